"""Pins for the FP64 oracle: facts fixed by the paper and by mathematics, not by
the oracle itself.

Every function takes the oracle module and a loaded library handle, raises
AssertionError on failure, and is used twice: by ``test_oracle_pins.py`` on the
real oracle, and by ``test_oracle_mutations.py`` on deliberately broken copies
(each must fail at least one pin).

Sources of truth used here, none of which is the oracle's own code:
  * exhaustive best-subset search on tiny inputs (Section 1: greedy OMP versus
    the C(N, S) exhaustive search);
  * numpy's least-squares routine on a given support (Algorithm 1's LS step);
  * closed forms: S = 1 is the matched filter; an orthonormal dictionary makes
    OMP top-S thresholding of A^T y;
  * exact recovery of noiseless sparse x when Tropp's Exact Recovery Condition
    holds (Section 1's recovery remark);
  * invariants: residual orthogonal to the selected atoms (Section 4, numerical
    accuracy), non-increasing residual norm, Pythagoras;
  * metamorphic relations: column scaling (Appendix A), atom permutation,
    signal scaling;
  * scikit-learn's orthogonal_mp, an independent implementation.
"""
from __future__ import annotations

import itertools

import numpy as np


def _dict(M, N, seed, norms=None):
    g = np.random.default_rng(seed)
    A = g.standard_normal((N, M))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    if norms is not None:
        A *= g.uniform(norms[0], norms[1], size=(N, 1))
    return A.astype(np.float32)


def _lstsq(A, y, sup):
    As = A[sup].astype(np.float64).T
    x, *_ = np.linalg.lstsq(As, y.astype(np.float64), rcond=None)
    return x, y.astype(np.float64) - As @ x


def pin_s1_matched_filter(orc, lib):
    """S = 1: the pick minimises ||y - a_n x|| over all atoms, and x = a^T y / ||a||^2."""
    A = _dict(12, 40, 1, norms=(0.3, 3.0))
    Y = np.random.default_rng(2).standard_normal((30, 12)).astype(np.float32)
    o = orc.omp(A, Y, 1, lib=lib)
    A64 = A.astype(np.float64)
    for b in range(Y.shape[0]):
        y = Y[b].astype(np.float64)
        res = [np.linalg.norm(y - A64[n] * (A64[n] @ y) / (A64[n] @ A64[n])) for n in range(A.shape[0])]
        best = int(np.argmin(res))
        assert o["support"][b, 0] == best, (b, o["support"][b, 0], best)
        xc = (A64[best] @ y) / (A64[best] @ A64[best])
        assert abs(o["coef"][b, 0] - xc) <= 1e-12 * max(1.0, abs(xc))


def pin_bruteforce_tiny(orc, lib):
    """Tiny problems: every step's coefficients equal numpy LS on the picks so far,
    and ||r_OMP|| is never below the exhaustive best-subset residual."""
    g = np.random.default_rng(3)
    for trial in range(12):
        M, N, S = int(g.integers(5, 11)), int(g.integers(8, 17)), int(g.integers(1, 4))
        A = _dict(M, N, 100 + trial, norms=(0.5, 2.0))
        y = g.standard_normal(M).astype(np.float32)
        h = orc.omp_signal_history(A, y, S, lib=lib)
        sup = h["support"][: h["k"]]
        assert h["k"] == S
        assert len(set(sup.tolist())) == len(sup)
        for j in range(1, h["k"] + 1):
            x, r = _lstsq(A, y, sup[:j])
            np.testing.assert_allclose(h["coef_hist"][j - 1, :j], x, rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(h["rnorm_hist"][j], np.linalg.norm(r), rtol=1e-10, atol=1e-14)
        best = min(np.linalg.norm(_lstsq(A, y, list(c))[1]) for c in itertools.combinations(range(N), S))
        assert h["rnorm_hist"][S] >= best - 1e-12


def pin_greedy_choice(orc, lib):
    """Each pick maximises |a_n^T r| / ||a_n|| over unpicked atoms, with r the
    numpy-LS residual of the previous picks (the definition of the greedy step)."""
    g = np.random.default_rng(4)
    A = _dict(20, 60, 5, norms=(0.5, 2.0))
    A64 = A.astype(np.float64)
    nu = np.linalg.norm(A64, axis=1)
    for t in range(10):
        y = g.standard_normal(20).astype(np.float32)
        h = orc.omp_signal_history(A, y, 6, lib=lib)
        sup = h["support"][: h["k"]]
        for j in range(len(sup)):
            r = y.astype(np.float64) if j == 0 else _lstsq(A, y, sup[:j])[1]
            s = np.abs(A64 @ r) / nu
            s[sup[:j]] = -1
            assert sup[j] == int(np.argmax(s)), (t, j)
            np.testing.assert_allclose(h["s_best"][j], s.max(), rtol=1e-10)
            np.testing.assert_allclose(h["s_second"][j], np.sort(s)[-2], rtol=1e-10)


def pin_exact_recovery_erc(orc, lib):
    """Noiseless x whose support T satisfies Tropp's ERC, max_{n not in T} ||A_T^+ a_n||_1 < 1:
    OMP returns exactly T and x (Tropp 2004). Also the low-coherence [I | H/sqrt(M)] case."""
    g = np.random.default_rng(6)
    checked = 0
    for trial in range(40):
        M, N, K = 32, 64, 3
        A = _dict(M, N, 200 + trial)
        A64 = A.astype(np.float64)
        T = np.sort(g.choice(N, K, replace=False))
        pinv = np.linalg.pinv(A64[T].T)
        others = [n for n in range(N) if n not in set(T)]
        erc = max(np.abs(pinv @ A64[n]).sum() for n in others)
        if erc >= 1.0:
            continue
        checked += 1
        xs = np.sign(g.standard_normal(K)) * (1 + np.abs(g.standard_normal(K)))
        y = (xs @ A64[T]).astype(np.float32)
        o = orc.omp(A, y[None], K, lib=lib)
        assert set(o["support"][0].tolist()) == set(T.tolist())
        # coefficients equal LS on the float32-rounded y, which is x up to that rounding
        xl, _ = _lstsq(A, y, T)
        order = np.argsort(o["support"][0])
        np.testing.assert_allclose(o["coef"][0][order], xl, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(o["coef"][0][order], xs, rtol=1e-5, atol=1e-6)
    assert checked >= 10
    # [I | H / sqrt(M)] with H Hadamard: coherence 1/sqrt(M); S < (1 + sqrt(M)) / 2 guarantees recovery
    M = 16
    H = np.array([[1.0]])
    while H.shape[0] < M:
        H = np.block([[H, H], [H, -H]])
    A = np.concatenate([np.eye(M), H.T / np.sqrt(M)], axis=0).astype(np.float32)  # atoms are rows
    for trial in range(20):
        T = np.sort(g.choice(2 * M, 2, replace=False))
        xs = np.sign(g.standard_normal(2)) * (1 + np.abs(g.standard_normal(2)))
        y = (xs @ A[T].astype(np.float64)).astype(np.float32)
        o = orc.omp(A, y[None], 2, lib=lib)
        assert set(o["support"][0].tolist()) == set(T.tolist())


def pin_orthonormal_thresholding(orc, lib):
    """Orthonormal A (M = N): OMP is top-S hard thresholding of A^T y, x = (A^T y) on the support."""
    g = np.random.default_rng(7)
    M = 24
    Q, _ = np.linalg.qr(g.standard_normal((M, M)))
    A = Q.T.astype(np.float32)  # atoms = rows, orthonormal up to float32 rounding
    A64 = A.astype(np.float64)
    Y = g.standard_normal((8, M)).astype(np.float32)
    S = 5
    o = orc.omp(A, Y, S, lib=lib)
    nu = np.linalg.norm(A64, axis=1)
    for b in range(8):
        c = A64 @ Y[b].astype(np.float64)
        top = np.argsort(-np.abs(c) / nu, kind="stable")[:S]
        assert o["support"][b].tolist() == top.tolist()
        np.testing.assert_allclose(o["coef"][b], c[top] / nu[top] ** 2, rtol=1e-6, atol=1e-7)


def pin_invariants(orc, lib):
    """Residual orthogonal to the selected atoms (~1e-15 in FP64), ||r_k|| non-increasing,
    ||r_k||^2 = ||y||^2 - ||A_S x||^2 (Pythagoras for an orthogonal projection)."""
    A = _dict(48, 160, 8, norms=(0.5, 2.0))
    A64 = A.astype(np.float64)
    Y = np.random.default_rng(9).standard_normal((10, 48)).astype(np.float32)
    S = 12
    o = orc.omp(A, Y, S, lib=lib)
    for b in range(10):
        sup = o["support"][b]
        y = Y[b].astype(np.float64)
        fit = o["coef"][b] @ A64[sup]
        r = y - fit
        orth = np.abs(A64[sup] @ r).max() / (np.linalg.norm(y) * np.linalg.norm(A64[sup], axis=1).max())
        assert orth < 1e-13, orth
        rh = o["rnorm_hist"][b]
        assert np.all(np.diff(rh) <= 1e-12 * rh[0])
        np.testing.assert_allclose(rh[S] ** 2, y @ y - fit @ fit, rtol=1e-9, atol=1e-12 * (y @ y))
        np.testing.assert_allclose(rh[S], np.linalg.norm(r), rtol=1e-10)


def pin_metamorphic(orc, lib):
    """Column scaling (Appendix A): same support, x -> D^{-1} x. Atom permutation permutes
    the support. Signal scaling y -> alpha y, eps -> alpha eps: same support, x -> alpha x."""
    g = np.random.default_rng(10)
    A = _dict(40, 120, 11)
    Y = g.standard_normal((6, 40)).astype(np.float32)
    S = 8
    base = orc.omp(A, Y, S, lib=lib)
    d = np.exp2(g.integers(-3, 4, size=120)).astype(np.float32)  # powers of two: exact scaling
    sc = orc.omp(A * d[:, None], Y, S, lib=lib)
    assert np.array_equal(sc["support"], base["support"])
    np.testing.assert_allclose(sc["coef"] * d[sc["support"]], base["coef"], rtol=1e-10, atol=1e-12)
    perm = g.permutation(120)
    pe = orc.omp(A[perm], Y, S, lib=lib)
    assert np.array_equal(perm[pe["support"]], base["support"])
    np.testing.assert_allclose(pe["coef"], base["coef"], rtol=1e-10, atol=1e-12)
    al = np.float32(4.0)
    ys = orc.omp(A, Y * al, S, lib=lib)
    assert np.array_equal(ys["support"], base["support"])
    np.testing.assert_allclose(ys["coef"], base["coef"] * 4.0, rtol=1e-10, atol=1e-12)


def pin_tie_break_lowest(orc, lib):
    """Exact ties (duplicated atoms) go to the lowest index."""
    A = _dict(10, 20, 12)
    A[15] = A[4]
    A[17] = -A[9]
    y = (3.0 * A[4].astype(np.float64) + 0.1 * A[2]).astype(np.float32)
    o = orc.omp(A, y[None], 1, lib=lib)
    assert o["support"][0, 0] == 4
    y = (-5.0 * A[17].astype(np.float64) + 0.1 * A[3]).astype(np.float32)
    o = orc.omp(A, y[None], 1, lib=lib)
    assert o["support"][0, 0] == 9
    # Selected atoms are never re-selected, and all-zero scores go to the lowest
    # unselected index: atoms e0, e1, (e0+e1)/sqrt2 in R^3 and y = 2 e0 + e2.
    # Step 1 picks e0 (r = e2 exactly), every later score is exactly 0, so step 2
    # picks atom 1, and step 3 picks atom 2, which lies in span{e0, e1}.
    A3 = np.array([[1, 0, 0], [0, 1, 0], [np.sqrt(0.5), np.sqrt(0.5), 0]], np.float32)
    y3 = np.array([[2, 0, 1]], np.float32)
    o = orc.omp(A3, y3, 3, lib=lib)
    assert o["support"][0].tolist() == [0, 1, -1], o["support"]
    assert o["k"][0] == 2 and o["status"][0] == orc.SIG_DEPENDENT
    np.testing.assert_allclose(o["coef"][0, :2], [2.0, 0.0], atol=1e-15)


def pin_stop_rules(orc, lib):
    """Stop rules: y = 0 gives k = 0; eps >= ||y|| gives k = 0; a tolerance between two
    residual norms stops exactly there; non-finite y gives NONFINITE; a nearly dependent
    forced-last atom gives DEPENDENT."""
    A = _dict(16, 40, 13)
    Y = np.random.default_rng(14).standard_normal((3, 16)).astype(np.float32)
    Y[1] = 0
    o = orc.omp(A, Y, 5, lib=lib)
    assert o["k"][1] == 0 and o["support"][1, 0] == -1 and (o["status"][1] & orc.SIG_EPS)
    assert o["k"][0] == 5 and (o["status"][0] & orc.SIG_SMAX)
    yn = float(np.linalg.norm(Y[0].astype(np.float64)))
    o = orc.omp(A, Y[:1], 5, eps=yn * 1.0000001, lib=lib)
    assert o["k"][0] == 0
    full = orc.omp(A, Y[:1], 5, lib=lib)
    rh = full["rnorm_hist"][0]
    o = orc.omp(A, Y[:1], 5, eps=0.5 * (rh[2] + rh[3]), lib=lib)
    assert o["k"][0] == 3 and o["status"][0] == orc.SIG_EPS
    Yb = Y[:1].copy()
    Yb[0, 3] = np.nan
    o = orc.omp(A, Yb, 5, lib=lib)
    assert o["status"][0] == orc.SIG_NONFINITE and o["k"][0] == 0
    # two atoms 1e-4 rad apart: the second one is dependent at dep_tol = 1e-3
    a0 = np.zeros(3); a0[0] = 1.0
    a1 = np.array([1.0, 1e-4, 0.0]); a1 /= np.linalg.norm(a1)
    A2 = np.stack([a0, a1]).astype(np.float32)
    y = (a1 + 0.01 * np.array([0, 0, 1.0])).astype(np.float32)
    o = orc.omp(A2, y[None], 2, lib=lib)
    assert o["k"][0] == 1 and o["status"][0] == orc.SIG_DEPENDENT


def pin_per_signal_caps_and_tolerances(orc, lib):
    """Per-signal S_b and eps_b of a batch (Algorithm 1 runs independently per signal):
    a cap S_b keeps exactly the first S_b picks of the uncapped run (greedy picks do not
    depend on the cap); eps_b between two residual norms, computed here by numpy least
    squares on the uncapped run's prefixes, stops exactly between them; eps_b >= ||y_b||
    and S_b = 0 give k_b = 0; every signal equals a one-signal call with scalar S_b, eps_b."""
    g = np.random.default_rng(15)
    M, N, S, B = 24, 80, 8, 12
    A = _dict(M, N, 16, norms=(0.5, 2.0))
    Y = g.standard_normal((B, M)).astype(np.float32)
    full = orc.omp(A, Y, S, lib=lib)
    Sb = np.array([0, 1, 3, 8, 5, 8, 2, 8, 7, 4, 8, 6], np.int32)
    stop_at = np.array([-1, -1, -1, 2, -1, 5, -1, 0, 3, -1, 6, -1])  # eps_b between ||r_j|| and ||r_j+1||
    eps = np.zeros(B, np.float32)
    want_k = np.minimum(Sb, S).astype(int)
    for b in range(B):
        sup = full["support"][b]
        yb = Y[b].astype(np.float64)
        rn = [np.linalg.norm(yb)] + [np.linalg.norm(_lstsq(A, Y[b], sup[:j])[1]) for j in range(1, S + 1)]
        j = int(stop_at[b])
        if j >= 0:
            eps[b] = np.float32(0.5 * (rn[j] + rn[j + 1]))
            assert rn[j + 1] < eps[b] < rn[j]
            want_k[b] = min(want_k[b], j + 1)
    eps[4] = np.float32(np.linalg.norm(Y[4].astype(np.float64)) * 1.0001)  # eps >= ||y||
    want_k[4] = 0
    for kw in (dict(S_per_signal=Sb, eps_per_signal=eps), dict(S_per_signal=Sb), dict(eps_per_signal=eps)):
        o = orc.omp(A, Y, S, **kw, lib=lib)
        for b in range(B):
            kb = min(int(Sb[b]), S) if "S_per_signal" in kw else S
            if "eps_per_signal" in kw:
                kb = min(kb, int(want_k[b]) if stop_at[b] >= 0 or b == 4 else kb)
            assert o["k"][b] == kb, (kw.keys(), b, o["k"][b], kb)
            assert o["support"][b, :kb].tolist() == full["support"][b, :kb].tolist(), (b,)
            assert np.all(o["support"][b, kb:] == -1) and np.all(o["coef"][b, kb:] == 0.0)
            if kb > 0:
                x, _ = _lstsq(A, Y[b], full["support"][b, :kb])
                np.testing.assert_allclose(o["coef"][b, :kb], x, rtol=1e-10, atol=1e-12)
            eb = float(eps[b]) if "eps_per_signal" in kw else 0.0
            stopped_on_eps = eb > 0 and o["rnorm_hist"][b, kb] <= eb
            assert bool(o["status"][b] & orc.SIG_EPS) == stopped_on_eps, (b, o["status"][b])
            assert bool(o["status"][b] & orc.SIG_SMAX) == (kb >= (min(int(Sb[b]), S) if "S_per_signal" in kw else S))
            one = orc.omp(A, Y[b:b + 1], kb if kb < S else S, eb, lib=lib)
            assert one["support"][0, :kb].tolist() == o["support"][b, :kb].tolist()


def pin_sklearn_crosscheck(orc, lib):
    """scikit-learn's orthogonal_mp (unit-norm atoms) agrees on the plain 64x256 workload."""
    from sklearn.linear_model import orthogonal_mp
    from paper_2407_06434_amd import workloads
    w = workloads.plain_64x256()
    o = orc.omp(w.A, w.Y, w.S, lib=lib)
    X = orthogonal_mp(w.A.T.astype(np.float64), w.Y.T.astype(np.float64), n_nonzero_coefs=w.S)
    for b in range(w.B):
        assert set(np.nonzero(X[:, b])[0].tolist()) == set(o["support"][b].tolist())
    np.testing.assert_allclose(o["x"], X.T, rtol=1e-9, atol=1e-11)


def pin_forced_prefix(orc, lib):
    """Forced-prefix replay (the mode the GPU parity checker uses): the first nprefix_b
    picks are the forced atoms in order, whatever their scores, and the run then goes
    on greedily; at every step s_pick is the picked atom's |a^T r| / ||a|| and s_best
    and idx_best the largest such score over the atoms not yet picked and its atom,
    with r the least-squares residual on the picks so far (numpy here); nprefix_b = 0
    is the free run; a forced atom picked twice is refused."""
    import pytest
    g = np.random.default_rng(31)
    M, N, S, B = 20, 50, 7, 6
    A = _dict(M, N, 32, norms=(0.5, 2.0))
    Y = g.standard_normal((B, M)).astype(np.float32)
    free = orc.omp(A, Y, S, lib=lib)
    npre = np.array([0, 1, 3, 7, 2, 5], np.int32)
    pre = np.full((B, S), -1, np.int32)
    for b in range(B):
        pre[b, :npre[b]] = g.choice(N, int(npre[b]), replace=False)
    o = orc.omp(A, Y, S, prefix=pre, nprefix=npre, lib=lib)
    A64 = A.astype(np.float64)
    nu = np.linalg.norm(A64, axis=1)
    for b in range(B):
        assert o["k"][b] == S
        sup = o["support"][b, :S]
        assert sup[:npre[b]].tolist() == pre[b, :npre[b]].tolist(), b
        if npre[b] == 0:
            assert sup.tolist() == free["support"][b, :S].tolist()
        r = Y[b].astype(np.float64)
        for j in range(S):
            sc = np.abs(A64 @ r) / nu
            sc[sup[:j]] = -1.0
            best = int(np.argmax(sc))
            assert abs(o["s_best"][b, j] - sc[best]) <= 1e-10 * sc[best], (b, j)
            assert abs(o["s_pick"][b, j] - sc[sup[j]]) <= 1e-10 * sc[best], (b, j)
            assert o["idx_best"][b, j] == best, (b, j)
            if j >= npre[b]:
                assert sup[j] == best, (b, j)
            _, r = _lstsq(A, Y[b], sup[: j + 1])
        x, _ = _lstsq(A, Y[b], sup)
        np.testing.assert_allclose(o["coef"][b, :S], x, rtol=1e-9, atol=1e-12)
    twice = pre.copy()
    twice[3, 1] = twice[3, 0]
    with pytest.raises(ValueError):
        orc.omp(A, Y, S, prefix=twice, nprefix=npre, lib=lib)


PINS = [pin_s1_matched_filter, pin_bruteforce_tiny, pin_greedy_choice, pin_exact_recovery_erc,
        pin_orthonormal_thresholding, pin_invariants, pin_metamorphic, pin_tie_break_lowest,
        pin_stop_rules, pin_per_signal_caps_and_tolerances, pin_sklearn_crosscheck, pin_forced_prefix]
