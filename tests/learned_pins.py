"""Pins of the learned-proposal oracle (oracle/learned_oracle.py) against facts
that do not come from the oracle itself: the definition of the derivative
(central finite differences), the direct form of binary cross-entropy, closed
forms of Adam's first steps, torch's own bfloat16 conversion, Cauchy-Schwarz,
numpy's least-squares routine and stable sorting. Each pin takes the oracle
module, so that planted mistakes (tests/test_learned_oracle_mutations.py) can be
shown to fail one."""
import numpy as np


def _tiny(seed=0, n_in=7, hid=6, n_out=5):
    g = np.random.default_rng(seed)
    p = {"W1": g.normal(size=(hid, n_in)), "b1": g.normal(size=hid) * 0.3,
         "W2": g.normal(size=(hid, hid)) * 0.5, "b2": g.normal(size=hid) * 0.3,
         "W3": g.normal(size=(n_out, hid)) * 0.5, "b3": g.normal(size=n_out) * 0.3}
    F = g.normal(size=(4, n_in))
    T = (g.random(size=(4, n_out)) < 0.4).astype(float)
    return p, F, T


def pin_gradient_finite_differences(lo):
    """Every gradient entry matches a central difference of the loss (h = 1e-6)."""
    p, F, T = _tiny()
    loss, g = lo.backward(p, F, T)
    z, _ = lo.forward(p, F)
    assert abs(loss - lo.bce_loss(z, T)) < 1e-12
    h = 1e-6
    for k in p:
        it = np.nditer(p[k], flags=["multi_index"])
        for _ in it:
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k][it.multi_index] += h
            lp = lo.bce_loss(lo.forward(q, F)[0], T)
            q[k][it.multi_index] -= 2 * h
            lm = lo.bce_loss(lo.forward(q, F)[0], T)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][it.multi_index]) <= 1e-6 * max(1.0, abs(fd)), (k, it.multi_index, fd,
                                                                                  g[k][it.multi_index])


def pin_bce_direct_form(lo):
    """softplus(z) - t z equals -[t log s + (1-t) log(1-s)], s = 1/(1+e^-z), for moderate z;
    sigmoid is exact at 0 and symmetric."""
    z = np.linspace(-8, 8, 33)[None, :]
    for t in (0.0, 1.0):
        T = np.full_like(z, t)
        s = 1.0 / (1.0 + np.exp(-z))
        direct = -np.sum(t * np.log(s) + (1 - t) * np.log(1 - s))
        assert abs(lo.bce_loss(z, T) - direct) < 1e-9 * abs(direct)
    assert lo.sigmoid(np.array([0.0]))[0] == 0.5
    zz = np.array([-3.0, -0.5, 2.0, 30.0])
    assert np.allclose(lo.sigmoid(zz) + lo.sigmoid(-zz), 1.0, atol=1e-15)


def pin_adam_closed_forms(lo):
    """With zero moments, step 1 moves each parameter by lr g/(|g| + eps); a constant
    gradient keeps the bias-corrected step at lr g/(|g| + eps) for every t."""
    lr, eps = 1e-2, 1e-8
    p = {"w": np.array([1.0, -2.0, 0.5]), "c": np.array([0.0])}
    g = {"w": np.array([0.3, -4.0, 1e-3]), "c": np.array([2.0])}
    st = {}
    q = p
    for t in range(1, 6):
        q2 = lo.adam_step(q, g, st, lr, eps=eps)
        for k in p:
            step = lr * g[k] / (np.abs(g[k]) + eps)
            assert np.allclose(q[k] - q2[k], step, rtol=1e-7, atol=1e-13), (t, k)
        q = q2
    assert st["t"] == 5


def pin_bf16_rounding(lo):
    """Round to nearest even at the bfloat16 spacing, and agreement with torch's conversion."""
    import torch
    one = 1.0
    assert lo.bf16_round(np.array([one]))[0] == 1.0
    assert lo.bf16_round(np.array([1 + 2.0 ** -8]))[0] == 1.0              # tie -> even
    assert lo.bf16_round(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6  # tie -> even (up)
    assert lo.bf16_round(np.array([-(1 + 3 * 2.0 ** -8)]))[0] == -(1 + 2.0 ** -6)
    x = np.random.default_rng(3).normal(size=20000) * np.exp(np.random.default_rng(4).normal(size=20000) * 5)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lo.bf16_round(x), ref)


def pin_features(lo):
    """f_n = sqrt(M) when y is a multiple of atom n (Cauchy-Schwarz equality), 0 <= f <= sqrt(M),
    zero atoms and zero signals give 0."""
    g = np.random.default_rng(5)
    A = g.normal(size=(40, 16))
    A[7] = 0.0
    Y = np.vstack([3.0 * A[3], -0.5 * A[11], np.zeros(16), g.normal(size=16)])
    F = lo.features(A, Y)
    assert abs(F[0, 3] - 4.0) < 1e-13 and abs(F[1, 11] - 4.0) < 1e-13
    assert np.all(F >= 0) and np.all(F <= 4 + 1e-13)
    assert np.all(F[:, 7] == 0.0) and np.all(F[2] == 0.0)
    assert abs(F[3, 0] - 4 * abs(A[0] @ Y[3]) / np.linalg.norm(A[0]) / np.linalg.norm(Y[3])) < 1e-13


def pin_top_s(lo):
    """The S largest scores by a stable sort on (-score, index); ties go to the lowest index."""
    g = np.random.default_rng(6)
    sc = np.round(g.normal(size=(5, 50)), 1)  # many exact ties
    P = lo.top_s(sc, 8)
    for b in range(5):
        ref = np.lexsort((np.arange(50), -sc[b]))[:8]
        assert np.array_equal(P[b], ref)
    assert np.array_equal(lo.top_s(np.zeros((1, 6)), 3)[0], [0, 1, 2])


def pin_ls_check(lo):
    """Least squares on the proposal agrees with numpy's lstsq; a noiseless y = A_P x
    is fitted exactly; the residual is orthogonal to the proposed atoms."""
    g = np.random.default_rng(7)
    A = g.normal(size=(60, 24))
    P = np.array([[3, 10, 41, 7, 0], [59, 1, 2, 30, 31]])
    xs = g.normal(size=(2, 5))
    Y = np.vstack([A[P[0]].T @ xs[0], A[P[1]].T @ xs[1] + 0.1 * g.normal(size=24)])
    X, rn, acc = lo.ls_check(A, Y, P, np.array([1e-9, 1e-9]))
    assert np.allclose(X[0], xs[0], atol=1e-10) and rn[0] < 1e-10 and acc[0] and not acc[1]
    ref = np.linalg.lstsq(A[P[1]].T, Y[1], rcond=None)[0]
    assert np.allclose(X[1], ref, atol=1e-10)
    r = Y[1] - A[P[1]].T @ X[1]
    assert np.allclose(A[P[1]] @ r, 0.0, atol=1e-10)
    assert abs(rn[1] - np.linalg.norm(r)) < 1e-12


def pin_multi_hot(lo):
    T = lo.multi_hot(np.array([[2, 0, -1], [4, 4, 1]]), 6)
    assert np.array_equal(T, [[1, 0, 1, 0, 0, 0], [0, 1, 0, 0, 1, 0]])


PINS = [pin_gradient_finite_differences, pin_bce_direct_form, pin_adam_closed_forms, pin_bf16_rounding,
        pin_features, pin_top_s, pin_ls_check, pin_multi_hot]
