"""The parity checker itself, on the CPU.

Results are built by the oracle (with forced picks where a mistake is planted), so
they are self-consistent apart from the planted pick: the oracle's own result
passes; a wrong pick on a large residual fails with or without the FP32
residual-rounding tie bound; a different last pick taken on a residual near the
rounding level of y fails without that bound and, with it, is counted as
unresolved in FP32 (neither a failure nor a pass).
"""
import numpy as np

from tests import parity


def _as_gpu(r):
    k = r["k"].astype(np.int32)
    coef = np.where(r["support"] >= 0, r["coef"], 0.0).astype(np.float32)
    rn = r["rnorm_hist"][np.arange(len(k)), k].astype(np.float32)
    return dict(support=r["support"].copy(), coef=coef, status=(k << 8) | r["status"], rnorm=rn)


def _forced(orc, w, b, j, atom):
    """The oracle's run on signal b with pick j replaced by `atom` (later picks free)."""
    base = orc.omp(w.A, w.Y[b:b + 1], w.S)
    pre = base["support"][:, : j + 1].copy()
    pre[0, j] = atom
    return orc.omp(w.A, w.Y[b:b + 1], w.S, prefix=pre, nprefix=np.array([j + 1], np.int32))


def _worst_other(r, b, j, N):
    """The lowest-numbered atom that is neither among the first j picks nor pick j."""
    used = set(r["support"][b, :j].tolist()) | {int(r["support"][b, j])}
    return next(n for n in range(N) if n not in used)


def test_oracle_result_passes(orc):
    from paper_2407_06434_amd import workloads
    w = workloads.custom(32, 128, 8, 32, seed=32, k_true=32)
    r = orc.omp(w.A, w.Y, w.S)
    for rr in (False, True):
        rep = parity.check(w, _as_gpu(r), orc, residual_rounding=rr)
        assert rep["n_fail"] == 0 and rep["unresolved_fp32"] == 0 and rep["passed"] == w.B


def test_wrong_early_pick_fails_with_either_bound(orc):
    from paper_2407_06434_amd import workloads
    w = workloads.custom(32, 128, 1, 32, seed=32, k_true=32)
    r = orc.omp(w.A, w.Y, w.S)
    bad = _forced(orc, w, 0, 2, _worst_other(r, 0, 2, w.N))
    for rr in (False, True):
        rep = parity.check(w, _as_gpu(bad), orc, residual_rounding=rr, raise_on_fail=False)
        assert any("pick 2 " in f[1] for f in rep["fails"]), rep
        assert rep["passed"] == 0 and rep["unresolved_fp32"] == 0


def test_last_pick_on_a_rounding_level_residual(orc):
    from paper_2407_06434_amd import workloads
    w = workloads.custom(32, 128, 48, 32, seed=32, k_true=32)
    r = orc.omp(w.A, w.Y, w.S)
    rel = r["rnorm_hist"][:, 31] / r["rnorm_hist"][:, 0]
    b = int(np.argmin(rel))
    assert rel[b] < 2e-6  # the last pick is taken on a residual near FP32 rounding of y
    sub = workloads.Workload(w.name, w.A, w.Y[b:b + 1], w.S, 0.0)
    # the second-best atom at the last pick, from the state before it
    h = orc.omp(w.A, w.Y[b:b + 1], 31)
    res = w.Y[b].astype(np.float64) - h["x"][0] @ w.A.astype(np.float64)
    nu = np.linalg.norm(w.A.astype(np.float64), axis=1)
    score = np.abs(w.A.astype(np.float64) @ res) / nu
    score[h["support"][0]] = -1.0
    second = int(np.argsort(score)[-2])
    bad = _forced(orc, sub, 0, 31, second)
    strict = parity.check(sub, _as_gpu(bad), orc, raise_on_fail=False)
    assert any("pick 31 " in f[1] for f in strict["fails"]), strict
    loose = parity.check(sub, _as_gpu(bad), orc, residual_rounding=True, raise_on_fail=False)
    assert loose["n_fail"] == 0, loose
    assert loose["unresolved_fp32"] == 1 and loose["unresolved_fp32_picks"] == 1 and loose["passed"] == 0, loose
    # the FP64 form's checks take no rounding allowance
    strict64 = parity.check(sub, _as_gpu(bad), orc, residual_rounding=True, fp64=True, raise_on_fail=False)
    assert any("pick 31 " in f[1] for f in strict64["fails"]), strict64
