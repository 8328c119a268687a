"""Step-by-step comparison of a GPU solve with the FP64 oracle.

For every checked signal the GPU's pick sequence is replayed through the
oracle (forced-prefix mode): at each step the oracle scores every atom given
the GPU's own earlier picks, so a pick is judged against the exact argmax of
the same problem, and a legitimate near-tie divergence does not cascade into
false failures later on.

Rules (supports identical as index sets; a near-tie whose top-two gap is below
`tie` relative is allowed; coefficients within `coef_tol` relative):
  * every GPU pick p at step j has FP64 score s_p >= (1 - tie) * s_best;
  * where no pick was a near-tie, the support set equals the free-running
    oracle's support set;
  * the number of picks and the stop reason agree with the oracle, except where
    ||r|| sits within `stop_tol` of the tolerance, or is numerically zero
    (<= 1e-12 ||y||: "stop on an exactly zero residual" is then decided by
    rounding, which differs between FP32 and FP64);
  * coefficient j on the GPU's support agrees with the oracle's least squares
    on that support within coef_tol * max(|x_j|, 1e-2 max_i |x_i|);
  * FP32 limits, counted apart (`unresolved_fp32`, signals), never as passes:
    with `residual_rounding`, a pick below the tie bar whose score gap to the
    best atom is within rho_j = 2 (j + 1) u ||y|| (u = 2^-24: the FP32
    residual's rounding error at pick j, which bounds the error of every score;
    the gap can only be that small relative to the best score once the best
    score itself is at that level, e.g. when S = M fills the signal space); and
    a coefficient error above coef_tol but within (k + 1) kappa(A_S)^2 u, the
    forward error bound of FP32 Cholesky of the k x k Gram matrix (its backward
    error is bounded by gamma_{k+1} ||G||: Higham, Accuracy and Stability of
    Numerical Algorithms, Thm 10.3), which exceeds 1e-4 only on ill-conditioned
    supports (kappa ~ 1.7 for a 64-atom support of a 1024 x 4096 Gaussian
    dictionary gives 65 kappa^2 u ~ 1e-5). `fp64=True` (the FP64 form) turns both
    allowances off;
  * the final ||r|| agrees within 1e-4 ||y|| (float32 residual);
  * the dense X holds the coefficients on the support and zero elsewhere.
"""
from __future__ import annotations

import numpy as np

SIG_MASK = 0xFF


def check(w, gpu: dict, orc, idx=None, tie=1e-5, coef_tol=1e-4, stop_tol=1e-5, threads=None,
          S_per=None, eps_per=None, eps=None, raise_on_fail=True, residual_rounding=False, fp64=False,
          free=None) -> dict:
    """Check the GPU results `gpu` (support, coef, status, rnorm, optional X) on the
    signals `idx` (default all). `free`: the oracle's own run on those signals, if the
    caller already has it (it is recomputed otherwise)."""
    B = w.Y.shape[0]
    idx = np.arange(B) if idx is None else np.asarray(idx)
    A = w.A
    Y = w.Y[idx]
    S = w.S
    eps = w.eps if eps is None else eps
    S_per = w.S_per_signal if S_per is None else S_per
    eps_per = w.eps_per_signal if eps_per is None else eps_per
    Sp = None if S_per is None else np.asarray(S_per)[idx]
    Ep = None if eps_per is None else np.asarray(eps_per)[idx]

    g_sup = np.asarray(gpu["support"])[idx]
    g_coef = np.asarray(gpu["coef"])[idx]
    g_status = np.asarray(gpu["status"])[idx]
    g_rn = np.asarray(gpu["rnorm"])[idx]
    g_k = g_status >> 8
    g_bits = g_status & SIG_MASK

    if free is None:
        free = orc.omp(A, Y, S, eps, S_per_signal=Sp, eps_per_signal=Ep, threads=threads)
    rep = orc.omp(A, Y, S, eps, S_per_signal=Sp, eps_per_signal=Ep, prefix=g_sup,
                  nprefix=g_k.astype(np.int32), threads=threads)

    rh0 = rep["rnorm_hist"][:, 0]
    fails = []
    near_ties = 0
    exact_support = 0
    worst_coef = 0.0
    worst_ratio = 1.0
    unresolved = set()     # signals with an FP32-limited pick or coefficient
    unresolved_picks = 0
    unresolved_coefs = 0
    if fp64:
        residual_rounding = False
    for i, b in enumerate(idx):
        k = int(g_k[i])
        sup = g_sup[i, :k]
        if np.any(g_sup[i, k:] != -1):
            fails.append((b, "support not -1 padded"))
        sb = rep["s_best"][i, :k]
        sp = rep["s_pick"][i, :k]
        ratio = np.where(sb > 0, sp / np.where(sb > 0, sb, 1), 1.0)
        worst_ratio = min(worst_ratio, float(ratio.min()) if k else 1.0)
        tied = ratio < 1.0
        bad = ratio < 1.0 - tie
        if residual_rounding and k:
            # The GPU's residual r = y - A_S x is formed in FP32: its error is about
            # (j + 1) u ||y|| at pick j, so two scores closer than twice that are
            # ordered by rounding. Such picks are counted apart, not passed.
            rho = 2.0 * np.arange(1, k + 1) * 2.0 ** -24 * rh0[i]
            unres = bad & ((sb - sp) <= rho)
            if unres.any():
                unresolved.add(int(b))
                unresolved_picks += int(unres.sum())
            bad &= ~unres
        if np.any(bad):
            j = int(np.argmax(bad))
            fails.append((b, f"pick {j} atom {sup[j]} scores {ratio[j]:.8f} of the best atom "
                             f"{rep['idx_best'][i, j]}"))
        near_ties += int(tied.sum())
        same = set(sup.tolist()) == set(free["support"][i, :free["k"][i]].tolist())
        exact_support += int(same)
        if not same and not tied.any():
            fails.append((b, "support differs from the oracle without a near-tie"))
        # stopping: the replay must stop exactly where the GPU stopped
        ystop = Ep[i] if Ep is not None else eps
        rh = rep["rnorm_hist"][i]
        fin = rh[: k + 2][np.isfinite(rh[: k + 2])]
        boundary = bool(ystop > 0 and fin.size and np.min(np.abs(fin - ystop)) <= stop_tol * max(rh[0], 1e-30))
        if np.isfinite(rh[k]) and rh[k] <= 1e-12 * rh[0]:
            boundary = True
        if rep["k"][i] != k and not boundary:
            fails.append((b, f"GPU stopped after {k} picks, oracle after {rep['k'][i]}"))
        if (rep["status"][i] & 0x2F) != (g_bits[i] & 0x2F) and not boundary:
            fails.append((b, f"status GPU {g_bits[i]} oracle {rep['status'][i]}"))
        # coefficients on the GPU's own support
        if rep["k"][i] == k and k > 0:
            xo = rep["coef"][i, :k]
            xg = g_coef[i, :k].astype(np.float64)
            scale = np.maximum(np.abs(xo), 1e-2 * np.abs(xo).max())
            err = np.abs(xg - xo) / scale
            worst_coef = max(worst_coef, float(err.max()))
            if err.max() > coef_tol:
                kappa = np.linalg.cond(A[sup].astype(np.float64).T)
                if not fp64 and err.max() <= (k + 1) * kappa * kappa * 2.0 ** -24:
                    unresolved.add(int(b))
                    unresolved_coefs += 1
                else:
                    fails.append((b, f"coefficient error {err.max():.3e}"))
            if abs(g_rn[i] - rh[k]) > 1e-4 * rh[0] + 1e-4 * rh[k]:
                fails.append((b, f"rnorm GPU {g_rn[i]:.6e} oracle {rh[k]:.6e}"))
        if np.any(g_coef[i, k:] != 0):
            fails.append((b, "coef not 0 padded"))
        if "X" in gpu and gpu["X"] is not None:
            xr = np.asarray(gpu["X"])[b]
            dense = np.zeros_like(xr)
            dense[sup] = g_coef[i, :k]
            if not np.array_equal(xr, dense):
                fails.append((b, "dense X does not match support/coef"))
    failed = {int(f[0]) for f in fails}
    report = dict(checked=len(idx), exact_support=exact_support, near_tie_picks=near_ties,
                  worst_coef_rel=worst_coef, worst_pick_ratio=worst_ratio, fails=fails[:20],
                  n_fail=len(fails), unresolved_fp32=len(unresolved - failed),
                  unresolved_fp32_picks=unresolved_picks, unresolved_fp32_coefs=unresolved_coefs,
                  passed=len(idx) - len(failed | unresolved))
    if raise_on_fail and fails:
        raise AssertionError(f"parity failures ({len(fails)}): {fails[:10]}; report {report}")
    return report
