"""FP64 CPU oracle for Orthogonal Matching Pursuit (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The solver package never imports it, and
it imports nothing from the solver package.

The arithmetic lives in ``omp_oracle.c`` (Algorithm 1 of the paper, float64,
least squares from scratch by Householder QR at every step). This module only
builds that file with gcc and marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "omp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_omp.so")

SIG_EPS = 1
SIG_SMAX = 2
SIG_DEPENDENT = 4
SIG_NONFINITE = 8
SIG_EXHAUSTED = 32

# Dependency threshold on |R_kk| / ||a_n*|| (the distance of a picked atom to
# the span of the support, relative to its norm). The GPU path applies the
# same threshold to its Cholesky pivot, so both sides read the same quantity.
DEP_TOL = 1e-3

_lib = None


def build(src: str = _SRC, out: str = _LIB_PATH) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def load(path: Optional[str] = None):
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB_PATH
    if path is None and (not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(p)
    P = ctypes.c_void_p
    lib.oracle_omp_batch.restype = ctypes.c_int
    lib.oracle_omp_batch.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int64, ctypes.c_int, P,
                                     ctypes.c_int64, ctypes.c_int, P, ctypes.c_double, P, P, P,
                                     ctypes.c_double, P, P, P, P, P, P, P, P, P, ctypes.c_int]
    lib.oracle_omp_signal.restype = ctypes.c_int
    lib.oracle_omp_signal.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_int,
                                      ctypes.c_double, P, ctypes.c_int, ctypes.c_double, P, P, P, P,
                                      P, P, P, P, P, P]
    if path is None:
        _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def omp(A: np.ndarray, Y: np.ndarray, S: int, eps: float = 0.0, *,
        S_per_signal: Optional[np.ndarray] = None, eps_per_signal: Optional[np.ndarray] = None,
        prefix: Optional[np.ndarray] = None, nprefix: Optional[np.ndarray] = None,
        dep_tol: float = DEP_TOL, threads: Optional[int] = None, lib=None) -> dict:
    """Run the oracle on a batch.

    A: (N, M) float32 atom-major dictionary; Y: (B, M) float32 signals.
    prefix: optional (B, S) int32 forced picks, with nprefix[b] of them used.
    Returns a dict of per-signal arrays: support (B,S) int32 -1 padded, coef (B,S)
    float64 aligned with support, x (B,N) dense float64, rnorm_hist (B,S+1),
    s_best / s_second / s_pick (B,S), idx_best (B,S), k (B,), status (B,).
    """
    lib = lib or load()
    A = np.ascontiguousarray(A, dtype=np.float32)
    Y = np.ascontiguousarray(np.atleast_2d(Y), dtype=np.float32)
    N, M = A.shape
    B = Y.shape[0]
    assert Y.shape[1] == M
    S = int(S)
    sup = np.empty((B, S), np.int32)
    coef = np.empty((B, S), np.float64)
    rh = np.empty((B, S + 1), np.float64)
    sb = np.empty((B, S), np.float64)
    s2 = np.empty((B, S), np.float64)
    sp = np.empty((B, S), np.float64)
    ib = np.empty((B, S), np.int32)
    k = np.empty(B, np.int32)
    st = np.empty(B, np.int32)
    Sa = None if S_per_signal is None else np.ascontiguousarray(S_per_signal, dtype=np.int32)
    Ea = None if eps_per_signal is None else np.ascontiguousarray(eps_per_signal, dtype=np.float32)
    Pa = Na = None
    if prefix is not None:
        Pa = np.full((B, S), -1, np.int32)
        pre = np.asarray(prefix, dtype=np.int32)
        w = min(S, pre.shape[1])
        Pa[:, :w] = pre[:, :w]
        Na = np.ascontiguousarray(nprefix if nprefix is not None else np.full(B, w), dtype=np.int32)
    rc = lib.oracle_omp_batch(M, N, _ptr(A), M, B, _ptr(Y), M, S, _ptr(Sa), float(eps), _ptr(Ea),
                              _ptr(Pa), _ptr(Na), float(dep_tol), _ptr(sup), _ptr(coef), _ptr(rh),
                              _ptr(sb), _ptr(s2), _ptr(sp), _ptr(ib), _ptr(k), _ptr(st),
                              int(threads or default_threads()))
    if rc != 0:
        raise ValueError(f"oracle returned {rc} (-1: invalid forced prefix, -2: out of memory)")
    x = np.zeros((B, N), np.float64)
    rows, cols = np.nonzero(sup >= 0)
    x[rows, sup[rows, cols]] = coef[rows, cols]
    return dict(support=sup, coef=coef, x=x, rnorm_hist=rh, s_best=sb, s_second=s2, s_pick=sp,
                idx_best=ib, k=k, status=st)


def omp_signal_history(A: np.ndarray, y: np.ndarray, S: int, eps: float = 0.0,
                       dep_tol: float = DEP_TOL, lib=None) -> dict:
    """One signal, also returning the coefficient history coef_hist (S, S):
    row j holds the least-squares coefficients after pick j+1."""
    lib = lib or load()
    A = np.ascontiguousarray(A, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32).reshape(-1)
    N, M = A.shape
    sup = np.empty(S, np.int32)
    coef = np.empty(S, np.float64)
    ch = np.empty((S, S), np.float64)
    rh = np.empty(S + 1, np.float64)
    sb = np.empty(S, np.float64)
    s2 = np.empty(S, np.float64)
    sp = np.empty(S, np.float64)
    ib = np.empty(S, np.int32)
    k = np.empty(1, np.int32)
    st = np.empty(1, np.int32)
    rc = lib.oracle_omp_signal(M, N, _ptr(A), M, _ptr(y), S, float(eps), None, 0, float(dep_tol),
                               _ptr(sup), _ptr(coef), _ptr(ch), _ptr(rh), _ptr(sb), _ptr(s2), _ptr(sp),
                               _ptr(ib), _ptr(k), _ptr(st))
    if rc != 0:
        raise ValueError(f"oracle returned {rc}")
    return dict(support=sup, coef=coef, coef_hist=ch, rnorm_hist=rh, s_best=sb, s_second=s2,
                s_pick=sp, idx_best=ib, k=int(k[0]), status=int(st[0]))
