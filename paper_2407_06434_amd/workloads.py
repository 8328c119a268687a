"""Seeded synthetic workloads for batched Orthogonal Matching Pursuit.

This module only draws inputs. It holds none of the method's arithmetic: no
correlation, selection, least squares or residual. Both the solver's tests and
the FP64 oracle consume the arrays it returns, so the two sides always see the
same float32 bits.

Problem statement (Section 1 of the paper): y = A x + noise, with A an M x N
dictionary, x an S-sparse vector. The paper's realistic-application data
(image patches, face images, audio; Section 4, realistic-application table) is
not available, so these generators stand in for it with the shapes named below.

Layout. A is returned atom-major, shape (N, M): row n is atom a_n, contiguous
in m. Y is signal-major, shape (B, M).

Determinism. A is drawn from PCG64(1000 + cfg). The support, the values and the
noise each come from their own PCG64([2000 + cfg, stream]) generator and are
drawn row by row, so the first B' signals of a batch of B are identical to a
batch of B'. All draws are float64 and are cast to float32 exactly once.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    A: np.ndarray            # (N, M) float32, atom-major
    Y: np.ndarray            # (B, M) float32
    S: int                   # maximum sparsity (host scalar)
    eps: float               # scalar tolerance on ||r|| (<= 0: stop only on r == 0)
    S_per_signal: Optional[np.ndarray] = None    # (B,) int32 or None
    eps_per_signal: Optional[np.ndarray] = None  # (B,) float32 or None
    true_support: Optional[np.ndarray] = None    # (B, S_true) int64, -1 padded
    true_values: Optional[np.ndarray] = None     # (B, S_true) float64
    sigma: Optional[np.ndarray] = None           # (B,) noise std used per signal

    @property
    def M(self) -> int:
        return int(self.A.shape[1])

    @property
    def N(self) -> int:
        return int(self.A.shape[0])

    @property
    def B(self) -> int:
        return int(self.Y.shape[0])


def _rng(*seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(list(seed)))


def gaussian_dictionary(M: int, N: int, seed: int, column_norm: str = "none",
                        norm_range=(0.5, 2.0)) -> np.ndarray:
    """Atom-major (N, M) float64 dictionary with i.i.d. N(0, 1/M) entries.

    column_norm: "none" keeps the N(0, 1/M) draw; "unit" rescales every atom to
    unit norm; "uniform" rescales to unit norm and then multiplies atom n by a
    factor drawn from U[norm_range].
    """
    g = _rng(seed)
    A = g.standard_normal((N, M)) / np.sqrt(M)
    if column_norm in ("unit", "uniform"):
        A /= np.linalg.norm(A, axis=1, keepdims=True)
    if column_norm == "uniform":
        A *= g.uniform(norm_range[0], norm_range[1], size=(N, 1))
    return A


def sparse_signals(A64: np.ndarray, B: int, k: np.ndarray, seed: int, values: str,
                   noise_var: Optional[float] = None, snr_db: Optional[float] = None,
                   chunk: int = 256):
    """Draw B signals y_b = A x_b + e_b with |supp x_b| = k[b].

    values: "normal" draws N(0,1) values; "pm" draws +-(1 + |N(0,1)|).
    Noise is white Gaussian, either with a fixed variance or at a per-signal SNR
    in dB, sigma_b^2 = ||A x_b||^2 / (M 10^(snr/10)).
    Returns (Y float32 (B,M), support (B,kmax) int64 -1 padded, vals float64, sigma).
    """
    N, M = A64.shape
    kmax = int(np.max(k)) if B else 0
    g_sup, g_val, g_noise = _rng(seed, 0), _rng(seed, 1), _rng(seed, 2)
    Y = np.empty((B, M), dtype=np.float32)
    sup = np.full((B, kmax), -1, dtype=np.int64)
    vals = np.zeros((B, kmax), dtype=np.float64)
    sig = np.zeros(B, dtype=np.float64)
    for b0 in range(0, B, chunk):
        b1 = min(B, b0 + chunk)
        nb = b1 - b0
        keys = g_sup.random((nb, N))
        v = g_val.standard_normal((nb, kmax))
        e = g_noise.standard_normal((nb, M))
        clean = np.zeros((nb, M))
        for i in range(nb):
            kb = int(k[b0 + i])
            s = np.sort(np.argpartition(keys[i], kb - 1)[:kb]) if kb > 0 else np.zeros(0, np.int64)
            if values == "normal":
                xv = v[i, :kb]
            else:
                xv = np.sign(v[i, :kb]) * (1.0 + np.abs(v[i, :kb]))
            sup[b0 + i, :kb] = s
            vals[b0 + i, :kb] = xv
            clean[i] = xv @ A64[s]
        if snr_db is not None:
            sigma = np.sqrt(np.sum(clean * clean, axis=1) / (M * 10.0 ** (snr_db / 10.0)))
        else:
            sigma = np.full(nb, np.sqrt(noise_var if noise_var is not None else 0.0))
        sig[b0:b1] = sigma
        Y[b0:b1] = (clean + sigma[:, None] * e).astype(np.float32)
    return Y, sup, vals, sig


# ---------------------------------------------------------------------------
# The five workloads. Readings of unstated details:
#   * "N(0, v)" names the variance v, so the noise std is sqrt(v).
#   * "Gaussian" dictionaries without further detail are N(0, 1/M), not renormalised.
#   * "dB SNR" is per signal: sigma^2 = ||A x||^2 / (M 10^(SNR/10)).
#   * Where x values are unstated they are +-(1 + |N(0,1)|).
# ---------------------------------------------------------------------------

def plain_64x256(B: int = 100) -> Workload:
    """64x256 unit-norm dictionary, 8-sparse N(0,1) x, noise variance 1e-6, S=8."""
    A64 = gaussian_dictionary(64, 256, 1001, "unit")
    Y, sup, vals, sig = sparse_signals(A64, B, np.full(B, 8), 2001, "normal", noise_var=1e-6)
    return Workload("plain_64x256", A64.astype(np.float32), Y, 8, 0.0,
                    true_support=sup, true_values=vals, sigma=sig)


def batched_256x1024(B: int = 10000) -> Workload:
    """256x1024 dictionary, atom norms U[0.5,2], 32-sparse +-(1+|N|) x, noise variance 1e-4, S=32."""
    A64 = gaussian_dictionary(256, 1024, 1002, "uniform")
    Y, sup, vals, sig = sparse_signals(A64, B, np.full(B, 32), 2002, "pm", noise_var=1e-4)
    return Workload("batched_256x1024", A64.astype(np.float32), Y, 32, 0.0,
                    true_support=sup, true_values=vals, sigma=sig)


def bf16_1024x4096(B: int = 4096) -> Workload:
    """1024x4096 N(0,1/M) dictionary, 64-sparse +-(1+|N|) x at 30 dB SNR, S=64."""
    A64 = gaussian_dictionary(1024, 4096, 1003, "none")
    Y, sup, vals, sig = sparse_signals(A64, B, np.full(B, 64), 2003, "pm", snr_db=30.0)
    return Workload("bf16_1024x4096", A64.astype(np.float32), Y, 64, 0.0,
                    true_support=sup, true_values=vals, sigma=sig)


def face_8064x1207(B: int = 1200) -> Workload:
    """Tall dictionary of the face-recognition shape (8064-pixel images, 1207 training
    faces, S=30, B=1.2K; Section 4.2): unit-norm N(0,1/M) atoms standing in for the
    normalised face images, 30-sparse +-(1+|N|) x at 30 dB SNR."""
    A64 = gaussian_dictionary(8064, 1207, 1004, "unit")
    Y, sup, vals, sig = sparse_signals(A64, B, np.full(B, 30), 2004, "pm", snr_db=30.0)
    return Workload("face_8064x1207", A64.astype(np.float32), Y, 30, 0.0,
                    true_support=sup, true_values=vals, sigma=sig)


def uneven_pair(B_each: int = 10000):
    """Two dictionaries (128x512 and 512x2048, N(0,1/M)); per-signal S_i ~ U{4..64};
    true sparsity S_i; noise at 60 dB; eps_i = 1e-2 ||y_i||. Returns two Workloads."""
    out = []
    for j, (M, N) in enumerate(((128, 512), (512, 2048))):
        A64 = gaussian_dictionary(M, N, 1004 + 10 * j, "none")
        gS = _rng(2004 + 10 * j, 7)
        Si = gS.integers(4, 65, size=B_each).astype(np.int32)
        Y, sup, vals, sig = sparse_signals(A64, B_each, Si, 2004 + 10 * j, "pm", snr_db=60.0)
        eps_i = (1e-2 * np.linalg.norm(Y.astype(np.float64), axis=1)).astype(np.float32)
        out.append(Workload(f"uneven_{M}x{N}", A64.astype(np.float32), Y, 64, 0.0,
                            S_per_signal=Si, eps_per_signal=eps_i,
                            true_support=sup, true_values=vals, sigma=sig))
    return out


def learned_256x1024(B: int = 65536, stream: int = 0) -> Workload:
    """256x1024 N(0,1/M) dictionary, 32-sparse +-(1+|N|) x at 20 dB, S=32, eps_i = sigma_i sqrt(M).

    stream 0 is the evaluation set; other streams give disjoint training draws."""
    A64 = gaussian_dictionary(256, 1024, 1005, "none")
    Y, sup, vals, sig = sparse_signals(A64, B, np.full(B, 32), 2005 + 100 * stream, "pm", snr_db=20.0)
    eps_i = (sig * np.sqrt(256)).astype(np.float32)
    return Workload(f"learned_256x1024_s{stream}", A64.astype(np.float32), Y, 32, 0.0,
                    eps_per_signal=eps_i, true_support=sup, true_values=vals, sigma=sig)


def custom(M: int, N: int, B: int, S: int, seed: int = 7, values: str = "pm",
           snr_db: Optional[float] = 30.0, column_norm: str = "none", k_true: Optional[int] = None) -> Workload:
    """Arbitrary-size Gaussian workload for parity sweeps (ragged tiles, edge shapes)."""
    A64 = gaussian_dictionary(M, N, 5000 + seed, column_norm)
    kt = S if k_true is None else k_true
    Y, sup, vals, sig = sparse_signals(A64, B, np.full(B, kt), 6000 + seed, values,
                                       snr_db=snr_db, noise_var=None if snr_db is not None else 0.0)
    return Workload(f"custom_{M}x{N}_B{B}_S{S}", A64.astype(np.float32), Y, S, 0.0,
                    true_support=sup, true_values=vals, sigma=sig)


def mlp_init_params(n_in: int = 1024, n_hidden: int = 1024, n_out: int = 1024, seed: int = 3005,
                    prior: float = 32.0 / 1024.0, noise: float = 0.1) -> dict:
    """Initial weights of the support-proposal network, drawn here and passed to the
    library. Each layer starts as the identity (on the leading diagonal) plus
    He-uniform noise U(-s, s), s = noise * sqrt(6/fan_in); hidden biases are zero and
    the output bias is the log-odds of the prior support density. The untrained
    network therefore scores each atom by its matched-filter magnitude (the features),
    which training then refines. float32, W stored (out, in)."""
    g = _rng(seed)
    p = {}
    for name, (o, i) in (("1", (n_hidden, n_in)), ("2", (n_hidden, n_hidden)), ("3", (n_out, n_hidden))):
        lim = np.sqrt(6.0 / i) * noise
        W = g.uniform(-lim, lim, size=(o, i))
        W[np.arange(min(o, i)), np.arange(min(o, i))] += 1.0
        p["W" + name] = W.astype(np.float32)
        p["b" + name] = np.zeros(o, np.float32)
    p["b3"][:] = np.log(prior / (1.0 - prior))
    return p


WORKLOADS = {
    "plain_64x256": plain_64x256,
    "batched_256x1024": batched_256x1024,
    "bf16_1024x4096": bf16_1024x4096,
}
