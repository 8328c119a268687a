"""Training driver of the learned support proposal (argument marshalling and
the epoch loop only: labels, features, every training step and the learned
solve run in the library's HIP kernels through paper_2407_06434_amd.omp).

Labels are the supports of plain OMP (omp_solve) on the training signals. Each
epoch visits the training set in a fresh seeded permutation, passed to the
library as minibatch row indices; the learning rate follows a cosine decay.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from paper_2407_06434_amd import omp


def omp_labels(dictionary: omp.Dictionary, Y: torch.Tensor, S: int, eps_per_signal: Optional[torch.Tensor] = None,
               chunk: int = 65536) -> torch.Tensor:
    """Supports [B][S] (int32, -1 padded) of plain OMP on Y, computed in chunks."""
    out = torch.empty((Y.shape[0], S), dtype=torch.int32, device=Y.device)
    ws = None
    for i in range(0, Y.shape[0], chunk):
        j = min(Y.shape[0], i + chunk)
        eps = None if eps_per_signal is None else eps_per_signal[i:j].contiguous()
        if ws is None:
            ws = torch.empty(omp.workspace_bytes(dictionary.M, dictionary.N, j - i, S, dictionary.precision,
                                                 with_dict=True), dtype=torch.uint8, device=Y.device)
        r = omp.solve(dictionary.A, Y[i:j], S, precision=dictionary.precision, dictionary=dictionary,
                      eps_per_signal=eps, dense=False, workspace=ws)
        out[i:j] = r.support
    return out


def features(mlp: omp.MLP, dictionary: omp.Dictionary, Y: torch.Tensor, chunk: int = 65536) -> torch.Tensor:
    """BF16 features (int16 bits, [B][N]) in chunks."""
    return torch.cat([mlp.features(dictionary, Y[i:i + chunk]) for i in range(0, Y.shape[0], chunk)])


def train(mlp: omp.MLP, F: torch.Tensor, support: torch.Tensor, epochs: int, batch: int = 1024,
          lr: float = 1e-3, lr_final: float = 1e-5, seed: int = 0, log=None) -> list:
    """Adam over `epochs` passes; returns the mean loss of every epoch."""
    n = F.shape[0]
    steps = n // batch
    total = epochs * steps
    losses = torch.zeros(steps, dtype=torch.float32, device=F.device)
    hist = []
    t = 0
    for ep in range(epochs):
        perm = np.random.default_rng([seed, ep]).permutation(n).astype(np.int32)
        perm_d = torch.from_numpy(perm).to(F.device)
        for s in range(steps):
            frac = t / max(1, total - 1)
            rate = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * frac))
            mlp.train_step(F, support, rate, loss=losses[s:s + 1], rows=perm_d[s * batch:(s + 1) * batch])
            t += 1
        hist.append(float(losses.mean().item()))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.4f}")
    return hist
