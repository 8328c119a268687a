"""FP64 reference of the learned support proposal (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; it imports nothing from the solver package.

The learned proposal is an extension of the paper's method, not part of it. The
pieces follow their textbook definitions, written out plainly in float64 with
numpy matrix products as the only library steps:

* features: the magnitude of the first correlation of Algorithm 1, normalised
  and scaled to unit size, f_n = sqrt(M) |a_n^T y| / (||a_n|| ||y||) (0 for a
  zero atom or a zero signal);
* a multilayer perceptron with two ReLU hidden layers,
  h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3;
* the loss: binary cross-entropy with logits against the multi-hot support of
  the plain OMP solution, summed over the outputs and averaged over the batch,
  L = (1/B) sum_b sum_n [softplus(z_bn) - t_bn z_bn];
* its gradient by the chain rule (backpropagation), dL/dz = (sigmoid(z) - t)/B;
* Adam (Kingma and Ba, ICLR 2015, Algorithm 1) with bias correction;
* the proposal: the S largest scores z (ties to the lowest index);
* the check: the least-squares fit of y on the proposed atoms (Eq. 2 of the
  paper, x = argmin ||y - A_P x||) and its residual norm against eps.

Precision of the stored intermediates. The GPU path keeps features, hidden
activations, the output gradient and the back-propagated activation
gradients in BF16 (the network's declared precision: BF16 operands, FP32
accumulation). ``rnd`` names the rounding the oracle applies at exactly those
points (round to nearest even, the IEEE rule, written out below), so that both
sides take the same precision decisions; every other operation is float64.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), returned as
    float64. bfloat16 keeps the top 16 bits of the float32 encoding: the value is
    first rounded to float32 (numpy, nearest even), then the low 16 bits are
    rounded away by adding 0x7FFF plus the lowest kept bit (nearest, ties to
    even). Inf and NaN do not occur in the network's values."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def identity(x):
    return np.asarray(x, dtype=np.float64)


def features(A: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """f[b, n] = sqrt(M) |a_n^T y_b| / (||a_n|| ||y_b||); A is (N, M) atom-major, Y (B, M)."""
    A = np.asarray(A, np.float64)
    Y = np.asarray(Y, np.float64)
    an = np.linalg.norm(A, axis=1)
    yn = np.linalg.norm(Y, axis=1)
    C = Y @ A.T
    inv_a = np.where(an > 0, 1.0 / np.where(an > 0, an, 1.0), 0.0)
    inv_y = np.where(yn > 0, 1.0 / np.where(yn > 0, yn, 1.0), 0.0)
    return np.sqrt(A.shape[1]) * np.abs(C) * inv_a[None, :] * inv_y[:, None]


def multi_hot(support: np.ndarray, n_out: int) -> np.ndarray:
    """t[b, n] = 1 where n is in the support of signal b (-1 entries ignored)."""
    support = np.asarray(support)
    T = np.zeros((support.shape[0], n_out))
    for b in range(support.shape[0]):
        s = support[b][support[b] >= 0]
        T[b, s] = 1.0
    return T


def forward(params: dict, F: np.ndarray, rnd=identity):
    """The network: returns z and the cache of the layer inputs. W_l is (out, in)."""
    x0 = rnd(F)
    a1 = x0 @ rnd(params["W1"]).T + params["b1"]
    h1 = rnd(np.maximum(a1, 0.0))
    a2 = h1 @ rnd(params["W2"]).T + params["b2"]
    h2 = rnd(np.maximum(a2, 0.0))
    z = h2 @ rnd(params["W3"]).T + params["b3"]
    return z, dict(x0=x0, h1=h1, h2=h2)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def bce_loss(z: np.ndarray, T: np.ndarray) -> float:
    """(1/B) sum over the batch and outputs of softplus(z) - t z."""
    return float(np.sum(softplus(z) - T * z) / z.shape[0])


def backward(params: dict, F: np.ndarray, T: np.ndarray, rnd=identity):
    """Loss and gradients of every parameter by the chain rule."""
    z, c = forward(params, F, rnd)
    B = z.shape[0]
    dz = rnd((sigmoid(z) - T) / B)
    g = {"W3": dz.T @ c["h2"], "b3": dz.sum(axis=0)}
    dh2 = rnd((dz @ rnd(params["W3"])) * (c["h2"] > 0))
    g["W2"] = dh2.T @ c["h1"]
    g["b2"] = dh2.sum(axis=0)
    dh1 = rnd((dh2 @ rnd(params["W2"])) * (c["h1"] > 0))
    g["W1"] = dh1.T @ c["x0"]
    g["b1"] = dh1.sum(axis=0)
    return bce_loss(z, T), g


def adam_step(params: dict, grads: dict, state: dict, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, Algorithm 1): biased first and second moment
    estimates, bias correction with the step count t, then the update."""
    t = state.get("t", 0) + 1
    state["t"] = t
    out = {}
    for k, p in params.items():
        gk = np.asarray(grads[k], np.float64)
        m = beta1 * state.get("m_" + k, np.zeros_like(gk)) + (1 - beta1) * gk
        v = beta2 * state.get("v_" + k, np.zeros_like(gk)) + (1 - beta2) * gk * gk
        state["m_" + k], state["v_" + k] = m, v
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        out[k] = np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return out


def top_s(scores: np.ndarray, S: int) -> np.ndarray:
    """Indices of the S largest scores per row, by score descending, ties to the
    lowest index."""
    scores = np.asarray(scores)
    out = np.empty((scores.shape[0], S), np.int64)
    for b in range(scores.shape[0]):
        order = sorted(range(scores.shape[1]), key=lambda n: (-scores[b, n], n))
        out[b] = order[:S]
    return out


def ls_check(A: np.ndarray, Y: np.ndarray, P: np.ndarray, eps: np.ndarray):
    """Least squares of y_b on the atoms P[b] (Eq. 2), by QR of A_P; returns the
    coefficients (aligned with P), the residual norms and the acceptance
    ||r|| <= eps_b."""
    A = np.asarray(A, np.float64)
    Y = np.asarray(Y, np.float64)
    B, S = P.shape
    X = np.zeros((B, S))
    rn = np.zeros(B)
    for b in range(B):
        AP = A[P[b]].T  # (M, S)
        Q, R = np.linalg.qr(AP)
        X[b] = np.linalg.solve(R, Q.T @ Y[b])
        rn[b] = np.linalg.norm(Y[b] - AP @ X[b])
    return X, rn, rn <= np.asarray(eps, np.float64)
