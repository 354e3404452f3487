"""FP64 reference of the warm-start MLP (test infrastructure only).

A plain numpy definition of the network the HIP path trains: 192 inputs
(card masks, score features, padding), two ReLU layers of 256, two
outputs (policy logit, value); loss = per-parent cross-entropy of the
softmax of the logits over siblings against the target strategy (averaged
over parents) + value_weight/2 squared value error (averaged over rows).

With ``bf16=True`` every tensor the GPU feeds to a matrix multiply (inputs,
weights, hidden activations, output gradient, hidden gradients) is rounded
to bfloat16 (round to nearest even) at the same points as the GPU path,
which accumulates in FP32; with ``bf16=False`` everything stays FP64 (used to
pin the backward pass against finite differences).
"""
from __future__ import annotations

import numpy as np


N_IN = 192


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of bf16_round(x)."""
    return (np.asarray(bf16_round(x), np.float32).view(np.uint32) >> 16).astype(np.uint16)


def _q(x, on):
    return bf16_round(x) if on else np.asarray(x, np.float64)


def forward(W, X, bf16=True):
    """W = (W1, b1, W2, b2, W3, b3); X [M, N_IN].  Returns (H1, H2, Y) with H1,
    H2 the post-ReLU activations as fed to the next layer."""
    W1, b1, W2, b2, W3, b3 = W
    Xq = _q(X, bf16)
    H1 = _q(np.maximum(Xq @ _q(W1, bf16) + b1, 0.0), bf16)
    H2 = _q(np.maximum(H1 @ _q(W2, bf16) + b2, 0.0), bf16)
    Y = H2 @ _q(W3, bf16) + b3
    return H1, H2, Y


def loss_and_dY(Y, seg, tsig, tval, value_weight):
    """Per-parent softmax cross-entropy (rows seg[p]..seg[p+1]) and value MSE."""
    n_par = len(seg) - 1
    n_rows = Y.shape[0]
    dY = np.zeros_like(Y)
    lp = lv = 0.0
    for p in range(n_par):
        b, e = seg[p], seg[p + 1]
        z = Y[b:e, 0]
        ez = np.exp(z - z.max())
        pr = ez / ez.sum()
        dY[b:e, 0] = (pr - tsig[b:e]) / n_par
        lp -= np.sum(tsig[b:e] * np.log(np.maximum(pr, 1e-300))) / n_par
    dv = Y[:, 1] - tval
    dY[:, 1] = value_weight * dv / n_rows
    lv = 0.5 * value_weight * np.sum(dv * dv) / n_rows
    return lp + lv, dY


def backward(W, X, H1, H2, dY, bf16=True):
    """Gradients (dW1, db1, dW2, db2, dW3, db3) by the chain rule."""
    W1, b1, W2, b2, W3, b3 = W
    Xq = _q(X, bf16)
    dYq = _q(dY, bf16)
    dW3 = H2.T @ dYq
    db3 = dY.sum(axis=0)
    G2 = (dYq @ _q(W3, bf16).T) * (H2 > 0)
    G2q = _q(G2, bf16)
    dW2 = H1.T @ G2q
    db2 = G2.sum(axis=0)
    G1 = (G2q @ _q(W2, bf16).T) * (H1 > 0)
    G1q = _q(G1, bf16)
    dW1 = Xq.T @ G1q
    db1 = G1.sum(axis=0)
    return dW1, db1, dW2, db2, dW3, db3


def init_weights(rng, scale=1.0):
    """He-initialised weights (FP64)."""
    W1 = rng.normal(0, np.sqrt(2.0 / N_IN), (N_IN, 256)) * scale
    W2 = rng.normal(0, np.sqrt(2.0 / 256), (256, 256)) * scale
    W3 = rng.normal(0, np.sqrt(1.0 / 256), (256, 2)) * scale
    return [W1, np.zeros(256), W2, np.zeros(256), W3, np.zeros(2)]
