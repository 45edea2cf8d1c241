"""Fully connected network, squared-error loss and Adam in fp64 (test
infrastructure only; the reference for the library's cost-model kernels).

widths w_0 .. w_L; layer j maps a_j (n x w_j) to z_{j+1} = a_j W_j^T + b_j,
a_{j+1} = relu(z_{j+1}) except after the last layer.  Parameters are packed
layer by layer as W_j (w_{j+1} x w_j, row-major) then b_j.  Loss
L = mean over all n * w_L entries of (a_L - y)^2.  Gradients follow the chain
rule: dL/da_L = 2 (a_L - y) / (n w_L); dz = da * [z > 0] on hidden layers;
dW_j = dz_{j+1}^T a_j; db_j = column sums of dz_{j+1}; da_j = dz_{j+1} W_j.
Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def unpack(params: np.ndarray, widths: Sequence[int]) -> List[Tuple[np.ndarray, np.ndarray]]:
    out, o = [], 0
    for a, b in zip(widths[:-1], widths[1:]):
        W = params[o:o + a * b].reshape(b, a)
        o += a * b
        out.append((W, params[o:o + b]))
        o += b
    if o != len(params):
        raise ValueError("parameter count does not match the widths")
    return out


def forward(params: np.ndarray, widths: Sequence[int], X: np.ndarray):
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    acts, zs = [np.asarray(X, dtype=np.float64)], [None]
    for j, (W, b) in enumerate(layers):
        z = acts[-1] @ W.T + b
        zs.append(z)
        acts.append(np.maximum(z, 0.0) if j + 1 < len(layers) else z)
    return acts, zs


def loss_and_grad(params: np.ndarray, widths: Sequence[int], X: np.ndarray, Y: np.ndarray):
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    acts, zs = forward(params, widths, X)
    diff = acts[-1] - np.asarray(Y, dtype=np.float64)
    loss = float(np.mean(diff ** 2))
    da = 2.0 * diff / diff.size
    grads = []
    for j in range(len(layers) - 1, -1, -1):
        dz = da if j + 1 == len(layers) else da * (zs[j + 1] > 0)
        W, _ = layers[j]
        grads.append((dz.T @ acts[j], dz.sum(axis=0)))
        da = dz @ W
    grads.reverse()
    return loss, np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam_step(params, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    p = params - lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    return p, m, v
