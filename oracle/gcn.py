"""The plaintext FP64 GCN that the encrypted computation must reproduce
(test infrastructure only).

Layer (paper Sec. 2.2): X^{l+1} = sigma(A_hat X^l W^l), sigma(x) = x^2 (the
polynomial activation of Sec. 4.1) when the model has activations.
A_hat:
  "sym"  : D^-1/2 (A + I) D^-1/2, D the degrees of A + I, entry 1/sqrt(d_v d_u);
  "mean" : GraphSage MEAN over the sampled neighbours and the node itself
           (Sec. 2.2): entry 1 / (|S(v)| + 1) for u in S(v) and u = v.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np


def normalized_rows(n: int, neighbors: Sequence[np.ndarray], norm: str) -> List[List[Tuple[int, float]]]:
    """Row v of A_hat as (u, value) pairs sorted by u, self term included."""
    rows = []
    if norm == "sym":
        deg = [len(neighbors[v]) + 1 for v in range(n)]
        for v in range(n):
            us = sorted(set(int(u) for u in neighbors[v]) | {v})
            rows.append([(u, 1.0 / math.sqrt(deg[v] * deg[u])) for u in us])
    elif norm == "mean":
        for v in range(n):
            us = sorted(set(int(u) for u in neighbors[v]) | {v})
            val = 1.0 / len(us)
            rows.append([(u, val) for u in us])
    else:
        raise ValueError(norm)
    return rows


def dense_adjacency(n: int, rows) -> np.ndarray:
    a = np.zeros((n, n))
    for v, row in enumerate(rows):
        for u, val in row:
            a[v, u] = val
    return a


def aggregate(rows, x: np.ndarray) -> np.ndarray:
    """A_hat @ x, row by row."""
    out = np.zeros((len(rows), x.shape[1]))
    for v, row in enumerate(rows):
        for u, val in row:
            out[v] += val * x[u]
    return out


def gcn_forward(rows, x: np.ndarray, weights: Sequence[np.ndarray], activation: bool) -> List[np.ndarray]:
    """All layer outputs of the FP64 GCN; the last one is the model output."""
    outs = []
    h = x
    for w in weights:
        h = aggregate(rows, h) @ w
        if activation:
            h = h * h
        outs.append(h)
    return outs


def max_rel_error(approx: np.ndarray, exact: np.ndarray) -> float:
    """max_i |approx_i - exact_i| / max_i |exact_i| (error normalised by the
    output's infinity norm)."""
    return float(np.max(np.abs(approx - exact)) / np.max(np.abs(exact)))
