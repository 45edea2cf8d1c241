"""Data preparation around the library (host, no encryption arithmetic).

normalize  : the GCN's normalised adjacency A_hat (paper Sec. 2.2) as CSR with
             the diagonal: "sym" D^-1/2 (A + I) D^-1/2 (entry 1/sqrt(d_v d_u),
             d = degree + 1) or "mean" (GraphSage MEAN over the sampled
             neighbours and the node: 1 / (|S(v)| + 1)).
client_slots: the slot vectors the client encrypts for the first layer
             (client_slots_rep: the same in the case-1 layout of Sec. 3.2).
read_output : the n_v x F' output from decrypted slot vectors.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np


def normalize(n: int, neighbors: Sequence[np.ndarray], mode: str):
    rowptr = [0]
    col: List[int] = []
    val: List[float] = []
    if mode == "sym":
        deg = [len(neighbors[v]) + 1 for v in range(n)]
    for v in range(n):
        us = sorted(set(int(u) for u in neighbors[v]) | {v})
        for u in us:
            col.append(u)
            if mode == "sym":
                val.append(1.0 / math.sqrt(deg[v] * deg[u]))
            elif mode == "mean":
                val.append(1.0 / len(us))
            else:
                raise ValueError(mode)
        rowptr.append(len(col))
    return (np.array(rowptr, dtype=np.int32), np.array(col, dtype=np.int32), np.array(val, dtype=np.float64))


def client_slots(pi: np.ndarray, x: np.ndarray, M: int, copy_src: np.ndarray = None) -> np.ndarray:
    """Inter-CA (copy_src given): rows k*F + f hold copy k of column f,
    slot pi(v) = x[copy_src[k, v], f] (zero without a k-th term);
    otherwise rows f hold column f at slot pi(v)."""
    n, F = x.shape
    if copy_src is None:
        out = np.zeros((F, M))
        out[:, pi] = x.T
        return out
    K = copy_src.shape[0]
    out = np.zeros((K * F, M))
    for k in range(K):
        have = copy_src[k] >= 0
        out[k * F:(k + 1) * F][:, pi[have]] = x[copy_src[k][have]].T
    return out


def client_slots_rep(pi: np.ndarray, x: np.ndarray, M: int, copy_src: np.ndarray, t: int, B: int,
                     f_out: int) -> np.ndarray:
    """The case-1 layout of an Inter-CA first layer (paper Sec. 3.2, App. B): row k*J + j
    (J = ceil(F / t)) holds input columns j t + b (b < t) of copy k, column b repeated for
    every output column l < F' in the block starting at (b pow2(F') + l) B, node v at
    offset pi(v)."""
    n, F = x.shape
    K = copy_src.shape[0]
    J = -(-F // t)
    Fp = 1
    while Fp < f_out:
        Fp *= 2
    out = np.zeros((K * J, M))
    for k in range(K):
        have = copy_src[k] >= 0
        xs = x[copy_src[k][have]]
        for j in range(J):
            for b in range(min(t, F - j * t)):
                for l in range(f_out):
                    out[k * J + j, (b * Fp + l) * B + pi[have]] = xs[:, j * t + b]
    return out


def read_output(pi: np.ndarray, slots: Sequence[np.ndarray], f_out: int, t: int, B: int, packed: bool) -> np.ndarray:
    """Column l: slot pi(v) of ciphertext l (one column per ciphertext) or slot
    (l mod t) B + pi(v) of packed ciphertext l div t."""
    out = np.zeros((len(pi), f_out))
    for l in range(f_out):
        if packed:
            out[:, l] = np.real(slots[l // t][(l % t) * B + pi])
        else:
            out[:, l] = np.real(slots[l][pi])
    return out
