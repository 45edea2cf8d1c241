"""Seeded random graphs shaped like the paper's workloads (Sec. 4.1, Table 5).

All graphs are simple and undirected.  Node labels are shuffled with the same
generator so that the identity node order carries no structure (the
"without reordering" baseline of the node-order optimisation).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np


@dataclass
class Graph:
    """Undirected simple graph as sorted adjacency lists."""
    n: int
    adj: List[np.ndarray]          # adj[v] = sorted int64 neighbour ids (no v)

    @property
    def n_edges(self) -> int:
        return int(sum(len(a) for a in self.adj) // 2)

    @property
    def avg_degree(self) -> float:
        return 2.0 * self.n_edges / max(self.n, 1)

    def degrees(self) -> np.ndarray:
        return np.array([len(a) for a in self.adj], dtype=np.int64)


def _from_edge_set(n: int, edges: np.ndarray, rng: np.random.Generator,
                   shuffle: bool) -> Graph:
    if shuffle:
        perm = rng.permutation(n)
        edges = perm[edges]
    nbrs: List[list] = [[] for _ in range(n)]
    for a, b in edges.tolist():
        nbrs[a].append(b)
        nbrs[b].append(a)
    adj = [np.array(sorted(set(x)), dtype=np.int64) for x in nbrs]
    return Graph(n=n, adj=adj)


def erdos_renyi(n: int, avg_degree: float, seed: int, shuffle: bool = False) -> Graph:
    """G(n, p) with p = avg_degree / (n - 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = avg_degree / max(n - 1, 1)
    iu = np.triu_indices(n, k=1)
    keep = rng.random(len(iu[0])) < p
    edges = np.stack([iu[0][keep], iu[1][keep]], axis=1)
    return _from_edge_set(n, edges, rng, shuffle)


def _draw_edges(n_target: int, sampler, rng: np.random.Generator) -> np.ndarray:
    """Draw distinct non-loop undirected edges until n_target are collected."""
    seen = set()
    out = []
    while len(out) < n_target:
        need = n_target - len(out)
        a, b = sampler(2 * need + 16)
        for x, y in zip(a.tolist(), b.tolist()):
            if x == y:
                continue
            key = (x, y) if x < y else (y, x)
            if key in seen:
                continue
            seen.add(key)
            out.append(key)
            if len(out) == n_target:
                break
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def _power_law_weights(n: int, gamma: float) -> np.ndarray:
    i0 = max(1.0, n ** 0.5 / 10.0)
    w = (np.arange(n, dtype=np.float64) + i0) ** (-1.0 / (gamma - 1.0))
    return w / w.sum()


def chung_lu(n: int, avg_degree: float, seed: int, gamma: float = 2.5,
             shuffle: bool = True) -> Graph:
    """Power-law graph: endpoints drawn with probability proportional to
    w_i ~ (i + i0)^(-1/(gamma-1)); exactly round(avg_degree*n/2) edges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = _power_law_weights(n, gamma)
    n_target = int(round(avg_degree * n / 2))

    def sampler(k):
        return rng.choice(n, size=k, p=w), rng.choice(n, size=k, p=w)

    edges = _draw_edges(n_target, sampler, rng)
    return _from_edge_set(n, edges, rng, shuffle)


def dc_sbm(n: int, avg_degree: float, seed: int, blocks: int = 3,
           gamma: float = 2.5, mu: float = 0.2, shuffle: bool = True) -> Graph:
    """Degree-corrected stochastic block model: `blocks` equal communities,
    power-law weights inside each, a fraction `mu` of edges between blocks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [n // blocks + (1 if b < n % blocks else 0) for b in range(blocks)]
    starts = np.cumsum([0] + sizes)
    ws = [_power_law_weights(s, gamma) for s in sizes]
    n_target = int(round(avg_degree * n / 2))

    def sampler(k):
        inter = rng.random(k) < mu
        ba = rng.integers(0, blocks, size=k)
        shift = rng.integers(1, blocks, size=k)
        bb = np.where(inter, (ba + shift) % blocks, ba)
        a = np.empty(k, dtype=np.int64)
        b = np.empty(k, dtype=np.int64)
        for blk in range(blocks):
            ma = ba == blk
            mb = bb == blk
            a[ma] = starts[blk] + rng.choice(sizes[blk], size=int(ma.sum()), p=ws[blk])
            b[mb] = starts[blk] + rng.choice(sizes[blk], size=int(mb.sum()), p=ws[blk])
        return a, b

    edges = _draw_edges(n_target, sampler, rng)
    return _from_edge_set(n, edges, rng, shuffle)


def sample_neighbors(g: Graph, n_sample: int, seed: int) -> List[np.ndarray]:
    """Neighbour sampling without replacement (GraphSage-style, Sec. 2.2):
    min(n_sample, deg v) neighbours of every node, returned sorted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for v in range(g.n):
        a = g.adj[v]
        if len(a) <= n_sample:
            out.append(a.copy())
        else:
            pick = rng.choice(len(a), size=n_sample, replace=False)
            out.append(np.sort(a[pick]))
    return out


def skeleton_frames(n_joints: int, n_frames: int, seed: int, max_degree: int = 4) -> Graph:
    """A multi-frame skeleton graph: one seeded random tree of n_joints joints
    (each joint attached to a uniformly chosen earlier joint with fewer than
    max_degree bones), repeated over n_frames frames as disjoint copies; node
    f * n_joints + j is joint j of frame f.  The shape of the paper's
    action-recognition workload (Sec. 4.1: 25 joints, 256 frames) without
    any of its data."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = np.zeros(n_joints, dtype=np.int64)
    bones = []
    for j in range(1, n_joints):
        cand = [i for i in range(j) if deg[i] < max_degree]
        i = int(cand[rng.integers(len(cand))])
        bones.append((i, j))
        deg[i] += 1
        deg[j] += 1
    edges = np.array([(f * n_joints + a, f * n_joints + b) for f in range(n_frames) for a, b in bones],
                     dtype=np.int64).reshape(-1, 2)
    return _from_edge_set(n_joints * n_frames, edges, rng, shuffle=False)
