"""The workload configurations: CKKS parameter sizes, graph shape, feature and
weight distributions.  Sizes follow the paper's datasets (Sec. 4.1, Table 5)
as synthetic stand-ins; no dataset item is reproduced.

Seeds: base = 1000 * config_id + replicate; graph, sampling, features and
each weight matrix take base*10 + k for k = 0, 1, 2, 3, ...
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from .graphs import Graph, erdos_renyi, chung_lu, dc_sbm, sample_neighbors, skeleton_frames
from .features import (binary_features, uniform_features, tfidf_features,
                       gaussian_weights)


CONFIGS: Dict[str, dict] = {
    # One layer X' = A X W at N = 2^13 (4 x 50-bit primes + 1 x 60-bit special).
    "tiny": dict(id=1, log_n=13, n_q=4, q_bits=50, n_p=1, p_bits=60, log_scale=40,
                 graph=("er", 128, 4.0), norm="sym", n_sample=None,
                 features=("uniform", 32), dims=[32, 16], activation=False),
    # Two-layer x^2 GCN at N = 2^13 with an 8-prime chain: the small case of the
    # two-layer path (same plan structure as the citation-graph shape).
    "tiny2": dict(id=6, log_n=13, n_q=8, q_bits=50, n_p=2, p_bits=60, log_scale=40,
                  graph=("chung_lu", 200, 3.9), norm="mean", n_sample=4,
                  features=("binary", 48, 0.05), dims=[48, 16, 7], activation=True),
    # Deep chains for the radix-2 aggregation (one level per routing round):
    # the shapes of "tiny" and "tiny2" with enough primes for every round.
    "tiny_deep": dict(id=7, log_n=13, n_q=10, q_bits=50, n_p=2, p_bits=60, log_scale=40,
                      graph=("er", 128, 4.0), norm="sym", n_sample=None,
                      features=("uniform", 32), dims=[32, 16], activation=False),
    "tiny2_deep": dict(id=8, log_n=13, n_q=14, q_bits=50, n_p=2, p_bits=60, log_scale=40,
                       graph=("chung_lu", 200, 3.9), norm="mean", n_sample=4,
                       features=("binary", 48, 0.05), dims=[48, 16, 7], activation=True),
    # Citation-graph shape with the primes a radix-2 second layer needs
    # (log QP = 18 * 50 + 2 * 60 = 1020 bits at N = 2^16).
    "cora_deep": dict(id=9, log_n=16, n_q=18, q_bits=50, n_p=2, p_bits=60, log_scale=40,
                      graph=("chung_lu", 2708, 3.9), norm="mean", n_sample=4,
                      features=("binary", 1433, 0.013), dims=[1433, 16, 7], activation=True),
    # Action-recognition shape: 25-joint skeleton over 256 frames (6400 nodes),
    # 3-dimensional joint features, 3-layer x^2 GCN 3-64-128-128, N = 2^14.
    # Weights N(0, 1/F) keep the three squared layers at magnitudes near 1.
    "ntu": dict(id=10, log_n=14, n_q=10, q_bits=50, n_p=2, p_bits=60, log_scale=40,
                graph=("skeleton", 25, 256), norm="sym", n_sample=None,
                features=("uniform", 3), dims=[3, 64, 128, 128], activation=True, w_std="fan_in"),
    # The same model on 8 frames at N = 2^13: the small case of the 3-layer path.
    "ntu_small": dict(id=11, log_n=13, n_q=10, q_bits=50, n_p=2, p_bits=60, log_scale=40,
                      graph=("skeleton", 25, 8), norm="sym", n_sample=None,
                      features=("uniform", 3), dims=[3, 16, 16, 8], activation=True, w_std="fan_in"),
    # Citation-graph shape: 2708 nodes, 1433 binary features, 2-layer x^2 GCN.
    "cora": dict(id=2, log_n=16, n_q=8, q_bits=50, n_p=2, p_bits=60, log_scale=40,
                 graph=("chung_lu", 2708, 3.9), norm="mean", n_sample=4,
                 features=("binary", 1433, 0.013), dims=[1433, 16, 7], activation=True),
    # Larger citation-graph shape: 3327 nodes, 3703 binary features.
    "citeseer": dict(id=3, log_n=16, n_q=8, q_bits=50, n_p=2, p_bits=60, log_scale=40,
                     graph=("chung_lu", 3327, 2.7), norm="mean", n_sample=3,
                     features=("binary", 3703, 0.0085), dims=[3703, 16, 6], activation=True),
    # Clustered graph: 19717 nodes in 3 communities, TF-IDF-like features.
    "pubmed": dict(id=4, log_n=16, n_q=10, q_bits=50, n_p=2, p_bits=60, log_scale=40,
                   graph=("sbm", 19717, 4.5), norm="mean", n_sample=5,
                   features=("tfidf", 500, 0.10), dims=[500, 16, 3], activation=True),
}


@dataclass
class Workload:
    name: str
    params: dict                      # CKKS sizes: log_n, n_q, q_bits, n_p, p_bits, log_scale
    graph: Graph
    neighbors: List[np.ndarray]       # aggregation neighbours per node (sampled or full)
    norm: str                         # "sym" (D^-1/2 (A+I) D^-1/2) or "mean"
    x: np.ndarray                     # n x F features
    weights: List[np.ndarray]         # per-layer weight matrices
    activation: bool                  # x^2 after every layer
    meta: dict = field(default_factory=dict)


def _graph(spec, seed: int) -> Graph:
    kind, n, deg = spec
    if kind == "skeleton":
        return skeleton_frames(n, int(deg), seed)
    if kind == "er":
        return erdos_renyi(n, deg, seed)
    if kind == "chung_lu":
        return chung_lu(n, deg, seed)
    if kind == "sbm":
        return dc_sbm(n, deg, seed)
    raise ValueError(kind)


def make_workload(name: str, replicate: int = 0, n_nodes: Optional[int] = None,
                  dims: Optional[List[int]] = None) -> Workload:
    """Build a configuration's seeded inputs.  `n_nodes` / `dims` shrink it
    (used for small parity cases of a large configuration's shape)."""
    cfg = dict(CONFIGS[name])
    base = 1000 * cfg["id"] + replicate
    gspec = list(cfg["graph"])
    if n_nodes is not None:
        gspec[1] = n_nodes
    g = _graph(tuple(gspec), base * 10 + 0)
    if cfg["n_sample"] is None:
        nbrs = [a.copy() for a in g.adj]
    else:
        nbrs = sample_neighbors(g, cfg["n_sample"], base * 10 + 1)
    dims = list(dims if dims is not None else cfg["dims"])
    fspec = cfg["features"]
    if fspec[0] == "uniform":
        x = uniform_features(g.n, dims[0], base * 10 + 2)
    elif fspec[0] == "binary":
        x = binary_features(g.n, dims[0], fspec[2], base * 10 + 2)
    elif fspec[0] == "tfidf":
        x = tfidf_features(g.n, dims[0], fspec[2], base * 10 + 2)
    else:
        raise ValueError(fspec)
    ws = [gaussian_weights(dims[i], dims[i + 1], base * 10 + 3 + i,
                           std=dims[i] ** -0.5 if cfg.get("w_std") == "fan_in" else 0.1)
          for i in range(len(dims) - 1)]
    params = {k: cfg[k] for k in ("log_n", "n_q", "q_bits", "n_p", "p_bits", "log_scale")}
    return Workload(name=name, params=params, graph=g, neighbors=nbrs, norm=cfg["norm"],
                    x=x, weights=ws, activation=cfg["activation"],
                    meta=dict(config_id=cfg["id"], replicate=replicate,
                              n_sample=cfg["n_sample"], dims=dims))
