"""Learned cost model of the plan search: measurement, training, pruning.

The network (``ficgcn_mlp``: forward, backward and Adam in the library's
kernels) maps a candidate's local-adjacency features
(``ficgcn_candidate_features``) to the log of the latency, in ms, that the
batched SpIntra-CA layer of that candidate's plan takes on this GPU.  Training
data come from the kernels themselves: every candidate plan of a set of
seeded synthetic graphs is built, its operands filled with device-drawn
residues, and its layer timed.  ``ficgcn_plan_search`` then uses the network
to keep the few fastest-predicted candidates and lets the analytic judge pick
among them; with no network the judge builds every candidate.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

from . import ficgcn as fg
from . import graph

WIDTHS = (fg.N_FEATURES, 64, 64, 1)


@dataclass
class GraphCase:
    """One graph of the training or evaluation set."""
    name: str
    n_v: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    dims: List[int]
    weights: List[np.ndarray]


def synthetic_cases(n_cases: int, seed: int, dims=(16, 16, 7), n_range=(128, 2048)) -> List[GraphCase]:
    """Seeded graphs of the three generator families with log-uniform sizes,
    neighbour sampling and mean aggregation (as the citation shapes)."""
    from workload.graphs import chung_lu, dc_sbm, erdos_renyi, sample_neighbors
    from workload.features import gaussian_weights
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_cases):
        n = int(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))
        deg = float(rng.uniform(2.5, 6.0))
        kind = c % 3
        s = int(rng.integers(1 << 30))
        g = (erdos_renyi, chung_lu, dc_sbm)[kind](n, deg, s)
        nb = sample_neighbors(g, int(round(deg)), s + 1)
        rp, col, val = graph.normalize(n, nb, "mean")
        ws = [gaussian_weights(dims[i], dims[i + 1], s + 2 + i) for i in range(len(dims) - 1)]
        out.append(GraphCase("%s-%d" % (("er", "cl", "sbm")[kind], n), n, rp, col, val, list(dims), ws))
    return out


def features_of(ctx: fg.Context, case: GraphCase, cands: Sequence[fg.PlanOpts]) -> np.ndarray:
    return np.stack([fg.ficgcn_candidate_features(case.rowptr, case.col, case.n_v, case.dims, ctx.log_n, o)
                     for o in cands])


def measure_case(ctx: fg.Context, case: GraphCase, base: fg.PlanOpts, reps: int = 3, seed: int = 5,
                 max_keys: int = None, per_plan_keys: bool = False
                 ) -> Tuple[List[fg.PlanOpts], np.ndarray, np.ndarray]:
    """Times the batched SpIntra-CA layer of every candidate plan of one graph on this
    GPU: (candidates, features, median ms); a candidate needing more than max_keys
    rotation keys is not timed (NaN)."""
    cands = fg.ficgcn_plan_candidates(case.n_v, case.dims, ctx.log_n, base)
    ms = measure_plans(ctx, case, cands, bool(base.activation), reps, seed, max_keys, per_plan_keys)
    return cands, features_of(ctx, case, cands), ms


def measure_plans(ctx: fg.Context, case: GraphCase, opts: Sequence[fg.PlanOpts], activation: bool, reps: int = 3,
                  seed: int = 5, max_keys: int = None, per_plan_keys: bool = False) -> np.ndarray:
    """Median ms of the batched SpIntra-CA layer (the last layer) of the plan of each
    option set, operands filled with device-drawn residues, inputs uniform words.  Keys:
    one set for the plans' steps (with max_keys: plans taken by ascending key count while
    the set stays within max_keys keys), or (per_plan_keys) a set per plan freed after it;
    a plan left out is not timed (NaN)."""
    import torch
    plans = [fg.Plan(ctx, case.rowptr, case.col, case.val, case.n_v, case.dims, case.weights, opts=o) for o in opts]
    steps = [p.ficgcn_plan_rot_steps() for p in plans]
    ok = [max_keys is None or len(s_) <= max_keys for s_ in steps]
    ev = None
    if not per_plan_keys:
        union = set()
        if max_keys is not None:
            # one key set for the candidates in order of their key counts, up to max_keys keys in all
            for k in sorted(range(len(plans)), key=lambda i: len(steps[i])):
                if ok[k] and len(union | set(steps[k])) <= max_keys:
                    union |= set(steps[k])
                else:
                    ok[k] = False
        else:
            union = {x for s_ in steps for x in s_}
        _, ev = ctx.ckks_keygen(seed, sorted(union), with_relin=activation)
    ms = []
    li = len(case.dims) - 2    # the SpIntra-CA layer: the last one
    for k in range(len(plans)):
        if not ok[k]:
            ms.append(float("nan"))
            plans[k] = None
            continue
        p = plans[k]
        if per_plan_keys:
            _, ev = ctx.ckks_keygen(seed, steps[k], with_relin=activation)
        p.ficgcn_plan_fill_operands(seed)
        d = p.ficgcn_plan_info()[li]
        lv = d["level_in"]
        ins = [ctx.ct_buffer(lv) for _ in range(d["n_in_cts"])]
        for x in ins:
            x.random_(0, 1 << 49)     # residues below every 50-bit prime of the chain
        outs = [ctx.ct_buffer(lv) for _ in range(d["n_out_cts"])]
        times = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.ficgcn_gcn_layer(ev, li, ins, outs, mode=1)
            torch.cuda.synchronize()
            if r:
                times.append((time.perf_counter() - t0) * 1e3)
        ms.append(float(np.median(times)))
        del ins, outs, p
        plans[k] = None            # the plan's device operands are freed before the next one is filled
        if per_plan_keys:
            ev = None
    return np.array(ms)


def init_params(seed: int, widths=WIDTHS) -> np.ndarray:
    """He-normal weights, zero biases, packed as the library expects."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(widths[:-1], widths[1:]):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / a), size=(b, a)).ravel())
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def train(ctx: fg.Context, X: np.ndarray, y_ms: np.ndarray, epochs: int = 400, lr: float = 3e-3, batch: int = 64,
          seed: int = 0) -> Tuple[fg.Mlp, List[float]]:
    """Adam on mean squared error of log(ms), minibatches drawn on the host
    with a seeded permutation; every step runs in the library's kernels."""
    import torch
    net = fg.Mlp(ctx, WIDTHS, init_params(seed))
    xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    yd = torch.tensor(np.log(y_ms)[:, None], dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed + 1)
    n = len(X)
    losses = []
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n), device="cuda")
        tot = 0.0
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            xb = xd[idx].contiguous()
            yb = yd[idx].contiguous()
            tot += net.ficgcn_mlp_train_step(xb, yb, lr) * len(idx)
        losses.append(tot / n)
    return net, losses


def predict_ms(net: fg.Mlp, X: np.ndarray) -> np.ndarray:
    import torch
    xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    y = net.ficgcn_mlp_forward(xd)
    torch.cuda.synchronize()
    return np.exp(y.cpu().numpy()[:, 0])
