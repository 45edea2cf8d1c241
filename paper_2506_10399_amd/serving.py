"""Serving driver: a Poisson stream of encrypted 2-layer GCN requests through
the library's server (``ficgcn_server``: slots with their own streams,
admission by device-memory footprint, resident client keys).

Client side (per request): a seeded synthetic power-law graph and features,
the server's plan for it, the client's ciphertexts encrypted on the device
and parked in pinned host memory (the upload); after completion the client
decrypts the returned ciphertexts and checks them against the FP64 model.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from . import ficgcn as fg
from . import graph


@dataclass
class ClientRequest:
    name: str
    n_v: int
    dims: List[int]
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    x: np.ndarray
    weights: List[np.ndarray]
    plan: "fg.Plan" = None
    info: list = None
    inputs_host: object = None      # pinned torch tensor [n_in][2][L][N], or [n_in][L][N] when seeded
    output_host: object = None      # numpy [n_out][2][l_out+1][N]
    a_seed: Optional[int] = None    # public seed of seeded inputs (input i has ciphertext id i)
    packed_bits: int = 0            # seeded inputs' first polynomials packed at this many bits per residue
    result: dict = field(default_factory=dict)


def fp64_gcn(rp, col, val, x, weights):
    import scipy.sparse as sp
    n = len(rp) - 1
    A = sp.csr_matrix((val, col, rp), shape=(n, n))
    h = x
    for w in weights:
        h = A @ (h @ w)
        h = h * h
    return h


def make_requests(ctx: fg.Context, n_req: int, seed: int, n_range=(500, 4000), f_range=(64, 256), hidden: int = 16,
                  classes=(2, 10), model: Optional[fg.Mlp] = None, keep: int = 4,
                  corners: Sequence[tuple] = (), low_level: bool = False,
                  max_input_bytes: Optional[float] = None, log=None) -> List[ClientRequest]:
    """Graphs of log-uniform size and feature width (power-law, average
    degree 3-5, sampled neighbours + self, mean aggregation), binary features
    at 1%, N(0, 0.1^2) weights; plans by the paper's rule or, with a model,
    by the learned search.  corners: (n, F) shapes taken first (the range's
    extremes); low_level: the client encrypts at the lowest level the layers
    need; max_input_bytes: a drawn shape whose client ciphertexts would take the
    pool's total beyond this is skipped and the next one drawn (host memory); after 200
    skips in a row the pool is taken as full (fewer than n_req graphs)."""
    from workload.graphs import chung_lu, sample_neighbors
    from workload.features import binary_features, gaussian_weights
    rng = np.random.default_rng(seed)
    out = []
    total = 0.0
    corners = list(corners)
    r = 0
    skipped = 0
    while len(out) < n_req:
        if corners:
            n, F = corners.pop(0)
        else:
            n = int(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))
            F = int(np.exp(rng.uniform(np.log(f_range[0]), np.log(f_range[1]))))
        c = int(rng.integers(classes[0], classes[1] + 1))
        deg = float(rng.uniform(3.0, 5.0))
        s = int(rng.integers(1 << 30))
        if max_input_bytes is not None and out:
            # client ciphertexts before planning: (sampled neighbours + self) copies of F columns,
            # at most every prime of the chain
            est = (int(round(deg)) + 1) * F * 2 * ctx.L * ctx.N * 8.0
            if total + est > max_input_bytes:
                skipped += 1
                if skipped > 200:    # the pool is full: serve what it holds
                    if log:
                        log("pool full at %d graphs, %.1f GB" % (len(out), total / 1e9))
                    break
                if log and skipped <= 3:
                    log("skipped n=%d F=%d: about %.1f GB of ciphertexts beyond the pool's %.0f GB"
                        % (n, F, est / 1e9, max_input_bytes / 1e9))
                continue
        g = chung_lu(n, deg, s)
        nb = sample_neighbors(g, int(round(deg)), s + 1)
        rp, col, val = graph.normalize(n, nb, "mean")
        dims = [F, hidden, c]
        x = binary_features(n, F, 0.01, s + 2)
        ws = [gaussian_weights(dims[i], dims[i + 1], s + 3 + i) for i in range(2)]
        q = ClientRequest("req%d-n%d-F%d-c%d" % (r, n, F, c), n, dims, rp, col, val, x, ws)
        r += 1
        if model is not None:
            base = fg.PlanOpts(0, 1, 0, 0, 1, 0)
            base.low_level = int(low_level)
            base.max_key_bytes = 32e9   # keys of a graph's plan within an eighth of the device memory
            opts, _ = fg.ficgcn_plan_search(ctx, rp, col, val, n, dims, ws, base, model=model, keep=keep)
            q.plan = fg.Plan(ctx, rp, col, val, n, dims, ws, opts=opts)
        else:
            q.plan = fg.Plan(ctx, rp, col, val, n, dims, ws, activation=True, low_level=low_level)
        q.info = q.plan.ficgcn_plan_info()
        d0 = q.info[0]
        nbytes = d0["n_in_cts"] * 2 * (d0["level_in"] + 1) * ctx.N * 8.0
        if max_input_bytes is not None and out and total + nbytes > max_input_bytes:
            continue
        total += nbytes
        skipped = 0
        out.append(q)
        if log:
            log("planned %s: %d input ciphertexts, %.1f GB" % (q.name, d0["n_in_cts"], nbytes / 1e9))
    return out


def replicate(ctx: fg.Context, pool: Sequence[ClientRequest], n_req: int, seed: int) -> List[ClientRequest]:
    """A stream of n_req requests on graphs drawn uniformly from the pool: each request
    runs its pool entry's plan (the server encodes a plan's operands once and lets
    requests share it) on the entry's encrypted inputs, with its own output buffer."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_req):
        q = pool[int(rng.integers(len(pool)))]
        c = ClientRequest("%s#%d" % (q.name, r), q.n_v, q.dims, q.rowptr, q.col, q.val, q.x, q.weights)
        c.plan = q.plan
        c.info = q.info
        c.inputs_host = q.inputs_host
        c.a_seed = q.a_seed
        c.packed_bits = q.packed_bits
        c.output_host = np.zeros_like(q.output_host)
        out.append(c)
    return out


def client_keys(ctx: fg.Context, reqs: Sequence[ClientRequest], seed: int):
    """One client's keys covering every rotation its requests' plans use."""
    steps = set()
    for q in reqs:
        steps.update(q.plan.ficgcn_plan_rot_steps())
    return ctx.ckks_keygen(seed, sorted(steps), with_relin=True)


def encrypt_inputs(ctx: fg.Context, cl: fg.Keys, q: ClientRequest, seed: int, a_seed: Optional[int] = None,
                   whole: bool = False, packed_bits: int = 0):
    """The client's Inter-CA copies (copy k of column f at k*F + f, slots in
    the plan's node order), encrypted on the device, parked in pinned host
    memory; and a host buffer for the returned ciphertexts.  With a_seed the
    copies are seeded ciphertexts (uniform parts from the public a_seed, copy i
    with id i) and only their first polynomials are parked, half the upload,
    unless `whole` asks for both polynomials; packed_bits (seeded only) packs
    those residues at that many bits each (the widest prime's bit length)."""
    import torch
    pi = q.plan.ficgcn_plan_node_order()
    src = q.plan.ficgcn_plan_copy_sources(0)
    d0, dl = q.info[0], q.info[-1]
    lv = d0["level_in"]
    K, F = d0["K"], d0["f_in"]
    N, M = ctx.N, ctx.M
    half = a_seed is not None and not whole
    pk = packed_bits if half else 0
    shape = ((K * F, (lv + 1) * N * pk // 64) if pk else (K * F, lv + 1, N)) if half else (K * F, 2, lv + 1, N)
    try:
        host = torch.empty(shape, dtype=torch.int64, pin_memory=True)
    except RuntimeError:   # page-locked memory exhausted: a pageable buffer (the upload then blocks the slot)
        host = torch.empty(shape, dtype=torch.int64)
    dev = torch.empty((min(256, F), 2, lv + 1, N), dtype=torch.int64, device="cuda")
    packed = torch.empty((min(256, F),) + shape[1:], dtype=torch.int64, device="cuda") if pk else None
    for k in range(K):
        have = src[k] >= 0
        for f0 in range(0, F, dev.shape[0]):
            nf = min(dev.shape[0], F - f0)
            rows = np.zeros((nf, M))
            rows[:, pi[have]] = q.x[src[k][have], f0:f0 + nf].T
            pts = ctx.ckks_encode_batch(rows, 2.0 ** ctx.log_scale, lv)
            for i in range(nf):
                if a_seed is None:
                    ctx.ckks_encrypt(cl, pts[i], lv, seed, k * F + f0 + i, out=dev[i])
                else:
                    ctx.ckks_encrypt_seeded(cl, pts[i], lv, seed, a_seed, k * F + f0 + i, out=dev[i])
            if pk:
                for i in range(nf):
                    ctx.ckks_pack_residues(dev[i, 0], lv + 1, pk, out=packed[i])
            torch.cuda.synchronize()
            host[k * F + f0:k * F + f0 + nf].copy_(packed[:nf] if pk else dev[:nf, 0] if half else dev[:nf])
    q.inputs_host = host
    q.a_seed = a_seed if half else None
    q.packed_bits = pk
    q.output_host = np.zeros((dl["n_out_cts"], 2, dl["level_out"] + 1, N), dtype=np.uint64)


def decrypt_error(ctx: fg.Context, cl: fg.Keys, q: ClientRequest) -> float:
    import torch
    dl = q.info[-1]
    slots = []
    for o in q.output_host:
        # the returned words are the device's ciphertext words (evaluation form)
        d = torch.from_numpy(np.ascontiguousarray(o).view(np.int64)).to("cuda")
        slots.append(np.real(ctx.ckks_decrypt(cl, d, dl["level_out"], dl["scale_out"], ctx.M)))
    y = graph.read_output(q.plan.ficgcn_plan_node_order(), slots, dl["f_out"], dl["t"], dl["B"], dl["kind"] == 1)
    ref = fp64_gcn(q.rowptr, q.col, q.val, q.x, q.weights)
    return float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))


def run_stream(server: fg.Server, reqs: Sequence[ClientRequest], ev: fg.Keys, rate_per_s: float, seed: int,
               arrivals: Optional[Sequence[float]] = None) -> dict:
    """Submits the requests at Poisson arrival times (or the given offsets,
    seconds) and waits for all; returns the server's latency summary."""
    rng = np.random.default_rng(seed)
    if arrivals is None:
        arrivals = np.cumsum(rng.exponential(1.0 / rate_per_s, len(reqs))) if rate_per_s > 0 else np.zeros(len(reqs))
    t0 = time.perf_counter()
    ids = []
    for q, ta in zip(reqs, arrivals):
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ids.append(server.ficgcn_server_submit(q.plan, ev, q.inputs_host, len(q.inputs_host), q.output_host,
                                               len(q.output_host), a_seed=q.a_seed, packed_bits=q.packed_bits))
    for q, i in zip(reqs, ids):
        q.result = server.ficgcn_server_wait(i)
    return server.ficgcn_server_stats()
