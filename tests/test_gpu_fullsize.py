"""Full-size parity (N = 2^16, every node and feature) of both layers of the
citation-graph shapes (2708 x 1433 and 3327 x 3703) and the clustered shape
(19717 x 500, 10 + 2 primes), in the launch configuration the benchmark times.

The layer is linear in its inputs until the rescales, so with all 7165 input
ciphertexts zero except a few at random (copy, feature) positions the oracle
computes the exact result from those terms alone: Z_f = sum_k P_k (.) X_{k,f},
H_l = sum_f w_{f,l} Z_f, two rescales, then the relinearised square.  The
GPU runs the whole layer (fused matrix-core pass over every input, batched
rescales and relinearisation) in the batched and the graph form, from the
ciphertexts and from the inputs rearranged as the pass's operands; all 16
output ciphertexts must equal the oracle's words.

The second layer (combination, packing, baby-step/giant-step SpIntra-CA with
hundreds to thousands of shifts, rescale, relinearised square) runs on seeded
uniform input words; the oracle's output words for the same inputs and key seed
are stored as SHA-256 digests by tests/golden/make_fullsize_digests.py (tens of
minutes of oracle time).  The GPU takes the oracle's encoded masks, computed here
from the oracle's encoder in worker processes, and generates its keys from the
same seed (its key words equal the oracle's: test_gpu_ops)."""
import hashlib
import json
import multiprocessing as mp
import os
import sys

import numpy as np
import pytest

from oracle import ckks, gcn, planner, execute as ex, simulate as sim, encoding as enc
from oracle.params import Params
from workload import make_workload

pytestmark = pytest.mark.gpu


def _ct(c):
    return np.stack([c.c0, c.c1])


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
if GOLDEN not in sys.path:
    sys.path.insert(0, GOLDEN)
import make_fullsize_digests as mfd  # noqa: E402

NAMES = ["cora", "citeseer", "pubmed"]


@pytest.mark.parametrize("name", NAMES)
def test_first_layer_sparse_inputs_bit_exact(name):
    import torch
    from paper_2506_10399_amd import ficgcn as fg, graph
    w = make_workload(name)
    prm = Params.from_dict(w.params)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    opts = mfd.case_options(name)
    o = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, **opts)
    st = ex.schedule(prm, o)[0]
    lp = o.layers[0]
    K, F, Fo, lv = lp.K, lp.f_in, lp.f_out, st["level_in"]
    P = [enc.encode(prm, p, st["sP"], lv) for p in sim.inter_plaintexts(o, lp)]
    W = ex.weight_ints(w.weights[0], st["sW"])
    okeys = ckks.keygen(prm, 5, [], relin=True)
    rng = np.random.default_rng(17)
    picks = sorted({(int(rng.integers(K)), int(rng.integers(F))) for _ in range(3)} | {(K - 1, F - 1)})
    qs = prm.q_level(lv)
    X = {}
    for k, f in picks:
        c = [np.stack([rng.integers(0, q, prm.N, dtype=np.uint64) for q in qs]) for _ in range(2)]
        X[(k, f)] = ckks.Ciphertext(c[0], c[1], lv, st["scale_in"])
    # oracle: the layer restricted to the nonzero terms
    zero = lambda s: ckks.Ciphertext(np.zeros((lv + 1, prm.N), np.uint64), np.zeros((lv + 1, prm.N), np.uint64), lv, s)
    fs = sorted({f for _, f in picks})
    Z = {f: ckks.pt_mul_acc(prm, zero(st["scale_in"] * st["sP"]), [X[(k, g)] for k, g in picks if g == f],
                            [P[k] for k, g in picks if g == f]) for f in fs}
    want = []
    for l in range(Fo):
        h = ckks.scalar_mul_acc(prm, zero(st["scale_in"] * st["sP"] * st["sW"]), [Z[f] for f in fs],
                                [int(W[f, l]) for f in fs])
        h = ckks.rescale(prm, ckks.rescale(prm, h))
        want.append(_ct(ckks.ct_mul_relin(prm, okeys, h, h)))
    # GPU: the whole layer over all 7165 inputs, contiguous as the benchmark holds them
    ctx = fg.Context.from_dict(w.params)
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    p = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, activation=w.activation, **opts)
    assert np.array_equal(p.ficgcn_plan_node_order(), o.pi)
    assert p.ficgcn_plan_info()[0]["level_in"] == lv
    for i, pt in enumerate(P):
        p.ficgcn_plan_load_operand(0, i, pt.m)
    _, ev = ctx.ckks_keygen(5, [], with_relin=True)
    block = torch.zeros((K * F, 2, lv + 1, prm.N), dtype=torch.int64, device="cuda")
    for (k, f), c in X.items():
        ctx.ckks_ct_load(_ct(c), lv, out=block[k * F + f])
    ins = [block[i] for i in range(K * F)]
    d = p.ficgcn_plan_info()[0]
    outs = [ctx.ct_buffer(lv) for _ in range(Fo)]
    for mode in (1, 2, 2):          # batched, graph capture, graph replay
        for x in outs:
            x.zero_()
        p.ficgcn_gcn_layer(ev, 0, ins, outs, mode=mode)
        for l in range(Fo):
            got = ctx.ckks_poly_store(outs[l], d["level_out"], 2)
            assert np.array_equal(got, want[l]), (name, "mode", mode, "output", l, "picks", picks)
    # the same layer from the inputs rearranged as the matrix-core pass's operands
    packed = p.ficgcn_plan_pack_inputs(0, ins)
    # digits 0..5 as bytes, digit 6 as a nibble: 832 words per (wave, step), the last feature block padded
    assert packed.numel() == K * -(-F // 64) * (prm.N // 16) * (lv + 1) * 2 * 832
    assert packed.numel() < 0.85 * block.numel()
    for mode in (1, 2, 2):
        for x in outs:
            x.zero_()
        p.ficgcn_gcn_layer(ev, 0, None, outs, mode=mode)
        for l in range(Fo):
            got = ctx.ckks_poly_store(outs[l], d["level_out"], 2)
            assert np.array_equal(got, want[l]), (name, "rearranged, mode", mode, "output", l, "picks", picks)
    del block, packed
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", NAMES)
def test_second_layer_full_size_words(name):
    """Second layer at the full size: the digests of the GPU's output words (plain,
    batched, graph capture and replay) equal the oracle's."""
    import torch
    from paper_2506_10399_amd import ficgcn as fg, graph
    with open(os.path.join(GOLDEN, "fullsize_layer2_digests.json")) as f:
        want = json.load(f)[name]
    w, prm, o, sched, st, lp, words = mfd.setup(name)
    assert want["options"] == mfd.case_options(name) and want["key_seed"] == mfd.KEY_SEED
    assert want["input_seed"] == mfd.input_seed(name)
    assert mfd.digest(np.asarray(o.pi, dtype=np.int64).astype(np.uint64)) == want["node_order_sha256"]
    ctx = fg.Context.from_dict(w.params)
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    p = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, activation=w.activation,
                **mfd.case_options(name))
    assert np.array_equal(p.ficgcn_plan_node_order(), o.pi)
    d = p.ficgcn_plan_info()[mfd.LAYER]
    assert (d["level_in"], d["level_out"], d["n_shifts"], d["G"], d["t"]) == \
        (want["level_in"], want["level_out"], want["n_shifts"], want["G"], want["t"])
    ns = len(lp.shifts)
    n_pk = -(-lp.f_out // lp.t)
    assert p.ficgcn_plan_operand_count(mfd.LAYER) == n_pk * ns
    # the oracle's mask encodings, packed ciphertext by packed ciphertext, in chunks of shifts
    chunk = 256
    jobs = [(name, g, lo, min(ns, lo + chunk)) for g in range(n_pk) for lo in range(0, ns, chunk)]
    with mp.get_context("spawn").Pool(8) as pool:
        for g, lo, pts in pool.imap_unordered(mfd.encode_mask_chunk, jobs):
            for j, m in enumerate(pts):
                p.ficgcn_plan_load_operand(mfd.LAYER, g * ns + lo + j, m)
        pool.close()
        pool.join()
    print("[%s] %d masks loaded" % (name, n_pk * ns), flush=True)
    _, ev = ctx.ckks_keygen(mfd.KEY_SEED, p.ficgcn_plan_rot_steps(), with_relin=w.activation)
    ins = [ctx.ckks_ct_load(words[i], d["level_in"]) for i in range(lp.f_in)]
    outs = [ctx.ct_buffer(d["level_in"]) for _ in range(d["n_out_cts"])]
    assert d["n_out_cts"] == want["n_out"]
    for mode in (0, 1, 2, 2):     # plain, batched, graph capture, graph replay
        for x in outs:
            x.zero_()
        p.ficgcn_gcn_layer(ev, mfd.LAYER, ins, outs, mode=mode)
        got = [ctx.ckks_poly_store(x, d["level_out"], 2) for x in outs]
        for g, x in enumerate(got):
            assert [int(v) for v in x[0, 0, :4]] == want["head"][g], (name, "mode", mode, "ct", g)
            assert mfd.digest(x) == want["sha256"][g], (name, "mode", mode, "ct", g)
    del ins, outs, ev
    torch.cuda.empty_cache()
