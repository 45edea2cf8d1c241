"""GPU parity of the paper's latency-aware packing (Sec. 3.2, App. B): the first
layer in the case-1 layout (t input columns per ciphertext, each repeated for the
F' output columns; plaintexts A_hat_k (x) W-slice; ceil(log2 t) fold rotations)
and later layers combining the packed blocks by block rotations.

The oracle plans, encodes and encrypts; the library builds its own plan (equal
to the oracle's, checked on the host) and runs every layer in the plain, batched
and graph forms on the oracle's operands and ciphertexts: output words must equal
the oracle's.  A second pass encodes the operands with the library's encoder and
encrypts the client's case-1 slot vectors on the GPU; decrypted outputs must be
within 1e-3 of the FP64 GCN.

Cases: the tiny configuration at the rule's t = 2 (one layer, N = 2^13), the
two-layer shape on 100 nodes at t = 2 and t = 1 (x^2 after both layers), and the
three-layer skeleton shape at the rule's t."""
import numpy as np
import pytest

from oracle import ckks, gcn, planner, execute as ex
from oracle.params import Params
from workload import make_workload

pytestmark = pytest.mark.gpu

KEY_SEED, ENC_SEED = 21, 22

CASES = [("tiny", {}, "rule", None), ("tiny2", {"n_nodes": 100}, 2, None), ("tiny2", {"n_nodes": 100}, 1, 4),
         ("ntu_small", {}, "rule", None)]


def _ct(c):
    return np.stack([c.c0, c.c1])


def _setup(name, kw, first_pack, family):
    from paper_2506_10399_amd import ficgcn as fg, graph
    w = make_workload(name, **kw)
    prm = Params.from_dict(w.params)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    ref = gcn.gcn_forward(rows, w.x, w.weights, w.activation)[-1]
    o = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, family=family,
                           first_pack=first_pack)
    assert o.layers[0].pack == "rep"
    okeys = ckks.keygen(prm, KEY_SEED, o.rot_steps(prm.M), relin=w.activation)
    sched = ex.schedule(prm, o)
    ops = ex.encode_operands(prm, o, w.weights, sched)
    cts = ex.client_encrypt(prm, o, w.x, okeys, ENC_SEED)
    outs = ex.run(prm, o, okeys, cts, ops, sched)
    ctx = fg.Context.from_dict(w.params)
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    p = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, family=family or 0,
                activation=w.activation, first_pack=-1 if first_pack == "rule" else first_pack)
    assert np.array_equal(p.ficgcn_plan_node_order(), o.pi)
    cl, ev = ctx.ckks_keygen(KEY_SEED, p.ficgcn_plan_rot_steps(), with_relin=w.activation)
    return dict(w=w, prm=prm, ref=ref, o=o, ops=ops, cts=cts, outs=outs, ctx=ctx, p=p, cl=cl, ev=ev,
                graph=graph, fg=fg)


def _load_operands(e):
    p, o = e["p"], e["o"]
    for li, (lp, d) in enumerate(zip(o.layers, e["ops"])):
        if li == 0:
            flat = [pt.m for pt in d["P"]]
        else:
            if lp.family == 4:
                agg = [d["masks"][g][s][1] for g in range(len(d["masks"])) for s in lp.shifts]
            else:
                agg = [d["masks"][g][s].m for g in range(len(d["masks"])) for s in lp.shifts]
            cm = [d["CM"][s] for s in lp.comb_shifts]
            flat = agg + [x if isinstance(x, np.ndarray) else x.m for x in cm]
        assert len(flat) == p.ficgcn_plan_operand_count(li)
        for i, pt in enumerate(flat):
            p.ficgcn_plan_load_operand(li, i, pt)


def _run(e, mode, ins=None, outs=None):
    ctx, p = e["ctx"], e["p"]
    info = p.ficgcn_plan_info()
    lv0 = e["prm"].L - 1
    cur = ins if ins is not None else [ctx.ckks_ct_load(_ct(c), lv0) for c in e["cts"]]
    res = []
    for li, d in enumerate(info):
        o = outs[li] if outs is not None else [ctx.ct_buffer(d["level_in"]) for _ in range(d["n_out_cts"])]
        p.ficgcn_gcn_layer(e["ev"], li, cur, o, mode=mode)
        res.append((o, d["level_out"]))
        cur = o
    return res


def _decrypt(e, outs):
    lp = e["o"].layers[-1]
    d = e["p"].ficgcn_plan_info()[-1]
    slots = [np.real(e["ctx"].ckks_decrypt(e["cl"], x, d["level_out"], d["scale_out"], e["prm"].M)) for x in outs]
    t = e["prm"].M // lp.B
    y = e["graph"].read_output(e["o"].pi, slots, lp.f_out, t, lp.B, True)
    return gcn.max_rel_error(y, e["ref"])


@pytest.mark.parametrize("name,kw,first_pack,family", CASES)
def test_case1_layers_bit_exact_all_forms(name, kw, first_pack, family):
    import torch
    e = _setup(name, kw, first_pack, family)
    print("case", name, kw, first_pack, family, flush=True)
    _load_operands(e)
    for mode in (0, 1):
        for li, ((outs, lvo), want) in enumerate(zip(_run(e, mode), e["outs"])):
            for g, (a, b) in enumerate(zip(outs, want)):
                assert b.level == lvo
                assert np.array_equal(e["ctx"].ckks_poly_store(a, lvo, 2), _ct(b)), (name, "form", mode, "layer", li)
    # graph form on fixed buffers: capture, then replays with eager work between them
    ctx, info = e["ctx"], e["p"].ficgcn_plan_info()
    lv0 = e["prm"].L - 1
    ins = [ctx.ckks_ct_load(_ct(c), lv0) for c in e["cts"]]
    bufs = [[ctx.ct_buffer(d["level_in"]) for _ in range(d["n_out_cts"])] for d in info]
    for rep in range(3):
        res = _run(e, 2, ins, bufs)
        for li, ((outs, lvo), want) in enumerate(zip(res, e["outs"])):
            for a, b in zip(outs, want):
                assert np.array_equal(ctx.ckks_poly_store(a, lvo, 2), _ct(b)), (name, "graph replay", rep, li)
        for o in bufs:
            for x in o:
                x.zero_()
        _run(e, 1)
        torch.cuda.synchronize()
    assert _decrypt(e, _run(e, 1)[-1][0]) < 1e-3


@pytest.mark.parametrize("name,kw,first_pack,family", CASES[:2])
def test_case1_library_encoder_and_client_layout(name, kw, first_pack, family):
    """The library's own encoder for the operands and the client's case-1 slot vectors
    encrypted on the GPU: decrypted output within 1e-3 of the FP64 GCN."""
    e = _setup(name, kw, first_pack, family)
    ctx, p, prm, w = e["ctx"], e["p"], e["prm"], e["w"]
    p.ficgcn_plan_encode()
    d0 = p.ficgcn_plan_info()[0]
    rows = e["graph"].client_slots_rep(p.ficgcn_plan_node_order(), w.x, prm.M, p.ficgcn_plan_copy_sources(0),
                                       d0["t"], d0["B"], d0["f_out"])
    assert rows.shape[0] == d0["n_in_cts"]
    lv0 = prm.L - 1
    pts = ctx.ckks_encode_batch(rows, prm.scale, lv0)
    ins = [ctx.ckks_encrypt(e["cl"], pts[i], lv0, 5, i) for i in range(rows.shape[0])]
    assert _decrypt(e, _run(e, 1, ins)[-1][0]) < 1e-3
