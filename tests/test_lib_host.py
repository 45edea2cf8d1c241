"""Host-side checks of the HIP library (no GPU needed): the shared library
loads and exports every entry point include/ficgcn.h declares, the prime chain
equals the oracle's, and the C++ planner reproduces the oracle's plan exactly
(node order, copies, shifts, routing family, integer weights, rotation keys,
scale schedule)."""
import os
import re

import numpy as np
import pytest

from oracle import gcn, planner, execute as ex, simulate as sim
from oracle.params import Params
from workload import make_workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ficgcn.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:ficgcn_status|void|const char\*|size_t)\s+(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def fg():
    from paper_2506_10399_amd import ficgcn
    if not os.path.exists(ficgcn.LIB_PATH):
        pytest.fail("libficgcn.so is not built; run __graft_entry__.build()")
    return ficgcn


def test_header_symbols_exported(fg):
    import ctypes
    lib = ctypes.CDLL(fg.LIB_PATH)
    names = _declared()
    assert len(names) >= 40
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared entry points
    assert sorted(fg.exported_symbols()) == names


def test_binding_structs_match_the_header_layout(fg, tmp_path):
    """Every struct the binding mirrors has the header's size and each field's offset and
    width (a C program built with gcc from include/ficgcn.h prints them)."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    pairs = [("ckks_params", fg.CkksParams), ("ficgcn_plan_opts", fg.PlanOpts), ("ckks_operand", fg.Operand),
             ("ficgcn_search_stats", fg.SearchStats), ("ficgcn_request", fg.Request),
             ("ficgcn_request_result", fg.RequestResult), ("ficgcn_server_summary", fg.ServerSummary)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ficgcn.h"', 'int main(void) {']
    for cname, py in pairs:
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('  printf("%s %s %%zu %%zu\\n", offsetof(%s, %s), sizeof(((%s*)0)->%s));'
                         % (cname, f, cname, f, cname, f))
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): [int(v) for v in l.split()[2:]] for l in out if l}
    for cname, py in pairs:
        assert got[(cname, "size")] == [ctypes.sizeof(py)], cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == [getattr(py, f).offset, getattr(py, f).size], (cname, f)


@pytest.mark.parametrize("name", ["tiny", "tiny2", "cora", "pubmed"])
def test_prime_chain_matches_oracle(fg, name):
    w = make_workload(name, n_nodes=16, dims=[2, 2])
    ctx = fg.Context.from_dict(w.params)
    prm = Params.from_dict(w.params)
    assert ctx.ckks_ctx_moduli() == prm.q + prm.p
    for k in (1, -1, 5, 1000):
        assert ctx.ckks_galois_element(k) == pow(5, k % prm.M, 2 * prm.N)


def _plans(fg, name, mode, noo, family, t=None, TH=None, **kw):
    from paper_2506_10399_amd import graph
    w = make_workload(name, **kw)
    prm = Params.from_dict(w.params)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    o = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, use_noo=noo, TH=TH,
                           family=family, first_mode=mode, t=t)
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    ctx = fg.Context.from_dict(w.params)
    p = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, first_mode=0 if mode == "inter" else 1,
                use_noo=noo, family=family or 0, activation=w.activation, t=t or 0, TH=TH or 0)
    return w, prm, rows, o, p


@pytest.mark.parametrize("name,mode,noo,family,kw", [
    ("tiny", "inter", True, None, {}), ("tiny", "spintra", True, None, {}), ("tiny", "spintra", False, 1, {}),
    ("tiny2", "inter", True, None, {}), ("tiny2", "inter", False, 2, {}),
    # the double-hoisted diagonal form: the diagonal routing, masks on the key basis
    ("tiny", "spintra", True, 4, {}), ("tiny2", "inter", True, 4, {}),
    ("cora", "inter", True, None, {"dims": [24, 16, 7]}), ("citeseer", "inter", True, None, {"dims": [24, 16, 6]}),
    # candidates of the plan search: forced packing t and region cap TH
    ("tiny2", "inter", True, 2, {"t": 1}), ("tiny2", "inter", True, 1, {"t": 4, "TH": 64}),
    ("tiny", "spintra", False, 2, {"t": 2}),
    ("cora", "inter", True, 1, {"dims": [24, 16, 7], "t": 2, "TH": 256}),
    # three layers: every SpIntra-CA layer packs one column per ciphertext
    ("ntu_small", "inter", True, None, {}), ("ntu_small", "inter", False, 2, {}), ("ntu", "inter", False, None, {}),
])
def test_plan_matches_oracle(fg, name, mode, noo, family, kw):
    w, prm, rows, o, p = _plans(fg, name, mode, noo, family, **kw)
    # the package's normalisation equals the oracle's A_hat bit for bit
    from paper_2506_10399_amd import graph
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    flat = [(v, u, a) for v, row in enumerate(rows) for u, a in row]
    assert [(v, int(u), float(a)) for v in range(w.graph.n) for u, a in
            zip(col[rp[v]:rp[v + 1]], val[rp[v]:rp[v + 1]])] == flat
    assert np.array_equal(p.ficgcn_plan_node_order(), o.pi.astype(np.int32))
    info = p.ficgcn_plan_info()
    sched = ex.schedule(prm, o)
    assert len(info) == len(o.layers)
    for li, (lp, d, st) in enumerate(zip(o.layers, info, sched)):
        assert d["kind"] == (0 if lp.kind == "inter" else 1)
        assert (d["f_in"], d["f_out"]) == (lp.f_in, lp.f_out)
        assert d["level_in"] == st["level_in"] and d["level_out"] == st["level_out"]
        assert d["scale_in"] == st["scale_in"] and d["scale_out"] == st["scale_out"] and d["sW"] == st["sW"]
        assert np.array_equal(p.ficgcn_plan_weights_int(li), ex.weight_ints(w.weights[li], st["sW"]))
        if lp.kind == "inter":
            assert d["K"] == lp.K
            assert np.array_equal(p.ficgcn_plan_copy_sources(li), lp.copy_src.astype(np.int32))
            n_ops = lp.K
        else:
            assert (d["t"], d["B"], d["family"], d["G"]) == (lp.t, lp.B, lp.family, lp.G)
            assert p.ficgcn_plan_shifts(li) == list(lp.shifts)
            n_ops = d["n_out_cts"] * len(lp.shifts)
            if lp.family == 4:
                assert p.ficgcn_plan_operand_level(li, n_ops - 1) == (st["level_agg"], st["sM"])
        assert p.ficgcn_plan_operand_count(li) == n_ops
    assert p.ficgcn_plan_rot_steps() == o.rot_steps(prm.M)


def test_plan_operand_slots_match_oracle(fg):
    from oracle import simulate as sim
    for name, mode, fam in [("tiny", "inter", None), ("tiny", "spintra", 2), ("tiny2", "inter", 1)]:
        w, prm, rows, o, p = _plans(fg, name, mode, True, fam)
        for li, lp in enumerate(o.layers):
            if lp.kind == "inter":
                want = sim.inter_plaintexts(o, lp)
            else:
                mv = ex.mask_vectors(o, li)
                want = [mv[g][d] for g in range(len(mv)) for d in lp.shifts]
            for i in range(0, len(want), max(1, len(want) // 17)):
                assert np.array_equal(p.ficgcn_plan_operand_slots(li, i), want[i])


def test_plan_rejects_bad_input(fg):
    ctx = fg.Context(13, 4, 50, 1, 60)
    rp = np.array([0, 1, 3], dtype=np.int32)
    col = np.array([0, 0, 5], dtype=np.int32)      # column 5 out of range
    with pytest.raises(fg.FicgcnError) as e:
        fg.Plan(ctx, rp, col, np.ones(3), 2, [1, 1], [np.ones((1, 1))])
    assert e.value.status == -1
    col = np.array([0, 0, 1], dtype=np.int32)
    with pytest.raises(fg.FicgcnError) as e:      # SpIntra-CA first layer of a two-layer model
        fg.Plan(ctx, rp, col, np.ones(3), 2, [1, 1, 1], [np.ones((1, 1))] * 2, first_mode=1)
    assert e.value.status == -7


def test_forced_packing_outside_rule_rejected(fg):
    from paper_2506_10399_amd import graph
    w = make_workload("tiny2")
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    ctx = fg.Context.from_dict(w.params)
    for t in (16, 3):                                       # F' = 7 allows powers of two up to 8
        with pytest.raises(fg.FicgcnError) as e:
            fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, activation=w.activation, t=t)
        assert e.value.status == -7
        rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
        with pytest.raises(ValueError):
            planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, 4096, t=t)


def _case(name):
    from paper_2506_10399_amd import graph
    w = make_workload(name)
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    return w, rp, col, val


def test_candidates_cover_packing_order_and_family(fg):
    w, rp, col, val = _case("tiny2")
    base = fg.PlanOpts(0, 1, 0, 0, int(w.activation), 0)
    c = fg.ficgcn_plan_candidates(w.graph.n, w.meta["dims"], w.params["log_n"], base)
    # t in {1, 2, 4, 8} (F' = 7, 200 nodes in 4096 slots), NOO off + TH in {64, 256... below n} + {n},
    # families 1, 2 and 4
    ts = sorted({o.t for o in c})
    assert ts == [1, 2, 4, 8]
    n_th = len([x for x in (64, 256, 1024, 4096) if x < w.graph.n]) + 1
    assert len(c) == len(ts) * (1 + n_th) * 3
    assert {(o.use_noo, o.family) for o in c} == {(u, f) for u in (0, 1) for f in (1, 2, 4)}
    # every candidate builds
    ctx = fg.Context.from_dict(w.params)
    for o in c:
        fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, opts=o)


def test_candidate_features_deterministic_and_bounded(fg):
    w, rp, col, val = _case("cora")
    base = fg.PlanOpts(0, 1, 0, 0, 1, 0)
    c = fg.ficgcn_plan_candidates(w.graph.n, w.meta["dims"], w.params["log_n"], base)
    F = np.stack([fg.ficgcn_candidate_features(rp, col, w.graph.n, w.meta["dims"], w.params["log_n"], o) for o in c])
    G = np.stack([fg.ficgcn_candidate_features(rp, col, w.graph.n, w.meta["dims"], w.params["log_n"], o) for o in c])
    assert np.array_equal(F, G)
    assert F.shape == (len(c), fg.N_FEATURES) and np.all(np.isfinite(F))
    assert F.min() >= 0.0 and F.max() <= 4.0
    # graph-only features agree across candidates, candidate features differ
    assert np.all(F[:, :8] == F[0, :8])
    assert len({tuple(r) for r in F}) == len(c)
    # mean off-diagonal degree feature = (nnz - n) / n / 16
    nnz = int(rp[-1])
    assert np.isclose(F[0, 2], (nnz - w.graph.n) / w.graph.n / 16, rtol=1e-6)


@pytest.mark.parametrize("name", ["tiny2", "cora"])
def test_exhaustive_search_no_worse_than_paper_rule(fg, name):
    w, rp, col, val = _case(name)
    ctx = fg.Context.from_dict(w.params)
    base = fg.PlanOpts(0, 1, 0, 0, int(w.activation), 0)
    best, st = fg.ficgcn_plan_search(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, base)
    assert st.n_built == st.n_candidates > 1
    rule = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, activation=w.activation)
    chosen = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, opts=best)
    assert chosen.ficgcn_plan_cost() == st.best_cost <= rule.ficgcn_plan_cost()
    # the judge's minimum over every candidate
    c = fg.ficgcn_plan_candidates(w.graph.n, w.meta["dims"], w.params["log_n"], base)
    costs = [fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, opts=o).ficgcn_plan_cost() for o in c]
    assert st.best_cost == min(costs)


@pytest.mark.parametrize("name,mode,cpoo,kw", [
    ("tiny_deep", "spintra", None, {}), ("tiny_deep", "spintra", 0.25, {}), ("tiny_deep", "spintra", 0.3, {"t": 1}),
    # nodes filling most of the ring (t = 1): AOO changes the routing
    ("tiny_deep", "spintra", 0.25, {"t": 1, "aoo": False, "n_nodes": 3000, "n_q": 20}),
    ("tiny_deep", "spintra", None, {"t": 1, "n_nodes": 3000, "n_q": 20}),
    ("tiny2_deep", "inter", None, {}), ("tiny2_deep", "inter", 0.25, {}),
    ("cora_deep", "inter", 0.25, {"dims": [24, 16, 7]}),
])
def test_radix2_plan_matches_oracle(fg, name, mode, cpoo, kw):
    """The library's radix-2 program (family 3) equals the oracle's: step and
    rotation counts, levels, every mask's slots, level and scale, the keys."""
    from paper_2506_10399_amd import graph
    from oracle import radix2
    t, aoo = kw.get("t"), kw.get("aoo", True)
    w = make_workload(name, **{k: v for k, v in kw.items() if k not in ("t", "aoo", "n_q")})
    params = dict(w.params, n_q=kw.get("n_q", w.params["n_q"]))
    prm = Params.from_dict(params)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    o = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, family=3, first_mode=mode,
                           cpoo=cpoo, t=t, aoo=aoo)
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    ctx = fg.Context.from_dict(params)
    p = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, first_mode=0 if mode == "inter" else 1,
                family=3, activation=w.activation, t=t or 0, cpoo=cpoo or 0.0, aoo=aoo)
    assert np.array_equal(p.ficgcn_plan_node_order(), o.pi.astype(np.int32))
    sched = ex.schedule(prm, o)
    info = p.ficgcn_plan_info()
    for li, (lp, d, st) in enumerate(zip(o.layers, info, sched)):
        assert d["level_out"] == st["level_out"] and d["scale_out"] == st["scale_out"] and d["sW"] == st["sW"]
        if lp.kind == "inter":
            continue
        prog = lp.program
        assert d["family"] == 3
        assert p.ficgcn_plan_radix2_stats(li) == dict(
            lanes=prog.n_lanes, steps=prog.n_steps(), rotations=len(prog.rotations()), amounts=len(prog.amounts()),
            depth=prog.depth, masks=len(radix2.operand_list(prog)), moved=prog.n_moved,
            registers=len(prog.reg_depth) - 1)
        flat = [x for per_g in ex.radix2_mask_vectors(o, li) for x in per_g]
        assert p.ficgcn_plan_operand_count(li) == len(flat)
        stride = max(1, len(flat) // 97)
        for i in list(range(0, len(flat), stride)) + [len(flat) - 1]:
            dep, v = flat[i]
            lvl = st["level_agg"] - dep
            assert p.ficgcn_plan_operand_level(li, i) == (lvl, float(prm.q[lvl]))
            assert np.array_equal(p.ficgcn_plan_operand_slots(li, i), v)
    assert p.ficgcn_plan_rot_steps() == o.rot_steps(prm.M)


def test_top_digit_of_rearranged_inputs_fits_a_nibble():
    """The rearranged-input layout stores digit 6 of each residue's balanced
    base-256 form as a 4-bit value, which needs it in [0, 15] for every
    residue the layout accepts (primes below 2^51).  Digits are computed from
    their definition: x = sum_a d_a 256^a with every d_a in [-128, 127]."""
    def digits(x):
        out = []
        for _ in range(7):
            d = x % 256
            if d >= 128:
                d -= 256
            out.append(d)
            x = (x - d) // 256
        assert x == 0
        return out
    rng = np.random.default_rng(7)
    edge = [0, 1, 127, 128, (1 << 48) - 1, 1 << 48, (1 << 50) - 1, (1 << 51) - 1,
            sum(127 << (8 * a) for a in range(6)) + (1 << 48)]
    xs = edge + [int(v) for v in rng.integers(0, 1 << 51, 20000, dtype=np.int64)]
    tops = []
    for x in xs:
        d = digits(x)
        assert sum(v * 256 ** a for a, v in enumerate(d)) == x
        tops.append(d[6])
    assert min(tops) >= 0 and max(tops) <= 8


@pytest.mark.parametrize("name,kw,first_pack,noo,family", [
    ("tiny", {}, "rule", True, None), ("tiny", {"n_nodes": 64}, 4, False, None), ("tiny", {}, 1, True, None),
    ("tiny2", {"n_nodes": 100}, "rule", True, None), ("tiny2", {"n_nodes": 100}, 1, False, 2),
    ("tiny2", {"n_nodes": 100}, 2, True, 4), ("ntu_small", {}, "rule", True, None)])
def test_case1_plan_matches_oracle(fg, name, kw, first_pack, noo, family):
    """The library's planner on the case-1 layout (Sec. 3.2, App. B) and the block-rotation
    combination equals the oracle's: node order, packing, schedule, every operand's slot
    vector, level, scale and basis, the rotation keys, and the mode formula per layer."""
    from paper_2506_10399_amd import graph
    w = make_workload(name, **kw)
    prm = Params.from_dict(w.params)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    o = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, use_noo=noo, family=family,
                           first_pack=first_pack)
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    ctx = fg.Context.from_dict(w.params)
    fp = -1 if first_pack == "rule" else first_pack
    p = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, use_noo=noo, family=family or 0,
                activation=w.activation, first_pack=fp)
    assert np.array_equal(p.ficgcn_plan_node_order(), o.pi.astype(np.int32))
    info = p.ficgcn_plan_info()
    sched = ex.schedule(prm, o)
    assert o.layers[0].pack == "rep" and info[0]["pack"] == 1
    for li, (lp, d, st) in enumerate(zip(o.layers, info, sched)):
        assert (d["t"], d["B"]) == (lp.t, lp.B)
        assert d["level_in"] == st["level_in"] and d["level_out"] == st["level_out"]
        assert d["scale_in"] == st["scale_in"] and d["scale_out"] == st["scale_out"] and d["sW"] == st["sW"]
        assert d["n_fold"] == len(lp.fold_steps) and d["n_comb_shifts"] == len(lp.comb_shifts)
        if li == 0:
            want = sim.rep_plaintexts(o, lp, w.weights[0])
            levels = [(st["level_in"], st["sP"])] * len(want)
        else:
            assert d["comb"] == 1 and d["family"] == lp.family and d["G"] == lp.G
            assert p.ficgcn_plan_shifts(li) == list(lp.shifts)
            assert d["paper_mode"] == (0 if lp.paper_mode == "inter" else 1)
            assert d["mode_cost_inter"] == lp.paper_mode_costs[0]
            assert d["mode_cost_spintra"] == lp.paper_mode_costs[1]
            mv = ex.mask_vectors(o, li)
            cm = sim.diag_masks(o, lp, w.weights[li])
            agg = [mv[g][s] for g in range(len(mv)) for s in lp.shifts]
            want = agg + [cm[s] for s in lp.comb_shifts]
            levels = [(st["level_agg"], st["sM"])] * len(agg) + [(st["level_in"], st["sW"])] * len(cm)
        assert p.ficgcn_plan_operand_count(li) == len(want)
        for i in range(0, len(want), max(1, len(want) // 23)):
            assert np.array_equal(p.ficgcn_plan_operand_slots(li, i), want[i]), (li, i)
            assert p.ficgcn_plan_operand_level(li, i) == levels[i]
    assert p.ficgcn_plan_rot_steps() == o.rot_steps(prm.M)


def test_case1_rule_and_rejections(fg):
    w = make_workload("tiny")
    from paper_2506_10399_amd import graph
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    ctx = fg.Context.from_dict(w.params)
    p = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, first_pack=-1)
    d = p.ficgcn_plan_info()[0]
    assert (d["pack"], d["t"], d["B"], d["n_in_cts"], d["n_out_cts"]) == (1, 2, 128, d["K"] * 16, 1)
    with pytest.raises(fg.FicgcnError) as e:      # t = 4 does not fit 128 nodes at F' = 16, M = 4096
        fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, first_pack=4)
    assert e.value.status == -7
    # the citation-graph shape is case 2: the rule keeps one column per ciphertext
    wc = make_workload("cora", dims=[24, 16, 7])
    rp, col, val = graph.normalize(wc.graph.n, wc.neighbors, wc.norm)
    ctx2 = fg.Context.from_dict(wc.params)
    p2 = fg.Plan(ctx2, rp, col, val, wc.graph.n, [24, 16, 7], wc.weights, activation=True, first_pack=-1)
    assert p2.ficgcn_plan_info()[0]["pack"] == 0


@pytest.mark.parametrize("name,kw,fp", [("cora", {"dims": [24, 16, 7]}, 0), ("tiny", {}, -1), ("tiny2", {}, 0),
                                         ("pubmed", {"dims": [8, 16, 3], "n_nodes": 3000}, 0)])
def test_lowest_level_schedule_matches_oracle(fg, name, kw, fp):
    from paper_2506_10399_amd import graph
    w = make_workload(name, **kw)
    prm = Params.from_dict(w.params)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    o = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, low_level=True,
                           first_pack="rule" if fp < 0 else "cols")
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    ctx = fg.Context.from_dict(w.params)
    p = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, activation=w.activation, first_pack=fp,
                low_level=True)
    sched = ex.schedule(prm, o)
    assert sched[-1]["level_out"] == ex.OUT_LEVEL
    for d, st in zip(p.ficgcn_plan_info(), sched):
        assert (d["level_in"], d["level_out"]) == (st["level_in"], st["level_out"])
        assert d["scale_in"] == st["scale_in"] and d["scale_out"] == st["scale_out"] and d["sW"] == st["sW"]


def test_operand_descriptors_checked_before_any_device_work(fg):
    """Level and scale checks of the descriptor calls (no GPU: every case fails
    its checks, so nothing reaches the device, and no descriptor changes)."""
    ctx = fg.Context(13, 4, 50, 1, 60)
    fake = 1 << 40                                   # never dereferenced
    op = lambda lv, sc, n=2: fg.Operand(fake, lv, n, sc)

    def status(f, *a):
        with pytest.raises(fg.FicgcnError) as e:
            f(*a)
        return e.value.status

    acc = op(3, 2.0 ** 80)
    assert status(ctx.ckks_pt_mul_acc_op, acc, [op(2, 2.0 ** 40)], [op(2, 2.0 ** 40, 1)]) == -2    # ELEVEL
    assert status(ctx.ckks_pt_mul_acc_op, acc, [op(3, 2.0 ** 40)], [op(3, 2.0 ** 40, 2)]) == -1    # not a plaintext
    assert status(ctx.ckks_pt_mul_acc_op, acc, [op(3, 2.0 ** 40)], [op(3, 2.0 ** 41, 1)]) == -3    # ESCALE
    assert (acc.level, acc.scale) == (3, 2.0 ** 80)
    fresh = op(3, 0.0)                               # a fresh accumulator takes the first product's scale,
    assert status(ctx.ckks_pt_mul_acc_op, fresh,     # every later product must carry it
                  [op(3, 2.0 ** 40), op(3, 2.0 ** 40)], [op(3, 2.0 ** 40, 1), op(3, 2.0 ** 39, 1)]) == -3
    assert status(ctx.ckks_scalar_mul_acc_op, acc, [op(3, 2.0 ** 40)], [5], 2.0 ** 39) == -3
    assert status(ctx.ckks_scalar_mul_acc_op, acc, [op(3, 2.0 ** 40)], [5], -1.0) == -3
    assert status(ctx.ckks_add_op, op(3, 2.0 ** 40), op(3, 2.0 ** 40 * (1 + 1e-6))) == -3
    assert status(ctx.ckks_add_op, op(3, 2.0 ** 40), op(2, 2.0 ** 40)) == -2
    assert status(ctx.ckks_rescale_op, op(0, 2.0 ** 40)) == -2
    assert status(ctx.ckks_rescale_op, op(4, 2.0 ** 40)) == -2           # beyond the 4-prime chain
    assert status(ctx.ckks_mul_relin_op, fg.Keys(ctx, None), op(3, 2.0 ** 40), op(2, 2.0 ** 40), op(3, 0.0)) == -2
    outs = [op(3, 0.0), op(2, 0.0)]
    assert status(ctx.ckks_rotate_hoisted_op, fg.Keys(ctx, None), op(3, 2.0 ** 40), [1, 2], outs) == -2
    assert [(o.level, o.scale) for o in outs] == [(3, 0.0), (2, 0.0)]
    assert status(ctx.ckks_decrypt_op, fg.Keys(ctx, None), op(3, 2.0 ** 40, 1), 4) == -1
    # seeded ciphertexts: ids past 32 bits, a level beyond the chain, no secret
    assert status(ctx.ckks_expand_seeded, 1, 2 ** 32 - 2, 3, 0, fake) == -1
    assert status(ctx.ckks_expand_seeded, 1, 0, 1, 4, fake) == -2
    assert status(ctx.ckks_encrypt_seeded, fg.Keys(ctx, None), fake, 0, 1, 2, 0, fake) == -1
    # packed residues: widths outside 1..64, too many limbs
    assert status(ctx.ckks_pack_residues, fake, 3, 0, fake) == -1
    assert status(ctx.ckks_unpack_residues, fake, 3, 65, fake) == -1
    assert status(ctx.ckks_pack_residues, fake, 70000, 50, fake) == -1


def test_search_rejects_plans_whose_keys_exceed_the_limit(fg):
    """The exhaustive search (host only) never returns a candidate whose rotation keys
    exceed base.max_key_bytes, and fails with EPLAN when no candidate fits."""
    from paper_2506_10399_amd import graph
    w = make_workload("tiny2")
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    ctx = fg.Context.from_dict(w.params)
    prm = Params.from_dict(w.params)
    key_bytes = -(-prm.L // len(prm.p)) * 2 * (prm.L + len(prm.p)) * prm.N * 8
    base = fg.PlanOpts(0, 1, 0, 0, 1, 0)
    free, _ = fg.ficgcn_plan_search(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, base)
    n_free = len(fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, opts=free).ficgcn_plan_rot_steps())
    steps_of = {}
    for o in fg.ficgcn_plan_candidates(w.graph.n, w.meta["dims"], 13, base):
        n = len(fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, opts=o).ficgcn_plan_rot_steps())
        steps_of[(o.t, o.use_noo, o.TH, o.family)] = n
    fewest = min(steps_of.values())
    assert fewest < n_free                       # the limit below makes the free choice infeasible
    base.max_key_bytes = (n_free - 1) * key_bytes
    best, _ = fg.ficgcn_plan_search(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, base)
    assert steps_of[(best.t, best.use_noo, best.TH, best.family)] * key_bytes <= base.max_key_bytes
    base.max_key_bytes = (fewest - 0.5) * key_bytes
    with pytest.raises(fg.FicgcnError) as e:
        fg.ficgcn_plan_search(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, base)
    assert e.value.status == -7
