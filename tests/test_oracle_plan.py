"""Pins of the oracle's planner, slot simulator and encrypted executor: the
paper's cost formulas at hand-computed values, structural invariants of the
node-order optimisation, brute force over small placements, and the FP64 GCN."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import gcn, planner, simulate as sim, execute as ex, ckks
from oracle.params import Params
from workload import make_workload, Graph

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name, **kw):
    w = make_workload(name, **kw)
    return w, gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)


def test_j_objective_hand_values():
    with open(os.path.join(GOLD, "j_objective_cfg_tiny.txt")) as f:
        pairs = [tuple(map(int, l.split())) for l in f if l.strip() and not l.startswith("#")]
    for t, j in pairs:
        assert planner.j_objective(t, 32, 4) == j
    # feasible argmin for the tiny configuration (t N F' <= M: t <= 2)
    assert planner.paper_packing_t(32, 4, 128, 16, 4096) == 2
    # citation-graph shape: M <= N F' -> t = 1 (Sec. 3.2 case 2)
    assert planner.paper_packing_t(1433, 4, 2708, 16, 32768) == 1


def test_packing_ciphertext_counts_match_printed_table():
    with open(os.path.join(GOLD, "packing_ciphertext_counts.txt")) as f:
        rows = [list(map(int, l.split())) for l in f if l.strip() and not l.startswith("#")]
    for t, *counts in rows:
        assert [planner.ceil_div(F, t) for F in (1433, 32, 16)] == counts


def test_case2_count_and_mode_rule():
    # ceil(Fn/t) * ceil(N F' / ceil(M/t)) at t = 1 for the citation-graph shape
    assert planner.case2_pmults(1, 1433, 4, 2708, 16, 32768) == 1433 * 4 * 2
    # Inter-CA: 2 ceil(F n / t) vs SpIntra-CA: 10 c n log^2 N
    assert planner.paper_agg_mode(16, 4, 1, 2708, 0.01) == "spintra"
    assert planner.paper_agg_mode(16, 4, 1, 2708, 1.0) == "inter"
    assert planner.spintra_worst_case_rots(4, 1024) == 3 * 100


def test_sibling_definition():
    rows = [[(0, 1.0), (1, 1.0)], [(1, 1.0), (2, 1.0)], [(2, 1.0)], [(3, 1.0), (2, 1.0)]]
    sib = planner.siblings(rows)
    assert sib[0] == [1] and sib[1] == [0, 2] and sib[2] == [1, 3] and sib[3] == [2]


def test_noo_structure_invariants():
    w, rows = _rows("cora", n_nodes=600, dims=[8, 4, 3])
    B = 1024
    for TH in (64, 200, 1024):
        regions = planner.noo_regions(rows, TH)
        assert sorted(v for r in regions for v in r) == list(range(600))
        assert all(len(r) <= TH for r in regions)
        assert all(len(r) == TH for r in regions[:-1])
        slots = planner.interleave_slots([len(r) for r in regions], B)
        flat = sorted(s for sl in slots for s in sl)
        assert len(set(flat)) == 600 and flat[-1] < B
        pi = planner.noo_place(rows, regions, slots, 32768, wrap=False)
        assert len(set(pi.tolist())) == 600 and pi.min() >= 0 and pi.max() < B
        # every node sits on one of its region's interleaved slots
        for r, sl in zip(regions, slots):
            assert sorted(pi[r].tolist()) == sorted(sl)
    # the region's first node is the highest-degree node left
    deg = [len(s) for s in planner.support(rows)]
    regions = planner.noo_regions(rows, 200)
    assert deg[regions[0][0]] == max(deg)


def test_interleave_round_robin_with_blanks():
    assert planner.interleave_slots([2, 2, 1], 6) == [[0, 3], [1, 4], [2]]
    # region 2 exhausted after one round: its turn takes the blank (slot 5)
    assert planner.interleave_slots([3, 3, 1], 8) == [[0, 3, 6], [1, 4, 7], [2]]
    # blanks exhausted: exhausted region skipped
    assert planner.interleave_slots([3, 3, 1], 7) == [[0, 3, 5], [1, 4, 6], [2]]


def test_greedy_step_is_argmin_by_brute_force():
    """Each greedy placement equals the brute-force argmin of its objective
    (number of new distinct shifts, lowest slot on ties)."""
    w, rows = _rows("tiny", n_nodes=8, dims=[4, 2])
    regions = planner.noo_regions(rows, 8)
    slots = planner.interleave_slots([len(r) for r in regions], 8)
    pi = planner.noo_place(rows, regions, slots, 4096, wrap=False)
    placed = {}
    shifts = set()
    order = regions[0]
    for idx, x in enumerate(order):
        free = [s for s in slots[0] if s not in placed.values()]
        if idx == 0:
            best = free[0]
        else:
            def cost(pos):
                new = set()
                for u, _ in rows[x]:
                    if u != x and u in placed:
                        new.add(placed[u] - pos)
                for v, row in enumerate(rows):
                    if v != x and v in placed and any(u == x for u, _ in row):
                        new.add(pos - placed[v])
                return len(new - shifts)
            best = min(free, key=lambda p: (cost(p), p))
        assert pi[x] == best
        placed[x] = best
        for u, _ in rows[x]:
            if u != x and u in placed:
                shifts.add(placed[u] - best)
        for v, row in enumerate(rows):
            if v != x and v in placed and any(u == x for u, _ in row):
                shifts.add(best - placed[v])


def _walk(s, d, M):
    """Cells of a radix-2 demand, simulated round by round: in round r the value
    moves by sign(d) 2^r if bit r of |d| is set; while distance remains after the
    round it occupies (r, slot)."""
    cells, cur, mag, sg = [], s, abs(d), (1 if d > 0 else -1)
    r = 0
    while mag >> r:
        if (mag >> r) & 1:
            cur = (cur - sg * (1 << r)) % M
        if mag >> (r + 1):
            cells.append((r, cur))
        r += 1
    return cells


@pytest.mark.parametrize("seed,n,B,M", [(1, 8, 8, 8), (2, 8, 16, 16), (3, 7, 8, 64), (4, 8, 32, 32),
                                        (5, 6, 16, 128), (6, 8, 16, 16)])
def test_conflict_objective_greedy_is_argmin_by_brute_force(seed, n, B, M):
    """Stage 3 with the radix-2 objective: each placement is the brute-force
    argmin (lowest slot on ties) of the number of (round, slot) cells where the
    node's demands with placed nodes meet a placed demand of another source,
    every demand's cells simulated round by round from its bits."""
    rng = np.random.default_rng(seed)
    adj = [set() for _ in range(n)]
    for _ in range(2 * n):
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    rows = [[(v, 1.0)] + [(u, 1.0) for u in sorted(adj[v])] for v in range(n)]
    wrap = B == M
    red = lambda d: planner.reduce_shift(d, M, wrap)
    regions = planner.noo_regions(rows, n)
    slots = planner.interleave_slots([len(r) for r in regions], B)
    pi = planner.noo_place(rows, regions, slots, M, wrap, objective="conflicts")
    placed = {}
    occupied = {}                                    # (round, slot) -> sources

    def demands_of(x, pos):
        out = []
        for u, _ in rows[x]:
            if u != x and u in placed:
                out.append((u, placed[u], red(placed[u] - pos)))
        for v, row in enumerate(rows):
            if v != x and v in placed and any(u == x for u, _ in row):
                out.append((x, pos, red(pos - placed[v])))
        return out

    for idx, x in enumerate(regions[0]):
        free = [s_ for s_ in slots[0] if s_ not in placed.values()]
        if idx == 0:
            best = free[0]
        else:
            def cost(pos):
                return sum(1 for src, s_, d in demands_of(x, pos) for c in _walk(s_, d, M)
                           if occupied.get(c, set()) - {src})
            best = min(free, key=lambda p_: (cost(p_), p_))
        assert pi[x] == best, (seed, x)
        for src, s_, d in demands_of(x, best):
            for c in _walk(s_, d, M):
                occupied.setdefault(c, set()).add(src)
        placed[x] = best
    assert planner.demand_cells(5, 6, 16) == _walk(5, 6, 16) == [(0, 5), (1, 3)]


def test_conflict_objective_differs_from_shift_objective():
    """On the small two-layer shape the radix-2 objective places nodes differently
    from the distinct-shift objective, and the radix-2 program built on its order
    needs no more working ciphertexts."""
    from oracle import radix2
    w, rows = _rows("tiny2")
    regions = planner.noo_regions(rows, 1024)
    slots = planner.interleave_slots([len(r) for r in regions], 512)
    a = planner.noo_place(rows, regions, slots, 4096, False, objective="shifts")
    b = planner.noo_place(rows, regions, slots, 4096, False, objective="conflicts")
    assert not np.array_equal(a, b)
    lanes = [radix2.build_program(pi, rows, 4096, 512, False, None).n_lanes for pi in (a, b)]
    assert lanes[1] <= lanes[0], lanes           # 8 -> 7 working ciphertexts on this shape
    o_a = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, 4096, family=3)
    assert o_a.layers[1].family == 3
    assert np.array_equal(o_a.pi, planner.noo(rows, o_a.layers[1].B, 4096, 1024, "conflicts")[0])


def test_circulant_graph_routes_with_one_rotation():
    """A directed cycle v -> v+1 (identity order, one column): the only shifts
    are 0 and +1, i.e. one rotation (diagonal form)."""
    n = 64
    rows = [[(v, 0.5), ((v + 1) % n, 0.5)] for v in range(n)]
    plan = planner.build_plan(n, rows, [1, 1], False, 64, use_noo=False, family=1, first_mode="spintra")
    lp = plan.layers[0]
    assert lp.t == 1 and lp.B == 64
    # the wrap-around demand (n-1 -> 0) reduces to +1 with AOO
    assert lp.shifts == [0, 1] and planner.rotation_steps_of(lp) == [1]


def test_aoo_reduces_to_shortest_direction():
    assert planner.reduce_shift(4095, 4096, True) == -1
    assert planner.reduce_shift(2048, 4096, True) == 2048
    assert planner.reduce_shift(-2049, 4096, True) == 2047
    assert planner.reduce_shift(4095, 4096, False) == 4095


def test_bsgs_split_covers_every_shift():
    shifts = [-300, -17, 0, 3, 64, 65, 129, 511]
    G, c = planner.bsgs_split(shifts, 512)
    babies = {d % G for d in shifts}
    giants = {d // G for d in shifts}
    for d in shifts:
        assert (d // G) * G + d % G == d
    assert c == len(babies - {0}) + len(giants - {0})


@pytest.mark.parametrize("name,mode,noo,fam", [
    ("tiny", "inter", True, None), ("tiny", "spintra", True, 1), ("tiny", "spintra", False, 2),
    ("tiny", "spintra", True, 4), ("tiny2", "inter", True, 1), ("tiny2", "inter", False, 2)])
def test_slot_simulator_equals_fp64_gcn(name, mode, noo, fam):
    w, rows = _rows(name)
    ref = gcn.gcn_forward(rows, w.x, w.weights, w.activation)[-1]
    M = 2 ** (w.params["log_n"] - 1)
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, M, use_noo=noo,
                              family=fam, first_mode=mode)
    counts = dict(rot=0, pmult=0, smult=0, cmult=0)
    out = sim.run(plan, w.x, w.weights, counts)
    assert gcn.max_rel_error(out, ref) < 1e-12
    oc = planner.op_counts(plan)
    assert oc["rot"] == counts["rot"] and oc["pmult"] == counts["pmult"]
    assert oc["smult"] == counts["smult"] and oc["cmult"] == counts["cmult"]
    if mode == "inter":
        lp = plan.layers[0]
        # Inter-CA: PMult = Add = K F with K = n + 1 copies (Sec. 3.2, Table 1), no rotation
        assert oc["pmult"] >= lp.K * lp.f_in
        assert planner.op_counts(planner.Plan(plan.n_v, M, plan.B_pi, plan.pi, rows, [lp]))["rot"] == 0


def test_spintra_first_layer_of_deep_model_rejected():
    w, rows = _rows("tiny2")
    with pytest.raises(ValueError):
        planner.build_plan(w.graph.n, rows, w.meta["dims"], True, 4096, first_mode="spintra")


def test_mask_nonzeros_equal_adjacency_nonzeros():
    w, rows = _rows("tiny2")
    M = 2 ** (w.params["log_n"] - 1)
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, M)
    lp = plan.layers[1]
    mk = sim.masks(plan, lp, lp.f_out)
    nnz = sum(len(r) for r in rows)
    assert sum(int(np.count_nonzero(v)) for v in mk.values()) == nnz * lp.f_out


def test_gcn_normalisations():
    n = 4
    nb = [np.array([1]), np.array([0, 2]), np.array([1]), np.array([], dtype=np.int64)]
    rows = gcn.normalized_rows(n, nb, "sym")
    a = gcn.dense_adjacency(n, rows)
    A = np.array([[0, 1, 0, 0], [1, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 0]], float) + np.eye(4)
    d = A.sum(1)
    assert np.allclose(a, A / np.sqrt(np.outer(d, d)))
    rows = gcn.normalized_rows(n, nb, "mean")
    a = gcn.dense_adjacency(n, rows)
    assert np.allclose(a.sum(1), 1.0) and a[1, 0] == pytest.approx(1 / 3)


@pytest.mark.slow
@pytest.mark.parametrize("name,mode,fam", [("tiny", "inter", None), ("tiny", "spintra", None), ("tiny", "spintra", 2),
                                           ("tiny", "spintra", 4), ("tiny2", "inter", None)])
def test_encrypted_plan_decrypts_to_fp64_gcn(name, mode, fam):
    w, rows = _rows(name)
    prm = Params.from_dict(w.params)
    ref = gcn.gcn_forward(rows, w.x, w.weights, w.activation)[-1]
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, first_mode=mode, family=fam)
    keys = ckks.keygen(prm, 11, plan.rot_steps(prm.M), relin=w.activation)
    sched = ex.schedule(prm, plan)
    ops = ex.encode_operands(prm, plan, w.weights, sched)
    cts = ex.client_encrypt(prm, plan, w.x, keys, 12)
    outs = ex.run(prm, plan, keys, cts, ops, sched)
    y = ex.decrypt_output(prm, plan, keys, outs[-1])
    assert gcn.max_rel_error(y, ref) < 1e-3


def _hand_regions_fixture():
    with open(os.path.join(GOLD, "noo_regions_hand.txt")) as f:
        lines = [l.strip() for l in f if l.strip() and not l.startswith("#")]
    edges = [tuple(map(int, e.split("-"))) for e in lines[0].split()[1:]]
    n = int(lines[1].split()[1])
    cases = []
    for l in lines[2:]:
        head, body = l.split(":")
        cases.append((int(head.split()[1]), [list(map(int, r.split())) for r in body.split("|")]))
    return n, edges, cases


def test_noo_regions_hand_worked_example():
    """Alg. 1 stage 1 against regions worked out by hand (tests/golden): sibling BFS
    from the highest-degree node, ascending enqueue, restart inside the region when
    the BFS runs dry."""
    n, edges, cases = _hand_regions_fixture()
    adj = [set([v]) for v in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    rows = [[(u, 1.0) for u in sorted(adj[v])] for v in range(n)]
    for TH, want in cases:
        assert planner.noo_regions(rows, TH) == want, TH


def test_rule_packing_picks_the_papers_t():
    """App. B's rule on the case-1 layout: the tiny configuration (F 32, F' 16, 128 nodes,
    M 4096) packs t = 2; the citation-graph shapes and the clustered shape are case 2
    (M <= N F'), one column per ciphertext."""
    assert planner.rule_packing(32, 4, 128, 16, 4096) == ("rep", 2)
    assert planner.rep_block(2, 16, 128, 4096) == 128
    assert planner.rep_block(4, 16, 128, 4096) is None
    assert planner.rule_packing(1433, 4, 2708, 16, 32768) == ("cols", 1)
    assert planner.rule_packing(3703, 3, 3327, 16, 32768) == ("cols", 1)
    assert planner.rule_packing(500, 5, 19717, 16, 32768) == ("cols", 1)
    # a later layer wider than the packed capacity M / Bc (32 at t = 2, 16 at t = 1) falls
    # back to smaller t, then to one column per ciphertext
    assert planner.rule_packing(32, 4, 64, 16, 4096, later_widths=[40]) == ("rep", 4)
    assert planner.rule_packing(32, 4, 128, 16, 4096, later_widths=[20]) == ("rep", 2)
    assert planner.rule_packing(32, 4, 128, 16, 4096, later_widths=[40]) == ("cols", 1)
    w, rows = _rows("tiny")
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], False, 4096, first_pack="rule")
    assert plan.layers[0].pack == "rep" and plan.layers[0].t == 2 and plan.B_pi == 128


@pytest.mark.parametrize("n_nodes,t", [(128, 1), (128, 2), (64, 4)])
def test_case1_counts_equal_the_papers_formulas(n_nodes, t):
    """Sec. 3.2 case 1 / App. B: PMult = Add = ceil(F n / t) (n counted as the K = n + 1
    copies the layer reads) and ceil(log2 t) rotations, as equalities; the simulator
    performs exactly those operations and equals the FP64 GCN."""
    w, rows = _rows("tiny", n_nodes=n_nodes)
    F, Fo = w.meta["dims"]
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], False, 4096, first_pack=t)
    lp = plan.layers[0]
    oc = planner.op_counts(plan)
    assert oc["pmult"] == lp.K * math.ceil(F / t) and oc["add"] == lp.K * math.ceil(F / t)
    assert oc["rot"] == math.ceil(math.log2(t)) if t > 1 else oc["rot"] == 0
    assert oc["smult"] == 0 and oc["rescale"] == 1
    counts = dict(rot=0, pmult=0, smult=0, cmult=0)
    out = sim.run(plan, w.x, w.weights, counts)
    ref = gcn.gcn_forward(rows, w.x, w.weights, False)[-1]
    assert gcn.max_rel_error(out, ref) < 1e-12
    assert counts["pmult"] == oc["pmult"] and counts["rot"] == oc["rot"]


@pytest.mark.parametrize("name,kw,t,noo", [("tiny2", dict(n_nodes=100), 2, True), ("tiny2", dict(n_nodes=100), 1, False),
                                           ("ntu_small", {}, "rule", True)])
def test_case1_layout_deeper_models_equal_fp64(name, kw, t, noo):
    """Later layers on the packed blocks (block-rotation combination, then SpIntra-CA):
    the slot simulator equals the FP64 GCN and its operation counts equal op_counts."""
    w, rows = _rows(name, **kw)
    M = 2 ** (w.params["log_n"] - 1)
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, M, use_noo=noo, first_pack=t)
    assert plan.layers[0].pack == "rep" and all(lp.comb == "diag" for lp in plan.layers[1:])
    counts = dict(rot=0, pmult=0, smult=0, cmult=0)
    out = sim.run(plan, w.x, w.weights, counts)
    ref = gcn.gcn_forward(rows, w.x, w.weights, w.activation)[-1]
    assert gcn.max_rel_error(out, ref) < 1e-12
    oc = planner.op_counts(plan)
    assert all(oc[k] == counts[k] for k in counts)
    # the block combination's offsets span every (input block, output block) pair once
    lp = plan.layers[1]
    assert lp.comb_shifts == list(range(-(lp.f_out - 1), lp.f_in))


def test_aggregation_mode_formula_recorded_per_layer():
    """Sec. 3.3.2's argmin for later layers: Inter-CA 2 ceil(F n / t) against SpIntra-CA
    10 c n log2(N)^2; at the citation-graph shape's second layer (F 16, n 4, t 1, 2708
    nodes) Inter-CA wins unless c < 128 / 5201."""
    w, rows = _rows("cora", n_nodes=2708, dims=[8, 16, 7])
    for c, want in ((1.0, "inter"), (0.01, "spintra")):
        plan = planner.build_plan(w.graph.n, rows, [8, 16, 7], True, 32768, use_noo=False, agg_c=c)
        lp = plan.layers[1]
        n = plan.layers[0].K - 1
        assert lp.paper_mode == want
        assert lp.paper_mode_costs[0] == 2 * math.ceil(16 * n / 1)
        assert lp.paper_mode_costs[1] == pytest.approx(10 * c * n * math.log2(2708) ** 2)


@pytest.mark.slow
@pytest.mark.parametrize("name,kw", [("tiny", {}), ("tiny2", dict(n_nodes=100))])
def test_case1_encrypted_plan_decrypts_to_fp64_gcn(name, kw):
    w, rows = _rows(name, **kw)
    prm = Params.from_dict(w.params)
    ref = gcn.gcn_forward(rows, w.x, w.weights, w.activation)[-1]
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, first_pack="rule")
    assert plan.layers[0].pack == "rep" and plan.layers[0].t == 2
    keys = ckks.keygen(prm, 11, plan.rot_steps(prm.M), relin=w.activation)
    sched = ex.schedule(prm, plan)
    ops = ex.encode_operands(prm, plan, w.weights, sched)
    cts = ex.client_encrypt(prm, plan, w.x, keys, 12)
    outs = ex.run(prm, plan, keys, cts, ops, sched)
    y = ex.decrypt_output(prm, plan, keys, outs[-1])
    assert gcn.max_rel_error(y, ref) < 1e-3


def test_lowest_level_schedule():
    """With low_level the client encrypts at the level the layers consume plus the output's
    one spare prime: citation shape 2 (Inter-CA) + 2 + 1 (SpIntra-CA after x^2) = 5 -> level 6;
    tiny case-1 one-layer plan 1 -> level 2; the schedule then ends at level 1 exactly."""
    w, rows = _rows("cora", n_nodes=600, dims=[8, 16, 7])
    for L, lv0 in ((8, 6), (10, 6)):
        prm = Params.from_dict(dict(w.params, n_q=L))
        plan = planner.build_plan(w.graph.n, rows, [8, 16, 7], True, prm.M, low_level=True)
        sched = ex.schedule(prm, plan)
        assert ex.levels_needed(plan) == 5
        assert sched[0]["level_in"] == lv0 and sched[-1]["level_out"] == ex.OUT_LEVEL
        top = ex.schedule(prm, planner.build_plan(w.graph.n, rows, [8, 16, 7], True, prm.M))
        assert top[0]["level_in"] == L - 1 and top[-1]["level_out"] == L - 1 - 5
    w, rows = _rows("tiny")
    prm = Params.from_dict(w.params)
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], False, prm.M, first_pack="rule", low_level=True)
    assert ex.schedule(prm, plan)[0]["level_in"] == 2


@pytest.mark.slow
def test_lowest_level_encrypted_plan_decrypts_to_fp64_gcn():
    w, rows = _rows("tiny2")
    prm = Params.from_dict(w.params)
    ref = gcn.gcn_forward(rows, w.x, w.weights, w.activation)[-1]
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, low_level=True)
    sched = ex.schedule(prm, plan)
    assert sched[0]["level_in"] == 6 and sched[-1]["level_out"] == 1
    keys = ckks.keygen(prm, 11, plan.rot_steps(prm.M), relin=w.activation)
    ops = ex.encode_operands(prm, plan, w.weights, sched)
    cts = ex.client_encrypt(prm, plan, w.x, keys, 12)
    assert cts[0].level == 6
    outs = ex.run(prm, plan, keys, cts, ops, sched)
    y = ex.decrypt_output(prm, plan, keys, outs[-1])
    assert gcn.max_rel_error(y, ref) < 1e-3
