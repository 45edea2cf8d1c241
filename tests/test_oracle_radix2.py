"""Pins of the radix-2 SpIntra-CA program (Sec. 3.3 and the CPOO/AOO
optimisations of Sec. 3.3.1) in the oracle.

* The program's whole linear map, probed slot by slot with unit vectors,
  equals the block-diagonal adjacency A_hat in the node order, exactly
  (every output value is one demand's coefficient times its source value,
  so no rounding enters): a wrong sign, bit, slot or a doubled write fails.
* Special cases with closed forms: a circulant graph with offset delta takes
  popcount(|delta|) rotations and levels in one lane; a cycle takes the two
  rotations +-1 in one level; AOO turns the wrap-around demand of a ring
  into a shift of one.
* The rotation count stays under the paper's worst case (n - 1) log^2 N.
"""
import numpy as np
import pytest

from oracle import gcn, planner, radix2
from oracle.params import Params
from workload import make_workload


def _program_matrix(prog, M, B, n_cols):
    cols = []
    for j in range(M):
        e = np.zeros(M)
        e[j] = 1.0
        cols.append(radix2.run_slots(prog, e, B, n_cols))
    return np.stack(cols, axis=1)


def _expected_matrix(pi, rows, M, B, n_cols):
    E = np.zeros((M, M))
    for v, row in enumerate(rows):
        for u, a in row:
            for c in range(n_cols):
                E[c * B + pi[v], (c * B + pi[u]) % M] += a
    return E


def _random_rows(n, deg, seed):
    rng = np.random.default_rng(seed)
    adj = [set() for _ in range(n)]
    for _ in range(n * deg // 2):
        a, b = rng.integers(n, size=2)
        if a != b:
            adj[a].add(int(b))
            adj[b].add(int(a))
    rows = []
    for v in range(n):
        us = sorted(adj[v] | {v})
        w = rng.uniform(0.1, 1.0, len(us))
        rows.append([(u, float(x)) for u, x in zip(us, w)])
    return rows


@pytest.mark.parametrize("theta", [None, 0.25, 0.5])
@pytest.mark.parametrize("M,B,n_cols,noo", [(64, 64, 1, False), (64, 64, 1, True), (256, 64, 4, True),
                                            (256, 64, 3, False)])
def test_program_map_equals_adjacency_exactly(theta, M, B, n_cols, noo):
    n = 48
    rows = _random_rows(n, 5, seed=M + B + n_cols)
    if noo:
        pi, _ = planner.noo(rows, B, M, TH=16)
    else:
        pi = np.random.default_rng(3).permutation(B)[:n]
    prog = radix2.build_program(np.asarray(pi), rows, M, B, wrap=(B == M), theta=theta)
    got = _program_matrix(prog, M, B, n_cols)
    assert np.array_equal(got, _expected_matrix(pi, rows, M, B, n_cols))


@pytest.mark.parametrize("delta", [1, 5, 11, 21, 31, 50, 63])
def test_circulant_graph_takes_popcount_rotations(delta):
    """Every node needs the node delta ahead (identity order, one column):
    one lane, one rotation and one level per set bit of the AOO-reduced shift."""
    n = M = 64
    rows = [[(v, 0.5), ((v + delta) % n, 0.5)] for v in range(n)]
    prog = radix2.build_program(np.arange(n), rows, M, M, wrap=True)
    d = radix2.reduce_shift(delta, M, True)
    bits = bin(abs(d)).count("1")
    assert prog.n_lanes == 1
    assert len(prog.rotations()) == bits and prog.depth == bits
    assert prog.amounts() == sorted(int(np.sign(d)) * (1 << b) for b in range(7) if (abs(d) >> b) & 1)


def test_cycle_graph_two_rotations_one_level():
    n = M = 64
    rows = [[((v - 1) % n, 1 / 3), (v, 1 / 3), ((v + 1) % n, 1 / 3)] for v in range(n)]
    prog = radix2.build_program(np.arange(n), rows, M, M, wrap=True)
    assert prog.amounts() == [-1, 1] and len(prog.rotations()) == 2 and prog.depth == 1


def test_aoo_shortens_the_wrap_around_demand():
    """A ring's wrap-around demand is delta = M - 1 without AOO (six rounds)
    and -1 with it (Sec. 3.3.1)."""
    n = M = 64
    rows = [[(v, 0.5), ((v + 1) % n, 0.5)] for v in range(n)]
    with_aoo = radix2.build_program(np.arange(n), rows, M, M, wrap=True)
    without = radix2.build_program(np.arange(n), rows, M, M, wrap=False)
    assert with_aoo.depth == 1 and len(with_aoo.rotations()) == 1
    assert without.depth == 6 and len(without.rotations()) > len(with_aoo.rotations())
    for prog in (with_aoo, without):
        assert np.array_equal(_program_matrix(prog, M, M, 1), _expected_matrix(np.arange(n), rows, M, M, 1))


@pytest.mark.parametrize("name", ["tiny_deep", "tiny2_deep"])
def test_rotations_within_worst_case_and_cpoo_prunes(name):
    w = make_workload(name)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    M = 2 ** (w.params["log_n"] - 1)
    first = "spintra" if len(w.meta["dims"]) == 2 else "inter"
    base = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, M, family=3, first_mode=first)
    cp = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, M, family=3, first_mode=first, cpoo=0.25)
    n = max(sum(1 for u, _ in row if u != v) for v, row in enumerate(rows))
    worst = (n - 1) * planner.clog2(w.graph.n) ** 2
    pb, pc = base.layers[-1].program, cp.layers[-1].program
    assert len(pb.rotations()) <= worst
    assert len(pc.rotations()) < len(pb.rotations()) and pc.depth <= pb.depth
    # the depth is the number of rounds in which something moves, at most the bit length of max |delta|
    assert pb.depth <= max(abs(d) for d in base.layers[-1].shifts).bit_length()


@pytest.mark.slow
def test_encrypted_radix2_layer_decrypts_to_fp64():
    from oracle import ckks, execute as ex
    w = make_workload("tiny_deep")
    prm = Params.from_dict(w.params)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    ref = gcn.gcn_forward(rows, w.x, w.weights, w.activation)[-1]
    plan = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M, family=3,
                              first_mode="spintra", cpoo=0.25)
    keys = ckks.keygen(prm, 11, plan.rot_steps(prm.M), relin=False)
    sched = ex.schedule(prm, plan)
    assert sched[0]["level_out"] == sched[0]["level_agg"] - plan.layers[0].program.depth
    ops = ex.encode_operands(prm, plan, w.weights, sched)
    cts = ex.client_encrypt(prm, plan, w.x, keys, 12)
    outs = ex.run(prm, plan, keys, cts, ops, sched)
    assert outs[-1][0].level == sched[0]["level_out"]
    y = ex.decrypt_output(prm, plan, keys, outs[-1])
    assert gcn.max_rel_error(y, ref) < 1e-3
