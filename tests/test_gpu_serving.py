"""The serving loop on the GPU: continuous batching must not change results.

Each request's returned ciphertext words are the same when it runs alone and
when it runs in a mix with others on concurrent slots; decrypted, every
result is within 1e-3 of the FP64 model; a served request given the oracle's
operands and ciphertexts returns the oracle's words.  Admission respects the
device budget (resident keys and plan tables, slot arenas and scratch), a
request that can never fit is refused, and in steady state requests allocate
nothing (the slot arenas are reused)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PARAMS = dict(log_n=13, n_q=8, q_bits=50, n_p=2, p_bits=60, log_scale=40)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2506_10399_amd import ficgcn as fg, serving as sv
    assert torch.cuda.is_available()
    ctx = fg.Context.from_dict(PARAMS)
    reqs = sv.make_requests(ctx, 5, 31, n_range=(60, 500), f_range=(8, 40), classes=(2, 7))
    cl, ev = sv.client_keys(ctx, reqs, 77)
    for i, q in enumerate(reqs):
        sv.encrypt_inputs(ctx, cl, q, 1000 + i)
    return dict(fg=fg, sv=sv, ctx=ctx, reqs=reqs, cl=cl, ev=ev)


def _footprints(env):
    """Each request's footprint (arena + scratch bound) and the resident bytes (keys, plan tables)."""
    fg = env["fg"]
    srv = fg.Server(PARAMS, 1, 1 << 40)
    out = []
    for q in env["reqs"]:
        rid = srv.ficgcn_server_submit(q.plan, env["ev"], q.inputs_host, len(q.inputs_host), q.output_host,
                                       len(q.output_host))
        out.append(srv.ficgcn_server_wait(rid)["footprint_bytes"])
    st = srv.ficgcn_server_stats()
    srv.close()
    assert st["scratch_overruns"] == 0
    return out, st["resident_bytes"]


def test_alone_equals_mix(env):
    fg, sv, reqs = env["fg"], env["sv"], env["reqs"]
    alone = []
    for q in reqs:
        srv = fg.Server(PARAMS, 1, 1 << 40)
        st = sv.run_stream(srv, [q], env["ev"], 0.0, 1)
        assert st["completed"] == 1 and st["failed"] == 0
        alone.append(q.output_host.copy())
        srv.close()
    for q in reqs:
        q.output_host[:] = 0
    srv = fg.Server(PARAMS, 3, 1 << 40)
    st = sv.run_stream(srv, reqs, env["ev"], 0.0, 2)      # all at once: three slots busy
    srv.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_concurrent"] >= 2
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    for q, a in zip(reqs, alone):
        assert np.array_equal(q.output_host, a), q.name
        assert sv.decrypt_error(env["ctx"], env["cl"], q) < 1e-3, q.name


def test_admission_by_footprint(env):
    fg, sv, reqs = env["fg"], env["sv"], env["reqs"]
    fp, resident = _footprints(env)
    s_ = sorted(fp)
    # room for the largest request alone (and, when any two exceed it, for one at a time)
    budget = resident + s_[-1]
    srv = fg.Server(PARAMS, 3, budget)
    st = sv.run_stream(srv, reqs, env["ev"], 0.0, 3)
    srv.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_bytes"] <= budget
    if s_[0] + s_[1] > s_[-1]:
        assert st["max_concurrent"] == 1
    assert st["scratch_overruns"] == 0
    # a request that can never fit is refused at submission
    srv = fg.Server(PARAMS, 2, min(fp) - 1)
    q = reqs[int(np.argmin(fp))]
    with pytest.raises(fg.FicgcnError) as e:
        srv.ficgcn_server_submit(q.plan, env["ev"], q.inputs_host, len(q.inputs_host), q.output_host,
                                 len(q.output_host))
    assert e.value.status == -5
    srv.close()


def test_arenas_reused_in_steady_state(env):
    """The second pass over the same requests allocates no arena: every slot's
    arena already fits them."""
    fg, sv, reqs = env["fg"], env["sv"], env["reqs"]
    srv = fg.Server(PARAMS, 2, 1 << 40)
    sv.run_stream(srv, reqs, env["ev"], 0.0, 5)
    first = srv.ficgcn_server_stats()["arena_allocs"]
    assert 1 <= first <= 2 * len(reqs)
    sv.run_stream(srv, reqs, env["ev"], 0.0, 6)
    second = srv.ficgcn_server_stats()
    srv.close()
    assert second["arena_allocs"] == first
    assert second["completed"] == 2 * len(reqs) and second["scratch_overruns"] == 0


def test_served_request_returns_oracle_words():
    """A two-layer request served beside another, with the oracle's encoded
    operands and the oracle's ciphertexts, returns the oracle's output words; so
    does a second request of the same plan submitted at the same time."""
    import torch
    from oracle import ckks, gcn, planner, execute as ex
    from oracle.params import Params
    from workload import make_workload
    from paper_2506_10399_amd import ficgcn as fg, graph, serving as sv
    w = make_workload("tiny2")
    prm = Params.from_dict(w.params)
    rows = gcn.normalized_rows(w.graph.n, w.neighbors, w.norm)
    o = planner.build_plan(w.graph.n, rows, w.meta["dims"], w.activation, prm.M)
    okeys = ckks.keygen(prm, 41, o.rot_steps(prm.M), relin=True)
    sched = ex.schedule(prm, o)
    ops = ex.encode_operands(prm, o, w.weights, sched)
    cts = ex.client_encrypt(prm, o, w.x, okeys, 42)
    want = ex.run(prm, o, okeys, cts, ops, sched)[-1]
    ctx = fg.Context.from_dict(w.params)
    rp, col, val = graph.normalize(w.graph.n, w.neighbors, w.norm)
    p = fg.Plan(ctx, rp, col, val, w.graph.n, w.meta["dims"], w.weights, activation=True)
    assert np.array_equal(p.ficgcn_plan_node_order(), o.pi)
    _, ev = ctx.ckks_keygen(41, p.ficgcn_plan_rot_steps(), with_relin=True)
    info = p.ficgcn_plan_info()
    lv0, lvo = info[0]["level_in"], info[-1]["level_out"]
    host_in = torch.empty((len(cts), 2, lv0 + 1, ctx.N), dtype=torch.int64, pin_memory=True)
    for i, c in enumerate(cts):
        host_in[i].copy_(ctx.ckks_ct_load(np.stack([c.c0, c.c1]), lv0))
    operands = []
    for lp, d in zip(o.layers, ops):
        flat = d["P"] if lp.kind == "inter" else [d["masks"][g][s] for g in range(len(d["masks"])) for s in lp.shifts]
        operands.append(np.concatenate([pt.m.ravel() for pt in flat]))
    out_host = np.zeros((len(want), 2, lvo + 1, ctx.N), dtype=np.uint64)
    # another request on the same server at the same time (its own plan, the library's encoder)
    other = sv.make_requests(ctx, 1, 9, n_range=(100, 200), f_range=(8, 16))[0]
    cl2, ev2 = sv.client_keys(ctx, [other], 43)
    sv.encrypt_inputs(ctx, cl2, other, 44)
    out_again = np.zeros_like(out_host)
    srv = fg.Server(w.params, 3, 1 << 40)
    r1 = srv.ficgcn_server_submit(p, ev, host_in, len(cts), out_host, len(want), operands_host=operands)
    r2 = srv.ficgcn_server_submit(other.plan, ev2, other.inputs_host, len(other.inputs_host), other.output_host,
                                  len(other.output_host))
    # the same plan again at once: it shares the operands the first request loads
    r3 = srv.ficgcn_server_submit(p, ev, host_in, len(cts), out_again, len(want))
    for r in (r1, r2, r3):
        srv.ficgcn_server_wait(r)
    srv.close()
    for res in (out_host, out_again):
        for i, c in enumerate(want):
            dev = torch.from_numpy(res[i].view(np.int64)).cuda()
            got = ctx.ckks_poly_store(dev, lvo, 2)
            assert np.array_equal(got, np.stack([c.c0, c.c1])), ("output", i)


def test_poisson_stream_reports_latency(env):
    fg, sv, reqs = env["fg"], env["sv"], env["reqs"]
    srv = fg.Server(PARAMS, 2, 1 << 40)
    st = sv.run_stream(srv, reqs, env["ev"], 50.0, 4)
    srv.close()
    assert st["completed"] == len(reqs)
    lat = sorted(q.result["latency_ms"] for q in reqs)
    assert st["p50_ms"] == lat[(len(lat) + 1) // 2 - 1] and st["p99_ms"] == lat[-1]
    assert st["throughput_per_s"] > 0
    for q in reqs:
        assert abs(q.result["latency_ms"] - q.result["queue_ms"] - q.result["run_ms"]) < 1e-6


def test_seeded_inputs_return_the_words_of_whole_inputs(env):
    """A request sent as seeded ciphertexts (each input's first polynomial and a
    public seed; the server rebuilds the uniform parts) returns the words of the
    same ciphertexts sent whole, beside an unseeded request; the upload is half,
    and with the first polynomials packed at the primes' bit length smaller still."""
    import dataclasses
    fg, sv, ctx = env["fg"], env["sv"], env["ctx"]
    base = env["reqs"][1]
    whole = dataclasses.replace(base, result={})
    seeded = dataclasses.replace(base, result={})
    sv.encrypt_inputs(ctx, env["cl"], whole, 4001, a_seed=0xABCDEF, whole=True)
    sv.encrypt_inputs(ctx, env["cl"], seeded, 4001, a_seed=0xABCDEF)
    assert seeded.a_seed == 0xABCDEF and whole.a_seed is None
    assert seeded.inputs_host.numel() * 2 == whole.inputs_host.numel()
    assert bool((seeded.inputs_host == whole.inputs_host[:, 0]).all())
    packed = dataclasses.replace(base, result={})
    bits = max(m.bit_length() for m in ctx.ckks_ctx_moduli()[:PARAMS["n_q"]])
    sv.encrypt_inputs(ctx, env["cl"], packed, 4001, a_seed=0xABCDEF, packed_bits=bits)
    assert packed.packed_bits == bits and packed.inputs_host.numel() * 64 == seeded.inputs_host.numel() * bits
    other = dataclasses.replace(env["reqs"][0], result={}, output_host=np.zeros_like(env["reqs"][0].output_host))
    srv = fg.Server(PARAMS, 2, 1 << 40)
    st = sv.run_stream(srv, [seeded, other, whole, packed], env["ev"], 0.0, 9)
    assert st["completed"] == 4 and st["failed"] == 0
    assert np.array_equal(seeded.output_host, whole.output_host)
    assert np.array_equal(packed.output_host, whole.output_host)
    assert sv.decrypt_error(ctx, env["cl"], seeded) < 1e-3
    # a packed width below a prime's bit length is refused at submission
    with pytest.raises(fg.FicgcnError):
        srv.ficgcn_server_submit(packed.plan, env["ev"], packed.inputs_host, len(packed.inputs_host),
                                 packed.output_host, len(packed.output_host), a_seed=0xABCDEF, packed_bits=bits - 1)
    srv.close()
