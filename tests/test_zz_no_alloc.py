"""The relinearised product without device allocation (ckks_mul_relin_noalloc)
against the allocating entry point (ckks_mul_relin, itself pinned word for
word against the oracle): equal words on two calls in a row, the second at a
lower level (a smaller input), and ENOMEM, with nothing written, for a level
whose intermediates exceed the fixed array.

Parameters: N = 2^16 with 18 + 2 primes, so the top level needs more than the
64 MiB array (274 limbs of 512 KiB) while levels 5 and 1 fit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PARAMS = dict(log_n=16, n_q=18, q_bits=50, n_p=2, p_bits=60, log_scale=40)


def _need_bytes(level, alpha, N):
    l1 = level + 1
    ext, nd = l1 + alpha, -(-l1 // alpha)
    return (3 * l1 + nd * ext + 2 * ext) * N * 8


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2506_10399_amd import ficgcn as fg
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    ctx = fg.Context.from_dict(PARAMS)
    cl, ev = ctx.ckks_keygen(515, [], with_relin=True)
    return dict(fg=fg, ctx=ctx, cl=cl, ev=ev, rng=np.random.default_rng(5))


def _rand_ct(e, level, ct_id):
    ctx = e["ctx"]
    M = (1 << PARAMS["log_n"]) // 2
    z = e["rng"].uniform(-1, 1, M)
    pt = ctx.ckks_encode(z, 2.0 ** PARAMS["log_scale"], level)
    return z, ctx.ckks_encrypt(e["cl"], pt, level, 99, ct_id)


def test_noalloc_equals_allocating_entry_point(env):
    ctx = env["ctx"]
    limit = env["fg"].lib().ckks_mul_relin_noalloc_limit()
    assert limit == 64 << 20
    for lv, cid in ((5, 10), (1, 20)):        # second call: a smaller input
        assert _need_bytes(lv, PARAMS["n_p"], 1 << PARAMS["log_n"]) <= limit
        z1, x = _rand_ct(env, lv, cid)
        z2, y = _rand_ct(env, lv, cid + 1)
        want = ctx.ckks_mul_relin(env["ev"], x, y, lv)
        out = ctx.ct_buffer(lv)
        out.fill_(-1)
        ctx.ckks_mul_relin_noalloc(env["ev"], x, y, lv, out)
        got_w = ctx.ckks_poly_store(out, lv, 2)
        want_w = ctx.ckks_poly_store(want, lv, 2)
        assert np.array_equal(got_w, want_w), "level %d: words differ from ckks_mul_relin" % lv
        dec = ctx.ckks_decrypt(env["cl"], out, lv, 2.0 ** (2 * PARAMS["log_scale"]), len(z1))
        assert np.abs(dec - z1 * z2).max() < 1e-6


def test_noalloc_rejects_level_beyond_the_array(env):
    ctx, fg = env["ctx"], env["fg"]
    lv = PARAMS["n_q"] - 1
    assert _need_bytes(lv, PARAMS["n_p"], 1 << PARAMS["log_n"]) > fg.lib().ckks_mul_relin_noalloc_limit()
    _, x = _rand_ct(env, lv, 30)
    _, y = _rand_ct(env, lv, 31)
    out = ctx.ct_buffer(lv)
    out.fill_(7)
    with pytest.raises(fg.FicgcnError) as ei:
        ctx.ckks_mul_relin_noalloc(env["ev"], x, y, lv, out)
    assert ei.value.status == -5
    ctx.ckks_sync()
    assert bool((out == 7).all())
