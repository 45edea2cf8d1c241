"""GPU checks of the descriptor forms of the core operations (ckks_*_op): the
same words as the raw-pointer calls, the level and scale each output takes
(Sec. 2.1: scales multiply, a rescale divides by the dropped prime), and a
rejected call (ELEVEL / ESCALE) leaves its output buffer untouched."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2506_10399_amd import ficgcn as fg
    ctx = fg.Context(13, 4, 50, 1, 60)
    cl, ev = ctx.ckks_keygen(3, [1, 5], with_relin=True)
    rng = np.random.default_rng(5)
    z = rng.uniform(-1, 1, ctx.M)
    w = rng.uniform(-1, 1, ctx.M)
    lv = 3
    S = 2.0 ** 40
    pt = ctx.pt_buffer(lv)
    ctx.ckks_encode(z, S, lv, out=pt)
    pw = ctx.pt_buffer(lv)
    q = ctx.ckks_ctx_moduli()
    ctx.ckks_encode(w, float(q[lv]), lv, out=pw)
    return dict(torch=torch, fg=fg, ctx=ctx, cl=cl, ev=ev, z=z, w=w, lv=lv, S=S, pt=pt, pw=pw, q=q)


def _words(e, buf, level):
    return e["ctx"].ckks_poly_store(buf, level, 2)


def test_operand_calls_equal_raw_calls(env):
    e = env
    ctx, fg, lv, S, q = e["ctx"], e["fg"], e["lv"], e["S"], e["q"]
    x = ctx.ct_buffer(lv)
    X = ctx.operand(x, 0, 0.0)
    ctx.ckks_encrypt_op(e["cl"], ctx.operand(e["pt"], lv, S, 1), 7, 0, X)
    assert (X.level, X.scale) == (lv, S)
    ref = ctx.ct_buffer(lv)
    ctx.ckks_encrypt(e["cl"], e["pt"], lv, 7, 0, out=ref)
    assert np.array_equal(_words(e, x, lv), _words(e, ref, lv))
    # rotations
    outs = [ctx.ct_buffer(lv) for _ in range(2)]
    O = [ctx.operand(o, lv, 0.0) for o in outs]
    ctx.ckks_rotate_hoisted_op(e["ev"], X, [1, 5], O)
    raw = ctx.ckks_rotate_hoisted(e["ev"], x, lv, [1, 5])
    for a, b, o in zip(outs, raw, O):
        assert np.array_equal(_words(e, a, lv), _words(e, b, lv))
        assert (o.level, o.scale) == (lv, S)
    # plaintext MAC into a fresh accumulator, then a rescale
    acc = e["torch"].zeros_like(x)
    A = ctx.operand(acc, lv, 0.0)
    W = ctx.operand(e["pw"], lv, float(q[lv]), 1)
    ctx.ckks_pt_mul_acc_op(A, [X, O[0]], [W, W])
    assert A.scale == S * float(q[lv])
    acc2 = e["torch"].zeros_like(x)
    ctx.ckks_pt_mul_acc(acc2, lv, [x, outs[0]], [e["pw"], e["pw"]])
    assert np.array_equal(_words(e, acc, lv), _words(e, acc2, lv))
    ctx.ckks_rescale_op(A)
    ctx.ckks_rescale(acc2, lv)
    assert (A.level, A.scale) == (lv - 1, S * float(q[lv]) / float(q[lv]))
    assert np.array_equal(_words(e, acc, lv - 1), _words(e, acc2, lv - 1))
    got = np.real(ctx.ckks_decrypt_op(e["cl"], A, ctx.M))
    want = e["z"] * e["w"] + np.roll(e["z"], -1) * e["w"]
    assert np.max(np.abs(got - want)) < 1e-6
    # integer constants, add, relinearised product
    B = ctx.operand(e["torch"].zeros_like(x), lv, 0.0)
    ctx.ckks_scalar_mul_acc_op(B, [X, O[1]], [3, -2], float(q[lv]))
    assert B.scale == S * float(q[lv])
    b2 = e["torch"].zeros_like(x)
    ctx.ckks_scalar_mul_acc(b2, lv, [x, outs[1]], [3, -2])
    assert np.array_equal(_words(e, B.data, lv), _words(e, b2, lv))
    Y = ctx.operand(ctx.ct_buffer(lv), lv, 0.0)
    ctx.ckks_mul_relin_op(e["ev"], X, X, Y)
    assert (Y.level, Y.scale) == (lv, S * S)
    y2 = ctx.ckks_mul_relin(e["ev"], x, x, lv)
    assert np.array_equal(_words(e, Y.data, lv), _words(e, y2, lv))
    C = ctx.operand(ctx.ct_buffer(lv), lv, S)
    ctx.ckks_encrypt_op(e["cl"], ctx.operand(e["pt"], lv, S, 1), 7, 1, C)
    ctx.ckks_add_op(C, X)
    assert C.scale == S
    got = np.real(ctx.ckks_decrypt_op(e["cl"], C, ctx.M))
    assert np.max(np.abs(got - 2 * e["z"])) < 1e-6


def test_rejected_operand_call_leaves_output(env):
    e = env
    ctx, fg, lv, S = e["ctx"], e["fg"], e["lv"], e["S"]
    x = ctx.ct_buffer(lv)
    X = ctx.operand(x, 0, 0.0)
    ctx.ckks_encrypt_op(e["cl"], ctx.operand(e["pt"], lv, S, 1), 7, 2, X)
    acc = ctx.ct_buffer(lv)
    ctx.ckks_encrypt(e["cl"], e["pt"], lv, 7, 3, out=acc)
    before = _words(e, acc, lv)
    A = ctx.operand(acc, lv, S)
    for f, args, code in [
        (ctx.ckks_add_op, (A, ctx.operand(x, lv, 2 * S)), -3),
        (ctx.ckks_add_op, (A, ctx.operand(x, lv - 1, S)), -2),
        (ctx.ckks_pt_mul_acc_op, (A, [X], [ctx.operand(e["pw"], lv, 2.0, 1)]), -3),   # product scale 2 S, not S
        (ctx.ckks_mul_relin_op, (e["ev"], X, ctx.operand(x, lv - 1, S), A), -2),
    ]:
        with pytest.raises(fg.FicgcnError) as err:
            f(*args)
        assert err.value.status == code
        assert (A.level, A.scale) == (lv, S)
        assert np.array_equal(_words(e, acc, lv), before)
