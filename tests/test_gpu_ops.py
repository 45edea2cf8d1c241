"""GPU parity of every CKKS operation against the oracle, through the C ABI.

Inputs (ciphertexts, plaintexts, keys) come from the oracle; the GPU result is
read back in coefficient form and compared word for word.  Runs at the tiny
parameters (N = 2^13, 4 + 1 primes) and at the citation-graph parameters
(N = 2^16, 8 + 2 primes), i.e. in the launch shapes the benchmark uses."""
import numpy as np
import pytest

from oracle import ckks, encoding as enc
from oracle.params import Params

pytestmark = pytest.mark.gpu

PARAMS = {
    "tiny": dict(log_n=13, n_q=4, q_bits=50, n_p=1, p_bits=60, log_scale=40),
    "cora": dict(log_n=16, n_q=8, q_bits=50, n_p=2, p_bits=60, log_scale=40),
}
STEPS = [1, 3, -5, 100]
SEED = 4242


def _ct(c: ckks.Ciphertext) -> np.ndarray:
    return np.stack([c.c0, c.c1])


@pytest.fixture(scope="module", params=["tiny", "cora"])
def env(request):
    import torch
    from paper_2506_10399_amd import ficgcn as fg
    assert torch.cuda.is_available()
    d = PARAMS[request.param]
    prm = Params.from_dict(d)
    ctx = fg.Context.from_dict(d)
    steps = STEPS if request.param == "tiny" else STEPS[:2]
    okeys = ckks.keygen(prm, SEED, steps, relin=True)
    cl, ev = ctx.ckks_keygen(SEED, steps, with_relin=True)
    rng = np.random.default_rng(11)
    return dict(name=request.param, prm=prm, ctx=ctx, okeys=okeys, cl=cl, ev=ev, steps=steps, rng=rng, fg=fg)


def _rand_ct(e, level, ct_id):
    prm = e["prm"]
    z = e["rng"].uniform(-1, 1, prm.M)
    return z, ckks.encrypt(prm, 77, ct_id, e["okeys"].s, enc.encode(prm, z, prm.scale, level))


def test_prime_chain(env):
    assert env["ctx"].ckks_ctx_moduli() == env["prm"].q + env["prm"].p


def test_ntt_roundtrip_and_ring_product(env):
    prm, ctx = env["prm"], env["ctx"]
    lv = prm.L - 1
    mods = prm.q_level(lv)
    a = np.stack([np.stack([env["rng"].integers(0, q, prm.N, dtype=np.uint64) for q in mods]) for _ in range(2)])
    b = np.stack([env["rng"].integers(0, q, prm.N, dtype=np.uint64) for q in mods])
    da = ctx.ckks_ct_load(a, lv)
    assert np.array_equal(ctx.ckks_poly_store(da, lv, 2), a)
    db = ctx.ckks_pt_load(b, lv)
    acc = ctx.ct_buffer(lv)
    acc.zero_()
    ctx.ckks_pt_mul_acc(acc, lv, [da], [db])
    got = ctx.ckks_poly_store(acc, lv, 2)
    for c in range(2):
        assert np.array_equal(got[c], ckks.poly_mul(b, a[c], mods, prm))


def test_keygen_matches_oracle(env):
    prm, ctx = env["prm"], env["ctx"]
    tags = env["ev"].ckks_keys_tags()
    assert sorted(tags) == sorted([0] + list(env["okeys"].rot))
    for tag in tags:
        ok = env["okeys"].relin if tag == 0 else env["okeys"].rot[tag]
        got = env["ev"].ckks_keys_export(tag)
        for j in range(prm.beta):
            assert np.array_equal(got[j, 0], ok.b[j]), ("b", tag, j)
            assert np.array_equal(got[j, 1], ok.a[j]), ("a", tag, j)


def test_encrypt_matches_oracle(env):
    prm, ctx = env["prm"], env["ctx"]
    for lv in (prm.L - 1, 1):
        z = env["rng"].uniform(-1, 1, prm.M)
        pt = enc.encode(prm, z, prm.scale, lv)
        want = ckks.encrypt(prm, SEED, 9 + lv, env["okeys"].s, pt)
        dpt = ctx.ckks_pt_load(pt.m, lv)
        ct = ctx.ckks_encrypt(env["cl"], dpt, lv, SEED, 9 + lv)
        assert np.array_equal(ctx.ckks_poly_store(ct, lv, 2), _ct(want))
        # decrypt + decode on the GPU path
        got = ctx.ckks_decrypt(env["cl"], ct, lv, prm.scale, prm.M)
        assert np.abs(got - z).max() < 1e-6


def test_seeded_encryption_and_rebuild_match_oracle(env):
    """A seeded ciphertext (uniform part from a public seed) has the oracle's
    words; rebuilding the uniform parts of a batch from (seed, ids) restores each
    second polynomial, across the launch's chunk of 4096 ciphertexts at the tiny
    parameters, and leaves the first polynomials alone."""
    import torch
    prm, ctx, fg = env["prm"], env["ctx"], env["fg"]
    A_SEED = 0x5EED5EED
    for lv in (prm.L - 1, 1):
        z = env["rng"].uniform(-1, 1, prm.M)
        pt = enc.encode(prm, z, prm.scale, lv)
        want = ckks.encrypt(prm, SEED + 1, 30 + lv, env["okeys"].s, pt, a_seed=A_SEED)
        dpt = ctx.ckks_pt_load(pt.m, lv)
        ct = ctx.ckks_encrypt_seeded(env["cl"], dpt, lv, SEED + 1, A_SEED, 30 + lv)
        assert np.array_equal(ctx.ckks_poly_store(ct, lv, 2), _ct(want))
        assert np.abs(ctx.ckks_decrypt(env["cl"], ct, lv, prm.scale, prm.M) - z).max() < 1e-6
    for bad in (SEED + 1, SEED):     # the error seed, the key generation seed
        with pytest.raises(fg.FicgcnError) as ei:
            ctx.ckks_encrypt_seeded(env["cl"], dpt, 1, SEED + 1, bad, 0)
        assert ei.value.status == -1
    lv = 0 if env["name"] == "tiny" else 1
    count, id0 = (4100, 7) if env["name"] == "tiny" else (3, 7)
    buf = torch.randint(0, 1 << 40, (count, 2, lv + 1, prm.N), dtype=torch.int64, device="cuda")
    c0 = buf[:, 0].clone()
    ctx.ckks_expand_seeded(A_SEED, id0, count, lv, buf)
    torch.cuda.synchronize()
    assert torch.equal(buf[:, 0], c0)
    for z in sorted({0, 1, count // 2, count - 1} | ({4095, 4096} if count > 4096 else set())):
        got = ctx.ckks_poly_store(buf[z].contiguous(), lv, 2)[1]
        assert np.array_equal(got, ckks.seeded_uniform(prm, A_SEED, id0 + z, lv)), z
    ctx.ckks_expand_seeded(A_SEED, 0, 0, lv, buf)     # no ciphertexts: nothing to do
    with pytest.raises(fg.FicgcnError) as ei:
        ctx.ckks_expand_seeded(A_SEED, 0, 1, prm.L, buf)
    assert ei.value.status == -2


@pytest.mark.parametrize("bits", [50, 60, 64, 13])
def test_packed_residues_layout_and_round_trip(env, bits):
    """Residues packed at `bits` each form the limb's little-endian bit stream (checked
    against Python integers), and unpacking restores them; higher bits are dropped."""
    import torch
    if env["name"] != "tiny":
        pytest.skip("layout checked at the tiny ring degree")
    ctx, N = env["ctx"], env["prm"].N
    n_limbs = 3
    rng = np.random.default_rng(bits)
    hi = (1 << bits) if bits < 64 else (1 << 64)
    x = np.stack([rng.integers(0, hi, N, dtype=np.uint64) if bits < 64 else
                  rng.integers(0, 1 << 63, N, dtype=np.uint64) * np.uint64(2) + np.uint64(1) for _ in range(n_limbs)])
    if bits < 64:
        x[:, 5] |= np.uint64(1) << np.uint64(bits)     # a bit above the width: dropped
    dev = torch.from_numpy(x.view(np.int64)).to("cuda")
    packed = ctx.ckks_pack_residues(dev, n_limbs, bits)
    got = packed.cpu().numpy().view(np.uint64).reshape(n_limbs, N * bits // 64)
    mask = (1 << bits) - 1
    for li in range(n_limbs):
        stream = 0
        for r in range(N):
            stream |= (int(x[li, r]) & mask) << (r * bits)
        want = [(stream >> (64 * w)) & ((1 << 64) - 1) for w in range(N * bits // 64)]
        assert [int(v) for v in got[li]] == want, li
    back = ctx.ckks_unpack_residues(packed, n_limbs, bits).cpu().numpy().view(np.uint64).reshape(n_limbs, N)
    assert np.array_equal(back, x & np.uint64(mask) if bits < 64 else x)


def test_rotate_hoisted_matches_oracle(env):
    prm, ctx = env["prm"], env["ctx"]
    for lv in (prm.L - 1, 2):
        z, oct_ = _rand_ct(env, lv, 1 + lv)
        want = ckks.rotate_hoisted(prm, env["okeys"], oct_, env["steps"])
        dct = ctx.ckks_ct_load(_ct(oct_), lv)
        outs = ctx.ckks_rotate_hoisted(env["ev"], dct, lv, env["steps"])
        for k, o, wnt in zip(env["steps"], outs, want):
            assert np.array_equal(ctx.ckks_poly_store(o, lv, 2), _ct(wnt)), (lv, k)
        # a single rotation gives the same words (canonical rotation)
        one = ctx.ckks_rotate_hoisted(env["ev"], dct, lv, env["steps"][1:2])[0]
        assert np.array_equal(ctx.ckks_poly_store(one, lv, 2), _ct(want[1]))


def test_rotate_batch_matches_oracle(env):
    """Several ciphertexts and steps in one key-switch batch (shared sources
    hoisted, zero step copied) give the oracle's single-rotation words."""
    prm, ctx = env["prm"], env["ctx"]
    lv = prm.L - 1
    cts = [_rand_ct(env, lv, 40 + i)[1] for i in range(3)]
    dcts = [ctx.ckks_ct_load(_ct(c), lv) for c in cts]
    st = env["steps"]
    pairs = [(0, st[0]), (1, st[1]), (0, st[-1]), (2, 0), (2, st[0]), (1, st[0])]
    outs = ctx.ckks_rotate_batch(env["ev"], [dcts[i] for i, _ in pairs], lv, [k for _, k in pairs])
    for (i, k), o in zip(pairs, outs):
        want = cts[i] if k == 0 else ckks.rotate(prm, env["okeys"], cts[i], k)
        assert np.array_equal(ctx.ckks_poly_store(o, lv, 2), _ct(want)), (i, k)


def test_rotate_missing_key_is_enokey(env):
    ctx = env["ctx"]
    lv = 1
    dct = ctx.ct_buffer(lv)
    dct.zero_()
    with pytest.raises(env["fg"].FicgcnError) as e:
        ctx.ckks_rotate_hoisted(env["ev"], dct, lv, [7])
    assert e.value.status == -4


def test_pt_and_scalar_mac_and_add_match_oracle(env):
    prm, ctx = env["prm"], env["ctx"]
    lv = prm.L - 1
    cts = [_rand_ct(env, lv, 20 + i)[1] for i in range(3)]
    pts = [enc.encode(prm, env["rng"].uniform(-1, 1, prm.M), float(prm.q[lv]), lv) for _ in range(3)]
    consts = [123456789012, -987654321098, 5]
    acc0 = ckks.zero_ct(prm, lv, 1.0)
    want = ckks.pt_mul_acc(prm, acc0, cts, pts)
    want = ckks.scalar_mul_acc(prm, want, cts, consts)
    want = ckks.add(prm, want, cts[0])
    dcts = [ctx.ckks_ct_load(_ct(c), lv) for c in cts]
    dpts = [ctx.ckks_pt_load(p.m, lv) for p in pts]
    acc = ctx.ct_buffer(lv)
    acc.zero_()
    ctx.ckks_pt_mul_acc(acc, lv, dcts, dpts)
    ctx.ckks_scalar_mul_acc(acc, lv, dcts, consts)
    ctx.ckks_add(acc, dcts[0], lv)
    assert np.array_equal(ctx.ckks_poly_store(acc, lv, 2), _ct(want))


def test_rescale_matches_oracle(env):
    prm, ctx = env["prm"], env["ctx"]
    for lv in (prm.L - 1, 1):
        _, c = _rand_ct(env, lv, 30 + lv)
        want = ckks.rescale(prm, c)
        d = ctx.ckks_ct_load(_ct(c), lv)
        ctx.ckks_rescale(d, lv)
        got = ctx.ckks_poly_store(d, lv - 1, 2)
        assert np.array_equal(got, _ct(want))


def test_mul_relin_matches_oracle(env):
    prm, ctx = env["prm"], env["ctx"]
    lv = prm.L - 2
    z1, c1 = _rand_ct(env, lv, 40)
    z2, c2 = _rand_ct(env, lv, 41)
    want = ckks.ct_mul_relin(prm, env["okeys"], c1, c2)
    d1, d2 = ctx.ckks_ct_load(_ct(c1), lv), ctx.ckks_ct_load(_ct(c2), lv)
    out = ctx.ckks_mul_relin(env["ev"], d1, d2, lv)
    assert np.array_equal(ctx.ckks_poly_store(out, lv, 2), _ct(want))
    got = ctx.ckks_decrypt(env["cl"], out, lv, prm.scale ** 2, prm.M)
    assert np.abs(got - z1 * z2).max() < 1e-6


def test_encoder_decodes_within_precision(env):
    prm, ctx = env["prm"], env["ctx"]
    lv = prm.L - 1
    z = env["rng"].uniform(-1, 1, prm.M)
    d = ctx.ckks_encode(z, prm.scale, lv)
    m = ctx.ckks_poly_store(d, lv, 1)[0]
    want = enc.encode(prm, z, prm.scale, lv).m
    # independent FP64 FFTs may round a handful of coefficients differently
    assert np.mean(m != want) < 1e-3
    back = enc.decode(prm, ckks.Plaintext(m=m, level=lv, scale=prm.scale))
    assert np.abs(back - z).max() < 1e-9


def test_batch_encoder_at_mask_scale_and_range_error(env):
    """The device encoder in batches at the scale masks use (the prime the next
    rescale drops, about 2^50): a small fraction of coefficients may round the
    other way than the oracle's independent FFT, the decoded slots agree to
    1e-9; coefficients beyond 63 bits are rejected with ESCALE."""
    prm, ctx, fg = env["prm"], env["ctx"], env["fg"]
    lv = prm.L - 1
    rows = env["rng"].uniform(-1, 1, (5, prm.M))
    sM = float(prm.q[lv])
    d = ctx.ckks_encode_batch(rows, sM, lv)
    for i in range(len(rows)):
        m = ctx.ckks_poly_store(d[i], lv, 1)[0]
        want = enc.encode(prm, rows[i], sM, lv).m
        assert np.mean(m != want) < 0.05
        back = enc.decode(prm, ckks.Plaintext(m=m, level=lv, scale=sM))
        assert np.abs(back - rows[i]).max() < 1e-9
    with pytest.raises(fg.FicgcnError):
        ctx.ckks_encode_batch(rows[:2] * 1e9, 2.0 ** 62, lv)


def test_ntt_every_schedule_gives_the_same_words(env):
    """Every NTT schedule the autotuner may pick (column-pass size 2^(log_n/2 - 1 .. log_n/2 + 1),
    workgroup widths) computes the same transform: the ring product through
    it equals the oracle's, and the autotuner's choice is one of them."""
    prm, ctx = env["prm"], env["ctx"]
    lv = prm.L - 1
    mods = prm.q_level(lv)
    a = np.stack([env["rng"].integers(0, q, prm.N, dtype=np.uint64) for q in mods])
    b = np.stack([env["rng"].integers(0, q, prm.N, dtype=np.uint64) for q in mods])
    want = ckks.poly_mul(b, a, mods, prm)
    mid = prm.log_n // 2
    try:
        for split in (mid - 1, mid, mid + 1):
            if not (4 <= split <= 9 and 4 <= prm.log_n - split <= 9):
                continue
            for c0, c1 in ((16, 4), (4, 16), (1, 2)):
                ctx.ckks_ntt_config(split, c0, c1)
                da = ctx.ckks_pt_load(a, lv)
                db = ctx.ckks_pt_load(b, lv)
                ctx.ckks_ntt(da, lv + 1, 0, False)   # da, db: evaluation form; take da back and forth once more
                ctx.ckks_ntt(da, lv + 1, 0, True)
                got = ctx.ckks_poly_store(da, lv, 1)[0]
                assert np.array_equal(got, a), (split, c0, c1)
                ct = ctx.ckks_ct_load(np.stack([a, a]), lv)
                out = ctx.ct_buffer(lv)
                out.zero_()
                ctx.ckks_pt_mul_acc(out, lv, [ct], [db])
                assert np.array_equal(ctx.ckks_poly_store(out, lv, 2)[0], want), (split, c0, c1)
        with pytest.raises(env["fg"].FicgcnError):
            ctx.ckks_ntt_config(3, 16, 4)
        c0, c1, split = ctx.ckks_ntt_autotune(prm.L + prm.n_p)
        assert split in (mid - 1, mid, mid + 1) and c0 in (4, 8, 16) and c1 in (2, 4, 8, 16)
    finally:
        ctx.ckks_ntt_config(0, 16, 4)


@pytest.mark.parametrize("log_n", [9, 10, 11, 12, 14])
def test_encoder_every_ring_degree(log_n):
    """The device encoder's four-step FFT at every split shape (N1 x N2 from
    16 x 32 up): coefficients as the oracle's encoder gives them (a few may
    round the other way) and the slots decoded back within 1e-9."""
    import torch
    from paper_2506_10399_amd import ficgcn as fg
    assert torch.cuda.is_available()
    d = dict(log_n=log_n, n_q=3, q_bits=50, n_p=1, p_bits=60, log_scale=40)
    prm = Params.from_dict(d)
    ctx = fg.Context.from_dict(d)
    lv = prm.L - 1
    z = np.random.default_rng(log_n).uniform(-1, 1, prm.M)
    m = ctx.ckks_poly_store(ctx.ckks_encode(z, prm.scale, lv), lv, 1)[0]
    want = enc.encode(prm, z, prm.scale, lv).m
    assert np.mean(m != want) < 1e-3
    back = enc.decode(prm, ckks.Plaintext(m=m, level=lv, scale=prm.scale))
    assert np.abs(back - z).max() < 1e-9
