"""Pins of the oracle's CKKS scheme: canonical embedding against its O(N^2)
definition, exact integer identities for rescale / ModDown, and the slot
semantics of Sec. 2.1 (decrypt(Rot(Enc(v), k)) = v shifted left by k)."""
import numpy as np
import pytest

from oracle import ckks, encoding as enc, ntheory as nt
from oracle.params import Params

rng = np.random.default_rng(7)


@pytest.fixture(scope="module")
def small():
    prm = Params(log_n=6, n_q=4, q_bits=50, n_p=2, p_bits=60)
    keys = ckks.keygen(prm, 99, rot_steps=[1, 2, 3, 5, -1, -7, 8], relin=True)
    return prm, keys


@pytest.mark.parametrize("N", [8, 16, 64, 256])
def test_embedding_fft_equals_definition(N):
    z = rng.uniform(-1, 1, N // 2) + 1j * rng.uniform(-1, 1, N // 2)
    assert np.allclose(enc.embed_inverse(z, N), enc.embed_inverse_direct(z, N), atol=1e-12)
    m = rng.uniform(-1, 1, N)
    assert np.allclose(enc.embed(m, N), enc.embed_direct(m, N), atol=1e-10)
    # inverse pair
    assert np.allclose(enc.embed(enc.embed_inverse(z, N), N), z, atol=1e-12)


def test_automorphism_rotates_slots():
    N = 64
    z = rng.uniform(-1, 1, N // 2)
    m = enc.embed_inverse(z, N)
    for k in (1, 3, 7):
        g = pow(5, k, 2 * N)
        mg = np.zeros(N)
        for i in range(N):
            j = i * g % (2 * N)
            if j < N:
                mg[j] = m[i]
            else:
                mg[j - N] = -m[i]
        assert np.allclose(enc.embed(mg, N), np.roll(z, -k), atol=1e-12)


def test_encrypt_decrypt_roundtrip(small):
    prm, keys = small
    z = rng.uniform(-1, 1, prm.M)
    pt = enc.encode(prm, z, prm.scale, prm.L - 1)
    ct = ckks.encrypt(prm, 3, 0, keys.s, pt)
    assert np.abs(enc.decode(prm, ckks.decrypt(prm, keys.s, ct)) - z).max() < 1e-9


def test_rescale_is_rounded_division(small):
    prm, keys = small
    lv = 3
    mods = prm.q_level(lv)
    c = [int(x) for x in rng.integers(0, 2 ** 63, prm.N, dtype=np.uint64)]
    Q = 1
    for m in mods:
        Q *= m
    c = [(x * 0x5851F42D4C957F2D) % Q for x in c]
    rows = np.array([[x % m for x in c] for m in mods], dtype=np.uint64)
    ct = ckks.Ciphertext(rows, rows.copy(), lv, 1.0)
    out = ckks.rescale(prm, ct)
    ql = prm.q[lv]
    for j in range(prm.N):
        want = (c[j] + ql // 2) // ql
        got = nt.crt([int(out.c0[i][j]) for i in range(lv)], mods[:lv])
        assert got == want % (Q // ql)


def test_mod_down_is_rounded_division_up_to_bconv_overflow(small):
    prm, keys = small
    lv = 2
    basis = ckks.ext_basis(prm, lv)
    PQ = 1
    for m in basis:
        PQ *= m
    P = prm.P
    xs = [(int(v) * 0x9E3779B97F4A7C15) % PQ for v in rng.integers(0, 2 ** 63, prm.N, dtype=np.uint64)]
    x = np.array([[v % m for v in xs] for m in basis], dtype=np.uint64)
    out = ckks.mod_down(prm, x, lv)
    Qs = prm.q_level(lv)
    Q = 1
    for m in Qs:
        Q *= m
    for j, v in enumerate(xs):
        got = nt.crt([int(out[i][j]) for i in range(lv + 1)], Qs)
        r = (v + P // 2) // P
        # exact up to the fast base conversion overflow u in [0, alpha)
        assert any((r - u - got) % Q == 0 for u in range(prm.alpha))


def test_rotation_is_left_shift_of_slots(small):
    prm, keys = small
    z = rng.uniform(-1, 1, prm.M)
    ct = ckks.encrypt(prm, 3, 1, keys.s, enc.encode(prm, z, prm.scale, prm.L - 1))
    steps = [1, 2, 3, 5, -1, -7, 8]
    outs = ckks.rotate_hoisted(prm, keys, ct, steps)
    for k, o in zip(steps, outs):
        d = enc.decode(prm, ckks.decrypt(prm, keys.s, o))
        assert np.abs(d - np.roll(z, -k)).max() < 1e-7
        single = ckks.rotate(prm, keys, ct, k)
        assert np.array_equal(single.c0, o.c0) and np.array_equal(single.c1, o.c1)
    # Rot_2 o Rot_3 = Rot_5 in the slots
    r23 = ckks.rotate(prm, keys, ckks.rotate(prm, keys, ct, 2), 3)
    d = enc.decode(prm, ckks.decrypt(prm, keys.s, r23))
    assert np.abs(d - np.roll(z, -5)).max() < 1e-7
    with pytest.raises(KeyError):
        ckks.rotate(prm, keys, ct, 4)


def test_plain_and_scalar_mac_and_square(small):
    prm, keys = small
    lv = prm.L - 1
    z1, z2 = rng.uniform(-1, 1, prm.M), rng.uniform(-1, 1, prm.M)
    p1, p2 = rng.uniform(-1, 1, prm.M), rng.uniform(-1, 1, prm.M)
    c1 = ckks.encrypt(prm, 3, 10, keys.s, enc.encode(prm, z1, prm.scale, lv))
    c2 = ckks.encrypt(prm, 3, 11, keys.s, enc.encode(prm, z2, prm.scale, lv))
    q = prm.q[lv]
    pts = [enc.encode(prm, p1, float(q), lv), enc.encode(prm, p2, float(q), lv)]
    acc = ckks.pt_mul_acc(prm, ckks.zero_ct(prm, lv, prm.scale * q), [c1, c2], pts)
    d = enc.decode(prm, ckks.decrypt(prm, keys.s, ckks.rescale(prm, acc)))
    assert np.abs(d - (z1 * p1 + z2 * p2)).max() < 1e-8
    w = [0.25, -0.75]
    ints = [enc.encode_const(x, float(q)) for x in w]
    acc = ckks.scalar_mul_acc(prm, ckks.zero_ct(prm, lv, prm.scale * q), [c1, c2], ints)
    d = enc.decode(prm, ckks.decrypt(prm, keys.s, ckks.rescale(prm, acc)))
    assert np.abs(d - (0.25 * z1 - 0.75 * z2)).max() < 1e-8
    sq = ckks.ct_mul_relin(prm, keys, c1, c1)
    d = enc.decode(prm, ckks.decrypt(prm, keys.s, sq))
    assert np.abs(d - z1 * z1).max() < 1e-8


def test_switching_key_decrypts_to_gadget(small):
    """b_j + a_j s = e_j + [q_i in digit j] P s' on every prime of the key basis."""
    prm, keys = small
    key = keys.relin
    basis = prm.q + prm.p
    s_rns = ckks.small_to_rns(keys.s, basis)
    s2 = ckks.poly_mul(s_rns, s_rns, basis, prm)
    for j, digit in enumerate(prm.digits(prm.L - 1)):
        lhs = ckks.poly_add(key.b[j], ckks.poly_mul(key.a[j], s_rns, basis, prm), basis)
        for i, m in enumerate(basis):
            want = np.zeros(prm.N, dtype=np.uint64) if i not in digit else \
                np.array([int(v) * (prm.P % m) % m for v in s2[i]], dtype=np.uint64)
            diff = [(int(a) - int(b)) % m for a, b in zip(lhs[i], want)]
            diff = [d - m if d > m // 2 else d for d in diff]
            assert max(abs(d) for d in diff) <= 21


def test_masked_rotation_sum_slots_and_precision(small):
    """Double hoisting: sum_k Rot_k(ct) (.) m_k with the mask products on the
    key basis before one ModDown decodes to sum_k roll(z, -k) * m_k, at least
    as precisely as the form with one ModDown per rotation."""
    prm, keys = small
    z = rng.uniform(-1, 1, prm.M)
    lv = prm.L - 1
    ct = ckks.encrypt(prm, 3, 0, keys.s, enc.encode(prm, z, prm.scale, lv))
    steps = [1, 2, -7, 5]
    ms = [rng.uniform(-1, 1, prm.M) for _ in steps]
    sM = float(prm.q[lv])
    out = ckks.rotate_masked_sum(prm, keys, ct, steps, [enc.encode_ext(prm, m, sM, lv) for m in ms])
    assert out.c0.shape == (lv + 1, prm.N) and out.c1.shape == (lv + 1, prm.N)
    out.scale = prm.scale * sM
    got = np.real(enc.decode(prm, ckks.decrypt(prm, keys.s, ckks.rescale(prm, out))))
    want = sum(np.roll(z, -k) * m for k, m in zip(steps, ms))
    err = np.max(np.abs(got - want))
    assert err < 1e-8
    rots = ckks.rotate_hoisted(prm, keys, ct, steps)
    acc = ckks.pt_mul_acc(prm, ckks.zero_ct(prm, lv, prm.scale * sM), rots,
                          [enc.encode(prm, m, sM, lv) for m in ms])
    got1 = np.real(enc.decode(prm, ckks.decrypt(prm, keys.s, ckks.rescale(prm, acc))))
    assert err <= 2 * np.max(np.abs(got1 - want))
    # the extended encoding reduces the same integers over Q_l and P
    m_ext = enc.encode_ext(prm, ms[0], sM, lv)
    m_q = enc.encode(prm, ms[0], sM, lv).m
    assert np.array_equal(m_ext[: lv + 1], m_q) and m_ext.shape[0] == lv + 1 + prm.alpha
    with pytest.raises(ValueError):
        ckks.rotate_masked_sum(prm, keys, ct, [0], [m_ext])


def test_rotation_sum_one_moddown(small):
    """sum_g Rot_{k_g}(ct_g) over distinct ciphertexts with one ModDown: with one
    term it is the rotation itself word for word; with several it decodes to
    sum_g roll(z_g, -k_g), and its words differ from the sum of separate
    rotations only by the ModDown roundings (a difference that decrypts to a
    few units, far below the scale)."""
    prm, keys = small
    lv = prm.L - 1
    zs = [rng.uniform(-1, 1, prm.M) for _ in range(3)]
    cts = [ckks.encrypt(prm, 30 + i, i, keys.s, enc.encode(prm, z, prm.scale, lv)) for i, z in enumerate(zs)]
    one = ckks.rotate_sum(prm, keys, [cts[0]], [5])
    ref = ckks.rotate(prm, keys, cts[0], 5)
    assert np.array_equal(one.c0, ref.c0) and np.array_equal(one.c1, ref.c1)
    steps = [1, -7, 8]
    out = ckks.rotate_sum(prm, keys, cts, steps)
    got = np.real(enc.decode(prm, ckks.decrypt(prm, keys.s, out)))
    want = sum(np.roll(z, -k) for z, k in zip(zs, steps))
    assert np.max(np.abs(got - want)) < 1e-8
    sep = None
    for c, k in zip(cts, steps):
        r = ckks.rotate(prm, keys, c, k)
        sep = r if sep is None else ckks.add(prm, sep, r)
    assert not np.array_equal(sep.c0, out.c0)   # three roundings against one
    qs = prm.q_level(lv)
    diff = ckks.Ciphertext(c0=ckks.poly_sub(out.c0, sep.c0, qs), c1=ckks.poly_sub(out.c1, sep.c1, qs), level=lv,
                           scale=prm.scale)
    d = ckks.to_signed_coeffs(prm, ckks.decrypt(prm, keys.s, diff))
    assert max(abs(v) for v in d) < 2 ** 20
    with pytest.raises(ValueError):
        ckks.rotate_sum(prm, keys, [cts[0]], [0])


def _negacyclic_mod(a, b, q):
    """Brute-force negacyclic product mod q in Python integers."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += ai * int(b[j])
            else:
                out[k - n] -= ai * int(b[j])
    return [x % q for x in out]


def test_seeded_ciphertext_rebuilt_from_its_seed_decrypts_to_small_error(small):
    """A ciphertext whose uniform part comes from a public seed (Sec. 2.1's
    (-a s + e + m, a) with a rebuilt by the server from (a_seed, ct_id) alone):
    c0 + a s - m, the product taken by brute force, is one integer of magnitude
    at most 21 (a centred binomial of 21 coin pairs) in every residue; the second
    polynomial is exactly the rebuilt a; the error's seed changes c0 only by the
    difference of two such errors."""
    prm, keys = small
    lv = prm.L - 1
    z = rng.uniform(-1, 1, prm.M)
    pt = enc.encode(prm, z, prm.scale, lv)
    ct = ckks.encrypt(prm, 3, 17, keys.s, pt, a_seed=12345)
    a = ckks.seeded_uniform(prm, 12345, 17, lv)
    assert np.array_equal(ct.c1, a)
    s = [int(v) for v in keys.s]
    errs = []
    for i, q in enumerate(prm.q_level(lv)):
        As = _negacyclic_mod(a[i], s, q)
        e = [(int(ct.c0[i][j]) + As[j] - int(pt.m[i][j])) % q for j in range(prm.N)]
        errs.append([v - q if v > q // 2 else v for v in e])
    assert all(r == errs[0] for r in errs[1:])
    assert max(abs(v) for v in errs[0]) <= 21 and any(v != 0 for v in errs[0])
    # another error seed, same public seed: same a, c0 moves by a difference of errors
    ct2 = ckks.encrypt(prm, 4, 17, keys.s, pt, a_seed=12345)
    assert np.array_equal(ct2.c1, a)
    q0 = prm.q[0]
    d = [(int(x) - int(y)) % q0 for x, y in zip(ct.c0[0], ct2.c0[0])]
    assert max(min(v, q0 - v) for v in d) <= 42 and any(v != 0 for v in d)
    # the unseeded form draws a from the error's seed
    assert np.array_equal(ckks.encrypt(prm, 3, 17, keys.s, pt).c1, ckks.seeded_uniform(prm, 3, 17, lv))
    assert np.array_equal(ckks.encrypt(prm, 3, 17, keys.s, pt).c0,
                          ckks.encrypt(prm, 3, 17, keys.s, pt, a_seed=3).c0)


def test_seeded_uniform_residues_are_uniform():
    """Each residue of the rebuilt uniform part is a 128-bit word reduced mod q:
    over the 2^13 coefficients of each of four primes its mean is q/2 within five
    standard errors, and each of its ten low bits is set half the time within
    five standard errors."""
    prm = Params(log_n=13, n_q=4, q_bits=50, n_p=1, p_bits=60)
    a = ckks.seeded_uniform(prm, 2024, 5, prm.L - 1)
    for i, q in enumerate(prm.q_level(prm.L - 1)):
        x = a[i].astype(np.float64) / q
        n = x.size
        assert (a[i] < q).all()
        assert abs(x.mean() - 0.5) < 5 / np.sqrt(12 * n)
        for b in range(10):
            f = ((a[i] >> np.uint64(b)) & np.uint64(1)).mean()
            assert abs(f - 0.5) < 5 * 0.5 / np.sqrt(n)
