"""Pins of the oracle's arithmetic against definitions it does not share code
with: Python big integers, brute-force convolution, direct evaluation, a
published test vector."""
import os

import numpy as np
import pytest

from oracle import _ffi, ntheory as nt, sampler
from oracle.params import Params

GOLD = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(2024)


def test_mulmod_matches_python_integers():
    for bits in (30, 50, 60, 62):
        q = nt.ntt_primes(bits, 1, 2 ** 14)[0]
        a = rng.integers(0, q, 2000, dtype=np.uint64)
        b = rng.integers(0, q, 2000, dtype=np.uint64)
        got = _ffi.vec_mul(a, b, q)
        want = np.array([int(x) * int(y) % q for x, y in zip(a, b)], dtype=np.uint64)
        assert np.array_equal(got, want)
        assert _ffi.mulmod(q - 1, q - 1, q) == 1


def test_miller_rabin_against_trial_division():
    def trial(n):
        if n < 2:
            return False
        i = 2
        while i * i <= n:
            if n % i == 0:
                return False
            i += 1
        return True
    for n in range(0, 5000):
        assert nt.is_prime(n) == trial(n)
    # Carmichael numbers and a strong pseudoprime to base 2
    for n in (561, 1105, 1729, 2047, 3215031751, 3825123056546413051):
        assert not nt.is_prime(n)


@pytest.mark.parametrize("log_n", [4, 13, 16])
def test_prime_chain_definition(log_n):
    prm = Params(log_n=log_n, n_q=8, q_bits=50, n_p=2, p_bits=60)
    two_n = 2 * prm.N
    assert prm.q == sorted(prm.q, reverse=True)
    for q in prm.q:
        assert q < 2 ** 50 and q > 2 ** 49 and q % two_n == 1 and nt.is_prime(q)
    for p in prm.p:
        assert p < 2 ** 60 and p > 2 ** 59 and p % two_n == 1 and nt.is_prime(p)
    # no larger admissible prime was skipped
    x = prm.q[0] + two_n
    while x < 2 ** 50:
        assert not nt.is_prime(x)
        x += two_n
    for m in prm.q + prm.p:
        psi = prm.psi[m]
        assert pow(psi, prm.N, m) == m - 1 and pow(psi, two_n, m) == 1


@pytest.mark.parametrize("n", [4, 8, 16, 64])
def test_ntt_negacyclic_product_equals_brute_force(n):
    q = nt.ntt_primes(50, 1, 2 * n)[0]
    psi = nt.primitive_root_2n(q, 2 * n)
    a = rng.integers(0, q, n, dtype=np.uint64)
    b = rng.integers(0, q, n, dtype=np.uint64)
    # definition: sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j, in Python integers
    want = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                want[i + j] += int(a[i]) * int(b[j])
            else:
                want[i + j - n] -= int(a[i]) * int(b[j])
    want = np.array([w % q for w in want], dtype=np.uint64)
    assert np.array_equal(_ffi.negacyclic_mul(a, b, q, psi), want)
    assert np.array_equal(_ffi.negacyclic_mul_naive(a, b, q), want)


def test_ntt_is_evaluation_at_odd_powers_and_invertible():
    n = 32
    q = nt.ntt_primes(60, 1, 2 * n)[0]
    psi = nt.primitive_root_2n(q, 2 * n)
    a = rng.integers(0, q, n, dtype=np.uint64)
    f = _ffi.ntt_fwd(a, q, psi)
    for i in range(n):
        x = pow(psi, 2 * i + 1, q)
        assert int(f[i]) == sum(int(a[j]) * pow(x, j, q) for j in range(n)) % q
    assert np.array_equal(_ffi.ntt_inv(f, q, psi), a)
    big = Params(log_n=16, n_q=1, q_bits=50, n_p=1, p_bits=60)
    q = big.q[0]
    a = rng.integers(0, q, big.N, dtype=np.uint64)
    assert np.array_equal(_ffi.ntt_inv(_ffi.ntt_fwd(a, q, big.psi[q]), q, big.psi[q]), a)


def test_automorphism_definition_and_composition():
    n = 16
    q = nt.ntt_primes(50, 1, 2 * n)[0]
    a = rng.integers(0, q, n, dtype=np.uint64)
    for g in (3, 5, 25, 2 * n - 1):
        out = _ffi.automorph(a, g, q)
        want = [0] * n
        for i in range(n):
            k = i * g % (2 * n)
            if k < n:
                want[k] = int(a[i])
            else:
                want[k - n] = (q - int(a[i])) % q
        assert list(map(int, out)) == want
    g, h = 5, 13
    assert np.array_equal(_ffi.automorph(_ffi.automorph(a, g, q), h, q), _ffi.automorph(a, g * h % (2 * n), q))


def test_fast_bconv_error_is_multiple_of_source_product():
    prm = Params(log_n=6, n_q=4, q_bits=50, n_p=2, p_bits=60)
    src = prm.q[:3]
    B = src[0] * src[1] * src[2]
    xs = [int(v) for v in rng.integers(0, 2 ** 62, 64, dtype=np.uint64)]
    xs = [(x * 0x9E3779B97F4A7C15 + 12345) % B for x in xs]
    rows = np.array([[x % b for x in xs] for b in src], dtype=np.uint64)
    from oracle.ckks import fast_bconv
    for p in prm.p:
        out = fast_bconv(rows, src, [p])[0]
        for j, x in enumerate(xs):
            # FastBConv returns x + u B for some u in [0, k) (k = #source primes)
            ok = [(x + u * B) % p for u in range(len(src))]
            assert int(out[j]) in ok


def test_chacha20_rfc8439_vector():
    vals = {}
    with open(os.path.join(GOLD, "chacha20_rfc8439_2_3_2.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *rest = line.split()
            vals[k] = rest
    key = np.array([int(x, 16) for x in vals["key"]], dtype=np.uint32)
    nonce = np.array([int(x, 16) for x in vals["nonce"]], dtype=np.uint32)
    out = _ffi.chacha20_block(key, int(vals["counter"][0]), nonce)
    assert [int(x) for x in out] == [int(x, 16) for x in vals["out"]]


def test_sampler_distributions():
    t = sampler.ternary(5, (sampler.SK, 0, 0), 1 << 16)
    assert set(np.unique(t)) == {-1, 0, 1}
    assert abs(np.mean(t == 0) - 1 / 3) < 0.01
    e = sampler.cbd21(5, (sampler.CT_E, 0, 0), 1 << 16)
    assert np.abs(e).max() <= 21
    assert abs(e.mean()) < 0.05 and abs(e.var() - 10.5) < 0.3
    q = Params(log_n=4, n_q=1, q_bits=50, n_p=1, p_bits=60).q[0]
    u = sampler.uniform(5, (sampler.CT_A, 0, 0), 4096, q)
    # the 128-bit to mod-q map, spot-checked with Python integers
    w = sampler.stream_words(5, (sampler.CT_A, 0, 0), 16)
    for j in range(4):
        x = sum(int(w[4 * j + i]) << (32 * i) for i in range(4))
        assert int(u[j]) == x % q
    assert u.max() < q and abs(u.mean() / q - 0.5) < 0.02
