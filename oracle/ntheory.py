"""Number theory for the oracle, in Python integers (test infrastructure only).

Primes for the RNS chain (Sec. 2.1: Q is a product of word-sized primes q_i):
the `count` largest primes below 2^bits with p = 1 (mod 2N), in descending
order, so that the ring Z_p[X]/(X^N+1) has a negacyclic NTT.
"""
from __future__ import annotations

from typing import List

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (the first 12 prime bases)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(bits: int, count: int, two_n: int, exclude=()) -> List[int]:
    """The `count` largest primes p < 2^bits with p = 1 (mod two_n), descending."""
    out = []
    p = ((1 << bits) - 1) // two_n * two_n + 1
    if p >= (1 << bits):
        p -= two_n
    while len(out) < count:
        if p < 2:
            raise ValueError("not enough primes")
        if p not in exclude and is_prime(p):
            out.append(p)
        p -= two_n
    return out


def primitive_root_2n(q: int, two_n: int) -> int:
    """A primitive two_n-th root of unity mod q: x^((q-1)/two_n) for the first
    x = 2, 3, ... whose power has order exactly two_n (psi^(N) = -1)."""
    assert (q - 1) % two_n == 0
    e = (q - 1) // two_n
    x = 2
    while True:
        psi = pow(x, e, q)
        if pow(psi, two_n // 2, q) == q - 1:
            return psi
        x += 1


def inv(a: int, q: int) -> int:
    return pow(a % q, -1, q)


def crt(residues, moduli) -> int:
    """The unique x in [0, prod moduli) with x = r_i mod m_i."""
    m = 1
    for mi in moduli:
        m *= mi
    x = 0
    for r, mi in zip(residues, moduli):
        mh = m // mi
        x += int(r) * mh * inv(mh, mi)
    return x % m


def center(x: int, m: int) -> int:
    """Representative of x mod m in (-m/2, m/2]."""
    x %= m
    return x - m if x > m // 2 else x
