"""CKKS canonical-embedding encoding (test infrastructure only).

Slot j of a plaintext polynomial m(X) in Z[X]/(X^N+1) is m evaluated at
zeta^(5^j), zeta = exp(i pi / N), for j < M = N/2; the conjugate slots sit at
zeta^(-5^j).  Rotating the slots left by k is X -> X^(5^k) (paper Sec. 2.1).

encode: m_i = round_half_even(scale * (2/N) Re(sum_j z_j zeta^(-5^j i))), computed
        with one FP64 FFT over the N odd powers of zeta (the direct O(N M) sum
        is kept for tiny N as the definition the FFT form is pinned against);
decode: z_j = m(zeta^(5^j)) / scale with m the centred CRT lift.
Scalar constants: c -> round_half_even(c * scale) as one integer.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import _ffi
from . import ntheory as nt
from .ckks import Plaintext
from .params import Params


def slot_roots(N: int) -> np.ndarray:
    """r_j = 5^j mod 2N for j < N/2 (the odd exponent of slot j)."""
    M = N // 2
    r = np.empty(M, dtype=np.int64)
    x = 1
    for j in range(M):
        r[j] = x
        x = x * 5 % (2 * N)
    return r


def _values_on_odd_powers(z: np.ndarray, N: int) -> np.ndarray:
    """v_s = value at zeta^(2s+1): z_j at 5^j, conj(z_j) at -5^j."""
    r = slot_roots(N)
    v = np.zeros(N, dtype=np.complex128)
    v[(r - 1) // 2] = z
    v[((2 * N - r) - 1) // 2] = np.conj(z)
    return v


def embed_inverse(z: Sequence[complex], N: int) -> np.ndarray:
    """Real coefficients m with m(zeta^(5^j)) = z_j (no scaling, no rounding)."""
    M = N // 2
    zz = np.zeros(M, dtype=np.complex128)
    zz[: len(z)] = np.asarray(z, dtype=np.complex128)
    v = _values_on_odd_powers(zz, N)
    i = np.arange(N)
    return np.real(np.exp(-1j * np.pi * i / N) * np.fft.fft(v) / N)


def embed_inverse_direct(z: Sequence[complex], N: int) -> np.ndarray:
    """The definition, O(N M): m_i = (2/N) Re(sum_j z_j zeta^(-5^j i))."""
    M = N // 2
    zz = np.zeros(M, dtype=np.complex128)
    zz[: len(z)] = np.asarray(z, dtype=np.complex128)
    r = slot_roots(N)
    i = np.arange(N)
    ang = np.exp(-1j * np.pi * np.outer(r, i) / N)      # (M, N)
    return (2.0 / N) * np.real(zz @ ang)


def embed(m: np.ndarray, N: int) -> np.ndarray:
    """Slot values of real coefficients m: z_j = sum_i m_i zeta^(5^j i)."""
    i = np.arange(N)
    w = N * np.fft.ifft(np.asarray(m, dtype=np.float64) * np.exp(1j * np.pi * i / N))
    r = slot_roots(N)
    return w[(r - 1) // 2]


def embed_direct(m: np.ndarray, N: int) -> np.ndarray:
    r = slot_roots(N)
    i = np.arange(N)
    return np.exp(1j * np.pi * np.outer(r, i) / N) @ np.asarray(m, dtype=np.float64)


def round_coeffs(x: np.ndarray) -> np.ndarray:
    """round-half-even to int64 (|x| < 2^63)."""
    return np.rint(x).astype(np.int64)


def encode(prm: Params, z: Sequence[complex], scale: float, level: int) -> Plaintext:
    m = round_coeffs(embed_inverse(z, prm.N) * scale)
    mods = prm.q_level(level)
    return Plaintext(m=np.stack([_ffi.from_signed(m, q) for q in mods]), level=level, scale=scale)


def encode_ext(prm: Params, z: Sequence[complex], scale: float, level: int) -> np.ndarray:
    """The same integer coefficients as encode(), reduced over Q_l and then the
    special primes P (the key-switching basis): rows level + 1 + alpha."""
    m = round_coeffs(embed_inverse(z, prm.N) * scale)
    return np.stack([_ffi.from_signed(m, q) for q in prm.q_level(level) + prm.p])


def encode_int(prm: Params, m: np.ndarray, level: int, scale: float) -> Plaintext:
    mods = prm.q_level(level)
    return Plaintext(m=np.stack([_ffi.from_signed(np.asarray(m, dtype=np.int64), q) for q in mods]),
                     level=level, scale=scale)


def encode_const(c: float, scale: float) -> int:
    """A scalar constant as one integer: round_half_even(c * scale)."""
    return int(np.rint(np.float64(c) * np.float64(scale)))


def decode(prm: Params, pt: Plaintext, n_slots: int = None) -> np.ndarray:
    mods = prm.q_level(pt.level)
    Q = 1
    for q in mods:
        Q *= q
    # CRT lift, centred, as floats divided by the scale
    lift = [0.0] * prm.N
    res = [list(map(int, pt.m[i])) for i in range(len(mods))]
    hats = [Q // q for q in mods]
    coef = [h * nt.inv(h, q) for h, q in zip(hats, mods)]
    for j in range(prm.N):
        x = 0
        for i in range(len(mods)):
            x += res[i][j] * coef[i]
        lift[j] = float(nt.center(x % Q, Q)) / pt.scale
    z = embed(np.array(lift), prm.N)
    return z if n_slots is None else z[:n_slots]
