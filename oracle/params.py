"""CKKS parameter set (paper Sec. 2.1; hybrid key switching per Han-Ki 2020).

Ring degree N, M = N/2 complex slots, ciphertext modulus Q = q_0 ... q_{L-1}
(descending; a rescale drops the highest active index), special modulus
P = p_0 ... p_{alpha-1} used only inside key switching, key-switching digits of
alpha consecutive Q primes (beta = ceil(L / alpha) digits), scale Delta = 2^40.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

from . import ntheory as nt


@dataclass
class Params:
    log_n: int
    n_q: int
    q_bits: int
    n_p: int
    p_bits: int
    log_scale: int = 40
    q: List[int] = field(default_factory=list)
    p: List[int] = field(default_factory=list)
    psi: dict = field(default_factory=dict)

    def __post_init__(self):
        two_n = 2 * self.N
        if not self.q:
            self.q = nt.ntt_primes(self.q_bits, self.n_q, two_n)
        if not self.p:
            self.p = nt.ntt_primes(self.p_bits, self.n_p, two_n, exclude=set(self.q))
        for m in self.q + self.p:
            self.psi[m] = nt.primitive_root_2n(m, two_n)

    @property
    def N(self) -> int:
        return 1 << self.log_n

    @property
    def M(self) -> int:
        return self.N // 2

    @property
    def L(self) -> int:
        return self.n_q

    @property
    def alpha(self) -> int:
        return self.n_p

    @property
    def beta(self) -> int:
        return -(-self.n_q // self.n_p)

    @property
    def scale(self) -> float:
        return float(2 ** self.log_scale)

    @property
    def P(self) -> int:
        out = 1
        for m in self.p:
            out *= m
        return out

    def q_level(self, level: int) -> List[int]:
        """Active Q primes at `level` (level + 1 primes)."""
        return self.q[: level + 1]

    def digits(self, level: int) -> List[List[int]]:
        """Key-switching digits at `level`: index lists into q, alpha per digit,
        the last one truncated to the active primes."""
        act = level + 1
        return [list(range(j * self.alpha, min((j + 1) * self.alpha, act)))
                for j in range(-(-act // self.alpha))]

    @classmethod
    def from_dict(cls, d: dict) -> "Params":
        return cls(log_n=d["log_n"], n_q=d["n_q"], q_bits=d["q_bits"], n_p=d["n_p"],
                   p_bits=d["p_bits"], log_scale=d.get("log_scale", 40))
