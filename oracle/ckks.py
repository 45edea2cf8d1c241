"""RNS-CKKS scheme in the oracle (test infrastructure only).

Public results are in coefficient form: a polynomial over primes m_0..m_{k-1}
is a uint64 array of shape (k, N), row i holding residues mod m_i.  Ring
products go through the C core's NTT (a library step; the result is the
negacyclic product by definition).

Paper Sec. 2.1 fixes what is computed: a ciphertext c in R_Q^2 decrypts as
c . sk = m + e (mod Q), Q = q_0...q_{L-1}; every multiplication consumes one
level; rotation by k maps the slots (v_0, ..., v_{M-1}) to
(v_k, ..., v_{M-1}, v_0, ..., v_{k-1}).  The scheme's internals that the paper
leaves to its library follow the standard hybrid key switching (Han-Ki 2020):
  ModUp_j    digit j's residues extended to the other active Q primes and P
             by fast base conversion;
  inner      acc_{0,1} = sum_j D_j * swk_j;
  ModDown    round(x / P): y = [x + h]_P with h = floor(P/2), then
             (x_Q + h - FastBConv_{P->Q}(y)) * P^-1 mod q_i;
  rotation   canonical form: ModUp first, then the automorphism on each D_j,
             so hoisted and single rotations give the same words;
  rescale    round(c / q_l): y = (c_l + h) mod q_l with h = floor(q_l/2), then
             (c_i + h - y) * q_l^-1 mod q_i.
A floor division would leave a +1/2 mean error on every coefficient; times
the secret that error concentrates in the slots next to zeta^(+-1), so both
divisions round.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Sequence

import numpy as np

from . import _ffi
from . import ntheory as nt
from . import sampler
from .params import Params


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclass
class Ciphertext:
    c0: np.ndarray          # (level+1, N) coefficient form
    c1: np.ndarray
    level: int
    scale: float

    def copy(self) -> "Ciphertext":
        return Ciphertext(self.c0.copy(), self.c1.copy(), self.level, self.scale)


@dataclass
class Plaintext:
    m: np.ndarray           # (level+1, N) coefficient form
    level: int
    scale: float


@dataclass
class SwitchingKey:
    b: List[np.ndarray]     # per digit: (L + alpha, N) over q_0..q_{L-1}, p_0..
    a: List[np.ndarray]
    tag: int


@dataclass
class Keys:
    s: np.ndarray                        # ternary secret, int64 (N,)
    rot: Dict[int, SwitchingKey]         # Galois element -> key
    relin: SwitchingKey = None


# ----------------------------------------------------------------------------
# ring helpers
# ----------------------------------------------------------------------------
def small_to_rns(x: np.ndarray, moduli: Sequence[int]) -> np.ndarray:
    return np.stack([_ffi.from_signed(x, m) for m in moduli])


def poly_mul(a: np.ndarray, b: np.ndarray, moduli: Sequence[int], prm: Params) -> np.ndarray:
    return np.stack([_ffi.negacyclic_mul(a[i], b[i], m, prm.psi[m]) for i, m in enumerate(moduli)])


def poly_mul_sum(pairs, moduli: Sequence[int], prm: Params) -> np.ndarray:
    """sum_k a_k * b_k in the ring, evaluated as INTT(sum_k NTT(a_k) . NTT(b_k))
    per prime (the NTT is a ring isomorphism onto pointwise products)."""
    out = []
    for i, m in enumerate(moduli):
        psi = prm.psi[m]
        acc = np.zeros(prm.N, dtype=np.uint64)
        for a, b in pairs:
            acc = _ffi.vec_add(acc, _ffi.vec_mul(_ffi.ntt_fwd(a[i], m, psi), _ffi.ntt_fwd(b[i], m, psi), m), m)
        out.append(_ffi.ntt_inv(acc, m, psi))
    return np.stack(out)


def poly_add(a, b, moduli):
    return np.stack([_ffi.vec_add(a[i], b[i], m) for i, m in enumerate(moduli)])


def poly_sub(a, b, moduli):
    return np.stack([_ffi.vec_sub(a[i], b[i], m) for i, m in enumerate(moduli)])


def poly_neg(a, moduli):
    z = np.zeros_like(a[0])
    return np.stack([_ffi.vec_sub(z, a[i], m) for i, m in enumerate(moduli)])


def automorph(a, g: int, moduli):
    return np.stack([_ffi.automorph(a[i], g, m) for i, m in enumerate(moduli)])


def galois_element(k: int, prm: Params) -> int:
    """g = 5^(k mod M) mod 2N: X -> X^g rotates the slots left by k."""
    return pow(5, k % prm.M, 2 * prm.N)


def ext_basis(prm: Params, level: int) -> List[int]:
    """Key-switching basis at `level`: active Q primes, then P primes."""
    return prm.q_level(level) + prm.p


def _key_rows(prm: Params, level: int) -> List[int]:
    return list(range(level + 1)) + list(range(prm.L, prm.L + prm.alpha))


# ----------------------------------------------------------------------------
# key generation
# ----------------------------------------------------------------------------
def gen_secret(prm: Params, seed: int) -> np.ndarray:
    return sampler.ternary(seed, (sampler.SK, 0, 0), prm.N)


def gen_switching_key(prm: Params, seed: int, s: np.ndarray, s_prime: np.ndarray, tag: int) -> SwitchingKey:
    """swk_j = (-a_j s + e_j + [q_i in digit j] * P * s', a_j) over all L + alpha
    primes.  s_prime: (L + alpha, N) residues of the target key."""
    basis = prm.q + prm.p
    s_rns = small_to_rns(s, basis)
    P = prm.P
    bs, as_ = [], []
    for j, digit in enumerate(prm.digits(prm.L - 1)):
        a = np.stack([sampler.uniform(seed, (sampler.SWK_A, tag, j * 65536 + i), prm.N, m)
                      for i, m in enumerate(basis)])
        e = sampler.cbd21(seed, (sampler.SWK_E, tag, j), prm.N)
        e_rns = small_to_rns(e, basis)
        b = poly_sub(e_rns, poly_mul(a, s_rns, basis, prm), basis)
        for i in digit:
            m = basis[i]
            b[i] = _ffi.vec_add(b[i], _ffi.vec_scale(s_prime[i], P % m, m), m)
        bs.append(b)
        as_.append(a)
    return SwitchingKey(b=bs, a=as_, tag=tag)


def gen_rotation_key(prm: Params, seed: int, s: np.ndarray, k: int) -> SwitchingKey:
    g = galois_element(k, prm)
    basis = prm.q + prm.p
    s_g = automorph(small_to_rns(s, basis), g, basis)
    return gen_switching_key(prm, seed, s, s_g, tag=g)


def gen_relin_key(prm: Params, seed: int, s: np.ndarray) -> SwitchingKey:
    basis = prm.q + prm.p
    s_rns = small_to_rns(s, basis)
    return gen_switching_key(prm, seed, s, poly_mul(s_rns, s_rns, basis, prm), tag=0)


def keygen(prm: Params, seed: int, rot_steps: Sequence[int] = (), relin: bool = True) -> Keys:
    s = gen_secret(prm, seed)
    keys = Keys(s=s, rot={})
    for k in rot_steps:
        g = galois_element(k, prm)
        if g not in keys.rot:
            keys.rot[g] = gen_rotation_key(prm, seed, s, k)
    if relin:
        keys.relin = gen_relin_key(prm, seed, s)
    return keys


# ----------------------------------------------------------------------------
# encryption
# ----------------------------------------------------------------------------
def seeded_uniform(prm: Params, a_seed: int, ct_id: int, level: int) -> np.ndarray:
    """The uniform part a of ciphertext ct_id, as the server rebuilds it from a
    public seed: residue i is the uniform stream (CT_A, ct_id, i) keyed by a_seed,
    in coefficient form over Q_level.  A seeded ciphertext travels as (c0, a_seed,
    ct_id); its second polynomial is this array."""
    mods = prm.q_level(level)
    return np.stack([sampler.uniform(a_seed, (sampler.CT_A, ct_id, i), prm.N, m) for i, m in enumerate(mods)])


def encrypt(prm: Params, seed: int, ct_id: int, s: np.ndarray, pt: Plaintext, a_seed: int = None) -> Ciphertext:
    """Symmetric encryption (the client holds sk): (-a s + e + m, a) mod Q_level,
    e from the stream (CT_E, ct_id) of `seed`, a from seeded_uniform of a_seed
    (default: seed).  A public a_seed lets the client send c0 alone; it must key
    no other stream (the secret and the errors are drawn under their own seeds)."""
    mods = prm.q_level(pt.level)
    a = seeded_uniform(prm, seed if a_seed is None else a_seed, ct_id, pt.level)
    e = sampler.cbd21(seed, (sampler.CT_E, ct_id, 0), prm.N)
    c0 = poly_add(poly_sub(small_to_rns(e, mods), poly_mul(a, small_to_rns(s, mods), mods, prm), mods),
                  pt.m, mods)
    return Ciphertext(c0=c0, c1=a, level=pt.level, scale=pt.scale)


def decrypt(prm: Params, s: np.ndarray, ct: Ciphertext) -> Plaintext:
    mods = prm.q_level(ct.level)
    m = poly_add(ct.c0, poly_mul(ct.c1, small_to_rns(s, mods), mods, prm), mods)
    return Plaintext(m=m, level=ct.level, scale=ct.scale)


def to_signed_coeffs(prm: Params, pt: Plaintext) -> List[int]:
    """CRT-reconstruct and center each coefficient (Python integers)."""
    mods = prm.q_level(pt.level)
    Q = 1
    for m in mods:
        Q *= m
    return [nt.center(nt.crt([int(pt.m[i][j]) for i in range(len(mods))], mods), Q)
            for j in range(prm.N)]


# ----------------------------------------------------------------------------
# base conversion, ModUp, ModDown
# ----------------------------------------------------------------------------
def fast_bconv(rows: np.ndarray, src: Sequence[int], dst: Sequence[int]) -> np.ndarray:
    """sum_i [x_i (B/b_i)^-1]_{b_i} (B/b_i) mod p for each p in dst (non-centred)."""
    B = 1
    for b in src:
        B *= b
    hats = [B // b for b in src]
    hat_inv = np.array([nt.inv(h, b) for h, b in zip(hats, src)], dtype=np.uint64)
    out = []
    for p in dst:
        hat_mod_p = np.array([h % p for h in hats], dtype=np.uint64)
        out.append(_ffi.fast_bconv(rows, np.array(src, dtype=np.uint64), hat_inv, hat_mod_p, p))
    return np.stack(out)


def mod_up(prm: Params, a: np.ndarray, level: int, digit: List[int]) -> np.ndarray:
    """Digit `digit` (indices into q) of `a` (level+1, N) extended to the key
    basis (active Q primes then P): own residues copied, the rest converted."""
    basis = ext_basis(prm, level)
    src = [prm.q[i] for i in digit]
    others = [i for i in range(len(basis)) if i not in digit]
    conv = fast_bconv(a[digit], src, [basis[i] for i in others])
    out = np.empty((len(basis), prm.N), dtype=np.uint64)
    for r, i in enumerate(digit):
        out[i] = a[i]
    for r, i in enumerate(others):
        out[i] = conv[r]
    return out


def mod_down(prm: Params, x: np.ndarray, level: int) -> np.ndarray:
    """round(x / P) over the active Q primes: y = [x + floor(P/2)]_P,
    out_i = (x_i + floor(P/2) - FastBConv_{P->q_i}(y)) * P^-1 mod q_i."""
    qs = prm.q_level(level)
    k = len(qs)
    P = prm.P
    h = P // 2
    y = np.stack([_ffi.vec_add(x[k + j], np.full(prm.N, h % p, dtype=np.uint64), p)
                  for j, p in enumerate(prm.p)])
    conv = fast_bconv(y, prm.p, qs)
    out = np.empty((k, prm.N), dtype=np.uint64)
    for i, q in enumerate(qs):
        xi = _ffi.vec_add(x[i], np.full(prm.N, h % q, dtype=np.uint64), q)
        out[i] = _ffi.vec_scale(_ffi.vec_sub(xi, conv[i], q), nt.inv(P, q), q)
    return out


def _key_inner(prm: Params, D: List[np.ndarray], key: SwitchingKey, level: int):
    """acc_{0,1} = sum_j D_j * swk_j over the key basis at `level`."""
    basis = ext_basis(prm, level)
    rows = _key_rows(prm, level)
    acc0 = poly_mul_sum([(Dj, key.b[j][rows]) for j, Dj in enumerate(D)], basis, prm)
    acc1 = poly_mul_sum([(Dj, key.a[j][rows]) for j, Dj in enumerate(D)], basis, prm)
    return acc0, acc1


def key_switch(prm: Params, d: np.ndarray, level: int, key: SwitchingKey):
    """(u0, u1) with u0 + u1 s ~ d s' for the key's target s'."""
    D = [mod_up(prm, d, level, dg) for dg in prm.digits(level)]
    acc0, acc1 = _key_inner(prm, D, key, level)
    return mod_down(prm, acc0, level), mod_down(prm, acc1, level)


def rotate_hoisted(prm: Params, keys: Keys, ct: Ciphertext, steps: Sequence[int]) -> List[Ciphertext]:
    """Rotations of one ciphertext by each k in `steps`, sharing one ModUp:
    D_j = ModUp_j(c1); per k: acc = sum_j sigma_g(D_j) swk_{g,j};
    out = (sigma_g(c0) + ModDown(acc0), ModDown(acc1))."""
    lv = ct.level
    qs = prm.q_level(lv)
    basis = ext_basis(prm, lv)
    D = [mod_up(prm, ct.c1, lv, dg) for dg in prm.digits(lv)]
    outs = []
    for k in steps:
        if k % prm.M == 0:
            outs.append(ct.copy())
            continue
        g = galois_element(k, prm)
        if g not in keys.rot:
            raise KeyError("no rotation key for step %d" % k)
        Dg = [automorph(Dj, g, basis) for Dj in D]
        acc0, acc1 = _key_inner(prm, Dg, keys.rot[g], lv)
        c0 = poly_add(automorph(ct.c0, g, qs), mod_down(prm, acc0, lv), qs)
        outs.append(Ciphertext(c0=c0, c1=mod_down(prm, acc1, lv), level=lv, scale=ct.scale))
    return outs


def rotate(prm: Params, keys: Keys, ct: Ciphertext, k: int) -> Ciphertext:
    return rotate_hoisted(prm, keys, ct, [k])[0]


def rotate_masked_sum(prm: Params, keys: Keys, ct: Ciphertext, steps: Sequence[int],
                      masks_ext: Sequence[np.ndarray]) -> Ciphertext:
    """sum_k Rot_k(ct) (.) m_k for nonzero steps k, with the mask products taken
    on the key-switching basis before a single ModDown (double hoisting):
    D_j = ModUp_j(c1);  A = sum_k KeyInner(sigma_gk(D)) * m_k  over Q_l and P;
    out = (ModDown(A_0) + sum_k sigma_gk(c0) * m_k,  ModDown(A_1)).
    masks_ext[k]: the mask's integer coefficients reduced over Q_l then P
    (rows = ext_basis).  No rescale; scale = ct.scale * (mask scale)."""
    lv = ct.level
    qs = prm.q_level(lv)
    basis = ext_basis(prm, lv)
    D = [mod_up(prm, ct.c1, lv, dg) for dg in prm.digits(lv)]
    a0_terms, a1_terms, c0_terms = [], [], []
    for k, m in zip(steps, masks_ext):
        if k % prm.M == 0:
            raise ValueError("the identity shift is a plain mask product, not a key switch")
        g = galois_element(k, prm)
        if g not in keys.rot:
            raise KeyError("no rotation key for step %d" % k)
        Dg = [automorph(Dj, g, basis) for Dj in D]
        acc0, acc1 = _key_inner(prm, Dg, keys.rot[g], lv)
        a0_terms.append((acc0, m))
        a1_terms.append((acc1, m))
        c0_terms.append((automorph(ct.c0, g, qs), m[: lv + 1]))
    A0 = poly_mul_sum(a0_terms, basis, prm)
    A1 = poly_mul_sum(a1_terms, basis, prm)
    c0 = poly_add(mod_down(prm, A0, lv), poly_mul_sum(c0_terms, qs, prm), qs)
    return Ciphertext(c0=c0, c1=mod_down(prm, A1, lv), level=lv, scale=ct.scale)


def rotate_sum(prm: Params, keys: Keys, cts: Sequence[Ciphertext], steps: Sequence[int]) -> Ciphertext:
    """sum_g Rot_{k_g}(ct_g) over distinct ciphertexts with one ModDown (the
    giant-step sum of the baby-step/giant-step SpIntra-CA form):
    A = sum_g KeyInner(sigma_g(ModUp(c1_g))) over Q_l and P;
    out = (ModDown(A_0) + sum_g sigma_g(c0_g),  ModDown(A_1)).
    With one term this is rotate() word for word.  All inputs share level and
    scale; every step is a nonzero rotation."""
    if not cts or len(cts) != len(steps):
        raise ValueError("one step per ciphertext, at least one")
    lv = cts[0].level
    qs = prm.q_level(lv)
    basis = ext_basis(prm, lv)
    A0 = np.zeros((len(basis), prm.N), dtype=np.uint64)
    A1 = np.zeros_like(A0)
    c0 = np.zeros((lv + 1, prm.N), dtype=np.uint64)
    for ct, k in zip(cts, steps):
        if ct.level != lv:
            raise ValueError("level mismatch")
        if k % prm.M == 0:
            raise ValueError("the identity shift is a plain addition, not a key switch")
        g = galois_element(k, prm)
        if g not in keys.rot:
            raise KeyError("no rotation key for step %d" % k)
        D = [mod_up(prm, ct.c1, lv, dg) for dg in prm.digits(lv)]
        acc0, acc1 = _key_inner(prm, [automorph(Dj, g, basis) for Dj in D], keys.rot[g], lv)
        A0 = poly_add(A0, acc0, basis)
        A1 = poly_add(A1, acc1, basis)
        c0 = poly_add(c0, automorph(ct.c0, g, qs), qs)
    return Ciphertext(c0=poly_add(mod_down(prm, A0, lv), c0, qs), c1=mod_down(prm, A1, lv), level=lv,
                      scale=cts[0].scale)


# ----------------------------------------------------------------------------
# arithmetic
# ----------------------------------------------------------------------------
def rescale(prm: Params, ct: Ciphertext) -> Ciphertext:
    """Drop q_l with rounding: y = (c_l + h) mod q_l, h = floor(q_l / 2);
    c_i' = (c_i + h - y) * q_l^-1 mod q_i."""
    lv = ct.level
    if lv == 0:
        raise ValueError("cannot rescale at level 0")
    ql = prm.q[lv]
    h = ql // 2

    def one(c):
        y = _ffi.vec_add(c[lv], np.full(prm.N, h, dtype=np.uint64), ql)
        out = np.empty((lv, prm.N), dtype=np.uint64)
        for i in range(lv):
            q = prm.q[i]
            ci = _ffi.vec_add(c[i], np.full(prm.N, h % q, dtype=np.uint64), q)
            out[i] = _ffi.vec_scale(_ffi.vec_sub(ci, _ffi.vec_reduce(y, q), q), nt.inv(ql, q), q)
        return out

    return Ciphertext(c0=one(ct.c0), c1=one(ct.c1), level=lv - 1, scale=ct.scale / ql)


def drop_to(ct: Ciphertext, level: int) -> Ciphertext:
    """Level drop without division: keep the first level+1 residues."""
    return Ciphertext(ct.c0[: level + 1].copy(), ct.c1[: level + 1].copy(), level, ct.scale)


def add(prm: Params, x: Ciphertext, y: Ciphertext) -> Ciphertext:
    assert x.level == y.level
    mods = prm.q_level(x.level)
    return Ciphertext(poly_add(x.c0, y.c0, mods), poly_add(x.c1, y.c1, mods), x.level, x.scale)


def zero_ct(prm: Params, level: int, scale: float) -> Ciphertext:
    z = np.zeros((level + 1, prm.N), dtype=np.uint64)
    return Ciphertext(z, z.copy(), level, scale)


def pt_mul_acc(prm: Params, acc: Ciphertext, cts: Sequence[Ciphertext], pts: Sequence[Plaintext]) -> Ciphertext:
    """acc + sum_i pts[i] * cts[i] (no rescale)."""
    mods = prm.q_level(acc.level)
    for ct, pt in zip(cts, pts):
        assert ct.level == acc.level and pt.level == acc.level
    c0 = poly_add(acc.c0, poly_mul_sum([(pt.m, ct.c0) for ct, pt in zip(cts, pts)], mods, prm), mods)
    c1 = poly_add(acc.c1, poly_mul_sum([(pt.m, ct.c1) for ct, pt in zip(cts, pts)], mods, prm), mods)
    return Ciphertext(c0, c1, acc.level, acc.scale)


def scalar_mul_acc(prm: Params, acc: Ciphertext, cts: Sequence[Ciphertext], consts: Sequence[int]) -> Ciphertext:
    """acc + sum_i c_i * cts[i] for signed integer constants c_i (no rescale)."""
    mods = prm.q_level(acc.level)
    c0, c1 = acc.c0.copy(), acc.c1.copy()
    for ct, c in zip(cts, consts):
        assert ct.level == acc.level
        for i, m in enumerate(mods):
            cm = int(c) % m
            c0[i] = _ffi.vec_add(c0[i], _ffi.vec_scale(ct.c0[i], cm, m), m)
            c1[i] = _ffi.vec_add(c1[i], _ffi.vec_scale(ct.c1[i], cm, m), m)
    return Ciphertext(c0, c1, acc.level, acc.scale)


def ct_mul_relin(prm: Params, keys: Keys, x: Ciphertext, y: Ciphertext) -> Ciphertext:
    """(b1 b2, b1 a2 + a1 b2, a1 a2), then a1 a2 key-switched with the relin key.
    No rescale."""
    assert x.level == y.level
    lv = x.level
    mods = prm.q_level(lv)
    d0 = poly_mul(x.c0, y.c0, mods, prm)
    d1 = poly_add(poly_mul(x.c0, y.c1, mods, prm), poly_mul(x.c1, y.c0, mods, prm), mods)
    d2 = poly_mul(x.c1, y.c1, mods, prm)
    u0, u1 = key_switch(prm, d2, lv, keys.relin)
    return Ciphertext(poly_add(d0, u0, mods), poly_add(d1, u1, mods), lv, x.scale * y.scale)
