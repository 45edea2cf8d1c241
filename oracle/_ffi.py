"""ctypes access to the oracle's plain C core (oracle/core.c).

Test infrastructure only.  The shared object is built by ``oracle.build``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_core.so")

_lib = None

u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
sz = ctypes.c_size_t
u64 = ctypes.c_uint64
u32 = ctypes.c_uint32


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "or_mulmod": (u64, [u64, u64, u64]),
            "or_powmod": (u64, [u64, u64, u64]),
            "or_vec_mul": (None, [u64p, u64p, u64p, sz, u64]),
            "or_vec_add": (None, [u64p, u64p, u64p, sz, u64]),
            "or_vec_sub": (None, [u64p, u64p, u64p, sz, u64]),
            "or_vec_scale": (None, [u64p, u64, u64p, sz, u64]),
            "or_vec_reduce": (None, [u64p, u64p, sz, u64]),
            "or_vec_from_signed": (None, [i64p, u64p, sz, u64]),
            "or_ntt_fwd": (None, [u64p, sz, u64, u64]),
            "or_ntt_inv": (None, [u64p, sz, u64, u64]),
            "or_negacyclic_mul": (None, [u64p, u64p, u64p, sz, u64, u64]),
            "or_negacyclic_mul_naive": (None, [u64p, u64p, u64p, sz, u64]),
            "or_automorph": (None, [u64p, u64p, sz, u64, u64]),
            "or_fast_bconv": (None, [u64p, sz, u64p, sz, u64p, u64p, u64, u64p]),
            "or_chacha20_block": (None, [u32p, u32, u32p, u32p]),
            "or_chacha20_stream": (None, [u32p, u32p, u32, sz, u32p]),
            "or_uniform_from_words": (None, [u32p, sz, u64, u64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _c(a, dtype=np.uint64):
    return np.ascontiguousarray(a, dtype=dtype)


def mulmod(a: int, b: int, q: int) -> int:
    return int(lib().or_mulmod(a, b, q))


def vec_mul(a, b, q):
    a, b = _c(a), _c(b)
    out = np.empty_like(a)
    lib().or_vec_mul(a, b, out, a.size, q)
    return out


def vec_add(a, b, q):
    a, b = _c(a), _c(b)
    out = np.empty_like(a)
    lib().or_vec_add(a, b, out, a.size, q)
    return out


def vec_sub(a, b, q):
    a, b = _c(a), _c(b)
    out = np.empty_like(a)
    lib().or_vec_sub(a, b, out, a.size, q)
    return out


def vec_scale(a, c, q):
    a = _c(a)
    out = np.empty_like(a)
    lib().or_vec_scale(a, int(c) % q, out, a.size, q)
    return out


def vec_reduce(a, q):
    a = _c(a)
    out = np.empty_like(a)
    lib().or_vec_reduce(a, out, a.size, q)
    return out


def from_signed(a, q):
    a = _c(a, np.int64)
    out = np.empty(a.shape, dtype=np.uint64)
    lib().or_vec_from_signed(a, out, a.size, q)
    return out


def ntt_fwd(a, q, psi):
    out = _c(a).copy()
    lib().or_ntt_fwd(out, out.size, q, psi)
    return out


def ntt_inv(a, q, psi):
    out = _c(a).copy()
    lib().or_ntt_inv(out, out.size, q, psi)
    return out


def negacyclic_mul(a, b, q, psi):
    a, b = _c(a), _c(b)
    out = np.empty_like(a)
    lib().or_negacyclic_mul(a, b, out, a.size, q, psi)
    return out


def negacyclic_mul_naive(a, b, q):
    a, b = _c(a), _c(b)
    out = np.empty_like(a)
    lib().or_negacyclic_mul_naive(a, b, out, a.size, q)
    return out


def automorph(a, g, q):
    a = _c(a)
    out = np.empty_like(a)
    lib().or_automorph(a, out, a.size, g, q)
    return out


def fast_bconv(rows, src, hat_inv, hat_mod_p, p):
    rows = _c(rows)
    ks, n = rows.shape
    out = np.empty(n, dtype=np.uint64)
    lib().or_fast_bconv(rows, n, _c(src), ks, _c(hat_inv), _c(hat_mod_p), p, out)
    return out


def chacha20_block(key, counter, nonce):
    out = np.empty(16, dtype=np.uint32)
    lib().or_chacha20_block(_c(key, np.uint32), counter, _c(nonce, np.uint32), out)
    return out


def chacha20_stream(key, nonce, first, nblocks):
    out = np.empty(16 * nblocks, dtype=np.uint32)
    lib().or_chacha20_stream(_c(key, np.uint32), _c(nonce, np.uint32), first, nblocks, out)
    return out


def uniform_from_words(words, q):
    words = _c(words, np.uint32)
    n = words.size // 4
    out = np.empty(n, dtype=np.uint64)
    lib().or_uniform_from_words(words, n, q, out)
    return out
