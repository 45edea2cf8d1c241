"""Randomness of keys and ciphertexts, drawn from ChaCha20 (RFC 8439) streams.

Definition (shared by every implementation of the scheme, each written
independently):
  key      = 32-bit words (seed mod 2^32, seed >> 32, 0, 0, 0, 0, 0, 0)
  nonce    = three 32-bit words naming the stream (below)
  counter  = block index 0, 1, 2, ... ; a stream is its blocks' 16 words in order
  uniform mod q, coefficient j : words 4j..4j+3 read as a little-endian 128-bit
                                 integer, reduced mod q
  ternary, coefficient j       : x = words 2j, 2j+1 as a 64-bit integer; (x mod 3) - 1
  CBD(21), coefficient j       : x as above; popcount(x & (2^21-1)) - popcount((x >> 21) & (2^21-1))
Streams (nonce words):
  secret key                      (1, 0, 0)
  switching key 'a', tag T, digit j, basis index i   (2, T, j * 65536 + i)
  switching key 'e', tag T, digit j                  (3, T, j)
  ciphertext 'a', id c, prime index i                (4, c, i)
  ciphertext 'e', id c                               (5, c, 0)
The tag T of a rotation key is its Galois element; the relinearisation key has T = 0.
Basis index i counts Q primes 0..L-1 then special primes L..L+alpha-1.
"""
from __future__ import annotations

import numpy as np

from . import _ffi

SK, SWK_A, SWK_E, CT_A, CT_E = 1, 2, 3, 4, 5


def key_words(seed: int) -> np.ndarray:
    seed &= (1 << 64) - 1
    return np.array([seed & 0xFFFFFFFF, seed >> 32, 0, 0, 0, 0, 0, 0], dtype=np.uint32)


def stream_words(seed: int, nonce, n_words: int) -> np.ndarray:
    nblocks = -(-n_words // 16)
    w = _ffi.chacha20_stream(key_words(seed), np.array(nonce, dtype=np.uint32), 0, nblocks)
    return w[:n_words]


def uniform(seed: int, nonce, n: int, q: int) -> np.ndarray:
    return _ffi.uniform_from_words(stream_words(seed, nonce, 4 * n), q)


def _u64(seed, nonce, n):
    w = stream_words(seed, nonce, 2 * n).astype(np.uint64)
    return w[0::2] | (w[1::2] << np.uint64(32))


def ternary(seed: int, nonce, n: int) -> np.ndarray:
    x = _u64(seed, nonce, n)
    return (x % np.uint64(3)).astype(np.int64) - 1


def _popcount(x: np.ndarray) -> np.ndarray:
    c = np.zeros(x.shape, dtype=np.int64)
    for b in range(21):
        c += ((x >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return c


def cbd21(seed: int, nonce, n: int) -> np.ndarray:
    x = _u64(seed, nonce, n)
    m = np.uint64((1 << 21) - 1)
    return _popcount(x & m) - _popcount((x >> np.uint64(21)) & m)
