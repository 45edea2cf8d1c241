"""Seeded ciphertext words for parity cases that start in the middle of the path.

A ciphertext at level l is two polynomials of l + 1 residue rows; here every
residue is drawn uniformly from [0, q_i) with numpy's PCG64 generator, row by
row in (ciphertext, polynomial, prime) order.  No arithmetic of the method is
done here: the moduli are given by the caller."""
from __future__ import annotations

from typing import Sequence

import numpy as np


def uniform_ct_words(seed: int, moduli: Sequence[int], n: int, count: int) -> np.ndarray:
    """count ciphertexts as a uint64 array (count, 2, len(moduli), n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((count, 2, len(moduli), n), dtype=np.uint64)
    for c in range(count):
        for p in range(2):
            for i, q in enumerate(moduli):
                out[c, p, i] = rng.integers(0, int(q), n, dtype=np.uint64)
    return out
