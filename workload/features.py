"""Seeded feature matrices and weights with the paper's value distributions."""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def binary_features(n: int, f: int, density: float, seed: int) -> np.ndarray:
    """Binary bag-of-words rows: Bernoulli(density) entries, float64."""
    return (_rng(seed).random((n, f)) < density).astype(np.float64)


def uniform_features(n: int, f: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return _rng(seed).uniform(lo, hi, size=(n, f))


def tfidf_features(n: int, f: int, density: float, seed: int) -> np.ndarray:
    """TF-IDF-like rows: Bernoulli(density) mask times lognormal(0,1) values,
    each row scaled to unit L2 norm (rows with no entries stay zero)."""
    rng = _rng(seed)
    mask = rng.random((n, f)) < density
    vals = rng.lognormal(0.0, 1.0, size=(n, f))
    x = np.where(mask, vals, 0.0)
    norms = np.sqrt((x * x).sum(axis=1, keepdims=True))
    return np.divide(x, norms, out=np.zeros_like(x), where=norms > 0)


def gaussian_weights(f_in: int, f_out: int, seed: int, std: float = 0.1) -> np.ndarray:
    return _rng(seed).normal(0.0, std, size=(f_in, f_out))
