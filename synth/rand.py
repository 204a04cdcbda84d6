"""Seeded random numbers for synthetic inputs (numpy PCG64)."""

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_complex(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    """Complex128 array with independent N(0, scale^2/2) real and imaginary parts."""
    g = rng(seed)
    s = scale / np.sqrt(2.0)
    return (g.normal(0.0, s, shape) + 1j * g.normal(0.0, s, shape)).astype(np.complex128)


def random_positive(seed: int, n: int, lo: float, hi: float) -> np.ndarray:
    return rng(seed).uniform(lo, hi, n).astype(np.float64)
