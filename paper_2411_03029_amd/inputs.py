"""Seeded synthetic inputs shaped like the paper's workloads.

Shared by the tests, the smoke check and the benchmark; it holds none of the
butterfly's arithmetic.  The paper applies its operators to random input
tensors (sections 4.1-4.3); every draw here is numpy PCG64 in FP64 with the
seed given, real and imaginary parts i.i.d. N(0, 1).
"""
from __future__ import annotations

import numpy as np


def complex_normal(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rhs_batch(n: int, d: int, nrhs: int, config: int) -> np.ndarray:
    """nrhs inputs of shape (n,)*d; right-hand side q uses seed 1000*config + q."""
    return np.stack([complex_normal((n,) * d, 1000 * config + q) for q in range(nrhs)])


def gaussian_bumps(n: int, nbumps: int, seed: int) -> np.ndarray:
    """A smooth random field on the source cube y = j/n + (2, 0, 0): a sum of
    ``nbumps`` Gaussian bumps with centres uniform in the cube, widths uniform
    in [0.05, 0.2] and complex normal amplitudes (d = 3)."""
    rng = np.random.default_rng(seed)
    c = rng.random((nbumps, 3))
    sig = rng.uniform(0.05, 0.2, nbumps)
    amp = (rng.standard_normal(nbumps) + 1j * rng.standard_normal(nbumps)) / np.sqrt(2)
    g = np.arange(n) / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    out = np.zeros((n, n, n), dtype=np.complex128)
    for m in range(nbumps):
        r2 = (X - c[m, 0]) ** 2 + (Y - c[m, 1]) ** 2 + (Z - c[m, 2]) ** 2
        out += amp[m] * np.exp(-r2 / (2 * sig[m] ** 2))
    return out


def uneven_rhs_counts(count: int = 12, lo: int = 16, hi: int = 128, seed: int = 4) -> np.ndarray:
    """Right-hand-side counts of the uneven batched mix, uniform in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, count)


def nudft_points(n: int, d: int, seed: int = 11) -> np.ndarray:
    """Target coordinates of a type-2 non-uniform DFT: per mode, n numbers
    drawn uniformly in [0, n - 1] and sorted, shape (d, n).  Sorting makes a
    dyadic block of indices an interval of coordinates."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.uniform(0.0, n - 1.0, size=(d, n)), axis=1)
