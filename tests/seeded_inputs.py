"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds no arithmetic of the method: only seeded random numbers shaped as the
caller asks.  Callers supply any base profile (rest populations, mean field).
"""

from __future__ import annotations

import numpy as np


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """FP64 uniform numbers on [lo, hi) from numpy's PCG64 with the given seed."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def perturbed(base, shape, seed: int, rel: float) -> np.ndarray:
    """base[q] * (1 + rel * U(-1, 1)) broadcast over ``shape`` = (nq, ny, nx)."""
    base = np.asarray(base, dtype=np.float64).reshape((-1,) + (1,) * (len(shape) - 1))
    return base * (1.0 + rel * uniform(shape, seed))


def offset_noise(base, shape, seed: int, amp: float) -> np.ndarray:
    """base[q] + amp * U(-1, 1) broadcast over ``shape`` = (nq, ny, nx)."""
    base = np.asarray(base, dtype=np.float64).reshape((-1,) + (1,) * (len(shape) - 1))
    return base + amp * uniform(shape, seed)


def smooth_field(nx: int, ny: int, seed: int, kmax: int = 3, amp: float = 1.0) -> np.ndarray:
    """Sum of random low Fourier modes |k_x|, |k_y| <= kmax on the periodic
    grid (real, FP64), scaled so that max |value| = amp."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx)[None, :] / nx
    y = np.arange(ny)[:, None] / ny
    out = np.zeros((ny, nx))
    for kx in range(-kmax, kmax + 1):
        for ky in range(0, kmax + 1):
            if kx == 0 and ky == 0:
                continue
            a, b = rng.standard_normal(2)
            ph = 2.0 * np.pi * (kx * x + ky * y)
            out += a * np.cos(ph) + b * np.sin(ph)
    return amp * out / np.abs(out).max()
