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


# ---------------------------------------------------------------------------
# Rough fields for the full-size parity tests.  Every field is a sum of
# separable terms a_k[x] * b_k[y], so a window of any grid (and the whole
# grid, assembled on a device with the same products and the same order of
# additions) is produced from one-dimensional factors without forming the
# grid on the host.
# ---------------------------------------------------------------------------

ROUGH_MEAN = (1.0, 0.0, 0.0, 0.01, 0.0)
ROUGH_WAVE = (0.02, 0.03, 0.03, 0.01, 0.01)
ROUGH_NOISE = (0.008, 0.03, 0.03, 0.018, 0.018)


def rough_factors(nx: int, ny: int, seed: int, mean=ROUGH_MEAN, wave=ROUGH_WAVE, noise=ROUGH_NOISE):
    """Factors of five fields (rho, m_x, m_y, B_x, B_y) on a periodic nx x ny
    grid: per field a list of (a[nx], b[ny]) FP64 pairs whose outer products
    b[y] * a[x], added in list order, give the field.  Terms: the mean; one
    oblique wave sin(kx x + ky y + phase) of wavelength about 32 cells
    (written as two separable products); four grid-scale noise products
    noise * u[x] * v[y] with u, v uniform on [-1, 1) from PCG64(seed)."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    out = []
    for f in range(5):
        terms = [(np.full(nx, float(mean[f])), np.ones(ny))]
        kx = 2.0 * np.pi * max(1, nx // 32) * int(rng.integers(1, 3)) / nx
        ky = 2.0 * np.pi * max(1, ny // 32) * int(rng.integers(1, 3)) / ny
        ph = float(rng.uniform(0.0, 2.0 * np.pi))
        terms.append((wave[f] * np.sin(kx * x + ph), np.cos(ky * y)))
        terms.append((wave[f] * np.cos(kx * x + ph), np.sin(ky * y)))
        for _ in range(4):
            terms.append((noise[f] * rng.uniform(-1.0, 1.0, nx), rng.uniform(-1.0, 1.0, ny)))
        out.append(terms)
    return out


def assemble_rough(factors, xs, ys) -> np.ndarray:
    """[5, len(ys), len(xs)] FP64 fields of rough_factors at columns xs and rows
    ys (integer index arrays, e.g. a periodic window)."""
    xs = np.asarray(xs)
    ys = np.asarray(ys)
    out = np.empty((5, len(ys), len(xs)))
    for f, terms in enumerate(factors):
        acc = np.outer(terms[0][1][ys], terms[0][0][xs])
        for a, b in terms[1:]:
            acc = acc + np.outer(b[ys], a[xs])
        out[f] = acc
    return out


def assemble_rough_torch(factors, torch, device):
    """The whole grid of rough_factors as a [5, ny, nx] FP64 tensor on
    `device`, with the products and additions of assemble_rough (IEEE
    multiply and add in the same order, so the values are identical)."""
    ny, nx = len(factors[0][0][1]), len(factors[0][0][0])
    out = torch.empty((5, ny, nx), dtype=torch.float64, device=device)
    for f, terms in enumerate(factors):
        a0 = torch.from_numpy(terms[0][0]).to(device)
        b0 = torch.from_numpy(terms[0][1]).to(device)
        acc = torch.outer(b0, a0)
        for a, b in terms[1:]:
            acc = acc + torch.outer(torch.from_numpy(b).to(device), torch.from_numpy(a).to(device))
        out[f] = acc
        del acc
    return out
