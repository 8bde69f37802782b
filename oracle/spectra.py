"""Oracle for the radially binned kinetic and magnetic energy spectra.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper compares LES and DNS through total-energy spectra (Sec. 4, figure
``FinalTotEn``) without defining the binning.  Reading used here, on a
periodic N x N grid with integer wavenumbers k = (k_x, k_y), k_a in
[-N/2, N/2):
  a_hat(k) = (1/N^2) sum_x a(x) exp(-2 pi i k.x / N),
  E_K(n) = 1/2 sum_{k : round(|k|) = n} (|u_x_hat(k)|^2 + |u_y_hat(k)|^2),
  E_M(n) = the same with B_x, B_y,
with u = m / rho, n = 0 .. nbins - 1 and round(r) = floor(r + 1/2).  With this
normalisation sum_n E_K(n) is the mean of |u|^2 / 2 over the grid (Parseval).
The streamwise spectrum E_x(m) = 1/2 sum_{k : |k_x| = m} (...), m = 0 .. N/2,
follows single Fourier modes of the jet (the growth of its m = 1 mode is the
Kelvin-Helmholtz growth rate).
"""

from __future__ import annotations

import math

import numpy as np


def nbins(n: int) -> int:
    """Number of radial bins: every |k| with k_a in [-N/2, N/2) rounds below it."""
    return int(math.floor(math.sqrt(2.0) * (n // 2) + 0.5)) + 1


def bin_index(n: int) -> np.ndarray:
    """[N, N] bin of every wavenumber in numpy's FFT ordering."""
    k = np.fft.fftfreq(n) * n
    r = np.sqrt(k[None, :] ** 2 + k[:, None] ** 2)
    return np.floor(r + 0.5).astype(np.int64)


def spectrum(*fields) -> np.ndarray:
    """1/2 sum over the fields of |FFT(a) / N^2|^2, summed per radial bin."""
    n = fields[0].shape[0]
    assert all(a.shape == (n, n) for a in fields)
    p = sum(np.abs(np.fft.fft2(a) / (n * n)) ** 2 for a in fields)
    return 0.5 * np.bincount(bin_index(n).ravel(), weights=p.ravel(), minlength=nbins(n))


def energy_spectra(rho, mx, my, bx, by):
    """(E_K, E_M) of one state's moments."""
    return spectrum(mx / rho, my / rho), spectrum(bx, by)


def x_spectrum(*fields) -> np.ndarray:
    """1/2 sum over the fields of |FFT(a) / N^2|^2, summed per |k_x|."""
    n = fields[0].shape[0]
    p = sum(np.abs(np.fft.fft2(a) / (n * n)) ** 2 for a in fields).sum(axis=0)
    kx = np.abs(np.fft.fftfreq(n) * n).astype(np.int64)
    return 0.5 * np.bincount(kx, weights=p, minlength=n // 2 + 1)
