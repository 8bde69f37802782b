"""Fields made of single Fourier modes and their closed-form energy spectra
(test support for the spectra at sizes the oracle's FFTs do not reach).

A real mode A cos(2 pi (k_x x + k_y y) / n + phi) has transform coefficients
of modulus A / 2 at +k and -k (normalised by n^2), so it adds A^2 / 4 to the
half-sum over its radial bin round(|k|) and to x-bin |k_x|; modes with
distinct wavevectors (not equal up to sign) add.
"""

from __future__ import annotations

import math

import numpy as np

from oracle import spectra as S


def random_modes(rng, n: int, count: int):
    """``count`` modes (A, k_x, k_y, phi) with distinct wavevectors (no two
    equal up to sign), |k_a| < n/2, covering every residue of k_x and k_y
    modulo 4, both signs of k_x, an axis of each kind and a wavevector near
    the corner of the spectrum."""
    seen, modes = set(), []
    forced = [(4 * int(rng.integers(1, n // 16)) + r, 4 * int(rng.integers(1, n // 16)) + (r + 1) % 4)
              for r in range(4)]
    forced += [(-kx, ky) for kx, ky in forced] + [(0, 3), (5, 0), (n // 2 - 1, -(n // 2 - 1))]
    cand = forced + [tuple(int(v) for v in rng.integers(-n // 2 + 1, n // 2, size=2)) for _ in range(4 * count)]
    for kx, ky in cand:
        if (kx, ky) == (0, 0) or (kx, ky) in seen or (-kx, -ky) in seen:
            continue
        seen.add((kx, ky))
        modes.append((float(rng.uniform(0.1, 1.0)), kx, ky, float(rng.uniform(0, 2 * math.pi))))
        if len(modes) == count:
            break
    return modes


def mode_field_numpy(n: int, modes) -> np.ndarray:
    """The field of ``modes`` on the n x n grid (phase reduced modulo n in
    integers, so it is exactly periodic)."""
    xs = np.arange(n, dtype=np.int64)
    out = np.zeros((n, n))
    for A, kx, ky, ph in modes:
        out += A * np.cos(((ky * xs[:, None] + kx * xs[None, :]) % n) * (2.0 * math.pi / n) + ph)
    return out


def mode_spectra(n: int, fields):
    """Closed-form (radial bins, x-bins) of the fields, each a list of modes."""
    e, ex = np.zeros(S.nbins(n)), np.zeros(n // 2 + 1)
    for modes in fields:
        for A, kx, ky, _ in modes:
            e[int(math.floor(math.sqrt(kx * kx + ky * ky) + 0.5))] += A * A / 4
            ex[abs(kx)] += A * A / 4
    return e, ex
