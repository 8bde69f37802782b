"""Pins of the oracle's scalar diagnostics on states with closed-form values."""

import math

import numpy as np

from oracle import lbmhd_oracle as O


def _state(rho, mx, my, bx, by):
    return O.f_equilibrium(rho, mx, my, bx, by), O.g_equilibrium(rho, mx, my, bx, by)


def test_diagnostics_closed_forms():
    nx, ny = 40, 24
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    kx, ky = 2 * np.pi * 2 / nx, 2 * np.pi * 3 / ny
    A, U, C = 0.02, 0.03, 0.01
    rho = np.full((ny, nx), 1.25)
    # u_y = U sin(kx x): w = D_x u_y = U sin(kx) cos(kx x)
    uy = U * np.sin(kx * x)
    # B from a stream function -> D.B = 0; B_y = A sin(kx x), B_x = C cos(ky y)
    bx = C * np.cos(ky * y)
    by = A * np.sin(kx * x)
    f, g = _state(rho, 0 * rho, rho * uy, bx, by)
    o = O.Oracle(nx, ny, 0.01, 0.01)
    o.set_state(f, g)
    d = o.diagnostics()
    assert d["mass"] == 1.25 * nx * ny
    assert abs(d["mom_x"]) < 1e-15 and abs(d["mom_y"]) < 1e-14
    assert abs(d["e_kin"] - 1.25 * U * U / 4) < 1e-17
    assert abs(d["e_mag"] - (A * A + C * C) / 4) < 1e-17
    w_amp = U * math.sin(kx)
    assert abs(d["enstrophy"] - 0.5 * w_amp ** 2 / 2) < 1e-17
    # J_z = D_x B_y - D_y B_x = A sin(kx) cos(kx x) + C sin(ky) sin(ky y)
    assert abs(d["j2"] - (A ** 2 * math.sin(kx) ** 2 + C ** 2 * math.sin(ky) ** 2) / 2) < 1e-17
    assert d["divb_max"] < 1e-17 and d["nonfinite"] == 0
    # a non-finite population is counted once per cell
    f[3, 2, 5] = np.nan
    g[1, 0, 7, 9] = np.inf
    o.set_state(f, g)
    assert o.diagnostics()["nonfinite"] == 2


def test_divergence_diagnostic():
    nx = ny = 32
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    k = 2 * np.pi / nx
    rho = np.ones((ny, nx))
    bx = 0.01 * np.sin(k * x)
    f, g = _state(rho, 0 * rho, 0 * rho, bx, 0 * rho)
    o = O.Oracle(nx, ny, 0.01, 0.01)
    o.set_state(f, g)
    d = o.diagnostics()
    assert abs(d["divb_max"] - 0.01 * math.sin(k)) < 1e-17
    assert abs(d["divb_rms"] - 0.01 * math.sin(k) / math.sqrt(2)) < 1e-17
