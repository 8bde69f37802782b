"""Pins of the oracle's lattice constants, equilibria and moment algebra.

Each check compares the oracle with something the paper prints or with
mathematics the paper fixes, never with a retyping of the oracle's own code.
"""

import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import lbmhd_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


def test_velocities_match_printed():
    c = _load("lattice_velocities.txt")
    assert np.array_equal(O.CX, c[0]) and np.array_equal(O.CY, c[1])


def test_T_symbolic_rows_match_printed_matrix():
    # Sec. 2, FluidTMatrix: the symbolic rows must equal the printed integers.
    assert np.array_equal(O.T, _load("moment_matrix_T.txt"))


def test_T_rows_orthogonal_and_closed_form_inverse():
    T = _load("moment_matrix_T.txt")
    gram = T @ T.T
    assert np.array_equal(gram, np.diag(np.diag(gram)))
    norms = [9, 6, 6, 4, 4, 12, 12, 180, 20]
    assert list(np.diag(gram)) == norms
    # exact rational check of T^-1 = T^T diag(1/|row|^2)
    Tf = [[Fraction(int(v)) for v in row] for row in T]
    inv = [[Tf[k][i] / norms[k] for k in range(9)] for i in range(9)]
    for i in range(9):
        for j in range(9):
            s = sum(inv[i][k] * Tf[k][j] for k in range(9))
            assert s == (1 if i == j else 0)
    assert np.allclose(O.T_INV, np.array([[float(v) for v in r] for r in inv]), atol=1e-15, rtol=0)


def _random_macro(n, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2, n)
    mx, my = rng.uniform(-0.15, 0.15, (2, n))
    bx, by = rng.uniform(-0.08, 0.08, (2, n))
    return rho, mx, my, bx, by


def test_f_equilibrium_moments_reproduce_printed_table():
    """T f^eq (Sec. 2 ``feq``) must equal the KinMomentEq table entry by entry;
    this fixes the D2Q9 weights the paper calls 'appropriate'."""
    rho, mx, my, bx, by = _random_macro(50, 1)
    M = O.T @ O.f_equilibrium(rho, mx, my, bx, by)
    table = [
        rho,
        mx,
        my,
        mx * my / rho - bx * by,
        (mx ** 2 - my ** 2) / rho - bx ** 2 + by ** 2,
        -mx,
        -my,
        -3 * (mx ** 2 + my ** 2) / rho,
        5 * rho / 3 - 3 * (mx ** 2 + my ** 2) / rho,
    ]
    for k in range(9):
        assert np.allclose(M[k], table[k], rtol=0, atol=4e-15), k


def test_rest_state_moments():
    """T (w rho0) = (rho0, 0, ..., 0, 5 rho0 / 3): the rest equilibrium."""
    M = O.T @ (O.W9 * 1.7)
    assert np.allclose(M, [1.7, 0, 0, 0, 0, 0, 0, 0, 5 * 1.7 / 3], atol=1e-15, rtol=0)


def test_g_equilibrium_moments():
    """Sum_i g_i^eq = B and sum_i c_ib g_ia^eq = u_b B_a - B_b u_a
    (MagMomentEq N_a0, N_a1, N_a2 with u for rho u), second moment isotropic
    with c_s^2 = 1/3 (needed by eta = 1/(3 s_m) - 1/6)."""
    rho, mx, my, bx, by = _random_macro(40, 2)
    g = O.g_equilibrium(rho, mx, my, bx, by)
    ux, uy = mx / rho, my / rho
    assert np.allclose(g[:, 0].sum(0), bx, atol=1e-16, rtol=0)
    assert np.allclose(g[:, 1].sum(0), by, atol=1e-16, rtol=0)
    cx, cy = O.CX[:5], O.CY[:5]
    lam_xx = np.tensordot(cx, g[:, 0], axes=(0, 0))
    lam_xy = np.tensordot(cx, g[:, 1], axes=(0, 0))
    lam_yx = np.tensordot(cy, g[:, 0], axes=(0, 0))
    lam_yy = np.tensordot(cy, g[:, 1], axes=(0, 0))
    assert np.allclose(lam_xx, 0, atol=1e-17)
    assert np.allclose(lam_yy, 0, atol=1e-17)
    assert np.allclose(lam_xy, ux * by - bx * uy, atol=1e-16, rtol=0)
    assert np.allclose(lam_yx, uy * bx - by * ux, atol=1e-16, rtol=0)
    second = np.array([[np.sum(O.W5 * a * b) for b in (cx, cy)] for a in (cx, cy)])
    assert np.allclose(second, np.eye(2) / 3, atol=1e-16)


def test_g_rebuilt_from_moments_equals_population_form():
    rho, mx, my, bx, by = _random_macro(30, 3)
    zero = {(a, c): 0.0 * rho for a in range(2) for c in range(2)}
    lam = O.filtered_induction(rho, mx, my, bx, by, zero)
    assert np.allclose(O.g_equilibrium_from_moments(bx, by, lam),
                       O.g_equilibrium(rho, mx, my, bx, by), atol=2e-17, rtol=0)


def test_transport_rates():
    # nu = 1/(3 s) - 1/6 and eta = 1/(3 s_m) - 1/6 (Sec. 2)
    for nu in (1e-3, 2e-4, 1e-4, 5e-5, 0.1):
        s = O.relaxation_rates(nu)[3]
        assert abs(1 / (3 * s) - 1 / 6 - nu) < 1e-15
        sm = O.magnetic_rate(nu)
        assert abs(1 / (3 * sm) - 1 / 6 - nu) < 1e-15
    assert O.relaxation_rates(1e-3)[3] == pytest.approx(1.98807, abs=1e-5)
    r = O.relaxation_rates(0.1, s5=1.1, s7=0.7)
    assert list(r[:3]) == [0, 0, 0] and r[5] == 1.1 and r[6] == r[3] and r[7] == 0.7


def test_srt_moment_space_equals_population_bgk():
    """With every rate equal and Delta = 0, collision in moment space must equal
    plain BGK on populations toward ``feq`` (a route that never uses the
    moment table or T)."""
    from seeded_inputs import perturbed, offset_noise
    nx = ny = 12
    f = perturbed(O.W9, (9, ny, nx), 11, 0.2)
    g = offset_noise(np.zeros(10), (10, ny, nx), 12, 0.02).reshape(5, 2, ny, nx)
    o = O.Oracle(nx, ny, nu=0.07, eta=0.04)
    fs, gs = o.collide(f, g)
    rho, mx, my, bx, by = o._moments(f, g)
    s = o.rates[3]
    feq = O.f_equilibrium(rho, mx, my, bx, by)
    assert np.allclose(fs, f - s * (f - feq), atol=1e-15, rtol=0)
    geq = O.g_equilibrium(rho, mx, my, bx, by)
    assert np.allclose(gs, g - o.s_m * (g - geq), atol=2e-17, rtol=0)


def test_mrt_matches_bruteforce_population_operator():
    """Generic MRT: f* = f - S' (f - f^eq) with S' = T^-1 S T formed by a
    generic matrix inverse of the printed T, rates random in (0, 2)."""
    from seeded_inputs import perturbed, offset_noise
    rng = np.random.default_rng(5)
    nx, ny = 10, 8
    f = perturbed(O.W9, (9, ny, nx), 21, 0.2)
    g = offset_noise(np.zeros(10), (10, ny, nx), 22, 0.02).reshape(5, 2, ny, nx)
    s5, s6, s7, s8 = rng.uniform(0.2, 1.9, 4)
    o = O.Oracle(nx, ny, nu=0.05, eta=0.05, s5=s5, s6=s6, s7=s7, s8=s8)
    fs, _ = o.collide(f, g)
    T = _load("moment_matrix_T.txt")
    S = np.diag(o.rates)
    Sp = np.linalg.inv(T) @ S @ T
    rho, mx, my, bx, by = o._moments(f, g)
    feq = O.f_equilibrium(rho, mx, my, bx, by)
    ref = f - np.tensordot(Sp, f - feq, axes=(1, 0))
    assert np.allclose(fs, ref, atol=2e-15, rtol=0)


def test_splitmix64_published_vectors():
    with open(os.path.join(GOLDEN, "splitmix64_vectors.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            vals = [int(v) for v in line.split()]
            seed, expect = vals[0], vals[1:]
            got = O.splitmix64(seed, np.arange(len(expect)))
            assert [int(v) for v in got] == expect


def test_uniform_noise_range_and_mean():
    u = O.uniform_pm1(7, np.arange(200000))
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.01 and abs((u * u).mean() - 1 / 3) < 0.01
