"""Pins of the oracle's D2Q9 vector distribution (Sec. 2's own lattice for
g: ``MagTMatrix``, ``MagMomentEq``, SRT collision in moment space)."""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import lbmhd_oracle as O
from oracle import linear as L
from seeded_inputs import offset_noise, perturbed, smooth_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _printed(name):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, name)) if ln.strip() and not ln.startswith("#")]
    return np.array([[int(v) for v in r] for r in rows], dtype=np.int64)


def test_magnetic_moment_matrix_is_the_printed_one():
    assert np.array_equal(O.T_M.astype(np.int64), _printed("magnetic_moment_matrix_Tm.txt"))
    # invertible, and the inverse is exact on the integer matrix (rational check)
    M = [[Fraction(int(v)) for v in row] for row in _printed("magnetic_moment_matrix_Tm.txt")]
    inv = [[Fraction(O.T_M_INV[i, j]).limit_denominator(64) for j in range(9)] for i in range(9)]
    for i in range(9):
        for j in range(9):
            assert sum(inv[i][k] * M[k][j] for k in range(9)) == (1 if i == j else 0)


def test_table_fixes_the_d2q9_weights_and_the_closed_form():
    """The printed N^eq table (N4 = B/3, N8 = B/9, N0 = B) fixes symmetric
    weights (w0, w_axis, w_diag) = (4/9, 1/9, 1/36); with them T_m^-1 N^eq is
    geq of Sec. 2 on D2Q9: w'_i [B + 3 ((c.u) B - (c.B) u)]."""
    # sum w = 1, sum w c_x^2 = 2 w1 + 4 w2 = 1/3, sum w c_x^2 c_y^2 = 4 w2 = 1/9
    A = np.array([[1.0, 4.0, 4.0], [0.0, 2.0, 4.0], [0.0, 0.0, 4.0]])
    w0, w1, w2 = np.linalg.solve(A, [1.0, 1.0 / 3.0, 1.0 / 9.0])
    assert np.allclose([w0, w1, w2], [4 / 9, 1 / 9, 1 / 36], atol=1e-15)
    w = np.array([w0] + [w1] * 4 + [w2] * 4)
    rng = np.random.default_rng(4)
    rho = 1.0 + 0.1 * rng.random((6, 7))
    mx, my, bx, by = (0.05 * rng.standard_normal((6, 7)) for _ in range(4))
    geq = O.g_equilibrium_d2q9(rho, mx, my, bx, by)
    ux, uy = mx / rho, my / rho
    for i in range(9):
        cu = O.CX[i] * ux + O.CY[i] * uy
        cb = O.CX[i] * bx + O.CY[i] * by
        assert np.allclose(geq[i, 0], w[i] * (bx + 3 * (cu * bx - cb * ux)), rtol=0, atol=1e-16)
        assert np.allclose(geq[i, 1], w[i] * (by + 3 * (cu * by - cb * uy)), rtol=0, atol=1e-16)
    # the D2Q5 subset gives the same zeroth and first moments
    g5 = O.g_equilibrium(rho, mx, my, bx, by)
    for a in range(2):
        assert np.allclose(geq[:, a].sum(0), g5[:, a].sum(0), atol=1e-16)
        assert np.allclose(np.tensordot(O.CX.astype(float), geq[:, a], 1),
                           np.tensordot(O.CX[:5].astype(float), g5[:, a], 1), atol=1e-16)


def test_moment_space_srt_equals_population_bgk():
    """One collision in the moment space of T_m with a single rate equals BGK
    towards T_m^-1 N^eq in population space (with the closure on)."""
    nx, ny = 12, 10
    f = perturbed(O.W9, (9, ny, nx), 5, 0.1)
    g = O.g_equilibrium_d2q9(*[np.ones((ny, nx))] + [0.02 * smooth_field(nx, ny, s) for s in (1, 2, 3, 4)])
    g = g + offset_noise(np.zeros(18), (18, ny, nx), 6, 1e-3).reshape(9, 2, ny, nx)
    o = O.Oracle(nx, ny, 0.02, 0.03, delta=2.0, mag_lattice="d2q9")
    fstar, gstar = o.collide(f, g)
    rho, mx, my, Bx, By = O.Oracle._moments(f, g)
    _, _, R = O.closure_terms(rho, mx, my, Bx, By, o.k2)
    lam = O.filtered_induction(rho, mx, my, Bx, By, R)
    geq = np.tensordot(O.T_M_INV, O.magnetic_equilibrium_moments(Bx, By, lam), axes=(1, 0))
    assert np.allclose(gstar, g - o.s_m * (g - geq), rtol=0, atol=1e-15)
    # B is a collisional invariant
    assert np.allclose(gstar.sum(0), g.sum(0), rtol=0, atol=1e-16)


@pytest.mark.parametrize("case", [
    # nx, ny, kx, ky, nu, eta, u0, B0
    (32, 32, 1, 2, 0.05, 0.03, (0.03, -0.02), (0.04, 0.02)),
    (24, 16, 3, 1, 0.01, 0.08, (0.0, 0.05), (0.0, 0.03)),
])
def test_small_amplitude_dynamics_equal_linear_operator(case):
    """Fourier amplitude after n steps equals G(k)^n x(0) of the hand-linearised
    27-population operator (population-space SRT with the D2Q9 geq), to second
    order in the amplitude: pins T_m, the N^eq table and the streaming of all
    nine g directions."""
    nx, ny, kx, ky, nu, eta, u0, B0 = case
    rng = np.random.default_rng(3)
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    ph = np.cos(2 * np.pi * (kx * x / nx + ky * y / ny) + 0.3)
    amp = 1e-7
    a = rng.standard_normal(5) * amp
    one = np.ones((ny, nx))
    fields = (one + a[0] * ph, u0[0] * one + a[1] * ph, u0[1] * one + a[2] * ph, B0[0] * one + a[3] * ph,
              B0[1] * one + a[4] * ph)
    f = O.f_equilibrium(*fields) + amp * 0.1 * rng.standard_normal((9, 1, 1)) * ph
    g = O.g_equilibrium_d2q9(*fields) + amp * 0.1 * rng.standard_normal((9, 2, 1, 1)) * ph
    o = O.Oracle(nx, ny, nu, eta, mag_lattice="d2q9")
    o.set_state(f, g)

    def vec():
        ff, gg, _ = o.state()
        st = np.concatenate([ff, gg[:, 0], gg[:, 1]], 0)
        return np.fft.fft2(st, axes=(1, 2))[:, ky, kx] / (nx * ny)

    x0 = vec()
    rates, sm = L.rates_from(nu, eta)
    G = L.step_matrix((2 * np.pi * kx / nx, 2 * np.pi * ky / ny), rates, sm, 1.0, u0, B0, qg=9)
    n = 40
    o.step(n)
    pred = np.linalg.matrix_power(G, n) @ x0
    err = np.abs(vec() - pred).max() / np.abs(pred).max()
    assert err < 1e-6, err


@pytest.mark.parametrize("N", [256, 1024])
def test_resistivity_and_alfven_waves_on_d2q9(N):
    """B diffuses at eta k^2 with eta = 1/(3 s_m) - 1/6 (Sec. 2) on D2Q9 as on
    D2Q5; the Alfven wave has speed B0 and damping (nu + eta) k^2 / 2."""
    nu, eta, B0 = 0.05, 0.03, 0.004
    k = 2 * np.pi / N
    rates, sm = L.rates_from(nu, eta)
    lam = np.linalg.eigvals(L.step_matrix((0.0, k), rates, sm, qg=9))
    real_slow = sorted(-np.log(np.abs(lam[np.abs(np.angle(lam)) < 1e-9])) / k ** 2)
    assert any(abs(r - eta) / eta < 2 * k * k for r in real_slow)
    lam = np.linalg.eigvals(L.step_matrix((k, 0.0), rates, sm, 1.0, (0, 0), (B0, 0), qg=9))
    alf = lam[np.abs(np.abs(np.angle(lam)) / k - B0) < 1e-4]
    assert len(alf) == 2
    omega = math.sqrt(k * k * B0 * B0 - (0.5 * (nu - eta) * k * k) ** 2)
    assert abs(abs(np.angle(alf[0])) - omega) / omega < 2 * k * k
    damp = -np.log(np.abs(alf[0])) / k ** 2
    assert abs(damp - 0.5 * (nu + eta)) / (0.5 * (nu + eta)) < 1e-3


@pytest.mark.parametrize("delta", [0.0, 2.0])
def test_d2q9_conservation_and_divergence(delta):
    """Sum rho, m, B invariant over 100 steps.  With s_m = 1 the new field is
    B(x) = sum_i w_i [B + 3 c_i.Lam](x - c_i), and sum_i w_i c_ib a(x - c_i) is
    -1/3 of the isotropic 3x3 difference on D2Q9 (of the central one on
    D2Q5): the isotropic divergence of a field that starts with none stays at
    round-off (Lam is antisymmetric and the difference operators commute),
    while the central-difference one does not."""
    nx, ny = 24, 20
    f = perturbed(O.W9, (9, ny, nx), 9, 0.1)
    g = offset_noise(np.zeros(18), (18, ny, nx), 10, 0.01).reshape(9, 2, ny, nx)
    o = O.Oracle(nx, ny, 0.02, 0.03, delta=delta, mag_lattice="d2q9")
    o.set_state(f, g)
    m0 = [a.sum() for a in o.moments()]
    o.step(100)
    m1 = [a.sum() for a in o.moments()]
    assert np.allclose(m0, m1, rtol=0, atol=1e-12)
    # B from a flux function through the isotropic stencil: zero isotropic divergence
    y, x = np.mgrid[0:ny, 0:nx]
    psi = 0.01 * np.sin(2 * np.pi * x / nx) * np.cos(4 * np.pi * y / ny)

    def d_iso(a):
        e, w = np.roll(a, -1, 1), np.roll(a, 1, 1)
        n, s = np.roll(a, -1, 0), np.roll(a, 1, 0)
        ne, nw, se, sw = (np.roll(np.roll(a, dy, 0), dx, 1) for dx, dy in ((-1, -1), (1, -1), (-1, 1), (1, 1)))
        return (e - w) / 3 + (ne + se - nw - sw) / 12, (n - s) / 3 + (ne + nw - se - sw) / 12

    dpx, dpy = d_iso(psi)
    bx, by = 0.01 + dpy, -dpx
    one = np.ones((ny, nx))
    fields = (one, 0.02 * smooth_field(nx, ny, 11), 0.02 * smooth_field(nx, ny, 12), bx, by)
    assert np.abs(d_iso(bx)[0] + d_iso(by)[1]).max() < 1e-17
    o = O.Oracle(nx, ny, 0.01, 1.0 / 6.0, delta=delta, mag_lattice="d2q9")
    o.set_state(O.f_equilibrium(*fields), O.g_equilibrium_d2q9(*fields))
    o.step(100)
    _, _, _, Bx, By = o.moments()
    div_iso = np.abs(d_iso(Bx)[0] + d_iso(By)[1]).max()
    assert div_iso < 1e-16, div_iso
    assert o.diagnostics()["divb_max"] > 1e3 * div_iso   # the central-difference divergence is not conserved


def test_d2q9_and_d2q5_give_the_same_mhd():
    """Both magnetic lattices solve the same induction equation to the order
    of the Chapman-Enskog expansion: a 64^2 Kelvin-Helmholtz run differs in B
    by far less than B changes over the run, and the kinetic fields agree."""
    n = 64
    kh = dict(U0=0.05, delta_over_L=0.05, B0=0.01, rho0=1.0, pert_amp_over_U0=1e-2, noise_amp=1e-5, seed=1)
    runs = {}
    for lat in ("d2q5", "d2q9"):
        o = O.Oracle(n, n, 5e-3, 5e-3, delta=2.0, mag_lattice=lat)
        o.init_kh_jet(**kh)
        b0 = np.stack(o.moments()[3:5])
        o.step(400)
        runs[lat] = (np.stack(o.moments()), b0)
    m5, b0 = runs["d2q5"]
    m9, _ = runs["d2q9"]
    change = np.linalg.norm(m5[3:5] - b0)
    diff = np.linalg.norm(m9[3:5] - m5[3:5])
    assert 0 < diff < 0.05 * change, (diff, change)
    assert np.linalg.norm(m9[1:3] - m5[1:3]) < 1e-3 * np.linalg.norm(m5[1:3])
    with pytest.raises(ValueError):
        O.Oracle(n, n, 5e-3, 5e-3, grad_stencil="local_iso9", mag_lattice="d2q9")
