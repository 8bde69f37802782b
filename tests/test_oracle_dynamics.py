"""Pins of the oracle's timestep: exact linear dynamics (brute-force Fourier
operator), the transport coefficients of Sec. 2, conservation, the divergence
of B, and lattice symmetries."""

import math

import numpy as np
import pytest

from oracle import lbmhd_oracle as O
from oracle import linear as L
from seeded_inputs import perturbed, offset_noise, smooth_field


def _state_vector(o, kx, ky):
    f, g, _ = o.state()
    st = np.concatenate([f, g[:, 0], g[:, 1]], 0)
    F = np.fft.fft2(st, axes=(1, 2))
    return F[:, ky, kx] / (o.nx * o.ny)


def _wave_state(nx, ny, kx, ky, rho0, u0, B0, amp, seed):
    """Uniform equilibrium (rho0, u0, B0) plus a small cosine perturbation of
    every macroscopic field and of the populations' non-equilibrium part."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    ph = np.cos(2 * np.pi * (kx * x / nx + ky * y / ny) + 0.3)
    one = np.ones((ny, nx))
    a = rng.standard_normal(5) * amp
    rho = rho0 * one + a[0] * ph
    mx = rho0 * u0[0] * one + a[1] * ph
    my = rho0 * u0[1] * one + a[2] * ph
    bx = B0[0] * one + a[3] * ph
    by = B0[1] * one + a[4] * ph
    f = O.f_equilibrium(rho, mx, my, bx, by) + amp * 0.1 * rng.standard_normal((9, 1, 1)) * ph
    g = O.g_equilibrium(rho, mx, my, bx, by) + amp * 0.1 * rng.standard_normal((5, 2, 1, 1)) * ph
    return f, g


@pytest.mark.parametrize("case", [
    # nx, ny, kx, ky, nu, eta, ghost rates, u0, B0
    (32, 32, 1, 2, 0.05, 0.03, (1.3, 1.1, 1.7, 0.9), (0.03, -0.02), (0.04, 0.02)),
    (24, 16, 3, 1, 0.01, 0.08, (None, None, None, None), (0.0, 0.05), (0.0, 0.03)),
    (16, 20, 0, 3, 0.2, 0.002, (0.6, 1.9, 1.2, 1.5), (-0.04, 0.0), (0.05, -0.01)),
])
def test_small_amplitude_dynamics_equal_linear_operator(case):
    """The oracle's Fourier amplitude after n steps equals G(k)^n x(0) of the
    hand-linearised operator (population-form equilibria, printed T) to
    second order in the amplitude.  Catches wrong streaming direction, wrong
    rates, equilibrium or moment-row errors."""
    nx, ny, kx, ky, nu, eta, ghost, u0, B0 = case
    o = O.Oracle(nx, ny, nu, eta, *[None] * 0, s5=ghost[0], s6=ghost[1], s7=ghost[2], s8=ghost[3])
    f, g = _wave_state(nx, ny, kx, ky, 1.0, u0, B0, 1e-7, 3)
    o.set_state(f, g)
    x0 = _state_vector(o, kx, ky)
    rates, sm = L.rates_from(nu, eta, *ghost)
    G = L.step_matrix((2 * np.pi * kx / nx, 2 * np.pi * ky / ny), rates, sm, 1.0, u0, B0)
    n = 40
    o.step(n)
    pred = np.linalg.matrix_power(G, n) @ x0
    err = np.abs(_state_vector(o, kx, ky) - pred).max() / np.abs(pred).max()
    assert err < 1e-6, err


def _decay(G):
    return L.hydrodynamic_eigenvalues(G, 5)


@pytest.mark.parametrize("N", [256, 1024])
def test_shear_and_magnetic_diffusion_rates(N):
    """Shear wave decays as nu k^2, B diffusion as eta k^2 (Sec. 2 formulas),
    up to O(k^2) lattice corrections."""
    nu, eta = 0.05, 0.03
    k = 2 * np.pi / N
    rates, sm = L.rates_from(nu, eta)
    lam = np.linalg.eigvals(L.step_matrix((0.0, k), rates, sm))
    real_slow = sorted(-np.log(np.abs(lam[np.abs(np.angle(lam)) < 1e-9])) / k ** 2)
    tol = 2 * k * k
    assert any(abs(r - eta) / eta < tol for r in real_slow)
    assert any(abs(r - nu) / nu < tol for r in real_slow)


@pytest.mark.parametrize("ghost", [(None, None, None, None), (1.0, 1.0, 1.5, 1.2),
                                   (1.2, 0.8, 1.1, 1.7), (1.5, 1.5, 0.9, 1.9)])
def test_sound_damping_matches_paper_bulk_viscosity(ghost):
    """Sound moves at c_s = 1/sqrt(3) and decays at (xi + 4 nu / 3) k^2 / 2 with
    xi from the MRT formula of Sec. 2, for arbitrary ghost rates s7, s8: this
    pins rows M7, M8 of the moment-space collision."""
    nu = 0.05
    rates, sm = L.rates_from(nu, 0.03, *ghost)
    xi = L.bulk_viscosity(nu, rates[4], rates[7], rates[8])
    errs = []
    for N in (128, 512):
        k = 2 * np.pi / N
        lam = np.linalg.eigvals(L.step_matrix((k, 0.0), rates, sm))
        snd = lam[np.abs(np.abs(np.angle(lam)) / k - 1 / math.sqrt(3)) < 1e-3]
        assert len(snd) == 2
        damp = -np.log(np.abs(snd[0])) / k ** 2
        errs.append(abs(damp - 0.5 * (xi + 4 * nu / 3)))
    assert errs[1] < 1e-4 * max(abs(0.5 * (xi + 4 * nu / 3)), 1e-2)
    assert errs[1] < errs[0] / 8  # converges like k^2


def test_alfven_wave_speed_and_damping():
    """Alfven wave along B0: omega^2 = k^2 B0^2 / rho0 - ((nu - eta) k^2 / 2)^2,
    damping (nu + eta) k^2 / 2.
    The lattice adds an O(B0^2 / c_s^2) relative error to the damping, so B0 is
    kept small."""
    nu, eta, B0 = 0.05, 0.03, 0.004
    rates, sm = L.rates_from(nu, eta)
    for N in (256, 1024):
        k = 2 * np.pi / N
        lam = np.linalg.eigvals(L.step_matrix((k, 0.0), rates, sm, 1.0, (0, 0), (B0, 0)))
        alf = lam[np.abs(np.abs(np.angle(lam)) / k - B0) < 1e-4]
        assert len(alf) == 2
        # continuum dispersion relation of a resistive, viscous Alfven wave
        omega = math.sqrt(k * k * B0 * B0 - (0.5 * (nu - eta) * k * k) ** 2)
        assert abs(abs(np.angle(alf[0])) - omega) / omega < 2 * k * k
        damp = -np.log(np.abs(alf[0])) / k ** 2
        assert abs(damp - 0.5 * (nu + eta)) / (0.5 * (nu + eta)) < 1e-3


def test_advection_direction():
    """A shear wave in a uniform stream u0 moves with +u0: phase per step -k.u0."""
    nu, eta = 0.05, 0.05
    u0 = (0.0, 0.04)
    N = 512
    k = 2 * np.pi / N
    rates, sm = L.rates_from(nu, eta)
    lam, vec = np.linalg.eig(L.step_matrix((0.0, k), rates, sm, 1.0, u0, (0, 0)))
    macro = np.abs(L._macro_jacobian() @ vec)
    slow = np.abs(lam) > 0.99
    shear = lam[slow & (macro[1] > 100 * np.delete(macro, 1, axis=0).max(axis=0))]
    assert len(shear) == 1
    assert abs(np.angle(shear[0]) + k * u0[1]) < 1e-6 * k * u0[1]
    # decay nu k^2 up to the lattice's O(u0^2 / c_s^2) Galilean defect
    assert abs(-np.log(abs(shear[0])) / k ** 2 - nu) < 4 * u0[1] ** 2 * nu


def _random_state(nx, ny, seed, B_amp=0.03):
    f = perturbed(O.W9, (9, ny, nx), seed, 0.15)
    g = offset_noise(np.zeros(10), (10, ny, nx), seed + 1, B_amp / 5).reshape(5, 2, ny, nx)
    return f, g


@pytest.mark.parametrize("delta", [0.0, 2.0])
def test_conservation(delta):
    """Sum rho, sum m, sum B are invariant (periodic domain) to round-off."""
    nx, ny = 24, 20
    o = O.Oracle(nx, ny, nu=0.02, eta=0.03, delta=delta)
    f, g = _random_state(nx, ny, 40)
    o.set_state(f, g)
    d0 = o.diagnostics()
    steps = 200
    o.step(steps)
    d1 = o.diagnostics()
    cells = nx * ny
    eps = np.finfo(float).eps
    assert abs(d1["mass"] - d0["mass"]) <= 4 * eps * cells * steps
    for key in ("mom_x", "mom_y", "bsum_x", "bsum_y"):
        assert abs(d1[key] - d0[key]) <= 2 * eps * cells * steps, key


@pytest.mark.parametrize("delta", [0.0, 2.0])
def test_divergence_of_B_at_unit_magnetic_rate(delta):
    """With s_m = 1 (eta = 1/6) a divergence-free start keeps D.B at round-off
    (central differences) for every step, closure on or off: the paper's
    machine-accuracy statement (Sec. 3) under this reading."""
    nx = ny = 32
    o = O.Oracle(nx, ny, nu=0.01, eta=1.0 / 6.0, delta=delta)
    assert o.s_m == 1.0
    f, _ = _random_state(nx, ny, 50)
    A = smooth_field(nx, ny, 51, kmax=5, amp=0.05)
    bx = (O.shifted(A, 0, 1) - O.shifted(A, 0, -1)) / 2
    by = -(O.shifted(A, 1, 0) - O.shifted(A, -1, 0)) / 2
    rho = f.sum(0)
    mx = np.tensordot(O.CX.astype(float), f, axes=(0, 0))
    my = np.tensordot(O.CY.astype(float), f, axes=(0, 0))
    g = O.g_equilibrium(rho, mx, my, bx, by)
    o.set_state(f, g)
    bmax = max(abs(bx).max(), abs(by).max())
    for _ in range(20):
        o.step(10)
        d = o.diagnostics()
        assert d["divb_max"] <= 1e-14 * bmax, d["divb_max"]
    # at s_m != 1 the divergence is not a round-off invariant
    o2 = O.Oracle(nx, ny, nu=0.01, eta=0.01, delta=delta)
    o2.set_state(f, g)
    o2.step(5)
    assert o2.diagnostics()["divb_max"] > 1e-10 * bmax


def _rot90(f, g):
    """Rotate the state by +90 degrees: x' = -y, y' = x; c_1 -> c_2 -> c_3 -> c_4,
    c_5 -> c_6 -> c_7 -> c_8; vectors (a, b) -> (-b, a)."""
    perm = [0, 2, 3, 4, 1, 6, 7, 8, 5]          # destination of population i
    def rot_field(a):
        # new(x', y') = old(x, y) with x = y', y = -x'
        return np.rot90(a, k=1, axes=(-1, -2))
    fr = np.empty_like(f)
    for i in range(9):
        fr[perm[i]] = rot_field(f[i])
    gr = np.empty_like(g)
    for i in range(5):
        gr[perm[i], 0] = -rot_field(g[i, 1])
        gr[perm[i], 1] = rot_field(g[i, 0])
    return fr, gr


def _reflect_x(f, g):
    perm = [0, 3, 2, 1, 4, 6, 5, 8, 7]
    fr = np.empty_like(f)
    for i in range(9):
        fr[perm[i]] = np.roll(f[i][:, ::-1], 1, axis=-1)
    gr = np.empty_like(g)
    for i in range(5):
        gr[perm[i], 0] = -np.roll(g[i, 0][:, ::-1], 1, axis=-1)
        gr[perm[i], 1] = np.roll(g[i, 1][:, ::-1], 1, axis=-1)
    return fr, gr


@pytest.mark.parametrize("stencil", ["iso9", "central5"])
@pytest.mark.parametrize("transform", ["rot90", "reflect_x"])
def test_lattice_symmetry_equivariance(stencil, transform):
    """Stepping commutes with the lattice's rotation and reflection (closure on,
    MRT ghost rates distinct)."""
    tr = {"rot90": _rot90, "reflect_x": _reflect_x}[transform]
    n = 16
    f, g = _random_state(n, n, 60)
    a = O.Oracle(n, n, nu=0.03, eta=0.02, delta=3.0, s5=1.2, s6=1.2, s7=0.9, s8=1.6,
                 grad_stencil=stencil)
    b = O.Oracle(n, n, nu=0.03, eta=0.02, delta=3.0, s5=1.2, s6=1.2, s7=0.9, s8=1.6,
                 grad_stencil=stencil)
    a.set_state(*tr(f, g))
    b.set_state(f, g)
    a.step(3)
    b.step(3)
    fa, ga, _ = a.state()
    fb, gb = tr(*b.state()[:2])
    assert np.allclose(fa, fb, atol=1e-15, rtol=0)
    assert np.allclose(ga, gb, atol=1e-16, rtol=0)


def test_translation_equivariance():
    n = 12
    f, g = _random_state(n, n + 2, 70)
    a = O.Oracle(n, n + 2, nu=0.03, eta=0.02, delta=2.0)
    b = O.Oracle(n, n + 2, nu=0.03, eta=0.02, delta=2.0)
    sh = (3, -5)
    a.set_state(np.roll(f, sh, axis=(-2, -1)), np.roll(g, sh, axis=(-2, -1)))
    b.set_state(f, g)
    a.step(2)
    b.step(2)
    assert np.allclose(a.state()[0], np.roll(b.state()[0], sh, axis=(-2, -1)), atol=1e-15, rtol=0)


def test_kh_initial_state_fields():
    """Moments of the initial state equal the analytic double shear layer,
    with the seeded noise bounded by its amplitude."""
    nx, ny = 48, 64
    U0, dl, B0 = 0.05, 0.05, 0.01
    o = O.Oracle(nx, ny, 1e-3, 1e-3)
    o.init_kh_jet(U0=U0, delta_over_L=dl, B0=B0, rho0=1.0, pert_amp_over_U0=1e-3,
                  noise_amp=1e-5, seed=3)
    rho, mx, my, bx, by = o.moments()
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    d = dl * ny
    ux = U0 * (np.tanh((y - ny / 4) / d) - np.tanh((y - 3 * ny / 4) / d) - 1)
    assert np.allclose(rho, 1.0, atol=1e-15)
    assert np.allclose(mx, ux * np.ones((1, nx)), atol=1e-16)
    assert np.allclose(bx, B0, atol=1e-17) and np.allclose(by, 0, atol=1e-18)
    noise = my - 1e-3 * U0 * np.sin(2 * np.pi * x / nx)
    assert np.abs(noise).max() <= 1e-5 and np.abs(noise).max() > 0.9e-5
    # the u_y noise of cell (x, y) is SplitMix64 output y * nx + x mapped to [-1, 1)
    z = O.splitmix64(3, np.array([5 * nx + 7]))[0]
    expect = (2.0 * (int(z) >> 11) / 2 ** 53 - 1.0) * 1e-5
    assert abs(noise[5, 7] - expect) < 1e-16
    # the profile is periodic in y to round-off level relative to U0
    assert abs(ux[0, 0] - U0 * (np.tanh((ny - ny / 4) / d) - np.tanh((ny - 3 * ny / 4) / d) - 1)) < 1e-12 * U0


def test_sech2_jet_fields():
    """The jet of Sec. 4: profile, perturbations, Re = U0 L / nu = 50k at 1024^2
    with nu = 1e-3, solenoidal u and B, and the periodic centring."""
    n = 64
    o = O.Oracle(n, n, 1e-3, 1e-3)
    o.init_sech2_jet()
    rho, mx, my, bx, by = o.moments()
    U0, B0 = 4.88e-2, 0.005 * 4.88e-2
    x = np.arange(n)
    d = np.minimum(x, n - x)
    want_uy = U0 / np.cosh(8 * np.pi * d / n) ** 2 + 0.01 * U0 * np.sin(8 * np.pi * x / n)
    assert np.allclose(my[0] / rho[0], want_uy, rtol=0, atol=1e-15)
    assert np.allclose(mx[:, 0] / rho[:, 0], 0.01 * U0 * np.sin(8 * np.pi * x / n), rtol=0, atol=1e-15)
    assert np.allclose(by[0], B0 + 0.01 * B0 * np.sin(8 * np.pi * x / n), rtol=0, atol=1e-17)
    assert np.allclose(bx[:, 0], 0.01 * B0 * np.sin(8 * np.pi * x / n), rtol=0, atol=1e-17)
    # u_x depends on y only and u_y on x only: both fields are divergence-free
    assert np.allclose(mx / rho, (mx / rho)[:, :1]) and np.allclose(my / rho, (my / rho)[:1, :])
    assert np.allclose(bx, bx[:, :1]) and np.allclose(by, by[:1, :])
    # symmetric about x = 0 of the periodic box (the sech^2 part)
    jet = want_uy - 0.01 * U0 * np.sin(8 * np.pi * x / n)
    assert np.allclose(jet[1:], jet[1:][::-1])
    assert abs(U0 * 1024 / 1e-3 - 5e4) < 1e3     # Re quoted in Sec. 4
