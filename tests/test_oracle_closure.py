"""Pins of the oracle's subgrid closure against brute-force filtering.

``FilterExampleSmall`` (Sec. 2.1) states bar(XY) = bar X bar Y + Delta^2/12
(d bar X)(d bar Y) + O(Delta^4).  A Gaussian filter of variance Delta^2/12 has
exactly that second moment.  Filtering the unfiltered equilibrium moments of
smooth fields by brute force (spectral convolution) and comparing with the
oracle's closed-form filtered moments checks the constant 1/12, the sign of
every Reynolds and Maxwell term and which moment each one enters.
"""

import numpy as np
import pytest

from oracle import lbmhd_oracle as O
from seeded_inputs import smooth_field, perturbed, offset_noise

N = 256
RHO = 1.3


def _fields():
    return [smooth_field(N, N, s, kmax=3, amp=a)
            for s, a in ((1, 0.08), (2, 0.06), (3, 0.05), (4, 0.04))]


def _gauss(a, delta):
    k = 2 * np.pi * np.fft.fftfreq(N)
    k2 = k[None, :] ** 2 + k[:, None] ** 2
    return np.real(np.fft.ifft2(np.fft.fft2(a) * np.exp(-k2 * delta * delta / 24.0)))


def _errors(delta):
    rho = np.full((N, N), RHO)
    mx, my, bx, by = _fields()
    # brute force: filter the unfiltered equilibrium moments (population route)
    exact = np.tensordot(O.T, O.f_equilibrium(rho, mx, my, bx, by), axes=(1, 0))
    exact = np.array([_gauss(exact[k], delta) for k in range(9)])
    u = (mx / rho, my / rho)
    b = (bx, by)
    lam_exact = np.array([[_gauss(u[p] * b[a] - b[p] * u[a], delta) for a in range(2)]
                          for p in range(2)])
    fm = [_gauss(a, delta) for a in (mx, my, bx, by)]
    P, Q, R = O.closure_terms(rho, *fm, delta * delta / 12.0)
    zero = {(a, c): 0.0 * rho for a in range(2) for c in range(2)}
    with_c = O.filtered_equilibrium_moments(rho, *fm, P, Q)
    without = O.filtered_equilibrium_moments(rho, *fm, zero, zero)
    lam_c = O.filtered_induction(rho, *fm, R)
    lam_0 = O.filtered_induction(rho, *fm, zero)
    ratios = {}
    for k in (3, 4, 7, 8):
        ratios[k] = np.abs(with_c[k] - exact[k]).max() / np.abs(without[k] - exact[k]).max()
    ratios["lam_xy"] = np.abs(lam_c[0, 1] - lam_exact[0, 1]).max() / np.abs(lam_0[0, 1] - lam_exact[0, 1]).max()
    ratios["lam_yx"] = np.abs(lam_c[1, 0] - lam_exact[1, 0]).max() / np.abs(lam_0[1, 0] - lam_exact[1, 0]).max()
    # linear moments are untouched by filtering
    for k in (0, 1, 2, 5, 6):
        assert np.allclose(with_c[k], exact[k], atol=1e-13, rtol=0)
    return ratios


def test_closure_matches_bruteforce_gaussian_filter():
    small = _errors(4.0)
    for key, r in small.items():
        assert r < 0.01, (key, r)
    r8, r16 = _errors(8.0), _errors(16.0)
    for key in r8:
        # the remaining error is O(Delta^4): relative to O(Delta^2) it grows ~4x per doubling
        assert 3.0 < r16[key] / r8[key] < 5.0, (key, r8[key], r16[key])


def test_closure_is_exactly_linear_in_delta_squared():
    """One step from the same state: (f(Delta) - f(0)) is linear in Delta^2 up
    to rounding, and Delta = 0 reproduces the unfiltered step bit for bit."""
    nx, ny = 16, 12
    f = perturbed(O.W9, (9, ny, nx), 5, 0.15)
    g = offset_noise(np.zeros(10), (10, ny, nx), 6, 0.01).reshape(5, 2, ny, nx)
    out = {}
    for d in (0.0, 1.0, 2.0):
        o = O.Oracle(nx, ny, 0.02, 0.02, delta=d)
        o.set_state(f, g)
        o.step(1)
        out[d] = o.state()
    d1 = out[1.0][0] - out[0.0][0]
    d2 = out[2.0][0] - out[0.0][0]
    assert np.abs(d1).max() > 1e-6
    assert np.allclose(d2, 4 * d1, atol=1e-15, rtol=1e-9)
    g1 = out[1.0][1] - out[0.0][1]
    g2 = out[2.0][1] - out[0.0][1]
    assert np.abs(g1).max() > 1e-9
    assert np.allclose(g2, 4 * g1, atol=1e-16, rtol=1e-9)
    # closure_scale multiplies Delta^2
    o = O.Oracle(nx, ny, 0.02, 0.02, delta=1.0, closure_scale=4.0)
    o.set_state(f, g)
    o.step(1)
    assert np.allclose(o.state()[0], out[2.0][0], atol=1e-16, rtol=0)


def test_iso9_gradient_symbol():
    """The 3x3 stencil acting on exp(i k.x) multiplies it by
    i sin(k_x) (2 + cos k_y) / 3 (x component); central by i sin(k_x)."""
    n = 32
    x = np.arange(n)[None, :]
    y = np.arange(n)[:, None]
    kx, ky = 2 * np.pi * 3 / n, 2 * np.pi * 5 / n
    a = np.exp(1j * (kx * x + ky * y))
    dx, dy = O.grad_iso9(a)
    assert np.allclose(dx, 1j * np.sin(kx) * (2 + np.cos(ky)) / 3 * a, atol=1e-14)
    assert np.allclose(dy, 1j * np.sin(ky) * (2 + np.cos(kx)) / 3 * a, atol=1e-14)
    cx, cy = O.grad_central(a)
    assert np.allclose(cx, 1j * np.sin(kx) * a, atol=1e-14)
    assert np.allclose(cy, 1j * np.sin(ky) * a, atol=1e-14)


# ---------------------------------------------------------------------------
# Lagged (single-sweep) closure: gradients of the previous step's moments
# ---------------------------------------------------------------------------


def _kh_oracle(closure_time, delta=2.0, n=32):
    o = O.Oracle(n, n, 1e-3, 1e-3, delta=delta, s5=1.6, s6=1.6, s7=1.6, s8=1.6, closure_time=closure_time)
    o.init_kh_jet(U0=0.05, delta_over_L=0.1, B0=0.01, pert_amp_over_U0=0.05, noise_amp=1e-4, seed=3)
    return o


def test_lagged_first_step_is_synchronous_and_dns_is_unaffected():
    a, b = _kh_oracle("sync"), _kh_oracle("lagged")
    a.step(1)
    b.step(1)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.g, b.g)
    a, b = _kh_oracle("sync", delta=0.0), _kh_oracle("lagged", delta=0.0)
    a.step(5)
    b.step(5)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.g, b.g)


def test_lagged_conserves_and_stays_close_to_synchronous():
    """The lag moves the gradients by one step: the difference to the
    synchronous closure is a small fraction of the closure's own effect, and
    the collision invariants are kept exactly."""
    sync, lag, dns = _kh_oracle("sync"), _kh_oracle("lagged"), _kh_oracle("sync", delta=0.0)
    m0 = [x.sum() for x in lag.moments()]
    for o in (sync, lag, dns):
        o.step(40)
    m1 = [x.sum() for x in lag.moments()]
    assert all(abs(a - b) <= 1e-12 * max(1.0, abs(a)) for a, b in zip(m0, m1))
    d_lag = np.linalg.norm(lag.f - sync.f)
    d_closure = np.linalg.norm(sync.f - dns.f)
    # the jet starts from equilibria, so sound transients make the fields change
    # fast in the first steps: the lag costs 12 % of the closure's effect here,
    # about 1 % on smooth fields (below)
    assert d_closure > 0 and d_lag < 0.2 * d_closure
    n = 32
    y, x = np.mgrid[0:n, 0:n]
    rho = np.ones((n, n))
    fields = (0.05 * np.sin(2 * np.pi * y / n), 0.03 * np.sin(2 * np.pi * x / n),
              0.01 * np.sin(2 * np.pi * (x + y) / n), 0.01 * np.cos(2 * np.pi * y / n))
    out = []
    for ct, d in (("sync", 2.0), ("lagged", 2.0), ("sync", 0.0)):
        o = O.Oracle(n, n, 0.02, 0.02, delta=d, closure_time=ct)
        o.set_state(O.f_equilibrium(rho, *fields), O.g_equilibrium(rho, *fields))
        o.step(30)
        out.append(o.f)
    assert np.linalg.norm(out[1] - out[0]) < 0.03 * np.linalg.norm(out[0] - out[2])
    # after a re-injection of the state the next step is synchronous again
    lag.set_state(sync.f, sync.g, sync.t)
    sync.step(1)
    lag.step(1)
    assert np.array_equal(lag.f, sync.f)


def test_lagged_uses_the_previous_moments():
    """Step t of the lagged run equals a synchronous collision of S_t whose
    closure differentiates the moments of S_(t-1), as the initial state of a
    second, synchronous oracle would; the effect of the lag flips sign with
    the time direction of the change in the fields."""
    lag = _kh_oracle("lagged")
    f0, g0, _ = lag.state()
    lag.step(1)
    f1, g1, _ = lag.state()
    lag.step(1)
    # a synchronous oracle at S_1 differs from the lagged step exactly through the gradients
    s = _kh_oracle("sync")
    s.set_state(f1, g1, 1)
    s.step(1)
    assert not np.array_equal(s.f, lag.f)
    # replacing S_1's moments by S_0's in the closure reproduces the lagged step
    fs, gs = s.collide(f1, g1, grad_fields=O.Oracle._moments(f0, g0)[1:])
    f2, g2 = O.Oracle.stream(fs, gs)
    assert np.array_equal(f2, lag.f) and np.array_equal(g2, lag.g)


# ---------------------------------------------------------------------------
# Closure gradients from local non-equilibrium moments (vorticity by stencil)
# ---------------------------------------------------------------------------


def _solenoidal_state(n=64):
    """rho = 1 and divergence-free m and B from stream/flux functions."""
    y, x = np.mgrid[0:n, 0:n]
    q = 2 * np.pi / n
    mx = 0.02 * np.cos(q * y) - 0.01 * np.sin(q * (x + y))
    my = 0.01 * np.sin(q * (x + y)) - 0.015 * np.cos(q * x)
    bx = 0.01 + 0.01 * np.cos(q * y) + 0.005 * np.cos(q * (x - y))
    by = 0.005 * np.cos(q * (x - y))
    rho = np.ones((n, n))
    return O.f_equilibrium(rho, mx, my, bx, by), O.g_equilibrium(rho, mx, my, bx, by)


@pytest.mark.parametrize("nu", [0.02, 0.05])
def test_local_gradients_match_spectral_derivatives(nu):
    """After the non-equilibrium parts have formed (60 steps of a smooth,
    divergence-free flow), the gradients read off M3, M4 (strain), the g
    first moments (grad B) and the stencil vorticity equal the exact
    derivatives to first-order Chapman-Enskog accuracy: a wrong rate factor,
    sign or index shows up as an O(1) error."""
    n = 64
    o = O.Oracle(n, n, nu, nu)
    o.set_state(*_solenoidal_state(n))
    o.step(60)
    f, g, _ = o.state()
    gm, gb = O.local_gradients(f, g, o.rates, o.s_m, "iso9")
    _, mx, my, bx, by = o.moments()
    k = 2 * np.pi * np.fft.fftfreq(n)

    def d(a):
        A = np.fft.fft2(a)
        return np.real(np.fft.ifft2(1j * k[None, :] * A)), np.real(np.fft.ifft2(1j * k[:, None] * A))

    em = [d(mx), d(my)]
    eb = [d(bx), d(by)]
    scale_m = max(np.abs(em[a][b]).max() for a in range(2) for b in range(2))
    scale_b = max(np.abs(eb[a][b]).max() for a in range(2) for b in range(2))
    for a in range(2):
        for b in range(2):
            assert np.abs(gm[a][b] - em[a][b]).max() < 0.03 * scale_m, (a, b)
            assert np.abs(gb[a][b] - eb[a][b]).max() < 0.005 * scale_b, (a, b)


def test_local_gradient_les_step_conserves_and_is_close_to_the_stencil_les():
    n = 48
    f, g = _solenoidal_state(n)
    runs = {}
    for st, d in (("iso9", 3.0), ("local_iso9", 3.0), ("iso9", 0.0)):
        o = O.Oracle(n, n, 0.02, 0.02, delta=d, grad_stencil=st)
        o.set_state(f, g)
        o.step(30)
        runs[(st, d)] = o
    loc = runs[("local_iso9", 3.0)]
    m0 = [a.sum() for a in O.Oracle._moments(f, g)]
    m1 = [a.sum() for a in loc.moments()]
    assert all(abs(a - b) <= 1e-12 * max(1.0, abs(a)) for a, b in zip(m0, m1))
    d_loc = np.linalg.norm(loc.f - runs[("iso9", 3.0)].f)
    d_closure = np.linalg.norm(runs[("iso9", 3.0)].f - runs[("iso9", 0.0)].f)
    assert 0 < d_loc < 0.1 * d_closure
    with pytest.raises(ValueError):
        O.Oracle(n, n, 0.02, 0.02, delta=3.0, grad_stencil="local_iso9", closure_time="lagged")


# ---------------------------------------------------------------------------
# The density-gradient closure (FilterExampleLarge with Z = rho)
# ---------------------------------------------------------------------------

def _errors_varying_density(delta, full):
    """Residual ratios (closure vs brute force) / (no closure vs brute force)
    of the quotient moments M3, M4, M7, M8 and the induction moments, with a
    density that varies by +-20 %."""
    rho = RHO + smooth_field(N, N, 9, kmax=2, amp=0.25)
    mx, my, bx, by = _fields()
    exact = np.tensordot(O.T, O.f_equilibrium(rho, mx, my, bx, by), axes=(1, 0))
    exact = np.array([_gauss(exact[k], delta) for k in range(9)])
    u = (mx / rho, my / rho)
    b = (bx, by)
    lam_exact = np.array([[_gauss(u[p] * b[a] - b[p] * u[a], delta) for a in range(2)] for p in range(2)])
    fr = _gauss(rho, delta)
    fm = [_gauss(a, delta) for a in (mx, my, bx, by)]
    k2 = delta * delta / 12.0
    P, Q, R = (O.closure_terms_full if full else O.closure_terms)(fr, *fm, k2)
    zero = {(a, c): 0.0 * rho for a in range(2) for c in range(2)}
    with_c = O.filtered_equilibrium_moments(fr, *fm, P, Q)
    without = O.filtered_equilibrium_moments(fr, *fm, zero, zero)
    lam_c = O.filtered_induction(fr, *fm, R)
    lam_0 = O.filtered_induction(fr, *fm, zero)
    ratios = {}
    for k in (3, 4, 7, 8):
        ratios[k] = np.abs(with_c[k] - exact[k]).max() / np.abs(without[k] - exact[k]).max()
    for p, a, key in ((0, 1, "lam_xy"), (1, 0, "lam_yx")):
        ratios[key] = np.abs(lam_c[p, a] - lam_exact[p, a]).max() / np.abs(lam_0[p, a] - lam_exact[p, a]).max()
    return ratios


def test_density_gradient_closure_matches_bruteforce_filter():
    """With a varying density the full closure leaves an O(Delta^4) residual
    (ratio to the O(Delta^2) no-closure error grows ~4x per doubling of Delta
    and is below 1 % at Delta = 4), while the closure with density gradients
    dropped keeps an O(Delta^2) residual: a dropped or sign-flipped term of
    the bracket, or X and Y swapped in the induction product, fails."""
    full4, simple4 = _errors_varying_density(4.0, True), _errors_varying_density(4.0, False)
    for key, r in full4.items():
        assert r < 0.01, (key, r)
        assert simple4[key] > 5 * r, (key, r, simple4[key])
    f8, f16 = _errors_varying_density(8.0, True), _errors_varying_density(16.0, True)
    s8 = _errors_varying_density(8.0, False)
    for key in f8:
        assert 3.0 < f16[key] / f8[key] < 5.0, (key, f8[key], f16[key])
        # dropping the density terms leaves a residual of the closure's own order
        assert 0.7 < s8[key] / simple4[key] < 1.4 and s8[key] > 0.03, (key, simple4[key], s8[key])


def test_density_gradient_closure_closed_forms():
    """Exact derivatives of analytic fields: the bracket of FilterExampleLarge
    equals Z d(X/Z).d(Y/Z) (quotient rule), and with uniform density the full
    closure equals the simplified one."""
    n = 64
    x = np.arange(n)[None, :] * np.ones((n, 1)) * 2 * np.pi / n
    y = np.arange(n)[:, None] * np.ones((1, n)) * 2 * np.pi / n
    rho = 1.2 + 0.3 * np.sin(x + 2 * y)
    grho = (0.3 * np.cos(x + 2 * y), 0.6 * np.cos(x + 2 * y))
    m = (0.1 * np.cos(2 * x) * np.sin(y), 0.05 * np.sin(x - y))
    gm = [(-0.2 * np.sin(2 * x) * np.sin(y), 0.1 * np.cos(2 * x) * np.cos(y)),
          (0.05 * np.cos(x - y), -0.05 * np.cos(x - y))]
    B = (0.02 + 0.01 * np.sin(3 * y), 0.03 * np.cos(x))
    gb = [(0 * x, 0.03 * np.cos(3 * y)), (-0.03 * np.sin(x), 0 * x)]
    k2 = 0.7
    P, Q, R = O.closure_terms_full_from_gradients(rho, m, B, gm, gb, grho, k2)

    def dq(a, ga):   # gradient of a / rho
        return [(ga[b] - a * grho[b] / rho) / rho for b in range(2)]

    for a in range(2):
        for c in range(2):
            pa, pc, bc = dq(m[a], gm[a]), dq(m[c], gm[c]), dq(B[c], gb[c])
            assert np.allclose(P[a, c], k2 * rho * (pa[0] * pc[0] + pa[1] * pc[1]), rtol=1e-12, atol=1e-18)
            assert np.allclose(R[a, c], k2 * rho * (pa[0] * bc[0] + pa[1] * bc[1]), rtol=1e-12, atol=1e-18)
            assert np.allclose(Q[a, c], k2 * (gb[a][0] * gb[c][0] + gb[a][1] * gb[c][1]), rtol=1e-14, atol=0)
    flat = np.full((n, n), 1.3)
    P1, Q1, R1 = O.closure_terms_full(flat, m[0], m[1], B[0], B[1], k2)
    P0, Q0, R0 = O.closure_terms(flat, m[0], m[1], B[0], B[1], k2)
    for key in P0:
        assert np.array_equal(Q1[key], Q0[key])
        assert np.allclose(P1[key], P0[key], rtol=1e-14, atol=1e-20)
        assert np.allclose(R1[key], R0[key], rtol=1e-14, atol=1e-20)


def test_density_gradient_oracle_step():
    """A step of the density-gradient oracle: uniform density gives the
    simplified closure's step, varying density a different one that still
    conserves mass and momentum; local or lagged gradients are rejected."""
    nx, ny = 24, 16
    f = O.f_equilibrium(np.full((ny, nx), 1.0), 0.02 + 0.01 * smooth_field(nx, ny, 3),
                        0.01 * smooth_field(nx, ny, 4), 0.01 + 0 * smooth_field(nx, ny, 5),
                        0.01 * smooth_field(nx, ny, 6))
    g = offset_noise(np.zeros(10), (10, ny, nx), 7, 1e-3).reshape(5, 2, ny, nx) + \
        np.repeat(O.W5[:, None, None, None] * 0.01, 2, axis=1)
    runs = {}
    for full in (False, True):
        o = O.Oracle(nx, ny, 0.01, 0.02, delta=3.0, density_gradients=full)
        o.set_state(f, g)
        o.step(1)
        runs[full] = o.state()
    assert np.allclose(runs[True][0], runs[False][0], rtol=0, atol=1e-16)
    fv = perturbed(O.W9, (9, ny, nx), 8, 0.1)
    runs = {}
    for full in (False, True):
        o = O.Oracle(nx, ny, 0.01, 0.02, delta=3.0, density_gradients=full)
        o.set_state(fv, g)
        m0 = [a.sum() for a in o.moments()[:3]]
        o.step(3)
        m1 = [a.sum() for a in o.moments()[:3]]
        assert np.allclose(m0, m1, rtol=1e-13, atol=1e-13)
        runs[full] = o.state()
    assert np.abs(runs[True][0] - runs[False][0]).max() > 1e-9
    for kw in (dict(grad_stencil="local_iso9"), dict(closure_time="lagged")):
        with pytest.raises(ValueError):
            O.Oracle(nx, ny, 0.01, 0.02, delta=3.0, density_gradients=True, **kw)
