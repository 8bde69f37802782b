"""Pins of the learned-closure oracle (filtered DNS, closure samples, MLP,
Adam, the closure-correction hook) and of the spectra oracle.

Each test checks the oracle against something it does not compute itself:
closed forms of the Gaussian filter on single Fourier modes, brute-force
loops on tiny grids, the O(Delta^4) agreement of the exact subgrid terms with
the analytic closure of Sec. 2.1 (``FilterExampleSmall``), central finite
differences of the loss, torch's independent bfloat16 rounding and layers,
Adam's closed form under a constant gradient, and Parseval's identity.
"""

import math

import numpy as np
import pytest

from oracle import learned as L
from oracle import lbmhd_oracle as O
from oracle import spectra as S
import fourier_modes as FM
from seeded_inputs import smooth_field, perturbed, offset_noise


# ---------------------------------------------------------------------------
# Gaussian filter and subsampling
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("delta", [4.0, 16.0])
def test_gaussian_weights_moments(delta):
    """Sampled taps keep the second moment Delta^2/12 once sigma >~ 1 (the
    filter widths used, 4 and 16 fine cells); at sigma ~ 0.6 sampling
    changes it by a few percent."""
    w = L.gaussian_weights(delta)
    R = (len(w) - 1) // 2
    r = np.arange(-R, R + 1)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.array_equal(w, w[::-1])
    # second moment of a sampled Gaussian = sigma^2 up to terms ~exp(-2 pi^2 sigma^2)
    # and the 5-sigma truncation
    assert abs((w * r * r).sum() / (delta * delta / 12.0) - 1.0) < 5e-5


@pytest.mark.parametrize("factor", [1, 2, 4])
def test_filter_subsample_brute_force(factor):
    ny, nx, delta = 12, 16, 4.0
    a = np.random.default_rng(3).standard_normal((ny, nx))
    w = L.gaussian_weights(delta)
    R = (len(w) - 1) // 2
    out = L.filter_subsample(a, factor, delta)
    assert out.shape == (ny // factor, nx // factor)
    for Y in range(ny // factor):
        for X in range(nx // factor):
            s = 0.0
            for j in range(-R, R + 1):
                for i in range(-R, R + 1):
                    s += w[i + R] * w[j + R] * a[(factor * Y + j) % ny, (factor * X + i) % nx]
            assert abs(out[Y, X] - s) < 1e-13


def _transfer(k, n, delta):
    """Continuous Gaussian transfer exp(-q^2 sigma^2 / 2), q = 2 pi k / n."""
    q = 2 * math.pi * k / n
    return math.exp(-q * q * delta * delta / 24.0)


def test_filter_transfer_function():
    n, delta = 128, 16.0
    x = np.arange(n)
    for k in (1, 3, 7):
        a = np.cos(2 * np.pi * k * x / n)[None, :] * np.ones((n, 1))
        out = L.filter_subsample(a, 1, delta)
        assert np.max(np.abs(out - _transfer(k, n, delta) * a)) < 1e-5
        out = L.filter_subsample(a.T, 4, delta)           # along y, subsampled
        assert np.max(np.abs(out - _transfer(k, n, delta) * a.T[::4, ::4])) < 1e-5


@pytest.mark.parametrize("factor", [1, 4])
def test_exact_subgrid_single_mode_closed_form(factor):
    """All fields proportional to c = cos(q x), rho = 1: every filtered product
    minus product of filtered fields is (coefficients) * S with
    S = bar(c^2) - bar(c)^2 = (1 + T(2k) cos(2 q x))/2 - T(k)^2 cos^2(q x)."""
    n, k, delta = 64, 2, 8.0
    x = np.arange(n)
    c = np.cos(2 * np.pi * k * x / n)[None, :] * np.ones((n, 1))
    a1, a2, a3, a4 = 0.03, -0.05, 0.02, 0.07
    rho = np.ones((n, n))
    c12 = L.filtered_fields(rho, a1 * c, a2 * c, a3 * c, a4 * c, factor, delta)
    tau = L.exact_subgrid(c12)
    w = L.gaussian_weights(delta)
    R = (len(w) - 1) // 2
    r = np.arange(-R, R + 1)
    T1 = (w * np.cos(2 * np.pi * k * r / n)).sum()          # exact discrete transfer
    T2 = (w * np.cos(4 * np.pi * k * r / n)).sum()
    cs = c[::factor, ::factor]
    c2 = np.cos(4 * np.pi * k * x / n)[None, ::factor] * np.ones((n // factor, 1))
    Sx = 0.5 * (1 + T2 * c2) - T1 * T1 * cs * cs
    want = [(a1 * a1 + 0.5 * (a4 * a4 - a3 * a3)) * Sx,
            (a1 * a2 - a3 * a4) * Sx,
            (a2 * a2 + 0.5 * (a3 * a3 - a4 * a4)) * Sx,
            (a1 * a4 - a2 * a3) * Sx]
    for comp in range(4):
        assert np.max(np.abs(tau[comp] - want[comp])) < 1e-15, comp


def test_exact_subgrid_constant_fields_vanish():
    n = 16
    one = np.ones((n, n))
    c12 = L.filtered_fields(1.1 * one, 0.02 * one, -0.03 * one, 0.01 * one, 0.04 * one, 2, 4.0)
    assert np.max(np.abs(L.exact_subgrid(c12))) < 1e-17


def test_exact_minus_analytic_is_order_delta4():
    """On smooth fields with constant density the exact subgrid terms and the
    analytic closure (spectral gradients: no stencil error) agree to
    O(Delta^4): halving Delta shrinks the difference ~16x while the terms
    themselves shrink 4x.  A wrong sign, index or constant in either fails."""
    n, rho0 = 256, 1.2
    mx, my, bx, by = [smooth_field(n, n, s, kmax=3, amp=a)
                      for s, a in ((11, 0.08), (12, 0.06), (13, 0.05), (14, 0.04))]
    rho = np.full((n, n), rho0)
    kk = 2 * np.pi * np.fft.fftfreq(n)

    def spectral_grad(a):
        A = np.fft.fft2(a)
        return (np.real(np.fft.ifft2(1j * kk[None, :] * A)), np.real(np.fft.ifft2(1j * kk[:, None] * A)))

    saved = O.GRADIENTS.get("spectral")
    O.GRADIENTS["spectral"] = spectral_grad
    try:
        rel = {}
        for delta in (8.0, 4.0):
            # the filter is applied on the same grid the closure sees (factor 1)
            exact = L.exact_subgrid(L.filtered_fields(rho, mx, my, bx, by, 1, delta))
            c12 = L.filtered_fields(rho, mx, my, bx, by, 1, delta)
            ana = L.analytic_subgrid(c12[0], c12[1], c12[2], c12[3], c12[4], delta, "spectral")
            rel[delta] = [np.linalg.norm(exact[c] - ana[c]) / np.linalg.norm(ana[c]) for c in range(4)]
            assert max(rel[delta]) < (0.08 if delta == 8.0 else 0.02), rel
        for c in range(4):
            assert 3.0 < rel[8.0][c] / rel[4.0][c] < 5.0, rel   # relative error ~ Delta^2
    finally:
        if saved is None:
            del O.GRADIENTS["spectral"]
        else:
            O.GRADIENTS["spectral"] = saved


# ---------------------------------------------------------------------------
# Features
# ---------------------------------------------------------------------------


def test_feature_layout_brute_force():
    ny, nx = 5, 7
    rho = perturbed(np.ones(1), (1, ny, nx), 21, 0.1)[0]
    mx, my, bx, by = [offset_noise(np.zeros(1), (1, ny, nx), s, 0.05)[0] for s in (22, 23, 24, 25)]
    X = L.closure_features(rho, mx, my, bx, by)
    assert X.shape == (ny * nx, 64) and np.all(X[:, 63] == 0)
    ux, uy = mx / rho, my / rho
    def d(a, ax):          # central difference by explicit indexing
        out = np.empty_like(a)
        for y in range(ny):
            for x in range(nx):
                if ax == 0:
                    out[y, x] = 0.5 * (a[y, (x + 1) % nx] - a[y, (x - 1) % nx])
                else:
                    out[y, x] = 0.5 * (a[(y + 1) % ny, x] - a[(y - 1) % ny, x])
        return out
    fields = [rho, ux, uy, bx, by, d(uy, 0) - d(ux, 1), d(by, 0) - d(bx, 1)]
    for y in range(ny):
        for x in range(nx):
            for f, a in enumerate(fields):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        got = X[y * nx + x, f * 9 + (dy + 1) * 3 + (dx + 1)]
                        assert abs(got - a[(y + dy) % ny, (x + dx) % nx]) < 1e-16


def test_feature_vorticity_current_closed_form():
    """u_y = A sin(q x), u_x = C sin(q y): central-difference vorticity
    A sin(q) cos(q x) - C sin(q) cos(q y); the same for J_z with B."""
    n = 32
    q = 2 * np.pi / n
    y, x = np.mgrid[0:n, 0:n]
    A, C = 0.03, 0.02
    one = np.ones((n, n))
    X = L.closure_features(one, C * np.sin(q * y), A * np.sin(q * x), 2 * C * np.sin(q * y), 2 * A * np.sin(q * x))
    w = A * math.sin(q) * np.cos(q * x) - C * math.sin(q) * np.cos(q * y)
    assert np.max(np.abs(X[:, 5 * 9 + 4] - w.ravel())) < 1e-16
    assert np.max(np.abs(X[:, 6 * 9 + 4] - 2 * w.ravel())) < 1e-16


# ---------------------------------------------------------------------------
# bfloat16 rounding, MLP, Adam
# ---------------------------------------------------------------------------


def test_bf16_rounding():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, 2 ** -130]]).astype(np.float32)
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(L.bf16(v), want)
    # ties to even: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6
    assert L.bf16(1 + 2 ** -8) == 1.0 and L.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6


def _random_params(seed):
    p = L.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    for k in ("b1", "b2", "b3"):
        p[k] = 0.1 * rng.standard_normal(p[k].shape)
    return p


def test_mlp_forward_against_torch():
    torch = pytest.importorskip("torch")
    p = _random_params(7)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((33, 64))
    X[:, 63] = 0
    shift, scale = 0.1 * rng.standard_normal(64), 1 + rng.random(64)
    for rnd in (lambda a: a, L.bf16):
        y, _ = L.forward(p, X, shift, scale, rnd)
        def tb(a):
            return torch.from_numpy(np.asarray(a, dtype=np.float64))
        r = (lambda t: t) if rnd is not L.bf16 else (lambda t: t.to(torch.float32).to(torch.bfloat16).to(torch.float64))
        # FP32 normalisation (torch float32 arithmetic), pad column 0
        z32 = (torch.from_numpy(X.astype(np.float32)) - torch.from_numpy(shift.astype(np.float32))) \
            * torch.from_numpy(scale.astype(np.float32))
        z32[:, 63] = 0
        z = r(z32.to(torch.float64))
        h = r(torch.relu(z @ r(tb(p["w1"])) + tb(p["b1"])))
        h = r(torch.relu(h @ r(tb(p["w2"])) + tb(p["b2"])))
        want = (h @ r(tb(p["w3"])) + tb(p["b3"])).numpy()
        assert np.max(np.abs(y - want)) < 1e-12


def test_feature_stats_brute_force():
    rng = np.random.default_rng(14)
    n = 50
    X = rng.standard_normal((n, 64)) * 0.3 + 1.0
    X[:, 5 * 9 + 4] = 0.25                      # a constant field: scale 1
    T = rng.standard_normal((n, 4)) * 1e-5
    shift, scale, out_scale = L.feature_stats(X, T)
    for f in range(7):
        c = [X[i, 9 * f + 4] for i in range(n)]
        mu = sum(c) / n
        var = sum((v - mu) ** 2 for v in c) / n
        want_scale = 1.0 / math.sqrt(var) if var > 0 else 1.0
        for k in range(9 * f, 9 * f + 9):
            assert shift[k] == float(np.float32(mu))
            assert abs(scale[k] - want_scale) <= 1e-7 * want_scale
    assert shift[63] == 0 and scale[63] == 1
    for o in range(4):
        assert abs(out_scale[o] - math.sqrt(sum(T[i, o] ** 2 for i in range(n)) / n)) <= 1e-7 * out_scale[o]
    # the normalised centre features then have mean 0 and unit spread
    z = L.normalise(X, shift, scale)
    assert abs(z[:, 4].mean()) < 1e-6 and abs(z[:, 4].std() - 1) < 1e-6
    assert np.all(z[:, 63] == 0)


def test_mlp_gradients_finite_differences():
    p = _random_params(9)
    rng = np.random.default_rng(10)
    X = rng.standard_normal((6, 64))
    X[:, 63] = 0
    T = rng.standard_normal((6, 4))
    shift, scale = np.zeros(64), np.ones(64)
    ident = lambda a: a
    _, g = L.loss_and_grads(p, X, T, shift, scale, ident)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = L.loss_and_grads(p, X, T, shift, scale, ident)
            flat[idx] = old - h
            lm, _ = L.loss_and_grads(p, X, T, shift, scale, ident)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[k].reshape(-1)[idx] - fd) < 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_adam_constant_gradient_closed_form():
    """Under a constant gradient both bias-corrected moments equal g and g^2,
    so every step moves each parameter by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(11)
    p = {"a": rng.standard_normal((3, 4)), "b": rng.standard_normal(5)}
    p0 = {k: v.copy() for k, v in p.items()}
    g = {"a": rng.standard_normal((3, 4)), "b": rng.standard_normal(5)}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    lr, eps = 1e-3, 1e-8
    for t in range(1, 4):
        p, m, v = L.adam_step(p, g, m, v, t, lr, eps=eps)
    for k in p:
        want = p0[k] - 3 * lr * g[k] / (np.abs(g[k]) + eps)
        assert np.max(np.abs(p[k] - want)) < 1e-14


def test_adam_first_steps_against_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    p = {"a": rng.standard_normal(7)}
    tp = torch.tensor(p["a"].copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m, v = {"a": np.zeros(7)}, {"a": np.zeros(7)}
    for t in range(1, 6):
        g = {"a": rng.standard_normal(7)}
        p, m, v = L.adam_step(p, g, m, v, t, 1e-2)
        tp.grad = torch.tensor(g["a"])
        opt.step()
    assert np.max(np.abs(p["a"] - tp.detach().numpy())) < 1e-14


# ---------------------------------------------------------------------------
# Closure-correction hook of the oracle
# ---------------------------------------------------------------------------


def _random_state(nx, ny, seed):
    f = perturbed(O.W9, (9, ny, nx), seed, 0.15)
    g = offset_noise(np.zeros(10), (10, ny, nx), seed + 1, 0.01).reshape(5, 2, ny, nx)
    return f, g


@pytest.mark.parametrize("stencil", ["iso9", "central5"])
def test_hook_fed_the_analytic_closure_reproduces_les(stencil):
    """A DNS oracle (Delta = 0) whose correction returns the analytic closure's
    (tau_xx, tau_xy, tau_yy, eps) takes the same step as the LES oracle: the
    hook inserts each component where the analytic closure enters."""
    nx, ny, delta = 20, 14, 3.0
    f, g = _random_state(nx, ny, 31)

    def analytic(rho, mx, my, bx, by):
        return L.analytic_subgrid(rho, mx, my, bx, by, delta, stencil)

    les = O.Oracle(nx, ny, 0.02, 0.03, delta=delta, grad_stencil=stencil, s5=1.3, s6=1.5, s7=1.7, s8=1.1)
    hooked = O.Oracle(nx, ny, 0.02, 0.03, delta=0.0, grad_stencil=stencil, s5=1.3, s6=1.5, s7=1.7, s8=1.1,
                      closure_correction=analytic)
    dns = O.Oracle(nx, ny, 0.02, 0.03, delta=0.0, grad_stencil=stencil, s5=1.3, s6=1.5, s7=1.7, s8=1.1)
    for o in (les, hooked, dns):
        o.set_state(f, g)
        o.step(2)
    fl, gl = les.state()[:2]
    fh, gh = hooked.state()[:2]
    fd, gd = dns.state()[:2]
    assert np.max(np.abs(fh - fl)) < 1e-15 and np.max(np.abs(gh - gl)) < 1e-15
    assert np.max(np.abs(fd - fl)) > 1e-6            # the closure matters here


def test_held_correction_composes_from_constant_segments():
    """correction_every = K evaluates the correction at the first step after
    an injected state and at every t with t % K == 0, and holds it in between:
    the run equals segments of single-step oracles each fed the constant
    correction of its own starting state."""
    nx, ny, delta, K, t0, n = 16, 12, 2.0, 3, 2, 7
    f, g = _random_state(nx, ny, 35)
    calls = []

    def corr_of(rho, mx, my, bx, by):
        calls.append(1)
        return 0.3 * L.analytic_subgrid(rho, mx, my, bx, by, delta)

    kw = dict(delta=delta, s5=1.3, s6=1.5, s7=1.7, s8=1.1)
    held = O.Oracle(nx, ny, 0.02, 0.03, closure_correction=corr_of, correction_every=K, **kw)
    held.set_state(f, g, t=t0)
    held.step(n)
    assert len(calls) == 3                               # t = 2 (injected), 3, 6
    # segments [2, 3), [3, 6), [6, 9)
    fs, gs = f, g
    for a, b in ((2, 3), (3, 6), (6, 9)):
        c = 0.3 * L.analytic_subgrid(*O.Oracle._moments(fs, gs), delta)
        seg = O.Oracle(nx, ny, 0.02, 0.03, closure_correction=lambda *args, c=c: c, **kw)
        seg.set_state(fs, gs, t=a)
        seg.step(b - a)
        fs, gs, t = seg.state()
        assert t == b
    fh, gh, th = held.state()
    assert th == t0 + n
    assert np.max(np.abs(fh - fs)) < 1e-15 and np.max(np.abs(gh - gs)) < 1e-15
    # holding matters: evaluating every step gives a different state
    calls.clear()
    every = O.Oracle(nx, ny, 0.02, 0.03, closure_correction=corr_of, **kw)
    every.set_state(f, g, t=t0)
    every.step(n)
    assert len(calls) == n
    assert np.max(np.abs(every.state()[0] - fh)) > 1e-9
    # a new injected state evaluates again at once, whatever t is
    calls.clear()
    held.set_state(f, g, t=4)
    held.step(1)
    assert len(calls) == 1
    with pytest.raises(ValueError):
        O.Oracle(nx, ny, 0.02, 0.03, closure_correction=corr_of, correction_every=0)


def test_learned_correction_zero_network_and_ood():
    nx, ny = 12, 10
    f, g = _random_state(nx, ny, 41)
    p = L.init_params(3)
    for k in p:
        p[k] = np.zeros_like(p[k])
    p["b3"] = np.array([1.0, -2.0, 0.5, 3.0])
    shift, scale, out_scale = np.zeros(64), np.ones(64), np.array([1e-4, 2e-4, 3e-4, 4e-4])
    o = O.Oracle(nx, ny, 0.02, 0.03)
    o.set_state(f, g)
    rho, mx, my, bx, by = o.moments()
    corr = L.learned_correction(p, shift, scale, out_scale)(rho, mx, my, bx, by)
    assert corr.shape == (4, ny, nx)
    assert np.allclose(corr, (p["b3"] * out_scale)[:, None, None], rtol=0, atol=1e-20)
    # a cell whose rho feature is scaled past 6 falls back to the analytic closure
    scale2 = scale.copy()
    scale2[4] = 6.0 / np.median(rho)     # the centre rho feature passes 6 above the median
    corr2 = L.learned_correction(p, shift, scale2, out_scale)(rho, mx, my, bx, by)
    ood = rho * scale2[4] > 6.0
    assert ood.any() and (~ood).any()
    assert np.all(corr2[:, ood] == 0) and np.all(corr2[:, ~ood] == corr[:, ~ood])
    # a non-finite output (NaN bias) or input (NaN shift) falls back everywhere
    p_nan = dict(p, b3=np.array([np.nan, 0.0, 0.0, 0.0]))
    assert np.all(L.learned_correction(p_nan, shift, scale, out_scale)(rho, mx, my, bx, by) == 0)
    shift_nan = shift.copy()
    shift_nan[0] = np.nan
    assert np.all(L.learned_correction(p, shift_nan, scale, out_scale)(rho, mx, my, bx, by) == 0)


# ---------------------------------------------------------------------------
# Spectra
# ---------------------------------------------------------------------------


def test_spectrum_single_mode():
    n = 64
    y, x = np.mgrid[0:n, 0:n]
    a = 0.3 * np.sin(2 * np.pi * (3 * x + 4 * y) / n)
    E = S.spectrum(a)
    assert E.shape == (S.nbins(n),)
    assert abs(E[5] - 0.3 ** 2 / 4) < 1e-15
    assert np.max(np.abs(np.delete(E, 5))) < 1e-30


def test_spectrum_parseval_and_brute_force():
    n = 6
    rng = np.random.default_rng(13)
    a, b = rng.standard_normal((2, n, n))
    E = S.spectrum(a, b)
    assert abs(E.sum() - 0.5 * np.mean(a * a + b * b)) < 1e-14
    # brute-force DFT and binning
    want = np.zeros(S.nbins(n))
    for ky in range(-n // 2, n // 2):
        for kx in range(-n // 2, n // 2):
            s = 0.0
            for arr in (a, b):
                c = 0j
                for yy in range(n):
                    for xx in range(n):
                        c += arr[yy, xx] * np.exp(-2j * np.pi * (kx * xx + ky * yy) / n)
                s += abs(c / n ** 2) ** 2
            want[int(math.floor(math.hypot(kx, ky) + 0.5))] += 0.5 * s
    assert np.max(np.abs(E - want)) < 1e-15


def test_many_mode_closed_form_matches_the_oracle():
    """The closed form the GPU's large-grid spectra are checked against
    (A^2 / 4 per mode in its bin) equals the oracle's FFT spectra on a
    64 x 64 grid for fields of 12 random modes each."""
    n = 64
    rng = np.random.default_rng(64)
    sets = [FM.random_modes(rng, n, 12) for _ in range(2)]
    a, b = (FM.mode_field_numpy(n, m) for m in sets)
    e, ex = FM.mode_spectra(n, sets)
    assert np.max(np.abs(S.spectrum(a, b) - e)) < 1e-15
    assert np.max(np.abs(S.x_spectrum(a, b) - ex)) < 1e-15


def test_energy_spectra_sum_to_diagnostic_energies():
    n = 32
    f, g = _random_state(n, n, 51)
    o = O.Oracle(n, n, 0.02, 0.03)
    o.set_state(f, g)
    rho, mx, my, bx, by = o.moments()
    EK, EM = S.energy_spectra(rho, mx, my, bx, by)
    assert abs(EK.sum() - 0.5 * np.mean((mx * mx + my * my) / rho ** 2)) < 1e-15
    assert abs(EM.sum() - 0.5 * np.mean(bx * bx + by * by)) < 1e-15


def test_x_spectrum_single_modes_and_parseval():
    n = 32
    y, x = np.mgrid[0:n, 0:n]
    a = 0.2 * np.cos(2 * np.pi * (3 * x + 5 * y) / n) + 0.1 * np.sin(2 * np.pi * 7 * y / n)
    E = S.x_spectrum(a)
    assert E.shape == (n // 2 + 1,)
    assert abs(E[3] - 0.2 ** 2 / 4) < 1e-15 and abs(E[0] - 0.1 ** 2 / 4) < 1e-15
    assert np.max(np.abs(np.delete(E, [0, 3]))) < 1e-30
    b = np.random.default_rng(15).standard_normal((n, n))
    assert abs(S.x_spectrum(a, b).sum() - 0.5 * np.mean(a * a + b * b)) < 1e-14
    # the Nyquist column k_x = -n/2 lands in the last entry
    c = np.cos(np.pi * x)
    assert abs(S.x_spectrum(c)[n // 2] - 0.5) < 1e-15
