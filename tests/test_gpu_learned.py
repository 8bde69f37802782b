"""GPU parity of the learned closure, the filtered-DNS pipeline and the
spectra against the FP64 oracle (oracle/learned.py, oracle/spectra.py).

Tolerances.  FP64 paths (filter, spectra, the collision with a given
correction) are held to round-off.  The network runs in bfloat16 with FP32
accumulation on both sides' definitions, but the oracle accumulates in FP64:
a pre-activation that lands within ~1e-7 of a bfloat16 rounding boundary can
round the other way, changing that
activation by one bfloat16 step (2^-8 relative) and the output by at most
about |w| 2^-8.  The tests bound the worst row by a few such steps and
require the bulk of rows to agree to FP32 accumulation noise; measured
errors are printed.
"""

import math

import numpy as np
import pytest

from oracle import learned as L
from oracle import lbmhd_oracle as O
from oracle import spectra as S
import fourier_modes as FM
from seeded_inputs import perturbed, offset_noise

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09807_amd import learned as G
    return G


def _params(seed):
    """Oracle parameter dict with nonzero biases, all values FP32."""
    p = L.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.uniform(-0.2, 0.2, p[k].shape).astype(np.float32).astype(np.float64)
    return p


def _flat(p):
    return np.concatenate([p["w1"].ravel(), p["b1"], p["w2"].ravel(), p["b2"], p["w3"].ravel(),
                           p["b3"]]).astype(np.float32)


def _unflat(v):
    v = np.asarray(v, dtype=np.float64)
    return {"w1": v[0:4096].reshape(64, 64), "b1": v[4096:4160], "w2": v[4160:8256].reshape(64, 64),
            "b2": v[8256:8320], "w3": v[8320:8576].reshape(64, 4), "b3": v[8576:8580]}


def _norm(seed):
    rng = np.random.default_rng(seed)
    shift = rng.normal(0, 0.1, 7).astype(np.float32)
    scale = rng.uniform(0.5, 2.0, 7).astype(np.float32)
    out_scale = rng.uniform(1e-5, 1e-4, 4).astype(np.float32)
    s64 = np.zeros(64)
    c64 = np.ones(64)
    for f in range(7):
        s64[9 * f: 9 * f + 9] = shift[f]
        c64[9 * f: 9 * f + 9] = scale[f]
    return shift, scale, out_scale, s64, c64


def _features(n, seed, ood_rows=()):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 0.8, (n, 64)).astype(np.float32)
    X[:, 63] = 0
    for r in ood_rows:
        X[r, rng.integers(0, 63)] = 40.0
    return X


def _mlp(G, p, shift, scale, out_scale):
    m = G.Mlp(_flat(p))
    m.set_norm(shift, scale, out_scale)
    return m


def _compare_rows(got, want, label):
    d = np.abs(got - want).max(axis=1)
    scale = np.abs(want).max()
    print(f"{label}: max {d.max():.2e}, 99th pct {np.percentile(d, 99):.2e}, median {np.median(d):.2e}, "
          f"|y| max {scale:.2e}", flush=True)
    assert np.median(d) <= 2e-5 * max(scale, 1.0)
    assert np.percentile(d, 95) <= 1e-4 * max(scale, 1.0)
    assert d.max() <= 2e-2 * max(scale, 1.0)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("n", [1, 31, 1000, 70001])
def test_forward_matches_oracle(n):
    G = _gpu()
    p = _params(1)
    shift, scale, out_scale, s64, c64 = _norm(2)
    ood_rows = [r for r in (0, n // 2, n - 1) if r < n] if n > 1 else []
    X = _features(n, 3, ood_rows)
    m = _mlp(G, p, shift, scale, out_scale)
    y, ood = m.forward(torch.from_numpy(X).cuda())
    y = y.cpu().numpy().astype(np.float64)
    ood = ood.cpu().numpy()
    yo, _ = L.forward(p, X.astype(np.float64), s64, c64)
    oo = (np.abs(L.normalise(X, s64, c64)) > 6.0).any(axis=1)
    assert np.array_equal(ood.astype(bool), oo)
    if n > 1:
        assert oo[ood_rows].all()          # planted rows (a few random rows may exceed 6 too)
    _compare_rows(y, yo, f"forward n={n}")


def test_feature_stats_match_oracle():
    G = _gpu()
    rng = np.random.default_rng(5)
    n = 5003
    X = (rng.normal(0, 1, (n, 64)) * rng.uniform(1e-3, 1, 64) + rng.normal(0, 1, 64)).astype(np.float32)
    X[:, 5 * 9 + 4] = 0.125          # a constant field: scale 1
    X[:, 63] = 0
    T = (rng.normal(0, 1, (n, 4)) * [1e-5, 2e-5, 3e-6, 1e-6]).astype(np.float32)
    m = G.Mlp(_flat(_params(1)))
    m.fit_norm(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    nm = m.norm.cpu().numpy()
    shift, scale, out_scale = L.feature_stats(X.astype(np.float64), T.astype(np.float64))
    for f in range(7):
        assert abs(nm[f] - shift[9 * f]) <= 2.4e-7 * abs(shift[9 * f]) + 1e-30, f
        assert abs(nm[8 + f] - scale[9 * f]) <= 2.4e-7 * scale[9 * f], f
    assert nm[8 + 5] == 1.0
    assert np.all(np.abs(nm[16:20] - out_scale) <= 2.4e-7 * out_scale)


def _clear_of_bf16_boundaries(p, X, shift, scale, rel=1e-6):
    """Rows whose network inputs and pre-activations all lie further than
    `rel` (relative) from a bfloat16 rounding boundary and from zero, so that
    the GPU's FP32 and the oracle's FP64 forward pass round every one of them
    the same way (a value within ~1e-7 of a boundary may round to the
    neighbouring bfloat16 on one side, shifting that row's activation by one
    bfloat16 step)."""
    def ambiguous(v):
        return (L.bf16(v * (1 + rel)) != L.bf16(v * (1 - rel))) | (np.abs(v) < rel)
    z = L.normalise(X, shift, scale)
    bad = ambiguous(z)[:, :63].any(axis=1)
    zr = L.bf16(z)
    a1 = zr @ L.bf16(p["w1"]) + p["b1"]
    bad |= ambiguous(a1).any(axis=1)
    h1 = L.bf16(np.maximum(a1, 0.0))
    a2 = h1 @ L.bf16(p["w2"]) + p["b2"]
    bad |= ambiguous(a2).any(axis=1)
    return ~bad


@pytest.mark.parametrize("batch", [200, 5000])
def test_gradient_matches_oracle(batch):
    """Batch gradient and loss against the oracle's FP64 gradients of the same
    bfloat16 forward pass (straight through the roundings), per tensor within
    1e-5 relative L2.  The rows are drawn among those whose roundings the two
    sides cannot take differently (about 7 % of random rows are left out); the
    backward's matrix-core products carry the FP32 deltas in three bfloat16
    terms, so what remains is FP32 accumulation."""
    G = _gpu()
    p = _params(7)
    shift, scale, out_scale, s64, c64 = _norm(8)
    n = 8000
    X = _features(n, 9)
    rng = np.random.default_rng(10)
    T = (rng.normal(0, 1, (n, 4)) * out_scale).astype(np.float32)
    clear = np.flatnonzero(_clear_of_bf16_boundaries(p, X.astype(np.float64), s64, c64))
    print(f"{len(clear)} of {n} rows clear of bfloat16 rounding boundaries", flush=True)
    assert len(clear) >= batch
    idx = rng.permutation(clear)[:batch].astype(np.int32)
    m = _mlp(G, p, shift, scale, out_scale)
    grad, loss = m.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), torch.from_numpy(idx).cuda())
    g = _unflat(grad.cpu().numpy())
    Tn = (T[idx] / out_scale).astype(np.float64)          # FP32 division, as the kernel
    lo, go = L.loss_and_grads(p, X[idx].astype(np.float64), Tn, s64, c64)
    print(f"batch {batch}: loss gpu {loss.item():.8e} oracle {lo:.8e}", flush=True)
    assert abs(loss.item() - lo) <= 1e-6 * lo
    for k in go:
        err = np.linalg.norm(g[k] - go[k]) / np.linalg.norm(go[k])
        print(f"  grad {k}: relative L2 error {err:.2e}", flush=True)
        assert err <= 1e-5, k
    assert np.all(g["w1"][63] == 0)          # the pad input carries no gradient


def test_adam_and_train_step_match():
    G = _gpu()
    p = _params(11)
    shift, scale, out_scale, s64, c64 = _norm(12)
    n = 1000
    X = _features(n, 13)
    rng = np.random.default_rng(14)
    T = (rng.normal(0, 1, (n, 4)) * out_scale).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    a = _mlp(G, p, shift, scale, out_scale)
    b = _mlp(G, p, shift, scale, out_scale)
    po = {k: v.copy() for k, v in p.items()}
    mo = {k: np.zeros_like(v) for k, v in p.items()}
    vo = {k: np.zeros_like(v) for k, v in p.items()}
    for t in range(1, 4):
        idx = torch.from_numpy(rng.permutation(n)[:256].astype(np.int32)).cuda()
        grad, _ = a.gradient(Xd, Td, idx)
        go = _unflat(grad.cpu().numpy())
        a.adam(grad, 1e-3)
        b.train_step(Xd, Td, idx, 1e-3)
        po, mo, vo = L.adam_step(po, go, mo, vo, t, 1e-3)
        # the composed entry point is the two halves, bit for bit
        assert torch.equal(a.params, b.params) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
        pa = _unflat(a.params.cpu().numpy())
        for k in po:
            err = np.abs(pa[k] - po[k]).max()
            assert err <= 1e-6 * max(1.0, np.abs(po[k]).max()), (t, k, err)


def test_training_reduces_loss():
    """A few hundred steps fit a smooth function of the inputs (end-to-end
    check of forward, backward and optimiser on the GPU)."""
    G = _gpu()
    rng = np.random.default_rng(15)
    n = 8192
    X = _features(n, 16)
    w = rng.normal(0, 0.3, (63, 4))
    T = np.tanh(X[:, :63].astype(np.float64) @ w).astype(np.float32) * 1e-4
    m = G.Mlp(G.glorot_params(17))
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    m.fit_norm(Xd, Td)
    gen = torch.Generator(device="cuda").manual_seed(18)
    first = last = None
    for step in range(400):
        idx = torch.randperm(n, device="cuda", generator=gen)[:1024].to(torch.int32)
        loss = m.train_step(Xd, Td, idx, 3e-3)
        if step == 0:
            first = loss.item()
    last = m.train_step(Xd, Td, torch.arange(n, device="cuda", dtype=torch.int32), 1e-9).item()
    print(f"loss {first:.4e} -> {last:.4e}", flush=True)
    assert last < 0.1 * first


# ---------------------------------------------------------------------------
# filtered DNS pipeline
# ---------------------------------------------------------------------------


def _smooth_state(nx, ny, seed):
    """A near-equilibrium state with smooth, large-scale momentum and field."""
    y, x = np.mgrid[0:ny, 0:nx]
    rng = np.random.default_rng(seed)
    def mode():
        kx, ky = rng.integers(1, 4, 2)
        return np.sin(2 * np.pi * (kx * x / nx + ky * y / ny) + rng.uniform(0, 2 * np.pi))
    rho = 1.0 + 0.01 * mode()
    ux, uy = 0.04 * mode(), 0.03 * mode()
    bx, by = 0.01 + 0.02 * mode(), 0.015 * mode()
    f = O.f_equilibrium(rho, rho * ux, rho * uy, bx, by)
    g = O.g_equilibrium(rho, rho * ux, rho * uy, bx, by)
    f = f + offset_noise(np.zeros(9), (9, ny, nx), seed + 1, 1e-5)
    return f, g


def _sim_state(nx, ny, f, g, **kw):
    from paper_1705_09807_amd import Sim
    s = Sim(nx=nx, ny=ny, nu=0.02, eta=0.03, **kw)
    s.set_state(torch.from_numpy(np.concatenate([f, g[:, 0], g[:, 1]], 0)))
    return s


@pytest.mark.parametrize("nx,ny,factor,delta", [(96, 80, 4, 8.0), (64, 48, 1, 4.0), (128, 128, 4, 16.0),
                                                (40, 24, 8, 3.0)])
def test_filter_subsample_matches_oracle(nx, ny, factor, delta):
    G = _gpu()
    f, g = _smooth_state(nx, ny, 21)
    s = _sim_state(nx, ny, f, g)
    mom = s.moments()
    out = G.filter_subsample(mom, factor, delta).cpu().numpy()
    rho, mx, my, bx, by = mom.cpu().numpy()
    want = L.filtered_fields(rho, mx, my, bx, by, factor, delta)
    for k in range(12):
        err = np.abs(out[k] - want[k]).max() / np.abs(want[k]).max()
        assert err <= 1e-13, (k, err)


@pytest.mark.parametrize("stencil", ["iso9", "central5"])
def test_closure_samples_match_oracle(stencil):
    G = _gpu()
    nx, ny, factor, delta = 128, 96, 4, 16.0
    f, g = _smooth_state(nx, ny, 31)
    s = _sim_state(nx, ny, f, g)
    c12 = G.filter_subsample(s.moments(), factor, delta)
    X, T = G.closure_samples(c12, delta / factor, stencil)
    X, T = X.cpu().numpy(), T.cpu().numpy()
    c = c12.cpu().numpy()
    Xo = L.closure_features(c[0], c[1], c[2], c[3], c[4])
    To = (L.exact_subgrid(c) - L.analytic_subgrid(c[0], c[1], c[2], c[3], c[4], delta / factor, stencil))
    To = To.reshape(4, -1).T
    # FP64 on both sides, stored FP32: within one FP32 rounding (plus FP64 noise)
    assert np.all(np.abs(X - Xo) <= 1.2e-7 * np.abs(Xo) + 1e-12)
    err = np.abs(T - To).max(axis=0) / np.abs(To).max(axis=0)
    print(f"targets relative error per component {err}", flush=True)
    assert np.all(err <= 1e-6)


@pytest.mark.parametrize("n", [8, 64, 256])
def test_spectra_match_oracle(n):
    G = _gpu()
    f, g = _smooth_state(n, n, 41 + n)
    f = f + offset_noise(np.zeros(9), (9, n, n), 7, 1e-3)     # energy in every bin
    s = _sim_state(n, n, f, g)
    mom = s.moments()
    ek, em, ekx = [a.cpu().numpy() for a in G.spectra(mom)]
    rho, mx, my, bx, by = mom.cpu().numpy()
    EK, EM = S.energy_spectra(rho, mx, my, bx, by)
    EX = S.x_spectrum(mx / rho, my / rho)
    assert np.abs(ek - EK).max() <= 1e-13 * EK.sum()
    assert np.abs(em - EM).max() <= 1e-13 * EM.sum()
    assert np.abs(ekx - EX).max() <= 1e-13 * EX.sum()


def _mode_field(n, modes, device):
    """fourier_modes.mode_field_numpy on the device."""
    xs = torch.arange(n, device=device, dtype=torch.int64)
    out = torch.zeros((n, n), dtype=torch.float64, device=device)
    for A, kx, ky, ph in modes:
        ph_int = (ky * xs[:, None] + kx * xs[None, :]) % n
        out += A * torch.cos(ph_int.to(torch.float64) * (2.0 * math.pi / n) + ph)
        del ph_int
    return out


@pytest.mark.parametrize("n", [4096, 8192, 16384])
def test_spectra_exact_modes_large_grids(n):
    """Up to and beyond one LDS transform (n > 4096 takes the four-step
    path): velocity and field made of 40 random single Fourier modes each (every
    residue of k_x and k_y modulo 4, both signs, near the corner of the
    spectrum), rho = 1; every bin of E_K, E_M and E_x equals the closed form
    sum of A^2 / 4 within 1e-12 of the total (an index, twiddle or residue
    mistake moves a mode's energy to another bin)."""
    G = _gpu()
    rng = np.random.default_rng(n)
    dev = torch.device("cuda:0")
    mode_sets = [FM.random_modes(rng, n, 40) for _ in range(4)]
    mom = torch.empty((5, n, n), dtype=torch.float64, device=dev)
    mom[0].fill_(1.0)
    for i, modes in enumerate(mode_sets):
        mom[1 + i] = _mode_field(n, modes, dev)
    torch.cuda.synchronize()
    ek, em, ekx = [a.cpu().numpy() for a in G.spectra(mom)]
    del mom
    torch.cuda.empty_cache()
    EK, EX = FM.mode_spectra(n, mode_sets[:2])
    EM, _ = FM.mode_spectra(n, mode_sets[2:])
    for got, ref in ((ek, EK), (em, EM), (ekx, EX)):
        err = np.abs(got - ref).max() / ref.sum()
        print(f"n={n} max bin error / total = {err:.2e}", flush=True)
        assert err <= 1e-12


# ---------------------------------------------------------------------------
# the learned closure inside the timestep
# ---------------------------------------------------------------------------


def _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale, dtype="fp64", delta=2.0):
    s = _sim_state(nx, ny, f, g, delta=delta, closure="learned", dtype=dtype, s5=1.3, s6=1.5, s7=1.7, s8=1.1,
                   b_ref=(0.01, 0.0))
    m = _mlp(G, p, shift, scale, out_scale)
    s.set_closure_mlp(m.pack())
    torch.cuda.synchronize()
    return s


def _state_norm(f, g):
    rho, mx, my, bx, by = O.Oracle._moments(f, g)
    X = L.closure_features(rho, mx, my, bx, by)
    shift, scale, _ = L.feature_stats(X, np.ones((X.shape[0], 4)))
    out_scale = np.array([3e-5, 2e-5, 3e-5, 1e-5], dtype=np.float32)
    return shift[::9][:7].astype(np.float32), scale[::9][:7].astype(np.float32), out_scale, shift, scale


def test_step_requires_a_network():
    G = _gpu()
    from paper_1705_09807_amd.native import LbmError
    f, g = _smooth_state(32, 24, 51)
    s = _sim_state(32, 24, f, g, delta=2.0, closure="learned")
    with pytest.raises(LbmError):
        s.step(1)


_CORR_CASES = [(nx, ny, ood) for nx, ny in [(96, 64), (70, 37), (67, 33), (523, 77)] for ood in (False, True)]
# on a grid this small every 3x3 patch reaches the density extremes, so the
# out-of-range case would flag every cell: the in-range case only
_CORR_CASES.append((24, 18, False))
# taller grids whose last strip of the FP32-compute input-vector kernel is partial
# (512-, 256- and 64-lane strips) while its row segments run the three-row loop and
# end with one or two rows (segments of 5, 4, 2 and 5 rows on a 256-CU device)
_CORR_CASES += [(1100, 425, False), (1100, 340, False), (700, 99, False), (200, 300, False)]
# the widest rows the ABI accepts: 64 input-vector strips per row (the last one
# column short at 32767), network tiles shorter than the grid is wide, and a
# grid fewer rows tall than a tile, so every tile's vertical halo wraps
_CORR_CASES += [(32768, 4, False), (32767, 5, False)]


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("nx,ny,ood", _CORR_CASES)
def test_correction_of_state_matches_oracle(nx, ny, ood, dtype):
    """The correction of a state (moments of the stored state, features,
    network, out-of-range fallback) against the oracle's on the state the GPU
    holds, for FP64, FP32 and BF16 storage.  523 x 77 spans three strips of
    the input-vector kernel (the last ragged), ragged row segments and
    ragged network tiles in both directions; 24 x 18 is narrower than a
    strip and a tile in both directions, so every halo wraps around."""
    G = _gpu()
    f, g = _smooth_state(nx, ny, 61)
    p = _params(62)
    shift, scale, out_scale, s64, c64 = _state_norm(f, g)
    if ood:
        # a narrow density scale: cells with |rho - mean| above ~60% of the
        # largest deviation leave the training range and keep the analytic closure
        rho = f.sum(axis=0)
        scale[0] = np.float32(6.0 / (0.6 * np.abs(rho - shift[0]).max()))
        c64[:9] = scale[0]
    s = _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale, dtype=dtype)
    corr = s.closure_correction().cpu().numpy().astype(np.float64)
    st = s.get_state().cpu().numpy()
    fo, go = st[:9], np.stack([st[9:14], st[14:19]], axis=1)
    rho, mx, my, bx, by = O.Oracle._moments(fo, go)
    want = L.learned_correction(p, s64, c64, out_scale.astype(np.float64))(rho, mx, my, bx, by)
    zmax = np.abs(L.normalise(L.closure_features(rho, mx, my, bx, by), s64, c64)).max(axis=1)
    oo = zmax > 6.0
    decided = np.abs(zmax - 6.0) > 1e-4          # both sides decide these cells the same way
    got_ood = (corr == 0).all(axis=0).ravel()
    assert np.array_equal(got_ood[decided], oo[decided])
    if ood:
        # both branches exercised (the flagged share depends on the shape's field)
        assert 0.02 < oo.mean() < 0.98
    else:
        assert not oo.any()
    rows = lambda a: (a / out_scale[:, None, None]).reshape(4, -1).T[decided]
    _compare_rows(rows(corr), rows(want), f"correction {nx}x{ny} ood={ood} ({oo.mean():.0%} out of range)")


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_isolated_out_of_range_cells_zero_exactly_their_neighbourhoods(dtype):
    """Isolated cells whose density alone leaves the training range (all nine
    f populations scaled, so u, B and the vorticity and current around them
    keep their values): each must zero the correction of exactly the nine
    cells whose 3x3 patch holds it, and every other cell keeps the oracle's
    correction.  Each neighbour sees its culprit at another patch position,
    so all nine positions are checked on their own (inside a blob of flagged
    cells a missed position is hidden by the others).  Culprits sit at the
    grid's corner, at network-tile edges (every 64 columns, 16 rows) and at
    the FP32-compute input-vector kernel's strip edges (255/256, 511/512)."""
    G = _gpu()
    nx, ny = 523, 77
    f, g = _smooth_state(nx, ny, 71)
    p = _params(72)
    shift, scale, out_scale, s64, c64 = _state_norm(f, g)
    culprits = [(0, 0), (5, 63), (16, 64), (31, 127), (30, 253), (45, 254), (60, 508), (76, 300), (47, 522),
                (20, 255), (38, 256), (68, 511), (10, 512)]
    rho = f.sum(axis=0)
    want_ood = np.zeros((ny, nx), dtype=bool)
    for cy, cx in culprits:
        f[:, cy, cx] *= (float(shift[0]) + 8.0 / float(scale[0])) / rho[cy, cx]
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                want_ood[(cy + dy) % ny, (cx + dx) % nx] = True
    s = _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale, dtype=dtype)
    corr = s.closure_correction().cpu().numpy().astype(np.float64)
    st = s.get_state().cpu().numpy()
    fo, go = st[:9], np.stack([st[9:14], st[14:19]], axis=1)
    rho, mx, my, bx, by = O.Oracle._moments(fo, go)
    zmax = np.abs(L.normalise(L.closure_features(rho, mx, my, bx, by), s64, c64)).max(axis=1).reshape(ny, nx)
    assert np.array_equal(zmax > 6.0, want_ood)        # the input: only the culprits are out of range
    assert (np.abs(zmax - 6.0) > 0.1).all()
    got_ood = (corr == 0).all(axis=0)
    missed = np.argwhere(want_ood & ~got_ood)
    extra = np.argwhere(got_ood & ~want_ood)
    print(f"{dtype}: {want_ood.sum()} cells to zero, missed {missed[:8].tolist()}, extra {extra[:8].tolist()}",
          flush=True)
    assert np.array_equal(got_ood, want_ood)
    want = L.learned_correction(p, s64, c64, out_scale.astype(np.float64))(rho, mx, my, bx, by)
    rows = lambda a: (a / out_scale[:, None, None]).reshape(4, -1).T[~want_ood.ravel()]
    _compare_rows(rows(corr), rows(want), f"isolated out-of-range cells ({dtype})")


@pytest.mark.parametrize("dtype,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("nx,ny", [(64, 48), (67, 33)])
def test_learned_step_matches_oracle_given_the_correction(dtype, tol, nx, ny):
    """One learned-closure step from a given state equals the oracle step
    whose closure_correction returns the correction the GPU used."""
    G = _gpu()
    f, g = _smooth_state(nx, ny, 71)
    p = _params(72)
    shift, scale, out_scale, _, _ = _state_norm(f, g)
    s = _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale, dtype=dtype)
    st0 = s.get_state().cpu().numpy()
    for t0 in (0, 1):
        if t0 == 1:
            s.set_state(torch.from_numpy(st0), 1)
        corr = s.closure_correction().cpu().numpy().astype(np.float64)
        assert np.abs(corr).max() > 0
        s.step(1)
        got = s.get_state().cpu().numpy()
        o = O.Oracle(nx, ny, 0.02, 0.03, delta=2.0, s5=1.3, s6=1.5, s7=1.7, s8=1.1,
                     closure_correction=lambda *a: corr)
        o.set_state(st0[:9], np.stack([st0[9:14], st0[14:19]], axis=1))
        o.step(1)
        fo, go = o.state()[:2]
        want = np.concatenate([fo, go[:, 0], go[:, 1]], 0)
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        # and the correction mattered at this tolerance
        o2 = O.Oracle(nx, ny, 0.02, 0.03, delta=2.0, s5=1.3, s6=1.5, s7=1.7, s8=1.1)
        o2.set_state(st0[:9], np.stack([st0[9:14], st0[14:19]], axis=1))
        o2.step(1)
        f2, g2 = o2.state()[:2]
        effect = np.linalg.norm(np.concatenate([f2, g2[:, 0], g2[:, 1]], 0) - want) / np.linalg.norm(want)
        print(f"{dtype} {nx}x{ny} t0={t0}: relative L2 {err:.2e} (correction's effect {effect:.2e})", flush=True)
        assert err <= tol
        if dtype == "fp64":
            assert effect > 1e3 * tol
        s.set_state(torch.from_numpy(st0), 0)


@pytest.mark.parametrize("dtype,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_held_correction_matches_oracle(dtype, tol):
    """Correction interval 3 over 7 steps from a state injected at t = 2: the
    GPU evaluates the network at t = 2 (first step after the new state), 3 and
    6 and holds the correction in between, as the oracle with
    correction_every = 3 does when its hook returns the correction of the
    state the GPU holds at each step (that correction itself is checked
    against the oracle's network above)."""
    G = _gpu()
    nx, ny, K, t0, n = 64, 48, 3, 2, 7
    f, g = _smooth_state(nx, ny, 81)
    p = _params(82)
    shift, scale, out_scale, _, _ = _state_norm(f, g)
    s = _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale, dtype=dtype)
    s.set_correction_interval(K)
    st0 = s.get_state().cpu().numpy()
    s.set_state(torch.from_numpy(st0), t0)
    corrs = {}
    for t in range(t0, t0 + n):
        corrs[t] = s.closure_correction().cpu().numpy().astype(np.float64)
        s.step(1)
    got = s.get_state().cpu().numpy()
    kw = dict(delta=2.0, s5=1.3, s6=1.5, s7=1.7, s8=1.1)
    runs = {}
    for every in (K, 1):
        called = []
        o = O.Oracle(nx, ny, 0.02, 0.03, correction_every=every, **kw)
        o.closure_correction = lambda *a, o=o, called=called: (called.append(o.t), corrs[o.t])[1]
        o.set_state(st0[:9], np.stack([st0[9:14], st0[14:19]], axis=1), t=t0)
        o.step(n)
        fo, go = o.state()[:2]
        runs[every] = (np.concatenate([fo, go[:, 0], go[:, 1]], 0), called)
    want, called = runs[K]
    assert called == [2, 3, 6]
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    # holding the correction mattered at this tolerance
    effect = np.linalg.norm(runs[1][0] - want) / np.linalg.norm(want)
    print(f"{dtype}: relative L2 {err:.2e} (holding's effect {effect:.2e})", flush=True)
    assert err <= tol
    if dtype == "fp64":
        assert effect > 1e3 * tol
    # interval 1 is the every-step default, bit for bit
    a = _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale, dtype=dtype)
    b = _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale, dtype=dtype)
    b.set_correction_interval(1)
    a.step(3)
    b.step(3)
    assert torch.equal(a.get_state(), b.get_state())


@pytest.mark.parametrize("every", [1, 3])
@pytest.mark.parametrize("nx,ny", [(64, 48), (67, 33)])
def test_learned_run_matches_oracle_network(nx, ny, every):
    """Five FP64 learned steps (network every step, or every 3 steps with the
    correction held) against the oracle running its own network from the
    same host input: no value computed on the GPU enters the oracle.  The
    two networks agree to FP32 accumulation noise except for rare rows where
    a value within ~1e-7 of a bfloat16 rounding boundary rounds the other
    way, so the bound is set by the correction's own effect: the GPU run
    reproduces it to 1 % (a wrong sign, input permutation, output scale or
    cadence misses by O(1) of it)."""
    G = _gpu()
    f, g = _smooth_state(nx, ny, 91)
    p = _params(92)
    shift, scale, out_scale, s64, c64 = _state_norm(f, g)
    s = _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale, dtype="fp64")
    s.set_correction_interval(every)
    s.step(5)
    got = s.get_state().cpu().numpy()
    kw = dict(delta=2.0, s5=1.3, s6=1.5, s7=1.7, s8=1.1)
    hook = L.learned_correction(p, s64, c64, out_scale.astype(np.float64))
    runs = []
    for corr in (hook, None):
        o = O.Oracle(nx, ny, 0.02, 0.03, closure_correction=corr, correction_every=every, **kw)
        o.set_state(f, g)
        o.step(5)
        fo, go = o.state()[:2]
        runs.append(np.concatenate([fo, go[:, 0], go[:, 1]], 0))
    want, plain = runs
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    effect = np.linalg.norm(plain - want) / np.linalg.norm(want)
    print(f"{nx}x{ny} every {every}: relative L2 {err:.2e} (correction's effect {effect:.2e})", flush=True)
    assert effect > 1e-6
    assert err <= 1e-2 * effect


@pytest.mark.parametrize("every", [1, 3])
@pytest.mark.parametrize("nx,ny", [(300, 40), (1100, 20)])
def test_fp32_learned_run_matches_oracle_network(nx, ny, every):
    """FP32 storage on grids wide enough for the closure sweep's 256-lane
    strips (300 columns) and 512-lane strips (1100), each with a ragged last
    strip: five learned steps, the network every step or every 3 steps (the
    held correction then passes through the correction planes), against the
    oracle running its own network from the same host input.  Larger output
    scales than the FP64 test make the correction's effect (~1e-4) far
    exceed FP32 rounding, and the GPU run must reproduce it to 1 %."""
    G = _gpu()
    f, g = _smooth_state(nx, ny, 93)
    p = _params(94)
    shift, scale, _, s64, c64 = _state_norm(f, g)
    out_scale = np.array([3e-4, 2e-4, 3e-4, 1e-4], dtype=np.float32)
    s = _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale, dtype="fp32")
    s.set_correction_interval(every)
    s.step(5)
    got = s.get_state().cpu().numpy()
    kw = dict(delta=2.0, s5=1.3, s6=1.5, s7=1.7, s8=1.1)
    hook = L.learned_correction(p, s64, c64, out_scale.astype(np.float64))
    runs = []
    for corr in (hook, None):
        o = O.Oracle(nx, ny, 0.02, 0.03, closure_correction=corr, correction_every=every, **kw)
        o.set_state(f, g)
        o.step(5)
        fo, go = o.state()[:2]
        runs.append(np.concatenate([fo, go[:, 0], go[:, 1]], 0))
    want, plain = runs
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    effect = np.linalg.norm(plain - want) / np.linalg.norm(want)
    print(f"fp32 {nx}x{ny} every {every}: relative L2 {err:.2e} (correction's effect {effect:.2e})", flush=True)
    assert effect > 1e-5
    assert err <= 1e-2 * effect


# ---------------------------------------------------------------------------
# what the trained network gains (a priori, held-out seed)
# ---------------------------------------------------------------------------


def test_trained_network_beats_the_analytic_closure_a_priori():
    """Train on filtered DNS of two jets (256^2 DNS, Gaussian Delta = 16 fine
    cells, 4x subsampled to 64^2) with the GPU's own kernels, then compare the
    subgrid-term error on a held-out seed: analytic closure alone versus
    analytic plus the network's correction."""
    G = _gpu()
    from paper_1705_09807_amd import training as TR
    setup = TR.JetSetup(n_fine=256)
    Xtr, Ttr = TR.samples(setup, seeds=[1, 2], les_times=[500, 750, 1000, 1250])
    Xte, Tte = TR.samples(setup, seeds=[3], les_times=[750, 1000, 1250])
    mlp = G.Mlp(G.glorot_params(4))
    mlp.fit_norm(Xtr, Ttr)
    losses = TR.train(mlp, Xtr, Ttr, steps=1500, batch=2048, lr=3e-3)
    ana, lea, ood = TR.closure_errors(mlp, Xte, Tte)
    ana, lea = ana.cpu().numpy(), lea.cpu().numpy()
    ratio = lea / ana
    print(f"train loss {losses[0].item():.3e} -> {losses[-100:].mean().item():.3e}; held-out MSE ratio "
          f"learned/analytic per component {np.round(ratio, 3)}, total {lea.sum() / ana.sum():.3f}, "
          f"out of range {ood.item():.2%}", flush=True)
    assert np.isfinite(lea).all()
    assert lea.sum() < 0.8 * ana.sum()


@pytest.mark.parametrize("schedule", ["fused", "aa"])
@pytest.mark.parametrize("t0", [0, 1])
def test_init_from_moments_is_the_equilibrium(schedule, t0):
    """lbm_init_from_moments writes feq / geq (Sec. 2) of the given fields."""
    _gpu()
    from paper_1705_09807_amd import Sim
    nx, ny = 45, 31
    f, g = _smooth_state(nx, ny, 81)
    rho, mx, my, bx, by = O.Oracle._moments(f, g)
    mom = np.stack([rho, mx, my, bx, by])
    s = Sim(nx=nx, ny=ny, nu=0.02, eta=0.03, dtype="fp64", schedule=schedule)
    s.init_from_moments(torch.from_numpy(mom), t0)
    assert s.t == t0
    got = s.get_state().cpu().numpy()
    want = np.concatenate([O.f_equilibrium(rho, mx, my, bx, by),
                           O.g_equilibrium(rho, mx, my, bx, by)[:, 0],
                           O.g_equilibrium(rho, mx, my, bx, by)[:, 1]], 0)
    assert np.abs(got - want).max() <= 4e-16 * np.abs(want).max()
    back = s.moments().cpu().numpy()
    assert np.abs(back - mom).max() <= 1e-15


def test_non_finite_network_output_keeps_the_analytic_closure():
    """A network whose output is NaN leaves every cell on the analytic closure:
    the learned step then equals the analytic LES step."""
    _gpu()
    from paper_1705_09807_amd import learned as G
    nx, ny = 48, 40
    f, g = _smooth_state(nx, ny, 91)
    p = _params(92)
    p["b3"] = np.array([np.nan, 0.0, 0.0, 0.0])
    shift, scale, out_scale, s64, c64 = _state_norm(f, g)
    s = _learned_sim(G, nx, ny, f, g, p, shift, scale, out_scale)
    assert np.all(s.closure_correction().cpu().numpy() == 0)
    s.step(2)
    a = _sim_state(nx, ny, f, g, delta=2.0, s5=1.3, s6=1.5, s7=1.7, s8=1.1, b_ref=(0.01, 0.0))
    a.step(2)
    assert torch.equal(s.get_state(), a.get_state())


def test_full_size_learned_step_sampled():
    """The benchmark's learned leg: 1024^2 LES (Delta = 4, FP32 storage, MRT
    ghost rates 1.6) with the learned closure in its launch configuration,
    one step from the jet; 24 sampled cells against the oracle on the 7 x 7
    window around each, whose closure_correction hook returns the GPU's
    correction planes on that window (the network itself is checked against
    the oracle's above)."""
    G = _gpu()
    from paper_1705_09807_amd import Sim
    n, nu, B0 = 1024, 2e-4, 0.01
    kh = dict(U0=0.05, delta_over_L=1 / 40, B0=B0, rho0=1.0, pert_amp_over_U0=1e-2, noise_amp=1e-3)
    g4 = dict(s5=1.6, s6=1.6, s7=1.6, s8=1.6)
    p = _params(81)
    s = Sim(nx=n, ny=n, nu=nu, eta=nu, delta=4.0, dtype="fp32", b_ref=(B0, 0.0), closure="learned", **g4)
    s.init_kh_jet(seed=9, **kh)
    X = s.moments().cpu().numpy()
    feats = L.closure_features(*X[:, ::8, ::8])
    shift, scale, _ = L.feature_stats(feats, np.ones((feats.shape[0], 4)))
    m = _mlp(G, p, shift[::9][:7].astype(np.float32), scale[::9][:7].astype(np.float32),
             np.array([1e-3, 7e-4, 1e-3, 3e-4], dtype=np.float32))
    s.set_closure_mlp(m.pack())
    st0 = s.get_state().cpu().numpy()
    corr = s.closure_correction().cpu().numpy().astype(np.float64)
    assert np.abs(corr).max() > 0
    s.step(1)
    rng = np.random.default_rng(23)
    pts = [(0, 0), (n - 1, n - 1), (511, 512)] + [tuple(v) for v in rng.integers(0, n, size=(21, 2))]
    xs = torch.tensor([q[0] for q in pts], device=s.device)
    ys = torch.tensor([q[1] for q in pts], device=s.device)
    got = s.get_state()[:, ys, xs].cpu().numpy()
    win, half = 7, 3
    for k, (x, y) in enumerate(pts):
        gx = (x - half + np.arange(win)) % n
        gy = (y - half + np.arange(win)) % n
        w = st0[:, gy[:, None], gx[None, :]]
        cw = corr[:, gy[:, None], gx[None, :]]
        o = O.Oracle(win, win, nu, nu, delta=4.0, closure_correction=lambda *a, c=cw: c, **g4)
        o.set_state(w[:9], np.stack([w[9:14], w[14:19]], axis=1))
        o.step(1)
        fo, go_ = o.state()[:2]
        ref = np.concatenate([fo, go_[:, 0], go_[:, 1]], 0)[:, half, half]
        err = np.abs(got[:, k] - ref).max()
        assert err <= 2e-6, (x, y, err)
        if k < 4:   # the correction itself is far above the tolerance
            o0 = O.Oracle(win, win, nu, nu, delta=4.0, **g4)
            o0.set_state(w[:9], np.stack([w[9:14], w[14:19]], axis=1))
            o0.step(1)
            f0, g0 = o0.state()[:2]
            plain = np.concatenate([f0, g0[:, 0], g0[:, 1]], 0)[:, half, half]
            assert np.abs(plain - ref).max() > 50 * 2e-6, (x, y, np.abs(plain - ref).max())


@pytest.mark.parametrize("dtype", ["bf16", "fp16"])
def test_learned_step_16bit_beyond_the_caches_sampled(dtype):
    """16-bit storage with the state beyond the 256 MB Infinity Cache (2048^2:
    319 MB) runs the correction sweep in 256-lane strips; one learned step from
    the rounded state the GPU holds, 16 sampled cells against windowed oracle
    runs with the GPU's correction; bound: one rounding of each stored
    deviation (u |deviation|)."""
    G = _gpu()
    from paper_1705_09807_amd import Sim
    n, nu, B0 = 2048, 2e-4, 0.01
    unit = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}[dtype]
    kh = dict(U0=0.05, delta_over_L=1 / 40, B0=B0, rho0=1.0, pert_amp_over_U0=1e-2, noise_amp=1e-3)
    g4 = dict(s5=1.6, s6=1.6, s7=1.6, s8=1.6)
    p = _params(91)
    s = Sim(nx=n, ny=n, nu=nu, eta=nu, delta=4.0, dtype=dtype, b_ref=(B0, 0.0), closure="learned", **g4)
    s.init_kh_jet(seed=4, **kh)
    X = s.moments().cpu().numpy()
    feats = L.closure_features(*X[:, ::16, ::16])
    shift, scale, _ = L.feature_stats(feats, np.ones((feats.shape[0], 4)))
    m = _mlp(G, p, shift[::9][:7].astype(np.float32), scale[::9][:7].astype(np.float32),
             np.array([1e-3, 7e-4, 1e-3, 3e-4], dtype=np.float32))
    s.set_closure_mlp(m.pack())
    st0 = s.get_state().cpu().numpy()
    corr = s.closure_correction().cpu().numpy().astype(np.float64)
    s.step(1)
    rng = np.random.default_rng(29)
    pts = [(0, 0), (n - 1, n - 1), (255, 256), (256, 255)] + [tuple(v) for v in rng.integers(0, n, size=(12, 2))]
    xs = torch.tensor([q[0] for q in pts], device=s.device)
    ys = torch.tensor([q[1] for q in pts], device=s.device)
    got = s.get_state()[:, ys, xs].cpu().numpy()
    rest = np.concatenate([O.W9, O.W5 * B0, O.W5 * 0.0])
    win, half = 7, 3
    for k, (x, y) in enumerate(pts):
        gx = (x - half + np.arange(win)) % n
        gy = (y - half + np.arange(win)) % n
        w = st0[:, gy[:, None], gx[None, :]]
        cw = corr[:, gy[:, None], gx[None, :]]
        o = O.Oracle(win, win, nu, nu, delta=4.0, closure_correction=lambda *a, c=cw: c, **g4)
        o.set_state(w[:9], np.stack([w[9:14], w[14:19]], axis=1))
        o.step(1)
        fo, go_ = o.state()[:2]
        ref = np.concatenate([fo, go_[:, 0], go_[:, 1]], 0)[:, half, half]
        err = np.abs(got[:, k] - ref).max()
        bound = unit * np.abs(ref - rest).max() + 1e-6
        assert err <= bound, (x, y, err, bound)


def test_production_size_learned_bf16_step_sampled():
    """The production configuration's step: 16384^2 (268M cells), learned
    closure, BF16 storage, nu = eta = 5e-5, B0 = 0.02.  One step from the jet;
    12 sampled cells against windowed oracle runs fed the GPU's correction
    (windows gathered on the device); bound: one rounding of each stored
    deviation (u |deviation|)."""
    G = _gpu()
    from paper_1705_09807_amd import Sim
    n, nu, B0 = 16384, 5e-5, 0.02
    unit = 2.0 ** -8
    kh = dict(U0=0.05, delta_over_L=1 / 40, B0=B0, rho0=1.0, pert_amp_over_U0=1e-2, noise_amp=1e-3)
    g4 = dict(s5=1.6, s6=1.6, s7=1.6, s8=1.6)
    p = _params(97)
    s = Sim(nx=n, ny=n, nu=nu, eta=nu, delta=4.0, dtype="bf16", b_ref=(B0, 0.0), closure="learned", **g4)
    s.init_kh_jet(seed=6, **kh)
    mom = s.moments()
    X = mom[:, ::64, ::64].cpu().numpy()
    del mom
    feats = L.closure_features(*X)
    shift, scale, _ = L.feature_stats(feats, np.ones((feats.shape[0], 4)))
    m = _mlp(G, p, shift[::9][:7].astype(np.float32), scale[::9][:7].astype(np.float32),
             np.array([1e-3, 7e-4, 1e-3, 3e-4], dtype=np.float32))
    s.set_closure_mlp(m.pack())
    rng = np.random.default_rng(31)
    pts = [(0, 0), (n - 1, n - 1), (8191, 8192), (4095, 12288)] + [tuple(v) for v in rng.integers(0, n, size=(8, 2))]
    win, half = 7, 3
    iy = torch.tensor([[(y - half + i) % n for i in range(win)] for _, y in pts], device=s.device)
    ix = torch.tensor([[(x - half + i) % n for i in range(win)] for x, _ in pts], device=s.device)
    st = s.get_state()
    w0 = st[:, iy[:, :, None], ix[:, None, :]].cpu().numpy()      # [19, points, win, win]
    del st
    corr = s.closure_correction()
    cw0 = corr[:, iy[:, :, None], ix[:, None, :]].cpu().numpy().astype(np.float64)
    assert np.abs(cw0).max() > 0
    del corr
    torch.cuda.empty_cache()
    s.step(1)
    xs = torch.tensor([q[0] for q in pts], device=s.device)
    ys = torch.tensor([q[1] for q in pts], device=s.device)
    st = s.get_state()
    got = st[:, ys, xs].cpu().numpy()
    del st
    assert s.diagnostics()["nonfinite"] == 0
    s.close()
    torch.cuda.empty_cache()
    rest = np.concatenate([O.W9, O.W5 * B0, O.W5 * 0.0])
    for k, (x, y) in enumerate(pts):
        w, cw = w0[:, k], cw0[:, k]
        o = O.Oracle(win, win, nu, nu, delta=4.0, closure_correction=lambda *a, c=cw: c, **g4)
        o.set_state(w[:9], np.stack([w[9:14], w[14:19]], axis=1))
        o.step(1)
        fo, go_ = o.state()[:2]
        ref = np.concatenate([fo, go_[:, 0], go_[:, 1]], 0)[:, half, half]
        err = np.abs(got[:, k] - ref).max()
        bound = unit * np.abs(ref - rest).max() + 1e-6
        assert err <= bound, (x, y, err, bound)
