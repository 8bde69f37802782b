"""GPU parity of the 16-bit storage modes (FP16 deviations x 2^8, BF16
deviations; FP32 arithmetic) against the FP64 oracle.

Tolerances follow from the storage's unit roundoff u (FP16: 2^-11, BF16: 2^-8):
every step rounds each stored deviation once, to within u of its value, so
* one step from a given (already rounded) state: every population within
  u * max|deviation| (+ FP32 arithmetic noise);
* after n steps the per-field relative L2 error of rho, m and B, whose
  rounding errors accumulate like a random walk, within sqrt(n) * u.
Measured errors are printed.
"""

import math

import numpy as np
import pytest

from oracle import lbmhd_oracle as O
from seeded_inputs import perturbed, offset_noise

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

UNIT = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}
KH0 = dict(U0=0.05, delta_over_L=0.05, B0=0.01, rho0=1.0, pert_amp_over_U0=1e-3, noise_amp=1e-5)


def _sim(**kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09807_amd import Sim
    return Sim(**kw)


def pack(f, g):
    return np.concatenate([f, g[:, 0], g[:, 1]], 0)


def unpack(s):
    return s[:9], np.stack([s[9:14], s[14:19]], axis=1)


def deviation(state, bx0=0.0, by0=0.0):
    d = state.copy()
    d[:9] -= O.W9[:, None, None]
    d[9:14] -= O.W5[:, None, None] * bx0
    d[14:19] -= O.W5[:, None, None] * by0
    return d


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dtype", ["fp16", "bf16"])
def test_initial_state(dtype):
    nx, ny = 48, 40
    s = _sim(nx=nx, ny=ny, nu=1e-3, eta=1e-3, delta=2.0, dtype=dtype, b_ref=(0.01, 0.0))
    s.init_kh_jet(seed=7, **KH0)
    o = O.Oracle(nx, ny, 1e-3, 1e-3, delta=2.0)
    o.init_kh_jet(seed=7, **KH0)
    ref = pack(*o.state()[:2])
    dev = deviation(ref, 0.01)
    err = np.abs(s.get_state().cpu().numpy() - ref)
    # each stored deviation rounded once: within u * |deviation| (+ FP64->FP32 noise)
    assert np.all(err <= UNIT[dtype] * np.abs(dev) + 1e-9)


@pytest.mark.parametrize("dtype", ["fp16", "bf16"])
@pytest.mark.parametrize("schedule", ["fused", "aa"])
@pytest.mark.parametrize("delta", [0.0, 2.0])
@pytest.mark.parametrize("shape", [(33, 17), (68, 12), (258, 5), (300, 7)])
def test_one_step_from_random_state(dtype, schedule, delta, shape):
    """Odd widths (one cell per thread), widths divisible by 4 (the four-cell
    closure-off sweep), a width of two mod 4 (the two-cell one).  300 x 7:
    two row segments per row, the second ragged, and 14 workgroups in the
    one-dimensional grids (not a multiple of the 8 XCDs the workgroups are
    numbered over); likewise two closure-sweep strips, the second ragged."""
    nx, ny = shape
    f = perturbed(O.W9, (9, ny, nx), 5, 0.15)
    g = offset_noise(np.zeros(10), (10, ny, nx), 6, 0.01).reshape(5, 2, ny, nx)
    s = _sim(nx=nx, ny=ny, nu=0.02, eta=0.03, delta=delta, dtype=dtype, schedule=schedule)
    for t0 in (0, 1):
        s.set_state(torch.from_numpy(pack(f, g)), t0)
        st0 = s.get_state().cpu().numpy()       # the rounded state the GPU holds
        s.step(1)
        o = O.Oracle(nx, ny, 0.02, 0.03, delta=delta)
        o.set_state(*unpack(st0))
        o.step(1)
        ref = pack(*o.state()[:2])
        err = np.abs(s.get_state().cpu().numpy() - ref).max()
        bound = UNIT[dtype] * np.abs(deviation(ref)).max() + 1e-6
        print(f"{dtype} {schedule} delta={delta} t0={t0}: max error {err:.2e}, bound {bound:.2e}", flush=True)
        assert err <= bound


@pytest.mark.parametrize("dtype", ["fp16", "bf16"])
@pytest.mark.parametrize("ny", [512, 768, 1280])
def test_closure_sweep_segment_heights(dtype, ny):
    """64-column grids of 512, 768 and 1280 rows give the closure sweep
    segments of 2, 3 and 5 rows on a 256-CU device, so the FP16 sweep's
    three-way unrolled row loop ends in each of its phases; three steps, each
    from the rounded state the GPU holds, against the oracle."""
    nx = 64
    f = perturbed(O.W9, (9, ny, nx), 15, 0.15)
    g = offset_noise(np.zeros(10), (10, ny, nx), 16, 0.01).reshape(5, 2, ny, nx)
    s = _sim(nx=nx, ny=ny, nu=0.02, eta=0.03, delta=2.0, dtype=dtype)
    s.set_state(torch.from_numpy(pack(f, g)), 0)
    for step in range(3):
        st0 = s.get_state().cpu().numpy()
        s.step(1)
        o = O.Oracle(nx, ny, 0.02, 0.03, delta=2.0)
        o.set_state(*unpack(st0))
        o.step(1)
        ref = pack(*o.state()[:2])
        err = np.abs(s.get_state().cpu().numpy() - ref).max()
        bound = UNIT[dtype] * np.abs(deviation(ref)).max() + 1e-6
        print(f"{dtype} 64x{ny} step {step}: max error {err:.2e}, bound {bound:.2e}", flush=True)
        assert err <= bound


@pytest.mark.parametrize("dtype", ["fp16", "bf16"])
@pytest.mark.parametrize("steps", [100, 1000])
def test_kh_64_fields(dtype, steps):
    """Per-field relative L2 of rho, m, B after n steps of the 64^2 LES jet
    within sqrt(n) * u."""
    n = 64
    o = O.Oracle(n, n, 1e-3, 1e-3, delta=2.0)
    o.init_kh_jet(seed=1, **KH0)
    o.step(steps)
    mo = np.stack(o.moments())
    s = _sim(nx=n, ny=n, nu=1e-3, eta=1e-3, delta=2.0, dtype=dtype, b_ref=(0.01, 0.0))
    s.init_kh_jet(seed=1, **KH0)
    s.step(steps)
    m = s.moments().cpu().numpy()
    e = {"rho": rel(m[0], mo[0]), "m": rel(m[1:3], mo[1:3]), "B": rel(m[3:5], mo[3:5])}
    bound = math.sqrt(steps) * UNIT[dtype]
    print(f"{dtype} after {steps} steps: {e} (bound {bound:.2e})", flush=True)
    for key, v in e.items():
        assert v <= bound, (key, v, bound)


@pytest.mark.parametrize("dtype", ["fp16", "bf16"])
@pytest.mark.parametrize("delta", [0.0, 4.0])
def test_ragged_wide_sampled(dtype, delta):
    """Streaming stores on a ragged 5000 x 1701 grid (650 MB of 16-bit state):
    the closure-off sweep's 256-cell row segments end with one of 136 cells
    and its grid has 34 020 workgroups; the closure sweep's ten 512-lane
    strips end with one of 392 columns, in 51 segments of 34 rows (510
    workgroups).  Neither count is a multiple of the 8 XCDs over which the
    workgroups are numbered.  The jet (B0 = 0.01, nu = eta = 1e-4) after 3
    steps at cells on segment, strip and grid edges and at random, against
    the oracle on a window around each; bound: 3 roundings of u * |deviation|."""
    nx, ny, steps, nu, B0 = 5000, 1701, 3, 1e-4, 0.01
    kh = dict(U0=0.05, delta_over_L=1 / 40, B0=B0, rho0=1.0, pert_amp_over_U0=1e-3, noise_amp=1e-5)
    g4 = dict(s5=1.6, s6=1.6, s7=1.6, s8=1.6)
    s = _sim(nx=nx, ny=ny, nu=nu, eta=nu, delta=delta, dtype=dtype, b_ref=(B0, 0.0), **g4)
    s.init_kh_jet(seed=15, **kh)
    d0 = s.diagnostics()
    s.step(steps)
    rng = np.random.default_rng(16)
    pts = [(0, 0), (nx - 1, ny - 1), (nx - 1, 0), (0, ny - 1), (4863, 850), (4864, 851), (511, 33), (512, 34),
           (4607, 1666), (4608, 1700), (255, 1699), (256, 425)]
    pts += [(int(rng.integers(0, nx)), int(rng.integers(0, ny))) for _ in range(12)]
    xs = torch.tensor([p[0] for p in pts], device=s.device)
    ys = torch.tensor([p[1] for p in pts], device=s.device)
    st = s.get_state()
    got = st[:, ys, xs].cpu().numpy()
    del st
    win = 2 * (2 * steps + 1) + 1
    half = win // 2
    worst = 0.0
    for k, (x, y) in enumerate(pts):
        X, Y = np.meshgrid((x - half + np.arange(win)) % nx, (y - half + np.arange(win)) % ny)
        f, g = O.kh_jet_populations(X, Y, nx, ny, seed=15, **kh)
        o = O.Oracle(win, win, nu, nu, delta=delta, **g4)
        o.set_state(f, g)
        o.step(steps)
        ref = pack(*o.state()[:2])[:, half, half]
        dev = deviation(ref[:, None, None], B0)[:, 0, 0]
        err = np.abs(got[:, k] - ref).max()
        worst = max(worst, err / np.abs(dev).max())
        assert err <= (steps + 1) * UNIT[dtype] * np.abs(dev).max() + 1e-6, (x, y, err)
    print(f"{dtype} delta={delta} {nx}x{ny}: worst sampled error / max|deviation| = {worst:.2e}", flush=True)
    d = s.diagnostics()
    assert d["nonfinite"] == 0
    assert abs(d["mass"] - d0["mass"]) <= steps * UNIT[dtype] * 0.05 * nx * ny
    s.close()


@pytest.mark.parametrize("dtype", ["fp16", "bf16"])
@pytest.mark.parametrize("delta", [0.0, 4.0])
def test_full_size_8192_sampled(dtype, delta):
    """The 8192^2 jet (B0 = 0.01, nu = eta = 1e-4, MRT ghost rates 1.6) in the
    benchmark's launch configuration: 3 steps, 24 sampled cells against the
    oracle run on a window around each cell (state after k steps depends on
    the initial state within 2k cells).  Bound: 3 roundings of u * |deviation|."""
    n, steps, nu, B0 = 8192, 3, 1e-4, 0.01
    kh = dict(U0=0.05, delta_over_L=1 / 40, B0=B0, rho0=1.0, pert_amp_over_U0=1e-3, noise_amp=1e-5)
    g4 = dict(s5=1.6, s6=1.6, s7=1.6, s8=1.6)
    s = _sim(nx=n, ny=n, nu=nu, eta=nu, delta=delta, dtype=dtype, b_ref=(B0, 0.0), **g4)
    s.init_kh_jet(seed=13, **kh)
    d0 = s.diagnostics()
    s.step(steps)
    rng = np.random.default_rng(14)
    pts = [(0, 0), (n - 1, n - 1), (n // 4, n // 4)] + [tuple(v) for v in rng.integers(0, n, size=(21, 2))]
    xs = torch.tensor([p[0] for p in pts], device=s.device)
    ys = torch.tensor([p[1] for p in pts], device=s.device)
    st = s.get_state()
    got = st[:, ys, xs].cpu().numpy()
    del st
    win = 2 * (2 * steps + 1) + 1
    half = win // 2
    worst = 0.0
    for k, (x, y) in enumerate(pts):
        X, Y = np.meshgrid((x - half + np.arange(win)) % n, (y - half + np.arange(win)) % n)
        f, g = O.kh_jet_populations(X, Y, n, n, seed=13, **kh)
        o = O.Oracle(win, win, nu, nu, delta=delta, **g4)
        o.set_state(f, g)
        o.step(steps)
        ref = pack(*o.state()[:2])[:, half, half]
        dev = deviation(ref[:, None, None], B0)[:, 0, 0]
        err = np.abs(got[:, k] - ref).max()
        worst = max(worst, err / np.abs(dev).max())
        assert err <= (steps + 1) * UNIT[dtype] * np.abs(dev).max() + 1e-6, (x, y, err)
    print(f"{dtype} delta={delta}: worst sampled error / max|deviation| = {worst:.2e}", flush=True)
    d = s.diagnostics()
    assert d["nonfinite"] == 0
    # mass: each step rounds every stored deviation (|f_i - w_i rho0| <= 0.05 per cell summed)
    assert abs(d["mass"] - d0["mass"]) <= steps * UNIT[dtype] * 0.05 * n * n
