"""GPU parity of the single-sweep in-place schedule with lagged closure
gradients (LBM_SCHED_AA_LAGGED) against the oracle's closure_time='lagged'.
Same tolerances as the synchronous schedules: FP64 <= 1e-12 relative L2 at
every step of the 64^2 jet, FP32 <= 1e-5 after 100 steps, two-to-three steps
from random states within 1e-14 per population."""

import numpy as np
import pytest

from oracle import lbmhd_oracle as O
from sampled_windows import check_rough_sampled
from seeded_inputs import ROUGH_MEAN, assemble_rough_torch, offset_noise, perturbed, rough_factors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KH0 = dict(U0=0.05, delta_over_L=0.05, B0=0.01, rho0=1.0, pert_amp_over_U0=1e-3, noise_amp=1e-5)


def _sim(**kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_09807_amd import Sim
    return Sim(**kw)


def pack(f, g):
    return np.concatenate([f, g[:, 0], g[:, 1]], 0)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_kh_64_fp64_every_step():
    n, steps = 64, 500
    s = _sim(nx=n, ny=n, nu=1e-3, eta=1e-3, delta=2.0, dtype="fp64", schedule="aa_lagged")
    o = O.Oracle(n, n, 1e-3, 1e-3, delta=2.0, closure_time="lagged")
    s.init_kh_jet(seed=0, **KH0)
    o.init_kh_jet(seed=0, **KH0)
    worst = 0.0
    for k in range(1, steps + 1):
        s.step(1)
        o.step(1)
        mg, mo = s.moments().cpu().numpy(), np.stack(o.moments())
        for sl in (slice(0, 1), slice(1, 3), slice(3, 5)):
            e = rel(mg[sl], mo[sl])
            worst = max(worst, e)
            assert e <= 1e-12, (k, sl, e)
    print(f"lagged fp64: worst relative L2 over {steps} steps {worst:.2e}", flush=True)


def test_kh_64_fp32_100_steps():
    n = 64
    s = _sim(nx=n, ny=n, nu=1e-3, eta=1e-3, delta=2.0, dtype="fp32", schedule="aa_lagged", b_ref=(0.01, 0.0))
    o = O.Oracle(n, n, 1e-3, 1e-3, delta=2.0, closure_time="lagged")
    s.init_kh_jet(seed=1, **KH0)
    o.init_kh_jet(seed=1, **KH0)
    s.step(100)
    o.step(100)
    e = rel(s.get_state().cpu().numpy(), pack(*o.state()[:2]))
    print(f"lagged fp32 after 100 steps: {e:.2e}", flush=True)
    assert e <= 1e-5


@pytest.mark.parametrize("case", [(33, 17, 1.0, "iso9"), (70, 9, 4.0, "central5"), (130, 66, 4.0, "iso9"),
                                  (4, 4, 2.0, "iso9"), (257, 10, 2.0, "iso9")])
@pytest.mark.parametrize("t0", [0, 1])
def test_random_state_steps_fp64(case, t0):
    nx, ny, delta, stencil = case
    f = perturbed(O.W9, (9, ny, nx), 300 + nx, 0.15)
    g = offset_noise(np.zeros(10), (10, ny, nx), 301 + nx, 0.01).reshape(5, 2, ny, nx)
    s = _sim(nx=nx, ny=ny, nu=0.02, eta=0.03, delta=delta, grad_stencil=stencil, dtype="fp64", schedule="aa_lagged",
             s5=1.2, s6=0.9, s7=1.5, s8=1.1)
    o = O.Oracle(nx, ny, 0.02, 0.03, delta=delta, grad_stencil=stencil, s5=1.2, s6=0.9, s7=1.5, s8=1.1,
                 closure_time="lagged")
    s.set_state(torch.from_numpy(pack(f, g)), t=t0)
    o.set_state(f, g, t=t0)
    for _ in range(3):
        s.step(1)
        o.step(1)
        d = np.abs(s.get_state().cpu().numpy() - pack(*o.state()[:2])).max()
        assert d <= 1e-14, d


def test_lag_changes_the_result_and_restarts_synchronously():
    nx, ny = 48, 40
    f = perturbed(O.W9, (9, ny, nx), 7, 0.1)
    g = offset_noise(np.zeros(10), (10, ny, nx), 8, 0.01).reshape(5, 2, ny, nx)
    lag = _sim(nx=nx, ny=ny, nu=0.02, eta=0.03, delta=3.0, dtype="fp64", schedule="aa_lagged")
    syn = _sim(nx=nx, ny=ny, nu=0.02, eta=0.03, delta=3.0, dtype="fp64", schedule="aa")
    st = torch.from_numpy(pack(f, g))
    lag.set_state(st)
    syn.set_state(st)
    lag.step(1)
    syn.step(1)
    assert torch.equal(lag.get_state(), syn.get_state())          # the first step is synchronous
    lag.step(2)
    syn.step(2)
    assert (lag.get_state() - syn.get_state()).abs().max().item() > 1e-8
    mid = syn.get_state()
    lag.set_state(mid, syn.t)                                       # re-injection: synchronous again
    lag.step(1)
    syn.step(1)
    assert torch.equal(lag.get_state(), syn.get_state())


VARIANTS = [
    # label, schedule, grad_stencil, oracle closure_time
    ("local_fused", "fused", "local_iso9", "sync"),
    ("local_aa", "aa", "local_iso9", "sync"),
    ("lagged", "aa_lagged", "iso9", "lagged"),
]


@pytest.mark.parametrize("variant", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_full_size_variants_sampled(variant):
    """4096^2 FP32 LES (Delta = 4) of the lagged and local-gradient variants in
    the benchmark's launch configuration: 3 steps from rough fields, 24
    sampled cells against the oracle in the same mode on the 15 x 15 window
    around each; the same windows without the closure, and with the
    synchronous stencil closure, sit far outside the tolerance."""
    label, schedule, stencil, ctime = variant
    n, nu, steps, delta = 4096, 2e-4, 3, 4.0
    g4 = dict(s5=1.6, s6=1.6, s7=1.6, s8=1.6)
    s = _sim(nx=n, ny=n, nu=nu, eta=nu, delta=delta, dtype="fp32", schedule=schedule, grad_stencil=stencil,
             b_ref=(ROUGH_MEAN[3], ROUGH_MEAN[4]), **g4)
    factors = rough_factors(n, n, 19)
    s.init_from_moments(assemble_rough_torch(factors, torch, s.device))
    s._keep = None
    s.step(steps)
    rng = np.random.default_rng(31)
    pts = [(0, 0), (n - 1, n - 1), (255, 256), (256, 255), (511, 127), (512, 128)] + \
        [tuple(int(v) for v in q) for q in rng.integers(0, n, size=(18, 2))]
    xs = torch.tensor([q[0] for q in pts], device=s.device)
    ys = torch.tensor([q[1] for q in pts], device=s.device)
    got = s.get_state()[:, ys, xs].cpu().numpy()
    gaps = [("no closure", dict(delta=0.0, grad_stencil="iso9", closure_time="sync"), 100.0),
            ("synchronous stencil closure", dict(grad_stencil="iso9", closure_time="sync"), 30.0)]
    check_rough_sampled(got, pts, n, steps, factors, 1e-7, gaps=gaps, say=print,
                        nu=nu, eta=nu, delta=delta, grad_stencil=stencil, closure_time=ctime, **g4)
    s.close()


RAGGED_VARIANTS = VARIANTS + [("stencil_aa", "aa", "iso9", "sync")]


@pytest.mark.parametrize("variant", RAGGED_VARIANTS, ids=[v[0] for v in RAGGED_VARIANTS])
def test_ragged_variants_sampled(variant):
    """The same variants, and the in-place schedule with the stencil closure,
    on a ragged 5000 x 1701 grid: the in-place kernels' 256-cell row segments
    end with one of 136 cells and their grid has 34 020 workgroups (not a
    multiple of the 8 XCDs they are numbered over).  3 steps from rough
    fields, cells at segment and grid edges and at random."""
    label, schedule, stencil, ctime = variant
    nx, ny, nu, steps, delta = 5000, 1701, 2e-4, 3, 4.0
    g4 = dict(s5=1.6, s6=1.6, s7=1.6, s8=1.6)
    s = _sim(nx=nx, ny=ny, nu=nu, eta=nu, delta=delta, dtype="fp32", schedule=schedule, grad_stencil=stencil,
             b_ref=(ROUGH_MEAN[3], ROUGH_MEAN[4]), **g4)
    factors = rough_factors(nx, ny, 23)
    s.init_from_moments(assemble_rough_torch(factors, torch, s.device))
    s._keep = None
    s.step(steps)
    rng = np.random.default_rng(37)
    pts = [(0, 0), (nx - 1, ny - 1), (nx - 1, 0), (0, ny - 1), (255, 850), (256, 851), (4863, 1700),
           (4864, 33), (511, 34), (512, 1666)]
    pts += [(int(rng.integers(0, nx)), int(rng.integers(0, ny))) for _ in range(10)]
    xs = torch.tensor([q[0] for q in pts], device=s.device)
    ys = torch.tensor([q[1] for q in pts], device=s.device)
    got = s.get_state()[:, ys, xs].cpu().numpy()
    gaps = [("no closure", dict(delta=0.0, grad_stencil="iso9", closure_time="sync"), 100.0)]
    check_rough_sampled(got, pts, nx, steps, factors, 1e-7, gaps=gaps, say=print, ny=ny,
                        nu=nu, eta=nu, delta=delta, grad_stencil=stencil, closure_time=ctime, **g4)
    s.close()
