"""GPU parity of the closure with gradients from local non-equilibrium
moments (LBM_STENCIL_LOCAL_*: strain from M3, M4, grad B from the first
moments of g, vorticity from the stencil) against the oracle's
grad_stencil='local_*'.  Tolerances as for the stencil closure."""

import numpy as np
import pytest

from oracle import lbmhd_oracle as O
from seeded_inputs import perturbed, offset_noise

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


@pytest.mark.parametrize("schedule", ["fused", "aa"])
def test_kh_64_fp64_every_step(schedule):
    n, steps = 64, 300
    s = _sim(nx=n, ny=n, nu=1e-3, eta=1e-3, delta=2.0, dtype="fp64", schedule=schedule, grad_stencil="local_iso9")
    o = O.Oracle(n, n, 1e-3, 1e-3, delta=2.0, grad_stencil="local_iso9")
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
    print(f"local {schedule} fp64: worst relative L2 over {steps} steps {worst:.2e}", flush=True)


@pytest.mark.parametrize("schedule", ["fused", "aa"])
def test_kh_64_fp32_100_steps(schedule):
    n = 64
    s = _sim(nx=n, ny=n, nu=1e-3, eta=1e-3, delta=2.0, dtype="fp32", schedule=schedule, grad_stencil="local_iso9",
             b_ref=(0.01, 0.0))
    o = O.Oracle(n, n, 1e-3, 1e-3, delta=2.0, grad_stencil="local_iso9")
    s.init_kh_jet(seed=1, **KH0)
    o.init_kh_jet(seed=1, **KH0)
    s.step(100)
    o.step(100)
    e = rel(s.get_state().cpu().numpy(), pack(*o.state()[:2]))
    print(f"local {schedule} fp32 after 100 steps: {e:.2e}", flush=True)
    assert e <= 1e-5


@pytest.mark.parametrize("case", [(33, 17, 1.0, "local_iso9"), (70, 9, 4.0, "local_central5"),
                                  (130, 66, 4.0, "local_iso9"), (4, 4, 2.0, "local_iso9"),
                                  (257, 10, 2.0, "local_iso9"), (513, 6, 3.0, "local_central5")])
@pytest.mark.parametrize("schedule", ["fused", "aa"])
@pytest.mark.parametrize("t0", [0, 1])
def test_random_state_steps_fp64(case, schedule, t0):
    nx, ny, delta, stencil = case
    f = perturbed(O.W9, (9, ny, nx), 400 + nx, 0.15)
    g = offset_noise(np.zeros(10), (10, ny, nx), 401 + nx, 0.01).reshape(5, 2, ny, nx)
    s = _sim(nx=nx, ny=ny, nu=0.02, eta=0.03, delta=delta, grad_stencil=stencil, dtype="fp64", schedule=schedule,
             s5=1.2, s6=0.9, s7=1.5, s8=1.1)
    o = O.Oracle(nx, ny, 0.02, 0.03, delta=delta, grad_stencil=stencil, s5=1.2, s6=0.9, s7=1.5, s8=1.1)
    s.set_state(torch.from_numpy(pack(f, g)), t=t0)
    o.set_state(f, g, t=t0)
    for _ in range(2):
        s.step(1)
        o.step(1)
        d = np.abs(s.get_state().cpu().numpy() - pack(*o.state()[:2])).max()
        assert d <= 1e-14, d
