"""Filtered-DNS training of the learned closure, composed from the ABI.

Every numerical step runs in the library's kernels: the DNS timestep, the
moments, the Gaussian filter and subsampling, the closure samples (network
inputs and exact-minus-analytic targets), the normalisation statistics, the
network's forward and backward passes and Adam.  This module only sequences
the calls and concatenates or indexes device tensors.

Grid convention: a DNS on an N x N grid is filtered with a Gaussian of width
`delta_fine` fine cells and sampled every `factor` cells; the LES it trains
runs on the (N/factor)^2 grid with Delta = delta_fine / factor of its own
cells.  At constant Reynolds number the DNS viscosity is factor times the
LES one and one LES step spans factor DNS steps.
"""

from __future__ import annotations

from dataclasses import dataclass

from . import learned as G
from .sim import Sim


@dataclass
class JetSetup:
    """A Kelvin-Helmholtz jet and the lattice parameters of the DNS that
    resolves it.  With `modes` empty the jet is lbm_init_kh_jet's (one
    sin(2 pi x / L) perturbation); otherwise the DNS starts from
    jet_fields(): the same shear layers with the given streamwise modes,
    amplitude mode_amp * U0 each and seeded phases, concentrated on the two
    layers, plus seeded white noise."""
    n_fine: int = 256
    factor: int = 4
    delta_fine: float = 16.0
    nu_les: float = 2e-4
    eta_les: float = 0.0          # <= 0: equal to nu_les
    ghost: float = 1.6
    U0: float = 0.05
    delta_over_L: float = 1.0 / 40.0
    B0: float = 0.01
    pert_amp_over_U0: float = 0.02
    noise_amp: float = 2e-3
    dtype: str = "fp32"
    modes: tuple = ()
    mode_amp: float = 0.01

    @property
    def nu_dns(self) -> float:
        return self.nu_les * self.factor

    @property
    def eta(self) -> float:
        return self.eta_les if self.eta_les > 0 else self.nu_les

    @property
    def eta_dns(self) -> float:
        return self.eta * self.factor

    @property
    def n_les(self) -> int:
        return self.n_fine // self.factor

    @property
    def delta_les(self) -> float:
        return self.delta_fine / self.factor

    def kh(self, seed: int) -> dict:
        return dict(U0=self.U0, delta_over_L=self.delta_over_L, B0=self.B0, rho0=1.0,
                    pert_amp_over_U0=self.pert_amp_over_U0, noise_amp=self.noise_amp, seed=seed)


def jet_fields(setup: JetSetup, n: int, seed: int, device="cuda:0"):
    """[5, n, n] float64 input fields (rho, m_x, m_y, B_x, B_y) of the
    multi-mode jet: u_x = U0 [tanh((y - L/4)/d) - tanh((y - 3L/4)/d) - 1],
    u_y = U0 mode_amp sum_m sin(2 pi m x / L + phi_m) (g(y - L/4) + g(y - 3L/4))
    with g(s) = exp(-(s / 2d)^2), phases phi_m uniform from `seed`, plus
    noise_amp times seeded uniform noise on [-1, 1); rho = 1, B = (B0, 0).
    This is an input recipe (seeded synthetic initial data), not a step of
    the method."""
    import math

    import torch
    gen = torch.Generator().manual_seed(int(seed))
    L = float(n)
    d = setup.delta_over_L * L
    y = torch.arange(n, dtype=torch.float64)[:, None]
    x = torch.arange(n, dtype=torch.float64)[None, :]
    ux = setup.U0 * (torch.tanh((y - L / 4) / d) - torch.tanh((y - 3 * L / 4) / d) - 1.0) * torch.ones_like(x)
    env = torch.exp(-((y - L / 4) / (2 * d)) ** 2) + torch.exp(-((y - 3 * L / 4) / (2 * d)) ** 2)
    uy = torch.zeros(n, n, dtype=torch.float64)
    for m in setup.modes:
        phi = float(torch.rand(1, generator=gen, dtype=torch.float64)) * 2 * math.pi
        uy += setup.U0 * setup.mode_amp * torch.sin(2 * math.pi * m * x / L + phi) * env
    uy += setup.noise_amp * (2 * torch.rand(n, n, generator=gen, dtype=torch.float64) - 1)
    mom = torch.stack([torch.ones(n, n, dtype=torch.float64), ux, uy,
                       torch.full((n, n), setup.B0, dtype=torch.float64), torch.zeros(n, n, dtype=torch.float64)])
    return mom.to(device)


def dns(setup: JetSetup, seed: int) -> Sim:
    g = setup.ghost
    s = Sim(nx=setup.n_fine, ny=setup.n_fine, nu=setup.nu_dns, eta=setup.eta_dns, delta=0.0, s5=g, s6=g, s7=g, s8=g,
            dtype=setup.dtype, b_ref=(setup.B0, 0.0))
    if setup.modes:
        s.init_from_moments(jet_fields(setup, setup.n_fine, seed, s.device))
    else:
        s.init_kh_jet(**setup.kh(seed))
    return s


def les(setup: JetSetup, seed: int, closure: str = "analytic", mlp=None, dtype=None) -> Sim:
    """The LES of the same jet on the coarse grid (analytic or learned closure)."""
    g = setup.ghost
    s = Sim(nx=setup.n_les, ny=setup.n_les, nu=setup.nu_les, eta=setup.eta, delta=setup.delta_les,
            s5=g, s6=g, s7=g, s8=g, dtype=dtype or setup.dtype, b_ref=(setup.B0, 0.0), closure=closure)
    s.init_kh_jet(**setup.kh(seed))
    if closure == "learned":
        s.set_closure_mlp(mlp.pack())
    return s


def filtered(setup: JetSetup, sim: Sim):
    """[12, n_les, n_les] filtered fields and products of a DNS state."""
    return G.filter_subsample(sim.moments(), setup.factor, setup.delta_fine)


def samples(setup: JetSetup, seeds, les_times, stencil="iso9", progress=None):
    """(X, T) closure samples of every coarse cell at the given LES times
    (DNS times factor x larger) for each seed, concatenated on the device.
    `progress(seed, t)` (optional) is called after each snapshot."""
    import torch
    xs, ts = [], []
    for seed in seeds:
        s = dns(setup, seed)
        for t in sorted(les_times):
            s.step(t * setup.factor - s.t)
            X, T = G.closure_samples(filtered(setup, s), setup.delta_les, stencil)
            xs.append(X)
            ts.append(T)
            if progress is not None:
                progress(seed, t)
        s.close()
    return torch.cat(xs), torch.cat(ts)


def train(mlp, X, T, steps: int, batch: int = 4096, lr: float = 2e-3, seed: int = 0, lr_final: float = 1e-4):
    """Adam over random mini-batches with a geometric learning-rate decay from
    lr to lr_final; returns the loss of every step (device tensor)."""
    import torch
    gen = torch.Generator(device=X.device).manual_seed(int(seed))
    n = X.shape[0]
    losses = torch.empty(steps, device=X.device)
    for k in range(steps):
        idx = torch.randint(0, n, (batch,), device=X.device, generator=gen, dtype=torch.int32)
        rate = lr * (lr_final / lr) ** (k / max(steps - 1, 1))
        losses[k:k + 1] = mlp.train_step(X, T, idx, rate)
    return losses


def closure_errors(mlp, X, T):
    """A-priori mean squared errors of the subgrid terms, per component, for
    the analytic closure alone (T itself: exact minus analytic) and with the
    network's correction (T - out_scale * y; out-of-distribution rows keep the
    analytic closure).  Returns (analytic, learned, ood_fraction) as tensors."""
    y, ood = mlp.forward(X)
    corr = y * mlp.norm[16:20]
    corr = corr.masked_fill(ood.bool()[:, None], 0.0)
    return (T.double() ** 2).mean(0), ((T - corr).double() ** 2).mean(0), ood.float().mean()
