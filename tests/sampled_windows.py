"""Sampled parity at full size: the oracle on a window around each sampled cell.

After k steps a cell depends only on the initial state within 2k cells (one
cell per step from streaming, one from the closure's 3x3 stencil), so an
oracle run on the periodic window of half-width 2k + 1 around the cell gives
that cell's reference exactly.  The gap check runs the same windows with a
different closure (no closure, the other stencil) to show that the
comparison can see the closure: a kernel that dropped or mis-indexed it would
land at least that far away.
"""

from __future__ import annotations

import numpy as np

from oracle import lbmhd_oracle as O
from seeded_inputs import assemble_rough


def window(x: int, y: int, n: int, steps: int, ny: int | None = None):
    """Column and row indices of the periodic window around (x, y) on an
    n x ny grid (ny = n if not given), and the window position of (x, y)."""
    half = 2 * steps + 1
    idx = np.arange(2 * half + 1) - half
    return (x + idx) % n, (y + idx) % (n if ny is None else ny), half


def pack(f, g):
    return np.concatenate([f, g[:, 0], g[:, 1]], 0)


def oracle_cell(mom, steps: int, lattice: str = "d2q5", **oracle_kw) -> np.ndarray:
    """Populations of the window's centre cell after `steps` oracle steps from
    the unfiltered equilibria of the window fields mom [5, w, w]."""
    w = mom.shape[-1]
    half = w // 2
    o = O.Oracle(w, w, mag_lattice=lattice, **oracle_kw)
    o.set_state(O.f_equilibrium(*mom), O.g_equilibrium_for(lattice, *mom))
    o.step(steps)
    return pack(*o.state()[:2])[:, half, half]


def check_rough_sampled(got, pts, n, steps, factors, tol, gaps=(), lattice="d2q5", say=print, ny=None,
                        **oracle_kw):
    """got [npop, npts]: the GPU's populations at the sampled cells pts after
    `steps` steps from the equilibria of the rough fields `factors` on an
    n x ny grid (ny = n if not given).  Each
    cell must be within `tol` (max abs) of the oracle with `oracle_kw`; for
    each (label, kw, factor) in `gaps`, the oracle with those keyword changes
    must sit at least factor * tol away at every sampled cell.  Returns the
    worst error and the smallest gap of each label."""
    worst = 0.0
    smallest = {label: np.inf for label, _, _ in gaps}
    need = {label: factor * tol for label, _, factor in gaps}
    for k, (x, y) in enumerate(pts):
        xs, ys, _ = window(x, y, n, steps, ny)
        mom = assemble_rough(factors, xs, ys)
        ref = oracle_cell(mom, steps, lattice, **oracle_kw)
        err = float(np.abs(got[:, k] - ref).max())
        worst = max(worst, err)
        assert err <= tol, (x, y, err, tol)
        for label, kw, _ in gaps:
            other = oracle_cell(mom, steps, lattice, **{**oracle_kw, **kw})
            smallest[label] = min(smallest[label], float(np.abs(other - ref).max()))
    say(f"  worst error {worst:.3e} (tol {tol:.1e}); smallest gaps "
        + ", ".join(f"{k} {v:.3e} ({v / tol:.0f} x tol)" for k, v in smallest.items()))
    for label, g in smallest.items():
        assert g >= need[label], (label, g, need[label])
    return worst, smallest
