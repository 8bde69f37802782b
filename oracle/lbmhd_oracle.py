"""Plain FP64 NumPy oracle of the filtered LB-MHD timestep.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Paper: Flint & Vahala, arXiv 1705.09807.  Citations name the paper's section
and the LaTeX label of the equation (``feq``, ``FluidTMatrix``, ...).

State and conventions
---------------------
* Periodic grid of ``nx`` x ``ny`` nodes at x = i, y = j (lattice units,
  dx = dt = 1).  Arrays are indexed ``[..., y, x]``.
* ``f[9, ny, nx]``: D2Q9 scalar distribution (filtered density, momentum).
* ``g[5, 2, ny, nx]``: vector distribution on the D2Q5 subset of the same
  velocities, ``g[i, alpha]`` = component alpha of g_i (filtered B);
  ``g[9, 2, ny, nx]`` with ``mag_lattice="d2q9"`` (all nine velocities,
  collision in the moment space of ``MagTMatrix``).
* The stored state at time t is post-streaming (what the next collision
  consumes).  Two arrays, no in-place tricks.

Readings of the paper used here (each is also listed in the design notes):
* The magnetic distribution uses D2Q5 with weights (1/3, 1/6 x 4), the only
  D2Q5 weights with c_s^2 = 1/3, which the resistivity formula of Sec. 2
  (eta = 1/(3 s_m) - 1/6) requires.  The paper itself writes D2Q9 for g.
* The magnetic equilibrium moments use u = rho u / rho (as in the g
  equilibrium ``geq`` and the induction term of ``FinalMagnetic``), not the
  momentum written in the ``MagMomentEq`` table.
* The subgrid terms follow ``FilterExampleSmall`` applied to every nonlinear
  equilibrium moment with filtered-density gradients dropped, as Sec. 3 does
  for M3; the closure strength is Delta^2/12 times ``closure_scale`` (1 =
  as printed in Sec. 3).
* ``density_gradients=True`` keeps the filtered-density terms of
  ``FilterExampleLarge`` (Z = rho) in the Reynolds and induction products.
* Gradients are synchronous (taken from the current post-streaming moments)
  with a 3x3 isotropic stencil by default; diagnostics use central
  differences.
"""

from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Lattice constants (Sec. 2)
# ---------------------------------------------------------------------------

#: D2Q9 velocities, Sec. 2 (the lattice-vector equation after ``MagTMatrix``).
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.int64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.int64)

#: D2Q9 weights.  Sec. 2 only says "appropriate lattice weights"; these are the
#: weights for which T f^eq reproduces the ``KinMomentEq`` table (pinned by test).
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)

#: D2Q5 weights for the vector distribution (first five D2Q9 velocities).
W5 = np.array([1 / 3] + [1 / 6] * 4)


def moment_matrix() -> np.ndarray:
    """The 9x9 moment transform T built from its symbolic rows, Sec. 2
    ``FluidTMatrix``: 1, c_x, c_y, c_x c_y, c_x^2 - c_y^2, 3 c_x c_y^2 - 2 c_x,
    3 c_y c_x^2 - 2 c_y, 4 - 9 (c_x^2 + c_y^2 - 2 c_x^2 c_y^2),
    4 - 4 (c_x^2 + c_y^2) + 3 c_x^2 c_y^2."""
    cx = CX.astype(np.float64)
    cy = CY.astype(np.float64)
    one = np.ones(9)
    rows = [
        one,
        cx,
        cy,
        cx * cy,
        cx ** 2 - cy ** 2,
        3 * cx * cy ** 2 - 2 * cx,
        3 * cy * cx ** 2 - 2 * cy,
        4 * one - 9 * (cx ** 2 + cy ** 2 - 2 * cx ** 2 * cy ** 2),
        4 * one - 4 * (cx ** 2 + cy ** 2) + 3 * cx ** 2 * cy ** 2,
    ]
    return np.array(rows)


T = moment_matrix()
T_INV = np.linalg.inv(T)


def magnetic_moment_matrix() -> np.ndarray:
    """The 9x9 transform T_m of the D2Q9 vector distribution built from its
    symbolic rows, Sec. 2 ``MagTMatrix``: 1, c_x, c_y, c_x c_y, c_x^2, c_y^2,
    c_x^2 c_y, c_x c_y^2, c_x^2 c_y^2."""
    cx = CX.astype(np.float64)
    cy = CY.astype(np.float64)
    rows = [np.ones(9), cx, cy, cx * cy, cx ** 2, cy ** 2, cx ** 2 * cy, cx * cy ** 2, cx ** 2 * cy ** 2]
    return np.array(rows)


T_M = magnetic_moment_matrix()
T_M_INV = np.linalg.inv(T_M)

#: Magnetic lattices: number of velocities of g (the first n of the D2Q9 set).
MAG_LATTICES = {"d2q5": 5, "d2q9": 9}


def relaxation_rates(nu: float, s5=None, s6=None, s7=None, s8=None) -> np.ndarray:
    """Diagonal of the MRT rate matrix in moment space.

    s3 = s4 from nu = 1/(3 s) - 1/6 (Sec. 2, viscosity formula).  The
    conserved moments M0..M2 get rate 0.  Ghost rates s5..s8 default to s3,
    i.e. the single-relaxation-time collision the runs of Sec. 3 use."""
    s = 2.0 / (6.0 * nu + 1.0)
    ghost = [s if v is None or v <= 0 else float(v) for v in (s5, s6, s7, s8)]
    return np.array([0.0, 0.0, 0.0, s, s] + ghost)


def magnetic_rate(eta: float) -> float:
    """s_m from eta = 1/(3 s_m) - 1/6 (Sec. 2, resistivity formula)."""
    return 2.0 / (6.0 * eta + 1.0)


# ---------------------------------------------------------------------------
# Equilibria
# ---------------------------------------------------------------------------


def f_equilibrium(rho, mx, my, Bx, By) -> np.ndarray:
    """f_i^(eq) of Sec. 2 ``feq``, population form, with u = rho u / rho."""
    ux = mx / rho
    uy = my / rho
    usq = ux * ux + uy * uy
    bsq = Bx * Bx + By * By
    out = np.empty((9,) + np.shape(rho))
    for i in range(9):
        cu = CX[i] * ux + CY[i] * uy
        cb = CX[i] * Bx + CY[i] * By
        c2 = CX[i] ** 2 + CY[i] ** 2
        out[i] = W9[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq) \
            + 4.5 * W9[i] * (0.5 * bsq * c2 - cb * cb)
    return out


def g_equilibrium(rho, mx, my, Bx, By) -> np.ndarray:
    """Vector g_i^(eq) of Sec. 2 ``geq`` on D2Q5, with u = rho u / rho:
    g_i = w'_i [B + 3 ((c_i.u) B - (c_i.B) u)]."""
    ux = mx / rho
    uy = my / rho
    out = np.empty((5, 2) + np.shape(rho))
    for i in range(5):
        cu = CX[i] * ux + CY[i] * uy
        cb = CX[i] * Bx + CY[i] * By
        out[i, 0] = W5[i] * (Bx + 3.0 * (cu * Bx - cb * ux))
        out[i, 1] = W5[i] * (By + 3.0 * (cu * By - cb * uy))
    return out


def magnetic_equilibrium_moments(Bx, By, lam) -> np.ndarray:
    """N^(eq)_{alpha i}, i = 0..8, of the D2Q9 vector distribution, Sec. 2
    ``MagMomentEq`` with u in place of rho u (the R2 reading): N0 = B_a,
    N1 = Lam[x, a], N2 = Lam[y, a], N3 = 0, N4 = N5 = B_a / 3,
    N6 = Lam[y, a] / 3, N7 = Lam[x, a] / 3, N8 = B_a / 9, where
    Lam[b, a] = u_b B_a - B_b u_a (or its filtered value).  The table marks
    N4, N5 with (0) instead of (eq); they are read as equilibria like the
    rest.  Returns [9, 2, ...]."""
    B = (Bx, By)
    out = np.empty((9, 2) + np.shape(Bx))
    for a in range(2):
        out[0, a] = B[a]
        out[1, a] = lam[0, a]
        out[2, a] = lam[1, a]
        out[3, a] = 0.0 * B[a]
        out[4, a] = B[a] / 3.0
        out[5, a] = B[a] / 3.0
        out[6, a] = lam[1, a] / 3.0
        out[7, a] = lam[0, a] / 3.0
        out[8, a] = B[a] / 9.0
    return out


def unfiltered_induction(rho, mx, my, Bx, By) -> np.ndarray:
    """Lam[b, a] = u_b B_a - B_b u_a with u = rho u / rho."""
    u = (mx / rho, my / rho)
    B = (Bx, By)
    lam = np.empty((2, 2) + np.shape(rho))
    for b in range(2):
        for a in range(2):
            lam[b, a] = u[b] * B[a] - B[b] * u[a]
    return lam


def g_equilibrium_d2q9(rho, mx, my, Bx, By) -> np.ndarray:
    """Vector g^(eq) on D2Q9 (the lattice Sec. 2 uses for g): the moments of
    ``MagMomentEq`` mapped back to populations, T_m^-1 N^(eq).  [9, 2, ...]."""
    neq = magnetic_equilibrium_moments(Bx, By, unfiltered_induction(rho, mx, my, Bx, By))
    return np.tensordot(T_M_INV, neq, axes=(1, 0))


def g_equilibrium_for(lattice: str, rho, mx, my, Bx, By) -> np.ndarray:
    """g^(eq) on the named magnetic lattice ('d2q5' or 'd2q9')."""
    return g_equilibrium(rho, mx, my, Bx, By) if lattice == "d2q5" else g_equilibrium_d2q9(rho, mx, my, Bx, By)


# ---------------------------------------------------------------------------
# Periodic finite differences
# ---------------------------------------------------------------------------


def shifted(a, dx: int, dy: int):
    """a(x + dx, y + dy) on the periodic grid."""
    return np.roll(a, (-dy, -dx), axis=(-2, -1))


def grad_iso9(a):
    """3x3 isotropic gradient: D_x a = (a_E - a_W)/3 + (a_NE + a_SE - a_NW - a_SW)/12,
    D_y likewise.  This is 3 sum_i w_i c_i a(x + c_i) with the D2Q9 weights; the
    paper leaves the stencil open (Sec. 3, remark on derivatives)."""
    e, w = shifted(a, 1, 0), shifted(a, -1, 0)
    n, s = shifted(a, 0, 1), shifted(a, 0, -1)
    ne, nw = shifted(a, 1, 1), shifted(a, -1, 1)
    se, sw = shifted(a, 1, -1), shifted(a, -1, -1)
    dx = (e - w) / 3.0 + (ne + se - nw - sw) / 12.0
    dy = (n - s) / 3.0 + (ne + nw - se - sw) / 12.0
    return dx, dy


def grad_central(a):
    """Central differences (a_E - a_W)/2, (a_N - a_S)/2."""
    dx = (shifted(a, 1, 0) - shifted(a, -1, 0)) / 2.0
    dy = (shifted(a, 0, 1) - shifted(a, 0, -1)) / 2.0
    return dx, dy


GRADIENTS = {"iso9": grad_iso9, "central5": grad_central}


# ---------------------------------------------------------------------------
# Filtered equilibria with the subgrid closure (Sec. 2.1 and Sec. 3)
# ---------------------------------------------------------------------------


def closure_terms_from_gradients(rho, gm, gb, k2: float):
    """The P, Q, R dictionaries of ``closure_terms`` from given gradients
    gm[a][b] = D_b m_a and gb[a][b] = D_b B_a."""
    P, Q, R = {}, {}, {}
    for a in range(2):
        for c in range(2):
            P[a, c] = k2 / rho * (gm[a][0] * gm[c][0] + gm[a][1] * gm[c][1])
            Q[a, c] = k2 * (gb[a][0] * gb[c][0] + gb[a][1] * gb[c][1])
            R[a, c] = k2 / rho * (gm[a][0] * gb[c][0] + gm[a][1] * gb[c][1])
    return P, Q, R


def local_gradients(f, g, rates, s_m: float, stencil: str = "iso9"):
    """Closure gradients from local non-equilibrium moments, with a stencil
    only for the vorticity (Sec. 3 notes that D2Q9 cannot give every
    derivative locally).  First-order Chapman-Enskog for the pre-collision
    populations, f^neq = -(1/s) (d_t + c.grad) f^eq:
      * M3 - M3^eq = -(2 rho / (3 s3)) S_xy and M4 - M4^eq = -(2 rho / (3 s4))
        (S_xx - S_yy), S the strain rate of u, with the unfiltered equilibria
        of ``KinMomentEq``; incompressibility closes S_xx = -S_yy;
      * Lam_ba - Lam^eq_ba = -(1 / (3 s_m)) D_b B_a (the O(Ma^2) time derivative
        of Lam^eq dropped), Lam_ba = sum_i c_ib g_ia, Lam^eq_ba = u_b B_a - B_b u_a;
      * the vorticity w_m = D_x m_y - D_y m_x from the stencil;
    and D m = rho D u (density gradients dropped, as in Sec. 3).  Returns
    (gm, gb) with gm[a][b] = D_b m_a, gb[a][b] = D_b B_a."""
    rho = f.sum(axis=0)
    mx = np.tensordot(CX.astype(np.float64), f, axes=(0, 0))
    my = np.tensordot(CY.astype(np.float64), f, axes=(0, 0))
    Bx = g[:, 0].sum(axis=0)
    By = g[:, 1].sum(axis=0)
    M = np.tensordot(T, f, axes=(1, 0))
    m3eq = mx * my / rho - Bx * By
    m4eq = (mx * mx - my * my) / rho - Bx * Bx + By * By
    sxy = -1.5 * rates[3] / rho * (M[3] - m3eq)
    sd = -1.5 * rates[4] / rho * (M[4] - m4eq)
    sxx, syy = 0.5 * sd, -0.5 * sd
    grad = GRADIENTS[stencil]
    dmx, dmy = grad(mx), grad(my)
    wm = dmy[0] - dmx[1]
    gm = [(rho * sxx, rho * sxy - 0.5 * wm), (rho * sxy + 0.5 * wm, rho * syy)]
    c = (CX[:5].astype(np.float64), CY[:5].astype(np.float64))
    lam = [[np.tensordot(c[b], g[:, a], axes=(0, 0)) for a in range(2)] for b in range(2)]   # lam[b][a]
    ux, uy = mx / rho, my / rho
    lam_eq = [[np.zeros_like(rho), ux * By - Bx * uy], [uy * Bx - By * ux, np.zeros_like(rho)]]
    gb = [[-3.0 * s_m * (lam[b][a] - lam_eq[b][a]) for b in range(2)] for a in range(2)]
    return gm, gb


def closure_terms(rho, mx, my, Bx, By, k2: float, stencil: str = "iso9"):
    """Delta^2 corrections of the nonlinear equilibrium products.

    ``FilterExampleSmall`` gives  bar(XY) = bar X bar Y + Delta^2/12 (d_b bar X)(d_b bar Y).
    Applied with density gradients dropped (Sec. 3) to

    * the Reynolds product  m_a m_c / rho  ->  + k2/rho (d_b m_a)(d_b m_c),
    * the Maxwell product   B_a B_c        ->  + k2 (d_b B_a)(d_b B_c),
    * the induction product m_a B_c / rho  ->  + k2/rho (d_b m_a)(d_b B_c),

    with k2 = closure_scale * Delta^2 / 12.  Returns the dictionaries
    ``P[a,c]`` = k2/rho (d_b m_a)(d_b m_c), ``Q[a,c]`` = k2 (d_b B_a)(d_b B_c) and
    ``R[a,c]`` = k2/rho (d_b m_a)(d_b B_c) for a, c in {0 (x), 1 (y)}."""
    grad = GRADIENTS[stencil]
    gm = [grad(mx), grad(my)]       # gm[a][b] = D_b m_a
    gb = [grad(Bx), grad(By)]       # gb[a][b] = D_b B_a
    return closure_terms_from_gradients(rho, gm, gb, k2)


def closure_terms_full_from_gradients(rho, m, B, gm, gb, grho, k2: float):
    """``FilterExampleLarge`` with Z = rho, density gradients kept:

        bar(XY/Z) - bar X bar Y / bar Z
          = Delta^2/(12 Z) [ (d_b X)(d_b Y)
                             - (d_b Z / Z) (X d_b Y + Y d_b X - X Y d_b Z / Z) ],

    applied to the Reynolds product m_a m_c / rho (P) and the induction
    product m_a B_c / rho (R); the Maxwell product B_a B_c has no divisor and
    keeps ``FilterExampleSmall`` (Q).  m = (m_x, m_y), B = (B_x, B_y),
    gm[a][b] = D_b m_a, gb[a][b] = D_b B_a, grho[b] = D_b rho; k2 = closure
    strength times Delta^2/12.  Same dictionaries as ``closure_terms``."""
    P, Q, R = {}, {}, {}
    for a in range(2):
        for c in range(2):
            pp = np.zeros_like(rho)
            rr = np.zeros_like(rho)
            qq = np.zeros_like(rho)
            for b in range(2):
                lr = grho[b] / rho
                pp = pp + gm[a][b] * gm[c][b] - lr * (m[a] * gm[c][b] + m[c] * gm[a][b] - m[a] * m[c] * lr)
                rr = rr + gm[a][b] * gb[c][b] - lr * (m[a] * gb[c][b] + B[c] * gm[a][b] - m[a] * B[c] * lr)
                qq = qq + gb[a][b] * gb[c][b]
            P[a, c] = k2 / rho * pp
            Q[a, c] = k2 * qq
            R[a, c] = k2 / rho * rr
    return P, Q, R


def closure_terms_full(rho, mx, my, Bx, By, k2: float, stencil: str = "iso9"):
    """``closure_terms_full_from_gradients`` with every gradient (of m, B and
    rho) from the named 3x3 stencil."""
    grad = GRADIENTS[stencil]
    return closure_terms_full_from_gradients(rho, (mx, my), (Bx, By), [grad(mx), grad(my)], [grad(Bx), grad(By)],
                                             grad(rho), k2)


def filtered_equilibrium_moments(rho, mx, my, Bx, By, P, Q) -> np.ndarray:
    """Filtered M_i^(eq), i = 0..8: the ``KinMomentEq`` table evaluated on the
    filtered invariants (Sec. 2.1, filtered equilibrium moments) plus the
    Delta^2 term of every nonlinear entry ("similarly for the other filtered
    equilibrium moments", with the density-gradient terms dropped as in the
    simplified M3 of Sec. 3).  M5, M6 are linear and get no correction."""
    meq = np.empty((9,) + np.shape(rho))
    meq[0] = rho
    meq[1] = mx
    meq[2] = my
    # M3: rho u_x rho u_y / rho - B_x B_y  (Sec. 3, simplified M3)
    meq[3] = mx * my / rho - Bx * By + P[0, 1] - Q[0, 1]
    # M4: ((rho u_x)^2 - (rho u_y)^2)/rho - B_x^2 + B_y^2
    meq[4] = (mx * mx - my * my) / rho - Bx * Bx + By * By \
        + P[0, 0] - P[1, 1] - Q[0, 0] + Q[1, 1]
    meq[5] = -mx
    meq[6] = -my
    # M7: -3 ((rho u_x)^2 + (rho u_y)^2)/rho
    meq[7] = -3.0 * (mx * mx + my * my) / rho - 3.0 * (P[0, 0] + P[1, 1])
    # M8: 5 rho/3 - 3 ((rho u_x)^2 + (rho u_y)^2)/rho
    meq[8] = 5.0 * rho / 3.0 - 3.0 * (mx * mx + my * my) / rho - 3.0 * (P[0, 0] + P[1, 1])
    return meq


def filtered_induction(rho, mx, my, Bx, By, R) -> np.ndarray:
    """Filtered first moments of g^(eq):  Lam[b, a] = sum_i c_ib g_ia^(eq)
    = bar(u_b B_a - B_b u_a)  (``MagMomentEq`` N_a1, N_a2 with u in place of
    rho u), each product filtered by ``FilterExampleSmall`` with density
    gradients dropped: + R[b, a] - R[a, b]."""
    m = (mx, my)
    B = (Bx, By)
    lam = np.empty((2, 2) + np.shape(rho))
    for b in range(2):
        for a in range(2):
            lam[b, a] = (m[b] * B[a] - B[b] * m[a]) / rho + R[b, a] - R[a, b]
    return lam


def g_equilibrium_from_moments(Bx, By, lam) -> np.ndarray:
    """Vector g^(eq) rebuilt from its zeroth moment B and first moments Lam on
    D2Q5: g_ia = w'_i (B_a + 3 sum_b c_ib Lam[b, a])  (reproduces ``geq`` when
    Lam is unfiltered, since sum_i w'_i c_ib c_ic = delta_bc / 3)."""
    B = (Bx, By)
    out = np.empty((5, 2) + np.shape(Bx))
    for i in range(5):
        for a in range(2):
            out[i, a] = W5[i] * (B[a] + 3.0 * (CX[i] * lam[0, a] + CY[i] * lam[1, a]))
    return out


# ---------------------------------------------------------------------------
# SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), counter form
# ---------------------------------------------------------------------------

_GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """Output number ``counter + 1`` of the SplitMix64 sequence started at
    state ``seed``: z = seed + (counter + 1) * gamma, then the 64-bit finaliser
    with shifts 30, 27, 31 and the two published multipliers."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counter.astype(np.uint64) + np.uint64(1)) * _GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, counter: np.ndarray) -> np.ndarray:
    """Uniform on [-1, 1): 2 * (top 53 bits * 2^-53) - 1."""
    z = splitmix64(seed, counter)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


# ---------------------------------------------------------------------------
# Kelvin-Helmholtz initial state
# ---------------------------------------------------------------------------


def kh_jet_populations(x, y, nx, ny, U0=0.05, delta_over_L=0.05, B0=0.01, rho0=1.0,
                       pert_amp_over_U0=1e-3, noise_amp=1e-5, seed=0, lattice="d2q5"):
    """Initial populations at integer nodes (x, y) (arrays of equal shape) of
    an nx x ny grid.  Double shear layer u_x = U0 [tanh((y - L/4)/d) -
    tanh((y - 3L/4)/d) - 1] with L = ny, d = delta_over_L * ny;
    u_y = pert * U0 sin(2 pi x / nx) + noise_amp * xi, xi uniform on [-1, 1)
    from SplitMix64 on the cell index y * nx + x; B = (B0, 0); rho = rho0.
    Populations are the unfiltered equilibria ``feq`` and ``geq`` (Sec. 2).
    Returns (f[9, ...], g[q, 2, ...]) with q = 5 or 9 for the magnetic
    lattice."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    L = float(ny)
    d = delta_over_L * L
    yf = y.astype(np.float64)
    ux = U0 * (np.tanh((yf - L / 4.0) / d) - np.tanh((yf - 3.0 * L / 4.0) / d) - 1.0)
    uy = pert_amp_over_U0 * U0 * np.sin(2.0 * math.pi * x.astype(np.float64) / nx) \
        + noise_amp * uniform_pm1(seed, y * nx + x)
    rho = np.full(x.shape, float(rho0))
    bx = np.full(x.shape, float(B0))
    by = np.zeros(x.shape)
    return (f_equilibrium(rho, rho * ux, rho * uy, bx, by),
            g_equilibrium_for(lattice, rho, rho * ux, rho * uy, bx, by))


def sech2_jet_populations(x, y, nx, ny, U0=4.88e-2, B0=0.005 * 4.88e-2, pert=0.01, k=4, rho0=1.0,
                          lattice="d2q5"):
    """The magnetized Kelvin-Helmholtz jet of Sec. 4 at integer nodes (x, y):
    u_y = U0 sech^2(2 pi k d / nx) + pert U0 sin(2 pi k x / nx),
    u_x = pert U0 sin(2 pi k y / ny),
    B_x = pert B0 sin(2 pi k y / ny),  B_y = B0 + pert B0 sin(2 pi k x / nx),
    rho = rho0, with d the periodic distance of x from 0 (the printed profile
    sech^2(8 pi x / L) centred on x = 0 of the periodic box) and the mean field
    along the jet.  The paper: k = 4, pert = 0.01, U0 = 4.88e-2, B0 = 0.005 U0,
    nu = eta = 1e-3 at 1024^2.  Populations are the unfiltered equilibria."""
    xf = np.asarray(x, dtype=np.float64)
    yf = np.asarray(y, dtype=np.float64)
    d = np.minimum(xf, nx - xf)
    uy = U0 / np.cosh(2.0 * math.pi * k * d / nx) ** 2 + pert * U0 * np.sin(2.0 * math.pi * k * xf / nx)
    ux = pert * U0 * np.sin(2.0 * math.pi * k * yf / ny)
    bx = pert * B0 * np.sin(2.0 * math.pi * k * yf / ny)
    by = B0 + pert * B0 * np.sin(2.0 * math.pi * k * xf / nx)
    rho = np.full(xf.shape, float(rho0))
    return (f_equilibrium(rho, rho * ux, rho * uy, bx, by),
            g_equilibrium_for(lattice, rho, rho * ux, rho * uy, bx, by))


# ---------------------------------------------------------------------------
# The oracle
# ---------------------------------------------------------------------------


class Oracle:
    """Filtered LB-MHD on an nx x ny periodic grid, FP64, two-array state.

    Parameters mirror the C ABI: nu, eta (transport coefficients), optional
    MRT ghost rates s5..s8 (<= 0 or None: equal to s3), delta (filter width;
    0 = DNS), closure_scale (multiplies Delta^2/12), grad_stencil ('iso9' or
    'central5')."""

    def __init__(self, nx: int, ny: int, nu: float, eta: float, delta: float = 0.0,
                 closure_scale: float = 1.0, s5=None, s6=None, s7=None, s8=None,
                 grad_stencil: str = "iso9", closure_correction=None, closure_time: str = "sync",
                 density_gradients: bool = False, mag_lattice: str = "d2q5", correction_every: int = 1):
        if nx < 4 or ny < 4:
            raise ValueError("grid must be at least 4 x 4")
        self.nx, self.ny = int(nx), int(ny)
        self.nu, self.eta = float(nu), float(eta)
        self.delta = float(delta)
        self.closure_scale = float(closure_scale)
        self.k2 = self.closure_scale * self.delta ** 2 / 12.0
        self.rates = relaxation_rates(nu, s5, s6, s7, s8)
        self.s_m = magnetic_rate(eta)
        if not all(0.0 < r < 2.0 for r in list(self.rates[3:]) + [self.s_m]):
            raise ValueError("relaxation rates must lie in (0, 2)")
        self.grad_stencil = grad_stencil
        # optional learned correction: (rho, m_x, m_y, B_x, B_y) -> [4, ny, nx] of
        # (tau_xx, tau_xy, tau_yy, eps) added to the analytic closure terms
        self.closure_correction = closure_correction
        # the correction is evaluated from the state being collided at every
        # step t with t % correction_every == 0 and at the first step after an
        # initial or injected state, and held in between
        if int(correction_every) < 1:
            raise ValueError("correction_every must be >= 1")
        self.correction_every = int(correction_every)
        self._corr = None
        # "sync": gradients of the moments of the state being collided (Sec. 2.1,
        # Sec. 3).  "lagged": gradients of the previous step's moments (the
        # single-sweep variant of the in-place schedule); the first step after
        # an initial or injected state uses that state's own moments.  The 1/rho
        # of the closure is always the current density.
        if closure_time not in ("sync", "lagged"):
            raise ValueError("closure_time must be 'sync' or 'lagged'")
        # grad_stencil "local_iso9" / "local_central5": strain and grad B from
        # local non-equilibrium moments, vorticity from the named stencil
        self.local = grad_stencil.startswith("local_")
        self.stencil = grad_stencil[6:] if self.local else grad_stencil
        if self.stencil not in GRADIENTS:
            raise ValueError("unknown gradient stencil")
        if self.local and closure_time != "sync":
            raise ValueError("local gradients are taken from the current populations (closure_time='sync')")
        self.closure_time = closure_time
        # density_gradients: the full ``FilterExampleLarge`` closure (filtered
        # density gradients kept), synchronous stencil gradients only
        self.density_gradients = bool(density_gradients)
        if self.density_gradients and (self.local or closure_time != "sync"):
            raise ValueError("the density-gradient closure takes synchronous stencil gradients")
        # mag_lattice "d2q9": the vector distribution on all nine velocities with
        # the collision in the moment space of ``MagTMatrix`` (Sec. 2's own
        # lattice for g); "d2q5" is the five-velocity subset (R1)
        if mag_lattice not in MAG_LATTICES:
            raise ValueError("mag_lattice must be 'd2q5' or 'd2q9'")
        if mag_lattice == "d2q9" and self.local:
            raise ValueError("local gradients are defined for the D2Q5 vector distribution")
        self.mag_lattice = mag_lattice
        self.qg = MAG_LATTICES[mag_lattice]
        self._prev = None
        self.f = np.zeros((9, self.ny, self.nx))
        self.g = np.zeros((self.qg, 2, self.ny, self.nx))
        self.t = 0

    # -- initial and injected states ------------------------------------
    def init_kh_jet(self, U0=0.05, delta_over_L=0.05, B0=0.01, rho0=1.0,
                    pert_amp_over_U0=1e-3, noise_amp=1e-5, seed=0):
        """Kelvin-Helmholtz double shear layer on the whole grid at t = 0
        (see ``kh_jet_populations``)."""
        x = np.arange(self.nx, dtype=np.int64)[None, :] * np.ones((self.ny, 1), dtype=np.int64)
        y = np.arange(self.ny, dtype=np.int64)[:, None] * np.ones((1, self.nx), dtype=np.int64)
        self.f, self.g = kh_jet_populations(x, y, self.nx, self.ny, U0, delta_over_L, B0, rho0,
                                            pert_amp_over_U0, noise_amp, seed, self.mag_lattice)
        self.t = 0
        self._prev = None
        self._corr = None

    def init_sech2_jet(self, U0=4.88e-2, B0=0.005 * 4.88e-2, pert=0.01, k=4, rho0=1.0):
        """The magnetized jet of Sec. 4 on the whole grid at t = 0 (see
        ``sech2_jet_populations``)."""
        x = np.arange(self.nx, dtype=np.int64)[None, :] * np.ones((self.ny, 1), dtype=np.int64)
        y = np.arange(self.ny, dtype=np.int64)[:, None] * np.ones((1, self.nx), dtype=np.int64)
        self.f, self.g = sech2_jet_populations(x, y, self.nx, self.ny, U0, B0, pert, k, rho0, self.mag_lattice)
        self.t = 0
        self._prev = None
        self._corr = None

    def set_state(self, f, g, t: int = 0):
        self.f = np.array(f, dtype=np.float64).reshape(9, self.ny, self.nx)
        self.g = np.array(g, dtype=np.float64).reshape(self.qg, 2, self.ny, self.nx)
        self.t = int(t)
        self._prev = None
        self._corr = None

    def state(self):
        """(f, g, t): copies of the post-streaming populations at time t."""
        return self.f.copy(), self.g.copy(), self.t

    # -- the method ------------------------------------------------------
    @staticmethod
    def _moments(f, g):
        """rho = sum f_i, rho u = sum c_i f_i, B = sum g_i (Sec. 2, after ``LBMagEqn``)."""
        rho = f.sum(axis=0)
        mx = np.tensordot(CX.astype(np.float64), f, axes=(0, 0))
        my = np.tensordot(CY.astype(np.float64), f, axes=(0, 0))
        Bx = g[:, 0].sum(axis=0)
        By = g[:, 1].sum(axis=0)
        return rho, mx, my, Bx, By

    def moments(self):
        """(rho, m_x, m_y, B_x, B_y) at the current time, each [ny, nx]."""
        return self._moments(self.f, self.g)

    def collide(self, f, g, grad_fields=None):
        """One collision (Sec. 2 ``LBKinEqn``/``LBMagEqn``, Sec. 3): moments,
        synchronous gradients, filtered equilibria, MRT relaxation of f in
        moment space (``Transformation``), SRT relaxation of g.  Returns the
        post-collision (f*, g*).

        The f collision is the right-hand side of ``LBKinEqn`` with the rate
        tensor s' = T^-1 S T:  f* = f + s' (f^eq - f) = f - T^-1 S (M - M^eq),
        M = T f.  Relaxation acts on the moments; conserved moments (rate 0)
        contribute nothing.  `grad_fields` (m_x, m_y, B_x, B_y), when given,
        are the fields the closure differentiates instead of the current ones."""
        rho, mx, my, Bx, By = self._moments(f, g)
        if self.local:
            gm_loc, gb_loc = local_gradients(f, g, self.rates, self.s_m, self.stencil)
            P, Q, R = closure_terms_from_gradients(rho, gm_loc, gb_loc, self.k2)
        elif self.density_gradients:
            P, Q, R = closure_terms_full(rho, mx, my, Bx, By, self.k2, self.stencil)
        else:
            gm = (mx, my, Bx, By) if grad_fields is None else grad_fields
            P, Q, R = closure_terms(rho, gm[0], gm[1], gm[2], gm[3], self.k2, self.stencil)
        meq = filtered_equilibrium_moments(rho, mx, my, Bx, By, P, Q)
        lam = filtered_induction(rho, mx, my, Bx, By, R)
        if self.closure_correction is not None:
            # tau_xy enters M3, tau_xx - tau_yy M4, -3 (tau_xx + tau_yy) M7 and M8,
            # eps the induction moment Lam[x, y] = -Lam[y, x]
            if self._corr is None or self.t % self.correction_every == 0:
                self._corr = self.closure_correction(rho, mx, my, Bx, By)
            c = self._corr
            meq[3] = meq[3] + c[1]
            meq[4] = meq[4] + c[0] - c[2]
            meq[7] = meq[7] - 3.0 * (c[0] + c[2])
            meq[8] = meq[8] - 3.0 * (c[0] + c[2])
            lam[0, 1] = lam[0, 1] + c[3]
            lam[1, 0] = lam[1, 0] - c[3]
        M = np.tensordot(T, f, axes=(1, 0))
        fstar = f - np.tensordot(T_INV, self.rates[:, None, None] * (M - meq), axes=(1, 0))
        if self.qg == 9:
            # D2Q9 g: relax N = T_m g towards the filtered ``MagMomentEq`` table,
            # one rate s_m for every moment (SRT), and map back
            N = np.tensordot(T_M, g, axes=(1, 0))
            neq = magnetic_equilibrium_moments(Bx, By, lam)
            gstar = np.tensordot(T_M_INV, N - self.s_m * (N - neq), axes=(1, 0))
        else:
            geq = g_equilibrium_from_moments(Bx, By, lam)
            gstar = g - self.s_m * (g - geq)
        return fstar, gstar

    @staticmethod
    def stream(fstar, gstar):
        """Streaming in population space: f_i(x + c_i, t + 1) = f*_i(x, t)."""
        f = np.empty_like(fstar)
        g = np.empty_like(gstar)
        for i in range(9):
            f[i] = np.roll(fstar[i], (CY[i], CX[i]), axis=(0, 1))
        for i in range(gstar.shape[0]):
            g[i] = np.roll(gstar[i], (CY[i], CX[i]), axis=(-2, -1))
        return f, g

    def step(self, n: int = 1):
        for _ in range(int(n)):
            if self.closure_time == "lagged":
                cur = self._moments(self.f, self.g)[1:]
                src = cur if self._prev is None else self._prev
                fstar, gstar = self.collide(self.f, self.g, grad_fields=src)
                self._prev = cur
            else:
                fstar, gstar = self.collide(self.f, self.g)
            self.f, self.g = self.stream(fstar, gstar)
            self.t += 1

    # -- diagnostics -------------------------------------------------------
    def diagnostics(self) -> dict:
        """Scalar diagnostics of the current state, FP64 with exact summation
        (math.fsum).  Domain means: kinetic energy 1/2 |m|^2/rho, magnetic
        energy 1/2 |B|^2, enstrophy 1/2 w^2 (w = D_x u_y - D_y u_x), current
        J_z^2 (J_z = D_x B_y - D_y B_x); divergence D_x B_x + D_y B_y as max and
        rms; raw sums of rho, m, B; count of non-finite cells.  D = central
        differences."""
        rho, mx, my, Bx, By = self.moments()
        n = float(self.nx * self.ny)
        ux, uy = mx / rho, my / rho
        dux, duy = grad_central(ux), grad_central(uy)
        dbx, dby = grad_central(Bx), grad_central(By)
        omega = duy[0] - dux[1]
        jz = dby[0] - dbx[1]
        divb = dbx[0] + dby[1]
        finite = np.isfinite(self.f).all(axis=0) & np.isfinite(self.g).all(axis=(0, 1))

        def fs(a):
            return math.fsum(np.ravel(a).tolist())

        return {
            "t": self.t,
            "mass": fs(rho),
            "mom_x": fs(mx),
            "mom_y": fs(my),
            "bsum_x": fs(Bx),
            "bsum_y": fs(By),
            "e_kin": fs(0.5 * (mx * mx + my * my) / rho) / n,
            "e_mag": fs(0.5 * (Bx * Bx + By * By)) / n,
            "enstrophy": fs(0.5 * omega * omega) / n,
            "j2": fs(jz * jz) / n,
            "divb_max": float(np.max(np.abs(divb))),
            "divb_rms": math.sqrt(fs(divb * divb) / n),
            "nonfinite": int(np.count_nonzero(~finite)),
        }
