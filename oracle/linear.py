"""Brute-force linearisation of one LB-MHD timestep in Fourier space.

TEST INFRASTRUCTURE ONLY (see the package docstring).

About a uniform equilibrium (rho0, u0, B0) a small perturbation of the
9 + 2q populations (f_0..f_8, g_x0..g_x(q-1), g_y0..g_y(q-1); q = 5 for the
D2Q5 vector distribution, 9 for D2Q9) with wave vector k evolves as
x(t + 1) = G(k) x(t), G = Phi(k) (I - C):

* C is the collision linearised by hand from the population-form equilibria
  of Sec. 2 (``feq``, ``geq``) -- not from the moment table the oracle uses --
  and the MRT relaxation T^-1 S T (``FluidTMatrix``) with T typed in from the
  printed integer matrix, plus SRT for g (``LBMagEqn``) in population space
  (for D2Q9 g this bypasses the ``MagTMatrix`` route the oracle takes).
* Phi(k) = diag(exp(-i k.c_q)) is streaming f_q(x + c_q) = f*_q(x).

The subgrid closure is quadratic in gradients and drops out of the
linearisation, so this pins the unfiltered step only.  The eigenvalues of G
give the exact discrete decay rates and frequencies of shear, sound, Alfven
and magnetic-diffusion waves; the continuum limits are the transport
coefficients of Sec. 2.
"""

from __future__ import annotations

import numpy as np

# Velocities and the moment matrix as printed in Sec. 2 (lattice vectors and
# ``FluidTMatrix``), typed in independently of the oracle's symbolic rows.
_CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
_CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
_T_PRINTED = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [4, -5, -5, -5, -5, 4, 4, 4, 4],
    [4, 0, 0, 0, 0, -1, -1, -1, -1],
], dtype=np.float64)
_W = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])
_WM = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])

NQ = 19


def _gweights(qg: int) -> np.ndarray:
    """Weights of the vector distribution: D2Q5 (1/3, 1/6 x4) or the D2Q9 ones."""
    return _WM if qg == 5 else _W


def _macro_jacobian(qg: int = 5) -> np.ndarray:
    """d(rho, m_x, m_y, B_x, B_y) / d(9 + 2 qg populations)."""
    nq = 9 + 2 * qg
    D = np.zeros((5, nq))
    D[0, :9] = 1.0
    D[1, :9] = _CX
    D[2, :9] = _CY
    D[3, 9:9 + qg] = 1.0
    D[4, 9 + qg:nq] = 1.0
    return D


def equilibrium_jacobian(rho0: float, u0, B0, qg: int = 5) -> np.ndarray:
    """d(f^eq, g^eq) / d(rho, m_x, m_y, B_x, B_y) at (rho0, rho0 u0, B0),
    differentiated by hand from ``feq`` and ``geq`` (u = m / rho)."""
    ux, uy = float(u0[0]), float(u0[1])
    bx, by = float(B0[0]), float(B0[1])
    u = (ux, uy)
    b = (bx, by)
    wm = _gweights(qg)
    J = np.zeros((9 + 2 * qg, 5))
    for i in range(9):
        c = (_CX[i], _CY[i])
        cu = c[0] * ux + c[1] * uy
        cb = c[0] * bx + c[1] * by
        c2 = c[0] ** 2 + c[1] ** 2
        usq = ux * ux + uy * uy
        # w rho [1 + 3 c.m/rho + 9/2 (c.m)^2/rho^2 - 3/2 m^2/rho^2]
        J[i, 0] = _W[i] * (1.0 - 4.5 * cu * cu + 1.5 * usq)
        for a in range(2):
            J[i, 1 + a] = _W[i] * (3.0 * c[a] + 9.0 * cu * c[a] - 3.0 * u[a])
            # 9/2 w [1/2 B^2 c^2 - (B.c)^2]
            J[i, 3 + a] = 4.5 * _W[i] * (b[a] * c2 - 2.0 * cb * c[a])
    for i in range(qg):
        c = (_CX[i], _CY[i])
        cu = c[0] * ux + c[1] * uy
        cb = c[0] * bx + c[1] * by
        for a in range(2):
            row = 9 + qg * a + i
            # w' [B_a + 3 ((c.m) B_a - (c.B) m_a) / rho]
            J[row, 0] = -3.0 * wm[i] * (cu * b[a] - cb * u[a]) / rho0
            for bb in range(2):
                J[row, 1 + bb] = 3.0 * wm[i] * (c[bb] * b[a] - cb * (1.0 if a == bb else 0.0)) / rho0
                J[row, 3 + bb] = wm[i] * ((1.0 if a == bb else 0.0)
                                          + 3.0 * (cu * (1.0 if a == bb else 0.0) - c[bb] * u[a]))
    return J


def collision_matrix(rates, s_m: float, rho0: float = 1.0, u0=(0.0, 0.0), B0=(0.0, 0.0),
                     qg: int = 5) -> np.ndarray:
    """Linear map x -> x* of one collision, (9 + 2 qg) square (real)."""
    rates = np.asarray(rates, dtype=np.float64)
    nq = 9 + 2 * qg
    K = np.zeros((nq, nq))
    K[:9, :9] = np.linalg.solve(_T_PRINTED, np.diag(rates) @ _T_PRINTED)
    K[9:, 9:] = s_m * np.eye(2 * qg)
    Jeq = equilibrium_jacobian(rho0, u0, B0, qg) @ _macro_jacobian(qg)
    return np.eye(nq) - K @ (np.eye(nq) - Jeq)


def streaming_phase(k, qg: int = 5) -> np.ndarray:
    """diag(exp(-i k.c_q)) for the 9 + 2 qg populations."""
    kx, ky = float(k[0]), float(k[1])
    cx = np.concatenate([_CX, _CX[:qg], _CX[:qg]])
    cy = np.concatenate([_CY, _CY[:qg], _CY[:qg]])
    return np.diag(np.exp(-1j * (kx * cx + ky * cy)))


def step_matrix(k, rates, s_m: float, rho0: float = 1.0, u0=(0.0, 0.0), B0=(0.0, 0.0), qg: int = 5) -> np.ndarray:
    """G(k): Fourier amplitude at wave vector k after one collide-stream step."""
    return streaming_phase(k, qg) @ collision_matrix(rates, s_m, rho0, u0, B0, qg)


def rates_from(nu: float, eta: float, s5=None, s6=None, s7=None, s8=None):
    """(rates[9], s_m) from nu, eta (Sec. 2 transport formulas) and ghost rates."""
    s = 2.0 / (6.0 * nu + 1.0)
    ghost = [s if v is None else float(v) for v in (s5, s6, s7, s8)]
    return np.array([0.0, 0.0, 0.0, s, s] + ghost), 2.0 / (6.0 * eta + 1.0)


def hydrodynamic_eigenvalues(G: np.ndarray, n: int) -> np.ndarray:
    """The n eigenvalues of G with largest modulus (the slow modes)."""
    lam = np.linalg.eigvals(G)
    return lam[np.argsort(-np.abs(lam))][:n]


def bulk_viscosity(nu: float, s4: float, s7: float, s8: float) -> float:
    """xi of Sec. 2: -1/9 - 1/(9 s4) - 1/(15 s7) + 2/(5 s8)."""
    return -1.0 / 9.0 - 1.0 / (9.0 * s4) - 1.0 / (15.0 * s7) + 2.0 / (5.0 * s8)
