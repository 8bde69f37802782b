"""Oracle for the learned subgrid closure: filtered DNS, closure samples, MLP.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Filtered DNS.  The filter is the convolution of Sec. 1 (``VelFilter``) with a
Gaussian kernel of variance Delta^2/12 -- the second moment that the
Delta-expansion ``FilterExampleSmall`` (Sec. 2.1) assumes -- applied on the
periodic fine grid and sampled every `factor` cells.  Discrete weights:
w(r) = exp(-r^2 / (2 sigma^2)) for |r| <= R = ceil(5 sigma), normalised to sum
1, applied separably in x and y.

Closure samples.  On the coarse grid the exact subgrid terms are the filtered
nonlinear products minus the products of the filtered fields:
  R_ab = bar(m_a m_b / rho) - bar m_a bar m_b / bar rho,
  Q_ab = bar(B_a B_b) - bar B_a bar B_b,
  tau_xx = R_xx + (Q_yy - Q_xx)/2,  tau_yy = R_yy + (Q_xx - Q_yy)/2,
  tau_xy = R_xy - Q_xy,
  eps    = bar((m_x B_y - m_y B_x)/rho) - (bar m_x bar B_y - bar m_y bar B_x)/bar rho,
the same four quantities the analytic closure models (Sec. 2.1, Sec. 3).
The learned network predicts exact minus analytic.  Inputs: the 3x3 patch of
(rho, u_x, u_y, B_x, B_y, w, J_z) around a coarse cell (w, J_z by central
differences), index = field * 9 + (dy + 1) * 3 + (dx + 1), padded to 64.

MLP 63 -> 64 -> 64 -> 4, ReLU hidden activations, inputs normalised as
z = (x - shift) * scale with one shift and scale per input field (the mean
and inverse standard deviation of the field's centre feature), outputs
multiplied by out_scale (the root mean square of each target).  The GPU
rounds the normalised inputs, both hidden activations and all weights to
bfloat16 (round to nearest even) and accumulates in FP32; the reference below
does the same roundings and accumulates in FP64.  The normalisation itself is
FP32 arithmetic on both sides, because its bfloat16 rounding and the
out-of-distribution test |z| > 6 are decisions that must be taken in the same
precision.
"""

from __future__ import annotations

import math

import numpy as np

from . import lbmhd_oracle as O

N_IN, N_PAD, N_HID, N_OUT = 63, 64, 64, 4


# ---------------------------------------------------------------------------
# Gaussian filter and subsampling
# ---------------------------------------------------------------------------


def gaussian_weights(delta: float) -> np.ndarray:
    """Normalised taps w(-R..R) of a Gaussian with variance delta^2/12."""
    sigma = delta / math.sqrt(12.0)
    R = int(math.ceil(5.0 * sigma))
    r = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-r * r / (2.0 * sigma * sigma))
    return w / w.sum()


def filter_subsample(a: np.ndarray, factor: int, delta: float) -> np.ndarray:
    """bar a(X, Y) = sum_{dx, dy} w(dx) w(dy) a(factor X + dx, factor Y + dy)
    on the periodic grid; a is [ny, nx], the result [ny/factor, nx/factor]."""
    w = gaussian_weights(delta)
    R = (len(w) - 1) // 2
    ny, nx = a.shape
    xs = np.arange(0, nx, factor)
    ys = np.arange(0, ny, factor)
    tmp = np.zeros((ny, len(xs)))
    for k, d in enumerate(range(-R, R + 1)):
        tmp += w[k] * a[:, (xs + d) % nx]
    out = np.zeros((len(ys), len(xs)))
    for k, d in enumerate(range(-R, R + 1)):
        out += w[k] * tmp[(ys + d) % ny, :]
    return out


def filtered_fields(rho, mx, my, bx, by, factor: int, delta: float) -> np.ndarray:
    """The 12 filtered coarse fields: rho, m_x, m_y, B_x, B_y, then the products
    m_x m_x/rho, m_x m_y/rho, m_y m_y/rho, B_x B_x, B_x B_y, B_y B_y,
    (m_x B_y - m_y B_x)/rho."""
    fields = [rho, mx, my, bx, by,
              mx * mx / rho, mx * my / rho, my * my / rho,
              bx * bx, bx * by, by * by, (mx * by - my * bx) / rho]
    return np.stack([filter_subsample(f, factor, delta) for f in fields])


def exact_subgrid(c12: np.ndarray) -> np.ndarray:
    """[4, ny, nx]: tau_xx, tau_xy, tau_yy, eps from the filtered products."""
    rho, mx, my, bx, by = c12[:5]
    rxx = c12[5] - mx * mx / rho
    rxy = c12[6] - mx * my / rho
    ryy = c12[7] - my * my / rho
    qxx = c12[8] - bx * bx
    qxy = c12[9] - bx * by
    qyy = c12[10] - by * by
    eps = c12[11] - (mx * by - my * bx) / rho
    return np.stack([rxx + 0.5 * (qyy - qxx), rxy - qxy, ryy + 0.5 * (qxx - qyy), eps])


def analytic_subgrid(rho, mx, my, bx, by, delta: float, stencil: str = "iso9") -> np.ndarray:
    """The analytic closure (Delta^2/12 products of gradients, density
    gradients dropped) in the same four components."""
    P, Q, R = O.closure_terms(rho, mx, my, bx, by, delta * delta / 12.0, stencil)
    return np.stack([P[0, 0] + 0.5 * (Q[1, 1] - Q[0, 0]), P[0, 1] - Q[0, 1],
                     P[1, 1] + 0.5 * (Q[0, 0] - Q[1, 1]), R[0, 1] - R[1, 0]])


def closure_features(rho, mx, my, bx, by) -> np.ndarray:
    """[ny*nx, 64] inputs: 3x3 patches of (rho, u_x, u_y, B_x, B_y, w, J_z)."""
    ux, uy = mx / rho, my / rho
    dux, duy = O.grad_central(ux), O.grad_central(uy)
    dbx, dby = O.grad_central(bx), O.grad_central(by)
    omega = duy[0] - dux[1]
    jz = dby[0] - dbx[1]
    fields = [rho, ux, uy, bx, by, omega, jz]
    ny, nx = rho.shape
    X = np.zeros((ny * nx, N_PAD))
    for f, a in enumerate(fields):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                X[:, f * 9 + (dy + 1) * 3 + (dx + 1)] = O.shifted(a, dx, dy).ravel()
    return X


# ---------------------------------------------------------------------------
# MLP with bfloat16 roundings
# ---------------------------------------------------------------------------


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) through float32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int) -> dict:
    """Glorot-uniform weights, zero biases (FP32 values as float64)."""
    rng = np.random.default_rng(seed)
    def glorot(fan_in, fan_out):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=(fan_in, fan_out)).astype(np.float32).astype(np.float64)
    w1 = glorot(N_IN, N_HID)
    w1 = np.vstack([w1, np.zeros((1, N_HID))])          # row 63 multiplies the zero pad
    return {"w1": w1, "b1": np.zeros(N_HID), "w2": glorot(N_HID, N_HID), "b2": np.zeros(N_HID),
            "w3": glorot(N_HID, N_OUT), "b3": np.zeros(N_OUT)}


def feature_stats(X: np.ndarray, T: np.ndarray):
    """(shift[64], scale[64], out_scale[4]) as FP32 values: per field f the
    mean and 1/std (population) of the centre column X[:, 9 f + 4], expanded
    to the field's nine columns; the pad column 63 gets shift 0, scale 1;
    out_scale = RMS of each target column.  Zero spreads map to 1."""
    shift = np.zeros(N_PAD)
    scale = np.ones(N_PAD)
    for f in range(7):
        c = X[:, 9 * f + 4]
        mu = c.mean()
        sd = math.sqrt(np.mean((c - mu) ** 2))
        shift[9 * f: 9 * f + 9] = mu
        scale[9 * f: 9 * f + 9] = 1.0 / sd if sd > 0 else 1.0
    rms = np.sqrt(np.mean(T * T, axis=0))
    out_scale = np.where(rms > 0, rms, 1.0)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return f32(shift), f32(scale), f32(out_scale)


def normalise(X, shift, scale) -> np.ndarray:
    """z = (x - shift) * scale in FP32 arithmetic (pad column forced to 0)."""
    z = (np.asarray(X, np.float32) - np.asarray(shift, np.float32)) * np.asarray(scale, np.float32)
    z = z.astype(np.float64)
    z[:, N_IN:] = 0.0
    return z


def forward(p: dict, X: np.ndarray, shift: np.ndarray, scale: np.ndarray, rnd=bf16):
    """Normalised output y [n, 4] and the cached activations.  `rnd` is the
    rounding applied where the GPU rounds to bfloat16 (identity: exact math)."""
    z = rnd(normalise(X, shift, scale))
    a1 = z @ rnd(p["w1"]) + p["b1"]
    h1 = rnd(np.maximum(a1, 0.0))
    a2 = h1 @ rnd(p["w2"]) + p["b2"]
    h2 = rnd(np.maximum(a2, 0.0))
    y = h2 @ rnd(p["w3"]) + p["b3"]
    return y, (z, h1, h2)


def loss_and_grads(p: dict, X, T, shift, scale, rnd=bf16):
    """Mean squared error over samples and outputs of y against the
    normalised targets T, and its gradients with respect to the FP32 master
    parameters (straight through the bfloat16 roundings)."""
    y, (z, h1, h2) = forward(p, X, shift, scale, rnd)
    n = X.shape[0]
    r = y - T
    loss = float(np.mean(r * r))
    dy = 2.0 * r / (n * N_OUT)
    g = {"w3": h2.T @ dy, "b3": dy.sum(0)}
    d2 = (dy @ rnd(p["w3"]).T) * (h2 > 0)
    g["w2"], g["b2"] = h1.T @ d2, d2.sum(0)
    d1 = (d2 @ rnd(p["w2"]).T) * (h1 > 0)
    g["w1"], g["b1"] = z.T @ d1, d1.sum(0)
    return loss, g


def learned_correction(p: dict, shift, scale, out_scale, ood: float = 6.0):
    """Closure correction for ``Oracle(closure_correction=...)``: the network's
    (tau_xx, tau_xy, tau_yy, eps) corrections from the current moments; cells
    with any normalised input beyond `ood` (or not finite), or a non-finite
    output, fall back to the analytic closure (correction 0)."""
    def corr(rho, mx, my, bx, by):
        X = closure_features(rho, mx, my, bx, by)
        with np.errstate(invalid="ignore", over="ignore"):
            y, _ = forward(p, X, shift, scale)
            zn = np.abs(normalise(X, shift, scale))
            out = ~(zn <= ood).all(axis=1, keepdims=True) | ~np.isfinite(y).all(axis=1, keepdims=True)
            y = np.where(out, 0.0, y * out_scale)
        return y.T.reshape((N_OUT,) + rho.shape)
    return corr


def adam_step(p: dict, g: dict, m: dict, v: dict, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of every parameter, step t >= 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
