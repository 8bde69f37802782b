// Device helpers shared by the timestep kernels and the learned-closure
// kernels: the subgrid terms of the analytic closure and the 3x3 gradient.
#pragma once

#include <hip/hip_runtime.h>

#include "lbmhd.h"

namespace lbm {

// Subgrid terms of the filtered equilibria (Sec. 2.1 FilterExampleSmall with
// density gradients dropped, Sec. 3).  g*_ab = D_b m_a, h*_ab = D_b B_a; with
// k2 = closure_scale Delta^2 / 12:
//   P_ac = k2/rho sum_b D_b m_a D_b m_c   (Reynolds products m_a m_c / rho)
//   Q_ac = k2     sum_b D_b B_a D_b B_c   (Maxwell products B_a B_c)
//   R_ac = k2/rho sum_b D_b m_a D_b B_c   (induction products m_a B_c / rho)
// tau_xy = P_xy - Q_xy enters M3; tau_d = (P_xx - P_yy) - (Q_xx - Q_yy) enters
// M4; tau_s = P_xx + P_yy enters M7 and M8 (times -3); eps = R_xy - R_yx is
// the filtered part of the induction moment E = (u x B)_z.
template <typename C>
struct Closure {
  C tau_xy, tau_d, tau_s, eps;
};

// g = D m, h = D B (gxy = D_y m_x), k2 = closure strength x Delta^2 / 12.
// Reynolds P_ac = k2/rho (D m_a).(D m_c), Maxwell Q_ac = k2 (D B_a).(D B_c),
// induction R_ac = k2/rho (D m_a).(D' B_c); the induction product takes its
// B gradients from h' (equal to h except in the density-gradient closure).
template <typename C>
__device__ __forceinline__ Closure<C> closure_terms(C gxx, C gxy, C gyx, C gyy, C hxx, C hxy, C hyx, C hyy,
                                                    C pxx_, C pxy_, C pyx_, C pyy_, C inv_rho, C k2) {
  const C kr = k2 * inv_rho;
  const C pxx = kr * (gxx * gxx + gxy * gxy);
  const C pyy = kr * (gyx * gyx + gyy * gyy);
  const C pxy = kr * (gxx * gyx + gxy * gyy);
  const C qxx = k2 * (hxx * hxx + hxy * hxy);
  const C qyy = k2 * (hyx * hyx + hyy * hyy);
  const C qxy = k2 * (hxx * hyx + hxy * hyy);
  const C rxy = kr * (gxx * pyx_ + gxy * pyy_);
  const C ryx = kr * (gyx * pxx_ + gyy * pxy_);
  Closure<C> c;
  c.tau_xy = pxy - qxy;
  c.tau_d = (pxx - pyy) - (qxx - qyy);
  c.tau_s = pxx + pyy;
  c.eps = rxy - ryx;
  return c;
}

template <typename C>
__device__ __forceinline__ Closure<C> closure_terms(C gxx, C gxy, C gyx, C gyy, C hxx, C hxy, C hyx,
                                                    C hyy, C inv_rho, C k2) {
  return closure_terms(gxx, gxy, gyx, gyy, hxx, hxy, hyx, hyy, hxx, hxy, hyx, hyy, inv_rho, k2);
}

// FilterExampleLarge with Z = rho: the bracket of the expansion of
// bar(XY/rho) factors as (D X - X a).(D Y - Y a), a = D rho / rho, so every
// quotient product (Reynolds and induction) takes gradients corrected by
// their field times a, while the Maxwell product B_a B_c (no divisor)
// keeps the plain B gradients.  gr[k][b] = D_b of (m_x, m_y, B_x, B_y, rho).
template <typename C>
__device__ __forceinline__ Closure<C> closure_terms_full(const C gr[5][2], C mx, C my, C bx, C by, C inv_rho,
                                                         C k2) {
  const C ax = gr[4][0] * inv_rho, ay = gr[4][1] * inv_rho;
  return closure_terms(gr[0][0] - mx * ax, gr[0][1] - mx * ay, gr[1][0] - my * ax, gr[1][1] - my * ay,
                       gr[2][0], gr[2][1], gr[3][0], gr[3][1],
                       gr[2][0] - bx * ax, gr[2][1] - bx * ay, gr[3][0] - by * ax, gr[3][1] - by * ay, inv_rho, k2);
}

// Discrete gradient from a 3x3 neighbourhood (value at offset (dx, dy)).
// iso9: D_x a = (a_E - a_W)/3 + (a_NE + a_SE - a_NW - a_SW)/12 (and D_y by
// symmetry), i.e. 3 sum_i w_i c_i a(x + c_i); central5: (a_E - a_W)/2.
template <typename C, int STENCIL>
__device__ __forceinline__ void grad3x3(C e, C w, C n, C s, C ne, C nw, C se, C sw, C& dx, C& dy) {
  if ((STENCIL & 1) == LBM_STENCIL_ISO9) {  // the LOCAL variants use the same two stencils
    const C third = C(1.0 / 3.0), twelfth = C(1.0 / 12.0);
    dx = (e - w) * third + ((ne + se) - (nw + sw)) * twelfth;
    dy = (n - s) * third + ((ne + nw) - (se + sw)) * twelfth;
  } else {
    dx = (e - w) * C(0.5);
    dy = (n - s) * C(0.5);
  }
}

}  // namespace lbm
