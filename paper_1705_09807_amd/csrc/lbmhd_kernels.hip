// HIP kernels (gfx950) of the filtered lattice-Boltzmann MHD timestep.
//
// Method: Flint & Vahala, arXiv 1705.09807.  Sec. 2: kinetic equations
// (LBKinEqn, LBMagEqn), equilibria (feq, geq), moment transform
// (FluidTMatrix), equilibrium moments (KinMomentEq, MagMomentEq), transport
// coefficients; Sec. 2.1: filtered equilibrium moments built from the
// Delta-expansion FilterExampleSmall; Sec. 3: SRT runs, density gradients
// dropped (simplified M3).
//
// Storage: structure of arrays by lattice row.  Lattice row y holds the 19
// population rows f_0..f_8, g_x0..g_x4, g_y0..g_y4 (x fastest) one after
// another, each padded to a multiple of 64 elements.  FP32 stores f as the deviation
// f_i - w_i rho0 from the rest equilibrium, so that the small dynamic part
// keeps its digits; FP64 stores f itself (rho0 = 0 below); g is stored as is.
//
// Two schedules:
//  * fused (two buffers, pull streaming): a buffer holds post-collision
//    populations at their source cell; a sweep gathers f_q(x) from x - c_q
//    (loads shifted by at most one cell), collides and stores aligned rows.
//    With the closure on, one workgroup marches up a column strip and keeps
//    a 4-row ring of moments in LDS, so the 3x3 gradient stencil costs no
//    extra HBM pass.
//  * AA (one buffer, in place): even steps read and write the cell's own
//    slots (reversed), odd steps read from and write to the neighbours; the
//    read set of a cell equals its write set, so cells never race.  With the
//    closure on, a moment sweep writes m and B to four planes first.
//
// All arithmetic that defines the method (moments, closure, collision,
// equilibria) lives in the __device__ functions below and is shared by every
// kernel, so both schedules compute identical values.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lbmhd_device.h"
#include "lbmhd_internal.h"
#include "lbmhd_learned.h"
#include "lbmhd_mlp_device.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Lattice (Sec. 2): D2Q9 velocities; the vector distribution uses the first
// QG of them: five (D2Q5, the default) or all nine (D2Q9, Sec. 2's own
// lattice for g).  Population q: f_q (q < 9), g_x,q-9 (9 .. 8+QG),
// g_y,q-9-QG (9+QG .. 8+2QG); NPOP = 9 + 2 QG populations per cell.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int cx9(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int cy9(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp9(int i) {
  return i == 0 ? 0 : (i < 5 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
template <int QG> constexpr int kPop = 9 + 2 * QG;
template <int QG = 5>
__host__ __device__ constexpr int qbase(int q) { return q < 9 ? q : (q < 9 + QG ? q - 9 : q - 9 - QG); }
template <int QG = 5>
__host__ __device__ constexpr int qcx(int q) { return cx9(qbase<QG>(q)); }
template <int QG = 5>
__host__ __device__ constexpr int qcy(int q) { return cy9(qbase<QG>(q)); }
template <int QG = 5>
__host__ __device__ constexpr int qopp(int q) {
  return q < 9 ? opp9(q) : (q < 9 + QG ? 9 + opp9(q - 9) : 9 + QG + opp9(q - 9 - QG));
}
// D2Q9 weights (rest deviation of f, and g on D2Q9) and D2Q5 weights of the
// vector distribution.
__host__ __device__ constexpr double w9(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
__host__ __device__ constexpr double w5(int i) { return i == 0 ? 1.0 / 3.0 : 1.0 / 6.0; }
template <int QG>
__host__ __device__ constexpr double wg(int i) { return QG == 5 ? w5(i) : w9(i); }

static_assert(opp9(1) == 3 && opp9(2) == 4 && opp9(3) == 1 && opp9(4) == 2, "opposites");
static_assert(opp9(5) == 7 && opp9(6) == 8 && opp9(7) == 5 && opp9(8) == 6, "opposites");
static_assert(qcx(10) == 1 && qcy(16) == 1 && qopp(15) == 17, "vector planes");
static_assert(qcx<9>(14) == 1 && qcy<9>(20) == 1 && qopp<9>(23) == 25 && qopp<9>(14) == 16, "D2Q9 vector planes");
static_assert(kPop<5> == kQ, "D2Q5 population count");

template <typename S> struct ComputeOf { using type = float; };
template <> struct ComputeOf<double> { using type = double; };

// Storage codecs.  FP64 and FP32 store values as they are.  The 16-bit
// storage types hold the deviations (see below) for FP32 arithmetic: FP16
// scaled by 2^8, which lifts the small deviations out of the FP16 subnormal
// range (normal values start at 6.1e-5) while the largest ones (~0.1) stay
// far below 65504; BF16 unscaled (it has the FP32 exponent range).  All
// conversions round to nearest even.
template <typename S> struct Codec {
  static constexpr float kScale = 1.0f;
};
template <> struct Codec<_Float16> {
  static constexpr float kScale = 256.0f;
};
template <typename C, typename S>
__device__ __forceinline__ C decode(S v) {
  if constexpr (sizeof(S) == 2)
    return C(float(v) * (1.0f / Codec<S>::kScale));
  else
    return C(v);
}
template <typename S, typename C>
__device__ __forceinline__ S encode(C v) {
  if constexpr (sizeof(S) == 2)
    return S(float(v) * Codec<S>::kScale);
  else
    return S(v);
}

__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Rates in the compute type, with the 1/|row|^2 of T^-1 = T^T diag(1/|row|^2)
// folded in: |row|^2 = 9, 6, 6, 4, 4, 12, 12, 180, 20 for M0..M8.
template <typename C>
struct Rates {
  C s3q, s4q, s5q, s6q, s7q, s8q;
  C sm, k2, rho0;
  C bx0, by0;  // reference field of the stored g deviations
};

template <typename C>
static Rates<C> make_rates(const Launch& L) {
  Rates<C> r;
  r.s3q = C(L.rate[3] / 4.0);
  r.s4q = C(L.rate[4] / 4.0);
  r.s5q = C(L.rate[5] / 12.0);
  r.s6q = C(L.rate[6] / 12.0);
  r.s7q = C(L.rate[7] / 180.0);
  r.s8q = C(L.rate[8] / 20.0);
  r.sm = C(L.sm);
  r.k2 = C(L.k2);
  r.rho0 = C(L.rho0);
  r.bx0 = C(L.bref[0]);
  r.by0 = C(L.bref[1]);
  return r;
}

// ---------------------------------------------------------------------------
// Per-cell arithmetic of the method
// ---------------------------------------------------------------------------
template <typename C>
struct Mom {
  C drho, mx, my, dbx, dby;  // rho - rho0, rho u, B - B_ref
};

// rho = sum f_i, rho u = sum c_i f_i, B = sum g_i (Sec. 2), from the stored
// deviations f_i - w_i rho0 and g_i - w'_i B_ref (sum_i w_i = sum_i w'_i = 1,
// sum_i w_i c_i = 0).  Fixed summation order: every kernel gets bit-identical
// moments for a cell.
template <int QG, typename C>
__device__ __forceinline__ Mom<C> moments_of(const C* v) {
  Mom<C> m;
  m.drho = (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) + v[8];
  m.mx = ((v[1] - v[3]) + (v[5] - v[6])) + (v[8] - v[7]);
  m.my = ((v[2] - v[4]) + (v[5] - v[7])) + (v[6] - v[8]);
  if constexpr (QG == 5) {
    m.dbx = ((v[9] + v[10]) + (v[11] + v[12])) + v[13];
    m.dby = ((v[14] + v[15]) + (v[16] + v[17])) + v[18];
  } else {
    m.dbx = (((v[9] + v[10]) + (v[11] + v[12])) + ((v[13] + v[14]) + (v[15] + v[16]))) + v[17];
    m.dby = (((v[18] + v[19]) + (v[20] + v[21])) + ((v[22] + v[23]) + (v[24] + v[25]))) + v[26];
  }
  return m;
}

template <typename C>
__device__ __forceinline__ Mom<C> moments19(const C v[kQ]) {
  return moments_of<5>(v);
}

// One collision of the 19 populations of a cell (Sec. 2, Sec. 3).
//  f: the collision term of LBKinEqn with rate tensor s' = T^-1 S T, i.e.
//     f* = f - T^-1 S (M - M_eq), M = T f, M_eq the filtered KinMomentEq table
//     (rho u_x rho u_y / rho - B_x B_y + tau_xy, ...).  Conserved M0..M2 have
//     rate 0, so only rows 3..8 are formed, and T^-1 = T^T diag(1/|row|^2).
//     In deviation storage M(w rho0) = (rho0, 0, ..., 0, 5 rho0 / 3) shifts
//     only M8's equilibrium.
//  g: g* = g - s_m (g - g_eq), g_eq_i = w'_i (B + 3 [(c.u) B - (c.B) u]) on D2Q5
//     or D2Q9, which is g_eq_ix = w'_i (B_x - 3 c_iy E), g_eq_iy = w'_i (B_y +
//     3 c_ix E) with E = (m_x B_y - m_y B_x) / rho + eps.  On D2Q9 this is the
//     moment-space SRT of MagTMatrix / MagMomentEq: with one rate for every
//     moment, relaxing T_m g towards N^eq and mapping back is relaxing g
//     towards T_m^-1 N^eq, the D2Q9 geq.
template <int QG, typename C>
__device__ __forceinline__ void collide_q(C* v, const Mom<C>& m, const Closure<C>& cl, const Rates<C>& r) {
  const C rho = r.rho0 + m.drho;
  const C ir = C(1) / rho;
  const C mx = m.mx, my = m.my, bx = r.bx0 + m.dbx, by = r.by0 + m.dby;
  // rows 3..8 of T applied to the stored deviations
  const C d56 = v[5] - v[6], d78 = v[7] - v[8], d87 = v[8] - v[7];
  const C s14 = (v[1] + v[2]) + (v[3] + v[4]);
  const C s58 = (v[5] + v[6]) + (v[7] + v[8]);
  const C M3 = d56 + d78;
  const C M4 = (v[1] + v[3]) - (v[2] + v[4]);
  const C M5 = C(2) * (v[3] - v[1]) + d56 + d87;
  const C M6 = C(2) * (v[4] - v[2]) + (v[5] + v[6]) - (v[7] + v[8]);
  const C M7 = C(4) * v[0] - C(5) * s14 + C(4) * s58;
  const C M8 = C(4) * v[0] - s58;
  // filtered equilibrium moments (deviation form for M8)
  const C q2 = (mx * mx + my * my) * ir;
  const C e3 = mx * my * ir - bx * by + cl.tau_xy;
  const C e4 = (mx * mx - my * my) * ir - (bx * bx - by * by) + cl.tau_d;
  const C e7 = C(-3) * q2 - C(3) * cl.tau_s;
  const C e8 = C(5.0 / 3.0) * m.drho + e7;
  const C d3 = r.s3q * (M3 - e3);
  const C d4 = r.s4q * (M4 - e4);
  const C d5 = r.s5q * (M5 + mx);
  const C d6 = r.s6q * (M6 + my);
  const C d7 = r.s7q * (M7 - e7);
  const C d8 = r.s8q * (M8 - e8);
  const C g7 = C(5) * d7, h = C(4) * d7 - d8;
  v[0] -= C(4) * (d7 + d8);
  v[1] -= (d4 - C(2) * d5) - g7;
  v[2] -= (-d4 - C(2) * d6) - g7;
  v[3] -= (d4 + C(2) * d5) - g7;
  v[4] -= (C(2) * d6 - d4) - g7;
  v[5] -= (d3 + d5 + d6) + h;
  v[6] -= (d6 - d3 - d5) + h;
  v[7] -= (d3 - d5 - d6) + h;
  v[8] -= (d5 - d3 - d6) + h;
  // vector distribution, SRT; the w'_i B_ref part of the stored deviation
  // cancels against that of g_eq
  const C E = (mx * by - my * bx) * ir + cl.eps;
  const C E3 = C(3) * E;
#pragma unroll
  for (int i = 0; i < QG; ++i) {
    const C wi = C(wg<QG>(i));
    const C gx = wi * (m.dbx - C(cy9(i)) * E3);
    const C gy = wi * (m.dby + C(cx9(i)) * E3);
    v[9 + i] -= r.sm * (v[9 + i] - gx);
    v[9 + QG + i] -= r.sm * (v[9 + QG + i] - gy);
  }
}

template <typename C>
__device__ __forceinline__ void collide19(C v[kQ], const Mom<C>& m, const Closure<C>& cl, const Rates<C>& r) {
  collide_q<5>(v, m, cl, r);
}

// Closure gradients from local non-equilibrium moments (LOCAL stencils),
// with the stencil vorticity wm = D_x m_y - D_y m_x.  First-order
// Chapman-Enskog of the pre-collision populations: M3 - M3^eq =
// -(2 rho / (3 s3)) S_xy, M4 - M4^eq = -(2 rho / (3 s4)) (S_xx - S_yy) with the
// unfiltered equilibria, S_xx = -S_yy (incompressible), D m = rho D u; and
// D_b B_a = -3 s_m (Lam_ba - Lam^eq_ba), Lam_ba = sum_i c_ib g_ia, Lam^eq_xy =
// E, Lam^eq_yx = -E.  The stored deviations have the same M3, M4 and Lam
// (the rest state has none).  gr[k] = (D_x, D_y) of m_x, m_y, B_x, B_y.
template <typename C>
__device__ __forceinline__ void local_gradients(const C v[kQ], const Mom<C>& m, const Rates<C>& r, C wm,
                                                C gr[4][2]) {
  // evaluated as written (no contraction into FMAs), so every copy of an
  // unrolled row body gives the same bits
#pragma clang fp contract(off)
  const C rho = r.rho0 + m.drho;
  const C ir = C(1) / rho;
  const C bx = r.bx0 + m.dbx, by = r.by0 + m.dby;
  const C M3 = (v[5] - v[6]) + (v[7] - v[8]);
  const C M4 = (v[1] + v[3]) - (v[2] + v[4]);
  const C e3 = m.mx * m.my * ir - bx * by;
  const C e4 = (m.mx * m.mx - m.my * m.my) * ir - (bx * bx - by * by);
  // rho S: s3 = 4 s3q and s4 = 4 s4q exactly
  const C rsxy = C(-6) * r.s3q * (M3 - e3);
  const C rsxx = C(-3) * r.s4q * (M4 - e4);
  gr[0][0] = rsxx;
  gr[0][1] = rsxy - C(0.5) * wm;
  gr[1][0] = rsxy + C(0.5) * wm;
  gr[1][1] = -rsxx;
  const C E = (m.mx * by - m.my * bx) * ir;
  const C k = C(-3) * r.sm;
  gr[2][0] = k * (v[10] - v[12]);
  gr[2][1] = k * ((v[11] - v[13]) + E);
  gr[3][0] = k * ((v[15] - v[17]) - E);
  gr[3][1] = k * (v[16] - v[18]);
}

// ---------------------------------------------------------------------------
// Fused schedule (two buffers, pull streaming).  A buffer holds the
// post-collision populations of the previous step at their source cell, so
// the state at time t is f_q(x) = buf[q][x - c_q]: every sweep gathers with
// loads shifted by at most one cell and stores aligned, coalesced rows.
// ---------------------------------------------------------------------------

// Two consecutive stored values (one aligned load or store).
template <typename S> using Vec2 = S __attribute__((ext_vector_type(2)));
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// Addressing.  A buffer is ny lattice rows, each holding the NPOP population
// rows of that lattice row one after another, `pitch` elements apart:
// element (q, x, y) at (y * NPOP + q) * pitch + x.  Keeping the populations
// of a lattice row together means the workgroups that run at the same time
// read and write a few contiguous stretches of memory instead of one stretch
// per population plane.  An access is a wave-uniform row base (the lattice
// row's offset, 64-bit, plus q * pitch, in scalar registers) plus a 32-bit
// byte offset of the column, the scalar-base + vector-offset form of global
// loads and stores.
template <typename S>
__device__ __forceinline__ const S* at(const S* __restrict__ base, int64_t row_off, uint32_t col_off) {
  return reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + row_off + col_off);
}
template <typename S>
__device__ __forceinline__ S* at(S* __restrict__ base, int64_t row_off, uint32_t col_off) {
  return reinterpret_cast<S*>(reinterpret_cast<char*>(base) + row_off + col_off);
}

// Streaming store: non-temporal when the working set exceeds the caches.
template <bool NT, typename T>
__device__ __forceinline__ void store(T* p, T v) {
  if (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Byte offsets of the lattice rows y - 1, y, y + 1 (periodic) and of the
// columns x - 1, x, x + 1 of a cell.
struct Rows {
  int64_t s, c, n;
};
template <typename S, int QG = 5>
__device__ __forceinline__ Rows rows_of(int y, int ny, int64_t pitch) {
  const int64_t rb = int64_t(kPop<QG>) * pitch * int64_t(sizeof(S));
  Rows r;
  r.c = int64_t(y) * rb;
  r.s = int64_t(y == 0 ? ny - 1 : y - 1) * rb;
  r.n = int64_t(y + 1 == ny ? 0 : y + 1) * rb;
  return r;
}
struct Cols {
  uint32_t w, c, e;
};
template <typename S>
__device__ __forceinline__ Cols cols_of(int x, int nx) {
  Cols c;
  c.c = uint32_t(x) * uint32_t(sizeof(S));
  c.w = uint32_t(x == 0 ? nx - 1 : x - 1) * uint32_t(sizeof(S));
  c.e = uint32_t(x + 1 == nx ? 0 : x + 1) * uint32_t(sizeof(S));
  return c;
}

// f_q(x, y) = src[q][x - c_q][y - c_q] for one cell.
template <typename S, typename C, int QG = 5>
__device__ __forceinline__ void pull_cell(const S* __restrict__ src, int64_t pitch, const Rows& rw, const Cols& cl,
                                          C* v) {
#pragma unroll
  for (int q = 0; q < kPop<QG>; ++q) {
    const uint32_t xo = qcx<QG>(q) > 0 ? cl.w : (qcx<QG>(q) < 0 ? cl.e : cl.c);
    const int64_t yo = qcy<QG>(q) > 0 ? rw.s : (qcy<QG>(q) < 0 ? rw.n : rw.c);
    v[q] = decode<C>(*at(src + q * pitch, yo, xo));
  }
}

// Two horizontally adjacent cells x, x + 1 (x even, nx even): the c_x = 0
// populations come in one aligned two-element load.
template <typename S, typename C, int QG = 5>
__device__ __forceinline__ void pull_pair(const S* __restrict__ src, int64_t pitch, int nx, const Rows& rw, int x,
                                          C* a, C* b) {
  using V2 = Vec2<S>;
  const uint32_t es = uint32_t(sizeof(S));
  const uint32_t xw = uint32_t(x == 0 ? nx - 1 : x - 1) * es, x0 = uint32_t(x) * es, x1 = x0 + es;
  const uint32_t x2 = uint32_t(x + 2 == nx ? 0 : x + 2) * es;
#pragma unroll
  for (int q = 0; q < kPop<QG>; ++q) {
    const int64_t yo = qcy<QG>(q) > 0 ? rw.s : (qcy<QG>(q) < 0 ? rw.n : rw.c);
    const S* pq = src + q * pitch;
    if (qcx<QG>(q) == 0) {
      const V2 t = *reinterpret_cast<const V2*>(at(pq, yo, x0));
      a[q] = decode<C>(t.x);
      b[q] = decode<C>(t.y);
    } else if (qcx<QG>(q) > 0) {
      a[q] = decode<C>(*at(pq, yo, xw));
      b[q] = decode<C>(*at(pq, yo, x0));
    } else {
      a[q] = decode<C>(*at(pq, yo, x1));
      b[q] = decode<C>(*at(pq, yo, x2));
    }
  }
}

// Closure off (Delta = 0).  One row segment of 2 * 128 cells per workgroup,
// two cells per thread, aligned two-element stores.  Requires nx even.
// Measured against 64- and 256-thread segments and two rows per workgroup at
// 4096^2 and 8192^2 FP32: 0.4-4 % faster than each.
template <typename S, typename C, bool NT, int QG>
__global__ void __launch_bounds__(128)
k_fused_dns_pair(const S* __restrict__ src, S* __restrict__ dst, int nx, int ny, int64_t pitch, Rates<C> r) {
  using nv2 = Vec2<S>;
  const int x = (blockIdx.x * 128 + threadIdx.x) * 2;
  const int y = blockIdx.y;
  if (x >= nx) return;
  const Rows rw = rows_of<S, QG>(y, ny, pitch);
  C a[kPop<QG>], b[kPop<QG>];
  pull_pair<S, C, QG>(src, pitch, nx, rw, x, a, b);
  const Closure<C> cl = {C(0), C(0), C(0), C(0)};
  {
    const Mom<C> m = moments_of<QG>(a);
    collide_q<QG>(a, m, cl, r);
  }
  {
    const Mom<C> m = moments_of<QG>(b);
    collide_q<QG>(b, m, cl, r);
  }
  const uint32_t xo = uint32_t(x) * uint32_t(sizeof(S));
#pragma unroll
  for (int q = 0; q < kPop<QG>; ++q) {
    nv2 t;
    t.x = encode<S>(a[q]);
    t.y = encode<S>(b[q]);
    store<NT>(reinterpret_cast<nv2*>(at(dst + q * pitch, rw.c, xo)), t);
  }
}

template <typename S> using Vec4 = S __attribute__((ext_vector_type(4)));

// Closure off, any nx: one cell per thread, row segments of 256 cells.
template <typename S, typename C, bool NT, int QG>
__global__ void __launch_bounds__(256)
k_fused_dns(const S* __restrict__ src, S* __restrict__ dst, int nx, int ny, int64_t pitch, Rates<C> r) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= nx) return;
  const Rows rw = rows_of<S, QG>(y, ny, pitch);
  const Cols cl = cols_of<S>(x, nx);
  C v[kPop<QG>];
  pull_cell<S, C, QG>(src, pitch, rw, cl, v);
  const Mom<C> m = moments_of<QG>(v);
  const Closure<C> zero = {C(0), C(0), C(0), C(0)};
  collide_q<QG>(v, m, zero, r);
#pragma unroll
  for (int q = 0; q < kPop<QG>; ++q) store<NT>(at(dst + q * pitch, rw.c, cl.c), encode<S>(v[q]));
}

// Closure on, FP64 (FP32 compute runs k_fused_les_f, the same schedule with
// buffer addressing).  A workgroup of W + 64 lanes owns the column strip
// x0 .. x0+W-1 and marches up rows y0 .. y0+ry-1.  The moments (m_x, m_y,
// B_x - B_ref, B_y - B_ref) of the rows y-1 .. y+2 live in a 4-slot LDS ring
// indexed by column - x0 + 1.  Lanes 0..W-1 gather, collide and store their
// cells; one extra wave gathers the two halo columns (x0 - 1 and the column
// after the strip's last cell), so no collision wave carries extra loads
// (every wave of the workgroup waits at the per-row barrier for the slowest).
// Rows are software-pipelined two deep: the loads of row y+2 are issued
// before row y is collided.  A ring slot is rewritten only after the barrier
// that follows its last read.
//
// MODE kClosureCorr: four FP32 planes (tau_xx, tau_xy, tau_yy, eps) of a
// learned correction are added to the analytic subgrid terms of every cell.
// MODE kClosureFull: the ring carries rho - rho0 as a fifth field and the
// closure keeps the filtered-density gradient terms.
enum { kClosurePlain = 0, kClosureCorr = 1, kClosureFull = 2 };

template <typename S, typename C, int W, int STENCIL, bool NT, int MODE, int QG>
__global__ void __launch_bounds__(W + 64)
k_fused_les(const S* __restrict__ src, S* __restrict__ dst, int nx, int ny, int64_t pitch, int ry, Rates<C> r,
            const float* __restrict__ corr) {
  constexpr int NF = MODE == kClosureFull ? 5 : 4;
  __shared__ C ring[4][NF][W + 2];
  const int tid = threadIdx.x;
  const bool halo_wave = tid >= W;
  const int x0 = blockIdx.x * W;
  const int last = min(x0 + W, nx) - 1;      // last column of this strip
  const bool valid = !halo_wave && x0 + tid <= last;
  const int hl = tid - W;                    // lane within the halo wave
  const bool hlo = halo_wave && hl == 0;     // gathers the column left of the strip
  const bool hhi = halo_wave && hl == 1;     // gathers the column right of the strip
  const bool writer = valid || hlo || hhi;   // lanes that put moments into the ring
  const bool loader = !halo_wave || hl < 2;
  const int widx = hlo ? 0 : (hhi ? last - x0 + 2 : tid + 1);
  const int xc = hlo ? (x0 == 0 ? nx - 1 : x0 - 1)
                     : (hhi ? (last + 1 == nx ? 0 : last + 1) : (valid ? x0 + tid : last));
  const Cols cx = cols_of<S>(xc, nx);        // idle lanes address a valid cell, never stored
  const int y0 = blockIdx.y * ry;
  const int y1 = min(y0 + ry, ny);

  auto put = [&](int slot, const C* v) {
    const Mom<C> m = moments_of<QG>(v);
    ring[slot][0][widx] = m.mx;
    ring[slot][1][widx] = m.my;
    ring[slot][2][widx] = m.dbx;
    ring[slot][3][widx] = m.dby;
    if constexpr (NF == 5) ring[slot][4][widx] = m.drho;
  };
  auto wrapy = [&](int y) { return y < 0 ? y + ny : (y >= ny ? y - ny : y); };

  C cur[kPop<QG>], nxt[kPop<QG>], nn[kPop<QG>];
  if (loader) {
    pull_cell<S, C, QG>(src, pitch, rows_of<S, QG>(wrapy(y0 - 1), ny, pitch), cx, nn);
    if (writer) put(0, nn);
    pull_cell<S, C, QG>(src, pitch, rows_of<S, QG>(y0, ny, pitch), cx, cur);
    if (writer) put(1, cur);
    pull_cell<S, C, QG>(src, pitch, rows_of<S, QG>(wrapy(y0 + 1), ny, pitch), cx, nxt);
    if (writer) put(2, nxt);
  }
  __syncthreads();
  {
    // Rows rotated by copies.  The learned correction of row y + 1 is loaded
    // with row y + 2's populations, a row ahead of its use.
    const int64_t n = (int64_t)nx * ny;
    float cc[4] = {0.0f, 0.0f, 0.0f, 0.0f}, cn[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    auto load_corr = [&](int y, float (&c)[4]) __attribute__((always_inline)) {
      const int64_t ci = (int64_t)y * nx + x0 + tid;
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] = corr[k * n + ci];
    };
    if constexpr (MODE == kClosureCorr) {
      if (valid) load_corr(y0, cc);
    }
    for (int y = y0; y < y1; ++y) {
      const int s = y - y0 + 1;                 // ring slot of row y is s & 3
      const bool more = y + 1 < y1;             // row y + 2 is needed for row y + 1
      if (more && loader) pull_cell<S, C, QG>(src, pitch, rows_of<S, QG>(wrapy(y + 2), ny, pitch), cx, nn);
      if constexpr (MODE == kClosureCorr) {
        if (more && valid) load_corr(y + 1, cn);
      }
      if (valid) {
        const int sn = (s + 1) & 3, sc = s & 3, ss = (s - 1) & 3, l = tid + 1;
        C gr[NF][2];
#pragma unroll
        for (int k = 0; k < NF; ++k) {
          grad3x3<C, STENCIL>(ring[sc][k][l + 1], ring[sc][k][l - 1], ring[sn][k][l], ring[ss][k][l],
                              ring[sn][k][l + 1], ring[sn][k][l - 1], ring[ss][k][l + 1], ring[ss][k][l - 1], gr[k][0],
                              gr[k][1]);
        }
        const Mom<C> m = moments_of<QG>(cur);
        const C ir = C(1) / (r.rho0 + m.drho);
        Closure<C> cl;
        if constexpr (MODE == kClosureFull) {
          cl = closure_terms_full(gr, m.mx, m.my, r.bx0 + m.dbx, r.by0 + m.dby, ir, r.k2);
        } else {
          if constexpr (STENCIL >= LBM_STENCIL_LOCAL_ISO9 && QG == 5)
            local_gradients(cur, m, r, gr[1][0] - gr[0][1], gr);
          cl = closure_terms(gr[0][0], gr[0][1], gr[1][0], gr[1][1], gr[2][0], gr[2][1], gr[3][0], gr[3][1], ir,
                             r.k2);
        }
        if constexpr (MODE == kClosureCorr) {
          const C txx = C(cc[0]), txy = C(cc[1]), tyy = C(cc[2]), eps = C(cc[3]);
          cl.tau_xy += txy;
          cl.tau_d += txx - tyy;
          cl.tau_s += txx + tyy;
          cl.eps += eps;
        }
        collide_q<QG>(cur, m, cl, r);
        const int64_t yo = int64_t(y) * int64_t(kPop<QG>) * pitch * int64_t(sizeof(S));
#pragma unroll
        for (int q = 0; q < kPop<QG>; ++q) store<NT>(at(dst + q * pitch, yo, cx.c), encode<S>(cur[q]));
      }
      if (more && writer) put((s + 2) & 3, nn);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kPop<QG>; ++q) {
        cur[q] = nxt[q];
        nxt[q] = nn[q];
      }
      if constexpr (MODE == kClosureCorr) {
#pragma unroll
        for (int k = 0; k < 4; ++k) cc[k] = cn[k];
      }
    }
  }
}

// A cell's populations as stored (16-bit values decoded where they are used).
template <typename S, int QG>
struct RawCell {
  S v[kPop<QG>];
};
template <typename S, typename C, int QG>
__device__ __forceinline__ void decode_raw(const RawCell<S, QG>& c, C* v) {
#pragma unroll
  for (int q = 0; q < kPop<QG>; ++q) v[q] = decode<C>(c.v[q]);
}

// Buffer addressing of the wave-strip sweep: a buffer resource per lattice
// row (its base held in scalar registers), the population's row offset as
// the scalar offset and the column's byte offset as the per-lane offset, so a
// load or store costs no per-lane address arithmetic.  Raw resources
// (stride 0) of num_records = the lattice row's bytes; every access of a row
// lies inside it, except the stores of lanes that own no output column,
// which take an offset past num_records: the hardware's range check drops
// them, so the row body has no branch around its stores.  (nx <= 32768, as
// lbm_create requires, keeps a lattice row below 27 * 32768 * 4 B = 3.5 MB
// and a row of input vectors at 512 KB, far below kDropOffset.)
constexpr uint32_t kDropOffset = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), 0x00020000);
}
template <typename S>
__device__ __forceinline__ S buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(S) == 2)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, int(voff), int(soff), 0));
  else
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
}
template <typename S, bool NT>
__device__ __forceinline__ void buf_store(S v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  constexpr int aux = NT ? 2 : 0;  // non-temporal
  if constexpr (sizeof(S) == 2)
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, int(voff), int(soff), aux);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, int(voff), int(soff), aux);
}

// Buffer loads and stores of T (4, 8 or 16 bytes: one, two or four stored values).
template <typename T>
__device__ __forceinline__ T buf_load_v(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), 0));
  else if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, int(voff), int(soff), 0));
}
template <typename T, bool NT>
__device__ __forceinline__ void buf_store_v(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  constexpr int aux = NT ? 2 : 0;
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, int(voff), int(soff), aux);
  else if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, int(voff), int(soff), aux);
  else
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, int(voff), int(soff), aux);
}

// f_q(x, y) = src[q][x - c_q][y - c_q] of one cell, as stored; ys, yc, yn
// are the (periodic) rows y - 1, y, y + 1, pq the bytes between population
// rows.
template <typename S, int QG>
__device__ __forceinline__ void pull_raw(const S* __restrict__ src, uint32_t pq, int ys, int yc, int yn,
                                         const Cols& cl, RawCell<S, QG>& c) {
  const uint32_t rowb = uint32_t(kPop<QG>) * pq;
  const char* b = reinterpret_cast<const char*>(src);
  const __amdgpu_buffer_rsrc_t rs = row_rsrc(b + int64_t(ys) * rowb, rowb);
  const __amdgpu_buffer_rsrc_t rc = row_rsrc(b + int64_t(yc) * rowb, rowb);
  const __amdgpu_buffer_rsrc_t rn = row_rsrc(b + int64_t(yn) * rowb, rowb);
#pragma unroll
  for (int q = 0; q < kPop<QG>; ++q) {
    const uint32_t xo = qcx<QG>(q) > 0 ? cl.w : (qcx<QG>(q) < 0 ? cl.e : cl.c);
    const __amdgpu_buffer_rsrc_t rr = qcy<QG>(q) > 0 ? rs : (qcy<QG>(q) < 0 ? rn : rc);
    c.v[q] = buf_load<S>(rr, xo, uint32_t(q) * pq);
  }
}

// Workgroups go to the XCDs in turn: workgroup b of a one-dimensional grid
// runs on XCD b % 8.  xcd_contiguous renumbers the nb workgroups so that each
// XCD takes one contiguous range of work items, so neighbouring row segments
// (or strips) run side by side on one XCD and the cache lines at their common
// edge, which both read, come from that XCD's L2 instead of two.  A bijection
// of 0 .. nb-1 for any nb, so results do not depend on the XCD count of the
// device or partition; only the cache benefit assumes eight.  Measured with the same results: the closure sweep
// at 8192^2 FP32 1701-1750 against 1761-1782 us (its reads 1.03x instead of
// 1.12x the algorithmic bytes at 4096^2), the 16-bit DNS sweep at 8192^2
// 844-862 against 916-918 us (FP16); the FP32 pair kernel was 3 % slower with
// it and keeps its two-dimensional grid.
__device__ __forceinline__ int xcd_contiguous(int b, int nb) {
  const int xcd = b & 7, k = b >> 3, q = nb >> 3, rm = nb & 7;
  return xcd < rm ? xcd * (q + 1) + k : rm * (q + 1) + (xcd - rm) * q + k;
}

// Closure off, 16-bit storage, nx a multiple of 4: four cells per thread, so
// every population moves in one aligned 8-byte load and store per thread (plus
// one 2-byte load of the neighbour column for those that stream along x),
// addressed through a resource per lattice row.  Measured 7-9 % faster than
// two cells per thread at 8192^2 with FP16 and BF16 storage (slower with FP32,
// whose pair loads are already 8 bytes), and the buffer form 0-4 % faster
// than per-lane addresses (BF16 8192^2 884-893 against 901-916 us; for the
// FP32 pair kernel it measured up to 3 % slower, so that one keeps them).
template <typename S, typename C, bool NT>
__global__ void __launch_bounds__(64)
k_fused_dns_quad(const S* __restrict__ src, S* __restrict__ dst, int nx, int ny, int64_t pitch, Rates<C> r) {
  using V4 = Vec4<S>;
  const int nseg = (nx + 255) / 256;  // row segments of 256 cells
  const int vb = xcd_contiguous(blockIdx.x, gridDim.x);
  const int x = ((vb % nseg) * 64 + threadIdx.x) * 4;
  const int y = vb / nseg;
  if (x >= nx) return;
  const uint32_t es = uint32_t(sizeof(S)), pq = uint32_t(pitch) * es, rowb = uint32_t(kQ) * pq;
  const char* b = reinterpret_cast<const char*>(src);
  const int ys = y == 0 ? ny - 1 : y - 1, yn = y + 1 == ny ? 0 : y + 1;
  const __amdgpu_buffer_rsrc_t rs = row_rsrc(b + int64_t(ys) * rowb, rowb);
  const __amdgpu_buffer_rsrc_t rc = row_rsrc(b + int64_t(y) * rowb, rowb);
  const __amdgpu_buffer_rsrc_t rn = row_rsrc(b + int64_t(yn) * rowb, rowb);
  const uint32_t x0 = uint32_t(x) * es;
  const uint32_t xw = uint32_t(x == 0 ? nx - 1 : x - 1) * es;
  const uint32_t x4 = uint32_t(x + 4 == nx ? 0 : x + 4) * es;
  C v[4][kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const __amdgpu_buffer_rsrc_t rr = qcy(q) > 0 ? rs : (qcy(q) < 0 ? rn : rc);
    const uint32_t so = uint32_t(q) * pq;
    const V4 t = buf_load_v<V4>(rr, x0, so);
    if (qcx(q) == 0) {
      v[0][q] = decode<C>(t.x);
      v[1][q] = decode<C>(t.y);
      v[2][q] = decode<C>(t.z);
      v[3][q] = decode<C>(t.w);
    } else if (qcx(q) > 0) {
      v[0][q] = decode<C>(buf_load<S>(rr, xw, so));
      v[1][q] = decode<C>(t.x);
      v[2][q] = decode<C>(t.y);
      v[3][q] = decode<C>(t.z);
    } else {
      v[0][q] = decode<C>(t.y);
      v[1][q] = decode<C>(t.z);
      v[2][q] = decode<C>(t.w);
      v[3][q] = decode<C>(buf_load<S>(rr, x4, so));
    }
  }
  const Closure<C> cl = {C(0), C(0), C(0), C(0)};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const Mom<C> m = moments19(v[k]);
    collide19(v[k], m, cl, r);
  }
  const __amdgpu_buffer_rsrc_t d = row_rsrc(reinterpret_cast<char*>(dst) + int64_t(y) * rowb, rowb);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    V4 t;
    t.x = encode<S>(v[0][q]);
    t.y = encode<S>(v[1][q]);
    t.z = encode<S>(v[2][q]);
    t.w = encode<S>(v[3][q]);
    buf_store_v<V4, NT>(t, d, x0, uint32_t(q) * pq);
  }
}

// Closure on, FP32 compute (FP32, FP16 and BF16 storage): the schedule of
// k_fused_les, written for the buffer addressing above.  A workgroup of W + 64
// lanes owns the columns x0 .. x0+W-1 (W a multiple of 64, so every wave
// stores whole aligned cache lines) and marches up the rows y0 .. y1-1; the
// moment fields of rows y-1 .. y+2 live in a 4-slot LDS ring indexed by
// column - x0 + 1.  Per row a collision lane issues the loads of row y + 2,
// collides and stores row y from the ring, puts row y + 2's moments into the
// ring and meets the others at the row's barrier (which waits for LDS only).
// The row body has no branch around a memory operation: a lane past the last
// column loads the last column, drops its stores (kDropOffset) and puts its
// moments into a spare ring column (W + 2), so the compiler waits on each
// batch of loads alone; three register sets rotate the rows without copies.
// The last wave gathers the two halo columns (x0 - 1 and the column after the
// strip's last cell) two rows ahead, in a loop of its own with the same
// barrier per row.  Results are those of k_fused_les (same expressions).
template <typename S, int W, int STENCIL, bool NT, int MODE, int QG>
__global__ void __launch_bounds__(W + 64)
k_fused_les_f(const S* __restrict__ src, S* __restrict__ dst, int nx, int ny, int64_t pitch, int ry, Rates<float> r,
              const float* __restrict__ corr) {
  using C = float;
  constexpr int NF = MODE == kClosureFull ? 5 : 4;
  constexpr int NP = kPop<QG>;
  __shared__ C ring[4][NF][W + 3];
  const int tid = threadIdx.x;
  const int nstrip = (nx + W - 1) / W;
  const int vb = xcd_contiguous(blockIdx.x, gridDim.x);  // strip vb % nstrip of segment vb / nstrip
  const int x0 = (vb % nstrip) * W;
  const int last = min(x0 + W, nx) - 1;  // last column of this strip
  const int y0 = (vb / nstrip) * ry;
  const int y1 = min(y0 + ry, ny);
  const uint32_t pq = uint32_t(pitch) * uint32_t(sizeof(S));  // bytes between population rows
  const uint32_t rowb = uint32_t(NP) * pq;                    // bytes of a lattice row
  auto wrapy = [&](int y) { return y < 0 ? y + ny : (y >= ny ? y - ny : y); };
  auto slot = [&](int y) { return (y - y0 + 1) & 3; };  // ring slot of row y
  auto pull = [&](int y, const Cols& cx, RawCell<S, QG>& c) __attribute__((always_inline)) {
    pull_raw<S, QG>(src, pq, wrapy(y - 1), y, wrapy(y + 1), cx, c);
  };
  auto put = [&](int sl, int widx, const RawCell<S, QG>& c) __attribute__((always_inline)) {
    C v[NP];
    decode_raw<S, C, QG>(c, v);
    const Mom<C> m = moments_of<QG>(v);
    ring[sl][0][widx] = m.mx;
    ring[sl][1][widx] = m.my;
    ring[sl][2][widx] = m.dbx;
    ring[sl][3][widx] = m.dby;
    if constexpr (NF == 5) ring[sl][4][widx] = m.drho;
  };

  if (tid >= W) {
    // halo wave: lane 0 gathers the column left of the strip, the others the
    // column right of it (only lanes 0 and 1 put theirs into the ring)
    const int hl = tid - W;
    const int xc = hl == 0 ? (x0 == 0 ? nx - 1 : x0 - 1) : (last + 1 == nx ? 0 : last + 1);
    const int widx = hl == 0 ? 0 : (hl == 1 ? last - x0 + 2 : W + 2);
    const Cols cx = cols_of<S>(xc, nx);
    auto ahead = [&](int y) { return wrapy(y <= y1 ? y : y1); };  // rows past y1 are not needed
    RawCell<S, QG> ca, cb;
    pull(wrapy(y0 - 1), cx, ca);
    put(0, widx, ca);
    pull(y0, cx, ca);
    put(1, widx, ca);
    pull(wrapy(y0 + 1), cx, ca);
    put(2, widx, ca);
    pull(ahead(y0 + 2), cx, ca);
    __syncthreads();
    int y = y0;
    for (; y + 2 <= y1; y += 2) {  // rows y, y + 1: put rows y + 2 and y + 3
      pull(ahead(y + 3), cx, cb);
      put(slot(y + 2), widx, ca);
      __syncthreads();
      pull(ahead(y + 4), cx, ca);
      if (y + 3 <= y1) put(slot(y + 3), widx, cb);
      __syncthreads();
    }
    if (y < y1) __syncthreads();  // row y1 - 1 needs no further row
    return;
  }

  const bool valid = x0 + tid <= last;
  const int xc = valid ? x0 + tid : last;  // idle lanes address a valid cell, never stored
  const Cols cx = cols_of<S>(xc, nx);
  const int widx = valid ? tid + 1 : W + 2;
  const uint32_t xo_store = valid ? cx.c : kDropOffset;
  const int64_t n = (int64_t)nx * ny;
  float cc[4] = {0.0f, 0.0f, 0.0f, 0.0f}, cn[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  auto load_corr = [&](int y, float (&c)[4]) __attribute__((always_inline)) {
    const int64_t ci = (int64_t)y * nx + xc;
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = corr[k * n + ci];
  };

  // Row y: rcur holds it as stored, rt receives row y + 2 (row y + 1 again
  // for the segment's last row, whose ring slot is then never read).
  auto row = [&](const RawCell<S, QG>& rcur, RawCell<S, QG>& rt, int y) __attribute__((always_inline)) {
    const bool more = y + 1 < y1;
    pull(wrapy(more ? y + 2 : y + 1), cx, rt);
    if constexpr (MODE == kClosureCorr) load_corr(more ? y + 1 : y, cn);
    // the loads stay ahead of the collision (the scheduler would otherwise
    // sink them to their use to save registers)
    __builtin_amdgcn_sched_barrier(0);
    const int sc = slot(y), sn = slot(y + 1), ss = slot(y - 1), l = tid + 1;
    C gr[NF][2];
#pragma unroll
    for (int k = 0; k < NF; ++k)
      grad3x3<C, STENCIL>(ring[sc][k][l + 1], ring[sc][k][l - 1], ring[sn][k][l], ring[ss][k][l], ring[sn][k][l + 1],
                          ring[sn][k][l - 1], ring[ss][k][l + 1], ring[ss][k][l - 1], gr[k][0], gr[k][1]);
    C cur[NP];
    decode_raw<S, C, QG>(rcur, cur);
    const Mom<C> m = moments_of<QG>(cur);
    const C ir = C(1) / (r.rho0 + m.drho);
    Closure<C> cl;
    if constexpr (MODE == kClosureFull) {
      cl = closure_terms_full(gr, m.mx, m.my, r.bx0 + m.dbx, r.by0 + m.dby, ir, r.k2);
    } else {
      if constexpr (STENCIL >= LBM_STENCIL_LOCAL_ISO9 && QG == 5)
        local_gradients(cur, m, r, gr[1][0] - gr[0][1], gr);
      cl = closure_terms(gr[0][0], gr[0][1], gr[1][0], gr[1][1], gr[2][0], gr[2][1], gr[3][0], gr[3][1], ir, r.k2);
    }
    if constexpr (MODE == kClosureCorr) {
      cl.tau_xy += cc[1];
      cl.tau_d += cc[0] - cc[2];
      cl.tau_s += cc[0] + cc[2];
      cl.eps += cc[3];
    }
    collide_q<QG>(cur, m, cl, r);
    const __amdgpu_buffer_rsrc_t d = row_rsrc(reinterpret_cast<char*>(dst) + int64_t(y) * rowb, rowb);
#pragma unroll
    for (int q = 0; q < NP; ++q) buf_store<S, NT>(encode<S>(cur[q]), d, xo_store, uint32_t(q) * pq);
    __builtin_amdgcn_sched_barrier(0);
    put(slot(y + 2), widx, rt);
    if constexpr (MODE == kClosureCorr) {
#pragma unroll
      for (int k = 0; k < 4; ++k) cc[k] = cn[k];
    }
    __syncthreads();
  };

  RawCell<S, QG> ra, rb, rc;
  pull(wrapy(y0 - 1), cx, ra);
  put(0, widx, ra);
  pull(y0, cx, rb);
  put(1, widx, rb);
  pull(wrapy(y0 + 1), cx, rc);
  put(2, widx, rc);
  if constexpr (MODE == kClosureCorr) load_corr(y0, cc);
  __syncthreads();
  int y = y0;
  for (; y + 3 <= y1; y += 3) {  // one straight-line block of three rows
    row(rb, ra, y);
    row(rc, rb, y + 1);
    row(ra, rc, y + 2);
  }
  if (y < y1) row(rb, ra, y);
  if (y + 1 < y1) row(rc, rb, y + 1);
}

// ---------------------------------------------------------------------------
// AA schedule (one buffer, in place).
//  even t: load A[q][x],             store f*_q to A[opp q][x]
//  odd  t: load A[opp q][x - c_q],   store f*_q to A[q][x + c_q]
// Every kernel of the schedule runs one row segment of kAARow cells per
// workgroup (1-D row blocks keep each wave's accesses within DRAM rows;
// measured 1.1-1.25x faster than 64 x 4 tiles at 4096^2) and addresses a
// population row by its wave-uniform base plus a 32-bit byte offset.
// ---------------------------------------------------------------------------
constexpr int kAARow = 256;

// Row segment x0 .. x0 + kAARow - 1 of row y for this workgroup, from a
// one-dimensional grid numbered XCD-contiguously.
__device__ __forceinline__ void aa_segment(int nx, int& x0, int& y) {
  const int nseg = (nx + kAARow - 1) / kAARow;
  const int vb = xcd_contiguous(blockIdx.x, gridDim.x);
  x0 = (vb % nseg) * kAARow;
  y = vb / nseg;
}

template <typename S, typename C, bool ODD>
__device__ __forceinline__ void aa_load(const S* __restrict__ A, int64_t pitch, const Rows& rw, const Cols& cl,
                                        C v[kQ]) {
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    if (!ODD) {
      v[q] = decode<C>(*at(A + q * pitch, rw.c, cl.c));
    } else {
      const uint32_t xo = qcx(q) > 0 ? cl.w : (qcx(q) < 0 ? cl.e : cl.c);  // x - c_q
      const int64_t yo = qcy(q) > 0 ? rw.s : (qcy(q) < 0 ? rw.n : rw.c);
      v[q] = decode<C>(*at(A + qopp(q) * pitch, yo, xo));
    }
  }
}

template <typename S, typename C, bool ODD>
__device__ __forceinline__ void aa_store(S* __restrict__ A, int64_t pitch, const Rows& rw, const Cols& cl,
                                         const C v[kQ]) {
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    if (!ODD) {
      *at(A + qopp(q) * pitch, rw.c, cl.c) = encode<S>(v[q]);
    } else {
      const uint32_t xo = qcx(q) > 0 ? cl.e : (qcx(q) < 0 ? cl.w : cl.c);  // x + c_q
      const int64_t yo = qcy(q) > 0 ? rw.n : (qcy(q) < 0 ? rw.s : rw.c);
      *at(A + q * pitch, yo, xo) = encode<S>(v[q]);
    }
  }
}

template <typename S, typename C, bool ODD>
__global__ void __launch_bounds__(kAARow) k_aa_dns(S* __restrict__ A, int nx, int ny, int64_t pitch, Rates<C> r) {
  int x0, y;
  aa_segment(nx, x0, y);
  const int x = x0 + threadIdx.x;
  if (x >= nx) return;
  const Rows rw = rows_of<S>(y, ny, pitch);
  const Cols cl = cols_of<S>(x, nx);
  C v[kQ];
  aa_load<S, C, ODD>(A, pitch, rw, cl, v);
  const Mom<C> m = moments19(v);
  const Closure<C> zero = {C(0), C(0), C(0), C(0)};
  collide19(v, m, zero, r);
  aa_store<S, C, ODD>(A, pitch, rw, cl, v);
}

// Moment sweep of the in-place closure schedule: m_x, m_y, B_x, B_y of the
// state at time t into four dense planes of the compute type.
template <typename S, typename C, bool ODD>
__global__ void __launch_bounds__(kAARow)
k_aa_moments(const S* __restrict__ A, C* __restrict__ mb, int nx, int ny, int64_t pitch) {
  int x0, y;
  aa_segment(nx, x0, y);
  const int x = x0 + threadIdx.x;
  if (x >= nx) return;
  const Rows rw = rows_of<S>(y, ny, pitch);
  const Cols cl = cols_of<S>(x, nx);
  C v[kQ];
  aa_load<S, C, ODD>(A, pitch, rw, cl, v);
  const Mom<C> m = moments19(v);
  const int64_t n = (int64_t)nx * ny, c0 = (int64_t)y * nx + x;
  mb[c0] = m.mx;
  mb[n + c0] = m.my;
  mb[2 * n + c0] = m.dbx;
  mb[3 * n + c0] = m.dby;
}

// The (kAARow + 2) x 3 halo tile of four moment planes (rows y - 1 .. y + 1)
// for the gradient stencil of one row segment.  Columns beyond the first halo
// column of a ragged last segment are not needed and not loaded.
template <typename C>
__device__ __forceinline__ void stage_tile(C (&tile)[4][3][kAARow + 2], const C* __restrict__ mb, int nx, int ny,
                                           int x0, int y) {
  const int64_t n = (int64_t)nx * ny;
  for (int idx = threadIdx.x; idx < 3 * (kAARow + 2); idx += kAARow) {
    const int ly = idx / (kAARow + 2), lx = idx - ly * (kAARow + 2);
    const int gx0 = x0 + lx - 1;
    if (gx0 > nx) continue;
    const int gx = gx0 < 0 ? gx0 + nx : (gx0 == nx ? 0 : gx0);
    const int gy = wrap1(y + ly - 1, ny);
    const int64_t c = (int64_t)gy * nx + gx;
#pragma unroll
    for (int k = 0; k < 4; ++k) tile[k][ly][lx] = mb[k * n + c];
  }
}

template <typename C, int STENCIL>
__device__ __forceinline__ void tile_gradients(const C (&tile)[4][3][kAARow + 2], int lx, C gr[4][2]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    grad3x3<C, STENCIL>(tile[k][1][lx + 1], tile[k][1][lx - 1], tile[k][2][lx], tile[k][0][lx], tile[k][2][lx + 1],
                        tile[k][2][lx - 1], tile[k][0][lx + 1], tile[k][0][lx - 1], gr[k][0], gr[k][1]);
  }
}

// Collide sweep of the in-place closure schedule (synchronous gradients of
// the moment planes written by k_aa_moments).
template <typename S, typename C, bool ODD, int STENCIL>
__global__ void __launch_bounds__(kAARow)
k_aa_les(S* __restrict__ A, const C* __restrict__ mb, int nx, int ny, int64_t pitch, Rates<C> r) {
  __shared__ C tile[4][3][kAARow + 2];
  int x0, y;
  aa_segment(nx, x0, y);
  stage_tile(tile, mb, nx, ny, x0, y);
  __syncthreads();
  const int x = x0 + threadIdx.x;
  if (x >= nx) return;
  const Rows rw = rows_of<S>(y, ny, pitch);
  const Cols cl = cols_of<S>(x, nx);
  C v[kQ];
  aa_load<S, C, ODD>(A, pitch, rw, cl, v);
  const Mom<C> m = moments19(v);
  C gr[4][2];
  tile_gradients<C, STENCIL>(tile, threadIdx.x + 1, gr);
  const C ir = C(1) / (r.rho0 + m.drho);
  if constexpr (STENCIL >= LBM_STENCIL_LOCAL_ISO9) local_gradients(v, m, r, gr[1][0] - gr[0][1], gr);
  const Closure<C> cls = closure_terms(gr[0][0], gr[0][1], gr[1][0], gr[1][1], gr[2][0], gr[2][1], gr[3][0],
                                       gr[3][1], ir, r.k2);
  collide19(v, m, cls, r);
  aa_store<S, C, ODD>(A, pitch, rw, cl, v);
}

// Single-sweep in-place closure schedule (lagged gradients): the halo tile
// comes from the previous step's moment planes mb_prev, while the cell's own
// moments go to mb_next for the next step.  19 + 4 values read, 19 + 4
// written per cell.
template <typename S, typename C, bool ODD, int STENCIL>
__global__ void __launch_bounds__(kAARow)
k_aa_les_lagged(S* __restrict__ A, const C* __restrict__ mb_prev, C* __restrict__ mb_next, int nx, int ny,
                int64_t pitch, Rates<C> r) {
  __shared__ C tile[4][3][kAARow + 2];
  int x0, y;
  aa_segment(nx, x0, y);
  stage_tile(tile, mb_prev, nx, ny, x0, y);
  __syncthreads();
  const int x = x0 + threadIdx.x;
  if (x >= nx) return;
  const Rows rw = rows_of<S>(y, ny, pitch);
  const Cols cl = cols_of<S>(x, nx);
  C v[kQ];
  aa_load<S, C, ODD>(A, pitch, rw, cl, v);
  const Mom<C> m = moments19(v);
  const int64_t n = (int64_t)nx * ny, c0 = (int64_t)y * nx + x;
  mb_next[c0] = m.mx;
  mb_next[n + c0] = m.my;
  mb_next[2 * n + c0] = m.dbx;
  mb_next[3 * n + c0] = m.dby;
  C gr[4][2];
  tile_gradients<C, STENCIL>(tile, threadIdx.x + 1, gr);
  const C ir = C(1) / (r.rho0 + m.drho);
  const Closure<C> cls = closure_terms(gr[0][0], gr[0][1], gr[1][0], gr[1][1], gr[2][0], gr[2][1], gr[3][0],
                                       gr[3][1], ir, r.k2);
  collide19(v, m, cls, r);
  aa_store<S, C, ODD>(A, pitch, rw, cl, v);
}

// ---------------------------------------------------------------------------
// Natural-layout access for initial state, state IO, moments and diagnostics.
// `base` is the buffer holding the state at time t and `layout` says where
// population q of cell x sits in it:
//   kLayoutNatural: slot q of cell x                (AA buffer, even t)
//   kLayoutAAOdd:   slot opp(q) of cell x - c_q     (AA buffer, odd t)
//   kLayoutPull:    slot q of cell x - c_q          (fused buffers, any t)
// ---------------------------------------------------------------------------
constexpr int kLayoutNatural = 0;
constexpr int kLayoutAAOdd = 1;
constexpr int kLayoutPull = 2;

template <int QG = 5>
__device__ __forceinline__ int64_t natural_index(int q, int x, int y, int nx, int ny, int64_t pitch, int layout) {
  if (layout == kLayoutNatural) return ((int64_t)y * kPop<QG> + q) * pitch + x;
  const int xs = wrap1(x - qcx<QG>(q), nx), ys = wrap1(y - qcy<QG>(q), ny);
  return ((int64_t)ys * kPop<QG> + (layout == kLayoutAAOdd ? qopp<QG>(q) : q)) * pitch + xs;
}

// Rest values subtracted from the stored populations: w_q rho0 for f,
// w'_i B_ref for g (all zero for FP64 storage).
struct RestRef {
  double rho0, bx0, by0;
};

template <int QG = 5>
__device__ __forceinline__ double rest_value(int q, const RestRef& ref) {
  return q < 9 ? w9(q) * ref.rho0 : (q < 9 + QG ? wg<QG>(q - 9) * ref.bx0 : wg<QG>(q - 9 - QG) * ref.by0);
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output number counter + 1 of
// the sequence started at `seed`.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Unfiltered equilibria feq / geq (Sec. 2) of one cell's fields, evaluated in
// FP64 and rounded to the storage type.
template <typename S, int QG = 5>
__device__ __forceinline__ void write_equilibrium(S* __restrict__ base, int x, int y, int nx, int ny, int64_t pitch,
                                                  int layout, const RestRef& ref, double rho, double ux, double uy,
                                                  double bx, double by) {
  const double usq = ux * ux + uy * uy, bsq = bx * bx + by * by;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double cu = cx9(i) * ux + cy9(i) * uy;
    const double cb = cx9(i) * bx + cy9(i) * by;
    const double c2 = double(cx9(i) * cx9(i) + cy9(i) * cy9(i));
    const double feq = w9(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq) + 4.5 * w9(i) * (0.5 * bsq * c2 - cb * cb);
    base[natural_index<QG>(i, x, y, nx, ny, pitch, layout)] = encode<S>(feq - rest_value<QG>(i, ref));
  }
#pragma unroll
  for (int i = 0; i < QG; ++i) {
    const double cu = cx9(i) * ux + cy9(i) * uy;
    const double cb = cx9(i) * bx + cy9(i) * by;
    const double gx = wg<QG>(i) * (bx + 3.0 * (cu * bx - cb * ux));
    const double gy = wg<QG>(i) * (by + 3.0 * (cu * by - cb * uy));
    base[natural_index<QG>(9 + i, x, y, nx, ny, pitch, layout)] = encode<S>(gx - rest_value<QG>(9 + i, ref));
    base[natural_index<QG>(9 + QG + i, x, y, nx, ny, pitch, layout)] =
        encode<S>(gy - rest_value<QG>(9 + QG + i, ref));
  }
}

// Kelvin-Helmholtz double shear layer at the unfiltered equilibria.
template <typename S, int QG>
__global__ void __launch_bounds__(256)
k_init_kh(S* __restrict__ base, int nx, int ny, int64_t pitch, int layout, RestRef ref, lbm_kh_params kh) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const double L = double(ny), d = kh.delta_over_L * L;
  const double yy = double(y), xx = double(x);
  const double ux = kh.U0 * (tanh((yy - 0.25 * L) / d) - tanh((yy - 0.75 * L) / d) - 1.0);
  const uint64_t z = splitmix64_at(kh.seed, (uint64_t)y * (uint64_t)nx + (uint64_t)x);
  const double xi = 2.0 * (double(z >> 11) * 0x1.0p-53) - 1.0;
  const double uy = kh.pert_amp_over_U0 * kh.U0 * sin(2.0 * M_PI * xx / double(nx)) + kh.noise_amp * xi;
  write_equilibrium<S, QG>(base, x, y, nx, ny, pitch, layout, ref, kh.rho0, ux, uy, kh.B0, 0.0);
}

// The magnetized jet of Sec. 4 at the unfiltered equilibria.
template <typename S, int QG>
__global__ void __launch_bounds__(256)
k_init_sech2(S* __restrict__ base, int nx, int ny, int64_t pitch, int layout, RestRef ref, lbm_sech2_params jet) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const double xf = double(x), yf = double(y), d = fmin(xf, double(nx) - xf);
  const double kx = 2.0 * M_PI * double(jet.k) / double(nx), ky = 2.0 * M_PI * double(jet.k) / double(ny);
  const double ch = cosh(kx * d);
  const double uy = jet.U0 / (ch * ch) + jet.pert * jet.U0 * sin(kx * xf);
  const double ux = jet.pert * jet.U0 * sin(ky * yf);
  const double bx = jet.pert * jet.B0 * sin(ky * yf);
  const double by = jet.B0 + jet.pert * jet.B0 * sin(kx * xf);
  write_equilibrium<S, QG>(base, x, y, nx, ny, pitch, layout, ref, jet.rho0, ux, uy, bx, by);
}

// Equilibria of given fields: 5 FP64 planes rho, m_x, m_y, B_x, B_y.
template <typename S, int QG>
__global__ void __launch_bounds__(256)
k_init_moments(S* __restrict__ base, const double* __restrict__ mom, int nx, int ny, int64_t pitch, int layout,
               RestRef ref) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const int64_t n = (int64_t)nx * ny, c = (int64_t)y * nx + x;
  const double rho = mom[c];
  write_equilibrium<S, QG>(base, x, y, nx, ny, pitch, layout, ref, rho, mom[n + c] / rho, mom[2 * n + c] / rho,
                       mom[3 * n + c], mom[4 * n + c]);
}

template <typename S, int QG>
__global__ void __launch_bounds__(256)
k_get_state(const S* __restrict__ base, double* __restrict__ out, int nx, int ny, int64_t pitch, int layout,
            RestRef ref) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const int64_t n = (int64_t)nx * ny, c0 = (int64_t)y * nx + x;
#pragma unroll
  for (int q = 0; q < kPop<QG>; ++q) {
    const double v = decode<double>(base[natural_index<QG>(q, x, y, nx, ny, pitch, layout)]);
    out[q * n + c0] = v + rest_value<QG>(q, ref);
  }
}

template <typename S, int QG>
__global__ void __launch_bounds__(256)
k_set_state(S* __restrict__ base, const double* __restrict__ in, int nx, int ny, int64_t pitch, int layout,
            RestRef ref) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const int64_t n = (int64_t)nx * ny, c0 = (int64_t)y * nx + x;
#pragma unroll
  for (int q = 0; q < kPop<QG>; ++q) {
    const double v = in[q * n + c0];
    base[natural_index<QG>(q, x, y, nx, ny, pitch, layout)] = encode<S>(v - rest_value<QG>(q, ref));
  }
}

// rho, m_x, m_y, B_x, B_y in FP64 (5 dense planes).  With mark_nonfinite,
// rho is set to NaN where any population is NaN or infinite.  256-cell row
// segments (measured 1.2-1.4x faster than 64 x 4 tiles for the moment
// gathers).
template <typename S, int QG>
__global__ void __launch_bounds__(256)
k_moments_out(const S* __restrict__ base, double* __restrict__ out, int nx, int ny, int64_t pitch, int layout,
              RestRef ref, bool mark_nonfinite) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= nx) return;
  double v[kPop<QG>];
  bool finite = true;
#pragma unroll
  for (int q = 0; q < kPop<QG>; ++q) {
    v[q] = decode<double>(base[natural_index<QG>(q, x, y, nx, ny, pitch, layout)]);
    finite = finite && isfinite(v[q]);
  }
  const Mom<double> m = moments_of<QG>(v);
  const int64_t n = (int64_t)nx * ny, c0 = (int64_t)y * nx + x;
  out[c0] = (mark_nonfinite && !finite) ? __builtin_nan("") : ref.rho0 + m.drho;
  out[n + c0] = m.mx;
  out[2 * n + c0] = m.my;
  out[3 * n + c0] = ref.bx0 + m.dbx;
  out[4 * n + c0] = ref.by0 + m.dby;
}

// Input vectors of the learned correction (first stage; the network kernel is
// the second).  For every cell of a fused-schedule state (layout kLayoutPull):
// rho, m, B in FP32 from the gathered populations, u = m / rho, the central-
// difference vorticity and current, the seven fields normalised (FP32) and
// rounded to bfloat16, and the out-of-range flag (CellIn, 16 bytes).  Each
// wave walks its own strip of 64 columns down a segment of kCellInRows rows,
// independently of the other waves (no workgroup barrier): each lane gathers
// one column per row, u_x, u_y, B_x, B_y go to the wave's four-row LDS ring,
// and the row above the newest one is finished from the ring.  The strip's
// outer two columns and the rows just outside the segment are gathered for
// their neighbours only: 62 output columns per strip.  FP64 storage runs this
// kernel; FP32 compute runs k_cell_inputs_f below, whose aligned strips store
// whole lines (16384^2 BF16: 2.73 ms against 2.94 ms for this form, whose
// 62-column strips split the lines they store with their neighbours).
constexpr int kCellInW = 64, kCellInRows = 8;

__host__ __device__ constexpr int cell_input_strips(int nx) { return (nx + kCellInW - 3) / (kCellInW - 2); }

template <typename S>
__global__ void __launch_bounds__(256)
k_cell_inputs(const S* __restrict__ src, int nx, int ny, int64_t pitch, RestRef ref, int nstrips,
              const char* __restrict__ pk, CellIn* __restrict__ out) {
  using C = typename ComputeOf<S>::type;
  __shared__ float ring_all[4][4][4][kCellInW];  // wave, row slot, field (u_x, u_y, B_x, B_y), column
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int strip = blockIdx.x * 4 + wid;
  if (strip >= nstrips) return;
  float(*ring)[4][kCellInW] = ring_all[wid];
  const int xu = strip * (kCellInW - 2) - 1 + lane;  // unwrapped column, >= -1
  const int x = xu < 0 ? nx - 1 : xu % nx;
  const bool out_col = lane >= 1 && lane < kCellInW - 1 && xu < nx;
  const int y0 = blockIdx.y * kCellInRows;
  const int nrow = (y0 + kCellInRows <= ny ? kCellInRows : ny - y0);
  const lbm_mlp_norm* nm = reinterpret_cast<const lbm_mlp_norm*>(pk + kPkNorm);
  const Cols cl = cols_of<S>(x, nx);
  float pr = 0.0f, pux = 0.0f, puy = 0.0f, pbx = 0.0f, pby = 0.0f;  // own column, previous row
  for (int k = 0; k < nrow + 2; ++k) {
    int yk = y0 - 1 + k;
    yk = yk < 0 ? yk + ny : (yk >= ny ? yk - ny : yk);
    C v[kQ];
    pull_cell<S, C, 5>(src, pitch, rows_of<S>(yk, ny, pitch), cl, v);
    const Mom<C> m = moments19(v);
    const float r = float(C(ref.rho0) + m.drho);
    const float ux = float(m.mx) / r, uy = float(m.my) / r;
    const float bx = float(C(ref.bx0) + m.dbx), by = float(C(ref.by0) + m.dby);
    const int sl = k & 3;
    ring[sl][0][lane] = ux;
    ring[sl][1][lane] = uy;
    ring[sl][2][lane] = bx;
    ring[sl][3][lane] = by;
    // the wave's own LDS writes, visible to all its lanes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (k >= 2 && out_col) {
      // row yk - 1 (slot k - 1), between rows yk - 2 and yk
      const int sm = (k - 2) & 3, s0 = (k - 1) & 3;
      const float om = 0.5f * (ring[s0][1][lane + 1] - ring[s0][1][lane - 1]) - 0.5f * (ring[sl][0][lane] - ring[sm][0][lane]);
      const float jz = 0.5f * (ring[s0][3][lane + 1] - ring[s0][3][lane - 1]) - 0.5f * (ring[sl][2][lane] - ring[sm][2][lane]);
      const float f[7] = {pr, pux, puy, pbx, pby, om, jz};
      bool bad = false;
      f32x8 z;
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        z[i] = (f[i] - nm->shift[i]) * nm->scale[i];
        bad = bad || !(fabsf(z[i]) <= kOodLimit);  // NaN counts as out of range
      }
      z[7] = 0.0f;
      u32x4 w = __builtin_bit_cast(u32x4, to_bf16x8(z));
      w[3] = (w[3] & 0xFFFFu) | (bad ? unsigned(kCellOutOfRange) << 16 : 0u);
      out[(int64_t)(y0 + k - 2) * nx + x] = __builtin_bit_cast(CellIn, w);
    }
    pr = r;
    pux = ux;
    puy = uy;
    pbx = bx;
    pby = by;
  }
}

// Input vectors with FP32 compute (FP32, FP16, BF16 storage): the strip
// schedule of k_fused_les_f.  A workgroup of W + 64 lanes owns the columns
// x0 .. x0+W-1 (so each row's input vectors are whole aligned lines) and walks
// the rows y0 .. y1-1.  A lane keeps rho, u, B of the rows y-1, y, y+1 of its
// own column in registers and reads u_y, B_y of its two neighbour columns from
// an LDS row (two slots by row parity, one barrier per row); the last wave
// gathers the two halo columns.  Rows are gathered two ahead of their use with
// buffer loads, three register sets rotate through a three-times unrolled
// loop, and lanes past the strip's last column drop their stores through
// kDropOffset, so the row body has no branch around a memory operation.  The
// arithmetic is k_cell_inputs' (same expressions, same results).
struct CellFields {
  float r, ux, uy, bx, by;
};

template <typename S, int W>
__global__ void __launch_bounds__(W + 64)
k_cell_inputs_f(const S* __restrict__ src, int nx, int ny, int64_t pitch, int ry, RestRef ref,
                const char* __restrict__ pk, CellIn* __restrict__ out) {
  using C = float;
  constexpr int NP = kPop<5>;
  __shared__ float rowbuf[2][2][W + 3];  // row parity, field (u_y, B_y), column - x0 + 1 (W + 2: spare)
  const int tid = threadIdx.x;
  const int nstrip = (nx + W - 1) / W;
  const int vb = xcd_contiguous(blockIdx.x, gridDim.x);  // strip vb % nstrip of segment vb / nstrip
  const int x0 = (vb % nstrip) * W;
  const int last = min(x0 + W, nx) - 1;
  const int y0 = (vb / nstrip) * ry;
  const int y1 = min(y0 + ry, ny);
  const uint32_t pq = uint32_t(pitch) * uint32_t(sizeof(S));
  const lbm_mlp_norm* nm = reinterpret_cast<const lbm_mlp_norm*>(pk + kPkNorm);
  auto wrapy = [&](int y) { return y < 0 ? y + ny : (y >= ny ? y - ny : y); };
  auto ahead = [&](int y) { return wrapy(y <= y1 ? y : y1); };  // rows past y1 are not needed

  const bool halo = tid >= W;
  const int hl = tid - W;
  const bool valid = !halo && x0 + tid <= last;
  const int xc = halo ? (hl == 0 ? (x0 == 0 ? nx - 1 : x0 - 1) : (last + 1 == nx ? 0 : last + 1))
                      : (valid ? x0 + tid : last);
  const int widx = halo ? (hl == 0 ? 0 : (hl == 1 ? last - x0 + 2 : W + 2)) : (valid ? tid + 1 : W + 2);
  const Cols cx = cols_of<S>(xc, nx);
  const uint32_t xo_store = valid ? uint32_t(x0 + tid) * uint32_t(sizeof(CellIn)) : kDropOffset;
  const uint32_t orow = uint32_t(nx) * uint32_t(sizeof(CellIn));

  auto pull = [&](int y, RawCell<S, 5>& c) __attribute__((always_inline)) {
    pull_raw<S, 5>(src, pq, wrapy(y - 1), y, wrapy(y + 1), cx, c);
  };
  auto fields = [&](const RawCell<S, 5>& c, CellFields& f) __attribute__((always_inline)) {
    C v[NP];
    decode_raw<S, C, 5>(c, v);
    const Mom<C> m = moments19(v);
    f.r = float(C(ref.rho0) + m.drho);
    f.ux = float(m.mx) / f.r;
    f.uy = float(m.my) / f.r;
    f.bx = float(C(ref.bx0) + m.dbx);
    f.by = float(C(ref.by0) + m.dby);
  };
  auto share = [&](int y, const CellFields& f) __attribute__((always_inline)) {
    rowbuf[y & 1][0][widx] = f.uy;
    rowbuf[y & 1][1][widx] = f.by;
  };

  // Row y: fm, fc hold rows y - 1 and y, fn receives row y + 1 from rn (loaded
  // two rows ago); rt receives row y + 3.
  auto row = [&](const CellFields& fm, const CellFields& fc, CellFields& fn, const RawCell<S, 5>& rn,
                 RawCell<S, 5>& rt, int y) __attribute__((always_inline)) {
    pull(ahead(y + 3), rt);
    __builtin_amdgcn_sched_barrier(0);
    fields(rn, fn);
    share(y + 1, fn);
    {
      // the halo wave runs the same body on column 1 and drops its stores
      const int l = halo ? 1 : tid + 1;
      const float om = 0.5f * (rowbuf[y & 1][0][l + 1] - rowbuf[y & 1][0][l - 1]) - 0.5f * (fn.ux - fm.ux);
      const float jz = 0.5f * (rowbuf[y & 1][1][l + 1] - rowbuf[y & 1][1][l - 1]) - 0.5f * (fn.bx - fm.bx);
      const float f[7] = {fc.r, fc.ux, fc.uy, fc.bx, fc.by, om, jz};
      bool bad = false;
      f32x8 z;
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        z[i] = (f[i] - nm->shift[i]) * nm->scale[i];
        bad = bad || !(fabsf(z[i]) <= kOodLimit);  // NaN counts as out of range
      }
      z[7] = 0.0f;
      u32x4 w = __builtin_bit_cast(u32x4, to_bf16x8(z));
      w[3] = (w[3] & 0xFFFFu) | (bad ? unsigned(kCellOutOfRange) << 16 : 0u);
      const __amdgpu_buffer_rsrc_t d = row_rsrc(reinterpret_cast<char*>(out) + int64_t(y) * orow, orow);
      // non-temporal: the network kernel reads the vectors back after the
      // whole grid is written (16384^2 learned step 0.5-1 % faster, 1024^2 no slower)
      __builtin_amdgcn_raw_buffer_store_b128(w, d, int(xo_store), 0, 2);
    }
    __syncthreads();
  };

  CellFields fa, fb, fc;
  RawCell<S, 5> ra, rb, rc;
  pull(wrapy(y0 - 1), ra);
  fields(ra, fa);
  pull(y0, rb);
  fields(rb, fb);
  share(y0, fb);
  pull(ahead(y0 + 1), ra);
  pull(ahead(y0 + 2), rb);
  __syncthreads();
  int y = y0;
  for (; y + 3 <= y1; y += 3) {  // one straight-line block of three rows
    row(fa, fb, fc, ra, rc, y);
    row(fb, fc, fa, rb, ra, y + 1);
    row(fc, fa, fb, rc, rb, y + 2);
  }
  if (y < y1) row(fa, fb, fc, ra, rc, y);
  if (y + 1 < y1) row(fb, fc, fa, rb, ra, y + 1);
}

// ---------------------------------------------------------------------------
// Diagnostics: per-cell FP64 terms from the five moment planes, a fixed-order
// grid-stride accumulation per thread, wave and block reductions into one
// partial per workgroup, then a single-workgroup fixed-order final pass.
// Accumulators: 0 mass, 1-2 momentum, 3-4 sum B, 5 kinetic energy, 6 magnetic
// energy, 7 enstrophy, 8 J_z^2, 9 (div B)^2, 10 max |div B|, 11 non-finite.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void diag_combine(double* a, const double* b) {
#pragma unroll
  for (int k = 0; k < kDiagVals; ++k) a[k] = (k == 10) ? fmax(a[k], b[k]) : a[k] + b[k];
}

__device__ void block_reduce_diag(double* acc, double* out) {
  __shared__ double red[4][kDiagVals];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    double o[kDiagVals];
#pragma unroll
    for (int k = 0; k < kDiagVals; ++k) o[k] = __shfl_down(acc[k], off, 64);
    diag_combine(acc, o);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kDiagVals; ++k) red[wid][k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[kDiagVals];
#pragma unroll
    for (int k = 0; k < kDiagVals; ++k) t[k] = red[0][k];
    for (int w = 1; w < 4; ++w) diag_combine(t, red[w]);
#pragma unroll
    for (int k = 0; k < kDiagVals; ++k) out[k] = t[k];
  }
}

__global__ void __launch_bounds__(256)
k_diag_partial(const double* __restrict__ mom, double* __restrict__ partial, int nx, int ny) {
  const int64_t n = (int64_t)nx * ny;
  const double* rho = mom;
  const double* mx = mom + n;
  const double* my = mom + 2 * n;
  const double* bx = mom + 3 * n;
  const double* by = mom + 4 * n;
  double acc[kDiagVals];
#pragma unroll
  for (int k = 0; k < kDiagVals; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
    const int y = int(c / nx), x = int(c - (int64_t)y * nx);
    const int xe = x + 1 == nx ? 0 : x + 1, xw = x == 0 ? nx - 1 : x - 1;
    const int yn = y + 1 == ny ? 0 : y + 1, ys = y == 0 ? ny - 1 : y - 1;
    const int64_t cE = (int64_t)y * nx + xe, cW = (int64_t)y * nx + xw;
    const int64_t cN = (int64_t)yn * nx + x, cS = (int64_t)ys * nx + x;
    const double r = rho[c], mxc = mx[c], myc = my[c], bxc = bx[c], byc = by[c];
    const double uyE = my[cE] / rho[cE], uyW = my[cW] / rho[cW];
    const double uxN = mx[cN] / rho[cN], uxS = mx[cS] / rho[cS];
    const double w = (uyE - uyW) / 2.0 - (uxN - uxS) / 2.0;
    const double jz = (by[cE] - by[cW]) / 2.0 - (bx[cN] - bx[cS]) / 2.0;
    const double dv = (bx[cE] - bx[cW]) / 2.0 + (by[cN] - by[cS]) / 2.0;
    acc[0] += r;
    acc[1] += mxc;
    acc[2] += myc;
    acc[3] += bxc;
    acc[4] += byc;
    acc[5] += 0.5 * (mxc * mxc + myc * myc) / r;
    acc[6] += 0.5 * (bxc * bxc + byc * byc);
    acc[7] += 0.5 * w * w;
    acc[8] += jz * jz;
    acc[9] += dv * dv;
    acc[10] = fmax(acc[10], fabs(dv));
    acc[11] += isfinite(r) ? 0.0 : 1.0;
  }
  block_reduce_diag(acc, partial + (int64_t)blockIdx.x * kDiagVals);
}

__global__ void __launch_bounds__(256) k_diag_final(const double* __restrict__ partial, double* __restrict__ out,
                                                    int nparts) {
  double acc[kDiagVals];
#pragma unroll
  for (int k = 0; k < kDiagVals; ++k) acc[k] = 0.0;
  for (int p = threadIdx.x; p < nparts; p += blockDim.x) diag_combine(acc, partial + (int64_t)p * kDiagVals);
  block_reduce_diag(acc, out);
}

// ---------------------------------------------------------------------------
// Host side: layout and launchers
// ---------------------------------------------------------------------------
size_t storage_bytes(int dtype) {
  return dtype == LBM_FP64 ? 8 : (dtype == LBM_FP32 ? 4 : 2);
}

int64_t row_pitch(int nx) {
  // Population rows padded to a multiple of 64 elements (whole cache lines);
  // no padding at the power-of-two sizes of the benchmarks, where measured
  // paddings of 64 and 256 elements were slower.
  return ((int64_t)nx + 63) / 64 * 64;
}

int64_t buffer_elems(int nx, int ny, int qg) {
  // ny lattice rows of 9 + 2 qg population rows; rounded to 256 elements.
  const int64_t e = (int64_t)ny * (9 + 2 * qg) * row_pitch(nx);
  return (e + 255) / 256 * 256;
}

size_t buffer_offset_bytes(int nx, int ny, int dtype, int qg) {
  // The second buffer of the fused schedule starts 4 KB past a 64 KB boundary
  // after the first.  The closure sweep reads rows of one buffer while it
  // writes rows of the other; measured at 4096^2 and 8192^2 (FP32), offsets
  // that are multiples of 64 KB put both streams on the same memory channels
  // and cost 10-20 % (8192^2: 2164 us against 1757 us at 4 KB past them).
  const size_t one = (size_t)buffer_elems(nx, ny, qg) * storage_bytes(dtype);
  return (one + 65535) / 65536 * 65536 + 4096;
}

size_t state_bytes(int nx, int ny, int dtype, int schedule, int qg) {
  const size_t one = (size_t)buffer_elems(nx, ny, qg) * storage_bytes(dtype);
  return schedule == LBM_SCHED_FUSED ? buffer_offset_bytes(nx, ny, dtype, qg) + one : one;
}

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t work_layout(Launch& L) {
  const size_t n = (size_t)L.nx * (size_t)L.ny;
  const size_t cbytes = L.dtype == LBM_FP64 ? 8 : 4;  // compute type of the moment planes
  size_t off = 0;
  L.off_mb = off;
  if (L.schedule == LBM_SCHED_AA) off += align256(4 * n * cbytes);
  if (L.schedule == LBM_SCHED_AA_LAGGED) off += 2 * align256(4 * n * cbytes);
  L.off_diag = off;
  off += align256(5 * n * sizeof(double));
  const int64_t want = ((int64_t)n + 255) / 256;
  L.diag_blocks = (int)(want < kDiagBlocksMax ? (want < 1 ? 1 : want) : kDiagBlocksMax);
  L.off_part = off;
  off += align256((size_t)L.diag_blocks * kDiagVals * sizeof(double));
  L.off_final = off;
  off += align256(kDiagVals * sizeof(double));
  if (L.learned) {
    L.off_cellin = off;
    off += align256(16 * n);
    L.off_corr = off;
    off += align256(4 * n * sizeof(float));
    L.off_mlp = off;
    off += align256(LBM_MLP_PACKED_BYTES);
  }
  return off;
}

static dim3 tile_grid(int nx, int ny) { return dim3((nx + 63) / 64, (ny + 3) / 4); }

// Magnetic-lattice dispatch: f(std::integral_constant<int, QG>).  The D2Q9
// vector distribution is built for FP64 and FP32 storage (the ABI rejects
// the 16-bit types with it), so 16-bit storage instantiates D2Q5 only.
template <typename S, typename F>
static hipError_t by_lattice(const Launch& L, F&& f) {
  if constexpr (sizeof(S) >= 4) {
    if (L.qg == 9) return f(std::integral_constant<int, 9>{});
  }
  return f(std::integral_constant<int, 5>{});
}
static const dim3 kTile(64, 4);

// Row segments of the in-place schedule's kernels (one-dimensional grid, see
// aa_segment).
static dim3 aa_grid(const Launch& L) { return dim3((L.nx + kAARow - 1) / kAARow * L.ny); }

template <typename S>
static S* buffer_at(const Launch& L, int64_t t) {
  char* base = static_cast<char*>(L.state);
  if (L.schedule == LBM_SCHED_FUSED && (t & 1)) base += buffer_offset_bytes(L.nx, L.ny, L.dtype, L.qg);
  return reinterpret_cast<S*>(base);
}

static RestRef rest_ref(const Launch& L) { return RestRef{L.rho0, L.bref[0], L.bref[1]}; }

static int layout_at(const Launch& L, int64_t t) {
  if (L.schedule == LBM_SCHED_FUSED) return kLayoutPull;
  return (t & 1) ? kLayoutAAOdd : kLayoutNatural;
}

// Moment set k (0 or 1) of the lagged schedule.
template <typename C>
static C* moment_set(const Launch& L, int k) {
  const size_t n = (size_t)L.nx * (size_t)L.ny;
  const size_t stride = (4 * n * sizeof(C) + 255) / 256 * 256;
  return reinterpret_cast<C*>(static_cast<char*>(L.work) + L.off_mb + (size_t)k * stride);
}

// Rows per workgroup of the fused closure kernel.  Measured on MI355X over
// 1024^2 .. 16384^2 (512-lane FP32 strips): one workgroup per compute unit is
// fastest (every strip segment runs concurrently from start to end, and the
// two halo rows re-read per segment are amortised over many rows) as long as
// a segment then holds at most 128 rows (FP32) or 64 rows (FP64); larger
// grids run more, 64-row segments (4096^2: 440 us at 128 rows = one per
// compute unit, 444 us at 64; 8192^2: 1764 us at 64 rows, 1781 us at 512).
static int fused_rows(int nx, int ny, int strip, int cus, int cap) {
  const int64_t strips = (nx + strip - 1) / strip;
  const int64_t blocks = cus / strips > 1 ? cus / strips : 1;  // segments per strip column
  int64_t ry = (ny + blocks - 1) / blocks;
  if (ry > cap) ry = 64;
  return (int)(ry < 1 ? 1 : ry);
}

// Non-temporal stores pay off once the two population buffers no longer fit
// in the 256 MB Infinity Cache; below that the next step re-reads them from it.
static bool streaming_stores(const Launch& L) {
  return 2.0 * double(9 + 2 * L.qg) * double(L.nx) * double(L.ny) * double(storage_bytes(L.dtype)) > 256.0e6;
}

// FP32 compute runs k_fused_les_f, FP64 k_fused_les.
template <typename S, typename C, int W, bool NT, int MODE, int QG, int STENCIL>
static void launch_les_s(const Launch& L, const S* src, S* dst, const Rates<C>& r, const float* corr) {
  // Segments sized for one workgroup per compute unit, two for k_fused_les_f
  // beyond the Infinity Cache (two fit a compute unit; measured 4096^2 FP32
  // 448 against 466 us, 8192^2 within 1 % either way, while the cache-resident
  // 1024^2 sweep prefers one: 28.7 against 31.4 us).
  const int per_cu = (sizeof(C) == 4 && NT) ? 2 : 1;
  const int ry = fused_rows(L.nx, L.ny, W, L.cus * per_cu, sizeof(C) == 4 ? 128 : 64);
  const int strips = (L.nx + W - 1) / W, segs = (L.ny + ry - 1) / ry;
  if constexpr (sizeof(C) == 4)  // one-dimensional grid, numbered XCD-contiguously in the kernel
    hipLaunchKernelGGL((k_fused_les_f<S, W, STENCIL, NT, MODE, QG>), dim3(strips * segs), dim3(W + 64), 0, L.stream,
                       src, dst, L.nx, L.ny, L.pitch, ry, r, corr);
  else
    hipLaunchKernelGGL((k_fused_les<S, C, W, STENCIL, NT, MODE, QG>), dim3(strips, segs), dim3(W + 64), 0, L.stream,
                       src, dst, L.nx, L.ny, L.pitch, ry, r, corr);
}

template <typename S, typename C, int W, bool NT, int MODE, int QG>
static void launch_les_k(const Launch& L, const S* src, S* dst, const Rates<C>& r, const float* corr) {
  // the density-gradient closure and the D2Q9 vector distribution take
  // stencil gradients only
  if constexpr (MODE != kClosureFull && QG == 5) {
    if (L.stencil == LBM_STENCIL_LOCAL_ISO9) {
      launch_les_s<S, C, W, NT, MODE, QG, LBM_STENCIL_LOCAL_ISO9>(L, src, dst, r, corr);
      return;
    }
    if (L.stencil == LBM_STENCIL_LOCAL_CENTRAL5) {
      launch_les_s<S, C, W, NT, MODE, QG, LBM_STENCIL_LOCAL_CENTRAL5>(L, src, dst, r, corr);
      return;
    }
  }
  if (L.stencil == LBM_STENCIL_CENTRAL5)
    launch_les_s<S, C, W, NT, MODE, QG, LBM_STENCIL_CENTRAL5>(L, src, dst, r, corr);
  else
    launch_les_s<S, C, W, NT, MODE, QG, LBM_STENCIL_ISO9>(L, src, dst, r, corr);
}

template <typename S, typename C, int W, bool NT, int QG>
static void launch_les(const Launch& L, const S* src, S* dst, const Rates<C>& r, const float* corr) {
  if constexpr (QG == 5) {  // the learned correction is built for D2Q5
    if (corr) {
      launch_les_k<S, C, W, NT, kClosureCorr, QG>(L, src, dst, r, corr);
      return;
    }
  }
  if (L.full)
    launch_les_k<S, C, W, NT, kClosureFull, QG>(L, src, dst, r, nullptr);
  else
    launch_les_k<S, C, W, NT, kClosurePlain, QG>(L, src, dst, r, nullptr);
}

template <typename S, typename C, bool NT, int QG>
static void launch_fused(const Launch& L, const S* src, S* dst, const Rates<C>& r, const float* corr) {
  if (L.k2 == 0.0 && !corr) {
    if constexpr (sizeof(S) == 2 && QG == 5) {
      if ((L.nx & 3) == 0) {
        hipLaunchKernelGGL((k_fused_dns_quad<S, C, NT>), dim3((L.nx + 255) / 256 * L.ny), dim3(64), 0, L.stream, src,
                           dst, L.nx, L.ny, L.pitch, r);
        return;
      }
    }
    if ((L.nx & 1) == 0)
      hipLaunchKernelGGL((k_fused_dns_pair<S, C, NT, QG>), dim3((L.nx + 255) / 256, L.ny), dim3(128), 0, L.stream,
                         src, dst, L.nx, L.ny, L.pitch, r);
    else
      hipLaunchKernelGGL((k_fused_dns<S, C, NT, QG>), dim3((L.nx + 255) / 256, L.ny), dim3(256), 0, L.stream, src,
                         dst, L.nx, L.ny, L.pitch, r);
    return;
  }
  // Strip width: 512 lanes for wide grids with FP32 compute, 256 otherwise (the
  // LDS ring of a 512-lane FP64 strip would exceed 64 KB), 64 for narrow
  // grids.  Measured with the lattice-row layout and XCD-contiguous numbering:
  // 256-lane strips (two or four workgroups per compute unit) against 512 take
  // 0-10 % longer with FP32 storage at 4096^2 and 8192^2 and 16-18 % longer
  // with FP16 at 8192^2 (with the earlier two-dimensional grids: up to 1.6x).
  if constexpr (sizeof(C) == 4) {
    if (L.nx >= 1024) {
      launch_les<S, C, 512, NT, QG>(L, src, dst, r, corr);
      return;
    }
  }
  if (L.nx >= 256)
    launch_les<S, C, 256, NT, QG>(L, src, dst, r, corr);
  else
    launch_les<S, C, 64, NT, QG>(L, src, dst, r, corr);
}

template <typename S>
// The learned closure runs in the fused schedule only (checked at creation),
// so the state is always in the pull layout here.
static hipError_t cell_inputs_typed(const Launch& L, int64_t t, CellIn* out) {
  if (layout_at(L, t) != kLayoutPull) return hipErrorInvalidValue;
  const char* pk = static_cast<const char*>(L.work) + L.off_mlp;
  if constexpr (sizeof(typename ComputeOf<S>::type) == 4) {
    const int W = L.nx >= 1024 ? 512 : (L.nx >= 256 ? 256 : 64);
    const int ry = fused_rows(L.nx, L.ny, W, L.cus, 128);
    const dim3 g(((L.nx + W - 1) / W) * ((L.ny + ry - 1) / ry));  // numbered XCD-contiguously in the kernel
    if (W == 512)
      hipLaunchKernelGGL((k_cell_inputs_f<S, 512>), g, dim3(512 + 64), 0, L.stream, buffer_at<S>(L, t), L.nx, L.ny,
                         L.pitch, ry, rest_ref(L), pk, out);
    else if (W == 256)
      hipLaunchKernelGGL((k_cell_inputs_f<S, 256>), g, dim3(256 + 64), 0, L.stream, buffer_at<S>(L, t), L.nx, L.ny,
                         L.pitch, ry, rest_ref(L), pk, out);
    else
      hipLaunchKernelGGL((k_cell_inputs_f<S, 64>), g, dim3(64 + 64), 0, L.stream, buffer_at<S>(L, t), L.nx, L.ny,
                         L.pitch, ry, rest_ref(L), pk, out);
  } else {
    const int strips = cell_input_strips(L.nx);
    hipLaunchKernelGGL((k_cell_inputs<S>), dim3((strips + 3) / 4, (L.ny + kCellInRows - 1) / kCellInRows),
                       dim3(256), 0, L.stream, buffer_at<S>(L, t), L.nx, L.ny, L.pitch, rest_ref(L), strips, pk, out);
  }
  return hipGetLastError();
}

hipError_t launch_correction(const Launch& L, int64_t t, float* out) {
  CellIn* in = reinterpret_cast<CellIn*>(static_cast<char*>(L.work) + L.off_cellin);
  hipError_t e;
  switch (L.dtype) {
    case LBM_FP64: e = cell_inputs_typed<double>(L, t, in); break;
    case LBM_FP32: e = cell_inputs_typed<float>(L, t, in); break;
    case LBM_FP16: e = cell_inputs_typed<_Float16>(L, t, in); break;
    default: e = cell_inputs_typed<__bf16>(L, t, in); break;
  }
  if (e != hipSuccess) return e;
  return launch_mlp_correct(in, static_cast<char*>(L.work) + L.off_mlp, out, L.nx, L.ny, L.stream);
}

template <typename S, typename C, int STENCIL>
static void launch_aa_les(const Launch& L, S* A, const C* mb, const Rates<C>& r, bool odd) {
  if (odd)
    hipLaunchKernelGGL((k_aa_les<S, C, true, STENCIL>), aa_grid(L), dim3(kAARow), 0, L.stream, A, mb, L.nx, L.ny,
                       L.pitch, r);
  else
    hipLaunchKernelGGL((k_aa_les<S, C, false, STENCIL>), aa_grid(L), dim3(kAARow), 0, L.stream, A, mb, L.nx,
                       L.ny, L.pitch, r);
}

template <typename S>
static hipError_t step_typed(const Launch& L, int64_t t, bool corr_refresh) {
  using C = typename ComputeOf<S>::type;
  const Rates<C> r = make_rates<C>(L);
  const dim3 grid = aa_grid(L);
  const bool les = L.k2 != 0.0;
  if (L.schedule == LBM_SCHED_FUSED) {
    const S* src = buffer_at<S>(L, t);
    S* dst = buffer_at<S>(L, t + 1);
    const float* corr = nullptr;
    if (L.learned) {
      float* c = reinterpret_cast<float*>(static_cast<char*>(L.work) + L.off_corr);
      if (corr_refresh) {
        const hipError_t e = launch_correction(L, t, c);
        if (e != hipSuccess) return e;
      }
      corr = c;
    }
    return by_lattice<S>(L, [&](auto qg) {
      constexpr int QG = decltype(qg)::value;
      if (streaming_stores(L))
        launch_fused<S, C, true, QG>(L, src, dst, r, corr);
      else
        launch_fused<S, C, false, QG>(L, src, dst, r, corr);
      return hipGetLastError();
    });
  }
  S* A = static_cast<S*>(L.state);
  const bool odd = t & 1;
  if (les && L.schedule == LBM_SCHED_AA_LAGGED) {
    const C* prev = moment_set<C>(L, int(t & 1));
    C* next = moment_set<C>(L, int((t + 1) & 1));
    if (L.stencil == LBM_STENCIL_ISO9) {
      if (odd)
        hipLaunchKernelGGL((k_aa_les_lagged<S, C, true, LBM_STENCIL_ISO9>), grid, dim3(kAARow), 0, L.stream, A, prev, next,
                           L.nx, L.ny, L.pitch, r);
      else
        hipLaunchKernelGGL((k_aa_les_lagged<S, C, false, LBM_STENCIL_ISO9>), grid, dim3(kAARow), 0, L.stream, A, prev, next,
                           L.nx, L.ny, L.pitch, r);
    } else {
      if (odd)
        hipLaunchKernelGGL((k_aa_les_lagged<S, C, true, LBM_STENCIL_CENTRAL5>), grid, dim3(kAARow), 0, L.stream, A, prev,
                           next, L.nx, L.ny, L.pitch, r);
      else
        hipLaunchKernelGGL((k_aa_les_lagged<S, C, false, LBM_STENCIL_CENTRAL5>), grid, dim3(kAARow), 0, L.stream, A, prev,
                           next, L.nx, L.ny, L.pitch, r);
    }
    return hipGetLastError();
  }
  if (!les) {
    if (odd)
      hipLaunchKernelGGL((k_aa_dns<S, C, true>), grid, dim3(kAARow), 0, L.stream, A, L.nx, L.ny, L.pitch, r);
    else
      hipLaunchKernelGGL((k_aa_dns<S, C, false>), grid, dim3(kAARow), 0, L.stream, A, L.nx, L.ny, L.pitch, r);
    return hipGetLastError();
  }
  C* mb = reinterpret_cast<C*>(static_cast<char*>(L.work) + L.off_mb);
  if (odd)
    hipLaunchKernelGGL((k_aa_moments<S, C, true>), grid, dim3(kAARow), 0, L.stream, A, mb, L.nx, L.ny, L.pitch);
  else
    hipLaunchKernelGGL((k_aa_moments<S, C, false>), grid, dim3(kAARow), 0, L.stream, A, mb, L.nx, L.ny, L.pitch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (L.stencil) {
    case LBM_STENCIL_ISO9: launch_aa_les<S, C, LBM_STENCIL_ISO9>(L, A, mb, r, odd); break;
    case LBM_STENCIL_CENTRAL5: launch_aa_les<S, C, LBM_STENCIL_CENTRAL5>(L, A, mb, r, odd); break;
    case LBM_STENCIL_LOCAL_ISO9: launch_aa_les<S, C, LBM_STENCIL_LOCAL_ISO9>(L, A, mb, r, odd); break;
    default: launch_aa_les<S, C, LBM_STENCIL_LOCAL_CENTRAL5>(L, A, mb, r, odd);
  }
  return hipGetLastError();
}

template <typename S>
static hipError_t lag_prime_typed(const Launch& L, int64_t t) {
  using C = typename ComputeOf<S>::type;
  S* A = static_cast<S*>(L.state);
  C* mb = moment_set<C>(L, int(t & 1));
  if (t & 1)
    hipLaunchKernelGGL((k_aa_moments<S, C, true>), aa_grid(L), dim3(kAARow), 0, L.stream, A, mb, L.nx, L.ny,
                       L.pitch);
  else
    hipLaunchKernelGGL((k_aa_moments<S, C, false>), aa_grid(L), dim3(kAARow), 0, L.stream, A, mb, L.nx, L.ny,
                       L.pitch);
  return hipGetLastError();
}

hipError_t launch_lag_prime(const Launch& L, int64_t t) {
  switch (L.dtype) {
    case LBM_FP64: return lag_prime_typed<double>(L, t);
    case LBM_FP32: return lag_prime_typed<float>(L, t);
    case LBM_FP16: return lag_prime_typed<_Float16>(L, t);
    default: return lag_prime_typed<__bf16>(L, t);
  }
}

hipError_t launch_step(const Launch& L, int64_t t, bool corr_refresh) {
  switch (L.dtype) {
    case LBM_FP64: return step_typed<double>(L, t, corr_refresh);
    case LBM_FP32: return step_typed<float>(L, t, corr_refresh);
    case LBM_FP16: return step_typed<_Float16>(L, t, corr_refresh);
    default: return step_typed<__bf16>(L, t, corr_refresh);
  }
}

template <typename S>
static hipError_t init_typed(const Launch& L, const lbm_kh_params& kh) {
  return by_lattice<S>(L, [&](auto qg) {
    hipLaunchKernelGGL((k_init_kh<S, decltype(qg)::value>), tile_grid(L.nx, L.ny), kTile, 0, L.stream,
                       buffer_at<S>(L, 0), L.nx, L.ny, L.pitch, layout_at(L, 0), rest_ref(L), kh);
    return hipGetLastError();
  });
}

hipError_t launch_init_kh(const Launch& L, const lbm_kh_params& kh) {
  switch (L.dtype) {
    case LBM_FP64: return init_typed<double>(L, kh);
    case LBM_FP32: return init_typed<float>(L, kh);
    case LBM_FP16: return init_typed<_Float16>(L, kh);
    default: return init_typed<__bf16>(L, kh);
  }
}

template <typename S>
static hipError_t init_sech2_typed(const Launch& L, const lbm_sech2_params& jet) {
  return by_lattice<S>(L, [&](auto qg) {
    hipLaunchKernelGGL((k_init_sech2<S, decltype(qg)::value>), tile_grid(L.nx, L.ny), kTile, 0, L.stream,
                       buffer_at<S>(L, 0), L.nx, L.ny, L.pitch, layout_at(L, 0), rest_ref(L), jet);
    return hipGetLastError();
  });
}

hipError_t launch_init_sech2(const Launch& L, const lbm_sech2_params& jet) {
  switch (L.dtype) {
    case LBM_FP64: return init_sech2_typed<double>(L, jet);
    case LBM_FP32: return init_sech2_typed<float>(L, jet);
    case LBM_FP16: return init_sech2_typed<_Float16>(L, jet);
    default: return init_sech2_typed<__bf16>(L, jet);
  }
}

template <typename S>
static hipError_t init_moments_typed(const Launch& L, int64_t t, const double* mom) {
  return by_lattice<S>(L, [&](auto qg) {
    hipLaunchKernelGGL((k_init_moments<S, decltype(qg)::value>), tile_grid(L.nx, L.ny), kTile, 0, L.stream,
                       buffer_at<S>(L, t), mom, L.nx, L.ny, L.pitch, layout_at(L, t), rest_ref(L));
    return hipGetLastError();
  });
}

hipError_t launch_init_moments(const Launch& L, int64_t t, const double* mom) {
  switch (L.dtype) {
    case LBM_FP64: return init_moments_typed<double>(L, t, mom);
    case LBM_FP32: return init_moments_typed<float>(L, t, mom);
    case LBM_FP16: return init_moments_typed<_Float16>(L, t, mom);
    default: return init_moments_typed<__bf16>(L, t, mom);
  }
}

template <typename S>
static hipError_t get_typed(const Launch& L, int64_t t, double* out) {
  return by_lattice<S>(L, [&](auto qg) {
    hipLaunchKernelGGL((k_get_state<S, decltype(qg)::value>), tile_grid(L.nx, L.ny), kTile, 0, L.stream,
                       buffer_at<S>(L, t), out, L.nx, L.ny, L.pitch, layout_at(L, t), rest_ref(L));
    return hipGetLastError();
  });
}

hipError_t launch_get_state(const Launch& L, int64_t t, double* out) {
  switch (L.dtype) {
    case LBM_FP64: return get_typed<double>(L, t, out);
    case LBM_FP32: return get_typed<float>(L, t, out);
    case LBM_FP16: return get_typed<_Float16>(L, t, out);
    default: return get_typed<__bf16>(L, t, out);
  }
}

template <typename S>
static hipError_t set_typed(const Launch& L, int64_t t, const double* in) {
  return by_lattice<S>(L, [&](auto qg) {
    hipLaunchKernelGGL((k_set_state<S, decltype(qg)::value>), tile_grid(L.nx, L.ny), kTile, 0, L.stream,
                       buffer_at<S>(L, t), in, L.nx, L.ny, L.pitch, layout_at(L, t), rest_ref(L));
    return hipGetLastError();
  });
}

hipError_t launch_set_state(const Launch& L, int64_t t, const double* in) {
  switch (L.dtype) {
    case LBM_FP64: return set_typed<double>(L, t, in);
    case LBM_FP32: return set_typed<float>(L, t, in);
    case LBM_FP16: return set_typed<_Float16>(L, t, in);
    default: return set_typed<__bf16>(L, t, in);
  }
}

template <typename S>
static hipError_t moments_typed(const Launch& L, int64_t t, double* out, bool mark) {
  return by_lattice<S>(L, [&](auto qg) {
    hipLaunchKernelGGL((k_moments_out<S, decltype(qg)::value>), dim3((L.nx + 255) / 256, L.ny), dim3(256), 0,
                       L.stream, buffer_at<S>(L, t), out, L.nx, L.ny, L.pitch, layout_at(L, t), rest_ref(L), mark);
    return hipGetLastError();
  });
}

hipError_t launch_moments(const Launch& L, int64_t t, double* out, bool mark_nonfinite) {
  switch (L.dtype) {
    case LBM_FP64: return moments_typed<double>(L, t, out, mark_nonfinite);
    case LBM_FP32: return moments_typed<float>(L, t, out, mark_nonfinite);
    case LBM_FP16: return moments_typed<_Float16>(L, t, out, mark_nonfinite);
    default: return moments_typed<__bf16>(L, t, out, mark_nonfinite);
  }
}

hipError_t launch_diagnostics(const Launch& L, int64_t t, double* vals_host) {
  char* w = static_cast<char*>(L.work);
  double* mom = reinterpret_cast<double*>(w + L.off_diag);
  double* part = reinterpret_cast<double*>(w + L.off_part);
  double* fin = reinterpret_cast<double*>(w + L.off_final);
  hipError_t e = launch_moments(L, t, mom, true);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_partial, dim3(L.diag_blocks), dim3(256), 0, L.stream, mom, part, L.nx, L.ny);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, L.stream, part, fin, L.diag_blocks);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(vals_host, fin, kDiagVals * sizeof(double), hipMemcpyDeviceToHost, L.stream)) !=
      hipSuccess)
    return e;
  return hipStreamSynchronize(L.stream);
}

}  // namespace lbm
