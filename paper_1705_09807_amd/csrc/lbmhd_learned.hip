// HIP kernels (gfx950) of the learned subgrid closure, the filtered-DNS
// pipeline that trains it, and the energy spectra.
//
// Method: Flint & Vahala, arXiv 1705.09807.  The analytic closure (Sec. 2.1
// FilterExampleSmall, Sec. 3) keeps the Delta^2/12 term of the filtered
// products; the learned closure adds a per-cell correction of the same four
// subgrid terms (tau_xx, tau_xy, tau_yy, eps), predicted by a 63-64-64-4 ReLU
// network trained on filtered DNS (the convolution of Sec. 1, VelFilter, with
// a Gaussian of variance Delta^2/12).  The spectra are the radially binned
// kinetic and magnetic energies compared in Sec. 4.
//
// Network on the matrix cores.  One wave evaluates 32 cells at a time in the
// transposed form H^T = W^T X^T, so that every layer's output (rows = hidden
// units, columns = cells) is directly the B operand of the next layer:
// v_mfma_f32_32x32x16_bf16 with A = 32 rows of W^T x 16 inputs, B = 16
// inputs x 32 cells, D = 32 x 32 FP32 (lane l holds column l % 32 and, in
// register i, row (i/4)*8 + (l/32)*4 + i%4).  The 16-input blocks of layers 2
// and 3 take their B operand from eight consecutive accumulator registers,
// which hold hidden rows (2 b + j/4) * 8 + (l/32) * 4 + j % 4; the packed A
// operands use the same permutation of the contraction index.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "lbmhd_device.h"
#include "lbmhd_internal.h"
#include "lbmhd_learned.h"
#include "lbmhd_mlp_device.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Packing
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_mlp_pack(const float* __restrict__ p, const lbm_mlp_norm* __restrict__ norm, char* __restrict__ pk) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  __bf16* a = reinterpret_cast<__bf16*>(pk);
  if (e < 4096) {  // A1: W1^T rows
    const int ot = e / 2048, kb = (e / 512) % 4, l = (e / 8) % 64, j = e % 8;
    const int hid = ot * 32 + l % 32, k = kb * 16 + (l / 32) * 8 + j;
    a[kPkA1 / 2 + e] = __bf16(k < 63 ? p[LBM_MLP_OFF_W1 + k * 64 + hid] : 0.0f);
  } else if (e < 8192) {  // A2: W2^T rows, chained contraction order
    const int f = e - 4096;
    const int ot = f / 2048, kb = (f / 512) % 4, l = (f / 8) % 64, j = f % 8;
    const int out = ot * 32 + l % 32, k = chained_k(kb, l / 32, j);
    a[kPkA2 / 2 + f] = __bf16(p[LBM_MLP_OFF_W2 + k * 64 + out]);
  } else if (e < 10240) {  // A3: W3^T rows 0..3, rest zero
    const int f = e - 8192;
    const int kb = f / 512, l = (f / 8) % 64, j = f % 8;
    const int o = l % 32, k = chained_k(kb, l / 32, j);
    a[kPkA3 / 2 + f] = __bf16(o < 4 ? p[LBM_MLP_OFF_W3 + k * 4 + o] : 0.0f);
  } else if (e < 10240 + 64) {
    const int i = e - 10240;
    reinterpret_cast<float*>(pk + kPkB1)[i] = p[LBM_MLP_OFF_B1 + i];
    reinterpret_cast<float*>(pk + kPkB2)[i] = p[LBM_MLP_OFF_B2 + i];
    reinterpret_cast<float*>(pk + kPkB3)[i] = i < 4 ? p[LBM_MLP_OFF_B3 + i] : 0.0f;
  } else if (e < 10240 + 64 + 32) {
    const int i = e - 10240 - 64;
    reinterpret_cast<float*>(pk + kPkNorm)[i] = reinterpret_cast<const float*>(norm)[i];
  } else if (e < 10240 + 64 + 32 + 4096) {  // A1n: W1^T rows, patch-ordered inputs
    const int f = e - (10240 + 64 + 32);
    const int ot = f / 2048, kb = (f / 512) % 4, l = (f / 8) % 64, j = f % 8;
    const int hid = ot * 32 + l % 32, pos = kb * 2 + l / 32;
    // element j < 7: field j at pos; element 7: field pos at position 8
    const int k = j < 7 ? j * 9 + pos : (pos < 7 ? pos * 9 + 8 : -1);
    __bf16* c = reinterpret_cast<__bf16*>(pk + kPkA1n);
    c[f] = __bf16(k >= 0 ? p[LBM_MLP_OFF_W1 + k * 64 + hid] : 0.0f);
  }
}

// ---------------------------------------------------------------------------
// Forward on feature rows (inference of given inputs; also the parity probe
// of the matrix-core network)
// ---------------------------------------------------------------------------

// Layer-1 operands of this lane from feature row `row` of x (FP32): z =
// (x - shift) * scale per field, pad 0, rounded to bfloat16.  Sets *ood when
// any |z| exceeds the limit; zf (may be null) receives the rounded values.
__device__ __forceinline__ void row_operands(const float* __restrict__ x, int64_t row, const lbm_mlp_norm* nm,
                                             int h, bf16x8 zb[4], bool* ood, float* zf) {
  bool o = false;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const f32x4* src = reinterpret_cast<const f32x4*>(x + row * 64 + kb * 16 + h * 8);
    const f32x4 u = src[0], v = src[1];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = kb * 16 + h * 8 + j;
      const float xv = j < 4 ? u[j] : v[j - 4];
      float z = 0.0f;
      if (k < 63) {
        const int f = feat_field(k);
        z = (xv - nm->shift[f]) * nm->scale[f];
      }
      o = o || !(fabsf(z) <= kOodLimit);  // NaN counts as out of range
      zb[kb][j] = __bf16(z);
      if (zf) zf[kb * 8 + j] = float(zb[kb][j]);
    }
  }
  *ood = o;
}

__global__ void __launch_bounds__(256)
k_mlp_forward(const char* __restrict__ pk, const float* __restrict__ x, int64_t n, float* __restrict__ y,
              int32_t* __restrict__ ood_out) {
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const lbm_mlp_norm* nm = reinterpret_cast<const lbm_mlp_norm*>(pk + kPkNorm);
  MlpA w;
  load_mlp(pk, lane, w);
  for (int64_t g = wave; g * 32 < n; g += nwaves) {
    const int64_t row = g * 32 + (lane & 31);
    const int64_t rr = row < n ? row : n - 1;
    bf16x8 zb[4];
    bool o;
    row_operands(x, rr, nm, h, zb, &o, nullptr);
    const f32x4 v = mlp_wave(w, zb, reinterpret_cast<const float*>(pk + kPkB1), lane, nullptr, nullptr);
    // every lane takes part in the exchange (a short-circuit would leave the
    // flagged lane inactive and its partner would read nothing from it)
    const int partner = __shfl_xor(int(o), 32, 64);
    const bool oo = o || partner != 0;
    if (h == 0 && row < n) {
      *reinterpret_cast<f32x4*>(y + row * 4) = v;
      if (ood_out) ood_out[row] = oo ? 1 : 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Correction of a simulation state, second stage: the network on the per-cell
// input vectors (CellIn, 16 bytes per cell) that the first stage wrote from
// the state.  A workgroup loads the vectors of a 64 x 16 tile and its
// one-cell halo straight into LDS (one 16-byte load per cell, no register
// staging), then evaluates the network for its 1024 cells (each wave 8 groups
// of 32).  Layer 1 contracts over four 16-input blocks of patch positions
// (kPkA1n): a lane's operand of a block is one 16-byte LDS read whose last
// element is replaced by a field of position 8.  A cell is out of
// distribution when a flagged cell lies in its 3x3 neighbourhood (its 63
// inputs are exactly the seven fields there).  Output: four FP32 planes
// tau_xx, tau_xy, tau_yy, eps = out_scale * y, 0 for out-of-distribution cells
// and cells whose output is not finite.
// ---------------------------------------------------------------------------
constexpr int kCorrTX = 64, kCorrTY = 16;
constexpr int kCorrLX = kCorrTX + 2, kCorrLY = kCorrTY + 2, kCorrPL = kCorrLX * kCorrLY;

// LDS cell offset of patch position pos (< 9: row pos / 3, column pos % 3)
// of tile cell (ty, tx) from ty * LX + tx: the patch corner is at (ty, tx)
// in the tile with its one-cell halo.
__host__ __device__ constexpr int corr_patch_offset(int pos) { return (pos / 3) * kCorrLX + pos % 3; }

// Periodic wrap of v in [-1, n + kCorrLX) into [0, n).
__device__ __forceinline__ int wrap_halo(int v, int n, bool wide) {
  if (wide) {
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
  }
  v %= n;
  return v < 0 ? v + n : v;
}

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void global_void;

__global__ void __launch_bounds__(256, 2)
k_mlp_correct(const CellIn* __restrict__ in, const char* __restrict__ pk, float* __restrict__ corr, int nx, int ny) {
  constexpr int LX = kCorrLX, PL = kCorrPL, PER = (PL + 255) / 256;
  __shared__ CellIn zt[PER * 256];
  __shared__ __attribute__((aligned(16))) float bias[132];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, h = lane >> 5;
  const int x0 = blockIdx.x * kCorrTX, y0 = blockIdx.y * kCorrTY;
  const int64_t n = (int64_t)nx * ny;
  const bool wide_x = nx >= LX, wide_y = ny >= kCorrLY;
  // each wave fills 64 consecutive entries per pass (entry base + lane)
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + 256 * i;
    if (e < PL) {
      const int ly = e / LX, lx = e - ly * LX;
      const int gx = wrap_halo(x0 + lx - 1, nx, wide_x), gy = wrap_halo(y0 + ly - 1, ny, wide_y);
      __builtin_amdgcn_global_load_lds((global_void*)(in + ((int64_t)gy * nx + gx)),
                                       (lds_void*)(zt + 256 * i + 64 * wid), 16, 0, 0);
    }
  }
  if (tid < 132) bias[tid] = reinterpret_cast<const float*>(pk + kPkB1)[tid];
  const lbm_mlp_norm* nm = reinterpret_cast<const lbm_mlp_norm*>(pk + kPkNorm);
  MlpA w;
  load_mlp_n(pk, lane, w);
  const float os0 = nm->out_scale[0], os1 = nm->out_scale[1], os2 = nm->out_scale[2], os3 = nm->out_scale[3];
  __builtin_amdgcn_s_waitcnt(0);  // the loads into LDS are complete
  __syncthreads();
  for (int g = wid; g < kCorrTX * kCorrTY / 32; g += 4) {
    const int ty = g >> 1, tx = (g & 1) * 32 + (lane & 31), base = ty * LX + tx;
    CellIn v[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) v[kb] = zt[base + (h ? corr_patch_offset(2 * kb + 1) : corr_patch_offset(2 * kb))];
    const CellIn v8 = zt[base + corr_patch_offset(8)];
    bf16x8 zb[4];
    bool bad;
    patch_operands(v, v8, h, zb, &bad);
    // the two halves of a cell see complementary patch positions.  Every lane
    // takes part in the exchange: under a short-circuit only the lanes with
    // bad == false would run it, the value they send would be known to be 0,
    // and the compiler drops the exchange altogether.
    const int partner = __shfl_xor(int(bad), 32, 64);
    const bool pb = bad || partner != 0;
    const f32x4 y = mlp_wave(w, zb, bias, lane, nullptr, nullptr);
    const bool o = pb || !(isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]) && isfinite(y[3]));
    const int gx = x0 + tx, gy = y0 + ty;
    if (h == 0 && gx < nx && gy < ny) {
      float* cp = corr + ((int64_t)gy * nx + gx);
      // non-temporal stores: the planes are read by the next sweep, after the
      // whole grid is written (measured together with the input vectors'
      // non-temporal stores: the 16384^2 learned step 0.5-1 % faster)
      __builtin_nontemporal_store(o ? 0.0f : y[0] * os0, cp);
      __builtin_nontemporal_store(o ? 0.0f : y[1] * os1, cp + n);
      __builtin_nontemporal_store(o ? 0.0f : y[2] * os2, cp + 2 * n);
      __builtin_nontemporal_store(o ? 0.0f : y[3] * os3, cp + 3 * n);
    }
  }
}

// ---------------------------------------------------------------------------
// Training: forward and backward on the matrix cores.  A workgroup of two
// waves takes chunks of 64 batch rows (32 per wave in the forward).  With the
// batch row r, the loss L = sum (y - t)^2 / (4 batch) and straight-through
// gradients of the bfloat16 roundings:
//   d3 = dL/dy,  d2 = (d3 W3^T) [h2 > 0],  d1 = (d2 W2^T) [h1 > 0],
//   G3 = h2^T d3, G2 = h1^T d2, G1 = z^T d1, biases: column sums of d.
// d3 and d2 are formed in FP32 on the vector ALU (contraction over the four
// outputs).  d1^T = W2 d2^T is one matrix-core product in the transposed
// form of the forward (hidden units x rows, d2 in the accumulator layout of
// h2, so it is directly the B operand), and G2, G1 are products over the 64
// rows of the chunk from feature-major LDS tiles.  A delta enters the matrix
// cores as three bfloat16 terms, d = hi + mid + lo + O(2^-25 |d|), so the
// products carry the FP32 delta; activations and weights are bfloat16
// already.  (Two terms, 16 bits, left 1e-4 relative errors in G1 over 5000
// rows, where the row sums cancel.)  Each wave owns half of every weight gradient and accumulates it
// over its workgroup's chunks in a fixed order; per-workgroup partials are
// summed in a fixed order by k_mlp_reduce_groups and k_mlp_reduce.
// ---------------------------------------------------------------------------
constexpr int kTrainChunk = 64;
constexpr int kTrainBlocksMax = 1024;
constexpr int kGradStride = 8704;  // floats per partial (>= LBM_MLP_PARAMS, 256-byte multiple)
constexpr int kTs = 72;            // bfloat16 per feature row of an LDS tile (64 rows + pad)

struct TrainLds {
  __bf16 z[64][kTs], h1[64][kTs], h2[64][kTs];     // [feature][chunk row]
  __bf16 d2h[64][kTs], d2m[64][kTs], d2l[64][kTs], d1h[64][kTs], d1m[64][kTs], d1l[64][kTs];
  bf16x8 a2b[2][4][64];                            // A operands of d1^T = W2 d2^T
  float d3[4][kTrainChunk];
  float w3[64 * 4];                                // bfloat16-rounded W3
  double loss[128];
};

// hi + mid + lo bfloat16 split of eight floats (each remainder is exact in
// FP32, so the three terms carry 24 bits).
__device__ __forceinline__ void split_bf16x8(const float* v, bf16x8& hi, bf16x8& mid, bf16x8& lo) {
  f32x8 a, b, c;
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = v[j];
  hi = to_bf16x8(a);
#pragma unroll
  for (int j = 0; j < 8; ++j) b[j] = v[j] - float(hi[j]);
  mid = to_bf16x8(b);
#pragma unroll
  for (int j = 0; j < 8; ++j) c[j] = b[j] - float(mid[j]);
  lo = to_bf16x8(c);
}

// One 32 x 32 tile of sum_r A[m][r] B[n][r] over the 64 rows of the chunk,
// from feature-major LDS tiles (operands: 8 consecutive rows per lane); the
// B tile is split hi + mid + lo.
__device__ __forceinline__ f32x16 rows_product(f32x16 acc, const __bf16 (*a)[kTs], const __bf16 (*bh)[kTs],
                                               const __bf16 (*bm)[kTs], const __bf16 (*bl)[kTs], int ma, int nb,
                                               int lane) {
  const int r0 = (lane >> 5) * 8, la = lane & 31;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(&a[ma + la][kb * 16 + r0]);
    const bf16x8 hv = *reinterpret_cast<const bf16x8*>(&bh[nb + la][kb * 16 + r0]);
    const bf16x8 mv = *reinterpret_cast<const bf16x8*>(&bm[nb + la][kb * 16 + r0]);
    const bf16x8 lv = *reinterpret_cast<const bf16x8*>(&bl[nb + la][kb * 16 + r0]);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, hv, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, mv, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, lv, acc, 0, 0, 0);
  }
  return acc;
}

// ReLU'd bfloat16 activations of two accumulator tiles (as activate()), stored
// feature-major for chunk row sl; also returned as the next layer's B operands.
__device__ __forceinline__ void activate_to_lds(const f32x16 acc[2], bf16x8 hb[4], __bf16 (*dst)[kTs], int h,
                                                int sl) {
  activate(acc, hb, nullptr);
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[chained_k(kb, h, j)][sl] = hb[kb][j];
}

__global__ void __launch_bounds__(128)
k_mlp_train(const char* __restrict__ pk, const float* __restrict__ p, const float* __restrict__ x,
            const float* __restrict__ t, const int32_t* __restrict__ idx, int batch, float* __restrict__ partial,
            double* __restrict__ loss_part) {
  __shared__ TrainLds s;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, h = lane >> 5;
  const lbm_mlp_norm* nm = reinterpret_cast<const lbm_mlp_norm*>(pk + kPkNorm);
  const float* b1 = reinterpret_cast<const float*>(pk + kPkB1);
  const float* b2 = reinterpret_cast<const float*>(pk + kPkB2);
  const float* b3 = reinterpret_cast<const float*>(pk + kPkB3);
  const bf16x8* pa1 = reinterpret_cast<const bf16x8*>(pk + kPkA1);
  const bf16x8* pa2 = reinterpret_cast<const bf16x8*>(pk + kPkA2);
  const bf16x8* pa3 = reinterpret_cast<const bf16x8*>(pk + kPkA3);
  // A operands of d1^T = W2 d2^T: row i = ot*32 + lane%32 of W2, contraction
  // index j in the chained order of the accumulator layout
  for (int e = tid; e < 2 * 4 * 64; e += 128) {
    const int ot = e / 256, kb = (e / 64) % 4, l = e % 64;
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      v[j] = __bf16(p[LBM_MLP_OFF_W2 + (ot * 32 + (l & 31)) * 64 + chained_k(kb, l >> 5, j)]);
    s.a2b[ot][kb][l] = v;
  }
  for (int e = tid; e < 256; e += 128) s.w3[e] = bf16_round(p[LBM_MLP_OFF_W3 + e]);
  // gradient accumulators: wave wid owns rows [32 wid, 32 wid + 32) of G1 and
  // G2 (two 32 x 32 tiles each, columns 0..31 and 32..63); thread tid owns two
  // entries of G3 and one bias entry of b1 (tid >= 64) or b2 (tid < 64)
  f32x16 g1[2], g2[2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) g1[c][e] = g2[c][e] = 0.0f;
  float g3a = 0.0f, g3b = 0.0f, gb = 0.0f, gb3 = 0.0f;
  double loss = 0.0;
  const float inv = 2.0f / (float(batch) * 4.0f);
  const int chunks = (batch + kTrainChunk - 1) / kTrainChunk;
  const int sl = wid * 32 + (lane & 31);           // chunk row of this lane
  for (int c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int b = c * kTrainChunk + sl;
    const bool valid = b < batch;
    // forward (the operations of mlp_wave), activations to LDS
    {
      const int64_t row = idx[valid ? b : batch - 1];
      bf16x8 zb[4];
      float zf[32];
      bool o;
      row_operands(x, row, nm, h, zb, &o, zf);
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int j = 0; j < 8; ++j) s.z[kb * 16 + h * 8 + j][sl] = zb[kb][j];
      f32x16 acc[2];
      bf16x8 hb[4];
#pragma unroll
      for (int ot = 0; ot < 2; ++ot) {
        acc[ot] = bias_tile(b1, ot, h);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
          acc[ot] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pa1[(ot * 4 + kb) * 64 + lane], zb[kb], acc[ot], 0, 0, 0);
      }
      activate_to_lds(acc, hb, s.h1, h, sl);
#pragma unroll
      for (int ot = 0; ot < 2; ++ot) {
        acc[ot] = bias_tile(b2, ot, h);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
          acc[ot] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pa2[(ot * 4 + kb) * 64 + lane], hb[kb], acc[ot], 0, 0, 0);
      }
      activate_to_lds(acc, hb, s.h2, h, sl);
      f32x16 out;
#pragma unroll
      for (int i = 0; i < 16; ++i) out[i] = 0.0f;
      if (h == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = b3[i];
      }
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pa3[kb * 64 + lane], hb[kb], out, 0, 0, 0);
      if (h == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float r = out[q] - t[row * 4 + q] / nm->out_scale[q];
          s.d3[q][sl] = valid ? inv * r : 0.0f;
          if (valid) loss += double(r) * double(r);
        }
      }
    }
    __syncthreads();
    // d2 in the accumulator layout of h2 (element kb*8 + j: hidden
    // chained_k(kb, h, j)), then d1^T = W2 d2^T on the matrix cores
    {
      float d3v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) d3v[q] = s.d3[q][sl];
      bf16x8 dh[4], dm[4], dl[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        float d2[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int ck = chained_k(kb, h, j);
          const float* w3 = &s.w3[ck * 4];
          const float a = w3[0] * d3v[0] + w3[1] * d3v[1] + w3[2] * d3v[2] + w3[3] * d3v[3];
          d2[j] = float(s.h2[ck][sl]) > 0.0f ? a : 0.0f;
        }
        split_bf16x8(d2, dh[kb], dm[kb], dl[kb]);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int ck = chained_k(kb, h, j);
          s.d2h[ck][sl] = dh[kb][j];
          s.d2m[ck][sl] = dm[kb][j];
          s.d2l[ck][sl] = dl[kb][j];
        }
      }
#pragma unroll
      for (int ot = 0; ot < 2; ++ot) {
        f32x16 acc;
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const bf16x8 a = s.a2b[ot][kb][lane];
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, dh[kb], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, dm[kb], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, dl[kb], acc, 0, 0, 0);
        }
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          float d1[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int hid = ot * 32 + acc_row(half * 8 + j, h);
            d1[j] = float(s.h1[hid][sl]) > 0.0f ? acc[half * 8 + j] : 0.0f;
          }
          bf16x8 hi, mi, lo;
          split_bf16x8(d1, hi, mi, lo);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int hid = ot * 32 + acc_row(half * 8 + j, h);
            s.d1h[hid][sl] = hi[j];
            s.d1m[hid][sl] = mi[j];
            s.d1l[hid][sl] = lo[j];
          }
        }
      }
    }
    __syncthreads();
    // weight gradients over the chunk's rows
#pragma unroll
    for (int cn = 0; cn < 2; ++cn) {
      g2[cn] = rows_product(g2[cn], s.h1, s.d2h, s.d2m, s.d2l, wid * 32, cn * 32, lane);
      g1[cn] = rows_product(g1[cn], s.z, s.d1h, s.d1m, s.d1l, wid * 32, cn * 32, lane);
    }
    {
      // G3[j][o] for j = tid / 2, o = 2 (tid % 2) + {0, 1}; bias of d1 or d2
      const int j = tid >> 1, o = (tid & 1) * 2, bh = tid & 63;
      const __bf16(*dh)[kTs] = tid < 64 ? s.d2h : s.d1h;
      const __bf16(*dm)[kTs] = tid < 64 ? s.d2m : s.d1m;
      const __bf16(*dl)[kTs] = tid < 64 ? s.d2l : s.d1l;
      for (int r = 0; r < kTrainChunk; ++r) {
        const float hv = float(s.h2[j][r]);
        g3a += hv * s.d3[o][r];
        g3b += hv * s.d3[o + 1][r];
        gb += (float(dh[bh][r]) + float(dm[bh][r])) + float(dl[bh][r]);
      }
      if (tid < 4)
        for (int r = 0; r < kTrainChunk; ++r) gb3 += s.d3[tid][r];
    }
    __syncthreads();
  }
  float* out = partial + (int64_t)blockIdx.x * kGradStride;
#pragma unroll
  for (int cn = 0; cn < 2; ++cn)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int m = wid * 32 + acc_row(e, h), n = cn * 32 + (lane & 31);
      out[LBM_MLP_OFF_W1 + m * 64 + n] = g1[cn][e];
      out[LBM_MLP_OFF_W2 + m * 64 + n] = g2[cn][e];
    }
  out[LBM_MLP_OFF_W3 + (tid >> 1) * 4 + (tid & 1) * 2] = g3a;
  out[LBM_MLP_OFF_W3 + (tid >> 1) * 4 + (tid & 1) * 2 + 1] = g3b;
  out[(tid < 64 ? LBM_MLP_OFF_B2 : LBM_MLP_OFF_B1) + (tid & 63)] = gb;
  if (tid < 4) out[LBM_MLP_OFF_B3 + tid] = gb3;
  // loss: fixed-order sum over the lanes that hold outputs
  s.loss[tid] = loss;
  __syncthreads();
  if (tid == 0) {
    double a = 0.0;
    for (int k = 0; k < 128; ++k) a += s.loss[k];
    loss_part[blockIdx.x] = a;
  }
}

// Sum of the partial gradients (and of the loss partials) in a fixed order,
// in two launches so that the loads of many partials are in flight at once:
// each run of kReduceGroup consecutive partials is summed in order into its
// first partial (k_mlp_reduce_groups), then those group sums in order
// (k_mlp_reduce).  (One thread summing all partials in order, one launch,
// waited on each batch of loads: 34 us for 128 partials.)
constexpr int kReduceGroup = 16;

__global__ void __launch_bounds__(256)
k_mlp_reduce_groups(float* __restrict__ partial, int nparts, double* __restrict__ loss_part) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int b0 = blockIdx.y * kReduceGroup;
  const int nb = min(kReduceGroup, nparts - b0);
  if (i < LBM_MLP_PARAMS) {
    float v[kReduceGroup];
#pragma unroll
    for (int k = 0; k < kReduceGroup; ++k) v[k] = k < nb ? partial[(int64_t)(b0 + k) * kGradStride + i] : 0.0f;
    float g = v[0];
#pragma unroll
    for (int k = 1; k < kReduceGroup; ++k)
      if (k < nb) g += v[k];
    partial[(int64_t)b0 * kGradStride + i] = g;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss_part) {
    double a = loss_part[b0];
    for (int k = 1; k < nb; ++k) a += loss_part[b0 + k];
    loss_part[b0] = a;
  }
}

__global__ void __launch_bounds__(256)
k_mlp_reduce(const float* __restrict__ partial, int nparts, float* __restrict__ grad,
             const double* __restrict__ loss_part, float* __restrict__ loss_out, float loss_norm) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < LBM_MLP_PARAMS) {
    float g = 0.0f;
    for (int b = 0; b < nparts; b += kReduceGroup) g += partial[(int64_t)b * kGradStride + i];
    grad[i] = g;
  }
  if (i == 0 && loss_out) {
    double a = 0.0;
    for (int b = 0; b < nparts; b += kReduceGroup) a += loss_part[b];
    *loss_out = float(a * double(loss_norm));
  }
}

// Adam (Kingma & Ba 2015), bias corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void __launch_bounds__(256)
k_mlp_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ grad,
           float lr, float bc1, float bc2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= LBM_MLP_PARAMS) return;
  const float g = grad[i];
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ---------------------------------------------------------------------------
// Normalisation statistics: FP64 partial sums per workgroup, fixed-order
// final pass.  Pass 1: sums of the seven centre features and of the squared
// targets; pass 2: squared deviations from the means.
// ---------------------------------------------------------------------------
constexpr int kStatBlocks = 256;

__device__ void block_sum11(double* acc, double* out) {
  __shared__ double red[4][11];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int k = 0; k < 11; ++k) acc[k] += __shfl_down(acc[k], off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 11; ++k) red[wid][k] = acc[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 11; ++k) out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  __syncthreads();
}

__global__ void __launch_bounds__(256)
k_stats_pass(const float* __restrict__ x, const float* __restrict__ t, int64_t n, const double* __restrict__ mean,
             double* __restrict__ part) {
  double acc[11];
#pragma unroll
  for (int k = 0; k < 11; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += stride) {
#pragma unroll
    for (int f = 0; f < 7; ++f) {
      const double v = x[r * 64 + f * 9 + 4];
      if (mean) {
        const double d = v - mean[f];
        acc[f] += d * d;
      } else {
        acc[f] += v;
      }
    }
    if (!mean)
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        const double v = t[r * 4 + o];
        acc[7 + o] += v * v;
      }
  }
  block_sum11(acc, part + (int64_t)blockIdx.x * 11);
}

// mode 0: partial sums -> means (mean[0..6]) and target RMS; mode 1:
// squared deviations -> norm.
__global__ void __launch_bounds__(64)
k_stats_final(const double* __restrict__ part, int nparts, int64_t n, double* __restrict__ mean, int mode,
              lbm_mlp_norm* __restrict__ norm) {
  if (threadIdx.x != 0) return;
  double s[11];
  for (int k = 0; k < 11; ++k) s[k] = 0.0;
  for (int b = 0; b < nparts; ++b)
    for (int k = 0; k < 11; ++k) s[k] += part[(int64_t)b * 11 + k];
  const double dn = double(n);
  if (mode == 0) {
    for (int f = 0; f < 7; ++f) mean[f] = s[f] / dn;
    for (int o = 0; o < 4; ++o) mean[7 + o] = sqrt(s[7 + o] / dn);
    return;
  }
  lbm_mlp_norm nm;
  for (int k = 0; k < 8; ++k) {
    nm.shift[k] = 0.0f;
    nm.scale[k] = 1.0f;
  }
  for (int f = 0; f < 7; ++f) {
    const double sd = sqrt(s[f] / dn);
    nm.shift[f] = float(mean[f]);
    nm.scale[f] = sd > 0.0 ? float(1.0 / sd) : 1.0f;
  }
  for (int o = 0; o < 4; ++o) nm.out_scale[o] = mean[7 + o] > 0.0 ? float(mean[7 + o]) : 1.0f;
  for (int k = 0; k < 12; ++k) nm.pad[k] = 0.0f;
  *norm = nm;
}

// ---------------------------------------------------------------------------
// Filtered DNS: Gaussian taps, x pass (12 products, subsampled columns), y
// pass (subsampled rows).  FP64 throughout.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gauss_taps(double sigma2, int R, double* __restrict__ taps) {
  __shared__ double wv[256];
  const int r = threadIdx.x;
  if (r <= 2 * R) {
    const double d = double(r - R);
    wv[r] = exp(-d * d / (2.0 * sigma2));
  }
  __syncthreads();
  if (r == 0) {
    double s = 0.0;
    for (int k = 0; k <= 2 * R; ++k) s += wv[k];
    wv[255] = s;
  }
  __syncthreads();
  if (r <= 2 * R) taps[r] = wv[r] / wv[255];
}

__global__ void __launch_bounds__(64)
k_filter_x(const double* __restrict__ mom, int nx, int ny, int factor, int R, const double* __restrict__ taps,
           double* __restrict__ tmp) {
  const int cx = nx / factor;
  const int X = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y;
  if (X >= cx) return;
  const int64_t n = (int64_t)nx * ny;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int r = -R; r <= R; ++r) {
    int xx = (X * factor + r) % nx;
    if (xx < 0) xx += nx;
    const int64_t c = (int64_t)y * nx + xx;
    const double rho = mom[c], mx = mom[n + c], my = mom[2 * n + c], bx = mom[3 * n + c], by = mom[4 * n + c];
    const double w = taps[r + R];
    const double p[12] = {rho, mx, my, bx, by, mx * mx / rho, mx * my / rho, my * my / rho,
                          bx * bx, bx * by, by * by, (mx * by - my * bx) / rho};
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] += w * p[k];
  }
  const int64_t cn = (int64_t)cx * ny;
#pragma unroll
  for (int k = 0; k < 12; ++k) tmp[k * cn + (int64_t)y * cx + X] = acc[k];
}

__global__ void __launch_bounds__(64)
k_filter_y(const double* __restrict__ tmp, int nx, int ny, int factor, int R, const double* __restrict__ taps,
           double* __restrict__ out) {
  const int cx = nx / factor, cy = ny / factor;
  const int X = blockIdx.x * 64 + threadIdx.x, Y = blockIdx.y, k = blockIdx.z;
  if (X >= cx) return;
  const int64_t cn = (int64_t)cx * ny;
  double acc = 0.0;
  for (int r = -R; r <= R; ++r) {
    int yy = (Y * factor + r) % ny;
    if (yy < 0) yy += ny;
    acc += taps[r + R] * tmp[k * cn + (int64_t)yy * cx + X];
  }
  out[(int64_t)k * cx * cy + (int64_t)Y * cx + X] = acc;
}

// ---------------------------------------------------------------------------
// Training samples on the coarse grid: inputs and exact-minus-analytic
// targets of every cell (FP64 arithmetic, FP32 output).
// ---------------------------------------------------------------------------
template <int STENCIL>
__global__ void __launch_bounds__(256)
k_closure_samples(const double* __restrict__ c12, int nx, int ny, double k2, float* __restrict__ xo,
                  float* __restrict__ to) {
  const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const int64_t n = (int64_t)nx * ny;
  auto at = [&](int k, int dx, int dy) {
    int xx = (x + dx) % nx, yy = (y + dy) % ny;
    if (xx < 0) xx += nx;
    if (yy < 0) yy += ny;
    return c12[k * n + (int64_t)yy * nx + xx];
  };
  auto field = [&](int f, int dx, int dy) -> double {
    switch (f) {
      case 0: return at(0, dx, dy);
      case 1: return at(1, dx, dy) / at(0, dx, dy);
      case 2: return at(2, dx, dy) / at(0, dx, dy);
      case 3: return at(3, dx, dy);
      default: return at(4, dx, dy);
    }
  };
  const int64_t c = (int64_t)y * nx + x;
  float* xr = xo + c * 64;
  for (int f = 0; f < 7; ++f)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        double v;
        if (f < 5) {
          v = field(f, dx, dy);
        } else {
          const int a = f == 5 ? 2 : 4, b = f == 5 ? 1 : 3;  // w: (u_y, u_x); J_z: (B_y, B_x)
          v = 0.5 * (field(a, dx + 1, dy) - field(a, dx - 1, dy)) - 0.5 * (field(b, dx, dy + 1) - field(b, dx, dy - 1));
        }
        xr[f * 9 + (dy + 1) * 3 + (dx + 1)] = float(v);
      }
  xr[63] = 0.0f;
  // exact subgrid terms of the filtered products
  const double rho = at(0, 0, 0), mx = at(1, 0, 0), my = at(2, 0, 0), bx = at(3, 0, 0), by = at(4, 0, 0);
  const double rxx = at(5, 0, 0) - mx * mx / rho, rxy = at(6, 0, 0) - mx * my / rho, ryy = at(7, 0, 0) - my * my / rho;
  const double qxx = at(8, 0, 0) - bx * bx, qxy = at(9, 0, 0) - bx * by, qyy = at(10, 0, 0) - by * by;
  const double eps = at(11, 0, 0) - (mx * by - my * bx) / rho;
  // analytic closure of the filtered fields
  double g[4][2];
  for (int k = 0; k < 4; ++k)
    grad3x3<double, STENCIL>(at(1 + k, 1, 0), at(1 + k, -1, 0), at(1 + k, 0, 1), at(1 + k, 0, -1), at(1 + k, 1, 1),
                             at(1 + k, -1, 1), at(1 + k, 1, -1), at(1 + k, -1, -1), g[k][0], g[k][1]);
  const Closure<double> cl =
      closure_terms(g[0][0], g[0][1], g[1][0], g[1][1], g[2][0], g[2][1], g[3][0], g[3][1], 1.0 / rho, k2);
  const double a_xx = 0.5 * (cl.tau_s + cl.tau_d), a_yy = 0.5 * (cl.tau_s - cl.tau_d);
  float* tr = to + c * 4;
  tr[0] = float((rxx + 0.5 * (qyy - qxx)) - a_xx);
  tr[1] = float((rxy - qxy) - cl.tau_xy);
  tr[2] = float((ryy + 0.5 * (qxx - qyy)) - a_yy);
  tr[3] = float(eps - cl.eps);
}

// ---------------------------------------------------------------------------
// Spectra.  Two complex fields per state, z_u = u_x + i u_y and z_B = B_x + i
// B_y: over a bin that contains -k with every k, sum |Z(k)|^2 equals
// sum |A(k)|^2 + |B(k)|^2 of the real fields' transforms.  Row FFTs, then
// column FFTs that bin |Z|^2 / n^4 per column (deterministic: one thread per
// bin walks its k_y range in order), then a fixed-order sum over columns.
// Radix-2 decimation in time in LDS (bit-reversed load), FP64 twiddles from
// sincospi.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) { return __builtin_bitreverse32(v) >> (32 - bits); }

// floor(sqrt(v)) and ceil(sqrt(v)) of a non-negative integer, exact.
__device__ __forceinline__ int isqrt_floor(int64_t v) {
  int64_t r = (int64_t)sqrt(double(v));
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return (int)r;
}
__device__ __forceinline__ int isqrt_ceil(int64_t v) {
  const int r = isqrt_floor(v);
  return (int64_t)r * r == v ? r : r + 1;
}

__device__ void fft_lds(double2* a, int n, int bits) {
  for (int half = 1; half < n; half <<= 1) {
    __syncthreads();
    for (int j = threadIdx.x; j < n / 2; j += blockDim.x) {
      const int pos = j & (half - 1);
      const int i0 = ((j - pos) << 1) + pos, i1 = i0 + half;
      double s, c;
      sincospi(-double(pos) / double(half), &s, &c);
      const double2 u = a[i0], v = a[i1];
      const double tr = c * v.x - s * v.y, ti = c * v.y + s * v.x;
      a[i0] = make_double2(u.x + tr, u.y + ti);
      a[i1] = make_double2(u.x - tr, u.y - ti);
    }
  }
  __syncthreads();
}

// Column of a column-pass workgroup.  Workgroups are dealt to the 8 XCDs in
// turn; this gives each XCD a contiguous range of columns, so the workgroups
// that read neighbouring columns (the same cache lines of every row) share an
// L2.  n is a power of two >= 8.
__device__ __forceinline__ int column_of_block(int bx, int n) { return (bx & 7) * (n >> 3) + (bx >> 3); }

__global__ void __launch_bounds__(256)
k_fft_rows(const double* __restrict__ mom, int n, int bits, double2* __restrict__ work) {
  extern __shared__ double2 a[];
  const int y = blockIdx.x, pair = blockIdx.y;
  const int64_t nn = (int64_t)n * n;
  for (int x = threadIdx.x; x < n; x += blockDim.x) {
    const int64_t c = (int64_t)y * n + x;
    double re, im;
    if (pair == 0) {
      const double r = mom[c];
      re = mom[nn + c] / r;
      im = mom[2 * nn + c] / r;
    } else {
      re = mom[3 * nn + c];
      im = mom[4 * nn + c];
    }
    a[bitrev(x, bits)] = make_double2(re, im);
  }
  fft_lds(a, n, bits);
  for (int x = threadIdx.x; x < n; x += blockDim.x) work[pair * nn + (int64_t)y * n + x] = a[x];
}

__global__ void __launch_bounds__(256)
k_fft_cols(const double2* __restrict__ work, int n, int bits, int nbins, double* __restrict__ part,
           double* __restrict__ partx) {
  extern __shared__ double2 a[];
  const int kxi = column_of_block(blockIdx.x, n), pair = blockIdx.y;
  const int64_t nn = (int64_t)n * n;
  for (int y = threadIdx.x; y < n; y += blockDim.x) a[bitrev(y, bits)] = work[pair * nn + (int64_t)y * n + kxi];
  fft_lds(a, n, bits);
  const double inv = 1.0 / (double(n) * double(n));
  const int kx = kxi < n / 2 ? kxi : kxi - n;
  const int64_t kx2 = (int64_t)kx * kx;
  double* out = part + ((int64_t)pair * n + kxi) * nbins;
  // Bin b holds the k with floor(|k| + 1/2) = b, i.e. |k|^2 = 0 for b = 0 and
  // b^2 - b + 1 <= |k|^2 <= b^2 + b for b >= 1 (exact in integers).  One
  // thread per bin walks its |k_y| range upwards, +k_y before -k_y.
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    const int64_t lo = b == 0 ? 0 : (int64_t)b * b - b + 1 - kx2;
    const int64_t hi = (int64_t)b * b + b - kx2;
    double s = 0.0;
    if (hi >= 0) {
      const int a0 = lo <= 0 ? 0 : isqrt_ceil(lo);
      int a1 = isqrt_floor(hi);
      if (a1 > n / 2) a1 = n / 2;
      for (int ay = a0; ay <= a1; ++ay) {
        const int idx[2] = {ay == n / 2 ? n / 2 : ay, n - ay};
        const int cnt = (ay == 0 || ay == n / 2) ? 1 : 2;
        for (int u = 0; u < cnt; ++u) {
          const double2 z = a[idx[u]];
          s += (z.x * inv) * (z.x * inv) + (z.y * inv) * (z.y * inv);
        }
      }
    }
    out[b] = s;
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int yi = 0; yi < n; ++yi) {
      const double2 z = a[yi];
      s += (z.x * inv) * (z.x * inv) + (z.y * inv) * (z.y * inv);
    }
    partx[(int64_t)pair * n + kxi] = s;
  }
}

// Rows and columns longer than one LDS transform (n > kFftLds): n = n1 n2
// with n2 = kFftLds.  With x = j1 n2 + j2 and k = k1 + n1 k2 (w_m =
// exp(-2 pi i / m)),
//   X[k1 + n1 k2] = sum_j2 w_n2^(j2 k2) [w_n^(j2 k1) sum_j1 a[j1 n2 + j2] w_n1^(j1 k1)],
// so each workgroup takes one residue class k1: an n1-point DFT and a twiddle
// per element, then one n2-point FFT in LDS.  The column pass stores the
// scaled |Z|^2 per column; k_bin_cols then bins every column in the same
// order as k_fft_cols.
constexpr int kFftLds = 4096, kFftLdsBits = 12;

__device__ __forceinline__ double2 cmul_w(double2 v, double num, double den) {
  double s, c;
  sincospi(-2.0 * num / den, &s, &c);
  return make_double2(c * v.x - s * v.y, c * v.y + s * v.x);
}

__global__ void __launch_bounds__(256)
k_fft_rows_big(const double* __restrict__ mom, int n, int n1, double2* __restrict__ work) {
  extern __shared__ double2 a[];
  const int y = blockIdx.x, k1 = blockIdx.y, pair = blockIdx.z;
  const int64_t nn = (int64_t)n * n;
  for (int j2 = threadIdx.x; j2 < kFftLds; j2 += blockDim.x) {
    double2 s = make_double2(0.0, 0.0);
    for (int j1 = 0; j1 < n1; ++j1) {
      const int64_t c = (int64_t)y * n + (int64_t)j1 * kFftLds + j2;
      double re, im;
      if (pair == 0) {
        const double r = mom[c];
        re = mom[nn + c] / r;
        im = mom[2 * nn + c] / r;
      } else {
        re = mom[3 * nn + c];
        im = mom[4 * nn + c];
      }
      const double2 t = cmul_w(make_double2(re, im), double(j1 * k1), double(n1));
      s.x += t.x;
      s.y += t.y;
    }
    a[bitrev(j2, kFftLdsBits)] = cmul_w(s, double(j2) * double(k1), double(n));
  }
  fft_lds(a, kFftLds, kFftLdsBits);
  for (int k2 = threadIdx.x; k2 < kFftLds; k2 += blockDim.x)
    work[pair * nn + (int64_t)y * n + k1 + (int64_t)n1 * k2] = a[k2];
}

__global__ void __launch_bounds__(256)
k_fft_cols_big(const double2* __restrict__ work, int n, int n1, double* __restrict__ pw) {
  extern __shared__ double2 a[];
  const int kxi = column_of_block(blockIdx.x, n), k1 = blockIdx.y, pair = blockIdx.z;
  const int64_t nn = (int64_t)n * n;
  const double inv = 1.0 / (double(n) * double(n));
  for (int j2 = threadIdx.x; j2 < kFftLds; j2 += blockDim.x) {
    double2 s = make_double2(0.0, 0.0);
    for (int j1 = 0; j1 < n1; ++j1) {
      const double2 t =
          cmul_w(work[pair * nn + ((int64_t)j1 * kFftLds + j2) * n + kxi], double(j1 * k1), double(n1));
      s.x += t.x;
      s.y += t.y;
    }
    a[bitrev(j2, kFftLdsBits)] = cmul_w(s, double(j2) * double(k1), double(n));
  }
  fft_lds(a, kFftLds, kFftLdsBits);
  double* col = pw + pair * nn + (int64_t)kxi * n;
  for (int k2 = threadIdx.x; k2 < kFftLds; k2 += blockDim.x) {
    const double2 z = a[k2];
    col[k1 + (int64_t)n1 * k2] = (z.x * inv) * (z.x * inv) + (z.y * inv) * (z.y * inv);
  }
}

// Bins of one column of scaled |Z|^2 (k_fft_cols' walk and order).
__global__ void __launch_bounds__(256)
k_bin_cols(const double* __restrict__ pw, int n, int nbins, double* __restrict__ part, double* __restrict__ partx) {
  const int kxi = blockIdx.x, pair = blockIdx.y;
  const double* col = pw + (int64_t)pair * n * n + (int64_t)kxi * n;
  const int kx = kxi < n / 2 ? kxi : kxi - n;
  const int64_t kx2 = (int64_t)kx * kx;
  double* out = part + ((int64_t)pair * n + kxi) * nbins;
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    const int64_t lo = b == 0 ? 0 : (int64_t)b * b - b + 1 - kx2;
    const int64_t hi = (int64_t)b * b + b - kx2;
    double s = 0.0;
    if (hi >= 0) {
      const int a0 = lo <= 0 ? 0 : isqrt_ceil(lo);
      int a1 = isqrt_floor(hi);
      if (a1 > n / 2) a1 = n / 2;
      for (int ay = a0; ay <= a1; ++ay) {
        const int idx[2] = {ay == n / 2 ? n / 2 : ay, n - ay};
        const int cnt = (ay == 0 || ay == n / 2) ? 1 : 2;
        for (int u = 0; u < cnt; ++u) s += col[idx[u]];
      }
    }
    out[b] = s;
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int yi = 0; yi < n; ++yi) s += col[yi];
    partx[(int64_t)pair * n + kxi] = s;
  }
}

// Sums of the per-column bins in a fixed order: thread (bin, s) of a 64 x 16
// block adds the columns s, s + 16, s + 32, ... of its bin (consecutive bins
// are consecutive addresses), then the 16 partial sums are added in order of s.
__global__ void __launch_bounds__(1024)
k_spectra_final(const double* __restrict__ part, const double* __restrict__ partx, int n, int nbins,
                double* __restrict__ ek, double* __restrict__ em, double* __restrict__ ekx) {
  __shared__ double red[2][16][64];
  const int bl = threadIdx.x, sl = threadIdx.y;
  const int b = blockIdx.x * 64 + bl;
  double su = 0.0, sb = 0.0;
  if (b < nbins) {
    for (int k = sl; k < n; k += 16) {
      su += part[(int64_t)k * nbins + b];
      sb += part[((int64_t)n + k) * nbins + b];
    }
  }
  red[0][sl][bl] = su;
  red[1][sl][bl] = sb;
  __syncthreads();
  if (sl == 0 && b < nbins) {
    double tu = 0.0, tb = 0.0;
    for (int i = 0; i < 16; ++i) {
      tu += red[0][i][bl];
      tb += red[1][i][bl];
    }
    ek[b] = 0.5 * tu;
    em[b] = 0.5 * tb;
  }
  if (ekx && sl == 1 && b <= n / 2) {
    double x = partx[b];
    if (b != 0 && b != n / 2) x += partx[n - b];
    ekx[b] = 0.5 * x;
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static int train_blocks(int batch) {
  const int chunks = (batch + kTrainChunk - 1) / kTrainChunk;
  return chunks < kTrainBlocksMax ? chunks : kTrainBlocksMax;
}

// Work of a training step: packed network, per-workgroup partial gradients,
// loss partials, the reduced gradient.
size_t mlp_train_work_bytes(int batch) {
  const int blocks = train_blocks(batch);
  return (size_t)LBM_MLP_PACKED_BYTES + (size_t)blocks * kGradStride * sizeof(float) +
         ((size_t)blocks * sizeof(double) + 255) / 256 * 256 + (size_t)kGradStride * sizeof(float);
}

hipError_t launch_mlp_pack(const float* params, const lbm_mlp_norm* norm, void* packed, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((10240 + 64 + 32 + 4096 + 255) / 256), dim3(256), 0, st, params, norm,
                     static_cast<char*>(packed));
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const void* packed, const float* x, int64_t n, float* y, int32_t* ood, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t groups = (n + 31) / 32;
  int64_t blocks = (groups + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<const char*>(packed), x, n,
                     y, ood);
  return hipGetLastError();
}

hipError_t launch_mlp_gradient(const float* params, const lbm_mlp_norm* norm, const float* x, const float* t,
                               const int32_t* idx, int batch, void* work, float* grad, float* loss, hipStream_t st) {
  char* w = static_cast<char*>(work);
  const int blocks = train_blocks(batch);
  float* partial = reinterpret_cast<float*>(w + LBM_MLP_PACKED_BYTES);
  double* lpart = reinterpret_cast<double*>(w + LBM_MLP_PACKED_BYTES + (size_t)blocks * kGradStride * sizeof(float));
  hipError_t e = launch_mlp_pack(params, norm, w, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_train, dim3(blocks), dim3(128), 0, st, w, params, x, t, idx, batch, partial, lpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce_groups, dim3((LBM_MLP_PARAMS + 255) / 256, (blocks + kReduceGroup - 1) / kReduceGroup),
                     dim3(256), 0, st, partial, blocks, lpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((LBM_MLP_PARAMS + 255) / 256), dim3(256), 0, st, partial, blocks, grad, lpart,
                     loss, float(1.0 / (double(batch) * 4.0)));
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t step, double lr,
                           hipStream_t st) {
  const float bc1 = float(1.0 - pow(0.9, double(step)));
  const float bc2 = float(1.0 - pow(0.999, double(step)));
  hipLaunchKernelGGL(k_mlp_adam, dim3((LBM_MLP_PARAMS + 255) / 256), dim3(256), 0, st, params, m, v, grad, float(lr),
                     bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_mlp_train(float* params, float* m, float* v, int64_t step, double lr, const lbm_mlp_norm* norm,
                            const float* x, const float* t, const int32_t* idx, int batch, void* work,
                            float* loss, hipStream_t st) {
  const int blocks = train_blocks(batch);
  float* grad = reinterpret_cast<float*>(static_cast<char*>(work) + LBM_MLP_PACKED_BYTES +
                                         (size_t)blocks * kGradStride * sizeof(float) +
                                         ((size_t)blocks * sizeof(double) + 255) / 256 * 256);
  hipError_t e = launch_mlp_gradient(params, norm, x, t, idx, batch, work, grad, loss, st);
  if (e != hipSuccess) return e;
  return launch_mlp_adam(params, m, v, grad, step, lr, st);
}

// Training step without a caller-provided work buffer.  Its work (packed
// network, per-workgroup partial gradients, loss partials, reduced gradient;
// every byte the kernels read is written earlier in the same step, so nothing
// needs clearing) lives in this fixed device array, one copy per GPU that the
// library runs on, held until the process ends.  In host code `scratch` names
// a host-side stand-in, not device memory: kernels get the address that
// hipGetSymbolAddress returns on the current device, looked up once per device
// at the first call there.
static __device__ __align__(256) char scratch[LBM_MLP_TRAIN_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

bool mlp_train_noalloc_limit_ok(int batch) {
  return batch >= 1 && batch <= LBM_MLP_TRAIN_NOALLOC_BATCH && mlp_train_work_bytes(batch) <= sizeof(scratch);
}

hipError_t launch_mlp_train_noalloc(float* params, float* m, float* v, int64_t step, double lr,
                                    const lbm_mlp_norm* norm, const float* x, const float* t, const int32_t* idx,
                                    int batch, float* loss, hipStream_t st) {
  if (!mlp_train_noalloc_limit_ok(batch)) return hipErrorInvalidValue;
  void* work = nullptr;
  const hipError_t e = scratch_on_current_device(&work);
  if (e != hipSuccess) return e;
  return launch_mlp_train(params, m, v, step, lr, norm, x, t, idx, batch, work, loss, st);
}

size_t mlp_stats_work_bytes() { return (size_t)(kStatBlocks * 11 + 16) * sizeof(double); }

hipError_t launch_mlp_stats(const float* x, const float* t, int64_t n, lbm_mlp_norm* norm, void* work,
                            hipStream_t st) {
  double* part = static_cast<double*>(work);
  double* mean = part + kStatBlocks * 11;
  int64_t want = (n + 255) / 256;
  const int blocks = int(want < kStatBlocks ? want : kStatBlocks);
  hipLaunchKernelGGL(k_stats_pass, dim3(blocks), dim3(256), 0, st, x, t, n, (const double*)nullptr, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, part, blocks, n, mean, 0, norm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_pass, dim3(blocks), dim3(256), 0, st, x, t, n, (const double*)mean, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, part, blocks, n, mean, 1, norm);
  return hipGetLastError();
}

int filter_radius(double delta) { return (int)ceil(5.0 * (delta / sqrt(12.0))); }

size_t filter_work_bytes(int nx, int ny, int factor) {
  return 256 * sizeof(double) + (size_t)12 * (size_t)(nx / factor) * (size_t)ny * sizeof(double);
}

hipError_t launch_filter(const double* mom, int nx, int ny, int factor, double delta, double* out, void* work,
                         hipStream_t st) {
  const int R = filter_radius(delta);
  double* taps = static_cast<double*>(work);
  double* tmp = taps + 256;
  hipLaunchKernelGGL(k_gauss_taps, dim3(1), dim3(256), 0, st, delta * delta / 12.0, R, taps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int cx = nx / factor, cy = ny / factor;
  hipLaunchKernelGGL(k_filter_x, dim3((cx + 63) / 64, ny), dim3(64), 0, st, mom, nx, ny, factor, R, taps, tmp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_filter_y, dim3((cx + 63) / 64, cy, 12), dim3(64), 0, st, tmp, nx, ny, factor, R, taps, out);
  return hipGetLastError();
}

hipError_t launch_closure_samples(const double* c12, int nx, int ny, double delta, int stencil, float* x, float* t,
                                  hipStream_t st) {
  const dim3 g((nx + 63) / 64, (ny + 3) / 4), b(64, 4);
  const double k2 = delta * delta / 12.0;
  if (stencil == LBM_STENCIL_ISO9)
    hipLaunchKernelGGL(k_closure_samples<LBM_STENCIL_ISO9>, g, b, 0, st, c12, nx, ny, k2, x, t);
  else
    hipLaunchKernelGGL(k_closure_samples<LBM_STENCIL_CENTRAL5>, g, b, 0, st, c12, nx, ny, k2, x, t);
  return hipGetLastError();
}

hipError_t launch_mlp_correct(const void* cell_in, const void* packed, float* corr, int nx, int ny, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_correct, dim3((nx + kCorrTX - 1) / kCorrTX, (ny + kCorrTY - 1) / kCorrTY), dim3(256), 0, st,
                     static_cast<const CellIn*>(cell_in), static_cast<const char*>(packed), corr, nx, ny);
  return hipGetLastError();
}

int spectra_bins(int n) { return (int)floor(sqrt(2.0) * double(n / 2) + 0.5) + 1; }

size_t spectra_work_bytes(int n) {
  const size_t nn = (size_t)n * n;
  const size_t big = n > kFftLds ? 2 * nn * sizeof(double) : 0;  // scaled |Z|^2 of the long columns
  return 2 * nn * sizeof(double2) + big + (size_t)2 * n * spectra_bins(n) * sizeof(double) +
         (size_t)2 * n * sizeof(double);
}

hipError_t launch_spectra(const double* mom, int n, double* ek, double* em, double* ekx, void* work, hipStream_t st) {
  int bits = 0;
  while ((1 << bits) < n) ++bits;
  const int nb = spectra_bins(n);
  double2* cw = static_cast<double2*>(work);
  double* part = reinterpret_cast<double*>(cw + (size_t)2 * n * n);
  hipError_t e;
  if (n <= kFftLds) {
    double* partx = part + (size_t)2 * n * nb;
    const size_t lds = (size_t)n * sizeof(double2);
    hipLaunchKernelGGL(k_fft_rows, dim3(n, 2), dim3(256), lds, st, mom, n, bits, cw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fft_cols, dim3(n, 2), dim3(256), lds, st, cw, n, bits, nb, part, partx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    double* pw = part;
    part = pw + (size_t)2 * n * n;
    const int n1 = n / kFftLds;
    const size_t lds = (size_t)kFftLds * sizeof(double2);
    hipLaunchKernelGGL(k_fft_rows_big, dim3(n, n1, 2), dim3(256), lds, st, mom, n, n1, cw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_fft_cols_big, dim3(n, n1, 2), dim3(256), lds, st, cw, n, n1, pw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_cols, dim3(n, 2), dim3(256), 0, st, pw, n, nb, part, part + (size_t)2 * n * nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  double* partx = part + (size_t)2 * n * nb;
  const int fin = (nb > n / 2 + 1 ? nb : n / 2 + 1);
  hipLaunchKernelGGL(k_spectra_final, dim3((fin + 63) / 64), dim3(64, 16), 0, st, part, partx, n, nb, ek, em, ekx);
  return hipGetLastError();
}

}  // namespace lbm
