// Device helpers of the learned correction's network (63 -> 64 -> 64 -> 4
// on the matrix cores): operand types, the packed-network layout, and one
// wave's forward pass over 32 cells.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbmhd_learned.h"

namespace lbm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Eight floats rounded to bfloat16 (nearest even), two per conversion.
__device__ __forceinline__ unsigned pack2_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ bf16x8 to_bf16x8(const f32x8& v) {
  const u32x4 u = {pack2_bf16(v[0], v[1]), pack2_bf16(v[2], v[3]), pack2_bf16(v[4], v[5]), pack2_bf16(v[6], v[7])};
  return __builtin_bit_cast(bf16x8, u);
}

// Packed network (LBM_MLP_PACKED_BYTES): bfloat16 A operands in lane order,
// FP32 biases, the normalisation.
constexpr int kPkA1 = 0;       // [ot 2][kb 4][lane 64][8] bf16
constexpr int kPkA2 = 8192;    // [ot 2][kb 4][lane 64][8] bf16
constexpr int kPkA3 = 16384;   // [kb 4][lane 64][8] bf16 (rows >= 4 zero)
constexpr int kPkB1 = 20480;   // 64 floats
constexpr int kPkB2 = 20736;   // 64 floats
constexpr int kPkB3 = 20992;   // 4 floats (+ pad)
constexpr int kPkNorm = 21248;  // lbm_mlp_norm
// Layer 1 of the state-correction kernel, whose inputs come from the 3x3
// patch of per-cell input vectors (CellIn below).  Contraction block kb of
// lane half h holds patch position p = 2 kb + h (pos = 3 row + column):
// element j < 7 is field j at p, element 7 is field p at position 8 (none
// for p = 7), so the 63 inputs fill four 16-wide blocks.  [ot 2][kb 4][lane
// 64][8] bf16.
constexpr int kPkA1n = 21504;
static_assert(kPkNorm + (int)sizeof(lbm_mlp_norm) <= kPkA1n, "packed layout");
static_assert(kPkA1n + 2 * 4 * 64 * 16 <= LBM_MLP_PACKED_BYTES, "packed size");
static_assert(sizeof(lbm_mlp_norm) == 128, "norm size");

constexpr float kOodLimit = 6.0f;

// Hidden row held by accumulator register i of lane half h (one 32-row tile).
__host__ __device__ constexpr int acc_row(int i, int h) { return (i / 4) * 8 + h * 4 + i % 4; }
// Contraction index of element j of lane half h in 16-wide block kb of a
// layer fed by accumulator registers (layers 2 and 3).
__host__ __device__ constexpr int chained_k(int kb, int h, int j) {
  return (kb / 2) * 32 + (2 * (kb % 2) + j / 4) * 8 + h * 4 + j % 4;
}
static_assert(chained_k(1, 0, 0) == 16 && chained_k(0, 1, 4) == 12 && chained_k(3, 1, 7) == 63, "chain");

// Field of feature k < 63 (k / 9) and its 3x3 offset, by multiply-shift.
__device__ __forceinline__ int feat_field(int k) { return (k * 57) >> 9; }

__device__ __forceinline__ float bf16_round(float v) { return float(__bf16(v)); }

// A operands of the three layers; KB1 16-wide contraction blocks in layer 1.
template <int KB1>
struct MlpW {
  bf16x8 a1[2][KB1], a2[2][4], a3[4];
};
using MlpA = MlpW<4>;

__device__ __forceinline__ void load_mlp_at(const char* __restrict__ pk, int a1_off, int lane, MlpA& w) {
  const bf16x8* p1 = reinterpret_cast<const bf16x8*>(pk + a1_off);
  const bf16x8* p2 = reinterpret_cast<const bf16x8*>(pk + kPkA2);
  const bf16x8* p3 = reinterpret_cast<const bf16x8*>(pk + kPkA3);
#pragma unroll
  for (int ot = 0; ot < 2; ++ot)
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      w.a1[ot][kb] = p1[(ot * 4 + kb) * 64 + lane];
      w.a2[ot][kb] = p2[(ot * 4 + kb) * 64 + lane];
    }
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) w.a3[kb] = p3[kb * 64 + lane];
}

// Network on feature rows (layer 1 in feature order).
__device__ __forceinline__ void load_mlp(const char* __restrict__ pk, int lane, MlpA& w) {
  load_mlp_at(pk, kPkA1, lane, w);
}

// Network of the state-correction kernel (layer 1 in patch order).
__device__ __forceinline__ void load_mlp_n(const char* __restrict__ pk, int lane, MlpA& w) {
  load_mlp_at(pk, kPkA1n, lane, w);
}

// Per-cell input vector of the state-correction kernel (16 bytes): the seven
// normalised fields rounded to bfloat16, and in element 7 a flag, nonzero
// when any of them is out of range (|z| > kOodLimit or not finite).
using CellIn = bf16x8;
constexpr unsigned short kCellOutOfRange = 0x3F80;  // bfloat16 1.0

// Layer-1 B operands of lane half h from the input vectors of patch
// positions 2 kb + h (v[kb]) and 8 (v8), in the kPkA1n order; *bad is set
// when any of these five cells carries the out-of-range flag.
__device__ __forceinline__ void patch_operands(const CellIn v[4], const CellIn& v8, int h, bf16x8 zb[4], bool* bad) {
  const u32x4 w8 = __builtin_bit_cast(u32x4, v8);
  unsigned flags = w8[3] >> 16;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    u32x4 w = __builtin_bit_cast(u32x4, v[kb]);
    flags |= w[3] >> 16;
    // field 2 kb + h of position 8: low or high half of its word kb (word 3
    // high is the flag, not a field: position 7 takes no extra input)
    const unsigned extra = h ? (kb == 3 ? 0u : (w8[kb] & 0xFFFF0000u)) : (w8[kb] << 16);
    w[3] = (w[3] & 0xFFFFu) | extra;
    zb[kb] = __builtin_bit_cast(bf16x8, w);
  }
  *bad = flags != 0;
}

// Accumulator of one 32-row tile preset to the bias of its rows.
__device__ __forceinline__ f32x16 bias_tile(const float* __restrict__ b, int ot, int h) {
  f32x16 acc;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(b + ot * 32 + g * 8 + h * 4);
    acc[g * 4 + 0] = v[0];
    acc[g * 4 + 1] = v[1];
    acc[g * 4 + 2] = v[2];
    acc[g * 4 + 3] = v[3];
  }
  return acc;
}

typedef short i16x8 __attribute__((ext_vector_type(8)));

// ReLU of two accumulator tiles, rounded to bfloat16, as the four B operands
// of the next layer.  Rounding is monotonic and keeps the sign, so the ReLU
// is taken after it, on the packed bfloat16 bit patterns read as int16
// (negative values, -0 included, are negative int16 and become +0).  The
// rounded values go to hout (as floats) when given.
__device__ __forceinline__ void activate(const f32x16 acc[2], bf16x8 hb[4], float* hout) {
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    f32x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = acc[kb / 2][(kb % 2) * 8 + j];
    const bf16x8 v = to_bf16x8(a);
    const i16x8 bits = __builtin_elementwise_max(__builtin_bit_cast(i16x8, v), i16x8(0));
    hb[kb] = __builtin_bit_cast(bf16x8, bits);
    if (hout) {
#pragma unroll
      for (int j = 0; j < 8; ++j) hout[kb * 8 + j] = float(hb[kb][j]);
    }
  }
}

// The network on the 32 cells of a wave: zb = layer-1 B operands of this lane
// (cell lane % 32, inputs kb*16 + (lane/32)*8 + j in layer 1's contraction
// order).  Returns y in lanes 0..31 (components 0..3).  h1, h2 (32 floats
// each, may be null) receive the bfloat16 activations held by this lane,
// element kb*8 + j = hidden chained_k(kb, lane/32, j).
// Biases: b points at b1 (64 floats), b2 (64) and b3 (4) back to back, in
// LDS or global memory.
template <int KB1>
__device__ __forceinline__ f32x4 mlp_wave(const MlpW<KB1>& w, const bf16x8 zb[KB1], const float* __restrict__ b,
                                          int lane, float* h1, float* h2) {
  const int h = lane >> 5;
  const float* b1 = b;
  const float* b2 = b + 64;
  const float* b3 = b + 128;
  f32x16 acc[2];
  bf16x8 hb[4];
#pragma unroll
  for (int ot = 0; ot < 2; ++ot) {
    acc[ot] = bias_tile(b1, ot, h);
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb)
      acc[ot] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w.a1[ot][kb], zb[kb], acc[ot], 0, 0, 0);
  }
  activate(acc, hb, h1);
#pragma unroll
  for (int ot = 0; ot < 2; ++ot) {
    acc[ot] = bias_tile(b2, ot, h);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc[ot] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w.a2[ot][kb], hb[kb], acc[ot], 0, 0, 0);
  }
  activate(acc, hb, h2);
  f32x16 out;
#pragma unroll
  for (int i = 0; i < 16; ++i) out[i] = 0.0f;
  if (h == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = b3[i];
  }
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w.a3[kb], hb[kb], out, 0, 0, 0);
  f32x4 y;
  y[0] = out[0];
  y[1] = out[1];
  y[2] = out[2];
  y[3] = out[3];
  return y;
}

}  // namespace lbm
