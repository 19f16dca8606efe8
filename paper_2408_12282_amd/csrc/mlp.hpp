// mlp.hpp -- the per-pixel residual network (Sec. 3.2, Eq. 6) on the matrix
// cores, one wavefront per 64 pixels.
//
// Layers are computed transposed, Y^T = W X^T: M = output features, N = the
// wave's 64 pixels (4 blocks of 16), K = input features.  The 16x16 MFMA
// result leaves lane (pixel p, group g) holding outputs 4g..4g+3 of each
// 16-row block; instead of transposing, the next layer consumes those
// registers directly as its B operand and the weights are stored with the
// matching permutation of K (done once per call by the prep kernel).
//
// Two arithmetic forms share the code: FP32 operands on v_mfma_f32_16x16x4_f32
// and BF16 operands on v_mfma_f32_16x16x32_bf16, both with FP32 accumulation.
// In the BF16 form the weights are single BF16 numbers and an activation
// enters a forward product as two, hi = RNE(x) and lo = RNE(x - hi) (two
// products per k-step, 16 significant bits of the activation): a single
// rounding would turn differences of an FP32 ulp in the input into jumps of a
// BF16 ulp, which the high octaves of the position encoding make frequent.
// Weight gradients and upstream gradients use single BF16 numbers.
#pragma once
#include "common.hpp"

namespace sssgs {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// Eight floats to an eight-element BF16 operand, rounded to nearest even in
// pairs (one v_cvt_pk_bf16_f32 per pair, no repacking of halves).
__device__ __forceinline__ bf16x8 pack_bf16x8(float v0, float v1, float v2, float v3, float v4, float v5, float v6,
                                              float v7) {
  const bf16x2v p0 = __builtin_convertvector((f32x2v){v0, v1}, bf16x2v);
  const bf16x2v p1 = __builtin_convertvector((f32x2v){v2, v3}, bf16x2v);
  const bf16x2v p2 = __builtin_convertvector((f32x2v){v4, v5}, bf16x2v);
  const bf16x2v p3 = __builtin_convertvector((f32x2v){v6, v7}, bf16x2v);
  const uint4 u = make_uint4(__builtin_bit_cast(uint32_t, p0), __builtin_bit_cast(uint32_t, p1),
                             __builtin_bit_cast(uint32_t, p2), __builtin_bit_cast(uint32_t, p3));
  return __builtin_bit_cast(bf16x8, u);
}

// hi = RNE(v), lo = RNE(v - hi) of eight floats; v - hi is exact in FP32.
__device__ __forceinline__ void pack_bf16x8_split(const float (&v)[8], bf16x8 &hi, bf16x8 &lo) {
  hi = pack_bf16x8(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
  float r[8];
#pragma unroll
  for (int j = 0; j < 8; j++) r[j] = v[j] - (float)hi[j];
  lo = pack_bf16x8(r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7]);
}

struct MmaF32 {
  static constexpr int KS = 4;   // K per instruction
  static constexpr int KPL = 1;  // K elements held per lane
  static constexpr int NSPLIT = 1;  // numbers per activation in a forward product
  using Op = float;
  using Elem = float;
  __device__ static __forceinline__ f32x4 mma(Op a, Op b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ Elem cvt(float v) { return v; }
  __device__ static __forceinline__ float back(Elem v) { return v; }
};

struct MmaBF16 {
  static constexpr int KS = 32;
  static constexpr int KPL = 8;
  static constexpr int NSPLIT = 2;
  using Op = bf16x8;
  using Elem = __bf16;
  __device__ static __forceinline__ f32x4 mma(Op a, Op b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ Elem cvt(float v) { return (__bf16)v; }
  __device__ static __forceinline__ float back(Elem v) { return (float)v; }
};

// Input feature index of element j of k-step ks for lane group g.
//  layer 0 (input read from LDS):   natural order
//  layers >= 1 (input from the previous layer's accumulators): permuted
template <class M>
__host__ __device__ constexpr int feat_index(bool natural, int ks, int g, int j) {
  if (natural) return ks * M::KS + g * M::KPL + j;
  if (M::KPL == 8) return 32 * ks + 16 * (j >> 2) + 4 * g + (j & 3);
  return 16 * (ks >> 2) + 4 * g + (ks & 3);
}

// Prepared (permuted, converted) weights of one network.
template <class M, int WIDTH, int IN_PAD>
struct NetShape {
  static constexpr int MB = WIDTH / 16;          // 16-row blocks of a hidden layer
  static constexpr int KS0 = IN_PAD / M::KS;     // k-steps of layer 0
  static constexpr int KSH = WIDTH / M::KS;      // k-steps of layers >= 1
  static constexpr int L0 = MB * KS0 * 64;       // operands of layer 0
  static constexpr int LH = MB * KSH * 64;       // operands of a hidden layer
  static constexpr int LO = 1 * KSH * 64;        // operands of the output layer (6 rows in a 16-row block)
  static constexpr int total_ops(int hidden) { return L0 + (hidden - 1) * LH + LO; }
  // transposed layers of the backward (dX^T = W^T dY^T), k = output features of the forward layer
  static constexpr int KT_H = WIDTH / M::KS;     // k-steps over a hidden layer's outputs
  static constexpr int KT_O = (16 + M::KS - 1) / M::KS;  // k-steps over the padded output block
  static constexpr int MB0 = IN_PAD / 16;        // 16-row blocks of layer 0's input
  static constexpr int T0 = MB0 * KT_H * 64;     // W0^T operands
  static constexpr int TH = MB * KT_H * 64;      // W^T operands of a hidden layer
  static constexpr int TO = MB * KT_O * 64;      // W_out^T operands
  static constexpr int total_tops(int hidden) { return T0 + (hidden - 1) * TH + TO; }
};

}  // namespace sssgs
