// net_bwd.hpp -- wave-level pieces of the network backward (Sec. 3.2,
// Eq. 6) shared by the shading backward and the weight-gradient kernel:
// layer products on the matrix cores, ReLU masks, and the packing of a
// masked gradient into the next product's B operands.
#pragma once
#include "shade_common.hpp"

namespace sssgs {

// B-operand packing of a masked upstream gradient (D layout -> permuted K).
template <class M, int MB>
__device__ __forceinline__ void grad_to_ops(const f32x4 (&d)[MB][4], typename M::Op (&B)[(MB * 16) / M::KS][4]) {
  constexpr int KSN = (MB * 16) / M::KS;
#pragma unroll
  for (int ks = 0; ks < KSN; ks++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      if constexpr (M::KPL == 8) {
        const f32x4 &lo = d[2 * ks][nb], &hi = d[2 * ks + 1][nb];
        B[ks][nb] = pack_bf16x8(lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]);
      } else {
        B[ks][nb] = d[ks >> 2][nb][ks & 3];
      }
    }
}

// One product from single B operands H (K = KSN k-steps) to accumulators:
// the gradient products of the backward (dX^T = W^T dY^T).
template <class M, int MB, int KSN>
__device__ __forceinline__ void layer_mma(const typename M::Op *__restrict__ w, const typename M::Op (&H)[KSN][4],
                                          f32x4 (&acc)[MB][4], int lane) {
  // the first k-step takes a literal zero accumulator (an inline constant, no register clears)
#pragma unroll
  for (int ks = 0; ks < KSN; ks++)
#pragma unroll
    for (int mb = 0; mb < MB; mb++) {
      const typename M::Op a = w[(mb * KSN + ks) * 64 + lane];
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
        acc[mb][nb] = M::mma(a, H[ks][nb], ks == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[mb][nb]);
    }
}

// ReLU masks of one layer's outputs in D layout, one bit per (mb, nb, j).
template <int MB>
struct Mask {
  uint32_t w[(MB * 16 + 31) / 32];
  __device__ __forceinline__ void set_from(const f32x4 (&acc)[MB][4], const float *bias, int g) {
#pragma unroll
    for (int k = 0; k < (MB * 16 + 31) / 32; k++) w[k] = 0u;
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int b = mb * 16 + nb * 4 + j;
          if (acc[mb][nb][j] + bias[16 * mb + 4 * g + j] > 0.f) w[b >> 5] |= 1u << (b & 31);
        }
  }
  // From a layer's BF16 activation operands (permuted K order: operand slot
  // 4 (mb & 1) + j holds D-layout element (mb, nb, j)): the bit is set where
  // the activation is positive.  A BF16 half is positive iff, as the top half
  // of a signed 32-bit word, it is above zero.  This equals the pre-activation
  // test except below the smallest BF16 subnormal, and it lets the
  // pre-activations die as soon as the activations are packed.
  __device__ __forceinline__ void set_from_ops(const bf16x8 (&H)[(MB + 1) / 2][4]) {
#pragma unroll
    for (int k = 0; k < (MB * 16 + 31) / 32; k++) w[k] = 0u;
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
      for (int nb = 0; nb < 4; nb++) {
        const uint4 u = __builtin_bit_cast(uint4, H[mb >> 1][nb]);
        const uint32_t w0 = (mb & 1) ? u.z : u.x, w1 = (mb & 1) ? u.w : u.y;
        const uint32_t bits = (uint32_t)((int)(w0 << 16) > 0) | ((uint32_t)((int)w0 > 0xFFFF) << 1) |
                              ((uint32_t)((int)(w1 << 16) > 0) << 2) | ((uint32_t)((int)w1 > 0xFFFF) << 3);
        const int b = mb * 16 + nb * 4;
        w[b >> 5] |= bits << (b & 31);
      }
  }
  // Materialise the words here: otherwise the compiler may sink the
  // comparisons to the masks' use in the backward and keep the forward's
  // accumulators alive until then.
  __device__ __forceinline__ void pin() {
#pragma unroll
    for (int k = 0; k < (MB * 16 + 31) / 32; k++) asm volatile("" : "+v"(w[k]));
  }
  __device__ __forceinline__ void apply(f32x4 (&d)[MB][4]) const {
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int b = mb * 16 + nb * 4 + j;
          if (!((w[b >> 5] >> (b & 31)) & 1u)) d[mb][nb][j] = 0.f;
        }
  }
};

}  // namespace sssgs
