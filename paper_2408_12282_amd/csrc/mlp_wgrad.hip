// mlp_wgrad.hip -- weight and bias gradients of the per-pixel network
// (Sec. 3.2, Eq. 6), BF16 operands, width 64, three hidden layers.
//
// Input: the strip records of the split shading backward, i.e. per 64-pixel
// strip the BF16 network input rows as layer 0 reads them and the BF16
// gradients of the six network outputs.  Each wave takes whole strips: it
// recomputes the forward (for the activations and ReLU masks), runs the
// backward through the hidden layers, and adds
//   dW_l += dY_l^T X_l,   db_l += sum over pixels of dY_l
// for all four layers into accumulators that stay in registers across all
// its strips (221 floats per lane at input width 64).
//
// The products of the forward keep features along K (B operands: lane =
// pixel, eight features per lane).  The weight gradient contracts over
// pixels, so each 16x16 block is turned around by one 16x16x16 MFMA against
// the identity, which is exact (every product is x * 1 or x * 0 and the sum
// has a single non-zero term): the result leaves lane (feature f, group g)
// holding pixels 4g .. 4g+3 of the block, which is the operand form with
// pixels along K.
//
// Weights are staged in LDS once per workgroup.  Strips go to waves in a
// fixed pattern and the four waves of a workgroup add their sums into the
// workgroup's partial in a fixed order, so the result does not depend on
// timing.
#include "launch.hpp"
#include "net_bwd.hpp"

namespace sssgs {

namespace {

typedef short s16x4 __attribute__((ext_vector_type(4)));

constexpr int kWgradWaves = 4;

// Bits of BF16 1.0.
constexpr short kBf16One = 0x3F80;

// Half h (elements 4h .. 4h+3) of an eight-element operand, as the operand
// of the 16x16x16 instruction.
__device__ __forceinline__ s16x4 half_op(bf16x8 v, int h) {
  const s16x4 *p = reinterpret_cast<const s16x4 *>(&v);
  return p[h];
}

// D[p][n] = A[p][n]: pixel-row form of a 16-pixel x 16-feature block.
__device__ __forceinline__ f32x4 turn(s16x4 a, s16x4 eye) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, eye, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
}

// Operand with pixels along K from two pixel-row blocks: slot j of lane
// (f, g) is pixel 4g + (j & 3) of block 2kk + (j >> 2).
__device__ __forceinline__ bf16x8 pack_px(const f32x4 &lo, const f32x4 &hi) {
  return pack_bf16x8(lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]);
}

// The 16-feature block fb (= 2 ks + h) of features-along-K operands H[ks][nb]
// in pixels-along-K form P[kk] (pixels 32 kk .. 32 kk + 31); optionally adds
// the lane's share of the pixel sum to *sum.
__device__ __forceinline__ void block_px(const bf16x8 (&Hks)[4], int h, s16x4 eye, bf16x8 (&P)[2], float *sum) {
  f32x4 t[4];
#pragma unroll
  for (int nb = 0; nb < 4; nb++) t[nb] = turn(half_op(Hks[nb], h), eye);
  P[0] = pack_px(t[0], t[1]);
  P[1] = pack_px(t[2], t[3]);
  if (sum) {
    float s = 0.f;
#pragma unroll
    for (int nb = 0; nb < 4; nb++) s += (t[nb][0] + t[nb][1]) + (t[nb][2] + t[nb][3]);
    *sum += s;
  }
}

// dW[ob][ib] += dY^T X over the strip for a layer with NOB 16-row blocks
// of outputs and NIB 16-column blocks of inputs; db[ob] += pixel sums.
template <int NOB, int NIB>
__device__ __forceinline__ void layer_wgrad(const bf16x8 (&dY)[(NOB + 1) / 2][4], const bf16x8 (&X)[NIB / 2][4],
                                            s16x4 eye, f32x4 (&dW)[NOB][NIB], float (&db)[NOB]) {
  bf16x8 PY[NOB][2];
#pragma unroll
  for (int ob = 0; ob < NOB; ob++) block_px(dY[ob >> 1], ob & 1, eye, PY[ob], &db[ob]);
#pragma unroll
  for (int ib = 0; ib < NIB; ib++) {
    bf16x8 PX[2];
    block_px(X[ib >> 1], ib & 1, eye, PX, nullptr);
#pragma unroll
    for (int ob = 0; ob < NOB; ob++)
#pragma unroll
      for (int kk = 0; kk < 2; kk++) dW[ob][ib] = MmaBF16::mma(PY[ob][kk], PX[kk], dW[ob][ib]);
  }
}

// ReLU derivative from the layer's BF16 activations: zero d where the
// activation is not positive.  The activation operands H[ks][nb] hold, in
// slot 4 (mb & 1) + j, the feature that D-layout element (mb, nb, j) holds
// (both use the permuted K order), so the test needs no data movement.  A
// BF16 half is positive iff, read as the top half of a signed 32-bit word,
// it is above zero.  (This equals the pre-activation test except for
// pre-activations below the smallest BF16 subnormal.)
template <int MB>
__device__ __forceinline__ void relu_mask_from_ops(const bf16x8 (&H)[MB / 2][4], f32x4 (&d)[MB][4]) {
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      const uint4 u = __builtin_bit_cast(uint4, H[mb >> 1][nb]);
      const uint32_t w0 = (mb & 1) ? u.z : u.x, w1 = (mb & 1) ? u.w : u.y;
      if (!((int)(w0 << 16) > 0)) d[mb][nb][0] = 0.f;
      if (!((int)w0 > 0xFFFF)) d[mb][nb][1] = 0.f;
      if (!((int)(w1 << 16) > 0)) d[mb][nb][2] = 0.f;
      if (!((int)w1 > 0xFFFF)) d[mb][nb][3] = 0.f;
    }
}

// Layer-0 B operands of a strip from its record rows ([64][stride] BF16).
template <int KS0>
__device__ __forceinline__ void load_rows(const __bf16 *xr, int stride, bf16x8 (&X)[KS0][4], int g, int col) {
#pragma unroll
  for (int ks = 0; ks < KS0; ks++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
      X[ks][nb] = *reinterpret_cast<const bf16x8 *>(xr + (16 * nb + col) * stride + ks * 32 + g * 8);
}

// LDS of a workgroup (input width 64): forward weight operands and biases
// (shared); per wave the layer-1 and layer-2 activations of the current strip
// and the layer-1 weight-gradient sums (the other sums stay in registers).
// After the strips, the front of it holds the workgroup's total.
struct WgradLds {
  using NS = NetShape<MmaBF16, 64, 64>;
  using PO = ParamOffsets<64, 64>;
  static constexpr int NOPS = NS::total_ops(3);  // forward operands (16 B each)
  static constexpr int NBIAS = 3 * 64 + 8;       // b0 | b1 | b2 | b3 (6, padded to 8)
  static constexpr int HOPS = 2 * NS::KSH * 4 * 64;  // H1, H2 operands of one wave
  static constexpr int DW1 = NS::MB * NS::MB * 64;   // layer-1 sums of one wave (f32x4)
  static constexpr int OFF_B = NOPS * 16;
  static constexpr int OFF_H = OFF_B + NBIAS * 4;
  static constexpr int OFF_D = OFF_H + kWgradWaves * HOPS * 16;
  static constexpr int BYTES = OFF_D + kWgradWaves * DW1 * 16;
  static_assert(PO::total() * 4 <= OFF_D, "workgroup total must not overlap the layer-1 sums");
  static_assert(OFF_H % 16 == 0, "operand alignment");
};

// Input feature of column col of 16-column block ib of layer 0, whose
// operands hold features in natural order (8 consecutive per lane group).
__device__ __forceinline__ int l0_feature(int ib, int col) {
  return 32 * (ib >> 1) + 8 * (col >> 2) + 4 * (ib & 1) + (col & 3);
}

__device__ __forceinline__ void store_ops(bf16x8 *dst, const bf16x8 (&H)[2][4], int lane) {
#pragma unroll
  for (int ks = 0; ks < 2; ks++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) dst[(ks * 4 + nb) * 64 + lane] = H[ks][nb];
}

__device__ __forceinline__ void load_ops(const bf16x8 *src, bf16x8 (&H)[2][4], int lane) {
#pragma unroll
  for (int ks = 0; ks < 2; ks++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) H[ks][nb] = src[(ks * 4 + nb) * 64 + lane];
}

// Layer 1 (64 x 64): the strip's dY^T X added to the wave's sums in LDS.
__device__ __forceinline__ void layer1_wgrad_lds(const bf16x8 (&dY)[2][4], const bf16x8 (&X)[2][4], s16x4 eye,
                                                 f32x4 *d1, float (&db)[4], int lane) {
  bf16x8 PY[4][2];
#pragma unroll
  for (int ob = 0; ob < 4; ob++) block_px(dY[ob >> 1], ob & 1, eye, PY[ob], &db[ob]);
#pragma unroll
  for (int ib = 0; ib < 4; ib++) {
    bf16x8 PX[2];
    block_px(X[ib >> 1], ib & 1, eye, PX, nullptr);
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
      f32x4 t = d1[(ob * 4 + ib) * 64 + lane];
#pragma unroll
      for (int kk = 0; kk < 2; kk++) t = MmaBF16::mma(PY[ob][kk], PX[kk], t);
      d1[(ob * 4 + ib) * 64 + lane] = t;
    }
  }
}

__global__ __launch_bounds__(kWgradWaves * 64, 1) void mlp_wgrad_kernel(const void *__restrict__ wops_g,
                                                                       const void *__restrict__ tops_g,
                                                                       const float *__restrict__ params,
                                                                       const __bf16 *__restrict__ rec_x,
                                                                       const __bf16 *__restrict__ rec_o,
                                                                       int nstrips, float *__restrict__ partials) {
  using M = MmaBF16;
  using Op = bf16x8;
  using SL = WgradLds;
  using NS = SL::NS;
  using PO = SL::PO;
  constexpr int IN_PAD = 64;
  constexpr int MB = NS::MB, KS0 = NS::KS0, KSH = NS::KSH, IB0 = IN_PAD / 16;
  static_assert(KSH == 2 && KS0 == 2, "width-64 network with 64 inputs");
  __shared__ __attribute__((aligned(16))) char lds[SL::BYTES];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  Op *wl_base = reinterpret_cast<Op *>(lds);
  float *bl = reinterpret_cast<float *>(lds + SL::OFF_B);
  Op *hs = reinterpret_cast<Op *>(lds + SL::OFF_H) + w * SL::HOPS;  // H1 | H2
  f32x4 *d1 = reinterpret_cast<f32x4 *>(lds + SL::OFF_D) + w * SL::DW1;
  float *red = reinterpret_cast<float *>(lds);  // after the strips
  const Op *tops_base = reinterpret_cast<const Op *>(tops_g);

  {
    const uint4 *sw = reinterpret_cast<const uint4 *>(wops_g);
    uint4 *dw = reinterpret_cast<uint4 *>(wl_base);
    for (int i = threadIdx.x; i < SL::NOPS; i += blockDim.x) dw[i] = sw[i];
    for (int i = threadIdx.x; i < SL::NBIAS; i += blockDim.x) {
      const int l = i >> 6, o = i & 63;
      bl[i] = l < 3 ? params[PO::b(l) + o] : (o < 6 ? params[PO::b(3) + o] : 0.f);
    }
    for (int i = lane; i < SL::DW1; i += 64) d1[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  __syncthreads();

  s16x4 eye;
#pragma unroll
  for (int j = 0; j < 4; j++) eye[j] = (4 * g + j == col) ? kBf16One : (short)0;

  f32x4 dW0[MB][IB0], dW2[MB][MB], dW3[1][MB];
  float db0[MB], db1[MB], db2[MB], db3[1];
#pragma unroll
  for (int ob = 0; ob < MB; ob++) {
#pragma unroll
    for (int ib = 0; ib < IB0; ib++) dW0[ob][ib] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ib = 0; ib < MB; ib++) dW2[ob][ib] = f32x4{0.f, 0.f, 0.f, 0.f};
    dW3[0][ob] = f32x4{0.f, 0.f, 0.f, 0.f};
    db0[ob] = db1[ob] = db2[ob] = 0.f;
  }
  db3[0] = 0.f;

#pragma unroll 1
  for (int s = blockIdx.x * kWgradWaves + w; s < nstrips; s += gridDim.x * kWgradWaves) {
    const __bf16 *xr = rec_x + (size_t)s * 64 * IN_PAD;
    const __bf16 *orow = rec_o + (size_t)s * 64 * 8;
    // Weight operands are re-read for every strip (LDS and L2 hits): an
    // opaque zero offset keeps the compiler from hoisting those loop-invariant
    // loads out of the loop, which would pin them in registers.
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    const Op *wl = wl_base + z;
    const Op *tops = tops_base + z;
    // forward: activations (H1, H2 to LDS)
    Op H3[KSH][4];
    {
      Op X0[KS0][4];
      load_rows<KS0>(xr, IN_PAD, X0, g, col);
      f32x4 acc[MB][4];
      Op H[KSH][4];
#pragma unroll
      for (int ks = 0; ks < KS0; ks++)
#pragma unroll
        for (int mb = 0; mb < MB; mb++) {
          const Op a = wl[(mb * KS0 + ks) * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < 4; nb++)
            acc[mb][nb] = M::mma(a, X0[ks][nb], ks == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[mb][nb]);
        }
      acc_to_ops<M, MB>(acc, bl, g, H);
      store_ops(hs, H, lane);
      layer_mma<M, MB, KSH>(wl + NS::L0, H, acc, lane);
      acc_to_ops<M, MB>(acc, bl + 64, g, H);
      store_ops(hs + KSH * 4 * 64, H, lane);
      layer_mma<M, MB, KSH>(wl + NS::L0 + NS::LH, H, acc, lane);
      acc_to_ops<M, MB>(acc, bl + 128, g, H3);
    }
    // output layer: dY = output gradients, X = H3 (one 16-row block, rows 0..5)
    Op Bo[1][4];
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      uint2 v = make_uint2(0u, 0u);
      if (g < 2) v = *reinterpret_cast<const uint2 *>(orow + (16 * nb + col) * 8 + 4 * g);
      Bo[0][nb] = __builtin_bit_cast(bf16x8, make_uint4(v.x, v.y, 0u, 0u));
    }
    layer_wgrad<1, MB>(Bo, H3, eye, dW3, db3);
    f32x4 dH[MB][4];
    Op Bd[KSH][4];
    layer_mma<M, MB, NS::KT_O>(tops + NS::T0 + 2 * NS::TH, Bo, dH, lane);
    relu_mask_from_ops<MB>(H3, dH);
    grad_to_ops<M, MB>(dH, Bd);
    {
      Op X[KSH][4];
      load_ops(hs + KSH * 4 * 64, X, lane);  // H2
      layer_wgrad<MB, MB>(Bd, X, eye, dW2, db2);
      layer_mma<M, MB, NS::KT_H>(tops + NS::T0 + NS::TH, Bd, dH, lane);
      relu_mask_from_ops<MB>(X, dH);
    }
    grad_to_ops<M, MB>(dH, Bd);
    {
      Op X[KSH][4];
      load_ops(hs, X, lane);  // H1
      layer1_wgrad_lds(Bd, X, eye, d1, db1, lane);
      layer_mma<M, MB, NS::KT_H>(tops + NS::T0, Bd, dH, lane);
      relu_mask_from_ops<MB>(X, dH);
    }
    grad_to_ops<M, MB>(dH, Bd);
    {
      // the input rows again (cache-resident) rather than held across the strip
      Op X0[KS0][4];
      load_rows<KS0>(xr, IN_PAD, X0, g, col);
      layer_wgrad<MB, IB0>(Bd, X0, eye, dW0, db0);
    }
  }

  // ---- workgroup sums in a fixed order, then the partial
  __syncthreads();
  for (int i = threadIdx.x; i < PO::total(); i += blockDim.x) red[i] = 0.f;
  __syncthreads();
#pragma unroll 1
  for (int v = 0; v < kWgradWaves; v++) {
    if (w == v) {
      // lane (col, g) of tile (ob, ib): rows 16 ob + 4 g + j, column col of block ib
#pragma unroll
      for (int ob = 0; ob < MB; ob++)
#pragma unroll
        for (int ib = 0; ib < MB; ib++) {
          const f32x4 t1 = d1[(ob * 4 + ib) * 64 + lane];
#pragma unroll
          for (int j = 0; j < 4; j++) {
            const int o = 16 * ob + 4 * g + j;
            red[PO::w(0) + o * IN_PAD + l0_feature(ib, col)] += dW0[ob][ib][j];
            red[PO::w(1) + o * 64 + 16 * ib + col] += t1[j];
            red[PO::w(2) + o * 64 + 16 * ib + col] += dW2[ob][ib][j];
          }
        }
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int o = 4 * g + j;
        if (o < 6)
#pragma unroll
          for (int ib = 0; ib < MB; ib++) red[PO::w(3) + o * 64 + 16 * ib + col] += dW3[0][ib][j];
      }
      // bias sums: the four lane groups hold disjoint pixel subsets of the same outputs
#pragma unroll 1
      for (int gg = 0; gg < 4; gg++) {
        if (g == gg) {
#pragma unroll
          for (int ob = 0; ob < MB; ob++) {
            red[PO::b(0) + 16 * ob + col] += db0[ob];
            red[PO::b(1) + 16 * ob + col] += db1[ob];
            red[PO::b(2) + 16 * ob + col] += db2[ob];
          }
          if (col < 6) red[PO::b(3) + col] += db3[0];
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
  }
  float *part = partials + (size_t)blockIdx.x * PO::total();
  for (int i = threadIdx.x; i < PO::total(); i += blockDim.x) part[i] = red[i];
}

}  // namespace

int mlp_wgrad_grid(int nstrips) {
  int grid = (nstrips + kWgradWaves - 1) / kWgradWaves;
  if (grid > kWgradMaxBlocks) grid = kWgradMaxBlocks;
  return grid < 1 ? 1 : grid;
}

void launch_mlp_wgrad(const void *wops, const void *tops, const float *params, const __bf16 *rec_x,
                      const __bf16 *rec_o, int nstrips, float *partials, hipStream_t st) {
  mlp_wgrad_kernel<<<mlp_wgrad_grid(nstrips), kWgradWaves * 64, 0, st>>>(wops, tops, params, rec_x, rec_o, nstrips,
                                                                        partials);
}

}  // namespace sssgs
