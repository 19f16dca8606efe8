// mlp_wgrad.hip -- weight and bias gradients of the per-pixel network
// (Sec. 3.2, Eq. 6), BF16 operands, width 64, three hidden layers.
//
// Input: the strip records of the split shading backward, i.e. per 64-pixel
// strip the BF16 network input rows as layer 0 reads them (values and their
// BF16 remainders) and the BF16 gradients of the six network outputs.  The
// forward products take activations as hi + lo pairs (mlp.hpp); the weight
// gradients take hi.  Each wave takes whole strips: it
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

// Layer-0 B operands of a strip from its record rows ([64][stride] BF16),
// starting at element `first` of each row (0: the values, IN_PAD: the
// remainders).
template <int KS0>
__device__ __forceinline__ void load_rows(const __bf16 *xr, int stride, int first, bf16x8 (&X)[KS0][4], int g,
                                          int col) {
#pragma unroll
  for (int ks = 0; ks < KS0; ks++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
      X[ks][nb] = *reinterpret_cast<const bf16x8 *>(xr + (16 * nb + col) * stride + first + ks * 32 + g * 8);
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
    const __bf16 *xr = rec_x + (size_t)s * 64 * 2 * IN_PAD;
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
      Op X0[KS0][4], X0lo[KS0][4];
      load_rows<KS0>(xr, 2 * IN_PAD, 0, X0, g, col);
      load_rows<KS0>(xr, 2 * IN_PAD, IN_PAD, X0lo, g, col);
      f32x4 acc[MB][4];
      Op H[KSH][4], Hlo[KSH][4];
      act_mma<M, MB, KS0>(wl, X0, X0lo, acc, lane);
      acc_to_ops<M, MB>(acc, bl, g, H, Hlo);
      store_ops(hs, H, lane);
      act_mma<M, MB, KSH>(wl + NS::L0, H, Hlo, acc, lane);
      acc_to_ops<M, MB>(acc, bl + 64, g, H, Hlo);
      store_ops(hs + KSH * 4 * 64, H, lane);
      act_mma<M, MB, KSH>(wl + NS::L0 + NS::LH, H, Hlo, acc, lane);
      acc_to_ops<M, MB>(acc, bl + 128, g, H3, Hlo);
    }
    // output layer: dY = output gradients, X = H3 (one 16-row block, rows 0..5)
    Op Bo[1][4];
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      uint2 v = make_uint2(0u, 0u);
      if (g < 2) v = *reinterpret_cast<const uint2 *>(orow + (16 * nb + col) * 8 + 4 * g);
      Bo[0][nb] = __builtin_bit_cast(bf16x8, make_uint4(v.x, v.y, 0u, 0u));
    }
    f32x4 dH[MB][4];
    Op Bd[KSH][4];
    // each layer's backward product first: its weight loads (L2) are then in
    // flight while the independent weight-gradient products run
    layer_mma<M, MB, NS::KT_O>(tops + NS::T0 + 2 * NS::TH, Bo, dH, lane);
    layer_wgrad<1, MB>(Bo, H3, eye, dW3, db3);
    relu_mask_from_ops<MB>(H3, dH);
    grad_to_ops<M, MB>(dH, Bd);
    {
      Op X[KSH][4];
      load_ops(hs + KSH * 4 * 64, X, lane);  // H2
      layer_mma<M, MB, NS::KT_H>(tops + NS::T0 + NS::TH, Bd, dH, lane);
      layer_wgrad<MB, MB>(Bd, X, eye, dW2, db2);
      relu_mask_from_ops<MB>(X, dH);
    }
    grad_to_ops<M, MB>(dH, Bd);
    {
      Op X[KSH][4];
      load_ops(hs, X, lane);  // H1
      layer_mma<M, MB, NS::KT_H>(tops + NS::T0, Bd, dH, lane);
      layer1_wgrad_lds(Bd, X, eye, d1, db1, lane);
      relu_mask_from_ops<MB>(X, dH);
    }
    grad_to_ops<M, MB>(dH, Bd);
    {
      // the input rows again (cache-resident) rather than held across the strip
      Op X0[KS0][4];
      load_rows<KS0>(xr, 2 * IN_PAD, 0, X0, g, col);
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


// ---------------------------------------------------------------- generic form
//
// The weight and bias gradients of the other network forms (FP32; BF16 at
// width 128 or input width 96) from the feature-major operands the generic
// shading backward stores: dW_l = dY_l X_l^T and db_l = dY_l 1, contractions
// over all P pixels.  Split K: workgroup (s, y) sums pixels [s S, (s + 1) S)
// of one layer into row s of the partials (every element of the layer's
// slice written), and the fixed-order reduction over s follows, so the result
// does not depend on timing.  Operands are read straight from memory with
// pixels along K: BF16 as 8 consecutive pixels per lane (16 B), FP32 as a
// float4 of 4 pixels that serves 4 k-steps (the pixel order inside a sum is
// free, so k-step t takes pixel 4 g + t of the 16).  The four waves tile the
// layer's 16 x 16 blocks (WO x WI waves over output x input blocks); the bias
// sums are added on the vector ALUs from the dY operands the waves with
// wi = 0 already hold.  1024 pixels per workgroup give a few hundred
// workgroups per layer at 800x800 (one per CU would leave most of the chip
// idle).
constexpr int kGemmSplit = 1024;  // pixels per workgroup

template <class M, int R16, int K16>
struct GemmShape {
  static constexpr int WO = R16 < 4 ? R16 : 4, WI = 4 / WO;
  static constexpr int NOB = (R16 + WO - 1) / WO, NIB = (K16 + WI - 1) / WI;
  static constexpr int KC = M::KPL == 8 ? 32 : 16;  // pixels per step
};

template <class M, int R16, int K16>
__global__ __launch_bounds__(256) void wgrad_gemm_kernel(const typename M::Elem *__restrict__ dy0,
                                                         const typename M::Elem *__restrict__ x0, size_t layer_dy,
                                                         size_t layer_x, int rows_alloc, int rows, int cols,
                                                         size_t P, float *__restrict__ partials, int nparams,
                                                         int woff0, int param_step) {
  using E = typename M::Elem;
  using Op = typename M::Op;
  using GS = GemmShape<M, R16, K16>;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
  const int wo = w % GS::WO, wi = w / GS::WO;
  const E *dy = dy0 + (size_t)blockIdx.y * layer_dy;
  const E *x = x0 + (size_t)blockIdx.y * layer_x;
  const int woff = woff0 + blockIdx.y * param_step, boff = woff + rows * cols;
  const size_t pa = (size_t)blockIdx.x * kGemmSplit, pb = pa + kGemmSplit < P ? pa + kGemmSplit : P;
  f32x4 acc[GS::NOB][GS::NIB];
  float bsum[GS::NOB];
#pragma unroll
  for (int a = 0; a < GS::NOB; a++) {
    bsum[a] = 0.f;
#pragma unroll
    for (int b = 0; b < GS::NIB; b++) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  for (size_t p = pa; p < pb; p += GS::KC) {
    if constexpr (M::KPL == 8) {
      Op A[GS::NOB], B[GS::NIB];
#pragma unroll
      for (int a = 0; a < GS::NOB; a++) {
        const int r = 16 * (wo + GS::WO * a) + col;
        A[a] = r < rows_alloc ? *reinterpret_cast<const bf16x8 *>(dy + (size_t)r * P + p + 8 * g) : Op{};
#pragma unroll
        for (int j = 0; j < 8; j++) bsum[a] += (float)A[a][j];
      }
#pragma unroll
      for (int b = 0; b < GS::NIB; b++) {
        const int ib = wi + GS::WI * b;
        if (ib < K16) B[b] = *reinterpret_cast<const bf16x8 *>(x + (size_t)(16 * ib + col) * P + p + 8 * g);
      }
#pragma unroll
      for (int a = 0; a < GS::NOB; a++)
#pragma unroll
        for (int b = 0; b < GS::NIB; b++)
          if (wo + GS::WO * a < R16 && wi + GS::WI * b < K16) acc[a][b] = M::mma(A[a], B[b], acc[a][b]);
    } else {
      float4 A[GS::NOB], B[GS::NIB];
#pragma unroll
      for (int a = 0; a < GS::NOB; a++) {
        const int r = 16 * (wo + GS::WO * a) + col;
        A[a] = r < rows_alloc ? *reinterpret_cast<const float4 *>(dy + (size_t)r * P + p + 4 * g)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
        bsum[a] += (A[a].x + A[a].y) + (A[a].z + A[a].w);
      }
#pragma unroll
      for (int b = 0; b < GS::NIB; b++) {
        const int ib = wi + GS::WI * b;
        if (ib < K16) B[b] = *reinterpret_cast<const float4 *>(x + (size_t)(16 * ib + col) * P + p + 4 * g);
      }
#pragma unroll
      for (int a = 0; a < GS::NOB; a++)
#pragma unroll
        for (int b = 0; b < GS::NIB; b++)
          if (wo + GS::WO * a < R16 && wi + GS::WI * b < K16) {
            acc[a][b] = M::mma(A[a].x, B[b].x, acc[a][b]);
            acc[a][b] = M::mma(A[a].y, B[b].y, acc[a][b]);
            acc[a][b] = M::mma(A[a].z, B[b].z, acc[a][b]);
            acc[a][b] = M::mma(A[a].w, B[b].w, acc[a][b]);
          }
    }
  }
  // D layout: lane (col, g) holds block rows 4 g + j, block column col
  float *part = partials + (size_t)blockIdx.x * nparams;
#pragma unroll
  for (int a = 0; a < GS::NOB; a++)
#pragma unroll
    for (int b = 0; b < GS::NIB; b++) {
      const int ob = wo + GS::WO * a, ib = wi + GS::WI * b;
      if (ob >= R16 || ib >= K16) continue;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int o = 16 * ob + 4 * g + j, i = 16 * ib + col;
        if (o < rows && i < cols) part[woff + o * cols + i] = acc[a][b][j];
      }
    }
  // bias: lane (col, g) summed row 16 ob + col over its pixel group g; add
  // the four groups (lanes col, col + 16, col + 32, col + 48) in a fixed order
  if (wi == 0) {
#pragma unroll
    for (int a = 0; a < GS::NOB; a++) {
      const float s1 = __shfl_xor(bsum[a], 16, 64);
      const float s12 = bsum[a] + s1;
      const float tot = s12 + __shfl_xor(s12, 32, 64);
      const int ob = wo + GS::WO * a, o = 16 * ob + col;
      if (g == 0 && ob < R16 && o < rows) part[boff + o] = tot;
    }
  }
}

template <class M, int R16, int K16>
static void gemm_layer(const void *dy, const void *x, size_t ldy, size_t lx, int nl, int rows_alloc, int rows,
                       int cols, size_t P, float *partials, int nparams, int woff, int step, hipStream_t st) {
  const dim3 grid((unsigned)((P + kGemmSplit - 1) / kGemmSplit), nl);
  wgrad_gemm_kernel<M, R16, K16><<<grid, 256, 0, st>>>(reinterpret_cast<const typename M::Elem *>(dy),
                                                       reinterpret_cast<const typename M::Elem *>(x), ldy, lx,
                                                       rows_alloc, rows, cols, P, partials, nparams, woff, step);
}

template <class M, int WIDTH, int IN_PAD>
static void wgrad_gemm_t(const void *gx, const void *gdy, size_t P, float *partials, hipStream_t st) {
  using PO = ParamOffsets<WIDTH, IN_PAD>;
  using E = typename M::Elem;
  const E *X = reinterpret_cast<const E *>(gx), *Y = reinterpret_cast<const E *>(gdy);
  const int np = PO::total();
  const E *X1 = X + (size_t)IN_PAD * P, *X3 = X1 + 2 * (size_t)WIDTH * P;
  const E *Y1 = Y + (size_t)WIDTH * P, *Y3 = Y1 + 2 * (size_t)WIDTH * P;
  gemm_layer<M, WIDTH / 16, IN_PAD / 16>(Y, X, 0, 0, 1, WIDTH, WIDTH, IN_PAD, P, partials, np, PO::w(0), 0, st);
  gemm_layer<M, WIDTH / 16, WIDTH / 16>(Y1, X1, (size_t)WIDTH * P, (size_t)WIDTH * P, 2, WIDTH, WIDTH, WIDTH, P,
                                        partials, np, PO::w(1), PO::w(2) - PO::w(1), st);
  gemm_layer<M, 1, WIDTH / 16>(Y3, X3, 0, 0, 1, 8, 6, WIDTH, P, partials, np, PO::w(3), 0, st);
}

int wgrad_gemm_splits(size_t P) { return (int)((P + kGemmSplit - 1) / kGemmSplit); }

void launch_wgrad_gemm(int net, int width, int in_pad, const void *gx, const void *gdy, size_t P, float *partials,
                       hipStream_t st) {
  if (net == 1) {
    if (width == 64 && in_pad == 64) wgrad_gemm_t<MmaF32, 64, 64>(gx, gdy, P, partials, st);
    else if (width == 64 && in_pad == 96) wgrad_gemm_t<MmaF32, 64, 96>(gx, gdy, P, partials, st);
  } else if (net == 2) {
    if (width == 64 && in_pad == 64) wgrad_gemm_t<MmaBF16, 64, 64>(gx, gdy, P, partials, st);
    else if (width == 64 && in_pad == 96) wgrad_gemm_t<MmaBF16, 64, 96>(gx, gdy, P, partials, st);
    else if (width == 128 && in_pad == 64) wgrad_gemm_t<MmaBF16, 128, 64>(gx, gdy, P, partials, st);
    else if (width == 128 && in_pad == 96) wgrad_gemm_t<MmaBF16, 128, 96>(gx, gdy, P, partials, st);
  }
}

}  // namespace sssgs
