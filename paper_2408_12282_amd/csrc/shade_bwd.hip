// shade_bwd.hip -- backward of the per-pixel deferred shading (Sec. 3.2,
// Eq. 4, 6, 7): from dL/d(rgb) to dL/d(G-buffer), dL/d(T_final) and the
// operands of the network parameter gradients.
//
// One wave per 64-pixel strip (16 x 4).  With the per-pixel network the
// forward is recomputed on the matrix cores, Eq. 7's backward gives the
// gradients of the six network outputs, and dX^T = W^T dY^T runs through the
// transposed layers (consuming the accumulator layout directly) down to the
// gradient of the network input, whose per-pixel backward gives dL/dG.  The
// weight gradients dW = dY^T X, a contraction over all pixels, are left to
// mlp_wgrad.hip: the BF16 width-64 network (the headline form, split kernel
// below) leaves per strip its input rows and output gradients and the weight
// kernel recomputes the rest; the other forms (generic kernel below) store
// every layer's input X_l and pre-activation gradient dY_l, feature-major,
// for a split-K matrix-core contraction.
#include "launch.hpp"
#include "net_bwd.hpp"

namespace sssgs {

// -------------------------------------------------------------- per pixel

// Backward of everything after the network outputs (or of the light
// fall-off without network): fills dgbar (d L / d mean values) and returns
// d L / d a (direct part).  dnet_in: gradient w.r.t. the network input vector
// (or null), used for features, position encoding and directions.
template <int C, int F, int MODE>
__device__ __forceinline__ float shade_pixel_bwd(const PixShade &S, const float *gb, const float *gL,
                                                 const LightArgs &light, const float *dnet_in, float *dgbar) {
#pragma unroll
  for (int k = 0; k < C; k++) dgbar[k] = 0.f;
  float dA = 0.f, gLo[3];
  for (int c = 0; c < 3; c++) {
    dA += gL[c] * S.L[c];
    gLo[c] = S.a * gL[c];
  }
  float dfs[3], dfd[3], dcos = 0.f, dx[3] = {0.f, 0.f, 0.f}, dwo[3] = {0.f, 0.f, 0.f}, dwi[3] = {0.f, 0.f, 0.f};
  float dvi[3] = {0.f, 0.f, 0.f};
  if constexpr (MODE == 2) {
    const float sss = gb[kChSss] * S.ia;
    float dsss = 0.f;
    for (int c = 0; c < 3; c++) {
      const float B = S.fs[c] + S.fd[c];
      dsss += gLo[c] * (S.Lsss[c] - B * S.Lin[c] * S.cosI);
      dfs[c] = gLo[c] * (1.f - sss) * S.Lin[c] * S.cosI;
      dfd[c] = dfs[c];
      dcos += gLo[c] * (1.f - sss) * B * S.Lin[c];
      dgbar[kChFeat + c] += gLo[c] * (1.f - sss) * B * S.cosI;
      dgbar[kChFeat + 3 + c] += gLo[c] * sss;
    }
    dgbar[kChSss] += dsss;
  } else if constexpr (MODE == 0) {
    float dli2 = 0.f;
    for (int c = 0; c < 3; c++) {
      dfs[c] = gLo[c] * S.Lin[c] * S.cosI;
      dfd[c] = dfs[c];
      const float dLin = gLo[c] * (S.fs[c] + S.fd[c]) * S.cosI;
      dcos += gLo[c] * (S.fs[c] + S.fd[c]) * S.Lin[c];
      dli2 -= dLin * light.intensity[c] / (S.li2 * S.li2);
    }
    if (dot3(S.vi, S.vi) >= 1e-12f)
      for (int k = 0; k < 3; k++) dvi[k] += 2.f * dli2 * S.vi[k];
  } else {
    const float sss = gb[kChSss] * S.ia;
    float dsss = 0.f;
    for (int c = 0; c < 3; c++) {
      const float B = S.fs[c] + S.fd[c];
      dsss += gLo[c] * (S.Lsss[c] - B * S.Lin[c] * S.cosI);
      dfs[c] = gLo[c] * (1.f - sss) * S.Lin[c] * S.cosI;
      dfd[c] = dfs[c];
      dcos += gLo[c] * (1.f - sss) * B * S.Lin[c];
    }
    dgbar[kChSss] += dsss;
#pragma unroll
    for (int f = 0; f < F; f++) dgbar[kChFeat + f] += dnet_in[f];
    int p = F;
    float sn[3][6], cs[3][6];
#pragma unroll
    for (int ax = 0; ax < 3; ax++) pe_octaves(S.x[ax], sn[ax], cs[ax]);
#pragma unroll
    for (int oct = 0; oct < 6; oct++) {
      const float sc = (float)(1 << oct);
#pragma unroll
      for (int ax = 0; ax < 3; ax++) dx[ax] += dnet_in[p + ax] * (sc * kPi) * cs[ax][oct];
#pragma unroll
      for (int ax = 0; ax < 3; ax++) dx[ax] -= dnet_in[p + 3 + ax] * (sc * kPi) * sn[ax][oct];
      p += 6;
    }
    for (int k = 0; k < 3; k++) dwo[k] += dnet_in[p + k];
    for (int k = 0; k < 3; k++) dwi[k] += dnet_in[p + 3 + k];
  }
  // BRDF
  const float r = gb[kChRough] * S.ia, m = gb[kChMetal] * S.ia;
  float dD = 0.f, dGv = 0.f, dQ = 0.f, dVoH = 0.f, dm = 0.f;
  const float w = S.w, w4 = (w * w) * (w * w), w5 = w4 * w;
  for (int c = 0; c < 3; c++) {
    dD += dfs[c] * S.F[c] * S.Gv * S.Q;
    const float dF = dfs[c] * S.D * S.Gv * S.Q;
    dGv += dfs[c] * S.D * S.F[c] * S.Q;
    dQ += dfs[c] * S.D * S.F[c] * S.Gv;
    const float dF0 = dF * (1.f - w5);
    dVoH -= dF * (1.f - S.F0[c]) * 5.f * w4;
    const float b = gb[kChAlb + c] * S.ia;
    dgbar[kChAlb + c] += dfd[c] * (1.f - m) * (1.f / kPi) + dF0 * m;
    dm += -dfd[c] * b * (1.f / kPi) + dF0 * (b - 0.04f);
  }
  float dNoV = -dQ * S.Q / S.NoV, dNoL = -dQ * S.Q / S.NoL;
  const float dg1v = dGv * S.g1l, dg1l = dGv * S.g1v;
  dNoV += dg1v * S.k / (S.dv * S.dv);
  dNoL += dg1l * S.k / (S.dl * S.dl);
  const float dk = -dg1v * S.NoV * (1.f - S.NoV) / (S.dv * S.dv) - dg1l * S.NoL * (1.f - S.NoL) / (S.dl * S.dl);
  float dr = dk * (r + 1.f) * 0.25f;
  const float ag = S.ag, den = S.den;
  const float dag = dD * (2.f * ag / (kPi * den * den)) * (1.f - 2.f * ag * ag * S.NoH * S.NoH / den);
  const float dNoH = dD * (-2.f * ag * ag / (kPi * den * den * den)) * 2.f * S.NoH * (ag * ag - 1.f);
  dr += dag * 2.f * r;
  dgbar[kChRough] += dr;
  dgbar[kChMetal] += dm;
  const float dnov = S.nov > 1e-4f ? dNoV : 0.f;
  const float dnol = (S.nol > 1e-4f ? dNoL : 0.f) + (S.nol > 0.f ? dcos : 0.f);
  const float dnoh = S.noh > 0.f ? dNoH : 0.f;
  const float dvoh = S.voh > 0.f ? dVoH : 0.f;
  float dn[3], dh[3];
  for (int k = 0; k < 3; k++) {
    dn[k] = dnov * S.wo[k] + dnol * S.wi[k] + dnoh * S.h[k];
    dwo[k] += dnov * S.n[k] + dvoh * S.h[k];
    dwi[k] += dnol * S.n[k];
    dh[k] = dnoh * S.n[k] + dvoh * S.wo[k];
  }
  // normalisations v / max(|v|, eps)
  auto nbwd = [](const float *v, float l, const float *o, const float *dout, float *dv) {
    if (l > 1e-12f) {
      const float p = dot3(o, dout), il = 1.f / l;
      for (int k = 0; k < 3; k++) dv[k] += (dout[k] - o[k] * p) * il;
    } else {
      for (int k = 0; k < 3; k++) dv[k] += dout[k] * 1e12f;
    }
    (void)v;
  };
  float dhv[3] = {0.f, 0.f, 0.f};
  nbwd(S.hv, S.hl, S.h, dh, dhv);
  for (int k = 0; k < 3; k++) {
    dwo[k] += dhv[k];
    dwi[k] += dhv[k];
  }
  float dvo[3] = {0.f, 0.f, 0.f};
  nbwd(S.vo, S.lo, S.wo, dwo, dvo);
  nbwd(S.vi, S.li, S.wi, dwi, dvi);
  for (int k = 0; k < 3; k++) dx[k] -= dvo[k] + dvi[k];
  dgbar[kChDepth] += dot3(dx, S.ray);
  float dnr[3] = {0.f, 0.f, 0.f};
  nbwd(S.nraw, S.nlen, S.n, dn, dnr);
  for (int k = 0; k < 3; k++) dgbar[kChNrm + k] += dnr[k];
  return dA;
}

// -------------------------------------------------------------- kernel

// Per-pixel inputs of the shading backward (reloaded in each per-pixel phase
// instead of being kept live across the network phases).
template <int C>
__device__ __forceinline__ void load_pixel(const ShadeArgs &A, bool inside, size_t pix, size_t HW, float *gb,
                                           float &T, float *gL) {
  T = 1.f;
  for (int c = 0; c < 3; c++) gL[c] = 0.f;
  if (inside) {
#pragma unroll
    for (int c = 0; c < C; c++) gb[c] = A.gbuf[c * HW + pix];
    T = A.t_final[pix];
    for (int c = 0; c < 3; c++) gL[c] = A.drgb[c * HW + pix];
  } else {
#pragma unroll
    for (int c = 0; c < C; c++) gb[c] = 0.f;
  }
}

// Only what Eq. 7's backward needs (geometry and material channels, T, the
// upstream gradient): the feature planes are not read.
template <int C>
__device__ __forceinline__ void load_pixel_geo(const ShadeArgs &A, bool inside, size_t pix, size_t HW, float *gb,
                                               float &T, float *gL) {
  T = 1.f;
  for (int c = 0; c < 3; c++) gL[c] = 0.f;
#pragma unroll
  for (int c = 0; c < C; c++) gb[c] = 0.f;
  if (inside) {
#pragma unroll
    for (int c = 0; c < kChFeat; c++) gb[c] = A.gbuf[c * HW + pix];
    T = A.t_final[pix];
    for (int c = 0; c < 3; c++) gL[c] = A.drgb[c * HW + pix];
  }
}

template <int C, int F>
__device__ __forceinline__ void write_pixel_grads(const ShadeArgs &A, bool inside, size_t pix, size_t HW,
                                                  const PixShade &S, const float *gb, float *dgbar, float dA) {
  if (!inside) return;
  float dT = 0.f;
  if (!S.bg) {
#pragma unroll
    for (int k = 0; k < C; k++) dA -= dgbar[k] * gb[k] * S.ia * S.ia;
    dT = -dA;
  }
  if (A.dalpha_ext) dT -= A.dalpha_ext[pix];
  // rgb = ... + T_final background
  for (int c = 0; c < 3; c++) dT += A.drgb[c * HW + pix] * A.bgc[c];
  A.dT[pix] = dT;
#pragma unroll
  for (int k = 0; k < C; k++) {
    float v = S.bg ? 0.f : dgbar[k] * S.ia;
    if (A.dgbuf_ext) v += A.dgbuf_ext[k * HW + pix];
    A.dG[k * HW + pix] = v;
  }
}

// Without a per-pixel network (light fall-off, or radiances composited from
// the per-Gaussian network): one lane per pixel, one 256-lane workgroup per
// tile.
template <int F, int NET>
__global__ __launch_bounds__(256) void shade_bwd_plain_kernel(ShadeArgs A) {
  constexpr int C = kChFeat + F;
  const int tile = xcd_item(blockIdx.x, gridDim.x);
  const int tx = tile % A.cam.TX, ty = tile / A.cam.TX;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < A.cam.W && py < A.cam.H;
  if (!inside) return;
  const size_t HW = (size_t)A.cam.W * A.cam.H, pix = (size_t)py * A.cam.W + px;
  float gb[C], T, gL[3], dgbar[C];
  load_pixel<C>(A, true, pix, HW, gb, T, gL);
  PixShade S;
  shade_geometry<C>(gb, T, (float)px + 0.5f, (float)py + 0.5f, A.cam, A.light, NET == 3, S);
  if constexpr (NET == 3) combine_features(S, gb);
  if (S.bg) gL[0] = gL[1] = gL[2] = 0.f;
  const float dA = shade_pixel_bwd<C, F, NET == 3 ? 2 : 0>(S, gb, gL, A.light, nullptr, dgbar);
  write_pixel_grads<C, F>(A, true, pix, HW, S, gb, dgbar, dA);
}

// ---------------------------------------------------------------- split form
//
// For the BF16 width-64 network the weight gradients are left to a kernel of
// their own (mlp_wgrad.hip).  This kernel then only needs, per wave, the input
// rows until layer 0 has consumed them, dL/d(input) afterwards (same LDS),
// and the network outputs with their gradients: about 20 KB, and no
// workgroup-wide exchange, so each wave shades one strip on its own and two
// waves fit per SIMD.  For the weight-gradient kernel it leaves a record per
// strip: the BF16 network input rows as layer 0 reads them ([64][2 IN_PAD],
// the values rounded to BF16 followed by their BF16 remainders) and
// the BF16 gradients of the six network outputs as the transposed output
// layer reads them ([64][8], two zero pads).
template <int IN_PAD>
struct SplitLds {
  static constexpr int XS = in_row_stride<MmaBF16, IN_PAD>();  // bf16 input row stride (hi | lo)
  static constexpr int DS = IN_PAD + 1;                     // fp32 input-gradient row stride
  // floats per pixel: 6 outputs, 6 output gradients.  No odd padding (its
  // few accesses conflict): 20480 bytes in all, so that eight one-wave
  // workgroups share a CU's 160 KB.
  static constexpr int IO = 12;
  static constexpr int RB = (64 * XS * 2 > 64 * DS * 4) ? 64 * XS * 2 : 64 * DS * 4;
  static constexpr int BYTES = RB + 64 * IO * 4;
};
static_assert(SplitLds<64>::BYTES <= 160 * 1024 / 8, "eight split-backward workgroups per CU");

template <int F, int IN_PAD>
__global__ __launch_bounds__(64, 2) void shade_bwd_split_kernel(ShadeArgs A, __bf16 *__restrict__ rec_x,
                                                                __bf16 *__restrict__ rec_o) {
  using M = MmaBF16;
  using Op = bf16x8;
  using NS = NetShape<M, 64, IN_PAD>;
  using PO = ParamOffsets<64, IN_PAD>;
  using SL = SplitLds<IN_PAD>;
  constexpr int C = kChFeat + F;
  constexpr int MB = NS::MB;
  __shared__ __attribute__((aligned(16))) char lds[SL::BYTES];
  __bf16 *xs = reinterpret_cast<__bf16 *>(lds);
  float *dxin = reinterpret_cast<float *>(lds);  // after layer 0 of the forward has read xs
  float *io = reinterpret_cast<float *>(lds + SL::RB);
  const int lane = threadIdx.x;
  const int g = lane >> 4, col = lane & 15;
  const int strip = xcd_item(blockIdx.x, gridDim.x);
  const int tile = strip >> 2, sub = strip & 3;
  const int tx = tile % A.cam.TX, ty = tile / A.cam.TX;
  const int px = tx * kTile + col, py = ty * kTile + 4 * sub + g;
  const bool inside = px < A.cam.W && py < A.cam.H;
  const size_t HW = (size_t)A.cam.W * A.cam.H;
  const size_t pix = inside ? (size_t)py * A.cam.W + px : 0;
  const float uc = (float)px + 0.5f, vc = (float)py + 0.5f;
  const Op *__restrict__ wops = reinterpret_cast<const Op *>(A.wops);
  const Op *__restrict__ tops = reinterpret_cast<const Op *>(A.tops);
  const size_t rrow = (size_t)strip * 64 + lane;
  // clear the compositing backward's per-Gaussian accumulators on the side
  // (stores only; they overlap with this kernel's arithmetic)
  if (A.zero_buf) {
    const size_t nth = (size_t)gridDim.x * 64;
    for (size_t k = rrow; k < A.zero_count4; k += nth) A.zero_buf[k] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  // ---- A: network input row (LDS and record)
  {
    float gb[C], T, gL[3];
    load_pixel<C>(A, inside, pix, HW, gb, T, gL);
    PixShade S;
    shade_geometry<C>(gb, T, uc, vc, A.cam, A.light, true, S);
    build_net_input<F, IN_PAD, M>(gb, S, xs + lane * SL::XS);
  }
  __syncthreads();
  {
    // the strip's rows to its record, coalesced: consecutive lanes write
    // consecutive 16-byte chunks of the 64 rows
    static_assert(SL::XS % 8 == 0, "row stride in 16-byte chunks");
    constexpr int CH = 2 * IN_PAD / 8;  // chunks per row
    const uint4 *src = reinterpret_cast<const uint4 *>(xs);
    uint4 *dst = reinterpret_cast<uint4 *>(rec_x + (size_t)strip * 64 * 2 * IN_PAD);
#pragma unroll
    for (int q = lane; q < 64 * CH; q += 64) dst[q] = src[(q / CH) * (SL::XS / 8) + q % CH];
  }
  // ---- B: network forward: ReLU masks and outputs
  Mask<MB> m1, m2, m3;
  {
    f32x4 acc[MB][4];
    Op H[NS::KSH][4], Hlo[NS::KSH][4];
    layer0_mma<M, MB, NS::KS0>(wops, xs, SL::XS, acc, lane);
    acc_to_ops<M, MB>(acc, A.params + PO::b(0), g, H, Hlo);
    m1.set_from_ops(H);
    act_mma<M, MB, NS::KSH>(wops + NS::L0, H, Hlo, acc, lane);
    acc_to_ops<M, MB>(acc, A.params + PO::b(1), g, H, Hlo);
    m2.set_from_ops(H);
    act_mma<M, MB, NS::KSH>(wops + NS::L0 + NS::LH, H, Hlo, acc, lane);
    acc_to_ops<M, MB>(acc, A.params + PO::b(2), g, H, Hlo);
    m3.set_from_ops(H);
    f32x4 oacc[1][4];
    act_mma<M, 1, NS::KSH>(wops + NS::L0 + 2 * NS::LH, H, Hlo, oacc, lane);
    if (g < 2)
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int o = 4 * g + j;
          if (o < 6) io[(16 * nb + col) * SL::IO + o] = oacc[0][nb][j] + A.params[PO::b(3) + o];
        }
  }
  __syncthreads();
  // ---- C: Eq. 7 and the gradients of the network outputs.  The pixel's
  // G-buffer values stay in registers through D for E (the register budget of
  // two waves per SIMD holds them).
  float gb[C], T, gL[3];
  load_pixel<C>(A, inside, pix, HW, gb, T, gL);
  {
    PixShade S;
    shade_geometry<C>(gb, T, uc, vc, A.cam, A.light, true, S);
    if (S.bg) gL[0] = gL[1] = gL[2] = 0.f;
    float o[6];
    for (int k = 0; k < 6; k++) o[k] = io[lane * SL::IO + k];
    combine_net(S, gb[kChSss], o);
    const float sss = gb[kChSss] * S.ia;
    float d[8];
    for (int c = 0; c < 3; c++) {
      const float gLo = S.a * gL[c];
      const float dLin = gLo * (1.f - sss) * (S.fs[c] + S.fd[c]) * S.cosI;
      d[c] = o[c] > 0.f ? dLin : 0.f;
      d[3 + c] = gLo * sss * S.Lsss[c] * (1.f - S.Lsss[c]);
    }
    d[6] = d[7] = 0.f;
    bf16x8 r;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (k < 6) io[lane * SL::IO + 6 + k] = d[k];
      r[k] = (__bf16)d[k];
    }
    *reinterpret_cast<bf16x8 *>(rec_o + rrow * 8) = r;
  }
  __syncthreads();
  // ---- D: backward through the network to its inputs
  {
    Op Bo[NS::KT_O][4];
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      bf16x8 v;
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int o = 4 * g + j;
        v[j] = (__bf16)((j < 4 && o < 6) ? io[(16 * nb + col) * SL::IO + 6 + o] : 0.f);
      }
      Bo[0][nb] = v;
    }
    f32x4 dH[MB][4];
    Op Bd[NS::KSH][4];
    layer_mma<M, MB, NS::KT_O>(tops + NS::T0 + 2 * NS::TH, Bo, dH, lane);
    m3.apply(dH);
    grad_to_ops<M, MB>(dH, Bd);
    layer_mma<M, MB, NS::KT_H>(tops + NS::T0 + NS::TH, Bd, dH, lane);
    m2.apply(dH);
    grad_to_ops<M, MB>(dH, Bd);
    layer_mma<M, MB, NS::KT_H>(tops + NS::T0, Bd, dH, lane);
    m1.apply(dH);
    grad_to_ops<M, MB>(dH, Bd);
    f32x4 dX[NS::MB0][4];
    layer_mma<M, NS::MB0, NS::KT_H>(tops, Bd, dX, lane);
#pragma unroll
    for (int mb = 0; mb < NS::MB0; mb++)
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
#pragma unroll
        for (int j = 0; j < 4; j++) dxin[(16 * nb + col) * SL::DS + 16 * mb + 4 * g + j] = dX[mb][nb][j];
  }
  __syncthreads();
  // ---- E: per pixel backward of geometry, BRDF and Eq. 7
  {
    float dgbar[C];
    PixShade S;
    shade_geometry<C>(gb, T, uc, vc, A.cam, A.light, true, S);
    if (S.bg) gL[0] = gL[1] = gL[2] = 0.f;
    float o[6];
    for (int k = 0; k < 6; k++) o[k] = io[lane * SL::IO + k];
    combine_net(S, gb[kChSss], o);
    const float dA = shade_pixel_bwd<C, F, 1>(S, gb, gL, A.light, dxin + lane * SL::DS, dgbar);
    write_pixel_grads<C, F>(A, inside, pix, HW, S, gb, dgbar, dA);
  }
}

template <int F, int IN_PAD>
void launch_shade_bwd_split_t(const ShadeArgs &a, __bf16 *rec_x, __bf16 *rec_o, hipStream_t st) {
  const int nstrips = a.cam.TX * a.cam.TY * 4;
  shade_bwd_split_kernel<F, IN_PAD><<<nstrips, 64, 0, st>>>(a, rec_x, rec_o);
}

template void launch_shade_bwd_split_t<0, 64>(const ShadeArgs &, __bf16 *, __bf16 *, hipStream_t);
template void launch_shade_bwd_split_t<8, 64>(const ShadeArgs &, __bf16 *, __bf16 *, hipStream_t);
template void launch_shade_bwd_split_t<16, 64>(const ShadeArgs &, __bf16 *, __bf16 *, hipStream_t);


// ---------------------------------------------------------------- generic form
//
// The other network forms (FP32; BF16 at width 128 or input width 96).  One
// wave per strip.  The layer inputs are staged in LDS rows [64 px][RS] in
// natural feature order (BF16: values, then their remainders), so a layer
// holds only its own accumulators in registers and every width fits.  Per
// layer the kernel stores the weight-gradient operands feature-major over all
// strip pixels (P = strips x 64): X_l[k][P], the layer input as the weight
// gradient takes it (FP32, or the BF16 value), and dY_l[r][P], the gradient of
// the layer's pre-activation as it enters the products (FP32, or BF16).
template <class M, int WIDTH, int IN_PAD>
struct NetLds {
  using E = typename M::Elem;
  static constexpr int KMAX = WIDTH > IN_PAD ? WIDTH : IN_PAD;
  static constexpr int RS = M::NSPLIT * KMAX + XPad<M>::value;  // row stride (elements)
  static constexpr int DS = IN_PAD + 1;                          // FP32 input-gradient row stride
  static constexpr int IO = 13;                                  // outputs (6), their gradients (6), pad
  static constexpr int RB_ROWS = 64 * RS * (int)sizeof(E), RB_DX = 64 * DS * 4;
  static constexpr int RB = RB_ROWS > RB_DX ? RB_ROWS : RB_DX;
  static constexpr int BYTES = RB + 64 * IO * 4;
};

// Bias-added, ReLU-ed accumulators (D layout: lane (col, g) holds features
// 16 mb + 4 g + j of pixel 16 nb + col) into the LDS rows of the next layer's
// input (K features; BF16: value at f, remainder at K + f).
template <class M, int MB>
__device__ __forceinline__ void acc_to_rows(const f32x4 (&acc)[MB][4], const float *bias, int K,
                                            typename M::Elem *rows, int RS, int lane) {
  const int g = lane >> 4, col = lane & 15;
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      const int f = 16 * mb + 4 * g;
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; j++) v[j] = fmaxf(acc[mb][nb][j] + bias[f + j], 0.f);
      typename M::Elem *r = rows + (16 * nb + col) * RS;
      if constexpr (M::NSPLIT == 2) {
        const bf16x2v h0 = __builtin_convertvector((f32x2v){v[0], v[1]}, bf16x2v);
        const bf16x2v h1 = __builtin_convertvector((f32x2v){v[2], v[3]}, bf16x2v);
        const bf16x2v l0 = __builtin_convertvector((f32x2v){v[0] - (float)h0[0], v[1] - (float)h0[1]}, bf16x2v);
        const bf16x2v l1 = __builtin_convertvector((f32x2v){v[2] - (float)h1[0], v[3] - (float)h1[1]}, bf16x2v);
        *reinterpret_cast<uint2 *>(r + f) =
            make_uint2(__builtin_bit_cast(uint32_t, h0), __builtin_bit_cast(uint32_t, h1));
        *reinterpret_cast<uint2 *>(r + K + f) =
            make_uint2(__builtin_bit_cast(uint32_t, l0), __builtin_bit_cast(uint32_t, l1));
      } else {
        *reinterpret_cast<float4 *>(r + f) = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
}

// The first K elements of the lane's own row (its pixel) into column P0 + lane
// of a feature-major operand [K][P].
template <class M>
__device__ __forceinline__ void row_to_operand(const typename M::Elem *rows, int RS, int K,
                                               typename M::Elem *__restrict__ dst, size_t P, size_t P0, int lane) {
  const typename M::Elem *r = rows + lane * RS;
  typename M::Elem *d = dst + P0 + lane;
#pragma unroll 8
  for (int k = 0; k < K; k++) d[(size_t)k * P] = r[k];
}

// D-layout gradients (features 16 mb + 4 g + j of pixel 16 nb + col) into
// columns P0 .. P0 + 63 of a feature-major operand [R][P], rounded as the
// gradient products round them.
template <class M, int MB>
__device__ __forceinline__ void d_to_operand(const f32x4 (&d)[MB][4], typename M::Elem *__restrict__ dst, size_t P,
                                             size_t P0, int lane) {
  const int g = lane >> 4, col = lane & 15;
  // per-lane base; the row offsets (16 mb + j) P are wave-uniform
  typename M::Elem *const base = dst + (size_t)(4 * g) * P + P0 + col;
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      typename M::Elem *const row = base + (size_t)(16 * mb + j) * P;
#pragma unroll
      for (int nb = 0; nb < 4; nb++) row[16 * nb] = M::cvt(d[mb][nb][j]);
    }
}

template <int F, class M, int WIDTH, int IN_PAD>
__global__ __launch_bounds__(64, WIDTH == 64 ? 2 : 1) void shade_bwd_net_kernel(ShadeArgs A) {
  using E = typename M::Elem;
  using Op = typename M::Op;
  using NS = NetShape<M, WIDTH, IN_PAD>;
  using PO = ParamOffsets<WIDTH, IN_PAD>;
  using NL = NetLds<M, WIDTH, IN_PAD>;
  constexpr int C = kChFeat + F;
  constexpr int MB = NS::MB, RS = NL::RS;
  __shared__ __attribute__((aligned(16))) char lds[NL::BYTES];
  E *rows = reinterpret_cast<E *>(lds);
  float *dxin = reinterpret_cast<float *>(lds);  // after the forward
  float *io = reinterpret_cast<float *>(lds + NL::RB);
  const int lane = threadIdx.x;
  const int g = lane >> 4, col = lane & 15;
  const int strip = xcd_item(blockIdx.x, gridDim.x);
  const int tile = strip >> 2, sub = strip & 3;
  const int tx = tile % A.cam.TX, ty = tile / A.cam.TX;
  const int px = tx * kTile + col, py = ty * kTile + 4 * sub + g;
  const bool inside = px < A.cam.W && py < A.cam.H;
  const size_t HW = (size_t)A.cam.W * A.cam.H;
  const size_t pix = inside ? (size_t)py * A.cam.W + px : 0;
  const float uc = (float)px + 0.5f, vc = (float)py + 0.5f;
  const Op *__restrict__ nops = reinterpret_cast<const Op *>(A.nops);
  const Op *__restrict__ tops = reinterpret_cast<const Op *>(A.tops);
  const size_t P = A.gP, P0 = (size_t)strip * 64;
  E *const gx = reinterpret_cast<E *>(A.gx);
  E *const gdy = reinterpret_cast<E *>(A.gdy);
  // operand rows: X_0 [IN_PAD], X_1..X_3 [WIDTH]; dY_0..dY_2 [WIDTH], dY_3 [8]
  E *const X0 = gx, *const X1 = gx + (size_t)IN_PAD * P, *const X2 = X1 + (size_t)WIDTH * P,
          *const X3 = X2 + (size_t)WIDTH * P;
  E *const Y0 = gdy, *const Y1 = gdy + (size_t)WIDTH * P, *const Y2 = Y1 + (size_t)WIDTH * P,
          *const Y3 = Y2 + (size_t)WIDTH * P;
  // ---- A: network input row
  {
    float gb[C], T, gL[3];
    load_pixel<C>(A, inside, pix, HW, gb, T, gL);
    PixShade S;
    shade_geometry<C>(gb, T, uc, vc, A.cam, A.light, true, S);
    build_net_input<F, IN_PAD, M>(gb, S, rows + lane * RS);
  }
  __syncthreads();
  row_to_operand<M>(rows, RS, IN_PAD, X0, P, P0, lane);
  // ---- B: forward, layer inputs through the LDS rows; ReLU masks and outputs
  Mask<MB> m1, m2, m3;
  {
    f32x4 acc[MB][4];
    layer0_mma<M, MB, NS::KS0>(nops, rows, RS, acc, lane);
    m1.set_from(acc, A.params + PO::b(0), g);
    m1.pin();
    __syncthreads();
    acc_to_rows<M, MB>(acc, A.params + PO::b(0), WIDTH, rows, RS, lane);
    __syncthreads();
    row_to_operand<M>(rows, RS, WIDTH, X1, P, P0, lane);
    __builtin_amdgcn_sched_barrier(0);
    layer0_mma<M, MB, NS::KSH>(nops + NS::L0, rows, RS, acc, lane);
    m2.set_from(acc, A.params + PO::b(1), g);
    m2.pin();
    __syncthreads();
    acc_to_rows<M, MB>(acc, A.params + PO::b(1), WIDTH, rows, RS, lane);
    __syncthreads();
    row_to_operand<M>(rows, RS, WIDTH, X2, P, P0, lane);
    __builtin_amdgcn_sched_barrier(0);
    layer0_mma<M, MB, NS::KSH>(nops + NS::L0 + NS::LH, rows, RS, acc, lane);
    m3.set_from(acc, A.params + PO::b(2), g);
    m3.pin();
    __syncthreads();
    acc_to_rows<M, MB>(acc, A.params + PO::b(2), WIDTH, rows, RS, lane);
    __syncthreads();
    row_to_operand<M>(rows, RS, WIDTH, X3, P, P0, lane);
    f32x4 oacc[1][4];
    __builtin_amdgcn_sched_barrier(0);
    layer0_mma<M, 1, NS::KSH>(nops + NS::L0 + 2 * NS::LH, rows, RS, oacc, lane);
    if (g < 2)
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int o = 4 * g + j;
          if (o < 6) io[(16 * nb + col) * NL::IO + o] = oacc[0][nb][j] + A.params[PO::b(3) + o];
        }
  }
  __syncthreads();
  // ---- C: Eq. 7 and the gradients of the network outputs
  {
    float gb[C], T, gL[3];
    load_pixel_geo<C>(A, inside, pix, HW, gb, T, gL);
    PixShade S;
    shade_geometry<C>(gb, T, uc, vc, A.cam, A.light, true, S);
    if (S.bg) gL[0] = gL[1] = gL[2] = 0.f;
    float o[6];
    for (int k = 0; k < 6; k++) o[k] = io[lane * NL::IO + k];
    combine_net(S, gb[kChSss], o);
    const float sss = gb[kChSss] * S.ia;
    float d[8];
    for (int c = 0; c < 3; c++) {
      const float gLo = S.a * gL[c];
      const float dLin = gLo * (1.f - sss) * (S.fs[c] + S.fd[c]) * S.cosI;
      d[c] = o[c] > 0.f ? dLin : 0.f;
      d[3 + c] = gLo * sss * S.Lsss[c] * (1.f - S.Lsss[c]);
    }
    d[6] = d[7] = 0.f;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (k < 6) io[lane * NL::IO + 6 + k] = d[k];
      Y3[(size_t)k * P + P0 + lane] = M::cvt(d[k]);
    }
  }
  __syncthreads();
  // ---- D: backward through the network to its inputs
  {
    Op Bo[NS::KT_O][4];
#pragma unroll
    for (int ks = 0; ks < NS::KT_O; ks++)
#pragma unroll
      for (int nb = 0; nb < 4; nb++) {
        const float *r = io + (16 * nb + col) * NL::IO + 6;
        if constexpr (M::KPL == 8) {
          bf16x8 v;
#pragma unroll
          for (int j = 0; j < 8; j++) {
            const int o = feat_index<M>(false, ks, g, j);
            v[j] = (__bf16)(o < 6 ? r[o] : 0.f);
          }
          Bo[ks][nb] = v;
        } else {
          const int o = feat_index<M>(false, ks, g, 0);
          Bo[ks][nb] = o < 6 ? r[o] : 0.f;
        }
      }
    f32x4 dH[MB][4];
    Op Bd[NS::KSH][4];
    __builtin_amdgcn_sched_barrier(0);
    layer_mma<M, MB, NS::KT_O>(tops + NS::T0 + 2 * NS::TH, Bo, dH, lane);
    m3.apply(dH);
    d_to_operand<M, MB>(dH, Y2, P, P0, lane);
    grad_to_ops<M, MB>(dH, Bd);
    __builtin_amdgcn_sched_barrier(0);
    layer_mma<M, MB, NS::KT_H>(tops + NS::T0 + NS::TH, Bd, dH, lane);
    m2.apply(dH);
    d_to_operand<M, MB>(dH, Y1, P, P0, lane);
    grad_to_ops<M, MB>(dH, Bd);
    __builtin_amdgcn_sched_barrier(0);
    layer_mma<M, MB, NS::KT_H>(tops + NS::T0, Bd, dH, lane);
    m1.apply(dH);
    d_to_operand<M, MB>(dH, Y0, P, P0, lane);
    grad_to_ops<M, MB>(dH, Bd);
    f32x4 dX[NS::MB0][4];
    __builtin_amdgcn_sched_barrier(0);
    layer_mma<M, NS::MB0, NS::KT_H>(tops, Bd, dX, lane);
#pragma unroll
    for (int mb = 0; mb < NS::MB0; mb++)
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
#pragma unroll
        for (int j = 0; j < 4; j++) dxin[(16 * nb + col) * NL::DS + 16 * mb + 4 * g + j] = dX[mb][nb][j];
  }
  __syncthreads();
  // ---- E: per pixel backward of geometry, BRDF and Eq. 7
  {
    float gb[C], T, gL[3], dgbar[C];
    load_pixel<C>(A, inside, pix, HW, gb, T, gL);
    PixShade S;
    shade_geometry<C>(gb, T, uc, vc, A.cam, A.light, true, S);
    if (S.bg) gL[0] = gL[1] = gL[2] = 0.f;
    float o[6];
    for (int k = 0; k < 6; k++) o[k] = io[lane * NL::IO + k];
    combine_net(S, gb[kChSss], o);
    const float dA = shade_pixel_bwd<C, F, 1>(S, gb, gL, A.light, dxin + lane * NL::DS, dgbar);
    write_pixel_grads<C, F>(A, inside, pix, HW, S, gb, dgbar, dA);
  }
}

// Elements of the generic form's weight-gradient operands per pixel.
size_t net_operand_elems(int width, int in_pad) { return (size_t)in_pad + 6 * (size_t)width + 8; }

template <int F, int NET, int WIDTH, int IN_PAD>
void launch_shade_bwd_t(const ShadeArgs &a, hipStream_t st) {
  const int tiles = a.cam.TX * a.cam.TY;
  if constexpr (NET == 1 || NET == 2) {
    shade_bwd_net_kernel<F, typename NetTraits<NET>::M, WIDTH, IN_PAD><<<tiles * 4, 64, 0, st>>>(a);
  } else {
    shade_bwd_plain_kernel<F, NET><<<tiles, 256, 0, st>>>(a);
  }
}

#define SSSGS_SHADE_BWD(F, NET, WIDTH, IN_PAD) \
  template void launch_shade_bwd_t<F, NET, WIDTH, IN_PAD>(const ShadeArgs &, hipStream_t);
SSSGS_SHADE_INSTANCES(SSSGS_SHADE_BWD)

}  // namespace sssgs
