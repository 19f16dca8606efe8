// shade_common.hpp -- per-pixel shading math shared by the forward and
// backward shading kernels, and the wave-level network forward.
#pragma once
#include "mlp.hpp"

namespace sssgs {

struct ShadeArgs {
  CamArgs cam;
  LightArgs light;
  const float *gbuf;     // [C][H][W] premultiplied
  const float *t_final;  // [H][W]
  float *rgb;            // [3][H][W]
  float *alpha;          // [H][W] or null
  const void *wops;      // prepared forward weights (MmaF32::Op or MmaBF16::Op)
  const void *tops;      // prepared transposed weights (backward)
  const float *params;   // raw parameters (biases are read from here)
  // backward
  const float *drgb, *dgbuf_ext, *dalpha_ext;
  float *dG;             // [C][H][W] out
  float *dT;             // [H][W] out
  float *mlp_partials;   // [gridDim.x][nparams] out
  int nparams;
  float4 *zero_buf;      // or null: cleared by the split shading backward (the
  size_t zero_count4;    // compositing backward's accumulators, in float4)
  // generic network backward: forward weights with natural K order in every
  // layer, and the weight-gradient operands [rows][gP] it stores
  const void *nops;
  void *gx, *gdy;
  size_t gP;
  // colour behind the Gaussians: rgb = a L_out + T_final bgc
  float bgc[3];
};

// Point lights of one shading pass (image-based lighting by a sum over light
// samples): rgb = sum_k weight_k * (the single-light image of light k),
// added to the existing rgb when `accumulate` is set.
constexpr int kMaxLights = 32;
struct MultiLight {
  int K, accumulate;
  float pos[kMaxLights][3], intensity[kMaxLights][3], weight[kMaxLights][3];
};

// Shading modes NET: 0 point-light fall-off without network, 1 per-pixel
// network in FP32, 2 per-pixel network in BF16, 3 radiances composited from
// a per-Gaussian network (feature planes 0-2 incident light, 3-5 SSS).
template <int NET> constexpr bool kIsNet = NET == 1 || NET == 2;

template <int NET> struct NetTraits { using M = MmaF32; };
template <> struct NetTraits<2> { using M = MmaBF16; };

template <class M> struct XPad { static constexpr int value = 4; };
template <> struct XPad<MmaBF16> { static constexpr int value = 8; };

// LDS row of one pixel's network input: [hi IN_PAD | lo IN_PAD | pad] in the
// BF16 form (see mlp.hpp), [value IN_PAD | pad] in the FP32 form.
template <class M, int IN_PAD>
constexpr int in_row_stride() { return M::NSPLIT * IN_PAD + XPad<M>::value; }

// Entry p of a network input row.
template <class M, int IN_PAD>
__device__ __forceinline__ void put_in(typename M::Elem *row, int p, float v) {
  if constexpr (M::NSPLIT == 2) {
    const __bf16 hi = (__bf16)v;
    row[p] = hi;
    row[IN_PAD + p] = (__bf16)(v - (float)hi);
  } else {
    row[p] = M::cvt(v);
  }
}

constexpr float kPi = 3.14159265358979323846f;

struct PixShade {
  bool bg;
  float a, ia;
  float nraw[3], nlen, n[3];
  float ray[3], x[3];
  float vo[3], lo, wo[3], vi[3], li, wi[3], hv[3], hl, h[3];
  float nov, nol, noh, voh, NoV, NoL, NoH, VoH, cosI;
  float ag, den, D, k, dv, dl, g1v, g1l, Gv, Q, w;
  float F0[3], F[3], fs[3], fd[3];
  float li2, Lin[3], Lsss[3];
  float L[3];
};

__device__ __forceinline__ float dot3(const float *a, const float *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// v / max(|v|, 1e-12); returns |v|
__device__ __forceinline__ float norm3(const float *v, float *o) {
  const float l = sqrtf(dot3(v, v));
  const float inv = 1.f / fmaxf(l, 1e-12f);
  o[0] = v[0] * inv; o[1] = v[1] * inv; o[2] = v[2] * inv;
  return l;
}

// Geometry and BRDF of one pixel from its premultiplied G-buffer values.
template <int C>
__device__ __forceinline__ void shade_geometry(const float *gb, float T, float uc, float vc, const CamArgs &cam,
                                               const LightArgs &light, bool net, PixShade &S) {
  S.a = 1.f - T;
  S.bg = !(S.a >= 1e-6f);
  S.ia = S.bg ? 0.f : 1.f / S.a;
  for (int k = 0; k < 3; k++) S.nraw[k] = gb[kChNrm + k] * S.ia;
  S.nlen = norm3(S.nraw, S.n);
  const float rc0 = (uc - cam.cx) / cam.fx, rc1 = (vc - cam.cy) / cam.fy;
  const float dbar = gb[kChDepth] * S.ia;
  for (int k = 0; k < 3; k++) {
    S.ray[k] = cam.R[k] * rc0 + cam.R[3 + k] * rc1 + cam.R[6 + k];
    S.x[k] = cam.Cw[k] + dbar * S.ray[k];
    S.vo[k] = cam.Cw[k] - S.x[k];
    S.vi[k] = light.pos[k] - S.x[k];
  }
  S.lo = norm3(S.vo, S.wo);
  S.li = norm3(S.vi, S.wi);
  for (int k = 0; k < 3; k++) S.hv[k] = S.wo[k] + S.wi[k];
  S.hl = norm3(S.hv, S.h);
  S.nov = dot3(S.n, S.wo);
  S.nol = dot3(S.n, S.wi);
  S.noh = dot3(S.n, S.h);
  S.voh = dot3(S.wo, S.h);
  S.NoV = fmaxf(S.nov, 1e-4f);
  S.NoL = fmaxf(S.nol, 1e-4f);
  S.NoH = fmaxf(S.noh, 0.f);
  S.VoH = fmaxf(S.voh, 0.f);
  S.cosI = fmaxf(S.nol, 0.f);
  const float r = gb[kChRough] * S.ia, m = gb[kChMetal] * S.ia;
  // GGX distribution, alpha = roughness^2
  S.ag = r * r;
  S.den = S.NoH * S.NoH * (S.ag * S.ag - 1.f) + 1.f;
  S.D = S.ag * S.ag / (kPi * S.den * S.den);
  // Smith / Schlick-GGX shadowing, k = (r + 1)^2 / 8
  S.k = (r + 1.f) * (r + 1.f) * 0.125f;
  S.dv = S.NoV * (1.f - S.k) + S.k;
  S.dl = S.NoL * (1.f - S.k) + S.k;
  S.g1v = S.NoV / S.dv;
  S.g1l = S.NoL / S.dl;
  S.Gv = S.g1v * S.g1l;
  S.Q = 1.f / (4.f * S.NoV * S.NoL);
  S.w = 1.f - S.VoH;
  const float w2 = S.w * S.w, w5 = w2 * w2 * S.w;
  for (int c = 0; c < 3; c++) {
    const float b = gb[kChAlb + c] * S.ia;
    S.F0[c] = 0.04f * (1.f - m) + b * m;
    S.F[c] = S.F0[c] + (1.f - S.F0[c]) * w5;
    S.fs[c] = S.D * S.F[c] * S.Gv * S.Q;
    S.fd[c] = (1.f - m) * b * (1.f / kPi);
  }
  if (!net) {
    S.li2 = fmaxf(dot3(S.vi, S.vi), 1e-12f);
    for (int c = 0; c < 3; c++) {
      S.Lin[c] = light.intensity[c] / S.li2;
      S.L[c] = (S.fs[c] + S.fd[c]) * S.Lin[c] * S.cosI;
    }
  }
}

// Network input [features | sin/cos(2^k pi x) | w_o | w_i | 0 ...] into an LDS row.
// sin and cos of pi 2^k x for the position encoding's six octaves: octaves 0
// and 3 from sinpi/cospi, the others by angle doubling (sin 2a = 2 sin a
// cos a, cos 2a = (cos a - sin a)(cos a + sin a)).  A doubling at most
// doubles the absolute error and adds one rounding, so every value is within
// a few ulp of the direct evaluation, well below the error the FP32 position
// itself carries into the top octave (its rounding times 32 pi).
__device__ __forceinline__ void pe_octaves(float x, float (&s)[6], float (&c)[6]) {
  s[0] = sinpif(x);
  c[0] = cospif(x);
  s[3] = sinpif(8.f * x);
  c[3] = cospif(8.f * x);
#pragma unroll
  for (int k = 1; k < 6; k++) {
    if (k == 3) continue;
    s[k] = 2.f * s[k - 1] * c[k - 1];
    c[k] = (c[k - 1] - s[k - 1]) * (c[k - 1] + s[k - 1]);
  }
}

template <int F, int IN_PAD, class M>
__device__ __forceinline__ void build_net_input(const float *gb, const PixShade &S, typename M::Elem *row) {
  int p = 0;
#pragma unroll
  for (int f = 0; f < F; f++) put_in<M, IN_PAD>(row, p++, gb[kChFeat + f] * S.ia);
  float sv[3][6], cv[3][6];
#pragma unroll
  for (int ax = 0; ax < 3; ax++) pe_octaves(S.x[ax], sv[ax], cv[ax]);
#pragma unroll
  for (int oct = 0; oct < 6; oct++) {
#pragma unroll
    for (int ax = 0; ax < 3; ax++) put_in<M, IN_PAD>(row, p++, sv[ax][oct]);
#pragma unroll
    for (int ax = 0; ax < 3; ax++) put_in<M, IN_PAD>(row, p++, cv[ax][oct]);
  }
#pragma unroll
  for (int k = 0; k < 3; k++) put_in<M, IN_PAD>(row, p++, S.wo[k]);
#pragma unroll
  for (int k = 0; k < 3; k++) put_in<M, IN_PAD>(row, p++, S.wi[k]);
#pragma unroll
  for (; p < IN_PAD; p++) put_in<M, IN_PAD>(row, p, 0.f);
}

// Only the incident-direction entries of a network input row (after the
// features, the position encoding and w_o).
template <int F, int IN_PAD, class M>
__device__ __forceinline__ void set_net_light(const PixShade &S, typename M::Elem *row) {
#pragma unroll
  for (int k = 0; k < 3; k++) put_in<M, IN_PAD>(row, F + kNumPE + 3 + k, S.wi[k]);
}

__device__ __forceinline__ void combine_net(PixShade &S, float sss_pre, const float *o) {
  const float sss = sss_pre * S.ia;
  for (int c = 0; c < 3; c++) {
    S.Lin[c] = fmaxf(o[c], 0.f);
    S.Lsss[c] = 1.f / (1.f + expf(-o[3 + c]));
    S.L[c] = sss * S.Lsss[c] + (1.f - sss) * (S.fs[c] + S.fd[c]) * S.Lin[c] * S.cosI;
  }
}

// Eq. 7 with the composited radiances of a per-Gaussian network (pipeline
// figure): the incident light and SSS radiance are blended like the other
// channels, so their pixel values are the feature planes over alpha.
__device__ __forceinline__ void combine_features(PixShade &S, const float *gb) {
  const float sss = gb[kChSss] * S.ia;
  for (int c = 0; c < 3; c++) {
    S.Lin[c] = gb[kChFeat + c] * S.ia;
    S.Lsss[c] = gb[kChFeat + 3 + c] * S.ia;
    S.L[c] = sss * S.Lsss[c] + (1.f - sss) * (S.fs[c] + S.fd[c]) * S.Lin[c] * S.cosI;
  }
}

// ----------------------------------------------------------------- network

// Offsets into the packed parameter vector.
template <int WIDTH, int IN_PAD>
struct ParamOffsets {
  static constexpr int w(int l) {  // three hidden layers, six outputs
    return l == 0 ? 0 : WIDTH * IN_PAD + WIDTH + (l - 1) * (WIDTH * WIDTH + WIDTH);
  }
  static constexpr int rows(int l) { return l == 3 ? 6 : WIDTH; }
  static constexpr int cols(int l) { return l == 0 ? IN_PAD : WIDTH; }
  static constexpr int b(int l) { return w(l) + rows(l) * cols(l); }
  static constexpr int total() { return b(3) + 6; }
};

template <class M>
__device__ __forceinline__ typename M::Op load_op_lds(const typename M::Elem *p) {
  if constexpr (M::KPL == 8) return *reinterpret_cast<const bf16x8 *>(p);
  else return *p;
}

// Pack the bias-added, ReLU-ed accumulators of a layer into the next layer's
// B operands (permuted K order, see feat_index): H the activations (BF16: hi),
// Hlo the BF16 remainders (unused in the FP32 form).
template <class M, int MB>
__device__ __forceinline__ void acc_to_ops(const f32x4 (&acc)[MB][4], const float *bias, int g,
                                           typename M::Op (&H)[(MB * 16) / M::KS][4],
                                           typename M::Op (&Hlo)[(MB * 16) / M::KS][4]) {
  constexpr int KSN = (MB * 16) / M::KS;
#pragma unroll
  for (int ks = 0; ks < KSN; ks++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      if constexpr (M::KPL == 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const int mb = 2 * ks + (j >> 2), jj = j & 3;
          v[j] = fmaxf(acc[mb][nb][jj] + bias[16 * mb + 4 * g + jj], 0.f);
        }
        pack_bf16x8_split(v, H[ks][nb], Hlo[ks][nb]);
      } else {
        const int mb = ks >> 2, jj = ks & 3;
        H[ks][nb] = fmaxf(acc[mb][nb][jj] + bias[16 * mb + 4 * g + jj], 0.f);
      }
    }
}

// One forward product from activation operands (K = KSN k-steps): acc =
// W H, and in the BF16 form + W Hlo.  The first k-step takes a literal zero
// accumulator (an inline constant, no register clears).
template <class M, int MB, int KSN>
__device__ __forceinline__ void act_mma(const typename M::Op *__restrict__ w, const typename M::Op (&H)[KSN][4],
                                        const typename M::Op (&Hlo)[KSN][4], f32x4 (&acc)[MB][4], int lane) {
#pragma unroll
  for (int ks = 0; ks < KSN; ks++)
#pragma unroll
    for (int mb = 0; mb < MB; mb++) {
      const typename M::Op a = w[(mb * KSN + ks) * 64 + lane];
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
        acc[mb][nb] = M::mma(a, H[ks][nb], ks == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[mb][nb]);
      if constexpr (M::NSPLIT == 2)
#pragma unroll
        for (int nb = 0; nb < 4; nb++) acc[mb][nb] = M::mma(a, Hlo[ks][nb], acc[mb][nb]);
    }
}

// Layer 0 from the LDS input rows (row stride XS; natural K order; in the
// BF16 form the remainders follow at offset IN_PAD).
template <class M, int MB, int KS0>
__device__ __forceinline__ void layer0_mma(const typename M::Op *__restrict__ w, const typename M::Elem *xs, int XS,
                                           f32x4 (&acc)[MB][4], int lane) {
  constexpr int IN_PAD = KS0 * M::KS;
  const int g = lane >> 4, col = lane & 15;
#pragma unroll
  for (int ks = 0; ks < KS0; ks++) {
    typename M::Op B[4], Blo[4];
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      const typename M::Elem *r = xs + (16 * nb + col) * XS + ks * M::KS + g * M::KPL;
      B[nb] = load_op_lds<M>(r);
      if constexpr (M::NSPLIT == 2) Blo[nb] = load_op_lds<M>(r + IN_PAD);
    }
#pragma unroll
    for (int mb = 0; mb < MB; mb++) {
      const typename M::Op a = w[(mb * KS0 + ks) * 64 + lane];
#pragma unroll
      for (int nb = 0; nb < 4; nb++) acc[mb][nb] = M::mma(a, B[nb], ks == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[mb][nb]);
      if constexpr (M::NSPLIT == 2)
#pragma unroll
        for (int nb = 0; nb < 4; nb++) acc[mb][nb] = M::mma(a, Blo[nb], acc[mb][nb]);
    }
  }
}

// Forward of the whole network for the wave's 64 pixels.  xs: LDS rows of
// the inputs (row stride XS).  Writes the 6 outputs of pixel p (bias added,
// before the output activations) to outs[p * 8 + o].
template <class M, int WIDTH, int IN_PAD, bool SAVE>
__device__ __forceinline__ void net_forward_wave(const void *wops_v, const float *__restrict__ params,
                                                 const typename M::Elem *xs, int XS, float *outs, void *) {
  using Op = typename M::Op;
  using NS = NetShape<M, WIDTH, IN_PAD>;
  using PO = ParamOffsets<WIDTH, IN_PAD>;
  constexpr int MB = NS::MB, KS0 = NS::KS0, KSH = NS::KSH;
  const Op *__restrict__ wops = reinterpret_cast<const Op *>(wops_v);
  const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
  f32x4 acc[MB][4];
  Op H[KSH][4], Hlo[KSH][4];
  layer0_mma<M, MB, KS0>(wops, xs, XS, acc, lane);
  acc_to_ops<M, MB>(acc, params + PO::b(0), g, H, Hlo);
  const Op *wl = wops + NS::L0;
  // hidden layers 1, 2
#pragma unroll
  for (int l = 1; l < 3; l++) {
    act_mma<M, MB, KSH>(wl, H, Hlo, acc, lane);
    acc_to_ops<M, MB>(acc, params + PO::b(l), g, H, Hlo);
    wl += NS::LH;
  }
  // output layer: 6 rows of one 16-row block
  f32x4 oacc[1][4];
  act_mma<M, 1, KSH>(wl, H, Hlo, oacc, lane);
  if (g < 2) {
    const float *bo = params + PO::b(3);
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int o = 4 * g + j;
        outs[(16 * nb + col) * 8 + o] = oacc[0][nb][j] + (o < 6 ? bo[o] : 0.f);
      }
  }
}

// Instances: (F, NET, WIDTH, IN_PAD), NET as for kIsNet.
#define SSSGS_SHADE_INSTANCES(X) \
  X(0, 0, 64, 64) X(0, 1, 64, 64) X(0, 2, 64, 64) X(0, 2, 128, 64) \
  X(8, 0, 64, 64) X(8, 1, 64, 64) X(8, 2, 64, 64) X(8, 2, 128, 64) X(8, 3, 64, 64) \
  X(16, 0, 64, 64) X(16, 1, 64, 64) X(16, 2, 64, 64) X(16, 2, 128, 64) \
  X(32, 0, 64, 96) X(32, 1, 64, 96) X(32, 2, 64, 96) X(32, 2, 128, 96)

}  // namespace sssgs
