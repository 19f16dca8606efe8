// shade_bwd.hip -- backward of the per-pixel deferred shading (Sec. 3.2,
// Eq. 4, 6, 7): from dL/d(rgb) to dL/d(G-buffer), dL/d(T_final) and the
// network parameter gradients.
//
// Persistent grid; each wave shades 64-pixel strips (16 x 4).  The network
// forward is recomputed (layer 3 input kept, layers 1-2 recomputed as
// needed); input gradients use the transposed weights on the matrix cores
// (dX^T = W^T dY^T, consuming the accumulator layout directly); weight
// gradients dW = dY^T X are computed per workgroup over the strips of all its
// waves (K = 64 x waves pixels, staged through LDS) and added to a
// per-workgroup partial; the first strips store, later ones add with
// no-return float atomics, so no wave stalls on a read-modify-write, and
// every address is written by one wave only, so the sums are deterministic.
#include "launch.hpp"
#include "net_bwd.hpp"

namespace sssgs {

// Staging of the weight-gradient operands.  For BF16 (8 pixels per lane and
// k-step) both factors are stored feature-major [feat][px]; for FP32 (one
// pixel per lane and k-step) pixel-major [px][feat].
template <class M>
struct Stage {
  static constexpr bool FM = M::KPL == 8;  // feature-major
  static constexpr int PXS = 64 + 8;       // feature-major row stride (elements)
  __device__ static __forceinline__ int idx(int feat, int px, int fstride) {
    return FM ? feat * PXS + px : px * fstride + feat;
  }
};

// Workgroup weight gradient of one layer over the NW strips its waves have
// staged (K = 64 NW pixels): dW[o][k] = sum_p dY[o][p] X[k][p] and the bias
// gradient db[o] = sum_p dY[o][p] (the product with an all-ones column).
// Wave w computes the 16-row blocks mbo = w, w + NW, ... and stores them
// into (first call) or adds them to (later calls, with no-return float
// atomics) the workgroup's partial at W offset woff (row-major [rows][cols])
// and bias offset boff.  Every address of the partial is written by one wave
// only, so the sums are deterministic.
template <class M, int ROWS16, int KCOLS, int NW>
__device__ __forceinline__ void dw_block(const typename M::Elem *st_all, int stage_elems, int fst,
                                         float *__restrict__ part, int woff, int boff, int rows, int cols,
                                         bool first, int w, int lane) {
  using Op = typename M::Op;
  using E = typename M::Elem;
  using ST = Stage<M>;
  constexpr int MBO = ROWS16 / 16, NBK = KCOLS / 16, KSW = 64 / M::KS;
  const int g = lane >> 4, col = lane & 15;
  Op ones;
  if constexpr (M::KPL == 8) {
#pragma unroll
    for (int j = 0; j < 8; j++) ones[j] = (__bf16)(col == 0 ? 1.f : 0.f);
  } else {
    ones = col == 0 ? 1.f : 0.f;
  }
#pragma unroll 1
  for (int mbo = w; mbo < MBO; mbo += NW) {
    f32x4 acc[NBK + 1];
#pragma unroll
    for (int nbk = 0; nbk <= NBK; nbk++) acc[nbk] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int v = 0; v < NW; v++) {
      const E *dy = st_all + v * 2 * stage_elems;
      const E *xk = dy + stage_elems;
#pragma unroll
      for (int ks = 0; ks < KSW; ks++) {
        const int px0 = ks * M::KS + g * M::KPL;
        Op a;
        if constexpr (M::KPL == 8) a = *reinterpret_cast<const bf16x8 *>(dy + ST::idx(16 * mbo + col, px0, fst));
        else a = dy[ST::idx(16 * mbo + col, px0, fst)];
#pragma unroll
        for (int nbk = 0; nbk < NBK; nbk++) {
          Op b;
          if constexpr (M::KPL == 8) b = *reinterpret_cast<const bf16x8 *>(xk + ST::idx(16 * nbk + col, px0, fst));
          else b = xk[ST::idx(16 * nbk + col, px0, fst)];
          acc[nbk] = M::mma(a, b, acc[nbk]);
        }
        acc[NBK] = M::mma(a, ones, acc[NBK]);
      }
    }
    // D layout: lane (col, g) holds dW[16 mbo + 4 g + j][16 nbk + col]; the bias in column 0
#pragma unroll
    for (int nbk = 0; nbk < NBK; nbk++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int o = 16 * mbo + 4 * g + j, k = 16 * nbk + col;
        if (o < rows && k < cols) {
          float *p = part + woff + o * cols + k;
          if (first) *p = acc[nbk][j];
          else atomicAdd(p, acc[nbk][j]);
        }
      }
    if (col == 0)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int o = 16 * mbo + 4 * g + j;
        if (o < rows) {
          float *p = part + boff + o;
          if (first) *p = acc[NBK][j];
          else atomicAdd(p, acc[NBK][j]);
        }
      }
  }
}

// Write D-layout values (feature f = 16 mb + 4 g + j, pixel 16 nb + col) into a stage.
template <class M, int MB>
__device__ __forceinline__ void stage_d(const f32x4 (&d)[MB][4], typename M::Elem *st, int fstride, int lane) {
  using ST = Stage<M>;
  const int g = lane >> 4, col = lane & 15;
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
#pragma unroll
      for (int j = 0; j < 4; j++) st[ST::idx(16 * mb + 4 * g + j, 16 * nb + col, fstride)] = M::cvt(d[mb][nb][j]);
}

// Write B-operand activations (permuted features) into a stage at their true feature index.
template <class M, int KSN>
__device__ __forceinline__ void stage_ops(const typename M::Op (&H)[KSN][4], typename M::Elem *st, int fstride,
                                          int lane) {
  using ST = Stage<M>;
  const int g = lane >> 4, col = lane & 15;
#pragma unroll
  for (int ks = 0; ks < KSN; ks++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      if constexpr (M::KPL == 8) {
#pragma unroll
        for (int j = 0; j < 8; j++) st[ST::idx(feat_index<M>(false, ks, g, j), 16 * nb + col, fstride)] = H[ks][nb][j];
      } else {
        st[ST::idx(feat_index<M>(false, ks, g, 0), 16 * nb + col, fstride)] = H[ks][nb];
      }
    }
}

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
#pragma unroll
    for (int oct = 0; oct < 6; oct++) {
      const float sc = (float)(1 << oct);
      float cs[3], sn[3];
#pragma unroll
      for (int ax = 0; ax < 3; ax++) {
        sn[ax] = sinpif(sc * S.x[ax]);
        cs[ax] = cospif(sc * S.x[ax]);
      }
#pragma unroll
      for (int ax = 0; ax < 3; ax++) dx[ax] += dnet_in[p + ax] * (sc * kPi) * cs[ax];
#pragma unroll
      for (int ax = 0; ax < 3; ax++) dx[ax] -= dnet_in[p + 3 + ax] * (sc * kPi) * sn[ax];
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

// Waves per workgroup: bounded by the LDS each wave needs (160 KB per CU).
template <int NET, int WIDTH, int IN_PAD> struct BwdWaves {
  static constexpr int value = !kIsNet<NET> ? 4 : ((NET == 2 && WIDTH == 64 && IN_PAD == 64) ? 4 : 2);
};

int shade_bwd_waves(int net, int width, int in_pad) {
  return (net == 0 || net == 3) ? 4 : ((net == 2 && width == 64 && in_pad == 64) ? 4 : 2);
}

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
  A.dT[pix] = dT;
#pragma unroll
  for (int k = 0; k < C; k++) {
    float v = S.bg ? 0.f : dgbar[k] * S.ia;
    if (A.dgbuf_ext) v += A.dgbuf_ext[k * HW + pix];
    A.dG[k * HW + pix] = v;
  }
}

template <int F, int NET, int WIDTH, int IN_PAD>
__global__ __launch_bounds__((BwdWaves<NET, WIDTH, IN_PAD>::value * 64)) void shade_bwd_kernel(ShadeArgs A, int nstrips) {
  using M = typename NetTraits<NET>::M;
  using E = typename M::Elem;
  using Op = typename M::Op;
  using NS = NetShape<M, WIDTH, IN_PAD>;
  using PO = ParamOffsets<WIDTH, IN_PAD>;
  using ST = Stage<M>;
  constexpr int NW = BwdWaves<NET, WIDTH, IN_PAD>::value;
  constexpr int C = kChFeat + F;
  constexpr int MB = NS::MB;
  constexpr int XS = IN_PAD + XPad<M>::value;
  constexpr int FMAX = WIDTH > IN_PAD ? WIDTH : IN_PAD;
  constexpr int FST = FMAX + 4;  // pixel-major stage stride (FP32)
  constexpr int STAGE_ELEMS = ST::FM ? FMAX * ST::PXS : 64 * FST;
  constexpr int XS_ELEMS = 64 * XS;
  // per wave: network input rows, two weight-gradient stages, outputs + their gradients
  constexpr bool NETW = kIsNet<NET>;
  __shared__ E xs_all[NETW ? NW * XS_ELEMS : 1];
  __shared__ E st_all[NETW ? NW * 2 * STAGE_ELEMS : 1];
  __shared__ float io_all[NETW ? NW * 64 * 16 : 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  E *xs = xs_all + (NETW ? w * XS_ELEMS : 0);
  E *sdy = st_all + (NETW ? w * 2 * STAGE_ELEMS : 0);
  E *sxk = sdy + (NETW ? STAGE_ELEMS : 0);
  float *io = io_all + (NETW ? w * 64 * 16 : 0);  // [px][0..7] outputs, [px][8..15] output gradients
  float *dxin = reinterpret_cast<float *>(sdy);  // [64][IN_PAD + 1] after the last weight gradient
  float *part = A.mlp_partials ? A.mlp_partials + (size_t)blockIdx.x * A.nparams : nullptr;
  const size_t HW = (size_t)A.cam.W * A.cam.H;
  bool first = true;
  for (int s0 = blockIdx.x * NW; s0 < nstrips; s0 += gridDim.x * NW) {
    const int strip = s0 + w;
    const int tile = strip >> 2, sub = strip & 3;
    const int tx = tile % A.cam.TX, ty = tile / A.cam.TX;
    const int px = tx * kTile + (lane & 15), py = ty * kTile + 4 * sub + (lane >> 4);
    const bool inside = strip < nstrips && px < A.cam.W && py < A.cam.H;
    const size_t pix = inside ? (size_t)py * A.cam.W + px : 0;
    const float uc = (float)px + 0.5f, vc = (float)py + 0.5f;
    if constexpr (!NETW) {
      float gb[C], T, gL[3], dgbar[C];
      load_pixel<C>(A, inside, pix, HW, gb, T, gL);
      PixShade S;
      shade_geometry<C>(gb, T, uc, vc, A.cam, A.light, NET == 3, S);
      if constexpr (NET == 3) combine_features(S, gb);
      if (S.bg) gL[0] = gL[1] = gL[2] = 0.f;
      const float dA = shade_pixel_bwd<C, F, NET == 3 ? 2 : 0>(S, gb, gL, A.light, nullptr, dgbar);
      write_pixel_grads<C, F>(A, inside, pix, HW, S, gb, dgbar, dA);
    } else {
      // Weight operands are re-read for every strip (cache hits): an opaque
      // zero offset keeps the compiler from hoisting these loop-invariant
      // loads out of the persistent loop, which would pin them in registers.
      int z;
      asm volatile("v_mov_b32 %0, 0" : "=v"(z));
      const Op *wops = reinterpret_cast<const Op *>(A.wops) + z;
      const Op *tops = reinterpret_cast<const Op *>(A.tops) + z;
      // ---- A: network input rows
      {
        float gb[C], T, gL[3];
        load_pixel<C>(A, inside, pix, HW, gb, T, gL);
        PixShade S;
        shade_geometry<C>(gb, T, uc, vc, A.cam, A.light, true, S);
        build_net_input<F, IN_PAD, M>(gb, S, xs + lane * XS);
      }
      __syncthreads();
      // ---- B: network forward; keep the layer-3 input and the ReLU masks
      Mask<MB> m1, m2, m3;
      Op H3[NS::KSH][4];
      {
        f32x4 acc[MB][4];
        Op H[NS::KSH][4];
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      layer0_mma<M, MB, NS::KS0>(wops, xs, XS, acc, lane);
        m1.set_from(acc, A.params + PO::b(0), g);
        acc_to_ops<M, MB>(acc, A.params + PO::b(0), g, H);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      layer_mma<M, MB, NS::KSH>(wops + NS::L0, H, acc, lane);
        m2.set_from(acc, A.params + PO::b(1), g);
        acc_to_ops<M, MB>(acc, A.params + PO::b(1), g, H);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      layer_mma<M, MB, NS::KSH>(wops + NS::L0 + NS::LH, H, acc, lane);
        m3.set_from(acc, A.params + PO::b(2), g);
        acc_to_ops<M, MB>(acc, A.params + PO::b(2), g, H3);
      }
      {
        f32x4 oacc[1][4];
        layer_mma<M, 1, NS::KSH>(wops + NS::L0 + 2 * NS::LH, H3, oacc, lane);
        if (g < 2)
#pragma unroll
          for (int nb = 0; nb < 4; nb++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
              const int o = 4 * g + j;
              io[(16 * nb + col) * 16 + o] = oacc[0][nb][j] + (o < 6 ? A.params[PO::b(3) + o] : 0.f);
            }
      }
      __syncthreads();
      // ---- C: per pixel, Eq. 7 and the gradient of the network outputs
      {
        float gb[C], T, gL[3];
        load_pixel<C>(A, inside, pix, HW, gb, T, gL);
        PixShade S;
        shade_geometry<C>(gb, T, uc, vc, A.cam, A.light, true, S);
        if (S.bg) gL[0] = gL[1] = gL[2] = 0.f;
        float o[6];
        for (int k = 0; k < 6; k++) o[k] = io[lane * 16 + k];
        combine_net(S, gb[kChSss], o);
        const float sss = gb[kChSss] * S.ia;
        for (int c = 0; c < 3; c++) {
          const float gLo = S.a * gL[c];
          const float dLin = gLo * (1.f - sss) * (S.fs[c] + S.fd[c]) * S.cosI;
          io[lane * 16 + 8 + c] = o[c] > 0.f ? dLin : 0.f;
          io[lane * 16 + 11 + c] = gLo * sss * S.Lsss[c] * (1.f - S.Lsss[c]);
        }
        io[lane * 16 + 14] = 0.f;
        io[lane * 16 + 15] = 0.f;
      }
      __syncthreads();
      // ---- D: network backward
      Op Bd[NS::KSH][4];
      {
        f32x4 dO[1][4];
#pragma unroll
        for (int nb = 0; nb < 4; nb++)
#pragma unroll
          for (int j = 0; j < 4; j++) dO[0][nb][j] = (g < 2) ? io[(16 * nb + col) * 16 + 8 + 4 * g + j] : 0.f;
        stage_d<M, 1>(dO, sdy, FST, lane);
        stage_ops<M, NS::KSH>(H3, sxk, FST, lane);
        __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      dw_block<M, 16, WIDTH, NW>(st_all, STAGE_ELEMS, FST, part, PO::w(3), PO::b(3), 6, WIDTH, first, w, lane);
        Op Bo[NS::KT_O][4];
#pragma unroll
        for (int ks = 0; ks < NS::KT_O; ks++)
#pragma unroll
          for (int nb = 0; nb < 4; nb++) {
            if constexpr (M::KPL == 8) {
              bf16x8 v;
#pragma unroll
              for (int j = 0; j < 8; j++) v[j] = (__bf16)(j < 4 ? dO[0][nb][j] : 0.f);
              Bo[ks][nb] = v;
            } else {
              Bo[ks][nb] = dO[0][nb][ks];
            }
          }
        f32x4 dH[MB][4];
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      layer_mma<M, MB, NS::KT_O>(tops + NS::T0 + 2 * NS::TH, Bo, dH, lane);
        m3.apply(dH);                       // upstream of layer 2's pre-activation
        __syncthreads();
        stage_d<M, MB>(dH, sdy, FST, lane);
        grad_to_ops<M, MB>(dH, Bd);
      }
#pragma unroll 1
      for (int l = 2; l >= 1; l--) {
        // recompute this layer's input h_l from the input rows
        {
          f32x4 acc[MB][4];
          Op H[NS::KSH][4];
          __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      layer0_mma<M, MB, NS::KS0>(wops, xs, XS, acc, lane);
          acc_to_ops<M, MB>(acc, A.params + PO::b(0), g, H);
          if (l == 2) {
            __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      layer_mma<M, MB, NS::KSH>(wops + NS::L0, H, acc, lane);
            acc_to_ops<M, MB>(acc, A.params + PO::b(1), g, H);
          }
          stage_ops<M, NS::KSH>(H, sxk, FST, lane);
        }
        __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      dw_block<M, WIDTH, WIDTH, NW>(st_all, STAGE_ELEMS, FST, part, PO::w(l), PO::b(l), WIDTH, WIDTH, first, w,
                                    lane);
        f32x4 dH[MB][4];
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      layer_mma<M, MB, NS::KT_H>(tops + NS::T0 + (l - 1) * NS::TH, Bd, dH, lane);
        if (l == 2) m2.apply(dH);
        else m1.apply(dH);
        __syncthreads();
        stage_d<M, MB>(dH, sdy, FST, lane);
        grad_to_ops<M, MB>(dH, Bd);
      }
      // layer 0: weight gradient with the input rows, input gradient W0^T dpre0
      for (int k = 0; k < IN_PAD; k++) sxk[ST::idx(k, lane, FST)] = xs[lane * XS + k];
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
      dw_block<M, WIDTH, IN_PAD, NW>(st_all, STAGE_ELEMS, FST, part, PO::w(0), PO::b(0), WIDTH, IN_PAD, first, w,
                                     lane);
      {
        f32x4 dX[NS::MB0][4];
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_sched_barrier(0);
      layer_mma<M, NS::MB0, NS::KT_H>(tops, Bd, dX, lane);
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < NS::MB0; mb++)
#pragma unroll
          for (int nb = 0; nb < 4; nb++)
#pragma unroll
            for (int j = 0; j < 4; j++) dxin[(16 * nb + col) * (IN_PAD + 1) + 16 * mb + 4 * g + j] = dX[mb][nb][j];
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
        for (int k = 0; k < 6; k++) o[k] = io[lane * 16 + k];
        combine_net(S, gb[kChSss], o);
        const float *din = dxin + lane * (IN_PAD + 1);
        const float dA = shade_pixel_bwd<C, F, 1>(S, gb, gL, A.light, din, dgbar);
        write_pixel_grads<C, F>(A, inside, pix, HW, S, gb, dgbar, dA);
      }
      first = false;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- split form
//
// For the BF16 width-64 network the weight gradients are left to a kernel of
// their own (mlp_wgrad.hip).  This kernel then only needs, per wave, the input
// rows until layer 0 has consumed them, dL/d(input) afterwards (same LDS),
// and the network outputs with their gradients: about 20 KB, and no
// workgroup-wide exchange, so each wave shades one strip on its own and two
// waves fit per SIMD.  For the weight-gradient kernel it leaves a record per
// strip: the BF16 network input rows as layer 0 reads them ([64][IN_PAD]) and
// the BF16 gradients of the six network outputs as the transposed output
// layer reads them ([64][8], two zero pads).
template <int IN_PAD>
struct SplitLds {
  static constexpr int XS = IN_PAD + XPad<MmaBF16>::value;  // bf16 input row stride
  static constexpr int DS = IN_PAD + 1;                     // fp32 input-gradient row stride
  static constexpr int IO = 13;  // floats per pixel: 6 outputs, 6 output gradients, pad
  static constexpr int RB = (64 * XS * 2 > 64 * DS * 4) ? 64 * XS * 2 : 64 * DS * 4;
  static constexpr int BYTES = RB + 64 * IO * 4;
};

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
  const int strip = blockIdx.x;
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
    const uint4 *src = reinterpret_cast<const uint4 *>(xs + lane * SL::XS);
    uint4 *dst = reinterpret_cast<uint4 *>(rec_x + rrow * IN_PAD);
#pragma unroll
    for (int k = 0; k < IN_PAD / 8; k++) dst[k] = src[k];
  }
  __syncthreads();
  // ---- B: network forward: ReLU masks and outputs
  Mask<MB> m1, m2, m3;
  {
    f32x4 acc[MB][4];
    Op H[NS::KSH][4];
    layer0_mma<M, MB, NS::KS0>(wops, xs, SL::XS, acc, lane);
    acc_to_ops<M, MB>(acc, A.params + PO::b(0), g, H);
    m1.set_from_ops(H);
    layer_mma<M, MB, NS::KSH>(wops + NS::L0, H, acc, lane);
    acc_to_ops<M, MB>(acc, A.params + PO::b(1), g, H);
    m2.set_from_ops(H);
    layer_mma<M, MB, NS::KSH>(wops + NS::L0 + NS::LH, H, acc, lane);
    acc_to_ops<M, MB>(acc, A.params + PO::b(2), g, H);
    m3.set_from_ops(H);
    f32x4 oacc[1][4];
    layer_mma<M, 1, NS::KSH>(wops + NS::L0 + 2 * NS::LH, H, oacc, lane);
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
  // ---- C: Eq. 7 and the gradients of the network outputs
  {
    float gb[C], T, gL[3];
    load_pixel<C>(A, inside, pix, HW, gb, T, gL);
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
    float gb[C], T, gL[3], dgbar[C];
    load_pixel<C>(A, inside, pix, HW, gb, T, gL);
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
template void launch_shade_bwd_split_t<32, 96>(const ShadeArgs &, __bf16 *, __bf16 *, hipStream_t);

// Workgroups of the persistent grid: every workgroup gets at least one strip.
int shade_bwd_grid(int net, int width, int in_pad, int tiles, int max_blocks) {
  const int nw = shade_bwd_waves(net, width, in_pad), nstrips = tiles * 4;
  int grid = (nstrips + nw - 1) / nw;
  if (grid > max_blocks) grid = max_blocks;
  return grid < 1 ? 1 : grid;
}

template <int F, int NET, int WIDTH, int IN_PAD>
void launch_shade_bwd_t(const ShadeArgs &a, int nblocks, hipStream_t st) {
  constexpr int NW = BwdWaves<NET, WIDTH, IN_PAD>::value;
  const int grid = shade_bwd_grid(NET, WIDTH, IN_PAD, a.cam.TX * a.cam.TY, nblocks);
  shade_bwd_kernel<F, NET, WIDTH, IN_PAD><<<grid, NW * 64, 0, st>>>(a, a.cam.TX * a.cam.TY * 4);
}

#define SSSGS_SHADE_BWD(F, NET, WIDTH, IN_PAD) \
  template void launch_shade_bwd_t<F, NET, WIDTH, IN_PAD>(const ShadeArgs &, int, hipStream_t);
SSSGS_SHADE_INSTANCES(SSSGS_SHADE_BWD)

}  // namespace sssgs
