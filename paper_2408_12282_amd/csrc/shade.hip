// shade.hip -- per-pixel deferred shading (Sec. 3.2 "Per-Pixel Deferred
// Shading"): GGX BRDF (Eq. 4), residual network (Eq. 6, per pixel, or its
// per-Gaussian outputs composited into the G-buffer) and the SSS/BRDF
// combination (Eq. 7), forward, for one or several point lights over the same
// G-buffer (image-based lighting as a weighted sum of light samples, paper
// appendix "Image Based Lighting").  The backward lives in shade_bwd.hip.
//
// One 256-lane workgroup per 16x16 tile; wave w owns rows 4w..4w+3.  Each lane
// shades its pixel; the network runs per wave on the matrix cores with the
// wave's 64 pixels as the N dimension (see mlp.hpp).
#include "shade_common.hpp"

namespace sssgs {

// LDS writes of this wave visible to its own later reads (all lanes).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// MULTI = false: one light of weight 1 written (not added) -- the plain
// forward, compiled without the light loop.
template <int F, int NET, int WIDTH, int IN_PAD, bool MULTI>
__global__ __launch_bounds__(256) void shade_fwd_kernel(ShadeArgs A, MultiLight ML) {
  using M = typename NetTraits<NET>::M;
  using E = typename M::Elem;
  constexpr int C = kChFeat + F;
  constexpr int XS = in_row_stride<M, IN_PAD>();  // LDS row stride (elements)
  __shared__ E xs[kIsNet<NET> ? 4 * 64 * XS : 1];
  __shared__ float outs[kIsNet<NET> ? 4 * 64 * 8 : 1];
  const int tile = xcd_item(blockIdx.x, gridDim.x);
  const int tx = tile % A.cam.TX, ty = tile / A.cam.TX;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < A.cam.W && py < A.cam.H;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t HW = (size_t)A.cam.W * A.cam.H, pix = inside ? (size_t)py * A.cam.W + px : 0;
  float gb[C];
  float T = 1.f;
  if (inside) {
#pragma unroll
    for (int c = 0; c < C; c++) gb[c] = A.gbuf[c * HW + pix];
    T = A.t_final[pix];
  } else {
#pragma unroll
    for (int c = 0; c < C; c++) gb[c] = 0.f;
  }
  E *xrow = xs + (w * 64 + lane) * XS;
  float acc[3] = {0.f, 0.f, 0.f};
  const int K = MULTI ? ML.K : 1;
  for (int k = 0; k < K; k++) {
    if constexpr (MULTI && kIsNet<NET>) {
      // opaque per light: keeps the light-independent terms derived from the
      // G-buffer inside the loop instead of live across it and the network
#pragma unroll
      for (int c = 0; c < C; c++) asm volatile("" : "+v"(gb[c]));
      asm volatile("" : "+v"(T));
    }
    LightArgs L;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      L.pos[c] = ML.pos[k][c];
      L.intensity[c] = ML.intensity[k][c];
    }
    PixShade S;
    shade_geometry<C>(gb, T, (float)px + 0.5f, (float)py + 0.5f, A.cam, L, NET != 0, S);
    if constexpr (NET == 3) {
      combine_features(S, gb);
    } else if constexpr (NET != 0) {
      // the network input row differs between lights only in w_i
      if (k == 0) build_net_input<F, IN_PAD, M>(gb, S, xrow);
      else set_net_light<F, IN_PAD, M>(S, xrow);
      // each wave reads and writes only its own rows: a wave-level fence
      // suffices, and the four waves run the network independently
      wave_sync();
      // Over several lights an opaque zero offset keeps the compiler from
      // hoisting the loop-invariant weight and bias loads out of the light
      // loop, which would hold every layer's operands in registers at once.
      int z = 0;
      if constexpr (MULTI) asm volatile("v_mov_b32 %0, 0" : "=v"(z));
      net_forward_wave<M, WIDTH, IN_PAD, false>(reinterpret_cast<const char *>(A.wops) + z, A.params + z,
                                                xs + w * 64 * XS, XS, outs + w * 64 * 8, nullptr);
      wave_sync();
      combine_net(S, gb[kChSss], outs + (w * 64 + lane) * 8);
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const float v = (S.bg ? 0.f : S.a * S.L[c]) + T * A.bgc[c];
      acc[c] = MULTI ? __fmaf_rn(ML.weight[k][c], v, acc[c]) : v;
    }
  }
  if (inside) {
#pragma unroll
    for (int c = 0; c < 3; c++)
      A.rgb[c * HW + pix] = (MULTI && ML.accumulate) ? A.rgb[c * HW + pix] + acc[c] : acc[c];
    if (A.alpha) A.alpha[pix] = 1.f - T;
  }
}

template <int F, int NET, int WIDTH, int IN_PAD>
void launch_shade_fwd_t(const ShadeArgs &a, const MultiLight &ml, hipStream_t st) {
  bool multi = ml.K != 1 || ml.accumulate;
  for (int c = 0; c < 3; c++) multi = multi || ml.weight[0][c] != 1.f;
  if (multi) shade_fwd_kernel<F, NET, WIDTH, IN_PAD, true><<<a.cam.TX * a.cam.TY, 256, 0, st>>>(a, ml);
  else shade_fwd_kernel<F, NET, WIDTH, IN_PAD, false><<<a.cam.TX * a.cam.TY, 256, 0, st>>>(a, ml);
}

#define SSSGS_SHADE_FWD(F, NET, WIDTH, IN_PAD) \
  template void launch_shade_fwd_t<F, NET, WIDTH, IN_PAD>(const ShadeArgs &, const MultiLight &, hipStream_t);
SSSGS_SHADE_INSTANCES(SSSGS_SHADE_FWD)

}  // namespace sssgs
