// shade.hip -- per-pixel deferred shading (Sec. 3.2 "Per-Pixel Deferred
// Shading"): GGX BRDF (Eq. 4), residual network (Eq. 6) and the SSS/BRDF
// combination (Eq. 7), forward.  The backward lives in shade_bwd.hip.
//
// One 256-lane workgroup per 16x16 tile; wave w owns rows 4w..4w+3.  Each lane
// shades its pixel; the network runs per wave on the matrix cores with the
// wave's 64 pixels as the N dimension (see mlp.hpp).
#include "shade_common.hpp"

namespace sssgs {

template <int F, int NET, int WIDTH, int IN_PAD>
__global__ __launch_bounds__(256) void shade_fwd_kernel(ShadeArgs A) {
  using M = typename NetTraits<NET>::M;
  using E = typename M::Elem;
  constexpr int C = kChFeat + F;
  constexpr int XS = IN_PAD + XPad<M>::value;  // LDS row stride (elements)
  __shared__ E xs[NET ? 4 * 64 * XS : 1];
  __shared__ float outs[NET ? 4 * 64 * 8 : 1];
  const int tile = blockIdx.x;
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
  PixShade S;
  shade_geometry<C>(gb, T, (float)px + 0.5f, (float)py + 0.5f, A.cam, A.light, NET != 0, S);
  if constexpr (NET != 0) {
    E *xrow = xs + (w * 64 + lane) * XS;
    build_net_input<F, IN_PAD, M>(gb, S, xrow);
    __syncthreads();
    net_forward_wave<M, WIDTH, IN_PAD, false>(A.wops, A.params, xs + w * 64 * XS, XS, outs + w * 64 * 8, nullptr);
    __syncthreads();
    const float *o = outs + (w * 64 + lane) * 8;
    combine_net(S, gb[kChSss], o);
  }
  if (inside) {
#pragma unroll
    for (int c = 0; c < 3; c++) A.rgb[c * HW + pix] = S.bg ? 0.f : S.a * S.L[c];
    if (A.alpha) A.alpha[pix] = 1.f - T;
  }
}

template <int F, int NET, int WIDTH, int IN_PAD>
void launch_shade_fwd_t(const ShadeArgs &a, hipStream_t st) {
  shade_fwd_kernel<F, NET, WIDTH, IN_PAD><<<a.cam.TX * a.cam.TY, 256, 0, st>>>(a);
}

#define SSSGS_SHADE_FWD(F, NET, WIDTH, IN_PAD) \
  template void launch_shade_fwd_t<F, NET, WIDTH, IN_PAD>(const ShadeArgs &, hipStream_t);
SSSGS_SHADE_INSTANCES(SSSGS_SHADE_FWD)

}  // namespace sssgs
