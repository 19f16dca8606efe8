// composite.hip -- per-tile front-to-back alpha compositing of the deferred
// G-buffer (Sec. 3.1, Eq. 3) and its backward.
//
// One 256-lane workgroup per 16x16 tile, one pixel per lane.  Gaussian
// records of the tile's depth-ordered list are staged through LDS in batches
// of 256; each lane walks the batch, and the workgroup stops loading as soon
// as every pixel has terminated.  The backward walks the same list from each
// pixel's last contributor down, recovering transmittance by division instead
// of storing per-pixel lists, and reduces per-Gaussian gradients across the
// wavefront (DPP + readlane) before one vector atomic per Gaussian and wave.
#include "common.hpp"

namespace sssgs {

template <int C>
__global__ __launch_bounds__(256) void composite_fwd_kernel(const uint2 *__restrict__ ranges,
                                                            const uint32_t *__restrict__ sorted_g,
                                                            const float *__restrict__ records, int W, int H,
                                                            int TX, float *__restrict__ gbuf,
                                                            float *__restrict__ t_final,
                                                            uint32_t *__restrict__ n_contrib) {
  constexpr int RS = rec_stride(C);
  __shared__ float4 batch[256 * RS / 4];
  const int tile = blockIdx.x;
  const int tx = tile % TX, ty = tile / TX;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  float T = 1.f;
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; c++) acc[c] = 0.f;
  uint32_t last = 0;
  bool done = !inside;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += 256) {
    if (__syncthreads_count(done) == 256) break;
    const uint32_t e = b0 + threadIdx.x;
    if (e < rg.y) {
      const float *src = records + (size_t)sorted_g[e] * RS;
#pragma unroll
      for (int k = 0; k < RS / 4; k++) batch[threadIdx.x * (RS / 4) + k] = ld4(src + 4 * k);
    }
    __syncthreads();
    const int cnt = (int)min(256u, rg.y - b0);
    if (!done) {
      for (int j = 0; j < cnt; j++) {
        const float *r = reinterpret_cast<const float *>(&batch[j * (RS / 4)]);
        float dx, dy;
        const float pw = splat_power(r[0], r[1], r[2], r[3], r[4], pxc, pyc, dx, dy);
        if (pw > 0.f) continue;
        const float al = fminf(0.99f, splat_alpha_raw(r[5], pw));
        if (al < (1.f / 255.f)) continue;
        const float tn = T * (1.f - al);
        if (tn < 1e-4f) {
          done = true;
          break;
        }
        const float wgt = al * T;
#pragma unroll
        for (int c = 0; c < C; c++) acc[c] = __fmaf_rn(wgt, r[6 + c], acc[c]);
        T = tn;
        last = b0 - rg.x + j + 1;
      }
    }
  }
  if (inside) {
    const size_t pix = (size_t)py * W + px, HW = (size_t)W * H;
#pragma unroll
    for (int c = 0; c < C; c++) gbuf[c * HW + pix] = acc[c];
    t_final[pix] = T;
    n_contrib[pix] = last;
  }
}

// ---------------------------------------------------------------- wave reduction

template <int CTRL>
__device__ __forceinline__ float dppv(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 64 lanes; every lane gets the total.
__device__ __forceinline__ float wave_sum(float v) {
  v += dppv<0xB1>(v);   // quad_perm(1,0,3,2)
  v += dppv<0x4E>(v);   // quad_perm(2,3,0,1)
  v += dppv<0x141>(v);  // row_half_mirror
  v += dppv<0x140>(v);  // row_mirror: every lane holds its row (16 lanes) sum
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

template <int C>
__global__ __launch_bounds__(256) void composite_bwd_kernel(
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ sorted_g, const float *__restrict__ records,
    int W, int H, int TX, const float *__restrict__ t_final, const uint32_t *__restrict__ n_contrib,
    const float *__restrict__ dG, const float *__restrict__ dT, float *__restrict__ gacc) {
  constexpr int RS = rec_stride(C);
  constexpr int GS = grad_stride(C);
  constexpr int NV = 6 + C;
  __shared__ float4 batch[256 * RS / 4];
  __shared__ uint32_t gidx[256];
  __shared__ uint32_t maxlast;
  const int tile = blockIdx.x;
  const int tx = tile % TX, ty = tile / TX;
  const int lane = threadIdx.x & 63;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const size_t HW = (size_t)W * H, pix = inside ? (size_t)py * W + px : 0;
  if (threadIdx.x == 0) maxlast = 0;
  __syncthreads();
  float g[C];
  float Tfin = 1.f, dTfin = 0.f;
  uint32_t last = 0;
  if (inside) {
    Tfin = t_final[pix];
    dTfin = dT[pix];
    last = n_contrib[pix];
#pragma unroll
    for (int c = 0; c < C; c++) g[c] = dG[c * HW + pix];
    atomicMax(&maxlast, last);
  } else {
#pragma unroll
    for (int c = 0; c < C; c++) g[c] = 0.f;
  }
  __syncthreads();
  const uint32_t top = maxlast;
  float Tcur = Tfin, S = 0.f;
  for (int hi = (int)top; hi > 0; hi -= 256) {
    const int lo = hi > 256 ? hi - 256 : 0;
    __syncthreads();
    const int e = lo + (int)threadIdx.x;
    if (e < hi) {
      const uint32_t gi = sorted_g[rg.x + e];
      gidx[threadIdx.x] = gi;
      const float *src = records + (size_t)gi * RS;
#pragma unroll
      for (int k = 0; k < RS / 4; k++) batch[threadIdx.x * (RS / 4) + k] = ld4(src + 4 * k);
    }
    __syncthreads();
    for (int j = hi - 1; j >= lo; j--) {
      const float *r = reinterpret_cast<const float *>(&batch[(j - lo) * (RS / 4)]);
      float dx = 0.f, dy = 0.f;
      bool contrib = false;
      float al = 0.f, ex = 0.f, pw = 0.f;
      if ((uint32_t)j < last) {
        pw = splat_power(r[0], r[1], r[2], r[3], r[4], pxc, pyc, dx, dy);
        if (pw <= 0.f) {
          ex = fast_exp(pw);
          const float araw = __fmul_rn(r[5], ex);
          al = fminf(0.99f, araw);
          contrib = al >= (1.f / 255.f);
        }
      }
      if (__ballot(contrib) == 0ull) continue;
      float v[NV];
#pragma unroll
      for (int k = 0; k < NV; k++) v[k] = 0.f;
      if (contrib) {
        const float om = 1.f - al;
        const float Tb = Tcur / om;
        const float wgt = al * Tb;
        float eg = 0.f;
#pragma unroll
        for (int c = 0; c < C; c++) eg = __fmaf_rn(g[c], r[6 + c], eg);
        const float dal = (Tb * eg - S / om) - dTfin * Tfin / om;
        S = __fmaf_rn(wgt, eg, S);
        Tcur = Tb;
#pragma unroll
        for (int c = 0; c < C; c++) v[6 + c] = wgt * g[c];
        if (__fmul_rn(r[5], ex) < 0.99f) {
          const float dpw = dal * al;
          v[5] = dal * ex;
          v[0] = -dpw * (r[2] * dx + r[3] * dy);
          v[1] = -dpw * (r[4] * dy + r[3] * dx);
          v[2] = -0.5f * dpw * dx * dx;
          v[3] = -dpw * dx * dy;
          v[4] = -0.5f * dpw * dy * dy;
        }
      }
      // reduce each value over the wave, then lane k adds value k
      float mine = 0.f;
#pragma unroll
      for (int k = 0; k < NV; k++) {
        const float s = wave_sum(v[k]);
        if (lane == k) mine = s;
      }
      if (lane < NV) atomicAdd(gacc + (size_t)gidx[j - lo] * GS + lane, mine);
    }
  }
}

template <int C>
void launch_composite_fwd_t(const uint2 *ranges, const uint32_t *sorted_g, const float *records, int W, int H,
                            int TX, int TY, float *gbuf, float *t_final, uint32_t *n_contrib, hipStream_t st) {
  composite_fwd_kernel<C><<<TX * TY, 256, 0, st>>>(ranges, sorted_g, records, W, H, TX, gbuf, t_final, n_contrib);
}

template <int C>
void launch_composite_bwd_t(const uint2 *ranges, const uint32_t *sorted_g, const float *records, int W, int H,
                            int TX, int TY, const float *t_final, const uint32_t *n_contrib, const float *dG,
                            const float *dT, float *gacc, hipStream_t st) {
  composite_bwd_kernel<C><<<TX * TY, 256, 0, st>>>(ranges, sorted_g, records, W, H, TX, t_final, n_contrib, dG,
                                                   dT, gacc);
}

#define SSSGS_COMP_INST(C)                                                                                      \
  template void launch_composite_fwd_t<C>(const uint2 *, const uint32_t *, const float *, int, int, int, int,  \
                                          float *, float *, uint32_t *, hipStream_t);                          \
  template void launch_composite_bwd_t<C>(const uint2 *, const uint32_t *, const float *, int, int, int, int,  \
                                          const float *, const uint32_t *, const float *, const float *, float *, \
                                          hipStream_t);
SSSGS_COMP_INST(10)
SSSGS_COMP_INST(18)
SSSGS_COMP_INST(26)
SSSGS_COMP_INST(42)

}  // namespace sssgs
