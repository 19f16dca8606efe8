// composite.hip -- per-tile front-to-back alpha compositing of the deferred
// G-buffer (Sec. 3.1, Eq. 3) and its backward.
//
// One 256-lane workgroup per 16x16 tile, one pixel per lane.  Gaussian
// records of the tile's depth-ordered list are staged through LDS in batches
// of 256; each lane walks the batch, and the workgroup stops loading as soon
// as every pixel has terminated.  The backward walks the same list from each
// pixel's last contributor down, recovering transmittance by division instead
// of storing per-pixel lists; per-Gaussian gradients are reductions over the
// tile's pixels done on the matrix cores (see composite_bwd_kernel).
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

// ---------------------------------------------------------------- backward

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float cf32x4;

// Backward of the compositing, one workgroup per tile.  Each pixel walks its
// list from the last contributor down in batches of kBJ Gaussians, recovering
// transmittance by division, and produces three numbers per (pixel,
// Gaussian): the blend weight w = T alpha, dL/dpower and dL/dopacity.  Every
// per-Gaussian gradient is then a reduction over the tile's pixels of one of
// those numbers times a per-pixel factor:
//   dL/dchannel_c = sum_p w_p dG_p,c                      (w  x  dG)
//   dL/d(u, v, conic) from sum_p dpower_p * (1, x, y, x^2, xy, y^2)_p
//   dL/dopacity   = sum_p dopacity_p
// so the reductions run on the matrix cores (v_mfma_f32_16x16x4_f32, K = the
// tile's pixels) instead of one cross-lane reduction per value.
constexpr int kBJ = 16;  // Gaussians per backward batch

template <int C>
__global__ __launch_bounds__(256, 2) void composite_bwd_kernel(
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ sorted_g, const float *__restrict__ records,
    int W, int H, int TX, const float *__restrict__ t_final, const uint32_t *__restrict__ n_contrib,
    const float *__restrict__ dG, const float *__restrict__ dT, float *__restrict__ gacc) {
  constexpr int RS = rec_stride(C);
  constexpr int GS = grad_stride(C);
  constexpr int CP = (C + 15) / 16 * 16;  // channels padded to 16-column blocks
  constexpr int NBC = CP / 16;
  constexpr int DS = CP + 4;              // LDS row stride of dG
  __shared__ float dgs[256 * DS];         // dL/dG of the tile, [pixel][channel]
  __shared__ float4 recs[kBJ * RS / 4];   // records of the batch
  __shared__ uint32_t gidx[kBJ];
  __shared__ float mat[2 * 256 * kBJ];    // [pixel][j] weights, later dpower | dopacity
  constexpr int RED = 4 * kBJ * CP > 4 * 2 * kBJ * 16 ? 4 * kBJ * CP : 4 * 2 * kBJ * 16;
  __shared__ float red[RED];              // per-wave partial sums of the two reductions
  __shared__ uint32_t maxlast;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, col = lane & 15;
  const int tile = blockIdx.x;
  const int tx = tile % TX, ty = tile / TX;
  const int px = tx * kTile + (t & 15), py = ty * kTile + (t >> 4);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const size_t HW = (size_t)W * H, pix = inside ? (size_t)py * W + px : 0;
  if (t == 0) maxlast = 0;
  __syncthreads();
  float gch[C];
  float Tfin = 1.f, dTfin = 0.f;
  uint32_t last = 0;
  if (inside) {
    Tfin = t_final[pix];
    dTfin = dT[pix];
    last = n_contrib[pix];
#pragma unroll
    for (int c = 0; c < C; c++) gch[c] = dG[c * HW + pix];
    atomicMax(&maxlast, last);
  } else {
#pragma unroll
    for (int c = 0; c < C; c++) gch[c] = 0.f;
  }
#pragma unroll
  for (int c = 0; c < CP; c++) dgs[t * DS + c] = c < C ? gch[c] : 0.f;
  __syncthreads();
  const int top = (int)maxlast;
  float Tcur = Tfin, S = 0.f;
  for (int hi = top; hi > 0; hi -= kBJ) {
    const int lo = hi > kBJ ? hi - kBJ : 0, cnt = hi - lo;
    for (int k = t; k < kBJ * RS / 4; k += 256) {
      const int jj = k / (RS / 4), q4 = k % (RS / 4);
      if (jj < cnt) {
        const uint32_t gi = sorted_g[rg.x + lo + jj];
        if (q4 == 0) gidx[jj] = gi;
        recs[k] = ld4(records + (size_t)gi * RS + 4 * q4);
      }
    }
    __syncthreads();
    // ---- per pixel, last to first
    float wv[kBJ], pv[kBJ], qv[kBJ];
#pragma unroll
    for (int jj = kBJ - 1; jj >= 0; jj--) {
      wv[jj] = 0.f;
      pv[jj] = 0.f;
      qv[jj] = 0.f;
      if (jj < cnt && (uint32_t)(lo + jj) < last) {
        const float *r = reinterpret_cast<const float *>(&recs[jj * (RS / 4)]);
        float dx, dy;
        const float pw = splat_power(r[0], r[1], r[2], r[3], r[4], pxc, pyc, dx, dy);
        if (pw <= 0.f) {
          const float ex = fast_exp(pw);
          const float araw = __fmul_rn(r[5], ex);
          const float al = fminf(0.99f, araw);
          if (al >= (1.f / 255.f)) {
            const float om = 1.f - al;
            const float Tb = Tcur / om;
            const float wgt = al * Tb;
            float eg = 0.f;
#pragma unroll
            for (int c = 0; c < C; c++) eg = __fmaf_rn(gch[c], r[6 + c], eg);
            const float dal = (Tb * eg - S / om) - dTfin * Tfin / om;
            S = __fmaf_rn(wgt, eg, S);
            Tcur = Tb;
            wv[jj] = wgt;
            if (araw < 0.99f) {
              pv[jj] = dal * al;
              qv[jj] = dal * ex;
            }
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // keep record loads of later Gaussians from piling up in registers
    }
    // ---- channel gradients: D1[j][c] = sum_p w[p][j] dG[p][c]
#pragma unroll
    for (int k = 0; k < kBJ; k += 4) *reinterpret_cast<float4 *>(&mat[t * kBJ + k]) = make_float4(wv[k], wv[k + 1], wv[k + 2], wv[k + 3]);
    __syncthreads();
    {
      cf32x4 acc[NBC];
#pragma unroll
      for (int nc = 0; nc < NBC; nc++) acc[nc] = cf32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 16; ks++) {  // this wave's 64 pixels, 4 per step
        const int p = 64 * w + 4 * ks + g;
        const float a = mat[p * kBJ + col];
#pragma unroll
        for (int nc = 0; nc < NBC; nc++)
          acc[nc] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, dgs[p * DS + 16 * nc + col], acc[nc], 0, 0, 0);
      }
      // D layout: lane (col, g) holds rows j = 4 g + i, column c = 16 nc + col
#pragma unroll
      for (int nc = 0; nc < NBC; nc++)
#pragma unroll
        for (int i = 0; i < 4; i++) red[(w * kBJ + 4 * g + i) * CP + 16 * nc + col] = acc[nc][i];
    }
    __syncthreads();
    for (int k = t; k < kBJ * C; k += 256) {
      const int jj = k / C, c = k % C;
      if (jj < cnt) {
        const float s = (red[(0 * kBJ + jj) * CP + c] + red[(1 * kBJ + jj) * CP + c]) +
                        (red[(2 * kBJ + jj) * CP + c] + red[(3 * kBJ + jj) * CP + c]);
        if (s != 0.f) atomicAdd(gacc + (size_t)gidx[jj] * GS + 6 + c, s);
      }
    }
    // ---- geometric moments: rows 0..15 dpower, rows 16..31 dopacity, against
    // the pixel basis (1, x, y, x^2, xy, y^2) relative to the tile corner
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBJ; k += 4) {
      *reinterpret_cast<float4 *>(&mat[t * kBJ + k]) = make_float4(pv[k], pv[k + 1], pv[k + 2], pv[k + 3]);
      *reinterpret_cast<float4 *>(&mat[256 * kBJ + t * kBJ + k]) = make_float4(qv[k], qv[k + 1], qv[k + 2], qv[k + 3]);
    }
    __syncthreads();
    {
      cf32x4 acc[2] = {cf32x4{0.f, 0.f, 0.f, 0.f}, cf32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
      for (int ks = 0; ks < 16; ks++) {
        const int p = 64 * w + 4 * ks + g;
        const float x = (float)(p & 15) + 0.5f, y = (float)(p >> 4) + 0.5f;
        float b = 0.f;
        switch (col) {
          case 0: b = 1.f; break;
          case 1: b = x; break;
          case 2: b = y; break;
          case 3: b = x * x; break;
          case 4: b = x * y; break;
          case 5: b = y * y; break;
          default: b = 0.f;
        }
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(mat[p * kBJ + col], b, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(mat[256 * kBJ + p * kBJ + col], b, acc[1], 0, 0, 0);
      }
#pragma unroll
      for (int m = 0; m < 2; m++)
#pragma unroll
        for (int i = 0; i < 4; i++) red[(w * 2 * kBJ + 16 * m + 4 * g + i) * 16 + col] = acc[m][i];
    }
    __syncthreads();
    if (t < cnt) {
      float mo[6], sq = 0.f;
#pragma unroll
      for (int n = 0; n < 6; n++)
        mo[n] = (red[(0 * 2 * kBJ + t) * 16 + n] + red[(1 * 2 * kBJ + t) * 16 + n]) +
                (red[(2 * 2 * kBJ + t) * 16 + n] + red[(3 * 2 * kBJ + t) * 16 + n]);
      sq = (red[(0 * 2 * kBJ + 16 + t) * 16] + red[(1 * 2 * kBJ + 16 + t) * 16]) +
           (red[(2 * 2 * kBJ + 16 + t) * 16] + red[(3 * 2 * kBJ + 16 + t) * 16]);
      const float *r = reinterpret_cast<const float *>(&recs[t * (RS / 4)]);
      const float up = r[0] - (float)(tx * kTile), vp = r[1] - (float)(ty * kTile);
      // sums of dpower * dx, dy, dx^2, dx dy, dy^2 with dx = u - x, dy = v - y
      const float sx = up * mo[0] - mo[1], sy = vp * mo[0] - mo[2];
      const float sxx = up * up * mo[0] - 2.f * up * mo[1] + mo[3];
      const float sxy = up * vp * mo[0] - up * mo[2] - vp * mo[1] + mo[4];
      const float syy = vp * vp * mo[0] - 2.f * vp * mo[2] + mo[5];
      float *ga = gacc + (size_t)gidx[t] * GS;
      if (mo[0] != 0.f || sq != 0.f) {
        atomicAdd(ga + 0, -(r[2] * sx + r[3] * sy));
        atomicAdd(ga + 1, -(r[4] * sy + r[3] * sx));
        atomicAdd(ga + 2, -0.5f * sxx);
        atomicAdd(ga + 3, -sxy);
        atomicAdd(ga + 4, -0.5f * syy);
        atomicAdd(ga + 5, sq);
      }
    }
    __syncthreads();
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
