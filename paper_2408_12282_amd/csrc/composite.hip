// composite.hip -- per-tile front-to-back alpha compositing of the deferred
// G-buffer (Sec. 3.1, Eq. 3) and its backward.
//
// One 256-lane workgroup per 16x16 tile, one pixel per lane; wave w owns the
// 16x4 strip of rows 4w..4w+3.  Records of the tile's depth-ordered list are
// staged through LDS by the whole workgroup.  Each wave first tests the
// staged Gaussians' alpha boxes (see alpha_box in project.hip) against its
// strip with one ballot per 64 Gaussians and then walks only the Gaussians
// that can reach it; the boxes are conservative, so skipping the others
// changes no result.  The backward walks the same list from each pixel's last
// contributor down, recovering transmittance by division instead of storing
// per-pixel lists; per-Gaussian gradients are reductions over the tile's
// pixels done on the matrix cores (see composite_bwd_kernel).
#include "common.hpp"

namespace sssgs {

// Does the alpha box (int16 x_lo, x_hi | y_lo, y_hi packed in two dwords)
// reach the 16x4 strip with top-left pixel (sx, sy)?
__device__ __forceinline__ bool box_hits(uint2 bx, int sx, int sy) {
  const int xlo = (int)(short)(bx.x & 0xffffu), xhi = (int)bx.x >> 16;
  const int ylo = (int)(short)(bx.y & 0xffffu), yhi = (int)bx.y >> 16;
  return !(xlo > sx + kTile - 1 || xhi < sx || ylo > sy + 3 || yhi < sy);
}

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float cf32x4;

// Forward: each wave walks the hits of its strip in depth order and keeps,
// per pixel, only the transmittance recursion (alpha, T, the stopping test);
// the blend weights w = alpha T of up to kFG hits wait as rows [hit][pixel]
// in LDS, and the channel sums G[c][p] += sum_k channel_k,c w_k,p are one
// FP32 product per four hits on the matrix cores (v_mfma_f32_16x16x4_f32,
// channels x pixels, K = hits), accumulated in registers for the tile.
constexpr int kFG = 4;        // hits per flush of the weight rows (one k-step; the small LDS
                              // and register footprint lets seven workgroups share a CU)
constexpr int kFWS = 64 + 16;  // row stride of the weight rows (conflict-free column reads)

template <int C>
__global__ __launch_bounds__(256, C > 32 ? 4 : 6) void composite_fwd_kernel(const uint2 *__restrict__ ranges,
                                                                          const uint32_t *__restrict__ sorted_g,
                                                                          const float *__restrict__ records,
                                                                          const short4 *__restrict__ boxes, int W,
                                                                          int H, int TX, float *__restrict__ gbuf,
                                                                          float *__restrict__ t_final,
                                                                          uint32_t *__restrict__ n_contrib,
                                                                          uint32_t *__restrict__ tile_top) {
  constexpr int RS = rec_stride(C);
  constexpr int NB = 128;             // records per batch
  constexpr int CB = (C + 15) / 16;   // 16-channel row blocks of the sums
  static_assert(NB <= 256 && kFG % 4 == 0 && kFG <= 8, "record index in 8 bits, one or two k-steps per flush");
  __shared__ float4 batch[NB * RS / 4];
  __shared__ uint2 bbox[NB];
  __shared__ float wrow[4][kFG * kFWS];
  __shared__ uint32_t tmax;
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int tile = blockIdx.x;
  const int tx = tile % TX, ty = tile / TX;
  const int sx = tx * kTile, sy = ty * kTile + 4 * w;  // the wave's strip
  const int px = sx + (lane & 15), py = sy + (lane >> 4);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const uint2 *bxs = reinterpret_cast<const uint2 *>(boxes);
  const float *bf = reinterpret_cast<const float *>(batch);
  float *wr = wrow[w];
  float T = 1.f;
  // D layout of the sums: acc[cb][nb] lane l holds channel 16 cb + 4 (l / 16) + i
  // (i = 0..3) of pixel (l % 16, row nb) of the strip
  cf32x4 acc[CB][4];
#pragma unroll
  for (int cb = 0; cb < CB; cb++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) acc[cb][nb] = cf32x4{0.f, 0.f, 0.f, 0.f};
  uint32_t last = 0;
  bool done = !inside;
  int nk = 0;          // hits waiting in the weight rows (wave-uniform)
  uint64_t krec = 0;   // their records in the batch, 8 bits each
  auto flush = [&]() {
    // the last k-step's unused rows are zero (their channels are any staged record's)
    for (int s = nk; s < ((nk + 3) & ~3); s++) wr[s * kFWS + lane] = 0.f;
    for (int ks = 0; 4 * ks < nk; ks++) {
      const int s = 4 * ks + (lane >> 4);
      const int js = (int)((krec >> (8 * s)) & 0xffu);
      float a[CB];
#pragma unroll
      for (int cb = 0; cb < CB; cb++) {
        const int c = 16 * cb + (lane & 15);
        a[cb] = c < C ? bf[js * RS + 6 + (c < C ? c : 0)] : 0.f;
      }
      float b[4];
#pragma unroll
      for (int nb = 0; nb < 4; nb++) b[nb] = wr[s * kFWS + 16 * nb + (lane & 15)];
#pragma unroll
      for (int cb = 0; cb < CB; cb++)
#pragma unroll
        for (int nb = 0; nb < 4; nb++) acc[cb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[cb], b[nb], acc[cb][nb], 0, 0, 0);
    }
    nk = 0;
    krec = 0;
  };
  if (t == 0) tmax = 0;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += NB) {
    if (__syncthreads_count(done) == 256) break;
    const uint32_t e = b0 + t;
    if (t < NB && e < rg.y) {
      const uint32_t gi = sorted_g[e];
      const float *src = records + (size_t)gi * RS;
#pragma unroll
      for (int k = 0; k < RS / 4; k++) batch[t * (RS / 4) + k] = ld4(src + 4 * k);
      bbox[t] = bxs[gi];
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NB, rg.y - b0);
    for (int j0 = 0; j0 < cnt; j0 += 64) {
      bool h = false;
      if (j0 + lane < cnt) h = box_hits(bbox[j0 + lane], sx, sy);
      uint64_t m = __ballot(h);
      // groups of up to kFG hits in depth order: the alphas of a group are
      // independent of each other, only the transmittance recursion is serial
      while (m != 0 && __ballot(!done) != 0) {
        int js[kFG];
        int nv = 0;
#pragma unroll
        for (int s = 0; s < kFG; s++) {
          js[s] = m != 0 ? j0 + (int)__builtin_ctzll(m) : -1;
          nv += m != 0 ? 1 : 0;
          m &= m - 1;
        }
        krec = 0;
#pragma unroll
        for (int s = 0; s < kFG; s++) {
          const int j = js[s] >= 0 ? js[s] : js[0];
          krec |= (uint64_t)j << (8 * s);
          const float4 ha = batch[j * (RS / 4)], hb = batch[j * (RS / 4) + 1];  // u v a b | c opacity ..
          float dx, dy;
          const float pw = splat_power(ha.x, ha.y, ha.z, ha.w, hb.x, pxc, pyc, dx, dy);
          const float al = fminf(0.99f, __fmul_rn(hb.y, fast_exp(fminf(pw, 0.f))));
          const bool ok = js[s] >= 0 && !done && pw <= 0.f && al >= (1.f / 255.f);
          const float tn = T * (1.f - al);
          const bool keep = ok && !(tn < 1e-4f);
          done = done || (ok && tn < 1e-4f);
          wr[s * kFWS + lane] = keep ? al * T : 0.f;
          T = keep ? tn : T;
          last = keep ? b0 - rg.x + j + 1 : last;
        }
        nk = nv;
        flush();
      }
    }
  }
  if (inside) {
    const size_t pix = (size_t)py * W + px;
    t_final[pix] = T;
    n_contrib[pix] = last;
  }
  {
    const size_t HW = (size_t)W * H;
    const int qx = sx + (lane & 15);
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      const int qy = sy + nb;
      if (qx < W && qy < H) {
        const size_t pix = (size_t)qy * W + qx;
#pragma unroll
        for (int cb = 0; cb < CB; cb++)
#pragma unroll
          for (int i = 0; i < 4; i++) {
            const int c = 16 * cb + 4 * (lane >> 4) + i;
            if (c < C) gbuf[c * HW + pix] = acc[cb][nb][i];
          }
      }
    }
  }
  // the tile's largest last-contributor index: the backward's work per tile
  __syncthreads();
  atomicMax(&tmax, last);
  __syncthreads();
  if (t == 0) tile_top[blockIdx.x] = tmax;
}

// ---------------------------------------------------------------- backward

// Backward of the compositing, one workgroup per tile.  Each pixel walks its
// list from the last contributor down in batches of kBJ Gaussians, recovering
// transmittance with v_rcp_f32, and produces two numbers per (pixel, Gaussian):
// the blend weight w = T alpha and g = dL/dpower.  Every per-Gaussian gradient
// is a reduction over the tile's pixels of one of them times a per-pixel
// factor:
//   dL/dchannel_c = sum_p w_p dG_p,c
//   dL/d(u, v, conic) from the moments sum_p g_p (1, x, y, x^2, xy, y^2)_p
//   dL/dopacity   = sum_p g_p / opacity   (alpha = o e^power: dalpha/do = alpha/o)
// so the reductions run on the matrix cores with K = the wave's 64 pixels
// rather than as one cross-lane reduction per value.  The channel sums use
// BF16 operands in three terms, a_hi b_hi + a_hi b_lo + a_lo b_hi with
// x_hi = x truncated to BF16 and x_lo = x - x_hi rounded to BF16 (relative
// error about 2^-16 per product, accumulated in FP32), on
// v_mfma_f32_16x16x32_bf16: a sixth of the matrix-core time of FP32 operands.
// The moment sums must stay FP32-accurate: the geometry gradients recombine
// them as u^2 sum g - 2 u sum g x + sum g x^2, which cancels and would
// magnify a 2^-16 error.  With x, y measured from the tile centre every basis
// value has at most 8 significant bits, so g split exactly into three BF16
// parts gives exact products on v_mfma_f32_16x16x32_bf16, where only the
// FP32 accumulation rounds (as with FP32 operands, at a third of the time).
// The batch is staged in LDS (double-buffered; the next batch is fetched
// into registers while the current one is walked): the record headers, and
// the channels already split into BF16 high and low parts in the lane order
// of the products' A operand, so that each wave reads its operand with two
// 16-byte loads per lane at consecutive addresses.  Each wave skips the
// Gaussians whose alpha box misses its strip.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 cbf16x8;

// Two floats as BF16 high parts (truncation) and low parts (RNE of the
// remainder), each pair packed in one dword with the first float low.
__device__ __forceinline__ void split_bf16x2(float x, float y, uint32_t &h, uint32_t &l) {
  const uint32_t a = __float_as_uint(x), b = __float_as_uint(y);
  h = __builtin_amdgcn_perm(b, a, 0x07060302u);  // upper halves: a in the low, b in the high half
  const float ra = x - __uint_as_float(a & 0xffff0000u);
  const float rb = y - __uint_as_float(b & 0xffff0000u);
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  l = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){ra, rb}, b2));
}

// Eight floats as BF16 high and low parts.
__device__ __forceinline__ void split_bf16x8(const float (&v)[8], cbf16x8 &hi, cbf16x8 &lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int k = 0; k < 4; k++) split_bf16x2(v[2 * k], v[2 * k + 1], h[k], l[k]);
  hi = __builtin_bit_cast(cbf16x8, make_uint4(h[0], h[1], h[2], h[3]));
  lo = __builtin_bit_cast(cbf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

// Eight floats as three BF16 parts each, x = p1 + p2 + p3 exactly: p1 and p2
// are the top 8 significant bits of x and of the remainder (truncation), p3
// the last 8 (exact).
__device__ __forceinline__ void split3_bf16x8(const float (&v)[8], cbf16x8 &p1, cbf16x8 &p2, cbf16x8 &p3) {
  uint32_t a[4], b[4], c[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const float x = v[2 * k], y = v[2 * k + 1];
    a[k] = __builtin_amdgcn_perm(__float_as_uint(y), __float_as_uint(x), 0x07060302u);
    const float rx = x - __uint_as_float(__float_as_uint(x) & 0xffff0000u);
    const float ry = y - __uint_as_float(__float_as_uint(y) & 0xffff0000u);
    b[k] = __builtin_amdgcn_perm(__float_as_uint(ry), __float_as_uint(rx), 0x07060302u);
    const float sx = rx - __uint_as_float(__float_as_uint(rx) & 0xffff0000u);
    const float sy = ry - __uint_as_float(__float_as_uint(ry) & 0xffff0000u);
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    c[k] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){sx, sy}, b2));
  }
  p1 = __builtin_bit_cast(cbf16x8, make_uint4(a[0], a[1], a[2], a[3]));
  p2 = __builtin_bit_cast(cbf16x8, make_uint4(b[0], b[1], b[2], b[3]));
  p3 = __builtin_bit_cast(cbf16x8, make_uint4(c[0], c[1], c[2], c[3]));
}

__device__ __forceinline__ cf32x4 mma3(const cbf16x8 &ah, const cbf16x8 &al, const cbf16x8 &bh, const cbf16x8 &bl,
                                       cf32x4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
}

constexpr int kBJ = 16;       // Gaussians per backward batch
constexpr int kMS = 256 + 4;  // row stride of the [Gaussian][pixel] matrices (conflict-free column reads)

template <int C>
__global__ __launch_bounds__(256, C > 26 ? 2 : 3) void composite_bwd_kernel(
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ sorted_g, const float *__restrict__ records,
    const short4 *__restrict__ boxes, int W, int H, int TX, const float *__restrict__ t_final,
    const uint32_t *__restrict__ n_contrib, const float *__restrict__ dG, const float *__restrict__ dT,
    float *__restrict__ gacc, DetSlots det, const uint32_t *__restrict__ order) {
  constexpr int RS = rec_stride(C);
  constexpr int GS = grad_stride(C);
  constexpr int CP = (C + 15) / 16 * 16;  // channels padded to 16-column blocks
  constexpr int NBC = CP / 16;
  constexpr int RW = CP + 16;             // columns of the per-wave partial sums: channels | moments
  constexpr int KC = (C + 31) / 32;       // 32-channel k-steps of the per-pair dot products
  static_assert(RW <= 64, "per-wave partial sums must fit the wave's 64 columns");
  static_assert(kBJ == 16 && KC <= 2 && C % 2 == 0, "batch fetch roles below");
  // [j][pixel]: weights (rows 0..kBJ-1) and dL/dpower (rows kBJ..2kBJ-1).  A
  // wave only touches its own 64 pixel columns, so once its reductions are
  // done it stores its partial sums [j][channels | moments] over its own
  // columns of the weight rows.
  __shared__ float mat[2 * kBJ * kMS];
  __shared__ float4 hdr[2][2 * kBJ];         // u v a b | c opacity . . of each Gaussian
  __shared__ cbf16x8 aop[2][KC][2][64];      // channel A operands: [k-step][high, low][lane]
  __shared__ uint32_t gidx[2][kBJ];
  __shared__ uint32_t gq[2][kBJ];            // Gaussian indices of the batch fetched next
  __shared__ uint2 bbox[2][kBJ];
  __shared__ uint32_t maxlast;
  const int t = threadIdx.x, lane = t & 63, g = lane >> 4, col = lane & 15;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int tile = (int)order[blockIdx.x];  // heaviest tiles first
  const int tx = tile % TX, ty = tile / TX;
  const int sx = tx * kTile, sy = ty * kTile + 4 * w;  // the wave's 16x4 strip
  const int px = sx + (lane & 15), py = sy + (lane >> 4);
  const bool inside = px < W && py < H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const size_t HW = (size_t)W * H, pix = inside ? (size_t)py * W + px : 0;
  const uint2 *bxs = reinterpret_cast<const uint2 *>(boxes);
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
  // The tile's dL/dG is the B operand of every channel reduction below: lane
  // (col, g) of wave w needs dG[pixel 64 w + 32 kk + 8 g + i][channel 16 nc + col],
  // i = 0..7.  It is transposed once through LDS (the weight matrix is not in
  // use yet), split into BF16 high and low parts and kept in registers for
  // the whole tile, as are the moment basis values (1, x, y, x^2, xy, y^2)
  // of the same pixels, from the tile corner.
  // The same dL/dG is also the B operand of the per-batch products
  // eg[j][p] = sum_c channel_j,c dG[p][c] (K = channels): lane (col, g)
  // holds channels 32 ks + 8 g + i of pixel 16 nb + col of the wave's strip.
  cbf16x8 bh[2][NBC], bl[2][NBC], eh[KC][4], el[KC][4];
  float ev[KC][4][8];
#pragma unroll
  for (int nc = 0; nc < NBC; nc++) {
#pragma unroll
    for (int c = 0; c < 16; c++) mat[t * 17 + c] = 16 * nc + c < C ? gch[16 * nc + c] : 0.f;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 2; kk++) {
      float v[8];
#pragma unroll
      for (int i = 0; i < 8; i++) v[i] = mat[(64 * w + 32 * kk + 8 * g + i) * 17 + col];
      split_bf16x8(v, bh[kk][nc], bl[kk][nc]);
    }
    // channel block nc holds k-step nc / 2 for the lanes with g / 2 == nc % 2
    if ((g >> 1) == (nc & 1)) {
#pragma unroll
      for (int nb = 0; nb < 4; nb++)
#pragma unroll
        for (int i = 0; i < 8; i++) ev[nc >> 1][nb][i] = mat[(64 * w + 16 * nb + col) * 17 + 8 * (g & 1) + i];
    }
    __syncthreads();
  }
#pragma unroll
  for (int ks = 0; ks < KC; ks++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      // channels of a k-step beyond the last 16-column block were never loaded
      if (2 * ks + (g >> 1) >= NBC)
        for (int i = 0; i < 8; i++) ev[ks][nb][i] = 0.f;
      split_bf16x8(ev[ks][nb], eh[ks][nb], el[ks][nb]);
    }
  // moment basis of pixel 16 g + 8 kk + i of the wave (B operand of k-step
  // kk, element i; a lane's 16 pixels are a row of the strip): offsets from
  // the tile centre x = 8 kk + i - 15/2 and y = 4 w + g - 15/2, so column col
  // of the basis (1, x, y, x^2, xy, y^2) is mb0 + mb1 x + mb2 x^2 with
  // per-lane constants.  Every value is a multiple of 1/4 below 57 in
  // magnitude with at most 8 significant bits: exact in BF16.
  const float yb = (float)(4 * w + g) - 7.5f;
  const float mb0 = col == 0 ? 1.f : col == 2 ? yb : col == 5 ? yb * yb : 0.f;
  const float mb1 = col == 1 ? 1.f : col == 4 ? yb : 0.f;
  const float mb2 = col == 3 ? 1.f : 0.f;
  const int top = (int)maxlast;
  uint32_t wlast = last;  // the wave's largest last contributor
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, o, 64));
  wlast = __builtin_amdgcn_readfirstlane(wlast);
  // Batch fetch into registers, one role per thread.  Threads 0..127 hold
  // half h = t / 64 of the A operand of lane l = t % 64 in every k-step ks:
  // channels 32 ks + 8 g + 4 h + i (i = 0..3) of Gaussian col, read straight
  // from its record; threads 128..159 one 16-byte header chunk each;
  // threads 160..175 the Gaussian's index and alpha box.
  const int fl = t & 63, fh = (t >> 6) & 1;
  const bool rA = t < 128, rH = t >= 128 && t < 160, rI = t >= 160 && t < 176;
  const int f_j = rA ? (fl & 15) : rH ? (t - 128) >> 1 : t - 160;  // Gaussian of the batch
  const int f_off = rA ? 6 + 8 * (fl >> 4) + 4 * fh : 4 * (t & 1);  // first float in its record
  float f_v[4 * KC];
#pragma unroll
  for (int i = 0; i < 4 * KC; i++) f_v[i] = 0.f;
  uint32_t f_g = 0;
  uint2 f_box = make_uint2(0u, 0u);
  // A fetch takes its Gaussian's index from LDS, where the index threads put
  // it one batch earlier: no record load waits on an index load (a wait on a
  // load would also take in this wave's gradient atomics of the batch before).
  uint32_t f_gi2 = 0;  // index threads: their Gaussian's index two batches ahead
  auto load_index2 = [&](int lo_, int cnt_) {
    if (rI && f_j < cnt_) f_gi2 = sorted_g[rg.x + lo_ + f_j];
  };
  auto stage_index = [&](int slot, int cnt_) {
    if (rI && f_j < cnt_) gq[slot][f_j] = f_gi2;
  };
  auto fetch = [&](int cnt_, uint32_t gg) {
    if ((rA || rH || rI) && f_j < cnt_) {
      const float *src = records + (size_t)gg * RS + f_off;
      if (rA) {
        // two 8-byte-aligned float2 per k-step; a pair is loaded whenever its
        // first channel is below C (C even), so every channel used is loaded
#pragma unroll
        for (int ks = 0; ks < KC; ks++) {
          const int c0 = f_off - 6 + 32 * ks;
          if (c0 < C) {
            const float2 v = *reinterpret_cast<const float2 *>(src + 32 * ks);
            f_v[4 * ks] = v.x;
            f_v[4 * ks + 1] = v.y;
          }
          if (c0 + 2 < C) {
            const float2 v = *reinterpret_cast<const float2 *>(src + 32 * ks + 2);
            f_v[4 * ks + 2] = v.x;
            f_v[4 * ks + 3] = v.y;
          }
        }
      } else if (rH) {
        const float4 v = ld4(src);
        f_v[0] = v.x;
        f_v[1] = v.y;
        f_v[2] = v.z;
        f_v[3] = v.w;
      } else {
        f_g = gg;
        f_box = bxs[gg];
      }
    }
  };
  auto stage = [&](int buf, int cnt_) {
    const bool ok = f_j < cnt_;
    if (rA) {
      // channels past C and Gaussians past the batch are zero
#pragma unroll
      for (int ks = 0; ks < KC; ks++) {
        const int c0 = f_off - 6 + 32 * ks;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; i++) v[i] = ok && c0 + i < C ? f_v[4 * ks + i] : 0.f;
        uint2 hi, lo;
        split_bf16x2(v[0], v[1], hi.x, lo.x);
        split_bf16x2(v[2], v[3], hi.y, lo.y);
        reinterpret_cast<uint2 *>(&aop[buf][ks][0][fl])[fh] = hi;
        reinterpret_cast<uint2 *>(&aop[buf][ks][1][fl])[fh] = lo;
      }
    } else if (rH) {
      if (ok) hdr[buf][t - 128] = make_float4(f_v[0], f_v[1], f_v[2], f_v[3]);
    } else if (rI) {
      if (ok) {
        gidx[buf][f_j] = f_g;
        bbox[buf][f_j] = f_box;
      }
    }
  };
  if (top > 0) {
    const int lo0 = top > kBJ ? top - kBJ : 0, lo1 = lo0 > kBJ ? lo0 - kBJ : 0;
    const uint32_t g0 = ((rA || rH || rI) && f_j < top - lo0) ? sorted_g[rg.x + lo0 + f_j] : 0u;
    fetch(top - lo0, g0);
    stage(0, top - lo0);
    if (lo0 > 0) {
      load_index2(lo1, lo0 - lo1);
      stage_index(1, lo0 - lo1);
    }
  }
  __syncthreads();
  // U: dL/dT_final T_final plus the sum of w eg over the Gaussians behind the
  // current one (the part of dL/dalpha that the Gaussians behind contribute)
  float Tcur = Tfin, U = dTfin * Tfin;
  int buf = 0;
  for (int hi = top; hi > 0; hi -= kBJ, buf ^= 1) {
    const int lo = hi > kBJ ? hi - kBJ : 0, cnt = hi - lo;
    const int nlo = lo > kBJ ? lo - kBJ : 0, ncnt = lo - nlo;
    const int nnlo = nlo > kBJ ? nlo - kBJ : 0, nncnt = nlo - nnlo;
    // next batch, in flight during this one, and the indices of the one after
    if (ncnt > 0) fetch(ncnt, ((rA || rH || rI) && f_j < ncnt) ? gq[buf ^ 1][f_j] : 0u);
    if (nncnt > 0) load_index2(nnlo, nncnt);
    // Gaussians of the batch that can reach this wave's strip
    bool h = false;
    if (lane < cnt) h = box_hits(bbox[buf][lane], sx, sy);
    const uint32_t hm = (uint32_t)__ballot(h);
    // ---- eg[j][p] = channels_j . dG_p for the batch on the matrix cores
    // (three-term BF16 split), into this wave's columns of rows kBJ.. (each
    // lane reads its own eg[j] there before the walk overwrites it with g)
    {
      cbf16x8 ah[KC], al[KC];
#pragma unroll
      for (int ks = 0; ks < KC; ks++) {
        ah[ks] = aop[buf][ks][0][lane];
        al[ks] = aop[buf][ks][1][lane];
      }
#pragma unroll
      for (int nb = 0; nb < 4; nb++) {
        cf32x4 d = cf32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KC; ks++) d = mma3(ah[ks], al[ks], eh[ks][nb], el[ks][nb], d);
#pragma unroll
        for (int i = 0; i < 4; i++) mat[(kBJ + 4 * g + i) * kMS + 64 * w + 16 * nb + col] = d[i];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    // ---- per pixel, last to first over the Gaussians whose box reaches this
    // strip and whose index is below some pixel's last contributor; each
    // result goes straight to LDS and the rows of the others are zero.  The
    // next Gaussian's header and eg are read while the current one is
    // evaluated, and a lane's tests are selects rather than branches, so that
    // the walk is not a chain of LDS round trips.
    uint32_t m = hm;
    if ((uint32_t)hi > wlast) m &= wlast > (uint32_t)lo ? (1u << (wlast - (uint32_t)lo)) - 1u : 0u;
#pragma unroll
    for (int jj = 0; jj < kBJ; jj++)
      if (!((m >> jj) & 1u)) {
        mat[jj * kMS + t] = 0.f;
        mat[(kBJ + jj) * kMS + t] = 0.f;
      }
    if (m != 0u) {
      const int n = __builtin_popcount(m);
      int jj = 31 - __builtin_clz(m);
      float4 ha = hdr[buf][2 * jj];
      float2 hb = *reinterpret_cast<const float2 *>(&hdr[buf][2 * jj + 1]);  // c, opacity
      float eg = mat[(kBJ + jj) * kMS + t];
      for (int k = 0; k < n; k++) {
        m &= ~(1u << jj);
        const int jn = m != 0u ? 31 - __builtin_clz(m) : jj;
        const float4 na = hdr[buf][2 * jn];
        const float2 nb = *reinterpret_cast<const float2 *>(&hdr[buf][2 * jn + 1]);
        const float neg = mat[(kBJ + jn) * kMS + t];
        float dx, dy;
        const float pw = splat_power(ha.x, ha.y, ha.z, ha.w, hb.x, pxc, pyc, dx, dy);
        const float araw = __fmul_rn(hb.y, fast_exp(fminf(pw, 0.f)));
        const float al = fminf(0.99f, araw);
        const bool on = (uint32_t)(lo + jj) < last && pw <= 0.f && al >= (1.f / 255.f);
        const float inv = __builtin_amdgcn_rcpf(1.f - al);
        const float Tb = Tcur * inv;
        const float wgt = al * Tb;
        const float dal = Tb * eg - U * inv;
        const float Un = __fmaf_rn(wgt, eg, U);
        U = on ? Un : U;
        Tcur = on ? Tb : Tcur;
        mat[jj * kMS + t] = on ? wgt : 0.f;
        mat[(kBJ + jj) * kMS + t] = on && araw < 0.99f ? dal * al : 0.f;
        jj = jn;
        ha = na;
        hb = nb;
        eg = neg;
      }
    }
    // the reductions read only this wave's own columns: a wave-level fence
    // suffices, and a wave whose strip had few hits goes on to the matrix
    // cores while the others still walk
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // ---- reductions over this wave's 64 pixels (two steps of 32):
    //   [j][c]  = sum_p w[j][p] dG[p][c]
    //   [j][n]  = sum_p g[j][p] basis_n(p),  basis = (1, x, y, x^2, xy, y^2) from the tile centre
    {
      cf32x4 acc[NBC + 1];
#pragma unroll
      for (int nc = 0; nc <= NBC; nc++) acc[nc] = cf32x4{0.f, 0.f, 0.f, 0.f};
      float gv[16];
      {
        const float4 *gr = reinterpret_cast<const float4 *>(&mat[(kBJ + col) * kMS + 64 * w + 16 * g]);
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const float4 v = gr[q];
          gv[4 * q] = v.x;
          gv[4 * q + 1] = v.y;
          gv[4 * q + 2] = v.z;
          gv[4 * q + 3] = v.w;
        }
      }
#pragma unroll
      for (int kk = 0; kk < 2; kk++) {
        const float4 *wr = reinterpret_cast<const float4 *>(&mat[col * kMS + 64 * w + 32 * kk + 8 * g]);
        const float4 w0 = wr[0], w1 = wr[1];
        const float wv[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
        cbf16x8 wh, wl;
        split_bf16x8(wv, wh, wl);
#pragma unroll
        for (int nc = 0; nc < NBC; nc++) acc[nc] = mma3(wh, wl, bh[kk][nc], bl[kk][nc], acc[nc]);
      }
      // moments: g split exactly into three BF16 parts against the exact BF16
      // basis, so every product is exact and only the FP32 accumulation
      // rounds, as with FP32 operands, on v_mfma_f32_16x16x32_bf16 (a
      // third of the matrix-core time); the parts in separate accumulators
      cf32x4 am2 = cf32x4{0.f, 0.f, 0.f, 0.f}, am3 = cf32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 2; kk++) {
        float gk[8], bk[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
          gk[i] = gv[8 * kk + i];
          const float x = (float)(8 * kk + i) - 7.5f;
          bk[i] = mb0 + x * (mb1 + x * mb2);
        }
        cbf16x8 g1, g2, g3;
        split3_bf16x8(gk, g1, g2, g3);
        typedef float f8 __attribute__((ext_vector_type(8)));
        const cbf16x8 bb = __builtin_convertvector(
            (f8){bk[0], bk[1], bk[2], bk[3], bk[4], bk[5], bk[6], bk[7]}, cbf16x8);
        acc[NBC] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g1, bb, acc[NBC], 0, 0, 0);
        am2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g2, bb, am2, 0, 0, 0);
        am3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g3, bb, am3, 0, 0, 0);
      }
      acc[NBC] += am2 + am3;
      // D layout: lane (col, g) holds rows j = 4 g + i of column 16 nc + col
#pragma unroll
      for (int nc = 0; nc <= NBC; nc++)
#pragma unroll
        for (int i = 0; i < 4; i++) mat[(4 * g + i) * kMS + 64 * w + 16 * nc + col] = acc[nc][i];
    }
    if (ncnt > 0) stage(buf ^ 1, ncnt);
    if (nncnt > 0) stage_index(buf, nncnt);
    __syncthreads();
    if (det.slots) {
      // deterministic: the tile's sums of each Gaussian go to that Gaussian's
      // slot for this tile (no atomics); a fixed-order pass adds the slots
      for (int k = t; k < kBJ * C; k += 256) {
        const int jj = k / C, c = k % C;
        if (jj < cnt) {
          const float s = (mat[jj * kMS + 0 * 64 + c] + mat[jj * kMS + 1 * 64 + c]) +
                          (mat[jj * kMS + 2 * 64 + c] + mat[jj * kMS + 3 * 64 + c]);
          const size_t sl = det_slot(det, gidx[buf][jj], tx, ty);
          if (sl < det.cap) det.slots[sl * GS + 6 + c] = s;
        }
      }
    } else {
      for (int k = t; k < kBJ * C; k += 256) {
        const int jj = k / C, c = k % C;
        if (jj < cnt) {
          const float s = (mat[jj * kMS + 0 * 64 + c] + mat[jj * kMS + 1 * 64 + c]) +
                          (mat[jj * kMS + 2 * 64 + c] + mat[jj * kMS + 3 * 64 + c]);
          if (s != 0.f) atomicAdd(gacc + (size_t)gidx[buf][jj] * GS + 6 + c, s);
        }
      }
    }
    // the moment gradients on the last kBJ threads (the first ones carry two
    // rounds of channel sums)
    const int jm = t - (256 - kBJ);
    if (jm >= 0 && jm < cnt && det.slots) {
      float mo[6];
#pragma unroll
      for (int n = 0; n < 6; n++)
        mo[n] = (mat[jm * kMS + 0 * 64 + CP + n] + mat[jm * kMS + 1 * 64 + CP + n]) +
                (mat[jm * kMS + 2 * 64 + CP + n] + mat[jm * kMS + 3 * 64 + CP + n]);
      const float *r = reinterpret_cast<const float *>(&hdr[buf][2 * jm]);
      const float up = r[0] - (float)(tx * kTile + 8), vp = r[1] - (float)(ty * kTile + 8);
      const float mx = up * mo[0] - mo[1], my = vp * mo[0] - mo[2];
      const float mxx = up * up * mo[0] - 2.f * up * mo[1] + mo[3];
      const float mxy = up * vp * mo[0] - up * mo[2] - vp * mo[1] + mo[4];
      const float myy = vp * vp * mo[0] - 2.f * vp * mo[2] + mo[5];
      const size_t sl = det_slot(det, gidx[buf][jm], tx, ty);
      if (sl < det.cap) {
        float *ga = det.slots + sl * GS;
        ga[0] = -(r[2] * mx + r[3] * my);
        ga[1] = -(r[4] * my + r[3] * mx);
        ga[2] = -0.5f * mxx;
        ga[3] = -mxy;
        ga[4] = -0.5f * myy;
        ga[5] = mo[0] / r[5];
        det.flags[sl] = 1;
      }
    } else if (jm >= 0 && jm < cnt) {
      float mo[6];
#pragma unroll
      for (int n = 0; n < 6; n++)
        mo[n] = (mat[jm * kMS + 0 * 64 + CP + n] + mat[jm * kMS + 1 * 64 + CP + n]) +
                (mat[jm * kMS + 2 * 64 + CP + n] + mat[jm * kMS + 3 * 64 + CP + n]);
      if (mo[0] != 0.f || mo[1] != 0.f || mo[2] != 0.f) {
        const float *r = reinterpret_cast<const float *>(&hdr[buf][2 * jm]);
        const float up = r[0] - (float)(tx * kTile + 8), vp = r[1] - (float)(ty * kTile + 8);
        // sums of g dx, g dy, g dx^2, g dx dy, g dy^2 with dx = u - x, dy = v - y
        const float mx = up * mo[0] - mo[1], my = vp * mo[0] - mo[2];
        const float mxx = up * up * mo[0] - 2.f * up * mo[1] + mo[3];
        const float mxy = up * vp * mo[0] - up * mo[2] - vp * mo[1] + mo[4];
        const float myy = vp * vp * mo[0] - 2.f * vp * mo[2] + mo[5];
        float *ga = gacc + (size_t)gidx[buf][jm] * GS;
        atomicAdd(ga + 0, -(r[2] * mx + r[3] * my));
        atomicAdd(ga + 1, -(r[4] * my + r[3] * mx));
        atomicAdd(ga + 2, -0.5f * mxx);
        atomicAdd(ga + 3, -mxy);
        atomicAdd(ga + 4, -0.5f * myy);
        atomicAdd(ga + 5, mo[0] / r[5]);
      }
    }
    __syncthreads();
  }
}

template <int C>
void launch_composite_fwd_t(const uint2 *ranges, const uint32_t *sorted_g, const float *records, const short4 *boxes,
                            int W, int H, int TX, int TY, float *gbuf, float *t_final, uint32_t *n_contrib,
                            uint32_t *tile_top, hipStream_t st) {
  composite_fwd_kernel<C><<<TX * TY, 256, 0, st>>>(ranges, sorted_g, records, boxes, W, H, TX, gbuf, t_final,
                                                   n_contrib, tile_top);
}

template <int C>
void launch_composite_bwd_t(const uint2 *ranges, const uint32_t *sorted_g, const float *records, const short4 *boxes,
                            int W, int H, int TX, int TY, const float *t_final, const uint32_t *n_contrib,
                            const float *dG, const float *dT, float *gacc, const DetSlots &det,
                            const uint32_t *order, hipStream_t st) {
  composite_bwd_kernel<C><<<TX * TY, 256, 0, st>>>(ranges, sorted_g, records, boxes, W, H, TX, t_final, n_contrib,
                                                   dG, dT, gacc, det, order);
}

// Tiles in descending order of the forward's largest last-contributor index
// (the backward's work per tile), so that the longest workgroups start first
// and short ones fill the end: a counting sort on min(top, 4095) in one
// workgroup.  Ties land in arbitrary order (it only changes the dispatch
// order; every result is independent of it).
constexpr int kOrderBins = 4096;

__global__ __launch_bounds__(1024) void tile_order_kernel(const uint32_t *__restrict__ tile_top, int T,
                                                          uint32_t *__restrict__ order) {
  __shared__ uint32_t bins[kOrderBins];
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  for (int b = t; b < kOrderBins; b += 1024) bins[b] = 0;
  __syncthreads();
  for (int i = t; i < T; i += 1024) atomicAdd(&bins[kOrderBins - 1 - min(tile_top[i], (uint32_t)kOrderBins - 1)], 1u);
  __syncthreads();
  // exclusive scan: 4 bins per thread, then over the threads
  uint32_t v[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    v[k] = bins[4 * t + k];
    s += v[k];
  }
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t a = t >= o ? part[t - o] : 0u;
    __syncthreads();
    part[t] += a;
    __syncthreads();
  }
  uint32_t run = part[t] - s;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    bins[4 * t + k] = run;
    run += v[k];
  }
  __syncthreads();
  for (int i = t; i < T; i += 1024) {
    const uint32_t pos = atomicAdd(&bins[kOrderBins - 1 - min(tile_top[i], (uint32_t)kOrderBins - 1)], 1u);
    order[pos] = (uint32_t)i;
  }
}

void launch_tile_order(const uint32_t *tile_top, int T, uint32_t *order, hipStream_t st) {
  tile_order_kernel<<<1, 1024, 0, st>>>(tile_top, T, order);
}

// ---------------------------------------------------------------- deterministic sums
//
// The slots of Gaussian i are toff[i] .. toff[i] + area(i) - 1, one per tile
// of its rectangle in row-major order (toff: exclusive scan of the areas).
__global__ __launch_bounds__(256) void rect_area_kernel(const ushort4 *__restrict__ rects, uint32_t n,
                                                        uint32_t *__restrict__ area) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const ushort4 r = rects[i];
  area[i] = (uint32_t)(r.z - r.x) * (uint32_t)(r.w - r.y);
}

// Per Gaussian, the sum of its flagged slots in row-major tile order (one
// thread per float4 of the accumulator row); every row is written.
template <int GS>
__global__ __launch_bounds__(256) void slot_reduce_kernel(DetSlots det, uint32_t n, float *__restrict__ gacc) {
  constexpr int Q = GS / 4;
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)n * Q) return;
  const uint32_t i = (uint32_t)(k / Q), q = (uint32_t)(k % Q);
  const ushort4 r = det.rects[i];
  const size_t base = det.toff[i];
  size_t area = (size_t)(r.z - r.x) * (size_t)(r.w - r.y);
  if (base >= det.cap) area = 0;
  else if (area > det.cap - base) area = det.cap - base;
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
  for (size_t s = 0; s < area; s++) {
    if (det.flags[base + s]) {
      const float4 v = ld4(det.slots + (base + s) * GS + 4 * q);
      a.x += v.x;
      a.y += v.y;
      a.z += v.z;
      a.w += v.w;
    }
  }
  st4(gacc + (size_t)i * GS + 4 * q, a);
}

void launch_rect_area(const ushort4 *rects, uint32_t n, uint32_t *area, hipStream_t st) {
  if (n) rect_area_kernel<<<(n + 255) / 256, 256, 0, st>>>(rects, n, area);
}

void launch_slot_reduce(int C, const DetSlots &det, uint32_t n, float *gacc, hipStream_t st) {
  if (!n) return;
  const int GS = grad_stride(C);
  const size_t threads = (size_t)n * (GS / 4);
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  switch (GS) {
    case 16: slot_reduce_kernel<16><<<blocks, 256, 0, st>>>(det, n, gacc); break;
    case 24: slot_reduce_kernel<24><<<blocks, 256, 0, st>>>(det, n, gacc); break;
    case 32: slot_reduce_kernel<32><<<blocks, 256, 0, st>>>(det, n, gacc); break;
    default: slot_reduce_kernel<48><<<blocks, 256, 0, st>>>(det, n, gacc); break;
  }
}

#define SSSGS_COMP_INST(C)                                                                                      \
  template void launch_composite_fwd_t<C>(const uint2 *, const uint32_t *, const float *, const short4 *, int,  \
                                          int, int, int, float *, float *, uint32_t *, uint32_t *,             \
                                          hipStream_t);                                                        \
  template void launch_composite_bwd_t<C>(const uint2 *, const uint32_t *, const float *, const short4 *, int,  \
                                          int, int, int, const float *, const uint32_t *, const float *,      \
                                          const float *, float *, const DetSlots &, const uint32_t *,        \
                                          hipStream_t);
SSSGS_COMP_INST(10)
SSSGS_COMP_INST(18)
SSSGS_COMP_INST(26)
SSSGS_COMP_INST(42)

}  // namespace sssgs
