// bvh.hip -- each Gaussian's visibility of the point light, by tracing a
// shadow ray through the other Gaussians with a bounding-volume hierarchy
// (Sec. 3.2, "Incident Light").
//
// What is computed: for Gaussian i the ray from its centre towards the light,
// 0 < t <= |p - mu_i|.  Another Gaussian j occludes it where the ray's line
// passes densest through j: in j's whitened frame (S^-1 R^T (x - mu_j)) the
// line is u + t w, the densest point t* = -(u.w)/(w.w) at squared distance
// D2 = |u x w|^2 / |w|^2; if t* is on the segment and
// alpha = min(0.99, opacity exp(-D2/2)) >= 1/255, the ray keeps a factor
// (1 - alpha).  v_i is the product, 0 once below 1e-4.  The product does not
// depend on the order of the occluders and only decreases, so the traversal
// needs no depth order and a ray stops when it crosses the floor.
//
// The hierarchy is a linear BVH built on the GPU each call:
//   vis_prep    per block the box of its centres, then (vis_scene) the
//               box of all centres.
//   vis_morton  30-bit Morton code of each centre in that box.
//   radix sort  of the codes (stable: index order among equal codes).
//   vis_tree    binary radix tree over the sorted codes, one thread per
//               internal node (prefix lengths of equal codes continue with
//               the bits of the sorted positions, so every split is unique).
//   vis_block_box
//               per sorted leaf an FP64 record (whitening matrix, opacity,
//               centre) and the box of the ellipsoid D2 <= 2 ln(255 opacity)
//               outside of which alpha < 1/255 (so the box test is exact,
//               not a 3-sigma heuristic); unions of 16- and 256-leaf
//               blocks (vis_super_box: of 4096-leaf blocks).
//   vis_node_box
//               boxes without inter-thread synchronisation: every internal
//               node covers a contiguous range of sorted leaves, so its box
//               is the union over that range, taken from unions of aligned
//               units of 1, 16, 256 and 4096 leaves.
//   vis_pack    per internal node one 64-byte record: both children and
//               both child boxes (one cache line per visited node).
//   vis_trace   one thread per Gaussian in Morton order (coherent rays), a
//               per-lane stack in LDS, children tested at their parent; a
//               short stack first, the rare deeper rays again with a deep one.
// The leaf test is FP64 (the densest point is a small difference of large
// terms for a distant, thin Gaussian); boxes and the slab test are FP32 with
// the boxes widened outward.
#include "launch.hpp"

namespace sssgs {

namespace {

constexpr int kVisStack = 64;       // tree depth <= 30 code bits + 32 position bits
constexpr int kVisShortStack = 32;  // first pass; deeper rays are traced again
constexpr double kFloor = 1e-4;

__device__ __forceinline__ uint32_t ordered(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unordered(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}


// Record and box of Gaussian i, stored at its sorted leaf position k.
__device__ __forceinline__ void leaf_record(const VisArgs &A, int i, int k, float *box) {
  const int n = A.n;
  double q[4], ql = 0.0;
  for (int a = 0; a < 4; a++) {
    q[a] = A.quats[a * n + i];
    ql += q[a] * q[a];
  }
  ql = sqrt(ql);
  for (int a = 0; a < 4; a++) q[a] /= ql;
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double R[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                       2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
                       2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
  double s[3], mu[3];
  for (int a = 0; a < 3; a++) {
    s[a] = exp((double)A.log_scales[a * n + i]);
    mu[a] = A.means[a * n + i];
  }
  const double op = 1.0 / (1.0 + exp(-(double)A.logits[i]));
  double rec[16];
  // whitening S^-1 R^T: row a = column a of R over s_a
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int m = 0; m < 3; m++) rec[3 * a + m] = R[3 * m + a] / s[a];
  rec[9] = op;
#pragma unroll
  for (int a = 0; a < 3; a++) rec[10 + a] = mu[a];
  rec[13] = rec[14] = rec[15] = 0.0;
  // the whole 128-byte record in eight 16-byte stores
  double2 *out = reinterpret_cast<double2 *>(A.rec + (size_t)k * 16);
#pragma unroll
  for (int q = 0; q < 8; q++) out[q] = make_double2(rec[2 * q], rec[2 * q + 1]);
  if (255.0 * op > 1.0) {
    const double r = sqrt(2.0 * log(255.0 * op));
    for (int m = 0; m < 3; m++) {
      double e2 = 0.0;
      for (int a = 0; a < 3; a++) e2 += R[3 * m + a] * R[3 * m + a] * s[a] * s[a];
      const double e = r * sqrt(e2), pad = 1e-6 * (1.0 + fabs(mu[m]) + e);
      box[m] = (float)(mu[m] - e - pad);
      box[3 + m] = (float)(mu[m] + e + pad);
    }
  } else {  // alpha can never reach 1/255: an empty box
    for (int m = 0; m < 3; m++) {
      box[m] = __int_as_float(0x7F800000);
      box[3 + m] = -__int_as_float(0x7F800000);
    }
  }
}

// Min (k < 3) or max (k >= 3) of six ordered keys over the 256 threads of a
// block; the result in red[4] after the call.
__device__ __forceinline__ void block_minmax6(uint32_t key[6], uint32_t (*red)[6]) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int k = 0; k < 6; k++) {
      const uint32_t o = (uint32_t)__shfl_xor((int)key[k], off);
      key[k] = k < 3 ? min(key[k], o) : max(key[k], o);
    }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 6; k++) red[wave][k] = key[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    uint32_t r = red[0][k];
    for (int w = 1; w < 4; w++) r = k < 3 ? min(r, red[w][k]) : max(r, red[w][k]);
    red[4][k] = r;
  }
  __syncthreads();
}

// Each block's min / max of the centres (ordered keys; reduced over the blocks by vis_scene_kernel, not by global
// atomics: on this chip atomics of all blocks on the same six words serialise
// outside the per-XCD L2s).
__global__ __launch_bounds__(256) void vis_prep_kernel(VisArgs A) {
  __shared__ uint32_t red[5][6];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool live = i < A.n;
  uint32_t key[6];
#pragma unroll
  for (int m = 0; m < 3; m++) {
    const uint32_t k = live ? ordered(A.means[m * A.n + i]) : 0u;
    key[m] = live ? k : 0xFFFFFFFFu;
    key[3 + m] = k;
  }
  block_minmax6(key, red);
  if (threadIdx.x < 6) A.bpart[(size_t)blockIdx.x * 6 + threadIdx.x] = red[4][threadIdx.x];
}

// The box of all centres from the per-block keys (one block); clears the
// status word of this call.
__global__ __launch_bounds__(256) void vis_scene_kernel(VisArgs A, int nblocks) {
  __shared__ uint32_t red[5][6];
  uint32_t key[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
  for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
    for (int k = 0; k < 6; k++) {
      const uint32_t v = A.bpart[(size_t)b * 6 + k];
      key[k] = k < 3 ? min(key[k], v) : max(key[k], v);
    }
  block_minmax6(key, red);
  if (threadIdx.x < 6) A.scene[threadIdx.x] = red[4][threadIdx.x];
  if (threadIdx.x == 6) A.status[0] = 0u;
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {  // 10 bits -> every third bit
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__global__ __launch_bounds__(256) void vis_morton_kernel(VisArgs A, uint32_t *codes, uint32_t *idx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= A.n) return;
  uint32_t c[3];
  for (int m = 0; m < 3; m++) {
    const float lo = unordered(A.scene[m]), hi = unordered(A.scene[3 + m]);
    const float ext = hi - lo;
    float f = ext > 0.f ? (A.means[m * A.n + i] - lo) / ext : 0.f;
    f = fminf(fmaxf(f, 0.f), 1.f);
    c[m] = (uint32_t)fminf(f * 1024.f, 1023.f);
  }
  codes[i] = (spread10(c[0]) << 2) | (spread10(c[1]) << 1) | spread10(c[2]);
  idx[i] = (uint32_t)i;
}

// Length of the common prefix of sorted entries a and b (codes, then
// positions); -1 outside [0, n).
__device__ __forceinline__ int prefix(const uint32_t *code, int n, int a, int b) {
  if (b < 0 || b >= n) return -1;
  const uint32_t ca = code[a], cb = code[b];
  if (ca != cb) return __clz(ca ^ cb);
  return 32 + __clz((uint32_t)a ^ (uint32_t)b);
}

// Internal node i covers a range of sorted leaves that starts or ends at i;
// its children split the range where the prefix shortens.  Children >= 0 are
// internal nodes, < 0 leaves (~position).
__global__ __launch_bounds__(256) void vis_tree_kernel(VisArgs A) {
  const int n = A.n;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n - 1) return;
  const uint32_t *code = A.codes;
  const int d = prefix(code, n, i, i + 1) - prefix(code, n, i, i - 1) >= 0 ? 1 : -1;
  const int dmin = prefix(code, n, i, i - d);
  int lmax = 2;
  while (prefix(code, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int l = 0;
  for (int t = lmax >> 1; t >= 1; t >>= 1)
    if (prefix(code, n, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  const int dnode = prefix(code, n, i, j);
  int s = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (prefix(code, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  const int split = i + s * d + (d < 0 ? -1 : 0);
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  const int left = lo == split ? ~split : split;
  const int right = hi == split + 1 ? ~(split + 1) : split + 1;
  A.left[i] = left;
  A.right[i] = right;
  A.range_lo[i] = lo;
  A.range_hi[i] = hi;
}

__device__ __forceinline__ void box_empty(float *b) {
  for (int m = 0; m < 3; m++) {
    b[m] = __int_as_float(0x7F800000);
    b[3 + m] = -__int_as_float(0x7F800000);
  }
}

__device__ __forceinline__ void box_add(float *b, const float *g) {
  for (int m = 0; m < 3; m++) {
    b[m] = fminf(b[m], g[m]);
    b[3 + m] = fmaxf(b[3 + m], g[3 + m]);
  }
}

constexpr int kBoxBlock = 256;

// The leaves' records and boxes in sorted order (a leaf is then found by its
// position, with no gather through the permutation), and the union of the
// boxes of each block of 256 consecutive sorted leaves.
__global__ __launch_bounds__(kBoxBlock) void vis_block_box_kernel(VisArgs A) {
  __shared__ float red[6][kBoxBlock];
  const int t = threadIdx.x, k = blockIdx.x * kBoxBlock + t;
  float b[6];
  box_empty(b);
  if (k < A.n) {
    float g[6];
    leaf_record(A, (int)A.order[k], k, g);
    box_add(b, g);
    for (int m = 0; m < 6; m++) A.sbox[(size_t)k * 6 + m] = g[m];
  }
  // unions of 16 consecutive leaves (aligned groups of 16 lanes)
  {
    float u[6];
#pragma unroll
    for (int m = 0; m < 6; m++) u[m] = b[m];
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1)
#pragma unroll
      for (int m = 0; m < 6; m++) {
        const float o = __shfl_xor(u[m], off);
        u[m] = m < 3 ? fminf(u[m], o) : fmaxf(u[m], o);
      }
    if ((t & 15) == 0 && k < A.n)
#pragma unroll
      for (int m = 0; m < 6; m++) A.b16[(size_t)(k >> 4) * 6 + m] = u[m];
  }
  for (int m = 0; m < 6; m++) red[m][t] = b[m];
  __syncthreads();
  for (int w = kBoxBlock / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int m = 0; m < 3; m++) {
        red[m][t] = fminf(red[m][t], red[m][t + w]);
        red[3 + m][t] = fmaxf(red[3 + m][t], red[3 + m][t + w]);
      }
    __syncthreads();
  }
  if (t < 6) A.bbox[(size_t)blockIdx.x * 6 + t] = red[t][0];
}

// Unions of 4096 consecutive leaves from 16 unions of 256.
__global__ __launch_bounds__(256) void vis_super_box_kernel(VisArgs A, int nblocks) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s * 16 >= nblocks) return;
  float b[6];
  box_empty(b);
  const int e = min(nblocks, (s + 1) * 16);
  for (int bb = s * 16; bb < e; bb++) box_add(b, A.bbox + (size_t)bb * 6);
  for (int m = 0; m < 6; m++) A.b4k[(size_t)s * 6 + m] = b[m];
}

// Box of internal node i: the union over its leaf range [lo, hi], taken
// greedily as the largest aligned whole unit of 4096, 256, 16 or 1 leaves
// that starts at the next leaf and ends inside the range (at most 15 units
// of each size on the way up and on the way down, plus the 4096-leaf units).
__global__ __launch_bounds__(256) void vis_node_box_kernel(VisArgs A) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= A.n - 1) return;
  const int lo = A.range_lo[i], end = A.range_hi[i] + 1;
  float b[6];
  box_empty(b);
  for (int k = lo; k < end;) {
    const float *u;
    if ((k & 4095) == 0 && k + 4096 <= end) {
      u = A.b4k + (size_t)(k >> 12) * 6;
      k += 4096;
    } else if ((k & 255) == 0 && k + 256 <= end) {
      u = A.bbox + (size_t)(k >> 8) * 6;
      k += 256;
    } else if ((k & 15) == 0 && k + 16 <= end) {
      u = A.b16 + (size_t)(k >> 4) * 6;
      k += 16;
    } else {
      u = A.sbox + (size_t)k * 6;
      k += 1;
    }
    box_add(b, u);
  }
  for (int m = 0; m < 6; m++) A.nbox[(size_t)i * 6 + m] = b[m];
}

// Node record: children (int bits) in floats 0, 1; left box 4..9; right box 10..15.
__global__ __launch_bounds__(256) void vis_pack_kernel(VisArgs A) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= A.n - 1) return;
  const int ch[2] = {A.left[i], A.right[i]};
  float r[16];
  r[0] = __int_as_float(ch[0]);
  r[1] = __int_as_float(ch[1]);
  r[2] = r[3] = 0.f;
#pragma unroll
  for (int c = 0; c < 2; c++) {
    const float *g = ch[c] < 0 ? A.sbox + (size_t)(~ch[c]) * 6 : A.nbox + (size_t)ch[c] * 6;
#pragma unroll
    for (int m = 0; m < 6; m++) r[4 + 6 * c + m] = g[m];
  }
  // the whole 64-byte record in four 16-byte stores
  float4 *out = reinterpret_cast<float4 *>(A.nrec + (size_t)i * 16);
#pragma unroll
  for (int q = 0; q < 4; q++) out[q] = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
}

// Does the segment o + t d, 0 <= t <= tmax, meet the box (lo, hi)?  The
// entry and exit planes are chosen by the direction's sign (not by min/max
// of the two distances), so an empty box (lo = +inf, hi = -inf) enters at
// +inf and leaves at -inf: never a hit.
__device__ __forceinline__ bool slab(const float *box, const float *o, const float *inv, float tmax) {
  float t0 = 0.f, t1 = tmax;
#pragma unroll
  for (int m = 0; m < 3; m++) {
    const bool pos = inv[m] >= 0.f;
    const float near = pos ? box[m] : box[3 + m], far = pos ? box[3 + m] : box[m];
    t0 = fmaxf(t0, (near - o[m]) * inv[m]);
    t1 = fminf(t1, (far - o[m]) * inv[m]);
  }
  return t0 <= t1;
}


// Factor (1 - alpha_j) of occluder j on the ray (o, d, tmax), or 1.
__device__ __forceinline__ double occlusion(const double *rec, const double *o, const double *d, double tmax) {
  double u[3], w[3];
  for (int k = 0; k < 3; k++) {
    const double *Wk = rec + 3 * k;
    u[k] = Wk[0] * (o[0] - rec[10]) + Wk[1] * (o[1] - rec[11]) + Wk[2] * (o[2] - rec[12]);
    w[k] = Wk[0] * d[0] + Wk[1] * d[1] + Wk[2] * d[2];
  }
  const double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double ts = -(u[0] * w[0] + u[1] * w[1] + u[2] * w[2]) / ww;
  if (!(ts > 0.0 && ts <= tmax)) return 1.0;
  const double c0 = u[1] * w[2] - u[2] * w[1], c1 = u[2] * w[0] - u[0] * w[2], c2 = u[0] * w[1] - u[1] * w[0];
  const double D2 = (c0 * c0 + c1 * c1 + c2 * c2) / ww;
  const double alpha = fmin(0.99, rec[9] * exp(-0.5 * D2));
  return alpha >= 1.0 / 255.0 ? 1.0 - alpha : 1.0;
}

// One ray per thread with an LDS stack of S entries per lane.  The first pass
// (S = kVisShortStack, half the LDS, so the registers and not the LDS bound
// the occupancy) marks a ray whose stack would overflow with a NaN and drops
// it; the second (RETRY, S = kVisStack) traces only the rays so marked.  The
// visiting order does not depend on S, so every ray's product is the one a
// single deep-stack pass computes, bit for bit.
template <int S, bool RETRY>
__global__ __launch_bounds__(64, 5) void vis_trace_kernel(VisArgs A) {
  __shared__ int stack[S][64];
  const int lane = threadIdx.x;
  const int k = blockIdx.x * 64 + lane;
  if (k >= A.n) return;
  const int n = A.n;
  const int i = (int)A.order[k];
  if (RETRY && !__builtin_isnan(A.vis[i])) return;
  double o[3], d[3], len = 0.0;
  for (int m = 0; m < 3; m++) {
    o[m] = A.means[m * n + i];
    d[m] = (double)A.light[m] - o[m];
    len += d[m] * d[m];
  }
  len = sqrt(len);
  float of[3], inv[3];
  for (int m = 0; m < 3; m++) {
    d[m] /= len;
    of[m] = (float)o[m];
    const float dm = (float)d[m];
    inv[m] = dm != 0.f ? 1.f / dm : 1e30f;
  }
  const float tmaxf = (float)len * (1.f + 1e-6f) + 1e-6f;
  double T = 1.0;
  int sp = 0;
  if (n >= 2) {
    float rb[6];
    for (int m = 0; m < 6; m++) rb[m] = A.nbox[m];
    if (slab(rb, of, inv, tmaxf)) stack[sp++][lane] = 0;
  }
  bool overflow = false;
  while (sp > 0 && T >= kFloor && !overflow) {
    const int node = stack[--sp][lane];
    const float4 *nr = reinterpret_cast<const float4 *>(A.nrec + (size_t)node * 16);
    const float4 q0 = nr[0], q1 = nr[1], q2 = nr[2], q3 = nr[3];
    const int ch[2] = {__float_as_int(q0.x), __float_as_int(q0.y)};
    const float bx[2][6] = {{q1.x, q1.y, q1.z, q1.w, q2.x, q2.y}, {q2.z, q2.w, q3.x, q3.y, q3.z, q3.w}};
#pragma unroll
    for (int c = 0; c < 2; c++) {
      if (!slab(bx[c], of, inv, tmaxf)) continue;
      const int cn = ch[c];
      if (cn < 0) {
        if (~cn != k) T *= occlusion(A.rec + (size_t)(~cn) * 16, o, d, len);
      } else if (sp < S) {
        stack[sp++][lane] = cn;
      } else {
        overflow = true;
      }
    }
  }
  float v = T < kFloor ? 0.f : (float)T;
  if (overflow) {
    v = __int_as_float(0x7FC00000);  // NaN: the stack bound was exceeded
    if (RETRY) atomicOr(A.status, 1u);
  }
  A.vis[i] = v;
}

}  // namespace

void launch_visibility(const VisArgs &a0, uint32_t *keys_a, uint32_t *vals_a, uint32_t *keys_b, uint32_t *vals_b,
                       uint32_t *hist, uint32_t *partials, hipStream_t st) {
  VisArgs a = a0;
  const int n = a.n;
  if (n <= 0) return;
  const int g256 = (n + 255) / 256;
  vis_prep_kernel<<<g256, 256, 0, st>>>(a);
  vis_scene_kernel<<<1, 256, 0, st>>>(a, g256);
  vis_morton_kernel<<<g256, 256, 0, st>>>(a, keys_a, vals_a);
  const uint32_t *kin = keys_a, *vin = vals_a;
  for (int pass = 0; pass < 4; pass++) {
    uint32_t *ko = (pass & 1) ? keys_a : keys_b;
    uint32_t *vo = (pass & 1) ? vals_a : vals_b;
    launch_radix_pass(kin, vin, ko, vo, (uint32_t)n, nullptr, pass * kRadixBits, hist, partials, false, st);  // partials: >= 256 words
    kin = ko;
    vin = vo;
  }
  a.codes = kin;
  a.order = vin;
  if (n >= 2) {
    const int gi = (n - 1 + 255) / 256;
    vis_tree_kernel<<<gi, 256, 0, st>>>(a);
    const int nblocks = (n + kBoxBlock - 1) / kBoxBlock;
    vis_block_box_kernel<<<nblocks, kBoxBlock, 0, st>>>(a);
    vis_super_box_kernel<<<(nblocks + 16 * 256 - 1) / (16 * 256), 256, 0, st>>>(a, nblocks);
    vis_node_box_kernel<<<gi, 256, 0, st>>>(a);
    vis_pack_kernel<<<gi, 256, 0, st>>>(a);
  }
  vis_trace_kernel<kVisShortStack, false><<<(n + 63) / 64, 64, 0, st>>>(a);
  vis_trace_kernel<kVisStack, true><<<(n + 63) / 64, 64, 0, st>>>(a);
}

}  // namespace sssgs
