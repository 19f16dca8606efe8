// binning.hip -- tile binning by a least-significant-digit radix sort of
// (tile id | depth) keys.
//
// The key of an instance is (tile << 32 | depth bits); an LSD radix sort
// handles the 32 depth bits first and the tile bits last.  The depth passes
// run on the N Gaussians before they are expanded into M >> N instances:
// expansion emits a Gaussian's instances in its depth-sorted position and the
// later (tile) passes are stable, so the result is the same total order
// (tile, depth, index) as sorting all M 64-bit keys, at a fraction of the
// traffic.  Every pass is a stable 8-bit counting pass: per-block digit
// histograms, one exclusive scan over all of them (digit-major), and a
// scatter in which each block ranks its keys stably with wave ballots.
#include "common.hpp"

namespace sssgs {

// ------------------------------------------------------------------ scans

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan over a 256-thread block; returns the block total in `total`.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds4, uint32_t &total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t inc = wave_inclusive_scan(v, lane);
  if (lane == 63) lds4[w] = inc;
  __syncthreads();
  uint32_t off = 0;
  for (int k = 0; k < w; k++) off += lds4[k];
  total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
  __syncthreads();
  return off + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t *__restrict__ in, uint32_t n,
                                                                   uint32_t *__restrict__ partials) {
  __shared__ uint32_t lds[4];
  const uint32_t base = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; k++)
    if (base + k < n) s += in[base + k];
  uint32_t total;
  block_exclusive_scan(s, lds, total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// One block: exclusive scan of the block partials in place; the grand total
// goes to total_out[0] (and, when status is given, to the instance count).
__global__ __launch_bounds__(kScanThreads) void scan_partials_kernel(uint32_t *__restrict__ partials, uint32_t np,
                                                                     uint32_t *__restrict__ total_out) {
  __shared__ uint32_t lds[4];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < np; base += kScanThreads) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < np ? partials[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, lds, total);
    if (i < np) partials[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0 && total_out) total_out[0] = carry;
}

__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(const uint32_t *__restrict__ in,
                                                                 uint32_t *__restrict__ out, uint32_t n,
                                                                 const uint32_t *__restrict__ partials) {
  __shared__ uint32_t lds[4];
  const uint32_t base = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; k++) v[k] = base + k < n ? in[base + k] : 0u;
  const uint32_t s = v[0] + v[1] + v[2] + v[3];
  uint32_t total;
  uint32_t ex = block_exclusive_scan(s, lds, total) + partials[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
}

// ------------------------------------------------------------------ radix pass

__device__ __forceinline__ uint32_t load_count(uint32_t n_host, const uint32_t *n_dev) {
  if (!n_dev) return n_host;
  const uint32_t m = *n_dev;
  return m < n_host ? m : n_host;
}

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint32_t *__restrict__ keys, uint32_t n_host,
                                                                  const uint32_t *__restrict__ n_dev, int shift,
                                                                  uint32_t *__restrict__ hist, int nblocks) {
  __shared__ uint32_t h[kRadixBins];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const uint32_t n = load_count(n_host, n_dev);
  const uint32_t base = blockIdx.x * kSortItems;
#pragma unroll
  for (int r = 0; r < kSortRounds; r++) {
    const uint32_t idx = base + r * kSortThreads + t;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (kRadixBins - 1)], 1u);
  }
  __syncthreads();
  hist[t * nblocks + blockIdx.x] = h[t];
}

// Stable scatter of one 8-bit digit.  The block ranks its keys with wave
// ballots into block-local digit runs in LDS, then streams the runs out, so
// that consecutive lanes write consecutive global addresses.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    uint32_t *__restrict__ vals_out, uint32_t n_host, const uint32_t *__restrict__ n_dev, int shift,
    const uint32_t *__restrict__ hist_scan, int nblocks) {
  __shared__ uint32_t run[kRadixBins];   // running block-local position per digit
  __shared__ uint32_t loff[kRadixBins];  // block-local start of each digit's run
  __shared__ uint32_t gbase[kRadixBins]; // global start of this block's run of each digit
  __shared__ uint32_t wcnt[4][kRadixBins];
  __shared__ uint32_t wbase[4][kRadixBins];
  __shared__ uint32_t sk[kSortItems], sv[kSortItems];
  __shared__ uint32_t lds4[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t n = load_count(n_host, n_dev);
  const uint32_t base = blockIdx.x * kSortItems;
  if (base >= n) return;  // uniform per block
  const uint32_t cnt = min((uint32_t)kSortItems, n - base);
  uint32_t key[kSortRounds], val[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; r++) {
    const uint32_t idx = base + r * kSortThreads + t;
    key[r] = idx < n ? keys_in[idx] : 0u;
    val[r] = idx < n ? vals_in[idx] : 0u;
  }
  run[t] = 0;
  gbase[t] = hist_scan[t * nblocks + blockIdx.x];
#pragma unroll
  for (int k = 0; k < 4; k++) wcnt[k][t] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortRounds; r++)
    if (r * kSortThreads + t < (int)cnt) atomicAdd(&run[(key[r] >> shift) & (kRadixBins - 1)], 1u);
  __syncthreads();
  {
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(run[t], lds4, total);
    loff[t] = ex;
    run[t] = ex;
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < kSortRounds; r++) {
    const bool active = r * kSortThreads + t < (int)cnt;
    const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
    uint64_t match = __ballot(active);
#pragma unroll
    for (int b = 0; b < kRadixBits; b++) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bl = __ballot(bit);
      match &= bit ? bl : ~bl;
    }
    const uint32_t rank = __popcll(match & lt);
    if (active && rank == 0) wcnt[w][d] = __popcll(match);
    __syncthreads();
    {
      uint32_t s = run[t];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const uint32_t c = wcnt[k][t];
        wbase[k][t] = s;
        s += c;
        wcnt[k][t] = 0;
      }
      run[t] = s;
    }
    __syncthreads();
    if (active) {
      const uint32_t pos = wbase[w][d] + rank;
      sk[pos] = key[r];
      sv[pos] = val[r];
    }
  }
  __syncthreads();
  for (uint32_t i = t; i < cnt; i += kSortThreads) {
    const uint32_t k = sk[i], d = (k >> shift) & (kRadixBins - 1);
    const uint32_t pos = gbase[d] + (i - loff[d]);
    keys_out[pos] = k;
    vals_out[pos] = sv[i];
  }
}

// ------------------------------------------------------------------ expansion

// tiles touched by the Gaussian at each depth-sorted position
__global__ __launch_bounds__(256) void gather_tiles_kernel(const uint32_t *__restrict__ sorted_g,
                                                           const ushort4 *__restrict__ rects, uint32_t n,
                                                           uint32_t *__restrict__ tt) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const ushort4 r = rects[sorted_g[p]];
  tt[p] = (uint32_t)(r.z - r.x) * (uint32_t)(r.w - r.y);
}

// Writes each Gaussian's (tile, index) instances at its scanned offset.  The
// instances of a block's 256 consecutive (depth-ordered) Gaussians form one
// contiguous range of the output, which the block writes cooperatively: each
// output slot finds its Gaussian by a binary search over the block's offsets.
__global__ __launch_bounds__(256) void emit_kernel(const uint32_t *__restrict__ sorted_g,
                                                   const ushort4 *__restrict__ rects,
                                                   const uint32_t *__restrict__ offsets, uint32_t n, uint32_t cap,
                                                   int TX, uint32_t *__restrict__ inst_keys,
                                                   uint32_t *__restrict__ inst_vals, const uint32_t *__restrict__ m_dev,
                                                   int32_t *__restrict__ status) {
  __shared__ uint32_t soff[257];
  __shared__ uint32_t sg[256];
  __shared__ ushort4 srect[256];
  const int t = threadIdx.x;
  const uint32_t p0 = blockIdx.x * 256u, p = p0 + t;
  const uint32_t mtot = m_dev[0];
  if (p == 0) {
    status[kStatusMLo] = (int32_t)mtot;
    status[kStatusMHi] = 0;
    status[kStatusFlags] = mtot > cap ? kFlagOverflow : 0;
  }
  if (p0 >= n) return;  // only with n == 0 (one block is launched for the status word)
  const uint32_t nb = min(256u, n - p0);
  if ((uint32_t)t < nb) {
    const uint32_t g = sorted_g[p];
    const ushort4 r = rects[g];
    sg[t] = g;
    srect[t] = r;
    soff[t] = offsets[p];
    if ((uint32_t)t == nb - 1) soff[nb] = offsets[p] + (uint32_t)(r.z - r.x) * (uint32_t)(r.w - r.y);
  }
  __syncthreads();
  const uint32_t lo = soff[0], hi = min(soff[nb], cap);
  for (uint32_t o = lo + t; o < hi; o += 256u) {
    // the Gaussian k with soff[k] <= o < soff[k + 1] (empty ranges skipped by the search)
    int k = 0;
#pragma unroll
    for (int step = 128; step > 0; step >>= 1)
      if (k + step < (int)nb && soff[k + step] <= o) k += step;
    const ushort4 r = srect[k];
    const uint32_t wx = (uint32_t)(r.z - r.x), q = o - soff[k];
    const uint32_t ty = r.y + q / wx, tx = r.x + q % wx;
    inst_keys[o] = ty * (uint32_t)TX + tx;
    inst_vals[o] = sg[k];
  }
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *__restrict__ p, uint32_t v, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void tile_ranges_kernel(const uint32_t *__restrict__ keys,
                                                          const uint32_t *__restrict__ m_dev, uint32_t cap,
                                                          uint2 *__restrict__ ranges) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t m = load_count(cap, m_dev);
  if (i >= m) return;
  const uint32_t k = keys[i];
  if (i == 0 || keys[i - 1] != k) ranges[k].x = i;
  if (i + 1 == m || keys[i + 1] != k) ranges[k].y = i + 1;
}

// ------------------------------------------------------------------ host side

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Exclusive scan of n (host-known bound) u32 values; total written to total_dev.
void launch_scan(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *partials, uint32_t *total_dev,
                 hipStream_t st) {
  const uint32_t nb = n ? cdiv(n, kScanItems) : 1;
  scan_reduce_kernel<<<nb, kScanThreads, 0, st>>>(in, n, partials);
  scan_partials_kernel<<<1, kScanThreads, 0, st>>>(partials, nb, total_dev);
  if (n) scan_down_kernel<<<nb, kScanThreads, 0, st>>>(in, out, n, partials);
}

uint32_t radix_blocks(uint64_t n) { return n ? cdiv(n, kSortItems) : 1; }
uint32_t scan_partials_needed(uint64_t n) { return n ? cdiv(n, kScanItems) : 1; }

// One stable 8-bit pass (keys/vals in -> out) over min(n_host, *n_dev) items.
void launch_radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, uint32_t n_host,
                       const uint32_t *n_dev, int shift, uint32_t *hist, uint32_t *partials, hipStream_t st) {
  const uint32_t nb = radix_blocks(n_host);
  radix_hist_kernel<<<nb, kSortThreads, 0, st>>>(kin, n_host, n_dev, shift, hist, (int)nb);
  launch_scan(hist, hist, nb * kRadixBins, partials, nullptr, st);
  radix_scatter_kernel<<<nb, kSortThreads, 0, st>>>(kin, vin, kout, vout, n_host, n_dev, shift, hist, (int)nb);
}

void launch_gather_tiles(const uint32_t *sorted_g, const ushort4 *rects, uint32_t n, uint32_t *tt, hipStream_t st) {
  if (n) gather_tiles_kernel<<<cdiv(n, 256), 256, 0, st>>>(sorted_g, rects, n, tt);
}

void launch_emit(const uint32_t *sorted_g, const ushort4 *rects, const uint32_t *offsets, uint32_t n, uint32_t cap,
                 int TX, uint32_t *ik, uint32_t *iv, const uint32_t *m_dev, int32_t *status, hipStream_t st) {
  emit_kernel<<<n ? cdiv(n, 256) : 1, 256, 0, st>>>(sorted_g, rects, offsets, n, cap, TX, ik, iv, m_dev, status);
}

void launch_fill_u32(uint32_t *p, uint32_t v, uint32_t n, hipStream_t st) {
  if (n) fill_u32_kernel<<<cdiv(n, 256), 256, 0, st>>>(p, v, n);
}

void launch_tile_ranges(const uint32_t *keys, const uint32_t *m_dev, uint32_t cap, uint2 *ranges, hipStream_t st) {
  if (cap) tile_ranges_kernel<<<cdiv(cap, 256), 256, 0, st>>>(keys, m_dev, cap, ranges);
}

}  // namespace sssgs
