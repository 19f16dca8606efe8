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

// Down sweep.  SUM: the block adds the partials of the blocks before it
// itself (no separate scan of the partials); otherwise partials holds their
// exclusive scan.
template <bool SUM>
__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(const uint32_t *__restrict__ in,
                                                                 uint32_t *__restrict__ out, uint32_t n,
                                                                 const uint32_t *__restrict__ partials,
                                                                 uint32_t *__restrict__ total_out) {
  __shared__ uint32_t lds[4];
  const uint32_t base = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; k++) v[k] = base + k < n ? in[base + k] : 0u;
  uint32_t before = 0;
  if (SUM) {
    uint32_t p = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads) p += partials[i];
    uint32_t tot;
    block_exclusive_scan(p, lds, tot);
    before = tot;
  } else {
    before = partials[blockIdx.x];
  }
  const uint32_t s = v[0] + v[1] + v[2] + v[3];
  uint32_t total;
  uint32_t ex = block_exclusive_scan(s, lds, total) + before;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  // the grand total, from the last block (SUM form)
  if (SUM && total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) total_out[0] = before + total;
}

// ------------------------------------------------------------------ radix pass

__device__ __forceinline__ uint32_t load_count(uint32_t n_host, const uint32_t *n_dev) {
  if (!n_dev) return n_host;
  const uint32_t m = *n_dev;
  return m < n_host ? m : n_host;
}

// Per-block digit histograms: digit-major hist[digit][block] for the scan
// across blocks, or block-major hist[block][digit] (LOCAL) when the scatter
// derives its own offsets.
template <bool LOCAL>
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
  if (LOCAL) hist[blockIdx.x * kRadixBins + t] = h[t];
  else hist[t * nblocks + blockIdx.x] = h[t];
}

// Stable scatter of one 8-bit digit.  The block ranks its keys with wave
// ballots into block-local digit runs in LDS, then streams the runs out, so
// that consecutive lanes write consecutive global addresses.  The global
// start of each of the block's runs comes from the scanned digit-major
// histogram, or (LOCAL, few blocks) from the block-major counts directly:
// all blocks' counts of the thread's digit, and those of earlier blocks.
template <bool LOCAL>
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
  if (LOCAL) {
    // Each wave sums a quarter of the blocks' counts, a lane four digits per
    // 16-byte load (eight loads in flight), for all blocks and for the blocks
    // before this one; the quarters are added through LDS.
    const int q0 = (nblocks * w) >> 2, q1 = (nblocks * (w + 1)) >> 2;
    const uint4 *h4 = reinterpret_cast<const uint4 *>(hist_scan) + lane;
    uint4 tot4 = make_uint4(0u, 0u, 0u, 0u), bel4 = make_uint4(0u, 0u, 0u, 0u);
    for (int b0 = q0; b0 < q1; b0 += 8) {
      uint4 c[8];
#pragma unroll
      for (int k = 0; k < 8; k++) c[k] = b0 + k < q1 ? h4[(size_t)(b0 + k) * (kRadixBins / 4)] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (int k = 0; k < 8; k++) {
        tot4.x += c[k].x;
        tot4.y += c[k].y;
        tot4.z += c[k].z;
        tot4.w += c[k].w;
        if (b0 + k < (int)blockIdx.x) {
          bel4.x += c[k].x;
          bel4.y += c[k].y;
          bel4.z += c[k].z;
          bel4.w += c[k].w;
        }
      }
    }
    reinterpret_cast<uint4 *>(wcnt[w])[lane] = tot4;
    reinterpret_cast<uint4 *>(wbase[w])[lane] = bel4;
    __syncthreads();
    const uint32_t tot = (wcnt[0][t] + wcnt[1][t]) + (wcnt[2][t] + wcnt[3][t]);
    const uint32_t below = (wbase[0][t] + wbase[1][t]) + (wbase[2][t] + wbase[3][t]);
    uint32_t total;
    gbase[t] = block_exclusive_scan(tot, lds4, total) + below;
  } else {
    gbase[t] = hist_scan[t * nblocks + blockIdx.x];
  }
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

// Rectangle of super-bins (squares of 2^log2s tiles) covering a tile rectangle.
__device__ __forceinline__ ushort4 super_rect(ushort4 r, int log2s) {
  if (r.z <= r.x || r.w <= r.y) return make_ushort4(0, 0, 0, 0);
  return make_ushort4(r.x >> log2s, r.y >> log2s, ((r.z - 1) >> log2s) + 1, ((r.w - 1) >> log2s) + 1);
}

// Super-bins touched by the Gaussian at each depth-sorted position; the
// block's number of tiles touched goes to area_part[block].
__global__ __launch_bounds__(256) void gather_tiles_kernel(const uint32_t *__restrict__ sorted_g,
                                                           const ushort4 *__restrict__ rects, uint32_t n, int log2s,
                                                           uint32_t *__restrict__ tt, uint32_t *__restrict__ area_part) {
  __shared__ uint32_t lds4[4];
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t area = 0;
  if (p < n) {
    const ushort4 r = rects[sorted_g[p]];
    const ushort4 q = super_rect(r, log2s);
    tt[p] = (uint32_t)(q.z - q.x) * (uint32_t)(q.w - q.y);
    area = (uint32_t)(r.z - r.x) * (uint32_t)(r.w - r.y);
  }
  uint32_t total;
  block_exclusive_scan(area, lds4, total);
  if (threadIdx.x == 0) area_part[blockIdx.x] = total;
}

// Writes each Gaussian's (super-bin, index) instances at its scanned offset.  The
// instances of a block's 256 consecutive (depth-ordered) Gaussians form one
// contiguous range of the output, which the block writes cooperatively: each
// output slot finds its Gaussian by a binary search over the block's offsets.
__global__ __launch_bounds__(256) void emit_kernel(const uint32_t *__restrict__ sorted_g,
                                                   const ushort4 *__restrict__ rects,
                                                   const uint32_t *__restrict__ offsets, uint32_t n, uint32_t cap,
                                                   int TX, int log2s, uint32_t *__restrict__ inst_keys,
                                                   uint32_t *__restrict__ inst_vals) {
  __shared__ uint32_t soff[257];
  __shared__ uint32_t sg[256];
  __shared__ ushort4 srect[256], trect[256];
  const int t = threadIdx.x;
  const uint32_t p0 = blockIdx.x * 256u, p = p0 + t;
  if (p0 >= n) return;
  const uint32_t nb = min(256u, n - p0);
  if ((uint32_t)t < nb) {
    const uint32_t g = sorted_g[p];
    const ushort4 tr = rects[g];
    const ushort4 r = super_rect(tr, log2s);
    sg[t] = g;
    srect[t] = r;
    trect[t] = tr;
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
    // key: super-bin (8 bits), then the Gaussian's tile rectangle clipped to
    // the super-bin, in super-bin-local tile coordinates (log2s bits each)
    const ushort4 t4 = trect[k];
    const uint32_t s = 1u << log2s, bx = tx << log2s, by = ty << log2s;
    const uint32_t x0 = max((uint32_t)t4.x, bx) - bx, x1 = min((uint32_t)t4.z, bx + s) - bx - 1;
    const uint32_t y0 = max((uint32_t)t4.y, by) - by, y1 = min((uint32_t)t4.w, by + s) - by - 1;
    inst_keys[o] = (ty * (uint32_t)TX + tx) | (x0 << 8) | (x1 << (8 + log2s)) | (y0 << (8 + 2 * log2s)) |
                   (y1 << (8 + 3 * log2s));  // TX: super-bins per row
    inst_vals[o] = sg[k];
  }
}

__global__ void zero_u32_kernel(uint32_t *__restrict__ p) { *p = 0u; }

// ------------------------------------------------------------------ tile lists
//
// Tile lists from super-bin lists.  The depth-sorted Gaussians are expanded
// into (super-bin, Gaussian) instances -- a super-bin is a square of 2^log2s
// tiles, sized so that there are at most 256 -- and one stable 8-bit radix
// pass makes them super-bin-major, depth order kept within each super-bin.
// Each tile then filters its super-bin's list by its own rectangle test,
// which keeps the depth order: the tile's list is written as one contiguous,
// coalesced run.  One workgroup per tile counts its instances, one block scans
// the counts into tile offsets, and one workgroup per tile writes its run.
// The result is the order (tile, depth, index) of a stable sort of all
// (tile, depth) keys.

// [start, end) of super-bin sb in the radix pass output (digit-major scanned
// histogram; digits >= the number of super-bins are empty).
__device__ __forceinline__ uint2 superbin_range(const uint32_t *__restrict__ hist_scan, int nblocks, int sb,
                                                uint32_t ms) {
  const uint32_t a = hist_scan[(size_t)sb * nblocks];
  const uint32_t b = sb + 1 < kRadixBins ? hist_scan[(size_t)(sb + 1) * nblocks] : ms;
  return make_uint2(a, b);
}

// Does the clipped rectangle packed in a super-bin key cover the tile at
// super-bin-local coordinates (lx, ly)?
__device__ __forceinline__ bool key_covers(uint32_t key, int log2s, uint32_t lx, uint32_t ly) {
  const uint32_t m = (1u << log2s) - 1u;
  const uint32_t x0 = (key >> 8) & m, x1 = (key >> (8 + log2s)) & m;
  const uint32_t y0 = (key >> (8 + 2 * log2s)) & m, y1 = (key >> (8 + 3 * log2s)) & m;
  return lx >= x0 && lx <= x1 && ly >= y0 && ly <= y1;
}

constexpr int kTileItems = 4;  // list items per thread and step
static_assert(8 + 4 * kMaxSuperbinLog2 <= 32, "super-bin key layout");

__global__ __launch_bounds__(256) void tile_count_kernel(const uint32_t *__restrict__ sb_keys,
                                                         const uint32_t *__restrict__ hist_scan, int nblocks,
                                                         const uint32_t *__restrict__ ms_dev, uint32_t cap, int TX,
                                                         int SX, int log2s, uint32_t *__restrict__ counts) {
  __shared__ uint32_t lds4[4];
  const int t = blockIdx.x;
  const uint32_t tx = t % TX, ty = t / TX;
  const uint32_t lx = tx & ((1u << log2s) - 1u), ly = ty & ((1u << log2s) - 1u);
  const uint32_t ms = min(ms_dev[0], cap);
  const uint2 rg = superbin_range(hist_scan, nblocks, (int)(ty >> log2s) * SX + (int)(tx >> log2s), ms);
  uint32_t c = 0;
  for (uint32_t i0 = rg.x + threadIdx.x * kTileItems; i0 < rg.y; i0 += 256u * kTileItems) {
#pragma unroll
    for (int j = 0; j < kTileItems; j++)
      if (i0 + j < rg.y && key_covers(sb_keys[i0 + j], log2s, lx, ly)) c++;
  }
  uint32_t total;
  block_exclusive_scan(c, lds4, total);
  if (threadIdx.x == 0) counts[t] = total;
}

// One block: tile offsets (exclusive scan of the counts), the instance count
// (the sum of the per-block tiles-touched totals: exact also when the
// super-bin instances overflowed the capacity and the counts are incomplete)
// and the status word.
__global__ __launch_bounds__(256) void tile_scan_kernel(uint32_t *__restrict__ counts, int T,
                                                        const uint32_t *__restrict__ area_part, int nparts,
                                                        uint32_t cap, uint32_t *__restrict__ m_out,
                                                        int32_t *__restrict__ status) {
  __shared__ uint32_t lds4[4];
  uint32_t msum = 0;
  for (int i = threadIdx.x; i < nparts; i += 256) msum += area_part[i];
  uint32_t mtot;
  block_exclusive_scan(msum, lds4, mtot);
  // one block scan: thread k sums, then rewrites, a contiguous chunk of counts
  const int per = (T + 255) / 256, i0 = threadIdx.x * per;
  uint32_t s = 0;
  for (int k = 0; k < per; k++)
    if (i0 + k < T) s += counts[i0 + k];
  uint32_t total;
  uint32_t ex = block_exclusive_scan(s, lds4, total);
  for (int k = 0; k < per; k++)
    if (i0 + k < T) {
      const uint32_t v = counts[i0 + k];
      counts[i0 + k] = ex;
      ex += v;
    }
  if (threadIdx.x == 0) {
    const uint32_t m = mtot;
    m_out[0] = m;
    status[kStatusMLo] = (int32_t)m;
    status[kStatusMHi] = 0;
    status[kStatusFlags] = m > cap ? kFlagOverflow : 0;
  }
}

__global__ __launch_bounds__(256) void tile_write_kernel(const uint32_t *__restrict__ sb_keys,
                                                         const uint32_t *__restrict__ sb_list,
                                                         const uint32_t *__restrict__ hist_scan, int nblocks,
                                                         const uint32_t *__restrict__ ms_dev, int TX, int T, int SX,
                                                         int log2s, const uint32_t *__restrict__ tile_off,
                                                         const uint32_t *__restrict__ m_dev, uint32_t cap,
                                                         uint32_t *__restrict__ out_tiles,
                                                         uint32_t *__restrict__ out_gauss, uint2 *__restrict__ ranges) {
  __shared__ uint32_t lds4[4];
  const int t = blockIdx.x;
  const uint32_t m = m_dev[0];
  if (m > cap) {  // overflow: empty tiles, nothing written
    if (threadIdx.x == 0) ranges[t] = make_uint2(0u, 0u);
    return;
  }
  const uint32_t tx = t % TX, ty = t / TX;
  const uint32_t lx = tx & ((1u << log2s) - 1u), ly = ty & ((1u << log2s) - 1u);
  const uint2 rg =
      superbin_range(hist_scan, nblocks, (int)(ty >> log2s) * SX + (int)(tx >> log2s), min(ms_dev[0], cap));
  const uint32_t start = tile_off[t];
  uint32_t run = start;
  for (uint32_t c0 = rg.x; c0 < rg.y; c0 += 256u * kTileItems) {
    // thread k takes the contiguous items c0 + kTileItems k + j, so the
    // block-wide prefix of per-thread hit counts keeps the list order
    const uint32_t i0 = c0 + threadIdx.x * kTileItems;
    bool hit[kTileItems];
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < kTileItems; j++) {
      hit[j] = i0 + j < rg.y && key_covers(sb_keys[i0 + j], log2s, lx, ly);
      c += hit[j];
    }
    uint32_t total;
    uint32_t pos = run + block_exclusive_scan(c, lds4, total);
#pragma unroll
    for (int j = 0; j < kTileItems; j++)
      if (hit[j]) {
        out_tiles[pos] = (uint32_t)t;
        out_gauss[pos] = sb_list[i0 + j];
        pos++;
      }
    run += total;
  }
  if (threadIdx.x == 0) ranges[t] = make_uint2(start, run);
}


// ------------------------------------------------------------------ host side

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

constexpr uint32_t kScanSumBlocks = 4096;  // up to this many blocks a scan skips the partials pass

// Exclusive scan of n (host-known bound) u32 values; total written to total_dev.
void launch_scan(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *partials, uint32_t *total_dev,
                 hipStream_t st) {
  const uint32_t nb = n ? cdiv(n, kScanItems) : 1;
  scan_reduce_kernel<<<nb, kScanThreads, 0, st>>>(in, n, partials);
  if (n && nb <= kScanSumBlocks) {
    // few blocks: each down-sweep block sums the partials before it, the
    // last one writes the total
    scan_down_kernel<true><<<nb, kScanThreads, 0, st>>>(in, out, n, partials, total_dev);
    return;
  }
  scan_partials_kernel<<<1, kScanThreads, 0, st>>>(partials, nb, total_dev);
  if (n) scan_down_kernel<false><<<nb, kScanThreads, 0, st>>>(in, out, n, partials, nullptr);
}

uint32_t radix_blocks(uint64_t n) { return n ? cdiv(n, kSortItems) : 1; }
uint32_t scan_partials_needed(uint64_t n) { return n ? cdiv(n, kScanItems) : 1; }

// One stable 8-bit pass (keys/vals in -> out) over min(n_host, *n_dev) items.
void launch_radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, uint32_t n_host,
                       const uint32_t *n_dev, int shift, uint32_t *hist, uint32_t *partials, hipStream_t st,
                       bool digit_major) {
  const uint32_t nb = radix_blocks(n_host);
  if (!digit_major && nb <= kRadixLocalBlocks) {
    // two launches: each scatter block sums the (few) block histograms itself
    radix_hist_kernel<true><<<nb, kSortThreads, 0, st>>>(kin, n_host, n_dev, shift, hist, (int)nb);
    radix_scatter_kernel<true><<<nb, kSortThreads, 0, st>>>(kin, vin, kout, vout, n_host, n_dev, shift, hist, (int)nb);
    return;
  }
  radix_hist_kernel<false><<<nb, kSortThreads, 0, st>>>(kin, n_host, n_dev, shift, hist, (int)nb);
  launch_scan(hist, hist, nb * kRadixBins, partials, nullptr, st);
  radix_scatter_kernel<false><<<nb, kSortThreads, 0, st>>>(kin, vin, kout, vout, n_host, n_dev, shift, hist, (int)nb);
}



int superbin_log2(int TX, int TY) {
  int l = 0;
  while ((uint64_t)cdiv(TX, 1u << l) * cdiv(TY, 1u << l) > (uint64_t)kRadixBins) l++;
  return l;
}

// The super-bin key packs 8 bits of super-bin and four log2s-bit coordinates.
bool superbin_supported(int TX, int TY) { return superbin_log2(TX, TY) <= kMaxSuperbinLog2; }

uint32_t area_parts(uint32_t n) { return n ? cdiv(n, 256) : 1; }

void launch_superbin_expand(const uint32_t *sorted_g, const ushort4 *rects, uint32_t n, uint32_t cap, int TX, int TY,
                            uint32_t *tt, uint32_t *offs, uint32_t *ka, uint32_t *va, uint32_t *partials,
                            uint32_t *ms_dev, uint32_t *area_part, hipStream_t st) {
  const int log2s = superbin_log2(TX, TY);
  const int SX = (int)cdiv(TX, 1u << log2s);
  if (n) gather_tiles_kernel<<<cdiv(n, 256), 256, 0, st>>>(sorted_g, rects, n, log2s, tt, area_part);
  else zero_u32_kernel<<<1, 1, 0, st>>>(area_part);
  launch_scan(tt, offs, n, partials, ms_dev, st);
  if (n) emit_kernel<<<cdiv(n, 256), 256, 0, st>>>(sorted_g, rects, offs, n, cap, SX, log2s, ka, va);
}

void launch_tile_lists(uint32_t n, uint32_t cap, int TX, int TY, uint32_t *ka, uint32_t *va, uint32_t *kb,
                       uint32_t *vb, uint32_t *counts, uint32_t *hist, uint32_t *partials, const uint32_t *ms_dev,
                       const uint32_t *area_part, uint32_t *m_out, int32_t *status, uint2 *ranges, hipStream_t st) {
  const int log2s = superbin_log2(TX, TY);
  const int SX = (int)cdiv(TX, 1u << log2s);
  const int T = TX * TY;
  // one stable 8-bit pass: super-bin-major, depth order within each super-bin
  launch_radix_pass(ka, va, kb, vb, cap, ms_dev, 0, hist, partials, st, true);  // ranges read the scanned histogram
  const int nb = (int)radix_blocks(cap);
  tile_count_kernel<<<T, 256, 0, st>>>(kb, hist, nb, ms_dev, cap, TX, SX, log2s, counts);
  tile_scan_kernel<<<1, 256, 0, st>>>(counts, T, area_part, (int)area_parts(n), cap, m_out, status);
  tile_write_kernel<<<T, 256, 0, st>>>(kb, vb, hist, nb, ms_dev, TX, T, SX, log2s, counts, m_out, cap, ka, va,
                                       ranges);
}



}  // namespace sssgs
