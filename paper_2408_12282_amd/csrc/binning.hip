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
// counts, a scan down each digit's column of block counts (one workgroup per
// digit, active blocks only) giving the digit totals and each block's count
// before it, and a scatter in which each block ranks its keys stably with
// wave ballots.
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

// Exclusive scan over a block of NW waves; lds holds NW words.  Returns the
// block total in `total`.
template <int NW>
__device__ __forceinline__ uint32_t block_exclusive_scan_w(uint32_t v, uint32_t *lds, uint32_t &total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t inc = wave_inclusive_scan(v, lane);
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NW; k++) {
    const uint32_t c = lds[k];
    off += k < w ? c : 0u;
    tot += c;
  }
  total = tot;
  __syncthreads();
  return off + inc - v;
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

// Per-block digit counts, block-major: hist[block][digit].  Blocks past the
// item count write nothing (the column scan reads only the active blocks).
// Sixteen waves per block, each adding into one of four LDS copies of the
// counts (fewer waves queued on one address when a digit dominates).
constexpr int kHistThreads = 1024;
constexpr int kHistRounds = kSortItems / kHistThreads;
static_assert(kHistRounds * kHistThreads == kSortItems && kHistThreads == 4 * kRadixBins,
              "count block covers one scatter block; one thread per count entry");
__global__ __launch_bounds__(kHistThreads) void radix_hist_kernel(const uint32_t *__restrict__ keys, uint32_t n_host,
                                                                  const uint32_t *__restrict__ n_dev, int shift,
                                                                  uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[4][kRadixBins];
  const int t = threadIdx.x;
  const uint32_t n = load_count(n_host, n_dev);
  const uint32_t base = blockIdx.x * kSortItems;
  if (base >= n) return;  // uniform per block
  (&h[0][0])[t] = 0;
  __syncthreads();
  uint32_t *hc = h[(t >> 6) & 3];
#pragma unroll
  for (int r = 0; r < kHistRounds; r++) {
    const uint32_t idx = base + r * kHistThreads + t;
    if (idx < n) atomicAdd(&hc[(keys[idx] >> shift) & (kRadixBins - 1)], 1u);
  }
  __syncthreads();
  if (t < kRadixBins) hist[blockIdx.x * kRadixBins + t] = (h[0][t] + h[1][t]) + (h[2][t] + h[3][t]);
}

// One workgroup per digit d: hist[b][d] becomes the count of digit d in the
// blocks before b (exclusive scan down the column, over the active blocks
// only), and tot[d] the digit's total.  A thread takes four consecutive
// blocks per step.
__global__ __launch_bounds__(kSortThreads) void radix_colscan_kernel(uint32_t *__restrict__ hist, uint32_t n_host,
                                                                     const uint32_t *__restrict__ n_dev,
                                                                     uint32_t *__restrict__ tot) {
  __shared__ uint32_t lds4[4];
  const int d = blockIdx.x, t = threadIdx.x;
  const uint32_t n = load_count(n_host, n_dev);
  const uint32_t na = (n + kSortItems - 1) / kSortItems;
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < na; b0 += 4 * kSortThreads) {
    const uint32_t b = b0 + 4 * t;
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = b + k < na ? hist[(size_t)(b + k) * kRadixBins + d] : 0u;
    uint32_t total;
    uint32_t ex = carry + block_exclusive_scan((v[0] + v[1]) + (v[2] + v[3]), lds4, total);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      if (b + k < na) hist[(size_t)(b + k) * kRadixBins + d] = ex;
      ex += v[k];
    }
    carry += total;
  }
  if (t == 0) tot[d] = carry;
}

// Stable scatter of one 8-bit digit, kSortItems keys per block of
// kScatterWaves waves.  The block ranks its keys with wave ballots into
// block-local digit runs in LDS, then streams the runs out, so that
// consecutive lanes write consecutive global addresses.  The global start of
// the block's run of digit d is the start of digit d (exclusive scan of the
// digit totals) plus the count of digit d in earlier blocks: read from the
// column-scanned counts, or (LOCAL: few blocks, a host-known item count, no
// column scan) summed by the block itself from all blocks' counts -- each
// wave an eighth of the blocks, a lane four digits per 16-byte load with
// eight in flight, the eighths added through LDS.
constexpr int kScatterWaves = 8;
constexpr int kScatterThreads = 64 * kScatterWaves;
constexpr int kScatterRounds = kSortItems / kScatterThreads;
static_assert(kScatterRounds * kScatterThreads == kSortItems, "scatter block covers one count block");
template <bool LOCAL>
__global__ __launch_bounds__(kScatterThreads) void radix_scatter_kernel(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    uint32_t *__restrict__ vals_out, uint32_t n_host, const uint32_t *__restrict__ n_dev, int shift,
    const uint32_t *__restrict__ hist_col, const uint32_t *__restrict__ tot) {
  constexpr int NR = kScatterRounds * kScatterWaves;  // (round, wave) rows in item order
  __shared__ uint32_t rc[NR][kRadixBins];  // digit counts per (round, wave), then their prefix per digit
  __shared__ uint32_t loff[kRadixBins];    // block-local start of each digit's run
  __shared__ uint32_t gbase[kRadixBins];   // global start of this block's run of each digit
  __shared__ uint32_t wcnt[kScatterWaves][kRadixBins];
  __shared__ uint32_t wbase[kScatterWaves][kRadixBins];
  __shared__ uint32_t sk[kSortItems], sv[kSortItems];
  __shared__ uint32_t ldsw[kScatterWaves];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const bool dig = t < kRadixBins;  // the threads that own a digit
  const uint32_t n = load_count(n_host, n_dev);
  const uint32_t base = blockIdx.x * kSortItems;
  if (base >= n) return;  // uniform per block
  const uint32_t cnt = min((uint32_t)kSortItems, n - base);
  uint32_t key[kScatterRounds], val[kScatterRounds];
#pragma unroll
  for (int r = 0; r < kScatterRounds; r++) {
    const uint32_t idx = base + r * kScatterThreads + t;
    key[r] = idx < n ? keys_in[idx] : 0u;
    val[r] = idx < n ? vals_in[idx] : 0u;
  }
  uint32_t *rcf = &rc[0][0];
#pragma unroll
  for (int k = 0; k < NR * kRadixBins / kScatterThreads; k++) rcf[k * kScatterThreads + t] = 0u;
  uint32_t dt = 0, below = 0;
  if (LOCAL) {
    const int nblocks = (int)((n + kSortItems - 1) / kSortItems);
    const int q0 = (nblocks * w) / kScatterWaves, q1 = (nblocks * (w + 1)) / kScatterWaves;
    const uint4 *h4 = reinterpret_cast<const uint4 *>(hist_col) + lane;
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
    if (dig) {
#pragma unroll
      for (int k = 0; k < kScatterWaves; k++) {
        dt += wcnt[k][t];
        below += wbase[k][t];
      }
    }
  } else if (dig) {
    dt = tot[t];
    below = hist_col[blockIdx.x * kRadixBins + t];
  }
  {
    uint32_t total;
    const uint32_t ex = block_exclusive_scan_w<kScatterWaves>(dt, ldsw, total);
    if (dig) gbase[t] = ex + below;
  }
  // Rank every key among the block's keys of its digit that come before it
  // (item order r, w, lane): its rank among the equal digits of its wave and
  // round from the ballots, and the counts of the earlier (round, wave) rows,
  // summed per digit once for all rows -- three barriers for the whole block.
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t rank[kScatterRounds];
#pragma unroll
  for (int r = 0; r < kScatterRounds; r++) {
    const bool active = r * kScatterThreads + t < (int)cnt;
    const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
    uint64_t match = __builtin_amdgcn_ballot_w64(active);
#pragma unroll
    for (int b = 0; b < kRadixBits; b++) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bl = __builtin_amdgcn_ballot_w64(bit);
      match &= bit ? bl : ~bl;
    }
    rank[r] = __popcll(match & lt);
    if (active && rank[r] == 0) rc[r * kScatterWaves + w][d] = __popcll(match);
  }
  __syncthreads();
  {
    uint32_t s = 0;
    if (dig) {
#pragma unroll
      for (int k = 0; k < NR; k++) {
        const uint32_t c = rc[k][t];
        rc[k][t] = s;
        s += c;
      }
    }
    uint32_t total;
    const uint32_t ex = block_exclusive_scan_w<kScatterWaves>(s, ldsw, total);
    if (dig) loff[t] = ex;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kScatterRounds; r++) {
    if (r * kScatterThreads + t < (int)cnt) {
      const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
      const uint32_t pos = loff[d] + rc[r * kScatterWaves + w][d] + rank[r];
      sk[pos] = key[r];
      sv[pos] = val[r];
    }
  }
  __syncthreads();
  for (uint32_t i = t; i < cnt; i += kScatterThreads) {
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

// Super-bins touched by the Gaussian at each depth-sorted position, kScanItems
// positions per block (four per thread, coalesced): the block's sum of them
// goes to partials[block] -- the block sums of the exclusive scan that
// follows, which then needs no reduction pass of its own -- and its number of
// tiles touched to area_part[block].
__global__ __launch_bounds__(kScanThreads) void gather_tiles_kernel(const uint32_t *__restrict__ sorted_g,
                                                                    const ushort4 *__restrict__ rects, uint32_t n,
                                                                    int log2s, uint32_t *__restrict__ tt,
                                                                    uint32_t *__restrict__ partials,
                                                                    uint32_t *__restrict__ area_part) {
  __shared__ uint32_t lds4[4];
  uint32_t sum = 0, area = 0;
#pragma unroll
  for (int k = 0; k < kScanItems / kScanThreads; k++) {
    const uint32_t p = blockIdx.x * kScanItems + k * kScanThreads + threadIdx.x;
    if (p < n) {
      const ushort4 r = rects[sorted_g[p]];
      const ushort4 q = super_rect(r, log2s);
      const uint32_t c = (uint32_t)(q.z - q.x) * (uint32_t)(q.w - q.y);
      tt[p] = c;
      sum += c;
      area += (uint32_t)(r.z - r.x) * (uint32_t)(r.w - r.y);
    }
  }
  uint32_t total;
  block_exclusive_scan(sum, lds4, total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
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
// into (super-bin, Gaussian) instances -- a super-bin is a square of
// S = 2^log2s tiles on a side, sized so that there are at most 256 -- and one
// stable 8-bit radix pass makes them super-bin-major, depth order kept within
// each super-bin.  Each super-bin's list is cut into pieces of kPieceItems
// consecutive items, and one wave takes a piece: it reads each item once and,
// for every tile of the super-bin, one wave ballot per 64 items says which of
// them cover the tile, in list order.  Four kernels: the count kernel writes
// per (piece, tile) counts; one workgroup per super-bin turns them, per tile,
// into the count before each piece (and the tile's total); one block scans
// the totals into the tiles' list offsets in row-major tile order; the write
// kernel writes every tile's items at its offset plus the piece's prefix plus
// the item's ballot rank.  Pieces spread the work of the heaviest super-bins
// over the whole chip.  The result is the order (tile, depth, index) of a
// stable sort of all (tile, depth) keys.

constexpr int kPieceItems = 256;  // items per piece: four 64-item chunks, loaded together
constexpr int kPieceWaves = 4;    // waves per workgroup of the piece kernels
constexpr int kPieceGrid = 2048;  // at most this many workgroups; each wave loops over pieces
static_assert(8 + 4 * kMaxSuperbinLog2 <= 32, "super-bin key layout");

// Pieces of the super-bin lists: pf[sb] = first piece of super-bin sb,
// pf[256] = the number of pieces; beg / end = the super-bin's list.
struct PieceTable {
  uint32_t pf[kRadixBins + 1];
  uint32_t beg[kRadixBins], end[kRadixBins];
};

// Built by a 256-thread workgroup (thread = super-bin) from the super-bin
// totals of the radix pass.
__device__ void build_piece_table(PieceTable &pt, const uint32_t *__restrict__ sb_tot, uint32_t *lds4) {
  const int t = threadIdx.x;
  const uint32_t c = sb_tot[t];
  uint32_t total;
  const uint32_t b = block_exclusive_scan(c, lds4, total);
  pt.pf[t] = block_exclusive_scan((c + kPieceItems - 1) / kPieceItems, lds4, total);
  pt.beg[t] = b;
  pt.end[t] = b + c;
  if (t == 0) pt.pf[kRadixBins] = total;
  __syncthreads();
}

// Super-bin of piece p (< the number of pieces): the last sb with pf[sb] <= p.
__device__ __forceinline__ int piece_superbin(const PieceTable &pt, uint32_t p) {
  int lo = 0;
#pragma unroll
  for (int step = kRadixBins / 2; step > 0; step >>= 1)
    if (pt.pf[lo + step] <= p) lo += step;
  return lo;
}

// Tile rectangle of a super-bin key, in super-bin-local coordinates: x0, the
// width minus one, y0, the height minus one (log2s bits each after the 8-bit
// super-bin id).  A lane without an item gets a row offset no tile matches.
struct LocalRect {
  uint32_t x0, wx, y0, wy;
};

__device__ __forceinline__ LocalRect key_rect(uint32_t key, int log2s, bool valid) {
  const uint32_t m = (1u << log2s) - 1u;
  LocalRect r;
  r.x0 = (key >> 8) & m;
  r.wx = ((key >> (8 + log2s)) & m) - r.x0;
  r.y0 = valid ? (key >> (8 + 2 * log2s)) & m : 0xFFFFu;
  r.wy = ((key >> (8 + 3 * log2s)) & m) - ((key >> (8 + 2 * log2s)) & m);
  return r;
}

// The tiles of a super-bin are taken in blocks of up to 64 (lane j of a wave
// stands for local tile 64 tb + j, row-major in the super-bin): one block for
// S <= 8, S^2 / 64 blocks above.  Rows of block tb: [row0, row0 + nrows).
struct TileBlock {
  int row0, nrows;
};

__device__ __forceinline__ TileBlock tile_block(int log2s, int tb) {
  const int S = 1 << log2s, per = S * S < 64 ? S : 64 / S;
  return TileBlock{tb * per, per};
}

__device__ __forceinline__ int tile_blocks(int log2s) { return log2s <= 3 ? 1 : (1 << (2 * log2s)) / 64; }

// Global tile id of local tile (lx, ly) of super-bin sb, or -1 outside the grid.
__device__ __forceinline__ int tile_of(int sb, int SX, int log2s, int lx, int ly, int TX, int TY) {
  const int tx = ((sb % SX) << log2s) + lx, ty = ((sb / SX) << log2s) + ly;
  return tx < TX && ty < TY ? ty * TX + tx : -1;
}

// Items [i0, i1) (0 < i1 - i0 <= kPieceItems, wave-uniform) of a piece: the
// number covering each tile of block tb (lane j: tile j of the block).
__device__ uint32_t piece_tile_counts(const uint32_t *__restrict__ keys, uint32_t i0, uint32_t i1, int log2s,
                                      TileBlock blk, int lane) {
  const int S = 1 << log2s;
  const uint32_t last = i1 - 1u;
  uint32_t k[kPieceItems / 64];
#pragma unroll
  for (int q = 0; q < kPieceItems / 64; q++) k[q] = keys[min(i0 + 64u * q + lane, last)];
  uint32_t cnt = 0;
#pragma unroll
  for (int q = 0; q < kPieceItems / 64; q++) {
    const uint32_t c0 = i0 + 64u * q;
    if (c0 >= i1) break;
    const LocalRect r = key_rect(k[q], log2s, c0 + lane < i1);
    for (int ry = 0; ry < blk.nrows; ry++) {
      const bool rowhit = (uint32_t)(blk.row0 + ry) - r.y0 <= r.wy;
      if (__builtin_amdgcn_ballot_w64(rowhit) == 0ull) continue;
      for (int lx = 0; lx < S; lx++) {
        const uint64_t b = __builtin_amdgcn_ballot_w64(rowhit && (uint32_t)lx - r.x0 <= r.wx);
        if (lane == ry * S + lx) cnt += (uint32_t)__popcll(b);
      }
    }
  }
  return cnt;
}

// The same for super-bins of S = 2^L <= 8 tiles on a side (lane j = tile j):
// per 64-item chunk one ballot per column and per row, and per tile the
// intersection of the two lane masks, counted in scalar registers.
template <int L>
__device__ __forceinline__ uint32_t piece_tile_counts_t(const uint32_t *__restrict__ keys, uint32_t i0, uint32_t i1,
                                                        int lane) {
  constexpr int S = 1 << L, S2 = S * S;
  constexpr uint32_t m = S - 1;
  const uint32_t last = i1 - 1u;
  uint32_t k[kPieceItems / 64];
#pragma unroll
  for (int q = 0; q < kPieceItems / 64; q++) k[q] = keys[min(i0 + 64u * q + lane, last)];
  uint32_t sc[S2];
#pragma unroll
  for (int j = 0; j < S2; j++) sc[j] = 0;
#pragma unroll
  for (int q = 0; q < kPieceItems / 64; q++) {
    const uint32_t c0 = i0 + 64u * q;
    if (c0 < i1) {
      const uint32_t key = k[q];
      const bool valid = c0 + lane < i1;
      const uint32_t x0 = (key >> 8) & m, x1 = (key >> (8 + L)) & m;
      const uint32_t y0 = (key >> (8 + 2 * L)) & m, y1 = (key >> (8 + 3 * L)) & m;
      uint64_t col[S];
#pragma unroll
      for (int c = 0; c < S; c++) col[c] = __builtin_amdgcn_ballot_w64(x0 <= (uint32_t)c && (uint32_t)c <= x1);
#pragma unroll
      for (int r = 0; r < S; r++) {
        const uint64_t row = __builtin_amdgcn_ballot_w64(valid && y0 <= (uint32_t)r && (uint32_t)r <= y1);
        if (row == 0ull) continue;
#pragma unroll
        for (int c = 0; c < S; c++) sc[r * S + c] += (uint32_t)__popcll(col[c] & row);
      }
    }
  }
  uint32_t cnt = 0;
#pragma unroll
  for (int j = 0; j < S2; j++) cnt = lane == j ? sc[j] : cnt;
  return cnt;
}

// Piece p's list items, wave-uniform: [i0, i1) of super-bin sb.
struct Piece {
  int sb;
  uint32_t i0, i1;
};

__device__ __forceinline__ Piece piece_of(const PieceTable &pt, uint32_t p) {
  const int sb = piece_superbin(pt, p);
  const uint32_t i0 = pt.beg[sb] + (p - pt.pf[sb]) * kPieceItems;
  const uint32_t i1 = min(i0 + kPieceItems, pt.end[sb]);
  return Piece{__builtin_amdgcn_readfirstlane(sb), (uint32_t)__builtin_amdgcn_readfirstlane(i0),
               (uint32_t)__builtin_amdgcn_readfirstlane(i1)};
}

// pcnt[p * S^2 + j] = items of piece p covering local tile j of its super-bin.
// L >= 0: super-bins of 2^L tiles on a side (L <= 3); L < 0: any size
// (log2s), tiles in blocks of 64.
template <int L>
__global__ __launch_bounds__(kPieceWaves * 64) void tile_count_kernel(const uint32_t *__restrict__ sb_keys,
                                                                      const uint32_t *__restrict__ sb_tot, int log2s,
                                                                      uint32_t *__restrict__ pcnt) {
  __shared__ PieceTable pt;
  __shared__ uint32_t lds4[4];
  build_piece_table(pt, sb_tot, lds4);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int S2 = 1 << (2 * log2s);
  const uint32_t np = pt.pf[kRadixBins];
  const uint32_t p0 = __builtin_amdgcn_readfirstlane(blockIdx.x * kPieceWaves + w);
  for (uint32_t p = p0; p < np; p += gridDim.x * kPieceWaves) {
    const Piece pc = piece_of(pt, p);
    if constexpr (L >= 0) {
      const uint32_t c = piece_tile_counts_t<L>(sb_keys, pc.i0, pc.i1, lane);
      if (lane < (1 << (2 * L))) pcnt[(size_t)p * (1 << (2 * L)) + lane] = c;
    } else {
      for (int tb = 0; tb < tile_blocks(log2s); tb++) {
        const uint32_t c = piece_tile_counts(sb_keys, pc.i0, pc.i1, log2s, tile_block(log2s, tb), lane);
        const int j = 64 * tb + lane;
        if (j < S2) pcnt[(size_t)p * S2 + j] = c;
      }
    }
  }
}

// One workgroup per super-bin; a wave takes eight tiles at a time (their
// loads in flight together): pcnt becomes, per tile, the count of the
// super-bin's earlier pieces (exclusive scan over the pieces); counts[tile] =
// the tile's total.
__global__ __launch_bounds__(256) void tile_piece_scan_kernel(const uint32_t *__restrict__ sb_tot, int TX, int TY,
                                                              int SX, int log2s, uint32_t *__restrict__ pcnt,
                                                              uint32_t *__restrict__ counts) {
  __shared__ PieceTable pt;
  __shared__ uint32_t lds4[4];
  build_piece_table(pt, sb_tot, lds4);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sb = blockIdx.x, S = 1 << log2s, S2 = S * S;
  const uint32_t P0 = pt.pf[sb], npc = pt.pf[sb + 1] - P0;
  constexpr int G = 8;
  for (int j0 = G * w; j0 < S2; j0 += G * 4) {
    uint32_t carry[G];
#pragma unroll
    for (int g = 0; g < G; g++) carry[g] = 0;
    for (uint32_t k0 = 0; k0 < npc; k0 += 64) {
      const uint32_t k = k0 + lane, kc = min(k, npc - 1u);
      uint32_t v[G];
#pragma unroll
      for (int g = 0; g < G; g++) v[g] = j0 + g < S2 ? pcnt[(size_t)(P0 + kc) * S2 + j0 + g] : 0u;
#pragma unroll
      for (int g = 0; g < G; g++) {
        const uint32_t x = k < npc ? v[g] : 0u;
        const uint32_t inc = wave_inclusive_scan(x, lane);
        if (k < npc && j0 + g < S2) pcnt[(size_t)(P0 + k) * S2 + j0 + g] = carry[g] + inc - x;
        carry[g] += __shfl(inc, 63, 64);
      }
    }
#pragma unroll
    for (int g = 0; g < G; g++) {
      const int j = j0 + g;
      if (j < S2) {
        const int t = tile_of(sb, SX, log2s, j & (S - 1), j >> log2s, TX, TY);
        if (lane == 0 && t >= 0) counts[t] = carry[g];
      }
    }
  }
}

// One block of 1024 threads: tile offsets (exclusive scan of the counts, in
// place, 4096 tiles per step staged through LDS so that global accesses are
// coalesced), the tile ranges, the instance count (the sum of the per-block
// tiles-touched totals: exact also when the super-bin instances overflowed
// the capacity and the counts are incomplete) and the status word.  On
// overflow every range is empty.
constexpr int kTileScanThreads = 1024;

__global__ __launch_bounds__(kTileScanThreads) void tile_scan_kernel(uint32_t *__restrict__ counts, int T,
                                                                     const uint32_t *__restrict__ area_part,
                                                                     int nparts, uint32_t cap,
                                                                     uint32_t *__restrict__ m_out,
                                                                     int32_t *__restrict__ status,
                                                                     uint2 *__restrict__ ranges) {
  constexpr int NT = kTileScanThreads, NW = NT / 64;
  __shared__ uint32_t buf[4 * NT];
  __shared__ uint32_t lds[NW];
  const int t = threadIdx.x;
  uint32_t msum = 0;
  for (int i = t; i < nparts; i += NT) msum += area_part[i];
  uint32_t mtot;
  block_exclusive_scan_w<NW>(msum, lds, mtot);
  const bool over = mtot > cap;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < T; c0 += 4 * NT) {
    uint32_t orig[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int i = c0 + k * NT + t;
      orig[k] = i < T ? counts[i] : 0u;
      buf[k * NT + t] = orig[k];
    }
    __syncthreads();
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = buf[4 * t + k];
    uint32_t total;
    uint32_t ex = block_exclusive_scan_w<NW>((v[0] + v[1]) + (v[2] + v[3]), lds, total);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      buf[4 * t + k] = ex;
      ex += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int i = c0 + k * NT + t;
      if (i < T) {
        const uint32_t o = carry + buf[k * NT + t];
        counts[i] = o;
        ranges[i] = over ? make_uint2(0u, 0u) : make_uint2(o, o + orig[k]);
      }
    }
    carry += total;
    __syncthreads();
  }
  if (t == 0) {
    m_out[0] = mtot;
    status[kStatusMLo] = (int32_t)mtot;
    status[kStatusMHi] = 0;
    status[kStatusFlags] = over ? kFlagOverflow : 0;
  }
}

// Writes piece p's items of super-bin-local tile j at the tile's offset plus
// the piece's prefix plus the item's ballot rank, for super-bins of
// S = 2^L <= 8 tiles on a side: the tiles' output positions are kept in
// scalar registers.
// Marks a loaded value as complete here.  Loads and stores share one
// completion counter; without this the compiler may sink a load into a
// branch and then, where branches merge, wait for every outstanding
// operation (the stores included) before each store.  An empty asm that
// takes the register as input and output makes it wait for the loads once,
// before the stores start.
__device__ __forceinline__ void settle(uint32_t &x) { asm volatile("" : "+v"(x)); }

template <int L>
__device__ __forceinline__ void write_piece_t(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                                              uint32_t i0, uint32_t i1, uint32_t run, int lane,
                                              uint32_t *__restrict__ out_gauss) {
  constexpr int S = 1 << L, S2 = S * S;
  constexpr uint32_t m = S - 1;
  const uint32_t last = i1 - 1u;
  uint32_t k[kPieceItems / 64], v[kPieceItems / 64];
#pragma unroll
  for (int q = 0; q < kPieceItems / 64; q++) {
    const uint32_t i = min(i0 + 64u * q + lane, last);
    k[q] = keys[i];
    v[q] = vals[i];
  }
#pragma unroll
  for (int q = 0; q < kPieceItems / 64; q++) {
    settle(k[q]);
    settle(v[q]);
  }
  uint32_t base[S2];
#pragma unroll
  for (int j = 0; j < S2; j++) base[j] = __builtin_amdgcn_readlane(run, j);
#pragma unroll
  for (int q = 0; q < kPieceItems / 64; q++) {
    const uint32_t c0 = i0 + 64u * q;
    if (c0 < i1) {
      const uint32_t key = k[q];
      const bool valid = c0 + lane < i1;
      const uint32_t x0 = (key >> 8) & m, x1 = (key >> (8 + L)) & m;
      const uint32_t y0 = (key >> (8 + 2 * L)) & m, y1 = (key >> (8 + 3 * L)) & m;
#pragma unroll
      for (int r = 0; r < S; r++) {
        const bool rh = valid && y0 <= (uint32_t)r && (uint32_t)r <= y1;
#pragma unroll
        for (int c = 0; c < S; c++) {
          const bool hit = rh && x0 <= (uint32_t)c && (uint32_t)c <= x1;
          const uint64_t b = __builtin_amdgcn_ballot_w64(hit);
          const uint32_t pos =
              base[r * S + c] + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
          if (hit) out_gauss[pos] = v[q];
          base[r * S + c] += (uint32_t)__popcll(b);
        }
      }
    }
  }
}

template <int L>
__global__ __launch_bounds__(kPieceWaves * 64) void tile_write_kernel(
    const uint32_t *__restrict__ sb_keys, const uint32_t *__restrict__ sb_list, const uint32_t *__restrict__ sb_tot,
    int TX, int TY, int SX, int log2s, const uint32_t *__restrict__ pcnt, const uint32_t *__restrict__ tile_off,
    const uint32_t *__restrict__ m_dev, uint32_t cap, uint32_t *__restrict__ out_gauss) {
  __shared__ PieceTable pt;
  __shared__ uint32_t lds4[4];
  if (m_dev[0] > cap) return;  // overflow: nothing written, the ranges are empty (uniform per launch)
  build_piece_table(pt, sb_tot, lds4);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int S = 1 << log2s, S2 = S * S;
  const uint32_t np = pt.pf[kRadixBins];
  const uint32_t p0 = __builtin_amdgcn_readfirstlane(blockIdx.x * kPieceWaves + w);
  for (uint32_t p = p0; p < np; p += gridDim.x * kPieceWaves) {
    const Piece pc = piece_of(pt, p);
    if constexpr (L >= 0) {
      // lane j: first output position of tile j for this piece
      const int tj = lane < S2 ? tile_of(pc.sb, SX, L, lane & (S - 1), lane >> L, TX, TY) : -1;
      const uint32_t run = tj >= 0 ? tile_off[tj] + pcnt[(size_t)p * S2 + lane] : 0u;
      write_piece_t<L>(sb_keys, sb_list, pc.i0, pc.i1, run, lane, out_gauss);
      continue;
    }
    const uint32_t last = pc.i1 - 1u;
    uint32_t kv[kPieceItems / 64], vv[kPieceItems / 64];
#pragma unroll
    for (int q = 0; q < kPieceItems / 64; q++) {
      const uint32_t i = min(pc.i0 + 64u * q + lane, last);
      kv[q] = sb_keys[i];
      vv[q] = sb_list[i];
    }
#pragma unroll
    for (int q = 0; q < kPieceItems / 64; q++) {
      settle(kv[q]);
      settle(vv[q]);
    }
    for (int tb = 0; tb < tile_blocks(log2s); tb++) {
      const TileBlock blk = tile_block(log2s, tb);
      // lane j: next output position of tile j of the block
      const int j = 64 * tb + lane;
      const int tj = j < S2 ? tile_of(pc.sb, SX, log2s, j & (S - 1), j >> log2s, TX, TY) : -1;
      uint32_t run = tj >= 0 ? tile_off[tj] + pcnt[(size_t)p * S2 + j] : 0u;
#pragma unroll
      for (int q = 0; q < kPieceItems / 64; q++) {
        const uint32_t c0 = pc.i0 + 64u * q;
        if (c0 >= pc.i1) break;
        const LocalRect r = key_rect(kv[q], log2s, c0 + lane < pc.i1);
        for (int ry = 0; ry < blk.nrows; ry++) {
          const bool rowhit = (uint32_t)(blk.row0 + ry) - r.y0 <= r.wy;
          if (__builtin_amdgcn_ballot_w64(rowhit) == 0ull) continue;
          for (int lx = 0; lx < S; lx++) {
            const bool hit = rowhit && (uint32_t)lx - r.x0 <= r.wx;
            const uint64_t b = __builtin_amdgcn_ballot_w64(hit);
            if (b == 0ull) continue;
            const int jj = ry * S + lx;  // lane of the tile in this block
            const uint32_t base = __builtin_amdgcn_readlane(run, jj);
            if (hit) {
              const uint32_t rank =
                  __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
              out_gauss[base + rank] = vv[q];
            }
            if (lane == jj) run += (uint32_t)__popcll(b);
          }
        }
      }
    }
  }
}


// ------------------------------------------------------------------ host side

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

constexpr uint32_t kScanSumBlocks = 4096;  // up to this many blocks a scan skips the partials pass
constexpr uint32_t kRadixLocalBlocks = 256;  // up to this many blocks a pass without totals skips the column scan

// Exclusive scan of n (host-known bound) u32 values; total written to
// total_dev.  have_partials: partials already holds the block sums (blocks of
// kScanItems values).
void launch_scan(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *partials, uint32_t *total_dev,
                 hipStream_t st, bool have_partials) {
  const uint32_t nb = n ? cdiv(n, kScanItems) : 1;
  if (!have_partials) scan_reduce_kernel<<<nb, kScanThreads, 0, st>>>(in, n, partials);
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

// One stable 8-bit pass (keys/vals in -> out) over min(n_host, *n_dev) items;
// tot receives the 256 digit totals.
void launch_radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, uint32_t n_host,
                       const uint32_t *n_dev, int shift, uint32_t *hist, uint32_t *tot, bool want_tot,
                       hipStream_t st) {
  const uint32_t nb = radix_blocks(n_host);
  radix_hist_kernel<<<nb, kHistThreads, 0, st>>>(kin, n_host, n_dev, shift, hist);
  if (!want_tot && !n_dev && nb <= kRadixLocalBlocks) {
    // few blocks: each scatter block sums the block counts itself
    radix_scatter_kernel<true><<<nb, kScatterThreads, 0, st>>>(kin, vin, kout, vout, n_host, n_dev, shift, hist, tot);
    return;
  }
  radix_colscan_kernel<<<kRadixBins, kSortThreads, 0, st>>>(hist, n_host, n_dev, tot);
  radix_scatter_kernel<false><<<nb, kScatterThreads, 0, st>>>(kin, vin, kout, vout, n_host, n_dev, shift, hist, tot);
}

int superbin_log2(int TX, int TY) {
  int l = 0;
  while ((uint64_t)cdiv(TX, 1u << l) * cdiv(TY, 1u << l) > (uint64_t)kRadixBins) l++;
  return l;
}

// The super-bin key packs 8 bits of super-bin and four log2s-bit coordinates.
bool superbin_supported(int TX, int TY) { return superbin_log2(TX, TY) <= kMaxSuperbinLog2; }

uint32_t area_parts(uint32_t n) { return n ? cdiv(n, kScanItems) : 1; }

void launch_superbin_expand(const uint32_t *sorted_g, const ushort4 *rects, uint32_t n, uint32_t cap, int TX, int TY,
                            uint32_t *tt, uint32_t *offs, uint32_t *ka, uint32_t *va, uint32_t *partials,
                            uint32_t *ms_dev, uint32_t *area_part, hipStream_t st) {
  const int log2s = superbin_log2(TX, TY);
  const int SX = (int)cdiv(TX, 1u << log2s);
  if (n) gather_tiles_kernel<<<cdiv(n, kScanItems), kScanThreads, 0, st>>>(sorted_g, rects, n, log2s, tt, partials,
                                                                          area_part);
  else zero_u32_kernel<<<1, 1, 0, st>>>(area_part);
  launch_scan(tt, offs, n, partials, ms_dev, st, n > 0);
  if (n) emit_kernel<<<cdiv(n, 256), 256, 0, st>>>(sorted_g, rects, offs, n, cap, SX, log2s, ka, va);
}

static uint32_t piece_bound(uint32_t cap) { return cap / kPieceItems + kRadixBins; }

size_t tile_piece_words(int TX, int TY, uint32_t cap) {
  return (size_t)piece_bound(cap) << (2 * superbin_log2(TX, TY));
}

void launch_tile_lists(uint32_t n, uint32_t cap, int TX, int TY, uint32_t *ka, uint32_t *va, uint32_t *kb,
                       uint32_t *vb, uint32_t *counts, uint32_t *pcnt, uint32_t *hist, uint32_t *tot,
                       const uint32_t *ms_dev, const uint32_t *area_part, uint32_t *m_out, int32_t *status,
                       uint2 *ranges, hipStream_t st) {
  const int log2s = superbin_log2(TX, TY);
  const int SX = (int)cdiv(TX, 1u << log2s), SY = (int)cdiv(TY, 1u << log2s);
  const int T = TX * TY;
  // one stable 8-bit pass: super-bin-major, depth order within each super-bin;
  // tot = the super-bin list lengths
  launch_radix_pass(ka, va, kb, vb, cap, ms_dev, 0, hist, tot, true, st);
  const uint32_t gp = cdiv(piece_bound(cap), kPieceWaves), grid = gp < (uint32_t)kPieceGrid ? gp : (uint32_t)kPieceGrid;
  const dim3 gb(grid), bb(kPieceWaves * 64);
  switch (log2s) {
    case 0: tile_count_kernel<0><<<gb, bb, 0, st>>>(kb, tot, log2s, pcnt); break;
    case 1: tile_count_kernel<1><<<gb, bb, 0, st>>>(kb, tot, log2s, pcnt); break;
    case 2: tile_count_kernel<2><<<gb, bb, 0, st>>>(kb, tot, log2s, pcnt); break;
    case 3: tile_count_kernel<3><<<gb, bb, 0, st>>>(kb, tot, log2s, pcnt); break;
    default: tile_count_kernel<-1><<<gb, bb, 0, st>>>(kb, tot, log2s, pcnt); break;
  }
  tile_piece_scan_kernel<<<SX * SY, 256, 0, st>>>(tot, TX, TY, SX, log2s, pcnt, counts);
  tile_scan_kernel<<<1, kTileScanThreads, 0, st>>>(counts, T, area_part, (int)area_parts(n), cap, m_out, status,
                                                 ranges);
#define SSSGS_TILE_WRITE(LL) \
  tile_write_kernel<LL><<<gb, bb, 0, st>>>(kb, vb, tot, TX, TY, SX, log2s, pcnt, counts, m_out, cap, va)
  switch (log2s) {
    case 0: SSSGS_TILE_WRITE(0); break;
    case 1: SSSGS_TILE_WRITE(1); break;
    case 2: SSSGS_TILE_WRITE(2); break;
    case 3: SSSGS_TILE_WRITE(3); break;
    default: SSSGS_TILE_WRITE(-1); break;
  }
#undef SSSGS_TILE_WRITE
}



}  // namespace sssgs
