// common.hpp -- shared definitions of the gfx950 kernels behind libsssgs.so.
// The CPU oracle shares nothing with this file.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sssgs {

constexpr int kTile = 16;            // 16x16 pixel tiles
constexpr int kTilePix = kTile * kTile;
constexpr int kChAlb = 0, kChNrm = 3, kChRough = 6, kChMetal = 7, kChSss = 8, kChDepth = 9, kChFeat = 10;
constexpr int kNumPE = 36;           // 6 octaves x {sin, cos} x 3 axes
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;                     // keys per thread per radix block
constexpr int kSortItems = kSortThreads * kSortRounds;
constexpr int kMaxSuperbinLog2 = 6;              // super-bins of up to 64 x 64 tiles
constexpr int kScanThreads = 256;
constexpr int kScanItems = kScanThreads * 4;

// Floats per splat record: u, v, conic (a, b, c), opacity, C channels; padded to 16 B.
__host__ __device__ constexpr int rec_stride(int C) { return (6 + C + 3) / 4 * 4; }
// Per-Gaussian gradient accumulator: du dv dA dB dC dopacity | dchannels, padded to 16 B.
__host__ __device__ constexpr int grad_stride(int C) { return (6 + C + 3) / 4 * 4; }

struct CamArgs {
  float R[9], t[3], fx, fy, cx, cy;
  int W, H, TX, TY;
  float Cw[3];   // camera centre in world space
};

struct LightArgs {
  float pos[3], intensity[3];
};

// Work item of block b in a grid of G blocks such that the blocks one XCD
// runs take consecutive items.  The hardware deals workgroups to the eight
// XCDs round-robin (block b to XCD b mod 8), and each XCD has its own L2:
// with consecutive tiles on one XCD, the two tiles that share a 128-byte
// line of a planar per-pixel array are fetched into one L2, not two.  A
// bijection on [0, G): XCD x runs G/8 blocks (one more for x < G mod 8).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_item(int b, int G) {
  const int per = G / kXcds, rem = G % kXcds, x = b % kXcds, k = b / kXcds;
  return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void st4(float *p, float4 v) { *reinterpret_cast<float4 *>(p) = v; }

// Splat power at a pixel: -0.5 (a dx^2 + c dy^2) - b dx dy with dx = u - px.
// The operation sequence is pinned so that forward and backward kernels take
// bit-identical decisions.
__device__ __forceinline__ float splat_power(float u, float v, float ca, float cb, float cc, float px, float py,
                                             float &dx, float &dy) {
  dx = u - px;
  dy = v - py;
  float q = __fmul_rn(ca, __fmul_rn(dx, dx));
  q = __fmaf_rn(cc, __fmul_rn(dy, dy), q);
  return __fmaf_rn(-0.5f, q, -__fmul_rn(cb, __fmul_rn(dx, dy)));
}

// exp via the hardware exp2 (v_exp_f32) with a folded log2(e).
__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(__fmul_rn(x, 1.44269504088896341f)); }

__device__ __forceinline__ float splat_alpha_raw(float opacity, float power) { return __fmul_rn(opacity, fast_exp(power)); }

// Deterministic per-Gaussian gradient sums of the compositing backward: one
// slot per (Gaussian, tile of its rectangle); the slots of Gaussian i are
// toff[i] .. toff[i] + area(i) - 1 in row-major tile order.  slots == null:
// the sums are added with atomics instead.
struct DetSlots {
  float *slots;          // [instances][grad_stride(C)]
  uint8_t *flags;        // [instances]: 1 where a tile wrote the slot
  const ushort4 *rects;  // [n] tile rectangles x0, y0, x1, y1
  const uint32_t *toff;  // [n] first slot of each Gaussian
  size_t cap;            // slots available (the instance capacity): after an
                         // overflowed forward, slots beyond it are skipped
};

__device__ __forceinline__ size_t det_slot(const DetSlots &d, uint32_t i, int tx, int ty) {
  const ushort4 r = d.rects[i];
  return (size_t)d.toff[i] + (size_t)(ty - (int)r.y) * (size_t)(r.z - r.x) + (size_t)(tx - (int)r.x);
}

// Status word layout in the workspace.
constexpr int kStatusFlags = 0, kStatusMLo = 1, kStatusMHi = 2;
constexpr int kFlagOverflow = 1;

}  // namespace sssgs
