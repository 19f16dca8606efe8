// mlp_prep.hip -- conversion of the packed network parameters into per-lane
// matrix-core operands (forward: W with permuted K; backward: W^T with
// permuted K), the deterministic reduction of per-block weight gradients, and
// the L1 image loss of the training objective (Appendix "Losses").
#include "launch.hpp"
#include "shade_common.hpp"

namespace sssgs {

// Forward operands: layer l, 16-row block mb, k-step ks, lane -> W[row][feat].
// NATURAL: every layer's K in natural order (inputs read from LDS rows);
// otherwise layers >= 1 in the permuted order of the accumulator layout.
template <class M, int WIDTH, int IN_PAD, bool NATURAL>
__device__ __forceinline__ void prep_fwd_op(const float *__restrict__ params, typename M::Op *wops, int idx) {
  using NS = NetShape<M, WIDTH, IN_PAD>;
  using PO = ParamOffsets<WIDTH, IN_PAD>;
  if (idx >= NS::total_ops(3)) return;
  int layer, local;
  if (idx < NS::L0) {
    layer = 0; local = idx;
  } else if (idx < NS::L0 + 2 * NS::LH) {
    layer = 1 + (idx - NS::L0) / NS::LH; local = (idx - NS::L0) % NS::LH;
  } else {
    layer = 3; local = idx - NS::L0 - 2 * NS::LH;
  }
  const int ksn = layer == 0 ? NS::KS0 : NS::KSH;
  const int lane = local % 64, t = local / 64, ks = t % ksn, mb = t / ksn;
  const int row = 16 * mb + (lane & 15), g = lane >> 4;
  const float *W = params + PO::w(layer);
  const int rows = PO::rows(layer), cols = PO::cols(layer);
  typename M::Op o;
  if constexpr (M::KPL == 8) {
    for (int j = 0; j < 8; j++) {
      const int f = feat_index<M>(NATURAL || layer == 0, ks, g, j);
      o[j] = (__bf16)((row < rows && f < cols) ? W[row * cols + f] : 0.f);
    }
  } else {
    const int f = feat_index<M>(NATURAL || layer == 0, ks, g, 0);
    o = (row < rows && f < cols) ? W[row * cols + f] : 0.f;
  }
  wops[idx] = o;
}

// Backward operands of dX^T = W^T dY^T: M = the layer's input features
// (16-row blocks mb), K = the layer's output features in the permuted order
// of the accumulator layout.
template <class M, int WIDTH, int IN_PAD>
__device__ __forceinline__ void prep_bwd_op(const float *__restrict__ params, typename M::Op *tops, int idx) {
  using NS = NetShape<M, WIDTH, IN_PAD>;
  using PO = ParamOffsets<WIDTH, IN_PAD>;
  if (idx >= NS::total_tops(3)) return;
  int layer, local;
  if (idx < NS::T0) {
    layer = 0; local = idx;
  } else if (idx < NS::T0 + 2 * NS::TH) {
    layer = 1 + (idx - NS::T0) / NS::TH; local = (idx - NS::T0) % NS::TH;
  } else {
    layer = 3; local = idx - NS::T0 - 2 * NS::TH;
  }
  const int ktn = layer == 3 ? NS::KT_O : NS::KT_H;
  const int lane = local % 64, t = local / 64, ks = t % ktn, mb = t / ktn;
  const int colf = 16 * mb + (lane & 15), g = lane >> 4;  // input feature of the forward layer
  const float *W = params + PO::w(layer);
  const int rows = PO::rows(layer), cols = PO::cols(layer);
  typename M::Op o;
  if constexpr (M::KPL == 8) {
    for (int j = 0; j < 8; j++) {
      const int r = feat_index<M>(false, ks, g, j);
      o[j] = (__bf16)((r < rows && colf < cols) ? W[r * cols + colf] : 0.f);
    }
  } else {
    const int r = feat_index<M>(false, ks, g, 0);
    o = (r < rows && colf < cols) ? W[r * cols + colf] : 0.f;
  }
  tops[idx] = o;
}

// All requested operand sets in one launch: blocks [0, bw) write wops,
// [bw, bw + bn) nops, the rest tops (bw, bn = 0 for a set not requested).
template <class M, int WIDTH, int IN_PAD>
__global__ __launch_bounds__(256) void prep_kernel(const float *__restrict__ params, typename M::Op *wops,
                                                   typename M::Op *nops, typename M::Op *tops, int bw, int bn) {
  const int b = blockIdx.x;
  if (b < bw) prep_fwd_op<M, WIDTH, IN_PAD, false>(params, wops, b * 256 + threadIdx.x);
  else if (b < bw + bn) prep_fwd_op<M, WIDTH, IN_PAD, true>(params, nops, (b - bw) * 256 + threadIdx.x);
  else prep_bwd_op<M, WIDTH, IN_PAD>(params, tops, (b - bw - bn) * 256 + threadIdx.x);
}

template <class M, int WIDTH, int IN_PAD>
static void prep_t(const float *params, void *wops, void *tops, void *nops, hipStream_t st) {
  using NS = NetShape<M, WIDTH, IN_PAD>;
  using Op = typename M::Op;
  const int cf = (NS::total_ops(3) + 255) / 256, cb = (NS::total_tops(3) + 255) / 256;
  const int bw = wops ? cf : 0, bn = nops ? cf : 0, bt = tops ? cb : 0;
  if (bw + bn + bt == 0) return;
  prep_kernel<M, WIDTH, IN_PAD><<<bw + bn + bt, 256, 0, st>>>(params, (Op *)wops, (Op *)nops, (Op *)tops, bw, bn);
}

void launch_prep_weights(int net, int width, int in_pad, const float *params, void *wops, void *tops, void *nops,
                         hipStream_t st) {
  if (net == 1) {
    if (width == 64 && in_pad == 64) prep_t<MmaF32, 64, 64>(params, wops, tops, nops, st);
    else if (width == 64 && in_pad == 96) prep_t<MmaF32, 64, 96>(params, wops, tops, nops, st);
  } else if (net == 2) {
    if (width == 64 && in_pad == 64) prep_t<MmaBF16, 64, 64>(params, wops, tops, nops, st);
    else if (width == 64 && in_pad == 96) prep_t<MmaBF16, 64, 96>(params, wops, tops, nops, st);
    else if (width == 128 && in_pad == 64) prep_t<MmaBF16, 128, 64>(params, wops, tops, nops, st);
    else if (width == 128 && in_pad == 96) prep_t<MmaBF16, 128, 96>(params, wops, tops, nops, st);
  }
}

// Bytes for either operand set (FP32 elements; the BF16 set is half).
size_t prep_weight_bytes(int width, int in_pad) {
  const size_t rows = (size_t)width;
  const size_t elems_fwd = rows * in_pad + 2 * rows * width + 16 * (size_t)width;
  const size_t elems_bwd = (size_t)in_pad * width + 2 * (size_t)width * width + (size_t)width * 32;
  return 4 * (elems_fwd > elems_bwd ? elems_fwd : elems_bwd);
}

// Deterministic sum of per-block partials in one pass: a 1024-thread block
// takes 64 parameters; each of its 16 waves sums a contiguous sixteenth of
// the partials for them (a wave reads 256 contiguous bytes of a partial row,
// eight rows in flight), and the sixteen sums are added in a fixed pairwise
// order.
constexpr int kRedParams = 64, kRedGroups = 16;

__global__ __launch_bounds__(kRedParams * kRedGroups) void reduce_partials_kernel(const float *__restrict__ partials,
                                                                                   int nparts, int nparams,
                                                                                   float *__restrict__ out,
                                                                                   int accumulate) {
  __shared__ float q[kRedGroups][kRedParams];
  const int t = threadIdx.x % kRedParams, h = threadIdx.x / kRedParams;
  const int p = blockIdx.x * kRedParams + t;
  const int per = (nparts + kRedGroups - 1) / kRedGroups;
  const int b0 = h * per, b1 = min(nparts, b0 + per);
  float s = 0.f;
  if (p < nparams) {
    int b = b0;
    for (; b + 8 <= b1; b += 8) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; k++) v[k] = partials[(size_t)(b + k) * nparams + p];
#pragma unroll
      for (int k = 0; k < 8; k++) s += v[k];
    }
    for (; b < b1; b++) s += partials[(size_t)b * nparams + p];
  }
  q[h][t] = s;
  __syncthreads();
  for (int w = kRedGroups / 2; w >= 1; w >>= 1) {
    if (h < w) q[h][t] += q[h + w][t];
    __syncthreads();
  }
  if (h == 0 && p < nparams) out[p] = accumulate ? out[p] + q[0][t] : q[0][t];
}

// `scratch` is not used by the one-pass sum (kept for the workspace layout).
void launch_reduce_partials(const float *partials, int nparts, int nparams, float *scratch, float *out,
                            int accumulate, hipStream_t st) {
  (void)scratch;
  reduce_partials_kernel<<<(nparams + kRedParams - 1) / kRedParams, kRedParams * kRedGroups, 0, st>>>(
      partials, nparts, nparams, out, accumulate);
}

int reduce_scratch_floats(int) { return 0; }  // the one-pass sum needs no scratch

__global__ __launch_bounds__(256) void l1_kernel(const float *__restrict__ pred, const float *__restrict__ target,
                                                 int64_t count, float scale, float *__restrict__ loss_out,
                                                 float *__restrict__ grad) {
  __shared__ float red[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < count) {
    const float d = pred[i] - target[i];
    l = fabsf(d) * scale;
    if (grad) grad[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
  }
  for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0 && loss_out) atomicAdd(loss_out, (red[0] + red[1]) + (red[2] + red[3]));
}

void launch_l1_loss(const float *pred, const float *target, int64_t count, float scale, float *loss_out,
                    float *grad, hipStream_t st) {
  if (count <= 0) return;
  l1_kernel<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(pred, target, count, scale, loss_out, grad);
}

__global__ __launch_bounds__(256) void zero_f32_kernel(float *__restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

void launch_zero_f32(float *p, size_t n, hipStream_t st) {
  if (n) zero_f32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n);
}

}  // namespace sssgs
