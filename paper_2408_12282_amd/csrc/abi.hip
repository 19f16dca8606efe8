// abi.hip -- the C ABI of libsssgs.so (include/sssgs.h): argument checks,
// workspace layout and the sequence of kernel launches on the caller's stream.
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "sssgs.h"
#include <algorithm>
#include <cmath>
#include "launch.hpp"
#include "shade_common.hpp"

using namespace sssgs;

namespace {

thread_local std::string g_last_error;

// ---- optional per-stage timing with HIP events on the caller's stream
enum Stage {
  kStProject = 0, kStSortDepth, kStExpand, kStSortTiles, kStCompositeFwd, kStShadeFwd,
  kStShadeBwd, kStMlpWgrad, kStMlpReduce, kStCompositeBwd, kStProjectBwd, kStGmlpFwd, kStGmlpBwd, kStVisibility, kStCount
};
const char *kStageNames[kStCount] = {"project_fwd", "sort_depth", "expand",        "sort_tiles",
                                     "composite_fwd", "shade_fwd", "shade_bwd",     "mlp_wgrad",
                                     "mlp_reduce",  "composite_bwd", "project_bwd", "gmlp_fwd", "gmlp_bwd",
                                     "visibility"};
struct TimerRec {
  int stage;
  hipEvent_t a, b;
};
struct Timer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<TimerRec> recs;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Timer g_timer;

struct Scope {
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Scope(int s, hipStream_t stream) : stage(s), st(stream) {
    if (g_timer.on) {
      a = g_timer.get();
      if (a && hipEventRecord(a, st) != hipSuccess) a = nullptr;  // timing is best effort
    }
  }
  ~Scope() {
    if (g_timer.on && a) {
      hipEvent_t b = g_timer.get();
      if (b && hipEventRecord(b, st) == hipSuccess) g_timer.recs.push_back({stage, a, b});
    }
  }
};

sssgs_status fail(sssgs_status s, const char *msg) {
  g_last_error = msg;
  return s;
}

sssgs_status check_hip(const char *where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return SSSGS_ERR_HIP;
  }
  return SSSGS_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int in_pad_of(int in_dim) { return (in_dim + 31) / 32 * 32; }

struct Layout {
  size_t records, depth_keys, vals_a, keys_b, vals_b, keys_a, rects, radii, boxes, tt, offsets, partials, hist;
  size_t ik_a, iv_a, ik_b, iv_b, ranges, tcount, tpcnt, dtot, apart, t_final, tile_top, tile_order, n_contrib, status, m_total;
  size_t gacc, slots, sflags, dG, dT, wops, tops, nops, mlp_part, mlp_mid, rec_x, rec_o, gx, gdy;
  size_t total;
  int C, RS, GS, TX, TY, T;
  uint32_t nb_g, nb_i;
  int parts, nparams;
};

bool make_layout(int32_t n, int32_t W, int32_t H, int32_t F, int32_t mlp_width, int64_t cap, Layout &L) {
  if (n < 0 || W <= 0 || H <= 0 || cap < 0 || cap >= (int64_t(1) << 31)) return false;
  if (!(F == 0 || F == 8 || F == 16 || F == 32)) return false;
  if (!(mlp_width == 0 || mlp_width == 64 || mlp_width == 128)) return false;
  if (W > 16 * 65535 || H > 16 * 65535) return false;
  L.C = kChFeat + F;
  L.RS = rec_stride(L.C);
  L.GS = grad_stride(L.C);
  L.TX = (W + kTile - 1) / kTile;
  L.TY = (H + kTile - 1) / kTile;
  L.T = L.TX * L.TY;
  if (!superbin_supported(L.TX, L.TY)) return false;
  L.nb_g = radix_blocks((uint64_t)n);
  L.nb_i = radix_blocks((uint64_t)cap);
  const uint32_t nbmax = L.nb_g > L.nb_i ? L.nb_g : L.nb_i;
  const size_t nn = (size_t)(n > 0 ? n : 1), HW = (size_t)W * H, cc = (size_t)(cap > 0 ? cap : 1);
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t o = p;
    p = align256(p + bytes);
    return o;
  };
  L.records = take(nn * L.RS * 4);
  L.depth_keys = take(nn * 4);
  L.vals_a = take(nn * 4);
  L.keys_a = take(nn * 4);
  L.keys_b = take(nn * 4);
  L.vals_b = take(nn * 4);
  L.rects = take(nn * 8);
  L.radii = take(nn * 4);
  L.boxes = take(nn * 8);
  L.tt = take(nn * 4);
  L.offsets = take(nn * 4);
  size_t np = scan_partials_needed(nn);
  const size_t np2 = scan_partials_needed((uint64_t)nbmax * kRadixBins);
  if (np2 > np) np = np2;
  L.partials = take(np * 4);
  L.hist = take((size_t)nbmax * kRadixBins * 4);
  L.tcount = take((size_t)L.T * 4);
  L.tpcnt = take(tile_piece_words(L.TX, L.TY, (uint32_t)cc) * 4);
  L.dtot = take(kRadixBins * 4);  // digit totals of a radix pass
  L.apart = take((size_t)area_parts((uint32_t)nn) * 4);
  L.ik_a = take(cc * 4);
  L.iv_a = take(cc * 4);
  L.ik_b = take(cc * 4);
  L.iv_b = take(cc * 4);
  L.ranges = take((size_t)L.T * 8);
  L.t_final = take(HW * 4);
  L.tile_top = take((size_t)L.T * 4);
  L.tile_order = take((size_t)L.T * 4);
  L.n_contrib = take(HW * 4);
  L.status = take(16);
  L.m_total = take(16);
  L.gacc = take(nn * L.GS * 4);
  // deterministic per-Gaussian sums: one slot per tile instance, and its flag
  L.slots = take(cc * L.GS * 4);
  L.sflags = take((cc + 3) / 4 * 4);
  L.dG = take(HW * L.C * 4);
  L.dT = take(HW * 4);
  const int in_pad = in_pad_of(F + kNumPE + 6);
  L.nparams = mlp_width ? (int)sssgs_mlp_param_count(F + kNumPE + 6, mlp_width, 3, 6) : 0;
  const size_t nstrips = (size_t)L.T * 4, P = nstrips * 64;
  // one weight-gradient partial row per workgroup of the weight kernels
  L.parts = mlp_width ? std::max(mlp_wgrad_grid((int)nstrips), wgrad_gemm_splits(P)) : 0;
  L.wops = take(mlp_width ? prep_weight_bytes(mlp_width, in_pad) : 0);
  L.tops = take(mlp_width ? prep_weight_bytes(mlp_width, in_pad) : 0);
  L.nops = take(mlp_width ? prep_weight_bytes(mlp_width, in_pad) : 0);
  L.mlp_part = take(mlp_width ? (size_t)L.parts * L.nparams * 4 : 0);
  L.mlp_mid = take(mlp_width ? (size_t)reduce_scratch_floats(L.nparams) * 4 : 0);
  // strip records of the split shading backward (BF16 network, width 64, input width 64)
  const bool split = mlp_width == 64 && in_pad == 64;
  L.rec_x = take(split ? nstrips * 64 * 2 * 64 * 2 : 0);  // BF16 values and remainders
  L.rec_o = take(split ? nstrips * 64 * 8 * 2 : 0);
  // weight-gradient operands of the generic network backward (X_l, dY_l per
  // pixel; FP32 where an FP32 network of this width exists, else BF16)
  const size_t esz = mlp_width == 64 ? 4 : 2;
  const size_t xe = (size_t)in_pad + 3 * (size_t)mlp_width, ye = 3 * (size_t)mlp_width + 8;
  L.gx = take(mlp_width ? P * xe * esz : 0);
  L.gdy = take(mlp_width ? P * ye * esz : 0);
  L.total = p;
  return true;
}

CamArgs cam_args(const sssgs_camera *c, const Layout &L) {
  CamArgs a;
  for (int k = 0; k < 9; k++) a.R[k] = c->R[k];
  for (int k = 0; k < 3; k++) a.t[k] = c->t[k];
  a.fx = c->fx; a.fy = c->fy; a.cx = c->cx; a.cy = c->cy;
  a.W = c->width; a.H = c->height; a.TX = L.TX; a.TY = L.TY;
  for (int k = 0; k < 3; k++)
    a.Cw[k] = (float)(-((double)c->R[k] * c->t[0] + (double)c->R[3 + k] * c->t[1] + (double)c->R[6 + k] * c->t[2]));
  return a;
}

template <class T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

sssgs_status check_common(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                          const sssgs_mlp *mlp, const sssgs_options *opt, void *ws, int &net, int &width) {
  if (!g || !cam || !light || !opt || !ws) return fail(SSSGS_ERR_INVALID_ARG, "null argument");
  if (g->n < 0) return fail(SSSGS_ERR_INVALID_ARG, "n < 0");
  if (cam->width <= 0 || cam->height <= 0) return fail(SSSGS_ERR_INVALID_ARG, "image size must be >= 1");
  if (!(cam->fx > 0.f) || !(cam->fy > 0.f)) return fail(SSSGS_ERR_INVALID_ARG, "focal lengths must be > 0");
  if (!(g->feat_dim == 0 || g->feat_dim == 8 || g->feat_dim == 16 || g->feat_dim == 32))
    return fail(SSSGS_ERR_UNSUPPORTED, "feat_dim must be 0, 8, 16 or 32");
  if (!(g->sh_degree == -1 || g->sh_degree == 3)) return fail(SSSGS_ERR_UNSUPPORTED, "sh_degree must be -1 or 3");
  if (g->n > 0) {
    if (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->roughness || !g->metallic || !g->sss)
      return fail(SSSGS_ERR_INVALID_ARG, "null Gaussian parameter plane");
    if (g->sh_degree < 0 && !g->albedo) return fail(SSSGS_ERR_INVALID_ARG, "null albedo");
    if (g->sh_degree == 3 && !g->sh) return fail(SSSGS_ERR_INVALID_ARG, "null sh");
    if (g->feat_dim > 0 && !g->features) return fail(SSSGS_ERR_INVALID_ARG, "null features");
  }
  if (!(opt->precision == SSSGS_PREC_FP32 || opt->precision == SSSGS_PREC_BF16))
    return fail(SSSGS_ERR_INVALID_ARG, "precision must be FP32 or BF16");
  net = 0;
  width = 0;
  if (mlp && mlp->params) {
    if (mlp->hidden != 3 || mlp->out_dim != 6) return fail(SSSGS_ERR_UNSUPPORTED, "network must be 3 hidden layers, 6 outputs");
    if (mlp->in_dim != g->feat_dim + kNumPE + 6) return fail(SSSGS_ERR_INVALID_ARG, "mlp in_dim must equal F + 42");
    if (!(mlp->width == 64 || mlp->width == 128)) return fail(SSSGS_ERR_UNSUPPORTED, "network width must be 64 or 128");
    if (opt->precision == SSSGS_PREC_FP32 && mlp->width != 64)
      return fail(SSSGS_ERR_UNSUPPORTED, "FP32 network supports width 64 only");
    net = opt->precision == SSSGS_PREC_BF16 ? 2 : 1;
    width = mlp->width;
  }
  if (!(opt->radiance_features == 0 || opt->radiance_features == 1))
    return fail(SSSGS_ERR_INVALID_ARG, "radiance_features must be 0 or 1");
  if (opt->radiance_features) {
    if (net) return fail(SSSGS_ERR_INVALID_ARG, "radiance_features excludes the per-pixel network");
    if (g->feat_dim != 8) return fail(SSSGS_ERR_UNSUPPORTED, "radiance_features needs feat_dim 8");
  }
  if (!(opt->deterministic == 0 || opt->deterministic == 1))
    return fail(SSSGS_ERR_INVALID_ARG, "deterministic must be 0 or 1");
  for (int c = 0; c < 3; c++)
    if (!std::isfinite(opt->background[c])) return fail(SSSGS_ERR_INVALID_ARG, "background must be finite");
  return SSSGS_OK;
}

ProjIn proj_in(const sssgs_gaussians *g) {
  ProjIn p;
  p.n = g->n;
  p.means = g->means; p.log_scales = g->log_scales; p.quats = g->quats; p.opacity_logits = g->opacity_logits;
  p.albedo = g->albedo; p.roughness = g->roughness; p.metallic = g->metallic; p.sss = g->sss;
  p.features = g->features; p.sh = g->sh;
  return p;
}

template <int F>
void project_fwd_f(bool sh, const ProjIn &in, const CamArgs &cam, float *rec, uint32_t *k, uint32_t *v, ushort4 *r,
                   int32_t *rad, short4 *box, hipStream_t st) {
  if (sh) launch_project_fwd_t<F, true>(in, cam, rec, k, v, r, rad, box, st);
  else launch_project_fwd_t<F, false>(in, cam, rec, k, v, r, rad, box, st);
}

void project_fwd(int F, bool sh, const ProjIn &in, const CamArgs &cam, float *rec, uint32_t *k, uint32_t *v,
                 ushort4 *r, int32_t *rad, short4 *box, hipStream_t st) {
  switch (F) {
    case 0: project_fwd_f<0>(sh, in, cam, rec, k, v, r, rad, box, st); break;
    case 8: project_fwd_f<8>(sh, in, cam, rec, k, v, r, rad, box, st); break;
    case 16: project_fwd_f<16>(sh, in, cam, rec, k, v, r, rad, box, st); break;
    default: project_fwd_f<32>(sh, in, cam, rec, k, v, r, rad, box, st); break;
  }
}

template <int F>
void project_bwd_f(bool sh, const ProjIn &in, const CamArgs &cam, const float *gacc, const ProjGradOut &o,
                   hipStream_t st) {
  if (sh) launch_project_bwd_t<F, true>(in, cam, gacc, o, st);
  else launch_project_bwd_t<F, false>(in, cam, gacc, o, st);
}

void project_bwd(int F, bool sh, const ProjIn &in, const CamArgs &cam, const float *gacc, const ProjGradOut &o,
                 hipStream_t st) {
  switch (F) {
    case 0: project_bwd_f<0>(sh, in, cam, gacc, o, st); break;
    case 8: project_bwd_f<8>(sh, in, cam, gacc, o, st); break;
    case 16: project_bwd_f<16>(sh, in, cam, gacc, o, st); break;
    default: project_bwd_f<32>(sh, in, cam, gacc, o, st); break;
  }
}

void composite_fwd(int C, const Layout &L, void *ws, int W, int H, float *gbuf, hipStream_t st) {
  uint32_t *top = at<uint32_t>(ws, L.tile_top);
  const uint2 *rg = at<uint2>(ws, L.ranges);
  const uint32_t *sg = at<uint32_t>(ws, L.iv_a);
  const float *rec = at<float>(ws, L.records);
  const short4 *bx = at<short4>(ws, L.boxes);
  float *tf = at<float>(ws, L.t_final);
  uint32_t *nc = at<uint32_t>(ws, L.n_contrib);
  switch (C) {
    case 10: launch_composite_fwd_t<10>(rg, sg, rec, bx, W, H, L.TX, L.TY, gbuf, tf, nc, top, st); break;
    case 18: launch_composite_fwd_t<18>(rg, sg, rec, bx, W, H, L.TX, L.TY, gbuf, tf, nc, top, st); break;
    case 26: launch_composite_fwd_t<26>(rg, sg, rec, bx, W, H, L.TX, L.TY, gbuf, tf, nc, top, st); break;
    default: launch_composite_fwd_t<42>(rg, sg, rec, bx, W, H, L.TX, L.TY, gbuf, tf, nc, top, st); break;
  }
}

void composite_bwd(int C, const Layout &L, void *ws, int W, int H, const DetSlots &det, hipStream_t st) {
  // heaviest tiles first: dispatch order from the forward's per-tile work
  uint32_t *ord = at<uint32_t>(ws, L.tile_order);
  launch_tile_order(at<uint32_t>(ws, L.tile_top), L.T, ord, st);
  const uint2 *rg = at<uint2>(ws, L.ranges);
  const uint32_t *sg = at<uint32_t>(ws, L.iv_a);
  const float *rec = at<float>(ws, L.records);
  const short4 *bx = at<short4>(ws, L.boxes);
  const float *tf = at<float>(ws, L.t_final);
  const uint32_t *nc = at<uint32_t>(ws, L.n_contrib);
  const float *dG = at<float>(ws, L.dG);
  const float *dT = at<float>(ws, L.dT);
  float *ga = at<float>(ws, L.gacc);
  switch (C) {
    case 10: launch_composite_bwd_t<10>(rg, sg, rec, bx, W, H, L.TX, L.TY, tf, nc, dG, dT, ga, det, ord, st); break;
    case 18: launch_composite_bwd_t<18>(rg, sg, rec, bx, W, H, L.TX, L.TY, tf, nc, dG, dT, ga, det, ord, st); break;
    case 26: launch_composite_bwd_t<26>(rg, sg, rec, bx, W, H, L.TX, L.TY, tf, nc, dG, dT, ga, det, ord, st); break;
    default: launch_composite_bwd_t<42>(rg, sg, rec, bx, W, H, L.TX, L.TY, tf, nc, dG, dT, ga, det, ord, st); break;
  }
}

// Dispatch over (F, NET, WIDTH, IN_PAD) for the shading kernels.
template <bool BWD>
bool shade_dispatch(int F, int net, int width, const ShadeArgs &a, hipStream_t st, const MultiLight *ml = nullptr) {
  const int in_pad = in_pad_of(F + kNumPE + 6);
  const int w = (net == 1 || net == 2) ? width : 64;
#define SSSGS_TRY(F_, NET_, W_, P_)                                              \
  if (F == F_ && net == NET_ && w == W_ && in_pad == P_) {                     \
    if constexpr (BWD) launch_shade_bwd_t<F_, NET_, W_, P_>(a, st);            \
    else launch_shade_fwd_t<F_, NET_, W_, P_>(a, *ml, st);                     \
    return true;                                                                \
  }
  SSSGS_SHADE_INSTANCES(SSSGS_TRY)
#undef SSSGS_TRY
  return false;
}

}  // namespace

extern "C" {

int64_t sssgs_mlp_param_count(int32_t in_dim, int32_t width, int32_t hidden, int32_t out_dim) {
  if (in_dim <= 0 || width <= 0 || hidden <= 0 || out_dim <= 0) return 0;
  const int64_t ip = in_pad_of(in_dim);
  return (int64_t)width * ip + width + (int64_t)(hidden - 1) * ((int64_t)width * width + width) +
         (int64_t)out_dim * width + out_dim;
}

size_t sssgs_workspace_bytes(int32_t n, int32_t width, int32_t height, int32_t feat_dim, int32_t mlp_width,
                             int64_t instance_capacity) {
  Layout L;
  if (!make_layout(n, width, height, feat_dim, mlp_width, instance_capacity, L)) return 0;
  return L.total;
}

sssgs_status sssgs_workspace_layout(int32_t n, int32_t width, int32_t height, int32_t feat_dim, int32_t mlp_width,
                                    int64_t instance_capacity, sssgs_layout *out) {
  Layout L;
  if (!out) return fail(SSSGS_ERR_INVALID_ARG, "null layout");
  if (!make_layout(n, width, height, feat_dim, mlp_width, instance_capacity, L))
    return fail(SSSGS_ERR_INVALID_ARG, "bad layout arguments");
  out->records = L.records;
  out->rec_stride = L.RS;
  out->depth_keys = L.depth_keys;
  out->rects = L.rects;
  out->radii = L.radii;
  out->boxes = L.boxes;
  out->tile_ranges = L.ranges;
  out->sorted_gauss = L.iv_a;
  out->t_final = L.t_final;
  out->n_contrib = L.n_contrib;
  out->status = L.status;
  return SSSGS_OK;
}

}  // extern "C"

namespace {

// Forward of one view with nl >= 1 point lights: geometry, binning and
// compositing once, then the shading summed over the lights in passes of up
// to kMaxLights (weights: host [nl][3], null = all ones).
sssgs_status forward_impl(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *lights,
                          const float *weights, int nl, const sssgs_mlp *mlp, const sssgs_options *opt, void *ws,
                          size_t ws_bytes, int64_t cap, float *out_rgb, float *out_gbuffer, float *out_alpha,
                          int64_t *out_num_instances, void *stream) {
  int net, width;
  sssgs_status s = check_common(g, cam, lights, mlp, opt, ws, net, width);
  if (s != SSSGS_OK) return s;
  if (nl < 1) return fail(SSSGS_ERR_INVALID_ARG, "at least one light");
  for (int k = 0; k < nl * 3 && weights; k++)
    if (!std::isfinite(weights[k])) return fail(SSSGS_ERR_INVALID_ARG, "light weights must be finite");
  if (!out_rgb || !out_gbuffer || !out_alpha) return fail(SSSGS_ERR_INVALID_ARG, "null output");
  Layout L;
  if (!make_layout(g->n, cam->width, cam->height, g->feat_dim, width, cap, L))
    return fail(SSSGS_ERR_INVALID_ARG, "bad sizes");
  if (ws_bytes < L.total) return fail(SSSGS_ERR_INVALID_ARG, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  const CamArgs ca = cam_args(cam, L);
  const ProjIn in = proj_in(g);
  const uint32_t n = (uint32_t)g->n, ucap = (uint32_t)cap;
  const int W = cam->width, H = cam->height;
  float *rec = at<float>(ws, L.records);
  uint32_t *dk = at<uint32_t>(ws, L.depth_keys), *ka = at<uint32_t>(ws, L.keys_a), *kb = at<uint32_t>(ws, L.keys_b);
  uint32_t *va = at<uint32_t>(ws, L.vals_a), *vb = at<uint32_t>(ws, L.vals_b);
  ushort4 *rects = at<ushort4>(ws, L.rects);
  uint32_t *hist = at<uint32_t>(ws, L.hist), *part = at<uint32_t>(ws, L.partials);
  uint32_t *mtot = at<uint32_t>(ws, L.m_total);
  int32_t *status = at<int32_t>(ws, L.status);
  // 1. projection (Eq. 1-2): records, depth keys, tile rectangles
  {
    Scope sc(kStProject, st);
    project_fwd(g->feat_dim, g->sh_degree == 3, in, ca, rec, dk, va, rects, at<int32_t>(ws, L.radii),
                at<short4>(ws, L.boxes), st);
  }
  // 2. depth passes of the radix sort on the N Gaussians (stable, index order on ties)
  const uint32_t *kin = dk;
  const uint32_t *vin = va;
  {
    Scope sc(kStSortDepth, st);
    for (int pass = 0; pass < 4; pass++) {
      uint32_t *ko = (pass & 1) ? ka : kb;
      uint32_t *vo = (pass & 1) ? va : vb;
      launch_radix_pass(kin, vin, ko, vo, n, nullptr, pass * kRadixBits, hist, at<uint32_t>(ws, L.dtot), false, st);
      kin = ko;
      vin = vo;
    }
  }
  // sorted Gaussian indices are now in va
  // 3. expansion of the depth-sorted Gaussians into (super-bin, Gaussian)
  // instances; m_total holds [M, super-bin instances]
  uint32_t *tt = at<uint32_t>(ws, L.tt), *offs = at<uint32_t>(ws, L.offsets);
  uint32_t *ik_a = at<uint32_t>(ws, L.ik_a), *iv_a = at<uint32_t>(ws, L.iv_a);
  uint32_t *ik_b = at<uint32_t>(ws, L.ik_b), *iv_b = at<uint32_t>(ws, L.iv_b);
  uint2 *ranges = at<uint2>(ws, L.ranges);
  {
    Scope sc(kStExpand, st);
    launch_superbin_expand(va, rects, n, ucap, L.TX, L.TY, tt, offs, ik_a, iv_a, part, mtot + 1,
                           at<uint32_t>(ws, L.apart), st);
  }
  // 4-5. tile-major Gaussian-index lists, tile ranges, instance count and status
  {
    Scope sc(kStSortTiles, st);
    launch_tile_lists(n, ucap, L.TX, L.TY, ik_a, iv_a, ik_b, iv_b, at<uint32_t>(ws, L.tcount),
                      at<uint32_t>(ws, L.tpcnt), hist, at<uint32_t>(ws, L.dtot),
                      mtot + 1, at<uint32_t>(ws, L.apart), mtot, status, ranges, st);
  }
  // 6. compositing into the G-buffer (Eq. 3)
  {
    Scope sc(kStCompositeFwd, st);
    composite_fwd(L.C, L, ws, W, H, out_gbuffer, st);
  }
  // 7. deferred shading (Eq. 4, 6, 7), summed over the lights
  ShadeArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.cam = ca;
  sa.gbuf = out_gbuffer;
  sa.t_final = at<float>(ws, L.t_final);
  sa.rgb = out_rgb;
  for (int c = 0; c < 3; c++) sa.bgc[c] = opt->background[c];
  sa.alpha = out_alpha;
  if (net) {
    sa.params = mlp->params;
    sa.wops = at<void>(ws, L.wops);
    launch_prep_weights(net, width, in_pad_of(mlp->in_dim), mlp->params, at<void>(ws, L.wops), nullptr, nullptr,
                        st);
  }
  {
    Scope sc(kStShadeFwd, st);
    for (int k0 = 0; k0 < nl; k0 += kMaxLights) {
      MultiLight ml;
      memset(&ml, 0, sizeof(ml));
      ml.K = nl - k0 < kMaxLights ? nl - k0 : kMaxLights;
      ml.accumulate = k0 > 0;
      for (int k = 0; k < ml.K; k++)
        for (int c = 0; c < 3; c++) {
          ml.pos[k][c] = lights[k0 + k].pos[c];
          ml.intensity[k][c] = lights[k0 + k].intensity[c];
          ml.weight[k][c] = weights ? weights[(k0 + k) * 3 + c] : 1.f;
        }
      if (!shade_dispatch<false>(g->feat_dim, opt->radiance_features ? 3 : net, width, sa, st, &ml))
        return fail(SSSGS_ERR_UNSUPPORTED, "no shading kernel for this configuration");
    }
  }
  s = check_hip("forward launch");
  if (s != SSSGS_OK) return s;
  if (out_num_instances) {
    int32_t hs[4];
    if (hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return check_hip("instance count readback");
    *out_num_instances = (int64_t)(uint32_t)hs[kStatusMLo];
    if (hs[kStatusFlags] & kFlagOverflow) return fail(SSSGS_ERR_CAPACITY, "instance capacity exceeded");
  }
  return SSSGS_OK;
}

}  // namespace

extern "C" {

sssgs_status sssgs_render_forward(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                                  const sssgs_mlp *mlp, const sssgs_options *opt, void *ws, size_t ws_bytes,
                                  int64_t cap, float *out_rgb, float *out_gbuffer, float *out_alpha,
                                  int64_t *out_num_instances, void *stream) {
  return forward_impl(g, cam, light, nullptr, 1, mlp, opt, ws, ws_bytes, cap, out_rgb, out_gbuffer, out_alpha,
                      out_num_instances, stream);
}

sssgs_status sssgs_render_forward_lights(const sssgs_gaussians *g, const sssgs_camera *cam,
                                         const sssgs_light *lights, const float *weights, int32_t num_lights,
                                         const sssgs_mlp *mlp, const sssgs_options *opt, void *ws, size_t ws_bytes,
                                         int64_t cap, float *out_rgb, float *out_gbuffer, float *out_alpha,
                                         int64_t *out_num_instances, void *stream) {
  if (!lights || !weights) return fail(SSSGS_ERR_INVALID_ARG, "null lights or weights");
  return forward_impl(g, cam, lights, weights, num_lights, mlp, opt, ws, ws_bytes, cap, out_rgb, out_gbuffer,
                      out_alpha, out_num_instances, stream);
}

sssgs_status sssgs_render_backward(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                                   const sssgs_mlp *mlp, const sssgs_options *opt, void *ws, size_t ws_bytes,
                                   int64_t cap, const float *gbuffer, const float *dL_drgb,
                                   const float *dL_dgbuffer, const float *dL_dalpha, sssgs_gaussian_grads *grads,
                                   float *dL_dmlp, void *stream) {
  int net, width;
  sssgs_status s = check_common(g, cam, light, mlp, opt, ws, net, width);
  if (s != SSSGS_OK) return s;
  if (!gbuffer || !dL_drgb || !grads) return fail(SSSGS_ERR_INVALID_ARG, "null gbuffer, dL_drgb or grads");
  if (!(opt->accumulate_grads == 0 || opt->accumulate_grads == 1))
    return fail(SSSGS_ERR_INVALID_ARG, "accumulate_grads must be 0 or 1");
  Layout L;
  if (!make_layout(g->n, cam->width, cam->height, g->feat_dim, width, cap, L))
    return fail(SSSGS_ERR_INVALID_ARG, "bad sizes");
  if (ws_bytes < L.total) return fail(SSSGS_ERR_INVALID_ARG, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  const CamArgs ca = cam_args(cam, L);
  const int W = cam->width, H = cam->height;
  // 1. shading backward: dL/dG (premultiplied), dL/dT_final, network gradients
  ShadeArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.cam = ca;
  for (int k = 0; k < 3; k++) {
    sa.light.pos[k] = light->pos[k];
    sa.light.intensity[k] = light->intensity[k];
  }
  sa.gbuf = gbuffer;
  sa.t_final = at<float>(ws, L.t_final);
  sa.drgb = dL_drgb;
  sa.dgbuf_ext = dL_dgbuffer;
  sa.dalpha_ext = dL_dalpha;
  sa.dG = at<float>(ws, L.dG);
  sa.dT = at<float>(ws, L.dT);
  for (int c = 0; c < 3; c++) sa.bgc[c] = opt->background[c];
  const int ip = net ? in_pad_of(mlp->in_dim) : 0;
  // BF16 width-64 network with input width 64: the split shading backward and
  // the weight-gradient kernel that recomputes from its strip records; other
  // network forms: the generic backward and the split-K weight contraction
  const bool split = net == 2 && width == 64 && ip == 64;
  if (net) {
    sa.params = mlp->params;
    sa.wops = at<void>(ws, L.wops);
    sa.tops = at<void>(ws, L.tops);
    sa.nops = split ? nullptr : at<void>(ws, L.nops);
    sa.mlp_partials = at<float>(ws, L.mlp_part);
    sa.nparams = L.nparams;
    sa.gx = at<void>(ws, L.gx);
    sa.gdy = at<void>(ws, L.gdy);
    sa.gP = (size_t)L.T * 4 * 64;
    launch_prep_weights(net, width, ip, mlp->params, at<void>(ws, L.wops), at<void>(ws, L.tops),
                        split ? nullptr : at<void>(ws, L.nops), st);
  }
  int parts = 0;
  // the split shading backward clears the compositing accumulators as side
  // work when that is at most 16 float4 stores per thread
  const size_t gacc4 = (size_t)g->n * L.GS / 4;
  const bool fused_zero = split && gacc4 <= (size_t)L.T * 4 * 64 * 16;
  if (fused_zero) {
    sa.zero_buf = at<float4>(ws, L.gacc);
    sa.zero_count4 = gacc4;
  }
  if (split) {
    __bf16 *rx = at<__bf16>(ws, L.rec_x), *ro = at<__bf16>(ws, L.rec_o);
    {
      Scope sc(kStShadeBwd, st);
      switch (g->feat_dim) {
        case 0: launch_shade_bwd_split_t<0, 64>(sa, rx, ro, st); break;
        case 8: launch_shade_bwd_split_t<8, 64>(sa, rx, ro, st); break;
        default: launch_shade_bwd_split_t<16, 64>(sa, rx, ro, st); break;
      }
    }
    if (dL_dmlp) {
      Scope sc(kStMlpWgrad, st);
      launch_mlp_wgrad(sa.wops, sa.tops, sa.params, rx, ro, L.T * 4, sa.mlp_partials, st);
      parts = mlp_wgrad_grid(L.T * 4);
    }
  } else {
    {
      Scope sc(kStShadeBwd, st);
      if (!shade_dispatch<true>(g->feat_dim, opt->radiance_features ? 3 : net, width, sa, st))
        return fail(SSSGS_ERR_UNSUPPORTED, "no shading kernel for this configuration");
    }
    if (net && dL_dmlp) {
      Scope sc(kStMlpWgrad, st);
      launch_wgrad_gemm(net, width, ip, sa.gx, sa.gdy, sa.gP, sa.mlp_partials, st);
      parts = wgrad_gemm_splits(sa.gP);
    }
  }
  if (net && dL_dmlp) {
    Scope sc(kStMlpReduce, st);
    launch_reduce_partials(sa.mlp_partials, parts, L.nparams, at<float>(ws, L.mlp_mid), dL_dmlp,
                           opt->accumulate_grads, st);
  }
  // 2. compositing backward into the per-Gaussian accumulators
  DetSlots det;
  memset(&det, 0, sizeof(det));
  if (opt->deterministic && g->n > 0) {
    // slot offsets: exclusive scan of the tile-rectangle areas; flags cleared
    det.slots = at<float>(ws, L.slots);
    det.flags = at<uint8_t>(ws, L.sflags);
    det.rects = at<ushort4>(ws, L.rects);
    det.toff = at<uint32_t>(ws, L.offsets);
    det.cap = (size_t)cap;
    launch_rect_area(det.rects, (uint32_t)g->n, at<uint32_t>(ws, L.tt), st);
    launch_scan(at<uint32_t>(ws, L.tt), at<uint32_t>(ws, L.offsets), (uint32_t)g->n, at<uint32_t>(ws, L.partials),
                at<uint32_t>(ws, L.status) + 3, st);
    launch_zero_f32(at<float>(ws, L.sflags), (size_t)(cap + 3) / 4, st);
  } else if (!fused_zero) {
    launch_zero_f32(at<float>(ws, L.gacc), (size_t)(g->n) * L.GS, st);
  }
  {
    Scope sc(kStCompositeBwd, st);
    composite_bwd(L.C, L, ws, W, H, det, st);
    if (det.slots) launch_slot_reduce(L.C, det, (uint32_t)g->n, at<float>(ws, L.gacc), st);
  }
  // 3. projection backward
  ProjGradOut go;
  go.means = grads->means; go.log_scales = grads->log_scales; go.quats = grads->quats;
  go.opacity_logits = grads->opacity_logits; go.albedo = grads->albedo; go.roughness = grads->roughness;
  go.metallic = grads->metallic; go.sss = grads->sss; go.features = grads->features; go.sh = grads->sh;
  go.accumulate = opt->accumulate_grads;
  {
    Scope sc(kStProjectBwd, st);
    project_bwd(g->feat_dim, g->sh_degree == 3, proj_in(g), ca, at<float>(ws, L.gacc), go, st);
  }
  return check_hip("backward launch");
}

// ---- per-Gaussian network

int64_t sssgs_gaussian_mlp_param_count(void) { return gmlp_param_count(); }

namespace {
struct GmlpLayout {
  size_t wt, part, mid, act, dz, masks, total;
};
GmlpLayout gmlp_layout(int32_t n) {
  GmlpLayout L;
  const size_t np = (size_t)gmlp_param_count();
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at_ = p;
    p += (bytes + 255) / 256 * 256;
    return at_;
  };
  L.wt = take(np * 4);
  L.part = take((size_t)gmlp_wgrad_grid(n) * np * 4);
  L.mid = take((size_t)reduce_scratch_floats((int)np) * 4);
  L.act = take(gmlp_act_floats(n) * 4);
  L.dz = take(gmlp_dz_floats(n) * 4);
  L.masks = take(gmlp_mask_words(n) * 4);
  L.total = p;
  return L;
}

sssgs_status gmlp_check(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                        const float *visibility, const float *params, void *ws, size_t ws_bytes) {
  if (!g || !cam || !light || !params || !ws) return fail(SSSGS_ERR_INVALID_ARG, "null argument");
  if (g->n < 0) return fail(SSSGS_ERR_INVALID_ARG, "n < 0");
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !visibility))
    return fail(SSSGS_ERR_INVALID_ARG, "null Gaussian plane or visibility");
  if (ws_bytes < gmlp_layout(g->n).total) return fail(SSSGS_ERR_INVALID_ARG, "workspace too small");
  return SSSGS_OK;
}

GmlpArgs gmlp_args(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                   const float *visibility, const float *params, void *ws) {
  GmlpArgs a;
  memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.means = g->means; a.log_scales = g->log_scales; a.quats = g->quats; a.vis = visibility;
  for (int k = 0; k < 3; k++) {
    a.cam[k] = (float)(-((double)cam->R[k] * cam->t[0] + (double)cam->R[3 + k] * cam->t[1] +
                         (double)cam->R[6 + k] * cam->t[2]));
    a.light[k] = light->pos[k];
  }
  a.params = params;
  a.wt = at<float>(ws, gmlp_layout(g->n).wt);
  return a;
}
}  // namespace

size_t sssgs_gaussian_mlp_workspace_bytes(int32_t n) { return n < 0 ? 0 : gmlp_layout(n).total; }

sssgs_status sssgs_gaussian_mlp_forward(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                                        const float *visibility, const float *params, void *ws, size_t ws_bytes,
                                        float *out_features, void *stream) {
  sssgs_status s = gmlp_check(g, cam, light, visibility, params, ws, ws_bytes);
  if (s != SSSGS_OK) return s;
  if (g->n > 0 && !out_features) return fail(SSSGS_ERR_INVALID_ARG, "null out_features");
  hipStream_t st = (hipStream_t)stream;
  GmlpArgs a = gmlp_args(g, cam, light, visibility, params, ws);
  a.feat = out_features;
  const GmlpLayout L = gmlp_layout(g->n);
  a.act = at<float>(ws, L.act);
  a.masks = at<uint32_t>(ws, L.masks);
  a.ldn = gmlp_ldn(g->n);
  Scope sc(kStGmlpFwd, st);
  launch_gmlp_prep(params, at<float>(ws, gmlp_layout(g->n).wt), st);
  launch_gmlp_fwd(a, st);
  return check_hip("gaussian network forward launch");
}

sssgs_status sssgs_gaussian_mlp_backward(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                                         const float *visibility, const float *params, const float *dL_dfeatures,
                                         void *ws, size_t ws_bytes, float *dL_dmeans, float *dL_dlog_scales,
                                         float *dL_dquats, float *dL_dvisibility, float *dL_dparams,
                                         int32_t accumulate, void *stream) {
  sssgs_status s = gmlp_check(g, cam, light, visibility, params, ws, ws_bytes);
  if (s != SSSGS_OK) return s;
  if (!(accumulate == 0 || accumulate == 1)) return fail(SSSGS_ERR_INVALID_ARG, "accumulate must be 0 or 1");
  if (!dL_dparams) return fail(SSSGS_ERR_INVALID_ARG, "null dL_dparams");
  if (g->n > 0 && (!dL_dfeatures || !dL_dmeans || !dL_dlog_scales || !dL_dquats || !dL_dvisibility))
    return fail(SSSGS_ERR_INVALID_ARG, "null gradient array");
  hipStream_t st = (hipStream_t)stream;
  const GmlpLayout L = gmlp_layout(g->n);
  GmlpArgs a = gmlp_args(g, cam, light, visibility, params, ws);
  a.dfeat = dL_dfeatures;
  a.d_means = dL_dmeans; a.d_log_scales = dL_dlog_scales; a.d_quats = dL_dquats; a.d_vis = dL_dvisibility;
  a.partials = at<float>(ws, L.part);
  a.act = at<float>(ws, L.act);
  a.dz = at<float>(ws, L.dz);
  a.masks = at<uint32_t>(ws, L.masks);
  a.ldn = gmlp_ldn(g->n);
  a.accumulate = accumulate;
  Scope sc(kStGmlpBwd, st);
  launch_gmlp_prep(params, at<float>(ws, L.wt), st);
  launch_gmlp_bwd(a, st);
  launch_reduce_partials(a.partials, gmlp_wgrad_grid(g->n), gmlp_param_count(), at<float>(ws, L.mid), dL_dparams,
                         accumulate, st);
  return check_hip("gaussian network backward launch");
}

// ---- ray-traced visibility

namespace {
struct VisLayout {
  size_t rec, scene, bpart, ka, va, kb, vb, hist, part, left, right, rlo, rhi, sbox, b16, bbox, b4k, nbox, nrec, status, total;
};
VisLayout vis_layout(int32_t n) {
  VisLayout L;
  const size_t nn = (size_t)(n > 1 ? n : 2);
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t o = p;
    p = align256(p + bytes);
    return o;
  };
  L.rec = take(nn * 16 * 8);
  L.scene = take(6 * 4);
  L.bpart = take((nn + 255) / 256 * 6 * 4);
  L.ka = take(nn * 4);
  L.va = take(nn * 4);
  L.kb = take(nn * 4);
  L.vb = take(nn * 4);
  const uint32_t nb = radix_blocks((uint64_t)nn);
  size_t np = scan_partials_needed(nn);
  const size_t np2 = scan_partials_needed((uint64_t)nb * kRadixBins);
  if (np2 > np) np = np2;
  if (np < (size_t)kRadixBins) np = kRadixBins;  // also the digit totals of the radix passes
  L.hist = take((size_t)nb * kRadixBins * 4);
  L.part = take(np * 4);
  L.left = take(nn * 4);
  L.right = take(nn * 4);
  L.rlo = take(nn * 4);
  L.rhi = take(nn * 4);
  L.sbox = take(nn * 6 * 4);
  L.b16 = take((nn + 15) / 16 * 6 * 4);
  L.bbox = take((nn + 255) / 256 * 6 * 4);
  L.b4k = take((nn + 4095) / 4096 * 6 * 4);
  L.nbox = take(nn * 6 * 4);
  L.nrec = take(nn * 16 * 4);
  L.status = take(4);
  L.total = p;
  return L;
}
}  // namespace

size_t sssgs_visibility_workspace_bytes(int32_t n) { return n < 0 ? 0 : vis_layout(n).total; }

sssgs_status sssgs_trace_visibility(const sssgs_gaussians *g, const sssgs_light *light, void *ws, size_t ws_bytes,
                                    float *out_visibility, void *stream) {
  if (!g || !light || !ws) return fail(SSSGS_ERR_INVALID_ARG, "null argument");
  if (g->n < 0) return fail(SSSGS_ERR_INVALID_ARG, "n < 0");
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !out_visibility))
    return fail(SSSGS_ERR_INVALID_ARG, "null Gaussian plane or output");
  const VisLayout L = vis_layout(g->n);
  if (ws_bytes < L.total) return fail(SSSGS_ERR_INVALID_ARG, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  VisArgs a;
  memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.means = g->means; a.log_scales = g->log_scales; a.quats = g->quats; a.logits = g->opacity_logits;
  for (int k = 0; k < 3; k++) a.light[k] = light->pos[k];
  a.rec = at<double>(ws, L.rec);
  a.scene = at<uint32_t>(ws, L.scene);
  a.bpart = at<uint32_t>(ws, L.bpart);
  a.left = at<int>(ws, L.left); a.right = at<int>(ws, L.right);
  a.range_lo = at<int>(ws, L.rlo); a.range_hi = at<int>(ws, L.rhi);
  a.sbox = at<float>(ws, L.sbox);
  a.b16 = at<float>(ws, L.b16);
  a.bbox = at<float>(ws, L.bbox);
  a.b4k = at<float>(ws, L.b4k);
  a.nbox = at<float>(ws, L.nbox);
  a.nrec = at<float>(ws, L.nrec);
  a.status = at<uint32_t>(ws, L.status);
  a.vis = out_visibility;
  Scope sc(kStVisibility, st);
  launch_visibility(a, at<uint32_t>(ws, L.ka), at<uint32_t>(ws, L.va), at<uint32_t>(ws, L.kb),
                    at<uint32_t>(ws, L.vb), at<uint32_t>(ws, L.hist), at<uint32_t>(ws, L.part), st);
  return check_hip("visibility launch");
}

sssgs_status sssgs_l1_loss(const float *pred, const float *target, int64_t count, float scale, float *loss_out,
                           float *dL_dpred, void *stream) {
  if (count < 0) return fail(SSSGS_ERR_INVALID_ARG, "count < 0");
  if (count > 0 && (!pred || !target)) return fail(SSSGS_ERR_INVALID_ARG, "null pred or target");
  launch_l1_loss(pred, target, count, scale, loss_out, dL_dpred, (hipStream_t)stream);
  return check_hip("l1 launch");
}

size_t sssgs_image_loss_workspace_bytes(int32_t channels, int32_t height, int32_t width) {
  if (channels <= 0 || height <= 0 || width <= 0) return 0;
  return image_loss_workspace_bytes(channels, height, width);
}

sssgs_status sssgs_image_loss(const float *pred, const float *target, int32_t channels, int32_t height,
                              int32_t width, float lambda_dssim, void *ws, size_t ws_bytes, float *loss_out,
                              float *dL_dpred, void *stream) {
  if (channels <= 0 || height <= 0 || width <= 0) return fail(SSSGS_ERR_INVALID_ARG, "bad image size");
  if (!pred || !target || !loss_out || !ws) return fail(SSSGS_ERR_INVALID_ARG, "null pointer");
  if (ws_bytes < image_loss_workspace_bytes(channels, height, width))
    return fail(SSSGS_ERR_INVALID_ARG, "workspace too small");
  launch_image_loss(pred, target, channels, height, width, lambda_dssim, ws, loss_out, dL_dpred,
                    (hipStream_t)stream);
  return check_hip("image loss launch");
}

sssgs_status sssgs_adam_step(float *param, const float *grad, float *m, float *v, int64_t count, float lr,
                             float beta1, float beta2, float eps, int32_t step, void *stream) {
  if (count < 0 || step < 1) return fail(SSSGS_ERR_INVALID_ARG, "count < 0 or step < 1");
  if (count > 0 && (!param || !grad || !m || !v)) return fail(SSSGS_ERR_INVALID_ARG, "null pointer");
  launch_adam(param, grad, m, v, count, lr, beta1, beta2, eps, step, (hipStream_t)stream);
  return check_hip("adam launch");
}

sssgs_status sssgs_workspace_status(const void *ws, int32_t n, int32_t width, int32_t height, int32_t feat_dim,
                                    int32_t mlp_width, int64_t cap, void *stream, int32_t *flags_out,
                                    int64_t *num_out) {
  Layout L;
  if (!ws) return fail(SSSGS_ERR_INVALID_ARG, "null workspace");
  if (!make_layout(n, width, height, feat_dim, mlp_width, cap, L)) return fail(SSSGS_ERR_INVALID_ARG, "bad sizes");
  int32_t hs[4];
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(hs, static_cast<const char *>(ws) + L.status, sizeof(hs), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return check_hip("status readback");
  if (flags_out) *flags_out = hs[kStatusFlags];
  if (num_out) *num_out = (int64_t)(uint32_t)hs[kStatusMLo];
  return SSSGS_OK;
}

const char *sssgs_status_string(sssgs_status s) {
  switch (s) {
    case SSSGS_OK: return "ok";
    case SSSGS_ERR_INVALID_ARG: return "invalid argument";
    case SSSGS_ERR_CAPACITY: return "instance capacity exceeded";
    case SSSGS_ERR_UNSUPPORTED: return "unsupported configuration";
    case SSSGS_ERR_HIP: return "HIP error";
  }
  return "unknown status";
}

const char *sssgs_last_error(void) { return g_last_error.c_str(); }

sssgs_status sssgs_timing_enable(int32_t on) {
  g_timer.on = on != 0;
  return SSSGS_OK;
}

sssgs_status sssgs_timing_read(int32_t max_stages, double *total_ms, int32_t *launches, int32_t *n_stages) {
  if (!total_ms || !launches || !n_stages || max_stages < (int32_t)kStCount)
    return fail(SSSGS_ERR_INVALID_ARG, "timing_read needs arrays of sssgs_timing_stages() entries");
  for (int k = 0; k < kStCount; k++) {
    total_ms[k] = 0.0;
    launches[k] = 0;
  }
  sssgs_status s = SSSGS_OK;
  for (const TimerRec &r : g_timer.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      s = check_hip("timing read");
    } else {
      total_ms[r.stage] += ms;
      launches[r.stage] += 1;
    }
    g_timer.pool.push_back(r.a);
    g_timer.pool.push_back(r.b);
  }
  g_timer.recs.clear();
  *n_stages = kStCount;
  return s;
}

int32_t sssgs_timing_stages(void) { return kStCount; }

const char *sssgs_timing_stage_name(int32_t k) { return (k >= 0 && k < kStCount) ? kStageNames[k] : ""; }

}  // extern "C"

namespace sssgs {
// Error reporting for entry points defined in other sources (sssgs_last_error).
sssgs_status noalloc_fail(sssgs_status s, const char *msg) { return fail(s, msg); }
}  // namespace sssgs
