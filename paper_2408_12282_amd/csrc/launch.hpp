// launch.hpp -- host-side launchers of the kernels (defined next to them).
#pragma once
#include "common.hpp"

namespace sssgs {

struct ProjIn {
  int n;
  const float *means, *log_scales, *quats, *opacity_logits, *albedo, *roughness, *metallic, *sss, *features, *sh;
};
struct ProjGradOut {
  float *means, *log_scales, *quats, *opacity_logits, *albedo, *roughness, *metallic, *sss, *features, *sh;
  int accumulate;
};
struct ShadeArgs;
struct MultiLight;

template <int F, bool SH>
void launch_project_fwd_t(const ProjIn &in, const CamArgs &cam, float *records, uint32_t *keys, uint32_t *vals,
                          ushort4 *rects, int32_t *radii, short4 *boxes, hipStream_t st);
template <int F, bool SH>
void launch_project_bwd_t(const ProjIn &in, const CamArgs &cam, const float *gacc, const ProjGradOut &out,
                          hipStream_t st);

void launch_scan(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *partials, uint32_t *total_dev,
                 hipStream_t st, bool have_partials = false);
uint32_t radix_blocks(uint64_t n);
uint32_t scan_partials_needed(uint64_t n);
// One stable 8-bit pass over min(n_host, *n_dev) items (n_dev may be null):
// block-major digit counts in hist (radix_blocks(n_host) x 256); with
// want_tot the 256 digit totals in tot (tot is scratch of 256 words either way).
void launch_radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, uint32_t n_host,
                       const uint32_t *n_dev, int shift, uint32_t *hist, uint32_t *tot, bool want_tot,
                       hipStream_t st);
// Tile lists (Sec. 3.1 binning): super-bin expansion of the depth-sorted
// Gaussians, then the stable super-bin pass and the per-tile filtering into
// tile-major Gaussian-index lists with their ranges and the status word.
int superbin_log2(int TX, int TY);
bool superbin_supported(int TX, int TY);
uint32_t area_parts(uint32_t n);
size_t tile_piece_words(int TX, int TY, uint32_t cap);  // per-piece tile counts of the tile-list kernels
void launch_superbin_expand(const uint32_t *sorted_g, const ushort4 *rects, uint32_t n, uint32_t cap, int TX, int TY,
                            uint32_t *tt, uint32_t *offs, uint32_t *ka, uint32_t *va, uint32_t *partials,
                            uint32_t *ms_dev, uint32_t *area_part, hipStream_t st);
void launch_tile_lists(uint32_t n, uint32_t cap, int TX, int TY, uint32_t *ka, uint32_t *va, uint32_t *kb,
                       uint32_t *vb, uint32_t *counts, uint32_t *pcnt, uint32_t *hist, uint32_t *tot,
                       const uint32_t *ms_dev, const uint32_t *area_part, uint32_t *m_out, int32_t *status,
                       uint2 *ranges, hipStream_t st);

template <int C>
void launch_composite_fwd_t(const uint2 *ranges, const uint32_t *sorted_g, const float *records, const short4 *boxes,
                            int W, int H, int TX, int TY, float *gbuf, float *t_final, uint32_t *n_contrib,
                            uint32_t *tile_top, hipStream_t st);
template <int C>
void launch_composite_bwd_t(const uint2 *ranges, const uint32_t *sorted_g, const float *records, const short4 *boxes,
                            int W, int H, int TX, int TY, const float *t_final, const uint32_t *n_contrib,
                            const float *dG, const float *dT, float *gacc, const DetSlots &det,
                            const uint32_t *order, hipStream_t st);
void launch_tile_order(const uint32_t *tile_top, int T, uint32_t *order, hipStream_t st);
void launch_rect_area(const ushort4 *rects, uint32_t n, uint32_t *area, hipStream_t st);
void launch_slot_reduce(int C, const DetSlots &det, uint32_t n, float *gacc, hipStream_t st);

template <int F, int NET, int WIDTH, int IN_PAD>
void launch_shade_fwd_t(const ShadeArgs &a, const MultiLight &ml, hipStream_t st);
template <int F, int NET, int WIDTH, int IN_PAD>
void launch_shade_bwd_t(const ShadeArgs &a, hipStream_t st);
size_t net_operand_elems(int width, int in_pad);
// split form for the BF16 width-64 network: shading backward writing per-strip
// records (one 64-thread workgroup per strip), then the weight-gradient kernel
template <int F, int IN_PAD>
void launch_shade_bwd_split_t(const ShadeArgs &a, __bf16 *rec_x, __bf16 *rec_o, hipStream_t st);
constexpr int kWgradMaxBlocks = 256;
int mlp_wgrad_grid(int nstrips);
void launch_mlp_wgrad(const void *wops, const void *tops, const float *params, const __bf16 *rec_x,
                      const __bf16 *rec_o, int nstrips, float *partials, hipStream_t st);
int wgrad_gemm_splits(size_t P);
void launch_wgrad_gemm(int net, int width, int in_pad, const void *gx, const void *gdy, size_t P, float *partials,
                       hipStream_t st);

// network weight preparation and gradient reduction (mlp_prep.hip)
void launch_prep_weights(int net, int width, int in_pad, const float *params, void *wops, void *tops, void *nops,
                         hipStream_t st);
size_t prep_weight_bytes(int width, int in_pad);
void launch_reduce_partials(const float *partials, int nparts, int nparams, float *scratch, float *out,
                            int accumulate, hipStream_t st);
int reduce_scratch_floats(int nparams);
size_t image_loss_workspace_bytes(int C, int H, int W);
void launch_image_loss(const float *x, const float *y, int C, int H, int W, float lam, void *ws, float *loss,
                       float *grad, hipStream_t st);
void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t st);
void launch_l1_loss(const float *pred, const float *target, int64_t count, float scale, float *loss_out,
                    float *grad, hipStream_t st);
void launch_zero_f32(float *p, size_t n, hipStream_t st);

// Per-Gaussian network (gmlp.hip).
struct GmlpArgs {
  int n;
  const float *means, *log_scales, *quats, *vis;
  float cam[3], light[3];  // camera centre and light position (world)
  const float *params;     // packed weights and biases
  const float *wt;         // weights transposed per layer (launch_gmlp_prep)
  float *feat;             // forward: [8][n]
  const float *dfeat;      // backward: dL/d(features) [8][n]
  float *d_means, *d_log_scales, *d_quats;  // added to
  float *d_vis;            // written, or added when accumulate
  float *partials;         // [gmlp_wgrad_grid(n)][gmlp_param_count()]
  float *act, *dz;         // records [rows][ldn] (gmlp_act_floats, gmlp_dz_floats); act written by the forward
  uint32_t *masks;         // [5][ldn] Leaky-ReLU signs written by the forward
  size_t ldn;              // n rounded up to 64
  int accumulate;
};
constexpr int kGmlpMaxWaves = 512;
int gmlp_param_count();
int gmlp_wgrad_grid(int n);
size_t gmlp_ldn(int n);
size_t gmlp_act_floats(int n);
size_t gmlp_dz_floats(int n);
size_t gmlp_mask_words(int n);
void launch_gmlp_prep(const float *params, float *wt, hipStream_t st);
void launch_gmlp_fwd(const GmlpArgs &a, hipStream_t st);
void launch_gmlp_bwd(const GmlpArgs &a, hipStream_t st);

// Ray-traced light visibility of every Gaussian (bvh.hip).
struct VisArgs {
  int n;
  const float *means, *log_scales, *quats, *logits;
  float light[3];
  double *rec;                    // [n][16] per sorted leaf: whitening matrix (9), opacity, centre (3)
  uint32_t *scene;                // [6]: ordered-integer min / max of the centres
  uint32_t *bpart;                // [ceil(n / 256)][6]: the same per block of 256 Gaussians
  const uint32_t *codes, *order;  // sorted Morton codes and Gaussian indices (set by the launcher)
  int *left, *right;              // [n - 1] children (>= 0 internal node, < 0 leaf ~position)
  int *range_lo, *range_hi;       // [n - 1] sorted-leaf range of each internal node
  float *sbox;                    // [n][6] per sorted leaf: lo xyz, hi xyz of the alpha >= 1/255 ellipsoid
  float *b16;                     // [ceil(n / 16)][6] unions of 16-leaf blocks
  float *bbox;                    // [ceil(n / 256)][6] unions of 256-leaf blocks
  float *b4k;                     // [ceil(n / 4096)][6] unions of 4096-leaf blocks
  float *nbox;                    // [n - 1][6] internal node boxes
  float *nrec;                    // [n - 1][16] node records: children, both child boxes
  uint32_t *status;               // [1]: bit 0 = a traversal stack overflowed
  float *vis;                     // [n] out
};
void launch_visibility(const VisArgs &a, uint32_t *keys_a, uint32_t *vals_a, uint32_t *keys_b, uint32_t *vals_b,
                       uint32_t *hist, uint32_t *partials, hipStream_t st);

}  // namespace sssgs
