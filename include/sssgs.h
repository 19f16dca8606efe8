/*
 * sssgs.h -- C ABI of libsssgs.so: differentiable deferred Gaussian splatting
 * with GGX + residual-network shading on AMD Instinct MI355X (gfx950).
 *
 * Method: arxiv 2408.12282, "Subsurface Scattering for 3D Gaussian Splatting".
 *   Sec. 3.1, Eq. 1-2   Gaussians with covariance R S S^T R^T projected by the
 *                       EWA approximation Sigma' = J W Sigma W^T J^T.
 *   Sec. 3.1, Eq. 3     front-to-back alpha compositing of per-Gaussian values.
 *   Sec. 3.1, Eq. 4     Disney diffuse + microfacet specular BRDF.
 *   Sec. 3.2, Eq. 6-7   residual network for incident light and SSS radiance,
 *                       combined with the BRDF through the per-Gaussian sss.
 *   Sec. 3.2 "Per-Pixel Deferred Shading": composite properties into buffers,
 *                       back-project the composited depth, shade per pixel.
 *   Pipeline figure, appendix "Network": the network evaluated per Gaussian,
 *                       its radiances composited (sssgs_gaussian_mlp_*).
 *   Sec. 3.2 "Incident Light": per-Gaussian light visibility by ray tracing
 *                       through the Gaussians with a BVH (sssgs_trace_visibility).
 *
 * Conventions (all the paper leaves open):
 *   - Camera: p_cam = R p + t with x right, y down, z forward; pinhole fx, fy,
 *     cx, cy; pixel (i, j) is sampled at (i + 0.5, j + 0.5).
 *   - Gaussians with z <= 0.2 are culled; x/z and y/z are clamped to
 *     +-1.3 * (W/2)/fx and +-1.3 * (H/2)/fy inside the Jacobian; Sigma' gets
 *     +0.3 on its diagonal; radius = ceil(3 sqrt(lambda_max)) with the
 *     eigenvalue gap floored at 0.1; 16x16 tiles; a Gaussian is evaluated at
 *     a pixel iff the pixel's tile lies in its tile rectangle
 *     [floor((u-r)/16), floor((u+r+15)/16)) (clamped to the grid).
 *   - alpha = min(0.99, o exp(power)); skipped if power > 0 or alpha < 1/255;
 *     the walk stops before a Gaussian that would bring T below 1e-4.
 *   - Order inside a tile: ascending (float32 depth, Gaussian index).  The
 *     depth key is the float32 rounding of a float64 evaluation of z.
 *   - G-buffer channels, premultiplied (sum of T alpha value):
 *       [0..2] basecolour (albedo, or SH colour when sh_degree = 3)
 *       [3..5] normal (world; axis of the smallest scale, facing the camera)
 *       [6] roughness [7] metallic [8] sss [9] view-space depth
 *       [10 .. 10+F) features.                              C = 10 + F.
 *   - Shading uses the mean values G / a with a = 1 - T_final; a pixel with
 *     a < 1e-6 is background (rgb 0, no gradient).  rgb = a * L_out.
 *
 * Memory: every array pointer below is a DEVICE pointer owned by the caller.
 * Per-Gaussian arrays are structure-of-arrays float32 planes [k][n]; images
 * are planes [k][height][width].  The library allocates no device memory: the
 * caller passes one workspace buffer (size from sssgs_workspace_bytes) that
 * must stay untouched between a forward call and the backward call that uses
 * it.  All work is enqueued on the caller's HIP stream (hipStream_t passed as
 * void*; NULL = default stream); calls with distinct workspaces may overlap.
 *
 * Errors: every entry point returns an sssgs_status.  Arguments are checked
 * on the host before anything is enqueued; an invalid argument enqueues
 * nothing.  SSSGS_ERR_HIP reports a failed launch; sssgs_last_error() gives
 * the HIP error text.
 */
#ifndef SSSGS_H
#define SSSGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SSSGS_OK = 0,
  SSSGS_ERR_INVALID_ARG = -1, /* NULL pointer, bad size, bad shape */
  SSSGS_ERR_CAPACITY = -2,    /* more tile instances than instance_capacity */
  SSSGS_ERR_UNSUPPORTED = -3, /* feature width / network shape without a kernel */
  SSSGS_ERR_HIP = -4          /* a HIP call failed */
} sssgs_status;

/* Gaussian parameters (Sec. 3.1: mean, scale, rotation quaternion, opacity;
   R3DGS material attributes; Eq. 7 subsurfaceness; features for Eq. 6).
   opacity = sigmoid(opacity_logit), scale = exp(log_scale), the quaternion
   (w, x, y, z) is normalised inside. */
typedef struct {
  int32_t n;          /* number of Gaussians, >= 0 */
  int32_t feat_dim;   /* F in {0, 8, 16, 32} */
  int32_t sh_degree;  /* -1: albedo colour; 3: degree-3 SH colour (48 planes) */
  const float *means;          /* [3][n] */
  const float *log_scales;     /* [3][n] */
  const float *quats;          /* [4][n] */
  const float *opacity_logits; /* [n] */
  const float *albedo;         /* [3][n] (ignored when sh_degree = 3) */
  const float *roughness;      /* [n] */
  const float *metallic;       /* [n] */
  const float *sss;            /* [n] */
  const float *features;       /* [F][n]; may be NULL when F = 0 */
  const float *sh;             /* [48][n], plane k*3+c; NULL unless sh_degree = 3 */
} sssgs_gaussians;

/* Gradient outputs, same shapes as sssgs_gaussians.  A NULL plane is skipped. */
typedef struct {
  float *means, *log_scales, *quats, *opacity_logits, *albedo, *roughness, *metallic, *sss, *features, *sh;
} sssgs_gaussian_grads;

typedef struct {
  float R[9];   /* world -> camera rotation, row-major */
  float t[3];   /* p_cam = R p + t */
  float fx, fy, cx, cy;
  int32_t width, height; /* >= 1 each */
} sssgs_camera;

/* One point light of known position (OLAT, Sec. 3.2 "Incident Light"). */
typedef struct {
  float pos[3];
  float intensity[3]; /* used only without the network: L_in = I / |p_L - x|^2 */
} sssgs_light;

/* Residual network of Eq. 6, evaluated per pixel.  Input
   [mean features (F) | Fourier encoding of the surface point: for k = 0..5,
   sin then cos of 2^k pi x for x, y, z (36) | w_out (3) | w_in (3)], zero
   padded to in_pad = in_dim rounded up to 32.  `hidden` ReLU layers of
   `width`, then a linear layer to 6 outputs: ReLU of [0..2] is the incident
   light, sigmoid of [3..5] the SSS radiance.  params packs row-major
   W0 [width][in_pad], b0, (hidden-1) x (W [width][width], b), W_out [6][width],
   b_out.  params == NULL (or a NULL sssgs_mlp*) renders without the network:
   L_out = (f_s + f_d) L_in (n . w_in). */
typedef struct {
  int32_t in_dim;   /* must equal F + 42 */
  int32_t width;    /* 64 or 128 */
  int32_t hidden;   /* 3 */
  int32_t out_dim;  /* 6 */
  const float *params; /* device, sssgs_mlp_param_count() floats */
} sssgs_mlp;

typedef enum { SSSGS_PREC_FP32 = 0, SSSGS_PREC_BF16 = 1 } sssgs_precision;

typedef struct {
  int32_t precision;        /* network arithmetic, on the matrix cores with FP32
                               accumulation either way: FP32 operands, or BF16
                               weights with each activation entering a forward
                               product as two BF16 numbers (the value rounded,
                               then the rounded remainder) and single BF16
                               upstream gradients.  Everything else is FP32. */
  int32_t accumulate_grads; /* backward: 0 overwrite gradient outputs, 1 add */
  int32_t radiance_features; /* 1: the radiances of Eq. 7 come from a per-Gaussian
                               network (sssgs_gaussian_mlp_forward) passed as the
                               Gaussians' eight feature planes: the deferred
                               shading takes the incident light from composited
                               feature planes 0-2 and the SSS radiance from planes
                               3-5 (each divided by alpha like every channel).
                               Requires feat_dim = 8 (the 18-plane G-buffer) and
                               no per-pixel network (SSSGS_ERR_UNSUPPORTED /
                               SSSGS_ERR_INVALID_ARG otherwise).  0: per-pixel
                               network or point-light fall-off. */
  int32_t deterministic;    /* backward: 1 sums each Gaussian's per-tile partial
                               gradients in a fixed order (one slot per tile of
                               its rectangle, then a row-major pass), so two
                               backward calls give bit-identical gradients; 0
                               adds them with atomics (order-dependent FP32
                               rounding).  Network weight gradients are summed
                               in a fixed order either way. */
  float background[3];      /* colour behind the Gaussians: rgb = a L_out +
                               T_final background (3DGS composites over a
                               constant background; black reproduces a plain
                               a L_out).  Its gradient reaches the Gaussians
                               through T_final.  Finite values. */
} sssgs_options;

/* Number of floats in sssgs_mlp.params. */
int64_t sssgs_mlp_param_count(int32_t in_dim, int32_t width, int32_t hidden, int32_t out_dim);

/* Bytes of workspace for one view: n Gaussians, width x height pixels,
   feature width F, network width (0 without network) and room for
   instance_capacity (tile, Gaussian) instances.  Returns 0 on bad arguments,
   including images whose 16x16 tile grid cannot be covered by 256 super-bins
   of at most 64x64 tiles (both sides up to 16384 pixels are always accepted). */
size_t sssgs_workspace_bytes(int32_t n, int32_t width, int32_t height, int32_t feat_dim, int32_t mlp_width,
                             int64_t instance_capacity);

/* Forward pass: projection, binning (order (tile, depth, index): radix sort of
   the depth keys, stable super-bin pass, per-tile filtering),
   compositing into the G-buffer, deferred shading.
   out_rgb [3][H][W], out_gbuffer [C][H][W] and out_alpha [H][W] are required.
   out_num_instances (HOST pointer) may be NULL.  When it is non-NULL the call
   waits for the stream once, stores the number of tile instances M and
   returns SSSGS_ERR_CAPACITY if M > instance_capacity (outputs are then
   undefined; retry with a larger workspace).  When it is NULL the call never
   waits; an overflow is recorded in the workspace (sssgs_workspace_status),
   kernels stay in bounds and the outputs are undefined. */
sssgs_status sssgs_render_forward(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                                  const sssgs_mlp *mlp, const sssgs_options *opt, void *workspace,
                                  size_t workspace_bytes, int64_t instance_capacity, float *out_rgb,
                                  float *out_gbuffer, float *out_alpha, int64_t *out_num_instances,
                                  void *stream);

/* Forward pass under several point lights at once: image-based lighting as a
   sum over light samples of an environment map (Appendix "Image Based
   Lighting": the relit image is the sum of the single-light images scaled by
   the environment's illumination).  Projection, binning and compositing run
   once; the deferred shading is evaluated for every light on the same
   G-buffer and summed:
     out_rgb = sum_k weights[k] (per channel) * rgb(lights[k]),
   where rgb(light) is what sssgs_render_forward writes for that light.
   lights: HOST array of num_lights >= 1; weights: HOST array [num_lights][3]
   of finite values (neither may be NULL).  The network input differs between
   lights only in the incident direction.  Other arguments, outputs, the
   workspace and errors as for sssgs_render_forward; out_gbuffer and
   out_alpha do not depend on the lights.  Forward only. */
sssgs_status sssgs_render_forward_lights(const sssgs_gaussians *g, const sssgs_camera *cam,
                                         const sssgs_light *lights, const float *weights, int32_t num_lights,
                                         const sssgs_mlp *mlp, const sssgs_options *opt, void *workspace,
                                         size_t workspace_bytes, int64_t instance_capacity, float *out_rgb,
                                         float *out_gbuffer, float *out_alpha, int64_t *out_num_instances,
                                         void *stream);

/* Backward pass of the forward call that filled `workspace` (same g, cam,
   light, mlp, options; gbuffer = that call's out_gbuffer).  Upstream gradients
   dL_drgb [3][H][W] (required), dL_dgbuffer [C][H][W] and dL_dalpha [H][W]
   (either may be NULL).  Writes (or adds, per opt->accumulate_grads) the
   gradient of every non-NULL plane of `grads` and, when mlp->params is
   non-NULL and dL_dmlp is non-NULL, of the network parameters.
   Transmittance is recomputed by reverse traversal; nothing per pixel-Gaussian
   pair is stored by the forward.  With opt->deterministic the per-Gaussian
   sums are bit-reproducible (see sssgs_options). */
sssgs_status sssgs_render_backward(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                                   const sssgs_mlp *mlp, const sssgs_options *opt, void *workspace,
                                   size_t workspace_bytes, int64_t instance_capacity, const float *gbuffer,
                                   const float *dL_drgb, const float *dL_dgbuffer, const float *dL_dalpha,
                                   sssgs_gaussian_grads *grads, float *dL_dmlp, void *stream);

/* Per-Gaussian network (pipeline figure: Eq. 6 evaluated for each Gaussian
   before rasterisation, Sec. 3.2; layer sizes from the appendix "Network").
   Input per Gaussian (42 values): normal (the shortest rotation axis turned
   toward the camera, Sec. 3.1) | unit quaternion | scale exp(log_scale) |
   direction to the light | direction to the camera | distance to the light |
   visibility | sin, cos(2^k pi mu) for k = 0..3.  Trunk of 64, 32, 32 units with
   Leaky-ReLU (slope 0.01); incident-light head: 32 units (Leaky-ReLU) then 3
   outputs through a ReLU; SSS head: 3 outputs through a sigmoid.  params packs
   per layer W [rows][cols] row-major then b [rows], layers in the order trunk
   64x42, 32x64, 32x32, incident 32x32, 3x32, SSS 3x32
   (sssgs_gaussian_mlp_param_count() floats, device).
   Output out_features [8][n] (device): incident light (3) | SSS radiance (3) |
   visibility | 1 -- the feature planes of a render with feat_dim = 8 and
   options.radiance_features = 1, whose composited constant plane is alpha.
   Only n, means, log_scales and quats of `g` are read; visibility [n] (device).
   The light's position is used, not its intensity.  `workspace` (device,
   caller-owned) holds sssgs_gaussian_mlp_workspace_bytes(n) bytes.  FP32. */
int64_t sssgs_gaussian_mlp_param_count(void);
size_t sssgs_gaussian_mlp_workspace_bytes(int32_t n);
sssgs_status sssgs_gaussian_mlp_forward(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                                        const float *visibility, const float *params, void *workspace,
                                        size_t workspace_bytes, float *out_features, void *stream);
/* Backward of sssgs_gaussian_mlp_forward.  It reads the per-Gaussian records
   (layer activations and Leaky-ReLU signs) that the last forward call left
   in the same workspace: call it after a forward with the same n, Gaussians,
   camera, light, visibility and params, with the workspace untouched in
   between (the backward itself does not modify the records, so it may be
   called repeatedly).  dL_dfeatures [8][n]: gradient of the feature
   planes, e.g. the `features` gradient of sssgs_render_backward.  ADDS the
   network's contribution to dL_dmeans [3][n], dL_dlog_scales [3][n] and
   dL_dquats [4][n] (the render backward writes them first); writes (accumulate
   = 0) or adds (1) dL_dvisibility [n] and dL_dparams.  The weight gradient is
   summed in a fixed order (deterministic).  All device arrays. */
sssgs_status sssgs_gaussian_mlp_backward(const sssgs_gaussians *g, const sssgs_camera *cam, const sssgs_light *light,
                                         const float *visibility, const float *params, const float *dL_dfeatures,
                                         void *workspace, size_t workspace_bytes, float *dL_dmeans,
                                         float *dL_dlog_scales, float *dL_dquats, float *dL_dvisibility,
                                         float *dL_dparams, int32_t accumulate, void *stream);

/* Each Gaussian's visibility of the point light, by tracing a shadow ray
   through the other Gaussians with a bounding-volume hierarchy (Sec. 3.2,
   "Incident Light"; the visibility input of the per-Gaussian network).
   For Gaussian i the ray runs from its centre to light->pos.  Gaussian j
   (j != i) occludes it at the point of the ray's line where j is densest
   (in j's whitened frame S^-1 R^T (x - mu_j): t* = -(u.w)/(w.w), squared
   distance D2 = |u x w|^2/|w|^2) when that point lies on the segment and
   alpha = min(0.99, sigmoid(logit_j) exp(-D2/2)) >= 1/255; the visibility is
   the product of (1 - alpha) over the occluders, reported as 0 below 1e-4.
   Reads n, means, log_scales, quats and opacity_logits of `g`; writes
   out_visibility [n] (device).  The hierarchy (Morton-ordered radix tree over
   the ellipsoids where alpha can reach 1/255) is built in `workspace`
   (device, caller-owned, sssgs_visibility_workspace_bytes(n) bytes) on every
   call.  Deterministic.  A NaN output marks a ray whose traversal stack
   overflowed (it cannot with at most 2^31 Gaussians: the tree is at most 62
   levels deep). */
size_t sssgs_visibility_workspace_bytes(int32_t n);
sssgs_status sssgs_trace_visibility(const sssgs_gaussians *g, const sssgs_light *light, void *workspace,
                                    size_t workspace_bytes, float *out_visibility, void *stream);

/* Image loss of the training objective (Appendix "Losses": the L1 part),
   over `count` values: *loss_out (device) += sum |pred - target| * scale and
   dL_dpred = sign(pred - target) * scale (sign(0) = 0).  loss_out may be NULL. */
sssgs_status sssgs_l1_loss(const float *pred, const float *target, int64_t count, float scale, float *loss_out,
                           float *dL_dpred, void *stream);

/* Image loss of the training objective (Appendix "Losses"):
     L = (1 - lambda) mean|pred - target| + lambda (1 - mean SSIM(pred, target))
   over `channels` planes of height x width floats ([C][H][W], device), with the
   paper's lambda = 0.2 passed as lambda_dssim.  SSIM: local statistics under an
   11x11 Gaussian window (sigma 1.5, normalised), images extended with zeros
   outside their border, C1 = 0.01^2, C2 = 0.03^2 (data range 1).  Writes
   *loss_out (device, overwritten) and, when dL_dpred is not NULL,
   dL/dpred ([C][H][W], device, overwritten; sign(0) = 0 in the L1 part).
   `workspace` (device, caller-owned) holds at least
   sssgs_image_loss_workspace_bytes(channels, height, width) bytes.
   Deterministic: fixed summation order.  Errors: INVALID_ARG for
   non-positive sizes, null pointers or a short workspace. */
size_t sssgs_image_loss_workspace_bytes(int32_t channels, int32_t height, int32_t width);
sssgs_status sssgs_image_loss(const float *pred, const float *target, int32_t channels, int32_t height,
                              int32_t width, float lambda_dssim, void *workspace, size_t workspace_bytes,
                              float *loss_out, float *dL_dpred, void *stream);

/* The image loss above for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid
   allocation): the same computation and outputs as sssgs_image_loss, with the
   scratch in a fixed device array of SSSGS_NOALLOC_SCRATCH_BYTES that the
   library holds on each GPU it runs on until the process ends.  The call
   allocates nothing.  Images whose sssgs_image_loss_workspace_bytes exceed
   that size are rejected with SSSGS_ERR_INVALID_ARG (32 MiB: three channels
   of 1024 x 1024 do not fit, three of 800 x 800 do).  All calls on one GPU
   share the array: calls that overlap on one GPU (different streams, or
   threads) race and must be serialised by the caller; consecutive calls on
   one stream are ordered.  Nothing in the array needs to start at zero. */
#define SSSGS_NOALLOC_SCRATCH_BYTES (32u * 1024u * 1024u)
sssgs_status sssgs_image_loss_noalloc(const float *pred, const float *target, int32_t channels, int32_t height,
                                      int32_t width, float lambda_dssim, float *loss_out, float *dL_dpred,
                                      void *stream);

/* One Adam update (Appendix "Training": Adam with its default parameters) of
   `count` float parameters in place, all device arrays:
     m = beta1 m + (1 - beta1) g;  v = beta2 v + (1 - beta2) g^2;
     param -= lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps)
   with step >= 1 the index of this update.  The learning-rate schedule is the
   caller's (lr is passed per call).  Errors: INVALID_ARG for count < 0, step < 1
   or null pointers. */
sssgs_status sssgs_adam_step(float *param, const float *grad, float *m, float *v, int64_t count, float lr,
                             float beta1, float beta2, float eps, int32_t step, void *stream);

/* Device-side status of the last forward on this workspace (sizes as passed
   to sssgs_workspace_bytes): flags bit 0 set = instance capacity overflowed;
   num_instances = tiles touched by all Gaussians.  Waits for the stream. */
sssgs_status sssgs_workspace_status(const void *workspace, int32_t n, int32_t width, int32_t height,
                                    int32_t feat_dim, int32_t mlp_width, int64_t instance_capacity, void *stream,
                                    int32_t *flags_out, int64_t *num_instances_out);

/* Byte offsets of the regions a test may inspect (all inside the workspace). */
typedef struct {
  size_t records;        /* float [n][rec_stride]: u, v, conic a b c, opacity, channels */
  int32_t rec_stride;    /* floats per record */
  size_t depth_keys;     /* uint32 [n] float bits of the depth key */
  size_t rects;          /* uint16x4 [n]: x0, y0, x1, y1 tiles */
  size_t radii;          /* int32 [n] */
  size_t tile_ranges;    /* uint32x2 [tiles]: [start, end) into sorted_gauss */
  size_t sorted_gauss;   /* uint32 [capacity] Gaussian index per instance, tile-major */
  size_t t_final;        /* float [H][W] */
  size_t n_contrib;      /* uint32 [H][W] */
  size_t status;         /* int32[4]: flags, M low, M high, unused */
  size_t boxes;          /* int16x4 [n]: inclusive pixel bounds x_lo, x_hi, y_lo, y_hi
                            outside which alpha < 1/255 (empty: x_lo > x_hi) */
} sssgs_layout;

sssgs_status sssgs_workspace_layout(int32_t n, int32_t width, int32_t height, int32_t feat_dim, int32_t mlp_width,
                                    int64_t instance_capacity, sssgs_layout *out);

/* Optional stage timing.  While enabled, every stage of a forward or
   backward call (projection, depth sort, expansion, tile sort, ranges,
   compositing, shading, network-gradient reduction, compositing backward,
   projection backward) records a pair of HIP events on the call's stream.
   sssgs_timing_read waits for the recorded events, writes per-stage summed
   milliseconds and call counts into arrays of sssgs_timing_stages() entries
   and clears the record.  Process-wide; not thread-safe. */
sssgs_status sssgs_timing_enable(int32_t on);
sssgs_status sssgs_timing_read(int32_t max_stages, double *total_ms, int32_t *launches, int32_t *n_stages);
int32_t sssgs_timing_stages(void);
const char *sssgs_timing_stage_name(int32_t k);

const char *sssgs_status_string(sssgs_status s);
const char *sssgs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
