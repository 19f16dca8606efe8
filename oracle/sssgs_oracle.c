/*
 * sssgs_oracle.c -- plain FP64 CPU reference renderer (the oracle).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant generator
 * with the HIP library.
 *
 * What it computes (arxiv 2408.12282, "Subsurface Scattering for 3D Gaussian
 * Splatting"):
 *   - Sec. 3.1, Eq. 1-2: each Gaussian's 3D covariance from scale and unit
 *     quaternion, projected by the EWA approximation Sigma' = J W Sigma W^T J^T.
 *   - Sec. 3.1, Eq. 3: front-to-back alpha compositing; alpha = opacity times
 *     the 2D Gaussian at the pixel (text after Eq. 3).
 *   - Sec. 3.1, Eq. 4: Disney diffuse (1-m) b / pi and a microfacet specular
 *     term D F G / ((w_o.n)(w_i.n)) (read with the usual factor 4).
 *   - Sec. 3.2, Eq. 6: the residual network returning incident light and SSS
 *     radiance from a Fourier-encoded position plus directions.
 *   - Sec. 3.2, Eq. 7: L_out = sss L_sss + (1-sss)(f_s+f_d) L_in (n.w_i).
 *   - Pipeline figure and appendix "Network": with the network evaluated per
 *     Gaussian instead (the per-Gaussian network itself is in
 *     gaussian_mlp.py), its incident light and SSS radiance are blended like
 *     any other channel and Eq. 7 takes them from the composited buffers
 *     (og_mlp.radiance_features).
 *   - Sec. 3.2, "Per-Pixel Deferred Shading": properties are composited into
 *     image buffers first; the BRDF is evaluated per pixel at the surface point
 *     obtained by back-projecting the composited depth.
 * and the exact (almost-everywhere) derivative of all of it.
 *
 * The paper leaves the rasteriser conventions open; the readings used here
 * (pinhole camera, 16x16 tiles, 3-sigma tile rectangles, 0.3 px low-pass,
 * alpha cut-offs 1/255 and 0.99, exclusive stop at T < 1e-4, depth order with
 * index tie-break, shortest-axis normal, premultiplied G-buffer) are listed
 * with the design notes of the repository.
 *
 * Everything is evaluated per pixel from the definitions: the list of a pixel
 * is "all Gaussians whose tile rectangle contains the pixel's tile", ordered by
 * (depth rounded to float32, index).  Lists are built per tile only because all
 * pixels of a tile share them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <fenv.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TILE 16
#define CH_ALB 0
#define CH_NRM 3
#define CH_ROUGH 6
#define CH_METAL 7
#define CH_SSS 8
#define CH_DEPTH 9
#define CH_FEAT 10
#define NPE 36      /* 6 octaves x {sin,cos} x 3 axes */
#define MAXC 64
#define MAXW 256
#define MAXIN 256

typedef struct {
  int n, feat_dim, sh_degree; /* sh_degree -1: albedo colour; 3: SH colour */
  const double *means, *log_scales, *quats, *opacity_logits, *albedo, *roughness, *metallic, *sss,
      *features, *sh;
} og_gauss;

typedef struct {
  double R[9], t[3], fx, fy, cx, cy;
  int width, height;
} og_cam;

typedef struct {
  double pos[3], intensity[3];
} og_light;

typedef struct {
  int in_dim, in_pad, width, hidden, out_dim, bf16; /* params NULL: no network */
  const double *params;
  /* 1: no per-pixel network; feature channels 0-2 hold the blended incident
     light and 3-5 the blended SSS radiance of the per-Gaussian network */
  int radiance_features;
} og_mlp;

typedef struct {
  /* images */
  double *rgb, *gbuf, *alpha;
  double *gbuf_abs; /* diagnostic: sum of T alpha |value| per channel (scale of rounding errors) */
  double *net_margin; /* diagnostic: smallest |argument| of any ReLU of the network at the pixel, relative to
                         the sum of the magnitudes of its terms (|bias| + sum |w x|) */
  double *rgb_sens;   /* diagnostic [3][H][W]: sum_k |d rgb_c / d G_k| (|G_k| + sum|terms_k|) + |d rgb_c / d T| T,
                         the first-order change of rgb under unit relative perturbations of the G-buffer */
  int32_t *n_contrib;
  uint8_t *pix_flag;
  /* per Gaussian */
  double *mean2d, *conic, *depth, *opacity, *channels;
  int32_t *radius, *rect, *tiles_touched;
  uint8_t *g_flag;
  /* lists */
  int64_t *tile_ranges;
  int32_t *tile_list;
  int64_t list_capacity;
  int64_t *num_instances;
  uint64_t *signature;
} og_out;

typedef struct {
  const double *drgb, *dgbuf, *dalpha;
} og_upstream;

typedef struct {
  double *means, *log_scales, *quats, *opacity_logits, *albedo, *roughness, *metallic, *sss, *features,
      *sh, *mlp;
} og_grads;

/* ------------------------------------------------------------------------- */
/* Small vector helpers (FP64). */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* v / max(|v|, eps) */
static double normalize3(const double *v, double *out, double eps) {
  double l = sqrt(dot3(v, v));
  double d = l > eps ? l : eps;
  out[0] = v[0] / d; out[1] = v[1] / d; out[2] = v[2] / d;
  return l;
}

/* Backward of out = v / max(|v|,eps): given dout, add dv. */
static void normalize3_bwd(const double *v, double l, double eps, const double *dout, double *dv) {
  if (l > eps) {
    double o[3] = {v[0] / l, v[1] / l, v[2] / l};
    double p = dot3(o, dout);
    for (int k = 0; k < 3; k++) dv[k] += (dout[k] - o[k] * p) / l;
  } else {
    for (int k = 0; k < 3; k++) dv[k] += dout[k] / eps;
  }
}

/* Round to the nearest bfloat16 value (8 significant bits, ties to even). */
double og_round_bf16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e = ilogb(x);
  double scale = ldexp(1.0, e - 7);
  /* rint rounds half to even in the default (to-nearest) floating-point environment */
  return rint(x / scale) * scale;
}

/* Real orthonormal spherical harmonics up to degree 3 at unit direction d
   (no Condon-Shortley phase).  Constants are written from their closed forms. */
static void sh_basis(const double *d, double *Y) {
  const double pi = M_PI;
  double x = d[0], y = d[1], z = d[2];
  Y[0] = 0.5 * sqrt(1.0 / pi);
  double c1 = sqrt(3.0 / (4.0 * pi));
  Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
  double c2a = sqrt(15.0 / (4.0 * pi)), c2b = sqrt(5.0 / (16.0 * pi)), c2c = sqrt(15.0 / (16.0 * pi));
  Y[4] = c2a * x * y; Y[5] = c2a * y * z; Y[6] = c2b * (3.0 * z * z - 1.0); Y[7] = c2a * x * z;
  Y[8] = c2c * (x * x - y * y);
  double c3a = sqrt(35.0 / (32.0 * pi)), c3b = sqrt(105.0 / (4.0 * pi)), c3c = sqrt(21.0 / (32.0 * pi)),
         c3d = sqrt(7.0 / (16.0 * pi)), c3e = sqrt(105.0 / (16.0 * pi));
  Y[9] = c3a * y * (3.0 * x * x - y * y);
  Y[10] = c3b * x * y * z;
  Y[11] = c3c * y * (5.0 * z * z - 1.0);
  Y[12] = c3d * z * (5.0 * z * z - 3.0);
  Y[13] = c3c * x * (5.0 * z * z - 1.0);
  Y[14] = c3e * z * (x * x - y * y);
  Y[15] = c3a * x * (x * x - 3.0 * y * y);
}

/* Jacobian dY[k][j] = dY_k / dd_j of the polynomials above (d treated as free). */
static void sh_basis_jac(const double *d, double J[16][3]) {
  const double pi = M_PI;
  double x = d[0], y = d[1], z = d[2];
  memset(J, 0, sizeof(double) * 48);
  double c1 = sqrt(3.0 / (4.0 * pi));
  J[1][1] = c1; J[2][2] = c1; J[3][0] = c1;
  double c2a = sqrt(15.0 / (4.0 * pi)), c2b = sqrt(5.0 / (16.0 * pi)), c2c = sqrt(15.0 / (16.0 * pi));
  J[4][0] = c2a * y; J[4][1] = c2a * x;
  J[5][1] = c2a * z; J[5][2] = c2a * y;
  J[6][2] = c2b * 6.0 * z;
  J[7][0] = c2a * z; J[7][2] = c2a * x;
  J[8][0] = c2c * 2.0 * x; J[8][1] = -c2c * 2.0 * y;
  double c3a = sqrt(35.0 / (32.0 * pi)), c3b = sqrt(105.0 / (4.0 * pi)), c3c = sqrt(21.0 / (32.0 * pi)),
         c3d = sqrt(7.0 / (16.0 * pi)), c3e = sqrt(105.0 / (16.0 * pi));
  J[9][0] = c3a * 6.0 * x * y; J[9][1] = c3a * (3.0 * x * x - 3.0 * y * y);
  J[10][0] = c3b * y * z; J[10][1] = c3b * x * z; J[10][2] = c3b * x * y;
  J[11][1] = c3c * (5.0 * z * z - 1.0); J[11][2] = c3c * y * 10.0 * z;
  J[12][2] = c3d * (15.0 * z * z - 3.0);
  J[13][0] = c3c * (5.0 * z * z - 1.0); J[13][2] = c3c * x * 10.0 * z;
  J[14][0] = c3e * 2.0 * x * z; J[14][1] = -c3e * 2.0 * y * z; J[14][2] = c3e * (x * x - y * y);
  J[15][0] = c3a * (3.0 * x * x - 3.0 * y * y); J[15][1] = -c3a * 6.0 * x * y;
}

/* Exposed for the tests (SH orthonormality pin). */
void og_sh_basis(const double *d, double *Y) { sh_basis(d, Y); }

/* ------------------------------------------------------------------------- */
/* Projection (Eq. 1-2).  One record per Gaussian with every intermediate the
   backward needs. */

typedef struct {
  int valid;            /* 0: culled (behind the near plane, degenerate or off-screen) */
  double pc[3];         /* camera-space mean */
  double s[3];          /* scales */
  double qn[4];         /* normalised quaternion */
  double qlen;
  double Rq[9];         /* rotation of the Gaussian, row-major */
  double V[9];          /* camera-space 3D covariance */
  double J[6];          /* 2x3 Jacobian */
  int clx, cly;         /* 1 when x/z (y/z) was clamped */
  double tx, ty;        /* (clamped) x/z, y/z */
  double a, b, c, det;  /* 2D covariance incl. low-pass */
  double conic[3];
  double u, v;          /* mean in pixels */
  int r;
  int rect[4];          /* x0, y0, x1, y1 (tile units, half-open) */
  float zkey;           /* depth rounded to float32: the order key */
  double o;             /* opacity */
  int kmin;             /* axis of the smallest scale */
  double nsign;         /* +1/-1 flip of the normal toward the camera */
  double dir[3], dirlen, dirraw[3]; /* SH view direction */
  double shval[3];      /* SH colour before the max(.,0) */
  double ch[MAXC];      /* composited channels */
  int gflag;
} proj_t;

static int og_channels(int feat_dim) { return CH_FEAT + feat_dim; }

static void quat_to_rot(const double *q, double *R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* dL/dq for R(q) given dL/dR (row-major). */
static void quat_to_rot_bwd(const double *q, const double *dR, double *dq) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  dq[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  dq[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
               2 * x * dR[8]);
  dq[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
               2 * y * dR[8]);
  dq[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4] + y * dR[5] + x * dR[6] +
               y * dR[7]);
}

static double frac_margin(double x) { /* distance of x to the nearest integer */
  double f = x - floor(x);
  return f < 1.0 - f ? f : 1.0 - f;
}

/* floor(v) clamped to [0, hi], clamped before the conversion to int */
static int floor_clamped(double v, int hi) {
  double f = floor(v);
  if (f < 0) f = 0;
  if (f > hi) f = hi;
  return (int)f;
}

static void project_one(const og_gauss *g, const og_cam *cam, int i, int TX, int TY, proj_t *P) {
  const int n = g->n;
  memset(P, 0, sizeof(*P));
  double mu[3] = {g->means[i], g->means[n + i], g->means[2 * n + i]};
  const double *Rw = cam->R;
  for (int k = 0; k < 3; k++) P->pc[k] = Rw[3 * k] * mu[0] + Rw[3 * k + 1] * mu[1] + Rw[3 * k + 2] * mu[2] + cam->t[k];
  double x = P->pc[0], y = P->pc[1], z = P->pc[2];
  P->zkey = (float)z;
  /* The order key is the float32 rounding of z; flag when z64 sits within a
     hair of a float32 rounding midpoint (two FP64 evaluations might round apart). */
  {
    double zk = (double)P->zkey;
    double ulp = fabs(nextafterf(P->zkey, INFINITY) - P->zkey);
    double dmid = fabs(fabs(z - zk) - 0.5 * ulp);
    /* an exact midpoint only arises from exact arithmetic, which rounds alike everywhere */
    if (dmid > 0 && dmid < 1e-12 * fabs(z)) P->gflag |= 1;
  }
  if (!(z > 0.2)) return; /* near plane */
  for (int k = 0; k < 3; k++) P->s[k] = exp(g->log_scales[k * n + i]);
  double q[4] = {g->quats[i], g->quats[n + i], g->quats[2 * n + i], g->quats[3 * n + i]};
  P->qlen = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; k++) P->qn[k] = q[k] / P->qlen;
  quat_to_rot(P->qn, P->Rq);
  /* Sigma = R S S^T R^T (Sec. 3.1, after Eq. 3) */
  double Sig[9];
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += P->Rq[3 * r + k] * P->s[k] * P->s[k] * P->Rq[3 * c + k];
      Sig[3 * r + c] = acc;
    }
  /* V = W Sigma W^T (Eq. 2) */
  double T1[9];
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += Rw[3 * r + k] * Sig[3 * k + c];
      T1[3 * r + c] = acc;
    }
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += T1[3 * r + k] * Rw[3 * c + k];
      P->V[3 * r + c] = acc;
    }
  /* J: Jacobian of the perspective map at the (clamped) mean direction (Eq. 2) */
  double limx = 1.3 * (0.5 * cam->width) / cam->fx, limy = 1.3 * (0.5 * cam->height) / cam->fy;
  double rx = x / z, ry = y / z;
  P->clx = rx < -limx || rx > limx;
  P->cly = ry < -limy || ry > limy;
  P->tx = rx < -limx ? -limx : (rx > limx ? limx : rx);
  P->ty = ry < -limy ? -limy : (ry > limy ? limy : ry);
  P->J[0] = cam->fx / z; P->J[1] = 0; P->J[2] = -cam->fx * P->tx / z;
  P->J[3] = 0; P->J[4] = cam->fy / z; P->J[5] = -cam->fy * P->ty / z;
  /* Sigma' = J V J^T + 0.3 I */
  double JV[6];
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 3; c++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += P->J[3 * r + k] * P->V[3 * k + c];
      JV[3 * r + c] = acc;
    }
  double S2[4];
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 2; c++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += JV[3 * r + k] * P->J[3 * c + k];
      S2[2 * r + c] = acc;
    }
  P->a = S2[0] + 0.3; P->b = S2[1]; P->c = S2[3] + 0.3;
  P->det = P->a * P->c - P->b * P->b;
  if (!(P->det > 0)) return;
  P->conic[0] = P->c / P->det; P->conic[1] = -P->b / P->det; P->conic[2] = P->a / P->det;
  double mid = 0.5 * (P->a + P->c);
  double disc = mid * mid - P->det;
  double lam = mid + sqrt(disc > 0.1 ? disc : 0.1);
  double r3 = 3.0 * sqrt(lam);
  double rr = ceil(r3);
  if (rr > 1e9) rr = 1e9; /* keeps the integer radius representable */
  P->r = (int)rr;
  P->u = cam->fx * x / z + cam->cx;
  P->v = cam->fy * y / z + cam->cy;
  double fx0 = (P->u - P->r) / TILE, fx1 = (P->u + P->r + TILE - 1) / TILE;
  double fy0 = (P->v - P->r) / TILE, fy1 = (P->v + P->r + TILE - 1) / TILE;
  P->rect[0] = floor_clamped(fx0, TX);
  P->rect[1] = floor_clamped(fy0, TY);
  P->rect[2] = floor_clamped(fx1, TX);
  P->rect[3] = floor_clamped(fy1, TY);
  {
    double m = frac_margin(r3);
    double m2 = frac_margin(fx0), m3 = frac_margin(fx1), m4 = frac_margin(fy0), m5 = frac_margin(fy1);
    if (m2 < m) m = m2;
    if (m3 < m) m = m3;
    if (m4 < m) m = m4;
    if (m5 < m) m = m5;
    if (m < 1e-9) P->gflag |= 2;
  }
  if ((P->rect[2] - P->rect[0]) * (P->rect[3] - P->rect[1]) == 0) return;
  P->valid = 1;
  P->o = 1.0 / (1.0 + exp(-g->opacity_logits[i]));
  /* normal: axis of the smallest scale, facing the camera (reading of Sec. 3.1 R3DGS paragraph) */
  double ls0 = g->log_scales[i], ls1 = g->log_scales[n + i], ls2 = g->log_scales[2 * n + i];
  P->kmin = 0;
  if (ls1 < ls0) P->kmin = 1;
  if (ls2 < (P->kmin == 0 ? ls0 : ls1)) P->kmin = 2;
  double nn[3] = {P->Rq[P->kmin], P->Rq[3 + P->kmin], P->Rq[6 + P->kmin]};
  double Cw[3];
  for (int k = 0; k < 3; k++) Cw[k] = -(Rw[k] * cam->t[0] + Rw[3 + k] * cam->t[1] + Rw[6 + k] * cam->t[2]);
  double tocam[3] = {Cw[0] - mu[0], Cw[1] - mu[1], Cw[2] - mu[2]};
  P->nsign = dot3(nn, tocam) < 0 ? -1.0 : 1.0;
  int C = og_channels(g->feat_dim);
  if (g->sh_degree >= 0) {
    for (int k = 0; k < 3; k++) P->dirraw[k] = mu[k] - Cw[k];
    P->dirlen = normalize3(P->dirraw, P->dir, 1e-12);
    double Y[16];
    sh_basis(P->dir, Y);
    for (int c = 0; c < 3; c++) {
      double acc = 0.5;
      for (int k = 0; k < 16; k++) acc += Y[k] * g->sh[(k * 3 + c) * n + i];
      P->shval[c] = acc;
      P->ch[CH_ALB + c] = acc > 0 ? acc : 0;
    }
  } else {
    for (int c = 0; c < 3; c++) P->ch[CH_ALB + c] = g->albedo[c * n + i];
  }
  for (int k = 0; k < 3; k++) P->ch[CH_NRM + k] = P->nsign * nn[k];
  P->ch[CH_ROUGH] = g->roughness[i];
  P->ch[CH_METAL] = g->metallic[i];
  P->ch[CH_SSS] = g->sss[i];
  P->ch[CH_DEPTH] = z;
  for (int f = 0; f < g->feat_dim; f++) P->ch[CH_FEAT + f] = g->features[f * n + i];
  (void)C;
}

/* ------------------------------------------------------------------------- */
/* Shading (Eq. 4, Eq. 6, Eq. 7, per-pixel deferred shading). */

typedef struct {
  double a, gbar[MAXC];
  double nraw[3], nlen, nrm[3];
  double ray[3], x[3];
  double vo[3], lo, wo[3], vi[3], li, wi[3], hv[3], hl, h[3];
  double nov_raw, nol_raw, noh_raw, voh_raw;
  double NoV, NoL, NoH, VoH, cosI;
  double ag, den, D, k, g1v, g1l, dv_, dl_, Gv, Q;
  double F0[3], F[3], fs[3], fd[3];
  double li2, Lin[3];
  double in[MAXIN];          /* network input (padded) */
  double act[8][MAXW];       /* layer inputs as the forward products use them (emulation: hi + lo) */
  double act_w[8][MAXW];     /* layer inputs as the weight gradient uses them (emulation: hi) */
  double pre[8][MAXW];       /* pre-activations */
  double out[8];
  double margin;             /* smallest |argument| / (sum of |terms|) of any ReLU */
  double Lsss[3];
  double L[3];
  int background;
} shade_t;

static const double *mlp_layer_w(const og_mlp *m, int layer, int *rows, int *cols, const double **bias) {
  const double *p = m->params;
  *rows = 0; *cols = 0; *bias = p;
  int in = m->in_pad;
  for (int l = 0; l <= m->hidden; l++) {
    int r = (l == m->hidden) ? m->out_dim : m->width;
    int c = (l == 0) ? in : m->width;
    if (l == layer) {
      *rows = r; *cols = c; *bias = p + (size_t)r * c;
      return p;
    }
    p += (size_t)r * c + r;
  }
  return NULL;
}

static size_t mlp_layer_offset(const og_mlp *m, int layer) {
  size_t off = 0;
  for (int l = 0; l < layer; l++) {
    int r = (l == m->hidden) ? m->out_dim : m->width;
    int c = (l == 0) ? m->in_pad : m->width;
    off += (size_t)r * c + r;
  }
  return off;
}

static double rb(const og_mlp *m, double v) { return m->bf16 ? og_round_bf16(v) : v; }

/* BF16 emulation of an activation entering a forward product: the value is
   carried as two bfloat16 numbers, hi = RNE(v) and lo = RNE(v - hi), so the
   product sees hi + lo (16 significant bits); the weight gradient takes hi. */
static void rb_act(const og_mlp *m, double v, double *prod, double *wgrad) {
  if (!m->bf16) { *prod = v; *wgrad = v; return; }
  double hi = og_round_bf16(v);
  *prod = hi + og_round_bf16(v - hi);
  *wgrad = hi;
}

static void shade_pixel(const og_cam *cam, const og_light *light, const og_mlp *mlp, int blend, int C, int F,
                        const double *G, double T, double uc, double vc, shade_t *S) {
  memset(S, 0, sizeof(*S));
  S->a = 1.0 - T;
  if (S->a < 1e-6) { S->background = 1; return; }
  for (int k = 0; k < C; k++) S->gbar[k] = G[k] / S->a;
  for (int k = 0; k < 3; k++) S->nraw[k] = S->gbar[CH_NRM + k];
  S->nlen = normalize3(S->nraw, S->nrm, 1e-12);
  double rc[3] = {(uc - cam->cx) / cam->fx, (vc - cam->cy) / cam->fy, 1.0};
  const double *Rw = cam->R;
  double Cw[3];
  for (int k = 0; k < 3; k++) {
    S->ray[k] = Rw[k] * rc[0] + Rw[3 + k] * rc[1] + Rw[6 + k] * rc[2];
    Cw[k] = -(Rw[k] * cam->t[0] + Rw[3 + k] * cam->t[1] + Rw[6 + k] * cam->t[2]);
  }
  double dbar = S->gbar[CH_DEPTH];
  for (int k = 0; k < 3; k++) S->x[k] = Cw[k] + dbar * S->ray[k];
  for (int k = 0; k < 3; k++) { S->vo[k] = Cw[k] - S->x[k]; S->vi[k] = light->pos[k] - S->x[k]; }
  S->lo = normalize3(S->vo, S->wo, 1e-12);
  S->li = normalize3(S->vi, S->wi, 1e-12);
  for (int k = 0; k < 3; k++) S->hv[k] = S->wo[k] + S->wi[k];
  S->hl = normalize3(S->hv, S->h, 1e-12);
  S->nov_raw = dot3(S->nrm, S->wo);
  S->nol_raw = dot3(S->nrm, S->wi);
  S->noh_raw = dot3(S->nrm, S->h);
  S->voh_raw = dot3(S->wo, S->h);
  S->NoV = S->nov_raw > 1e-4 ? S->nov_raw : 1e-4;
  S->NoL = S->nol_raw > 1e-4 ? S->nol_raw : 1e-4;
  S->NoH = S->noh_raw > 0 ? S->noh_raw : 0;
  S->VoH = S->voh_raw > 0 ? S->voh_raw : 0;
  S->cosI = S->nol_raw > 0 ? S->nol_raw : 0;
  double r = S->gbar[CH_ROUGH], m = S->gbar[CH_METAL];
  /* GGX microfacet distribution with alpha = roughness^2 */
  S->ag = r * r;
  S->den = S->NoH * S->NoH * (S->ag * S->ag - 1.0) + 1.0;
  S->D = S->ag * S->ag / (M_PI * S->den * S->den);
  /* Schlick-GGX shadowing with k = (r+1)^2/8, Smith product */
  S->k = (r + 1.0) * (r + 1.0) / 8.0;
  S->dv_ = S->NoV * (1.0 - S->k) + S->k;
  S->dl_ = S->NoL * (1.0 - S->k) + S->k;
  S->g1v = S->NoV / S->dv_;
  S->g1l = S->NoL / S->dl_;
  S->Gv = S->g1v * S->g1l;
  S->Q = 1.0 / (4.0 * S->NoV * S->NoL);
  double w = 1.0 - S->VoH, w5 = w * w * w * w * w;
  for (int c = 0; c < 3; c++) {
    double b = S->gbar[CH_ALB + c];
    S->F0[c] = 0.04 * (1.0 - m) + b * m;
    S->F[c] = S->F0[c] + (1.0 - S->F0[c]) * w5;
    S->fs[c] = S->D * S->F[c] * S->Gv * S->Q;
    S->fd[c] = (1.0 - m) * b / M_PI;
  }
  if (blend) {
    /* Eq. 7 with the composited radiances of the per-Gaussian network */
    double sss = S->gbar[CH_SSS];
    for (int c = 0; c < 3; c++) {
      S->Lin[c] = S->gbar[CH_FEAT + c];
      S->Lsss[c] = S->gbar[CH_FEAT + 3 + c];
      S->L[c] = sss * S->Lsss[c] + (1.0 - sss) * (S->fs[c] + S->fd[c]) * S->Lin[c] * S->cosI;
    }
    return;
  }
  if (!mlp) {
    S->li2 = dot3(S->vi, S->vi);
    if (S->li2 < 1e-12) S->li2 = 1e-12;
    for (int c = 0; c < 3; c++) {
      S->Lin[c] = light->intensity[c] / S->li2;
      S->L[c] = (S->fs[c] + S->fd[c]) * S->Lin[c] * S->cosI;
    }
    return;
  }
  /* network input: [features | gamma(x) | w_o | w_i | 0...] */
  int p = 0;
  for (int f = 0; f < F; f++) S->in[p++] = S->gbar[CH_FEAT + f];
  for (int oct = 0; oct < 6; oct++)
    for (int fn = 0; fn < 2; fn++)
      for (int ax = 0; ax < 3; ax++) {
        double arg = ldexp(M_PI, oct) * S->x[ax];
        S->in[p++] = fn == 0 ? sin(arg) : cos(arg);
      }
  for (int k = 0; k < 3; k++) S->in[p++] = S->wo[k];
  for (int k = 0; k < 3; k++) S->in[p++] = S->wi[k];
  for (; p < mlp->in_pad; p++) S->in[p] = 0;
  for (int k = 0; k < mlp->in_pad; k++) rb_act(mlp, S->in[k], &S->act[0][k], &S->act_w[0][k]);
  S->margin = INFINITY;
  for (int l = 0; l <= mlp->hidden; l++) {
    int rows = 0, cols = 0;
    const double *bias = NULL;
    const double *W = mlp_layer_w(mlp, l, &rows, &cols, &bias);
    for (int o = 0; o < rows; o++) {
      double acc = 0, mag = fabs(bias[o]);
      for (int c = 0; c < cols; c++) {
        acc += W[(size_t)o * cols + c] * S->act[l][c];
        mag += fabs(W[(size_t)o * cols + c] * S->act[l][c]);
      }
      acc += bias[o];
      S->pre[l][o] = acc;
      if (l < mlp->hidden) rb_act(mlp, acc > 0 ? acc : 0, &S->act[l + 1][o], &S->act_w[l + 1][o]);
      else S->out[o] = acc;
      /* decision margin of the ReLU: |argument| relative to the size of its terms */
      double rel = mag > 0 ? fabs(acc) / mag : INFINITY;
      if ((l < mlp->hidden || o < 3) && rel < S->margin) S->margin = rel;
    }
  }
  for (int c = 0; c < 3; c++) {
    S->Lin[c] = S->out[c] > 0 ? S->out[c] : 0;
    S->Lsss[c] = 1.0 / (1.0 + exp(-S->out[3 + c]));
  }
  double sss = S->gbar[CH_SSS];
  for (int c = 0; c < 3; c++)
    S->L[c] = sss * S->Lsss[c] + (1.0 - sss) * (S->fs[c] + S->fd[c]) * S->Lin[c] * S->cosI;
}

/* Backward of one pixel's shading.  gL = dLoss/d(rgb) (3).  Writes dG (C) and
   returns dLoss/dT_final; accumulates network-parameter gradients into dmlp. */
static double shade_pixel_bwd(const og_cam *cam, const og_light *light, const og_mlp *mlp, int blend, int C,
                              int F, const shade_t *S, const double *gL, double *dG, double *dmlp) {
  for (int k = 0; k < C; k++) dG[k] = 0;
  if (S->background) return 0.0;
  double a = S->a;
  double dgbar[MAXC];
  for (int k = 0; k < C; k++) dgbar[k] = 0;
  double dA = 0;
  double gLo[3];
  for (int c = 0; c < 3; c++) { dA += gL[c] * S->L[c]; gLo[c] = a * gL[c]; }
  double dfs[3], dfd[3], dLin[3] = {0, 0, 0}, dcos = 0, dx[3] = {0, 0, 0}, dwo[3] = {0, 0, 0}, dwi[3] = {0, 0, 0};
  double dvi[3] = {0, 0, 0};
  if (blend) {
    double sss = S->gbar[CH_SSS], dsss = 0;
    for (int c = 0; c < 3; c++) {
      double B = S->fs[c] + S->fd[c];
      dsss += gLo[c] * (S->Lsss[c] - B * S->Lin[c] * S->cosI);
      dfs[c] = gLo[c] * (1.0 - sss) * S->Lin[c] * S->cosI;
      dfd[c] = dfs[c];
      dcos += gLo[c] * (1.0 - sss) * B * S->Lin[c];
      dgbar[CH_FEAT + c] += gLo[c] * (1.0 - sss) * B * S->cosI;
      dgbar[CH_FEAT + 3 + c] += gLo[c] * sss;
    }
    dgbar[CH_SSS] += dsss;
  } else if (!mlp) {
    for (int c = 0; c < 3; c++) {
      dfs[c] = gLo[c] * S->Lin[c] * S->cosI;
      dfd[c] = dfs[c];
      dLin[c] = gLo[c] * (S->fs[c] + S->fd[c]) * S->cosI;
      dcos += gLo[c] * (S->fs[c] + S->fd[c]) * S->Lin[c];
    }
    double dli2 = 0;
    for (int c = 0; c < 3; c++) dli2 += -dLin[c] * light->intensity[c] / (S->li2 * S->li2);
    if (dot3(S->vi, S->vi) >= 1e-12)
      for (int k = 0; k < 3; k++) dvi[k] += dli2 * 2.0 * S->vi[k];
  } else {
    double sss = S->gbar[CH_SSS];
    double dLsss[3], dsss = 0;
    for (int c = 0; c < 3; c++) {
      double B = S->fs[c] + S->fd[c];
      dsss += gLo[c] * (S->Lsss[c] - B * S->Lin[c] * S->cosI);
      dLsss[c] = gLo[c] * sss;
      dfs[c] = gLo[c] * (1.0 - sss) * S->Lin[c] * S->cosI;
      dfd[c] = dfs[c];
      dLin[c] = gLo[c] * (1.0 - sss) * B * S->cosI;
      dcos += gLo[c] * (1.0 - sss) * B * S->Lin[c];
    }
    dgbar[CH_SSS] += dsss;
    double dout[8] = {0};
    for (int c = 0; c < 3; c++) {
      dout[c] = S->out[c] > 0 ? dLin[c] : 0;
      dout[3 + c] = dLsss[c] * S->Lsss[c] * (1.0 - S->Lsss[c]);
    }
    /* back through the network; emulation mode rounds the upstream gradient
       entering each product and the weights, as the tensor-core path does */
    double dcur[MAXW];
    for (int o = 0; o < mlp->out_dim; o++) dcur[o] = dout[o];
    double din[MAXIN];
    for (int l = mlp->hidden; l >= 0; l--) {
      int rows = 0, cols = 0;
      const double *bias = NULL;
      const double *W = mlp_layer_w(mlp, l, &rows, &cols, &bias);
      size_t off = mlp_layer_offset(mlp, l);
      double dprev[MAXIN];
      for (int c = 0; c < cols; c++) dprev[c] = 0;
      for (int o = 0; o < rows; o++) {
        double d = dcur[o];
        if (d == 0.0) continue;
        double dr = rb(mlp, d);
        if (dmlp) {
          /* bias: the sum of the upstream gradient as it enters the products */
          dmlp[off + (size_t)rows * cols + o] += dr;
          for (int c = 0; c < cols; c++) dmlp[off + (size_t)o * cols + c] += dr * S->act_w[l][c];
        }
        for (int c = 0; c < cols; c++) dprev[c] += W[(size_t)o * cols + c] * dr;
      }
      if (l > 0) {
        for (int c = 0; c < cols; c++) dcur[c] = S->pre[l - 1][c] > 0 ? dprev[c] : 0;
      } else {
        for (int c = 0; c < cols; c++) din[c] = dprev[c];
      }
    }
    int p = 0;
    for (int f = 0; f < F; f++) dgbar[CH_FEAT + f] += din[p++];
    for (int oct = 0; oct < 6; oct++)
      for (int fn = 0; fn < 2; fn++)
        for (int ax = 0; ax < 3; ax++) {
          double fr = ldexp(M_PI, oct);
          double arg = fr * S->x[ax];
          dx[ax] += din[p++] * (fn == 0 ? fr * cos(arg) : -fr * sin(arg));
        }
    for (int k = 0; k < 3; k++) dwo[k] += din[p++];
    for (int k = 0; k < 3; k++) dwi[k] += din[p++];
  }
  /* BRDF */
  double r = S->gbar[CH_ROUGH], m = S->gbar[CH_METAL];
  double dD = 0, dGv = 0, dQ = 0, dF0[3], dVoH = 0, dm = 0, db[3] = {0, 0, 0};
  double w = 1.0 - S->VoH, w4 = w * w * w * w, w5 = w4 * w;
  for (int c = 0; c < 3; c++) {
    dD += dfs[c] * S->F[c] * S->Gv * S->Q;
    double dF = dfs[c] * S->D * S->Gv * S->Q;
    dGv += dfs[c] * S->D * S->F[c] * S->Q;
    dQ += dfs[c] * S->D * S->F[c] * S->Gv;
    dF0[c] = dF * (1.0 - w5);
    dVoH += dF * (1.0 - S->F0[c]) * 5.0 * w4 * (-1.0);
    double b = S->gbar[CH_ALB + c];
    db[c] += dfd[c] * (1.0 - m) / M_PI;
    dm += -dfd[c] * b / M_PI;
    db[c] += dF0[c] * m;
    dm += dF0[c] * (b - 0.04);
  }
  double dNoV = dQ * (-S->Q / S->NoV), dNoL = dQ * (-S->Q / S->NoL);
  /* G */
  double dg1v = dGv * S->g1l, dg1l = dGv * S->g1v;
  dNoV += dg1v * S->k / (S->dv_ * S->dv_);
  dNoL += dg1l * S->k / (S->dl_ * S->dl_);
  double dk = dg1v * (-S->NoV * (1.0 - S->NoV) / (S->dv_ * S->dv_)) +
              dg1l * (-S->NoL * (1.0 - S->NoL) / (S->dl_ * S->dl_));
  double dr = dk * (r + 1.0) / 4.0;
  /* D */
  double ag = S->ag, den = S->den;
  double dag = dD * (2.0 * ag / (M_PI * den * den)) * (1.0 - 2.0 * ag * ag * S->NoH * S->NoH / den);
  double dNoH = dD * (-2.0 * ag * ag / (M_PI * den * den * den)) * 2.0 * S->NoH * (ag * ag - 1.0);
  dr += dag * 2.0 * r;
  dgbar[CH_ROUGH] += dr;
  dgbar[CH_METAL] += dm;
  for (int c = 0; c < 3; c++) dgbar[CH_ALB + c] += db[c];
  /* clamps */
  double dnov = S->nov_raw > 1e-4 ? dNoV : 0;
  double dnol = (S->nol_raw > 1e-4 ? dNoL : 0) + (S->nol_raw > 0 ? dcos : 0);
  double dnoh = S->noh_raw > 0 ? dNoH : 0;
  double dvoh = S->voh_raw > 0 ? dVoH : 0;
  double dn[3], dh[3];
  for (int k = 0; k < 3; k++) {
    dn[k] = dnov * S->wo[k] + dnol * S->wi[k] + dnoh * S->h[k];
    dwo[k] += dnov * S->nrm[k] + dvoh * S->h[k];
    dwi[k] += dnol * S->nrm[k];
    dh[k] = dnoh * S->nrm[k] + dvoh * S->wo[k];
  }
  double dhv[3] = {0, 0, 0};
  normalize3_bwd(S->hv, S->hl, 1e-12, dh, dhv);
  for (int k = 0; k < 3; k++) { dwo[k] += dhv[k]; dwi[k] += dhv[k]; }
  double dvo[3] = {0, 0, 0};
  normalize3_bwd(S->vo, S->lo, 1e-12, dwo, dvo);
  normalize3_bwd(S->vi, S->li, 1e-12, dwi, dvi);
  for (int k = 0; k < 3; k++) dx[k] += -dvo[k] - dvi[k];
  dgbar[CH_DEPTH] += dot3(dx, S->ray);
  double dnraw[3] = {0, 0, 0};
  normalize3_bwd(S->nraw, S->nlen, 1e-12, dn, dnraw);
  for (int k = 0; k < 3; k++) dgbar[CH_NRM + k] += dnraw[k];
  /* gbar = G / a */
  for (int k = 0; k < C; k++) {
    dG[k] = dgbar[k] / a;
    dA += -dgbar[k] * S->gbar[k] / a;
  }
  (void)cam;
  return -dA;
}

/* Exposed for the BRDF pins: evaluates (f_s + f_d) for one channel set. */
void og_brdf(const double *n, const double *wo, const double *wi, double basecolor, double rough,
             double metal, double *fs, double *fd) {
  double hv[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]}, h[3];
  normalize3(hv, h, 1e-12);
  double nov = dot3(n, wo), nol = dot3(n, wi), noh = dot3(n, h), voh = dot3(wo, h);
  double NoV = nov > 1e-4 ? nov : 1e-4, NoL = nol > 1e-4 ? nol : 1e-4;
  double NoH = noh > 0 ? noh : 0, VoH = voh > 0 ? voh : 0;
  double ag = rough * rough, den = NoH * NoH * (ag * ag - 1.0) + 1.0;
  double D = ag * ag / (M_PI * den * den);
  double k = (rough + 1.0) * (rough + 1.0) / 8.0;
  double Gv = NoV / (NoV * (1 - k) + k) * NoL / (NoL * (1 - k) + k);
  double F0 = 0.04 * (1 - metal) + basecolor * metal;
  double w = 1 - VoH;
  double F = F0 + (1 - F0) * w * w * w * w * w;
  *fs = D * F * Gv / (4 * NoV * NoL);
  *fd = (1 - metal) * basecolor / M_PI;
}

/* GGX D alone, for the normalisation pin. */
double og_ggx_d(double noh, double rough) {
  double ag = rough * rough, den = noh * noh * (ag * ag - 1.0) + 1.0;
  return ag * ag / (M_PI * den * den);
}

/* ------------------------------------------------------------------------- */
/* Tile lists. */

typedef struct {
  float z;
  int32_t i;
} keyidx_t;

static int cmp_keyidx(const void *pa, const void *pb) {
  const keyidx_t *a = (const keyidx_t *)pa, *b = (const keyidx_t *)pb;
  if (a->z < b->z) return -1;
  if (a->z > b->z) return 1;
  return (a->i > b->i) - (a->i < b->i);
}

static uint64_t mix64(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  return h;
}

/* ------------------------------------------------------------------------- */

/* background: colour behind the Gaussians (NULL: black).  The image is
   composited over it like one more, fully opaque layer at the back:
   rgb = a L_out + T_final background. */
int og_render(const og_gauss *g, const og_cam *cam, const og_light *light, const og_mlp *mlp_in,
              const int *crop, og_out *out, const og_upstream *up, og_grads *gr, int nthreads,
              const double *background) {
  const double bgc[3] = {background ? background[0] : 0.0, background ? background[1] : 0.0,
                         background ? background[2] : 0.0};
  const int n = g->n, W = cam->width, H = cam->height;
  const int TX = (W + TILE - 1) / TILE, TY = (H + TILE - 1) / TILE, T = TX * TY;
  const int F = g->feat_dim, C = og_channels(F);
  const int blend = mlp_in && mlp_in->radiance_features;
  const og_mlp *mlp = (!blend && mlp_in && mlp_in->params) ? mlp_in : NULL;
  if (C > MAXC) return -3;
  if (blend && F < 6) return -3;
  if (mlp && (mlp->width > MAXW || mlp->in_pad > MAXIN || mlp->out_dim != 6 || mlp->hidden + 1 > 8 ||
              mlp->in_dim != F + NPE + 6))
    return -3;
  /* Emulation of the bfloat16 tensor-core path: the weight matrices (not the
     biases) are rounded once; activations enter the forward products as a
     pair of bfloat16 numbers (hi + lo) and the weight gradient as hi alone;
     upstream gradients are rounded once where they enter a product
     (shade_pixel / shade_pixel_bwd). */
  og_mlp mlp_round;
  double *wround = NULL;
  if (mlp && mlp->bf16) {
    mlp_round = *mlp;
    size_t np0 = mlp_layer_offset(mlp, mlp->hidden + 1);
    wround = (double *)malloc(sizeof(double) * np0);
    memcpy(wround, mlp->params, sizeof(double) * np0);
    for (int l = 0; l <= mlp->hidden; l++) {
      int rows = 0, cols = 0;
      const double *bias = NULL;
      mlp_layer_w(mlp, l, &rows, &cols, &bias);
      size_t off = mlp_layer_offset(mlp, l);
      for (size_t k = 0; k < (size_t)rows * cols; k++) wround[off + k] = og_round_bf16(wround[off + k]);
    }
    mlp_round.params = wround;
    mlp = &mlp_round;
  }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int cx0 = 0, cy0 = 0, cx1 = W, cy1 = H;
  if (crop) { cx0 = crop[0]; cy0 = crop[1]; cx1 = crop[2]; cy1 = crop[3]; }

  proj_t *P = (proj_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(proj_t));
  if (!P) return -2;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; i++) project_one(g, cam, i, TX, TY, &P[i]);

  /* per-Gaussian outputs */
  for (int i = 0; i < n; i++) {
    if (out->mean2d) { out->mean2d[i] = P[i].u; out->mean2d[n + i] = P[i].v; }
    if (out->conic) for (int k = 0; k < 3; k++) out->conic[k * n + i] = P[i].conic[k];
    if (out->depth) out->depth[i] = P[i].pc[2];
    if (out->opacity) out->opacity[i] = P[i].o;
    if (out->radius) out->radius[i] = P[i].valid ? P[i].r : 0;
    if (out->rect) for (int k = 0; k < 4; k++) out->rect[k * n + i] = P[i].valid ? P[i].rect[k] : 0;
    if (out->tiles_touched)
      out->tiles_touched[i] = P[i].valid ? (P[i].rect[2] - P[i].rect[0]) * (P[i].rect[3] - P[i].rect[1]) : 0;
    if (out->g_flag) out->g_flag[i] = (uint8_t)P[i].gflag;
    if (out->channels) for (int k = 0; k < C; k++) out->channels[(size_t)k * n + i] = P[i].valid ? P[i].ch[k] : 0;
  }

  /* per-tile lists in (float32 depth, index) order */
  int64_t *cnt = (int64_t *)calloc((size_t)T + 1, sizeof(int64_t));
  for (int i = 0; i < n; i++) {
    if (!P[i].valid) continue;
    for (int ty = P[i].rect[1]; ty < P[i].rect[3]; ty++)
      for (int tx = P[i].rect[0]; tx < P[i].rect[2]; tx++) cnt[ty * TX + tx + 1]++;
  }
  for (int t = 0; t < T; t++) cnt[t + 1] += cnt[t];
  int64_t M = cnt[T];
  if (out->num_instances) *out->num_instances = M;
  keyidx_t *lists = (keyidx_t *)malloc(sizeof(keyidx_t) * (size_t)(M > 0 ? M : 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T + 1));
  memcpy(fill, cnt, sizeof(int64_t) * (size_t)(T + 1));
  for (int i = 0; i < n; i++) {
    if (!P[i].valid) continue;
    for (int ty = P[i].rect[1]; ty < P[i].rect[3]; ty++)
      for (int tx = P[i].rect[0]; tx < P[i].rect[2]; tx++) {
        keyidx_t e = {P[i].zkey, i};
        lists[fill[ty * TX + tx]++] = e;
      }
  }
#pragma omp parallel for schedule(dynamic, 4)
  for (int t = 0; t < T; t++) qsort(lists + cnt[t], (size_t)(cnt[t + 1] - cnt[t]), sizeof(keyidx_t), cmp_keyidx);
  if (out->tile_ranges)
    for (int t = 0; t < T; t++) { out->tile_ranges[2 * t] = cnt[t]; out->tile_ranges[2 * t + 1] = cnt[t + 1]; }
  if (out->tile_list && M <= out->list_capacity)
    for (int64_t e = 0; e < M; e++) out->tile_list[e] = lists[e].i;

  /* gradient accumulators (per thread) */
  int nth = 1;
#ifdef _OPENMP
  nth = omp_get_max_threads();
#endif
  const int GS = 6 + C; /* du dv dA dB dC dopacity | dchannels */
  double *gacc = NULL, *macc = NULL;
  size_t np = 0;
  if (up) {
    gacc = (double *)calloc((size_t)nth * (size_t)(n > 0 ? n : 1) * GS, sizeof(double));
    if (mlp) {
      np = mlp_layer_offset(mlp, mlp->hidden + 1);
      macc = (double *)calloc((size_t)nth * np, sizeof(double));
    }
  }
  uint64_t *sigs = (uint64_t *)calloc((size_t)T, sizeof(uint64_t));

  const int tx0 = cx0 / TILE, tx1 = (cx1 + TILE - 1) / TILE, ty0 = cy0 / TILE, ty1 = (cy1 + TILE - 1) / TILE;
  const int ntiles_crop = (tx1 - tx0) * (ty1 - ty0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int ti = 0; ti < ntiles_crop; ti++) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    int tx = tx0 + ti % (tx1 - tx0), ty = ty0 + ti / (tx1 - tx0);
    int t = ty * TX + tx;
    const keyidx_t *L = lists + cnt[t];
    int64_t len = cnt[t + 1] - cnt[t];
    uint64_t sig = mix64(0x1234, (uint64_t)t);
    for (int64_t e = 0; e < len; e++) sig = mix64(sig, (uint64_t)L[e].i);
    double *Gp = (double *)malloc(sizeof(double) * MAXC);
    double *Ga = (double *)malloc(sizeof(double) * MAXC);
    shade_t *S = (shade_t *)malloc(sizeof(shade_t));
    for (int py = ty * TILE; py < (ty + 1) * TILE && py < H; py++)
      for (int px = tx * TILE; px < (tx + 1) * TILE && px < W; px++) {
        if (px < cx0 || px >= cx1 || py < cy0 || py >= cy1) continue;
        size_t pix = (size_t)py * W + px;
        double uc = px + 0.5, vc = py + 0.5;
        /* Eq. 3: front-to-back compositing */
        double Tr = 1.0;
        for (int k = 0; k < C; k++) { Gp[k] = 0; Ga[k] = 0; }
        int32_t last = 0;
        uint8_t flag = 0;
        double tr_unc = 0.0; /* relative uncertainty of Tr under a float32 evaluation */
        for (int64_t e = 0; e < len; e++) {
          const proj_t *q = &P[L[e].i];
          double dx = q->u - uc, dy = q->v - vc;
          double pw = -0.5 * (q->conic[0] * dx * dx + q->conic[2] * dy * dy) - q->conic[1] * dx * dy;
          if (fabs(pw) < 1e-6) flag |= 4;
          if (pw > 0) { sig = mix64(sig, (uint64_t)(e * 4 + 1)); continue; }
          double araw = q->o * exp(pw);
          double al = araw < 0.99 ? araw : 0.99;
          /* relative change of alpha = change of the power when the mean and
             the conic are rounded to float32 (half an ulp, 2^-24 relative) */
          const double hu = 0x1p-24;
          double a_unc = 1e-5 + 2.0 * (fabs(q->conic[0] * dx + q->conic[1] * dy) * fabs(q->u) * hu +
                                       fabs(q->conic[2] * dy + q->conic[1] * dx) * fabs(q->v) * hu +
                                       (0.5 * fabs(q->conic[0]) * dx * dx + 0.5 * fabs(q->conic[2]) * dy * dy +
                                        fabs(q->conic[1] * dx * dy)) * hu);
          if (fabs(araw - 0.99) < a_unc * 0.99) flag |= 8;
          if (fabs(al - 1.0 / 255.0) < a_unc * (1.0 / 255.0)) flag |= 1;
          if (al < 1.0 / 255.0) { sig = mix64(sig, (uint64_t)(e * 4 + 1)); continue; }
          double tn = Tr * (1.0 - al);
          tr_unc += al / (1.0 - al) * (a_unc - 1e-5);
          if (fabs(tn - 1e-4) < (1e-5 + tr_unc) * 1e-4) flag |= 2;
          if (tn < 1e-4) { sig = mix64(sig, (uint64_t)(e * 4 + 2)); break; }
          for (int k = 0; k < C; k++) {
            Gp[k] += Tr * al * q->ch[k];
            Ga[k] += Tr * al * fabs(q->ch[k]);
          }
          Tr = tn;
          last = (int32_t)(e + 1);
          sig = mix64(sig, (uint64_t)(e * 4 + 3));
        }
        if (fabs((1.0 - Tr) - 1e-6) < 1e-5 * 1e-6) flag |= 16;
        if (out->gbuf) for (int k = 0; k < C; k++) out->gbuf[(size_t)k * H * W + pix] = Gp[k];
        if (out->gbuf_abs) for (int k = 0; k < C; k++) out->gbuf_abs[(size_t)k * H * W + pix] = Ga[k];
        if (out->alpha) out->alpha[pix] = 1.0 - Tr;
        if (out->n_contrib) out->n_contrib[pix] = last;
        if (out->pix_flag) out->pix_flag[pix] = flag;
        shade_pixel(cam, light, mlp, blend, C, F, Gp, Tr, uc, vc, S);
        if (out->net_margin) out->net_margin[pix] = (mlp && !S->background) ? S->margin : INFINITY;
        if (out->rgb_sens) {
          for (int c = 0; c < 3; c++) {
            double e[3] = {0, 0, 0}, dGs[MAXC];
            e[c] = 1.0;
            double dTs = shade_pixel_bwd(cam, light, mlp, blend, C, F, S, e, dGs, NULL) + bgc[c];
            double sacc = fabs(dTs) * Tr;
            for (int k = 0; k < C; k++) sacc += fabs(dGs[k]) * (fabs(Gp[k]) + Ga[k]);
            out->rgb_sens[(size_t)c * H * W + pix] = sacc;
          }
        }
        if (out->rgb)
          for (int c = 0; c < 3; c++) out->rgb[(size_t)c * H * W + pix] = S->a * S->L[c] * !S->background + Tr * bgc[c];
        if (!up) continue;
        /* ---- backward ---- */
        double gL[3], dG[MAXC];
        for (int c = 0; c < 3; c++) gL[c] = up->drgb ? up->drgb[(size_t)c * H * W + pix] : 0;
        double dT = shade_pixel_bwd(cam, light, mlp, blend, C, F, S, gL,
                                    dG, macc ? macc + (size_t)tid * np : NULL);
        if (up->dgbuf) for (int k = 0; k < C; k++) dG[k] += up->dgbuf[(size_t)k * H * W + pix];
        if (up->dalpha) dT -= up->dalpha[pix];
        for (int c = 0; c < 3; c++) dT += gL[c] * bgc[c]; /* rgb = ... + T_final background */
        /* reverse traversal: T before each contributor recovered by division */
        double Tcur = Tr, Sfx = 0; /* Sfx = sum over later contributors of w_j (dG . ch_j) */
        double *ga = gacc + ((size_t)tid * n) * GS;
        for (int64_t e = last - 1; e >= 0; e--) {
          const proj_t *q = &P[L[e].i];
          double dx = q->u - uc, dy = q->v - vc;
          double pw = -0.5 * (q->conic[0] * dx * dx + q->conic[2] * dy * dy) - q->conic[1] * dx * dy;
          if (pw > 0) continue;
          double ex = exp(pw);
          double araw = q->o * ex;
          double al = araw < 0.99 ? araw : 0.99;
          if (al < 1.0 / 255.0) continue;
          double Tb = Tcur / (1.0 - al);
          double wgt = Tb * al;
          double eg = 0;
          for (int k = 0; k < C; k++) eg += dG[k] * q->ch[k];
          double dal = Tb * eg - Sfx / (1.0 - al) - dT * Tr / (1.0 - al);
          Sfx += wgt * eg;
          Tcur = Tb;
          double *acc = ga + (size_t)L[e].i * GS;
          for (int k = 0; k < C; k++) acc[6 + k] += wgt * dG[k];
          if (araw < 0.99) {
            double dpw = dal * al;
            acc[5] += dal * ex;
            /* pw = -0.5 (A dx^2 + Cc dy^2) - B dx dy ; dx = u - uc */
            acc[0] += dpw * (-(q->conic[0] * dx + q->conic[1] * dy));
            acc[1] += dpw * (-(q->conic[2] * dy + q->conic[1] * dx));
            acc[2] += dpw * (-0.5 * dx * dx);
            acc[3] += dpw * (-dx * dy);
            acc[4] += dpw * (-0.5 * dy * dy);
          }
        }
      }
    sigs[t] = sig;
    free(Gp);
    free(Ga);
    free(S);
  }
  if (out->signature) {
    uint64_t s = 0;
    for (int t = 0; t < T; t++) s = mix64(s, sigs[t]);
    *out->signature = s;
  }

  if (up && gr) {
    /* reduce thread partials */
    for (int th = 1; th < nth; th++) {
      double *dst = gacc, *src = gacc + (size_t)th * n * GS;
      for (size_t k = 0; k < (size_t)n * GS; k++) dst[k] += src[k];
      if (macc) for (size_t k = 0; k < np; k++) macc[k] += macc[(size_t)th * np + k];
    }
    if (gr->mlp && mlp) for (size_t k = 0; k < np; k++) gr->mlp[k] = macc[k];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
      const proj_t *q = &P[i];
      double dmu[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dol = 0;
      double dch[MAXC];
      for (int k = 0; k < C; k++) dch[k] = 0;
      if (q->valid) {
        const double *acc = gacc + (size_t)i * GS;
        for (int k = 0; k < C; k++) dch[k] = acc[6 + k];
        double du = acc[0], dv = acc[1], dA = acc[2], dB = acc[3], dCc = acc[4], dop = acc[5];
        dol = dop * q->o * (1.0 - q->o);
        double dpc[3] = {0, 0, 0};
        const double fx = cam->fx, fy = cam->fy;
        double x = q->pc[0], y = q->pc[1], z = q->pc[2];
        /* mean2D */
        dpc[0] += du * fx / z;
        dpc[1] += dv * fy / z;
        dpc[2] += -du * fx * x / (z * z) - dv * fy * y / (z * z);
        /* depth channel */
        dpc[2] += dch[CH_DEPTH];
        /* conic (A,B,C) = (c,-b,a)/det */
        double a = q->a, b = q->b, c = q->c, det = q->det, d2 = det * det;
        double da = dA * (-c * c / d2) + dB * (b * c / d2) + dCc * (1.0 / det - a * c / d2);
        double db = dA * (2.0 * b * c / d2) + dB * (-1.0 / det - 2.0 * b * b / d2) + dCc * (2.0 * a * b / d2);
        double dc = dA * (1.0 / det - a * c / d2) + dB * (a * b / d2) + dCc * (-a * a / d2);
        /* Sigma' = J V J^T : G = dL/dSigma' (symmetric, off-diagonal db/2) */
        double Gm[4] = {da, 0.5 * db, 0.5 * db, dc};
        double dV[9], dJ[6];
        for (int r = 0; r < 3; r++)
          for (int s = 0; s < 3; s++) {
            double acc2 = 0;
            for (int u = 0; u < 2; u++)
              for (int v = 0; v < 2; v++) acc2 += q->J[3 * u + r] * Gm[2 * u + v] * q->J[3 * v + s];
            dV[3 * r + s] = acc2;
          }
        for (int u = 0; u < 2; u++)
          for (int r = 0; r < 3; r++) {
            double acc2 = 0;
            for (int v = 0; v < 2; v++)
              for (int s = 0; s < 3; s++) acc2 += 2.0 * Gm[2 * u + v] * q->J[3 * v + s] * q->V[3 * s + r];
            dJ[3 * u + r] = acc2;
          }
        /* J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]] */
        dpc[2] += dJ[0] * (-fx / (z * z)) + dJ[4] * (-fy / (z * z));
        if (!q->clx) { /* tx = x/z: J02 = -fx x / z^2 */
          dpc[0] += dJ[2] * (-fx / (z * z));
          dpc[2] += dJ[2] * (2.0 * fx * x / (z * z * z));
        } else {
          dpc[2] += dJ[2] * (fx * q->tx / (z * z));
        }
        if (!q->cly) {
          dpc[1] += dJ[5] * (-fy / (z * z));
          dpc[2] += dJ[5] * (2.0 * fy * y / (z * z * z));
        } else {
          dpc[2] += dJ[5] * (fy * q->ty / (z * z));
        }
        /* p_c = Rw mu + t */
        const double *Rw = cam->R;
        for (int k = 0; k < 3; k++) dmu[k] += Rw[k] * dpc[0] + Rw[3 + k] * dpc[1] + Rw[6 + k] * dpc[2];
        /* V = Rw Sigma Rw^T -> dSigma = Rw^T dV Rw */
        double dS[9], tmp[9];
        for (int r = 0; r < 3; r++)
          for (int s = 0; s < 3; s++) {
            double acc2 = 0;
            for (int k = 0; k < 3; k++) acc2 += Rw[3 * k + r] * dV[3 * k + s];
            tmp[3 * r + s] = acc2;
          }
        for (int r = 0; r < 3; r++)
          for (int s = 0; s < 3; s++) {
            double acc2 = 0;
            for (int k = 0; k < 3; k++) acc2 += tmp[3 * r + k] * Rw[3 * k + s];
            dS[3 * r + s] = acc2;
          }
        /* Sigma = M M^T, M = Rq diag(s): dM = (dS + dS^T) M */
        double Mm[9], dM[9];
        for (int r = 0; r < 3; r++)
          for (int k = 0; k < 3; k++) Mm[3 * r + k] = q->Rq[3 * r + k] * q->s[k];
        for (int r = 0; r < 3; r++)
          for (int k = 0; k < 3; k++) {
            double acc2 = 0;
            for (int s = 0; s < 3; s++) acc2 += (dS[3 * r + s] + dS[3 * s + r]) * Mm[3 * s + k];
            dM[3 * r + k] = acc2;
          }
        double dRq[9];
        for (int r = 0; r < 3; r++)
          for (int k = 0; k < 3; k++) dRq[3 * r + k] = dM[3 * r + k] * q->s[k];
        for (int k = 0; k < 3; k++) {
          double ds = 0;
          for (int r = 0; r < 3; r++) ds += dM[3 * r + k] * q->Rq[3 * r + k];
          dls[k] = ds * q->s[k];
        }
        /* normal channel = nsign * column kmin of Rq */
        for (int r = 0; r < 3; r++) dRq[3 * r + q->kmin] += q->nsign * dch[CH_NRM + r];
        double dqn[4];
        quat_to_rot_bwd(q->qn, dRq, dqn);
        double pdot = 0;
        for (int k = 0; k < 4; k++) pdot += q->qn[k] * dqn[k];
        for (int k = 0; k < 4; k++) dq[k] = (dqn[k] - q->qn[k] * pdot) / q->qlen;
        /* SH colour */
        if (g->sh_degree >= 0 && gr->sh) {
          double Y[16], JY[16][3], ddir[3] = {0, 0, 0};
          sh_basis(q->dir, Y);
          sh_basis_jac(q->dir, JY);
          for (int c = 0; c < 3; c++) {
            double dcol = q->shval[c] > 0 ? dch[CH_ALB + c] : 0;
            for (int k = 0; k < 16; k++) {
              gr->sh[(size_t)(k * 3 + c) * n + i] = dcol * Y[k];
              for (int j = 0; j < 3; j++) ddir[j] += dcol * g->sh[(k * 3 + c) * n + i] * JY[k][j];
            }
          }
          double ddr[3] = {0, 0, 0};
          normalize3_bwd(q->dirraw, q->dirlen, 1e-12, ddir, ddr);
          for (int k = 0; k < 3; k++) dmu[k] += ddr[k];
        }
      } else if (g->sh_degree >= 0 && gr->sh) {
        for (int k = 0; k < 48; k++) gr->sh[(size_t)k * n + i] = 0;
      }
      if (gr->means) for (int k = 0; k < 3; k++) gr->means[k * n + i] = dmu[k];
      if (gr->log_scales) for (int k = 0; k < 3; k++) gr->log_scales[k * n + i] = dls[k];
      if (gr->quats) for (int k = 0; k < 4; k++) gr->quats[k * n + i] = dq[k];
      if (gr->opacity_logits) gr->opacity_logits[i] = dol;
      if (gr->albedo) for (int c = 0; c < 3; c++) gr->albedo[c * n + i] = g->sh_degree >= 0 ? 0 : dch[CH_ALB + c];
      if (gr->roughness) gr->roughness[i] = dch[CH_ROUGH];
      if (gr->metallic) gr->metallic[i] = dch[CH_METAL];
      if (gr->sss) gr->sss[i] = dch[CH_SSS];
      if (gr->features) for (int f = 0; f < F; f++) gr->features[(size_t)f * n + i] = dch[CH_FEAT + f];
    }
  }
  free(wround);
  free(gacc);
  free(macc);
  free(sigs);
  free(lists);
  free(fill);
  free(cnt);
  free(P);
  return 0;
}
