// project.hip -- EWA projection of 3D Gaussians (Sec. 3.1, Eq. 1-2) and its
// backward.  One thread per Gaussian, structure-of-arrays loads.
//
// The geometry runs in FP64 registers (full rate on CDNA) and is stored as
// FP32.  That makes the integer decisions taken here -- radius, tile
// rectangle, float32 depth key -- reproducible by an FP64 reference.
#include "launch.hpp"

namespace sssgs {

// Real orthonormal SH basis, degrees 0..3 (no Condon-Shortley phase), at a
// unit direction; constants evaluated from their closed forms.
__device__ inline void sh_eval(double x, double y, double z, double *Y) {
  const double pi = 3.14159265358979323846;
  const double c0 = 0.5 * sqrt(1.0 / pi), c1 = sqrt(3.0 / (4.0 * pi));
  const double c2a = sqrt(15.0 / (4.0 * pi)), c2b = sqrt(5.0 / (16.0 * pi)), c2c = sqrt(15.0 / (16.0 * pi));
  const double c3a = sqrt(35.0 / (32.0 * pi)), c3b = sqrt(105.0 / (4.0 * pi)), c3c = sqrt(21.0 / (32.0 * pi));
  const double c3d = sqrt(7.0 / (16.0 * pi)), c3e = sqrt(105.0 / (16.0 * pi));
  const double xx = x * x, yy = y * y, zz = z * z;
  Y[0] = c0;
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  Y[4] = c2a * x * y;
  Y[5] = c2a * y * z;
  Y[6] = c2b * (3.0 * zz - 1.0);
  Y[7] = c2a * x * z;
  Y[8] = c2c * (xx - yy);
  Y[9] = c3a * y * (3.0 * xx - yy);
  Y[10] = c3b * x * y * z;
  Y[11] = c3c * y * (5.0 * zz - 1.0);
  Y[12] = c3d * z * (5.0 * zz - 3.0);
  Y[13] = c3c * x * (5.0 * zz - 1.0);
  Y[14] = c3e * z * (xx - yy);
  Y[15] = c3a * x * (xx - 3.0 * yy);
}

// Gradient of sum_k g_k Y_k(d) with respect to d (d treated as a free vector).
__device__ inline void sh_eval_grad(double x, double y, double z, const double *g, double *dd) {
  const double pi = 3.14159265358979323846;
  const double c1 = sqrt(3.0 / (4.0 * pi));
  const double c2a = sqrt(15.0 / (4.0 * pi)), c2b = sqrt(5.0 / (16.0 * pi)), c2c = sqrt(15.0 / (16.0 * pi));
  const double c3a = sqrt(35.0 / (32.0 * pi)), c3b = sqrt(105.0 / (4.0 * pi)), c3c = sqrt(21.0 / (32.0 * pi));
  const double c3d = sqrt(7.0 / (16.0 * pi)), c3e = sqrt(105.0 / (16.0 * pi));
  const double xx = x * x, yy = y * y, zz = z * z;
  double gx = 0, gy = 0, gz = 0;
  gy += g[1] * c1;
  gz += g[2] * c1;
  gx += g[3] * c1;
  gx += g[4] * c2a * y;  gy += g[4] * c2a * x;
  gy += g[5] * c2a * z;  gz += g[5] * c2a * y;
  gz += g[6] * c2b * 6.0 * z;
  gx += g[7] * c2a * z;  gz += g[7] * c2a * x;
  gx += g[8] * c2c * 2.0 * x;  gy -= g[8] * c2c * 2.0 * y;
  gx += g[9] * c3a * 6.0 * x * y;  gy += g[9] * c3a * 3.0 * (xx - yy);
  gx += g[10] * c3b * y * z;  gy += g[10] * c3b * x * z;  gz += g[10] * c3b * x * y;
  gy += g[11] * c3c * (5.0 * zz - 1.0);  gz += g[11] * c3c * 10.0 * y * z;
  gz += g[12] * c3d * (15.0 * zz - 3.0);
  gx += g[13] * c3c * (5.0 * zz - 1.0);  gz += g[13] * c3c * 10.0 * x * z;
  gx += g[14] * c3e * 2.0 * x * z;  gy -= g[14] * c3e * 2.0 * y * z;  gz += g[14] * c3e * (xx - yy);
  gx += g[15] * c3a * 3.0 * (xx - yy);  gy -= g[15] * c3a * 6.0 * x * y;
  dd[0] = gx; dd[1] = gy; dd[2] = gz;
}

// Everything the projection of one Gaussian produces (FP64).
struct Geo {
  bool valid;
  double px, py, pz;         // camera-space mean
  double s[3], qn[4], qlen;  // scales, unit quaternion, |q|
  double Rq[9];              // rotation of the Gaussian (row-major)
  double V[6];               // camera-space covariance (xx, xy, xz, yy, yz, zz)
  double J00, J02, J11, J12; // perspective Jacobian entries
  bool clx, cly;
  double tx, ty;
  double a, b, c, det;       // 2D covariance incl. +0.3
  double u, v;
  int r;
  int x0, y0, x1, y1;
  uint32_t key;
};

__device__ inline void rot_from_quat(const double *q, double *R) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// floor(v), clamped to [0, hi] before the conversion to int
__device__ inline int tile_floor(double v, int hi) { return (int)fmin(fmax(floor(v), 0.0), (double)hi); }

__device__ inline void project_geometry(const ProjIn &in, const CamArgs &cam, int i, Geo &G) {
  const int n = in.n;
  const double mx = in.means[i], my = in.means[n + i], mz = in.means[2 * n + i];
  G.px = fma((double)cam.R[0], mx, fma((double)cam.R[1], my, fma((double)cam.R[2], mz, (double)cam.t[0])));
  G.py = fma((double)cam.R[3], mx, fma((double)cam.R[4], my, fma((double)cam.R[5], mz, (double)cam.t[1])));
  G.pz = fma((double)cam.R[6], mx, fma((double)cam.R[7], my, fma((double)cam.R[8], mz, (double)cam.t[2])));
  G.valid = false;
  G.key = 0xFFFFFFFFu;
  G.r = 0;
  G.x0 = G.y0 = G.x1 = G.y1 = 0;
  if (!(G.pz > 0.2)) return;
  G.key = __float_as_uint(__double2float_rn(G.pz));
  for (int k = 0; k < 3; k++) G.s[k] = exp((double)in.log_scales[k * n + i]);
  double q[4];
  for (int k = 0; k < 4; k++) q[k] = in.quats[k * n + i];
  G.qlen = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; k++) G.qn[k] = q[k] / G.qlen;
  rot_from_quat(G.qn, G.Rq);
  // M = W Rq diag(s): camera-space factor of the covariance, V = M M^T
  double M[9];
  for (int r = 0; r < 3; r++)
    for (int k = 0; k < 3; k++)
      M[3 * r + k] = ((double)cam.R[3 * r] * G.Rq[k] + (double)cam.R[3 * r + 1] * G.Rq[3 + k] +
                      (double)cam.R[3 * r + 2] * G.Rq[6 + k]) * G.s[k];
  G.V[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  G.V[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  G.V[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  G.V[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  G.V[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  G.V[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  const double fx = cam.fx, fy = cam.fy, z = G.pz;
  const double limx = 1.3 * (0.5 * cam.W) / fx, limy = 1.3 * (0.5 * cam.H) / fy;
  const double rx = G.px / z, ry = G.py / z;
  G.clx = rx < -limx || rx > limx;
  G.cly = ry < -limy || ry > limy;
  G.tx = fmin(fmax(rx, -limx), limx);
  G.ty = fmin(fmax(ry, -limy), limy);
  G.J00 = fx / z;
  G.J02 = -fx * G.tx / z;
  G.J11 = fy / z;
  G.J12 = -fy * G.ty / z;
  // Sigma' = J V J^T with J = [[J00, 0, J02], [0, J11, J12]]
  const double t0x = G.J00 * G.V[0] + G.J02 * G.V[2];
  const double t0y = G.J00 * G.V[1] + G.J02 * G.V[4];
  const double t0z = G.J00 * G.V[2] + G.J02 * G.V[5];
  const double t1y = G.J11 * G.V[3] + G.J12 * G.V[4];
  const double t1z = G.J11 * G.V[4] + G.J12 * G.V[5];
  G.a = t0x * G.J00 + t0z * G.J02 + 0.3;
  G.b = t0y * G.J11 + t0z * G.J12;
  G.c = t1y * G.J11 + t1z * G.J12 + 0.3;
  G.det = G.a * G.c - G.b * G.b;
  if (!(G.det > 0.0)) return;
  const double mid = 0.5 * (G.a + G.c);
  const double lam = mid + sqrt(fmax(0.1, mid * mid - G.det));
  double rr = ceil(3.0 * sqrt(lam));
  if (rr > 1e9) rr = 1e9;
  G.r = (int)rr;
  G.u = fx * G.px / z + cam.cx;
  G.v = fy * G.py / z + cam.cy;
  G.x0 = tile_floor((G.u - rr) / kTile, cam.TX);
  G.y0 = tile_floor((G.v - rr) / kTile, cam.TY);
  G.x1 = tile_floor((G.u + rr + (kTile - 1)) / kTile, cam.TX);
  G.y1 = tile_floor((G.v + rr + (kTile - 1)) / kTile, cam.TY);
  G.valid = (G.x1 > G.x0) && (G.y1 > G.y0);
}

// Inclusive pixel bounds [x_lo, x_hi] x [y_lo, y_hi] outside of which the
// Gaussian's alpha stays below the 1/255 cut-off.  opacity e^power >= 1/255
// needs power >= -q with q = ln(255 opacity), an ellipse d^T Sigma^-1 d <= 2q
// whose half-extents are sqrt(2 q Sigma_xx) and sqrt(2 q Sigma_yy).  The bounds
// are widened by 1% + 1e-6 x the condition number of Sigma (the FP32 conic the
// compositing evaluates) and one pixel, so the FP32 decision can never fall
// outside them; empty (x_lo > x_hi) when no pixel can pass.
__device__ inline short4 alpha_box(const Geo &G, double opac) {
  const short4 empty = make_short4(32767, -32768, 32767, -32768);
  if (!G.valid || 255.0 * opac < 1.0 - 1e-6) return empty;
  const double q = fmax(log(255.0 * opac), 0.0);
  const double mid = 0.5 * (G.a + G.c), disc = sqrt(fmax(mid * mid - G.det, 0.0));
  const double lmax = mid + disc, lmin = G.det / lmax;
  const double grow = 1.01 + 1e-6 * lmax / lmin;
  const double ex = sqrt(2.0 * q * G.a) * grow + 1.0, ey = sqrt(2.0 * q * G.c) * grow + 1.0;
  auto clamp16 = [](double v) { return (short)fmin(fmax(v, -32768.0), 32767.0); };
  return make_short4(clamp16(ceil(G.u - ex - 0.5)), clamp16(floor(G.u + ex - 0.5)), clamp16(ceil(G.v - ey - 0.5)),
                     clamp16(floor(G.v + ey - 0.5)));
}

// Rq[3 r + k] for a run-time column k, by selects: an index into the array
// would send the whole array to scratch memory.
__device__ __forceinline__ double rq_col(const double *Rq, int r, int k) {
  return k == 0 ? Rq[3 * r] : (k == 1 ? Rq[3 * r + 1] : Rq[3 * r + 2]);
}

// Index of the smallest log-scale (first on ties) and the sign that turns
// that rotation axis toward the camera.
__device__ inline void normal_axis(const ProjIn &in, const CamArgs &cam, int i, const double *Rq, int &kmin,
                                   double &sign) {
  const int n = in.n;
  const float l0 = in.log_scales[i], l1 = in.log_scales[n + i], l2 = in.log_scales[2 * n + i];
  kmin = 0;
  float best = l0;
  if (l1 < best) { kmin = 1; best = l1; }
  if (l2 < best) { kmin = 2; }
  const double tc0 = cam.Cw[0] - (double)in.means[i];
  const double tc1 = cam.Cw[1] - (double)in.means[n + i];
  const double tc2 = cam.Cw[2] - (double)in.means[2 * n + i];
  const double d = rq_col(Rq, 0, kmin) * tc0 + rq_col(Rq, 1, kmin) * tc1 + rq_col(Rq, 2, kmin) * tc2;
  sign = d < 0.0 ? -1.0 : 1.0;
}

// One Gaussian: keys, values, rectangle, radius and culling box to memory,
// its record to the workgroup's LDS slot `sr` (zeros when it is culled).
template <int F, bool SH>
__device__ __forceinline__ void project_record(const ProjIn &in, const CamArgs &cam, int i, uint32_t *__restrict__ keys,
                                               uint32_t *__restrict__ vals, ushort4 *__restrict__ rects,
                                               int32_t *__restrict__ radii, short4 *__restrict__ boxes, float4 *sr) {
  constexpr int C = kChFeat + F;
  constexpr int RS = rec_stride(C);
  const int n = in.n;
  Geo G;
  project_geometry(in, cam, i, G);
  keys[i] = G.valid ? G.key : 0xFFFFFFFFu;
  vals[i] = (uint32_t)i;
  radii[i] = G.valid ? G.r : 0;
  rects[i] = G.valid ? make_ushort4((unsigned short)G.x0, (unsigned short)G.y0, (unsigned short)G.x1,
                                    (unsigned short)G.y1)
                     : make_ushort4(0, 0, 0, 0);
  const double opac = 1.0 / (1.0 + exp(-(double)in.opacity_logits[i]));
  boxes[i] = alpha_box(G, opac);
  if (!G.valid) {
#pragma unroll
    for (int k = 0; k < RS / 4; k++) sr[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  float rec[RS];
  rec[0] = (float)G.u;
  rec[1] = (float)G.v;
  rec[2] = (float)(G.c / G.det);
  rec[3] = (float)(-G.b / G.det);
  rec[4] = (float)(G.a / G.det);
  rec[5] = (float)opac;
  if (SH) {
    double d0 = (double)in.means[i] - cam.Cw[0], d1 = (double)in.means[n + i] - cam.Cw[1],
           d2 = (double)in.means[2 * n + i] - cam.Cw[2];
    const double dl = fmax(sqrt(d0 * d0 + d1 * d1 + d2 * d2), 1e-12);
    d0 /= dl; d1 /= dl; d2 /= dl;
    double Y[16];
    sh_eval(d0, d1, d2, Y);
    for (int c = 0; c < 3; c++) {
      double acc = 0.5;
      for (int k = 0; k < 16; k++) acc += Y[k] * (double)in.sh[(k * 3 + c) * n + i];
      rec[6 + kChAlb + c] = (float)fmax(acc, 0.0);
    }
  } else {
    for (int c = 0; c < 3; c++) rec[6 + kChAlb + c] = in.albedo[c * n + i];
  }
  int kmin;
  double sgn;
  normal_axis(in, cam, i, G.Rq, kmin, sgn);
  for (int r = 0; r < 3; r++) rec[6 + kChNrm + r] = (float)(sgn * rq_col(G.Rq, r, kmin));
  rec[6 + kChRough] = in.roughness[i];
  rec[6 + kChMetal] = in.metallic[i];
  rec[6 + kChSss] = in.sss[i];
  rec[6 + kChDepth] = __uint_as_float(G.key);
#pragma unroll
  for (int f = 0; f < F; f++) rec[6 + kChFeat + f] = in.features[f * n + i];
#pragma unroll
  for (int k = 6 + C; k < RS; k++) rec[k] = 0.f;
#pragma unroll
  for (int k = 0; k < RS; k += 4) sr[k / 4] = make_float4(rec[k], rec[k + 1], rec[k + 2], rec[k + 3]);
}

template <int F, bool SH>
__global__ __launch_bounds__(256) void project_fwd_kernel(ProjIn in, CamArgs cam, float *__restrict__ records,
                                                          uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                          ushort4 *__restrict__ rects, int32_t *__restrict__ radii,
                                                          short4 *__restrict__ boxes) {
  // the workgroup's records are staged in LDS and written out coalesced
  // (consecutive threads, consecutive 16-byte chunks): a thread writing its
  // own 128-byte record with 16-byte stores spread every store over 64 lines
  constexpr int RS = rec_stride(kChFeat + F);
  __shared__ float4 srec[256 * (RS / 4)];
  const int i0 = blockIdx.x * blockDim.x, i = i0 + threadIdx.x;
  const int nv = min(256, in.n - i0);
  if (i < in.n) project_record<F, SH>(in, cam, i, keys, vals, rects, radii, boxes, srec + threadIdx.x * (RS / 4));
  __syncthreads();
  float4 *dst = reinterpret_cast<float4 *>(records + (size_t)i0 * RS);
  for (int k = threadIdx.x; k < nv * (RS / 4); k += 256) dst[k] = srec[k];
}

__device__ __forceinline__ void put(float *p, int idx, double v, int acc) {
  if (!p) return;
  if (acc) p[idx] += (float)v;
  else p[idx] = (float)v;
}

// Backward of the projection: from the per-Gaussian accumulators
// [du, dv, dconic_a, dconic_b, dconic_c, dopacity | dchannels] to the
// parameter gradients.
template <int F, bool SH>
__global__ __launch_bounds__(256) void project_bwd_kernel(ProjIn in, CamArgs cam, const float *__restrict__ gacc,
                                                          ProjGradOut out) {
  constexpr int C = kChFeat + F;
  constexpr int GS = grad_stride(C);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= in.n) return;
  const int n = in.n, acc = out.accumulate;
  Geo G;
  project_geometry(in, cam, i, G);
  double dmu[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dlogit = 0;
  float dch[C];
#pragma unroll
  for (int k = 0; k < C; k++) dch[k] = 0.f;
  double shg[48];
  if (SH)
    for (int k = 0; k < 48; k++) shg[k] = 0;
  if (G.valid) {
    const float *ga = gacc + (size_t)i * GS;
    const double du = ga[0], dv = ga[1], dA = ga[2], dB = ga[3], dC = ga[4], dop = ga[5];
#pragma unroll
    for (int k = 0; k < C; k++) dch[k] = ga[6 + k];
    const double o = 1.0 / (1.0 + exp(-(double)in.opacity_logits[i]));
    dlogit = dop * o * (1.0 - o);
    const double fx = cam.fx, fy = cam.fy, x = G.px, y = G.py, z = G.pz, iz = 1.0 / z;
    double gx = du * fx * iz, gy = dv * fy * iz;
    double gz = -(du * fx * x + dv * fy * y) * iz * iz + (double)dch[kChDepth];
    // conic = (c, -b, a) / det
    const double a = G.a, b = G.b, c = G.c, det = G.det, id = 1.0 / det, id2 = id * id;
    const double da = -dA * c * c * id2 + dB * b * c * id2 + dC * (id - a * c * id2);
    const double db = 2.0 * dA * b * c * id2 - dB * (id + 2.0 * b * b * id2) + 2.0 * dC * a * b * id2;
    const double dc = dA * (id - a * c * id2) + dB * a * b * id2 - dC * a * a * id2;
    // Sigma' = J V J^T; symmetric upstream Gm = [[da, db/2], [db/2, dc]]
    const double g00 = da, g01 = 0.5 * db, g11 = dc;
    // dV = J^T Gm J (symmetric 3x3; J row0 = (J00, 0, J02), row1 = (0, J11, J12))
    const double J00 = G.J00, J02 = G.J02, J11 = G.J11, J12 = G.J12;
    double dV[9];
    {
      const double jr[3][2] = {{J00, 0.0}, {0.0, J11}, {J02, J12}};  // column r of J = (J[0][r], J[1][r])
      for (int r = 0; r < 3; r++)
        for (int s = 0; s < 3; s++) {
          const double u0 = jr[r][0], u1 = jr[r][1], w0 = jr[s][0], w1 = jr[s][1];
          dV[3 * r + s] = u0 * (g00 * w0 + g01 * w1) + u1 * (g01 * w0 + g11 * w1);
        }
    }
    // dJ = 2 Gm J V (only the entries J00, J02, J11, J12 are free)
    {
      const double Vf[9] = {G.V[0], G.V[1], G.V[2], G.V[1], G.V[3], G.V[4], G.V[2], G.V[4], G.V[5]};
      // (J V) rows
      double JV0[3], JV1[3];
      for (int s = 0; s < 3; s++) {
        JV0[s] = J00 * Vf[s] + J02 * Vf[6 + s];
        JV1[s] = J11 * Vf[3 + s] + J12 * Vf[6 + s];
      }
      const double dJ00 = 2.0 * (g00 * JV0[0] + g01 * JV1[0]);
      const double dJ02 = 2.0 * (g00 * JV0[2] + g01 * JV1[2]);
      const double dJ11 = 2.0 * (g01 * JV0[1] + g11 * JV1[1]);
      const double dJ12 = 2.0 * (g01 * JV0[2] + g11 * JV1[2]);
      gz += -dJ00 * fx * iz * iz - dJ11 * fy * iz * iz;
      if (!G.clx) {
        gx += -dJ02 * fx * iz * iz;
        gz += 2.0 * dJ02 * fx * x * iz * iz * iz;
      } else {
        gz += dJ02 * fx * G.tx * iz * iz;
      }
      if (!G.cly) {
        gy += -dJ12 * fy * iz * iz;
        gz += 2.0 * dJ12 * fy * y * iz * iz * iz;
      } else {
        gz += dJ12 * fy * G.ty * iz * iz;
      }
    }
    // p_cam = W mu + t
    for (int k = 0; k < 3; k++) dmu[k] += cam.R[k] * gx + cam.R[3 + k] * gy + cam.R[6 + k] * gz;
    // V = W Sigma W^T  ->  dSigma = W^T dV W
    double dS[9];
    for (int r = 0; r < 3; r++)
      for (int s = 0; s < 3; s++) {
        double t = 0;
        for (int k = 0; k < 3; k++)
          for (int l = 0; l < 3; l++) t += (double)cam.R[3 * k + r] * dV[3 * k + l] * (double)cam.R[3 * l + s];
        dS[3 * r + s] = t;
      }
    // Sigma = Rq diag(s^2) Rq^T:  with N = Rq diag(s), dN = (dS + dS^T) N
    double dRq[9];
    for (int r = 0; r < 3; r++)
      for (int k = 0; k < 3; k++) {
        double t = 0;
        for (int s = 0; s < 3; s++) t += (dS[3 * r + s] + dS[3 * s + r]) * G.Rq[3 * s + k] * G.s[k];
        dRq[3 * r + k] = t * G.s[k];
        dls[k] += t * G.Rq[3 * r + k] * G.s[k];
      }
    // normal channel: column kmin of Rq, signed toward the camera
    int kmin;
    double sgn;
    normal_axis(in, cam, i, G.Rq, kmin, sgn);
    for (int r = 0; r < 3; r++)
#pragma unroll
      for (int k = 0; k < 3; k++)
        if (k == kmin) dRq[3 * r + k] += sgn * (double)dch[kChNrm + r];
    // Rq(qn) -> dqn
    const double w = G.qn[0], qx = G.qn[1], qy = G.qn[2], qz = G.qn[3];
    double dqn[4];
    dqn[0] = 2.0 * (-qz * dRq[1] + qy * dRq[2] + qz * dRq[3] - qx * dRq[5] - qy * dRq[6] + qx * dRq[7]);
    dqn[1] = 2.0 * (qy * dRq[1] + qz * dRq[2] + qy * dRq[3] - 2.0 * qx * dRq[4] - w * dRq[5] + qz * dRq[6] +
                    w * dRq[7] - 2.0 * qx * dRq[8]);
    dqn[2] = 2.0 * (-2.0 * qy * dRq[0] + qx * dRq[1] + w * dRq[2] + qx * dRq[3] + qz * dRq[5] - w * dRq[6] +
                    qz * dRq[7] - 2.0 * qy * dRq[8]);
    dqn[3] = 2.0 * (-2.0 * qz * dRq[0] - w * dRq[1] + qx * dRq[2] + w * dRq[3] - 2.0 * qz * dRq[4] +
                    qy * dRq[5] + qx * dRq[6] + qy * dRq[7]);
    const double pd = G.qn[0] * dqn[0] + G.qn[1] * dqn[1] + G.qn[2] * dqn[2] + G.qn[3] * dqn[3];
    for (int k = 0; k < 4; k++) dq[k] = (dqn[k] - G.qn[k] * pd) / G.qlen;
    if (SH) {
      double e0 = (double)in.means[i] - cam.Cw[0], e1 = (double)in.means[n + i] - cam.Cw[1],
             e2 = (double)in.means[2 * n + i] - cam.Cw[2];
      const double el = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
      const double ed = fmax(el, 1e-12);
      const double d0 = e0 / ed, d1 = e1 / ed, d2 = e2 / ed;
      double Y[16];
      sh_eval(d0, d1, d2, Y);
      double gk[16];
      for (int k = 0; k < 16; k++) gk[k] = 0;
      for (int c = 0; c < 3; c++) {
        double accv = 0.5;
        for (int k = 0; k < 16; k++) accv += Y[k] * (double)in.sh[(k * 3 + c) * n + i];
        const double dcol = accv > 0.0 ? (double)dch[kChAlb + c] : 0.0;
        for (int k = 0; k < 16; k++) {
          shg[k * 3 + c] = dcol * Y[k];
          gk[k] += dcol * (double)in.sh[(k * 3 + c) * n + i];
        }
      }
      double dd[3];
      sh_eval_grad(d0, d1, d2, gk, dd);
      if (el > 1e-12) {
        const double p = d0 * dd[0] + d1 * dd[1] + d2 * dd[2];
        dmu[0] += (dd[0] - d0 * p) / el;
        dmu[1] += (dd[1] - d1 * p) / el;
        dmu[2] += (dd[2] - d2 * p) / el;
      } else {
        for (int k = 0; k < 3; k++) dmu[k] += dd[k] / 1e-12;
      }
    }
  }
  for (int k = 0; k < 3; k++) put(out.means, k * n + i, dmu[k], acc);
  for (int k = 0; k < 3; k++) put(out.log_scales, k * n + i, dls[k], acc);
  for (int k = 0; k < 4; k++) put(out.quats, k * n + i, dq[k], acc);
  put(out.opacity_logits, i, dlogit, acc);
  if (!SH)
    for (int c = 0; c < 3; c++) put(out.albedo, c * n + i, dch[kChAlb + c], acc);
  put(out.roughness, i, dch[kChRough], acc);
  put(out.metallic, i, dch[kChMetal], acc);
  put(out.sss, i, dch[kChSss], acc);
  for (int f = 0; f < F; f++) put(out.features, f * n + i, dch[kChFeat + f], acc);
  if (SH)
    for (int k = 0; k < 48; k++) put(out.sh, k * n + i, shg[k], acc);
}

// Host-side launchers (declared in launch.hpp).
template <int F, bool SH>
void launch_project_fwd_t(const ProjIn &in, const CamArgs &cam, float *records, uint32_t *keys, uint32_t *vals,
                          ushort4 *rects, int32_t *radii, short4 *boxes, hipStream_t st) {
  if (in.n == 0) return;
  project_fwd_kernel<F, SH><<<(in.n + 255) / 256, 256, 0, st>>>(in, cam, records, keys, vals, rects, radii, boxes);
}

template <int F, bool SH>
void launch_project_bwd_t(const ProjIn &in, const CamArgs &cam, const float *gacc, const ProjGradOut &out,
                          hipStream_t st) {
  if (in.n == 0) return;
  project_bwd_kernel<F, SH><<<(in.n + 255) / 256, 256, 0, st>>>(in, cam, gacc, out);
}

#define SSSGS_PROJ_INST(F, SH)                                                                              \
  template void launch_project_fwd_t<F, SH>(const ProjIn &, const CamArgs &, float *, uint32_t *, uint32_t *, \
                                            ushort4 *, int32_t *, short4 *, hipStream_t);                   \
  template void launch_project_bwd_t<F, SH>(const ProjIn &, const CamArgs &, const float *,                 \
                                            const ProjGradOut &, hipStream_t);
SSSGS_PROJ_INST(0, false)
SSSGS_PROJ_INST(8, false)
SSSGS_PROJ_INST(16, false)
SSSGS_PROJ_INST(32, false)
SSSGS_PROJ_INST(0, true)
SSSGS_PROJ_INST(8, true)
SSSGS_PROJ_INST(16, true)
SSSGS_PROJ_INST(32, true)

}  // namespace sssgs
