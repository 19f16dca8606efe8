// gmlp.hip -- the per-Gaussian network of the pipeline figure (Eq. 6
// evaluated for each Gaussian, Sec. 3.2; layer sizes from the appendix
// "Network"), forward and backward, FP32.
//
// Input, 42 values per Gaussian: normal (shortest rotation axis turned toward
// the camera) 3 | unit quaternion 4 | scale 3 | direction to the light 3 |
// direction to the camera 3 | light distance 1 | visibility 1 | sin, cos of
// 2^k pi mu for k = 0..3 (24).  Trunk 64-32-32 with Leaky-ReLU (slope 0.01);
// incident-light head 32 (Leaky-ReLU) -> 3 (ReLU); SSS head -> 3 (sigmoid).
// Output: eight feature planes [8][n] = L_in (3) | L_sss (3) | v | 1, which
// the projection and compositing blend like any other channel.
//
// One lane per Gaussian, one wave per workgroup.  Weights are wave-uniform and
// come through scalar loads: the forward walks the layer input (rolled loop
// over the input index, the input read from the lane's own LDS column) and
// keeps all outputs of the layer in registers, which needs the weights
// transposed ([cols][rows], prepared once per call); the backward walks the
// output gradient the same way with the weights as stored ([rows][cols]).
// The weight gradient sum_g dz[o][g] act[i][g] is a 16x16x4 FP32
// matrix-core product with K = Gaussians over records the backward stores
// (see the backward section); every wave keeps its sums in registers over
// its chunks and writes one partial row, reduced in fixed order afterwards.
#include "launch.hpp"

namespace sssgs {

namespace {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kGIn = 42;
constexpr float kSlope = 0.01f;
constexpr int kLS = 64;  // LDS row stride (floats) of the per-lane columns (lane l: word row * kLS + l)

// Packed parameter layout: per layer W [rows][cols] then b [rows].
struct GL { int rows, cols, w, b; };
constexpr GL mk(int rows, int cols, int off) { return GL{rows, cols, off, off + rows * cols}; }
constexpr GL kL0 = mk(64, kGIn, 0);
constexpr GL kL1 = mk(32, 64, kL0.b + 64);
constexpr GL kL2 = mk(32, 32, kL1.b + 32);
constexpr GL kLi = mk(32, 32, kL2.b + 32);
constexpr GL kLl = mk(3, 32, kLi.b + 32);
constexpr GL kLs = mk(3, 32, kLl.b + 3);
constexpr int kGParams = kLs.b + 3;
static_assert(kGParams == 7142, "per-Gaussian network parameter count");

// Weights and biases are read through the constant address space: with a
// wave-uniform index the compiler issues scalar loads (SGPR operands of the
// FMAs) instead of per-lane vector loads.
typedef const __attribute__((address_space(4))) float *cptr;
__device__ __forceinline__ cptr as_const(const float *p) { return (cptr)p; }

__device__ __forceinline__ float lrelu(float z) { return z > 0.f ? z : kSlope * z; }

// acc[r] = b[r] + sum_i W[r][i] in[i]; wt = W transposed ([COLS][ROWS]),
// in = the lane's LDS column (row stride kLS).
template <int ROWS, int COLS>
__device__ __forceinline__ void layer_fwd(cptr wt, cptr b, const float *in, float (&acc)[ROWS]) {
#pragma unroll
  for (int r = 0; r < ROWS; r++) acc[r] = b[r];
#pragma unroll 2
  for (int i = 0; i < COLS; i++) {
    const float xi = in[i * kLS];
#pragma unroll
    for (int r = 0; r < ROWS; r++) acc[r] = __fmaf_rn(wt[i * ROWS + r], xi, acc[r]);
  }
}

// d[c] = sum_r W[r][c] dz[r]; W as stored ([ROWS][COLS]), dz = the lane's LDS column.
template <int ROWS, int COLS>
__device__ __forceinline__ void layer_bwd(cptr w, const float *dz, float (&d)[COLS]) {
#pragma unroll
  for (int c = 0; c < COLS; c++) d[c] = 0.f;
#pragma unroll 2
  for (int r = 0; r < ROWS; r++) {
    const float g = dz[r * kLS];
#pragma unroll
    for (int c = 0; c < COLS; c++) d[c] = __fmaf_rn(w[r * COLS + c], g, d[c]);
  }
}

template <int N>
__device__ __forceinline__ void put_col(float *col, int row0, const float (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; k++) col[(row0 + k) * kLS] = v[k];
}

// The per-Gaussian quantities the input vector and its backward are built from.
struct GIn {
  float mu[3], qn[4], qlen, s[3], wi[3], dl, wo[3], dc, v, sign, nrm[3];
  int kmin;
};

__device__ __forceinline__ void gaussian_input(const GmlpArgs &A, int i, GIn &G) {
  const int n = A.n;
  for (int k = 0; k < 3; k++) G.mu[k] = A.means[k * n + i];
  float q[4];
  for (int k = 0; k < 4; k++) q[k] = A.quats[k * n + i];
  G.qlen = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; k++) G.qn[k] = q[k] / G.qlen;
  const float w = G.qn[0], x = G.qn[1], y = G.qn[2], z = G.qn[3];
  float R[9];
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
  float ls[3];
  for (int k = 0; k < 3; k++) ls[k] = A.log_scales[k * n + i];
  // shortest axis: first minimum of the log-scales
  G.kmin = 0;
  float best = ls[0];
  if (ls[1] < best) { G.kmin = 1; best = ls[1]; }
  if (ls[2] < best) G.kmin = 2;
  for (int k = 0; k < 3; k++) G.s[k] = expf(ls[k]);
  // side of the camera in FP64 (the sign is a decision; keep its margin small)
  {
    double qd[4], ql = 0.0;
    for (int k = 0; k < 4; k++) { qd[k] = q[k]; ql += qd[k] * qd[k]; }
    ql = sqrt(ql);
    for (int k = 0; k < 4; k++) qd[k] /= ql;
    const double W_ = qd[0], X = qd[1], Y = qd[2], Z = qd[3];
    double col[3];
    if (G.kmin == 0) { col[0] = 1.0 - 2.0 * (Y * Y + Z * Z); col[1] = 2.0 * (X * Y + W_ * Z); col[2] = 2.0 * (X * Z - W_ * Y); }
    else if (G.kmin == 1) { col[0] = 2.0 * (X * Y - W_ * Z); col[1] = 1.0 - 2.0 * (X * X + Z * Z); col[2] = 2.0 * (Y * Z + W_ * X); }
    else { col[0] = 2.0 * (X * Z + W_ * Y); col[1] = 2.0 * (Y * Z - W_ * X); col[2] = 1.0 - 2.0 * (X * X + Y * Y); }
    double d = 0.0;
    for (int k = 0; k < 3; k++) d += col[k] * ((double)A.cam[k] - (double)G.mu[k]);
    G.sign = d < 0.0 ? -1.f : 1.f;
  }
  // column kmin of R by 0/1 weights (exact; no indexing by kmin)
  const float m0 = G.kmin == 0 ? 1.f : 0.f, m1 = G.kmin == 1 ? 1.f : 0.f, m2 = G.kmin == 2 ? 1.f : 0.f;
  for (int k = 0; k < 3; k++) G.nrm[k] = G.sign * (m0 * R[3 * k] + m1 * R[3 * k + 1] + m2 * R[3 * k + 2]);
  float u[3], uo[3];
  for (int k = 0; k < 3; k++) {
    u[k] = A.light[k] - G.mu[k];
    uo[k] = A.cam[k] - G.mu[k];
  }
  G.dl = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  G.dc = sqrtf(uo[0] * uo[0] + uo[1] * uo[1] + uo[2] * uo[2]);
  const float il = 1.f / fmaxf(G.dl, 1e-12f), ic = 1.f / fmaxf(G.dc, 1e-12f);
  for (int k = 0; k < 3; k++) {
    G.wi[k] = u[k] * il;
    G.wo[k] = uo[k] * ic;
  }
  G.v = A.vis[i];
}

// The 42 input values into the lane's LDS column (rows row0 ..).
__device__ __forceinline__ void write_input(const GIn &G, float *col, int row0) {
  float *c = col + row0 * kLS;
  for (int k = 0; k < 3; k++) c[k * kLS] = G.nrm[k];
  for (int k = 0; k < 4; k++) c[(3 + k) * kLS] = G.qn[k];
  for (int k = 0; k < 3; k++) c[(7 + k) * kLS] = G.s[k];
  for (int k = 0; k < 3; k++) c[(10 + k) * kLS] = G.wi[k];
  for (int k = 0; k < 3; k++) c[(13 + k) * kLS] = G.wo[k];
  c[16 * kLS] = G.dl;
  c[17 * kLS] = G.v;
#pragma unroll
  for (int oct = 0; oct < 4; oct++) {
    const float sc = (float)(1 << oct);
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
      c[(18 + 6 * oct + ax) * kLS] = sinpif(sc * G.mu[ax]);
      c[(21 + 6 * oct + ax) * kLS] = cospif(sc * G.mu[ax]);
    }
  }
}

// ------------------------------------------------------------------ records
//
// The forward stores, unit-major ([row][ldn], ldn = n rounded up to 64), every
// layer's input activations, the heads' pre-activations and the Leaky-ReLU
// signs as bit masks; the backward reads them instead of recomputing the
// network, and the weight-gradient kernel streams them.

// Activation rows (layer inputs) and output-gradient rows of the records.
// Rows kAZ.. hold the heads' pre-activations (incident 3, SSS 3).
constexpr int kAX = 0, kAH1 = 42, kAH2 = 106, kAH3 = 138, kAE = 170, kAZ = 202, kARows = 208;
constexpr int kMaskRows = 5;  // Leaky-ReLU signs: h1 (two words), h2, h3, e
constexpr int kD0 = 0, kD1 = 64, kD2 = 96, kDI = 128, kDH = 160, kDRows = 166;

template <int N>
__device__ __forceinline__ void put_rows(float *rec, int row0, size_t ldn, size_t g, const float (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; k++) rec[(row0 + k) * ldn + g] = v[k];
}

template <int N>
__device__ __forceinline__ uint64_t sign_mask(const float (&z)[N]) {
  uint64_t m = 0;
#pragma unroll
  for (int k = 0; k < N; k++) m |= (z[k] > 0.f ? 1ull : 0ull) << k;
  return m;
}

__device__ __forceinline__ float slope(uint64_t m, int k) { return (m >> k) & 1ull ? 1.f : kSlope; }

// ------------------------------------------------------------------ forward

// Rows of the forward's LDS column: the layer input (up to 64 rows) and, for
// the heads, the trunk output at 0..31 and the incident hidden layer at 32..63.
__global__ __launch_bounds__(64) void gmlp_fwd_kernel(GmlpArgs A) {
  __shared__ float lds[64 * kLS];
  const int lane = threadIdx.x;
  const int i = blockIdx.x * 64 + lane;
  const bool live = i < A.n;
  const int gi = live ? i : 0;
  float *col = lds + lane;
  const cptr wt = as_const(A.wt), P = as_const(A.params);
  const bool rec = A.act != nullptr;  // keep the backward's records
  const size_t ldn = A.ldn;
  float *act = A.act;
  GIn G;
  gaussian_input(A, gi, G);
  write_input(G, col, 0);
  if (rec)
#pragma unroll
    for (int k = 0; k < kGIn; k++) act[(kAX + k) * ldn + i] = col[k * kLS];
  uint64_t m1, m2, m3, me;
  {
    float h[64];
    layer_fwd<64, kGIn>(wt + kL0.w, P + kL0.b, col, h);
    m1 = sign_mask(h);
#pragma unroll
    for (int k = 0; k < 64; k++) h[k] = lrelu(h[k]);
    put_col(col, 0, h);
    if (rec) put_rows(act, kAH1, ldn, i, h);
  }
  {
    float h[32];
    layer_fwd<32, 64>(wt + kL1.w, P + kL1.b, col, h);
    m2 = sign_mask(h);
#pragma unroll
    for (int k = 0; k < 32; k++) h[k] = lrelu(h[k]);
    put_col(col, 0, h);
    if (rec) put_rows(act, kAH2, ldn, i, h);
    layer_fwd<32, 32>(wt + kL2.w, P + kL2.b, col, h);
    m3 = sign_mask(h);
#pragma unroll
    for (int k = 0; k < 32; k++) h[k] = lrelu(h[k]);
    put_col(col, 0, h);   // trunk output
    if (rec) put_rows(act, kAH3, ldn, i, h);
    layer_fwd<32, 32>(wt + kLi.w, P + kLi.b, col, h);
    me = sign_mask(h);
#pragma unroll
    for (int k = 0; k < 32; k++) h[k] = lrelu(h[k]);
    put_col(col, 32, h);  // incident head, hidden
    if (rec) put_rows(act, kAE, ldn, i, h);
  }
  float zl[3], zs[3];
  layer_fwd<3, 32>(wt + kLl.w, P + kLl.b, col + 32 * kLS, zl);
  layer_fwd<3, 32>(wt + kLs.w, P + kLs.b, col, zs);
  if (rec) {
    const float z[6] = {zl[0], zl[1], zl[2], zs[0], zs[1], zs[2]};
    put_rows(act, kAZ, ldn, i, z);
    const uint32_t mw[kMaskRows] = {(uint32_t)m1, (uint32_t)(m1 >> 32), (uint32_t)m2, (uint32_t)m3, (uint32_t)me};
    for (int k = 0; k < kMaskRows; k++) A.masks[k * ldn + i] = mw[k];
  }
  if (live) {
    const size_t n = A.n;
    for (int c = 0; c < 3; c++) {
      A.feat[c * n + i] = fmaxf(zl[c], 0.f);
      A.feat[(3 + c) * n + i] = 1.f / (1.f + expf(-zs[c]));
    }
    A.feat[6 * n + i] = G.v;
    A.feat[7 * n + i] = 1.f;
  }
}

// Transposed copy of every weight matrix (same offsets), biases copied.
__global__ __launch_bounds__(256) void gmlp_prep_kernel(const float *__restrict__ params, float *__restrict__ wt) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kGParams) return;
  const GL Ls[6] = {kL0, kL1, kL2, kLi, kLl, kLs};
  for (int l = 0; l < 6; l++) {
    const GL L = Ls[l];
    if (p >= L.w && p < L.b) {
      const int r = (p - L.w) / L.cols, c = (p - L.w) % L.cols;
      wt[L.w + c * L.rows + r] = params[p];
      return;
    }
  }
  wt[p] = params[p];
}

// ----------------------------------------------------------------- backward
//
// Two kernels.  gmlp_bwd_kernel: one lane per Gaussian (high occupancy: one
// 64-row LDS column per lane); from the forward's records (signs and head
// pre-activations) it runs the backward through the layers and the chain to
// the Gaussian parameters, and stores every layer's output gradients
// unit-major ([unit][ldn]; lanes past n store zeros).  gmlp_wgrad_kernel:
// the weight gradients sum_g dz[o][g] a[i][g] on the matrix cores, streaming
// those records; one layer group per grid row.



__global__ __launch_bounds__(64) void gmlp_bwd_kernel(GmlpArgs A) {
  __shared__ float lds[64 * kLS];
  const int lane = threadIdx.x;
  const int i = blockIdx.x * 64 + lane;  // < ldn: the grid covers ldn / 64 blocks
  const bool live = i < A.n;
  const int gi = live ? i : 0;
  float *col = lds + lane;
  const cptr P = as_const(A.params);
  const size_t n = A.n, ldn = A.ldn;
  const float *act = A.act;
  float *dzr = A.dz;
  // ---- the forward's records: Leaky-ReLU signs and the heads' pre-activations
  const uint64_t m1 = (uint64_t)A.masks[i] | ((uint64_t)A.masks[ldn + i] << 32);
  const uint64_t m2 = A.masks[2 * ldn + i], m3 = A.masks[3 * ldn + i], me = A.masks[4 * ldn + i];
  float zl[3], lsss[3];
  for (int c = 0; c < 3; c++) {
    zl[c] = act[(kAZ + c) * ldn + i];
    lsss[c] = 1.f / (1.f + expf(-act[(kAZ + 3 + c) * ldn + i]));
  }
  // ---- backward
  float df[8];
  for (int c = 0; c < 8; c++) df[c] = live ? A.dfeat[c * n + i] : 0.f;
  float dzl[3], dzs[3];
  for (int c = 0; c < 3; c++) {
    dzl[c] = zl[c] > 0.f ? df[c] : 0.f;
    dzs[c] = df[3 + c] * lsss[c] * (1.f - lsss[c]);
  }
  {
    float hd[6] = {dzl[0], dzl[1], dzl[2], dzs[0], dzs[1], dzs[2]};
    put_rows(dzr, kDH, ldn, i, hd);
  }
  float dh3[32];
  {
    float dzi[32];
#pragma unroll
    for (int c = 0; c < 32; c++) {
      float d = 0.f, e = 0.f;
#pragma unroll
      for (int o = 0; o < 3; o++) {
        d = __fmaf_rn(P[kLl.w + o * 32 + c], dzl[o], d);
        e = __fmaf_rn(P[kLs.w + o * 32 + c], dzs[o], e);
      }
      dzi[c] = d * slope(me, c);
      dh3[c] = e;
    }
    put_col(col, 0, dzi);
    put_rows(dzr, kDI, ldn, i, dzi);
  }
  {
    float d[32];
    layer_bwd<32, 32>(P + kLi.w, col, d);
#pragma unroll
    for (int c = 0; c < 32; c++) d[c] = (dh3[c] + d[c]) * slope(m3, c);
    put_col(col, 0, d);  // dz2
    put_rows(dzr, kD2, ldn, i, d);
  }
  {
    float d[32];
    layer_bwd<32, 32>(P + kL2.w, col, d);
#pragma unroll
    for (int c = 0; c < 32; c++) d[c] *= slope(m2, c);
    put_col(col, 0, d);  // dz1
    put_rows(dzr, kD1, ldn, i, d);
  }
  {
    float d[64];
    layer_bwd<32, 64>(P + kL1.w, col, d);
#pragma unroll
    for (int c = 0; c < 64; c++) d[c] *= slope(m1, c);
    put_col(col, 0, d);  // dz0
    put_rows(dzr, kD0, ldn, i, d);
  }
  // ---- input gradient and the chain to the Gaussian parameters
  float dx[kGIn];
  layer_bwd<64, kGIn>(P + kL0.w, col, dx);
  if (!live) return;
  // the input's building blocks again (cheaper than keeping them live)
  GIn G;
  gaussian_input(A, gi, G);
  float dmu[3] = {0.f, 0.f, 0.f};
  // w_in = u / |u| and d = |u| with u = light - mu
  {
    const float p = G.wi[0] * dx[10] + G.wi[1] * dx[11] + G.wi[2] * dx[12];
    const float il = 1.f / G.dl;
    for (int k = 0; k < 3; k++) dmu[k] -= (dx[10 + k] - G.wi[k] * p) * il + dx[16] * G.wi[k];
  }
  {
    const float p = G.wo[0] * dx[13] + G.wo[1] * dx[14] + G.wo[2] * dx[15];
    const float ic = 1.f / G.dc;
    for (int k = 0; k < 3; k++) dmu[k] -= (dx[13 + k] - G.wo[k] * p) * ic;
  }
#pragma unroll
  for (int oct = 0; oct < 4; oct++) {
    const float sc = (float)(1 << oct), fr = sc * 3.14159265358979323846f;
#pragma unroll
    for (int ax = 0; ax < 3; ax++)
      dmu[ax] += fr * (dx[18 + 6 * oct + ax] * cospif(sc * G.mu[ax]) - dx[21 + 6 * oct + ax] * sinpif(sc * G.mu[ax]));
  }
  // normal = sign * column kmin of R(q^)
  float dR[9];
  for (int r = 0; r < 3; r++)
    for (int k = 0; k < 3; k++) dR[3 * r + k] = G.kmin == k ? G.sign * dx[r] : 0.f;
  const float w = G.qn[0], qx = G.qn[1], qy = G.qn[2], qz = G.qn[3];
  float dqn[4];
  dqn[0] = dx[3] + 2.f * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
  dqn[1] = dx[4] + 2.f * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.f * qx * dR[4] - w * dR[5] + qz * dR[6] +
                          w * dR[7] - 2.f * qx * dR[8]);
  dqn[2] = dx[5] + 2.f * (-2.f * qy * dR[0] + qx * dR[1] + w * dR[2] + qx * dR[3] + qz * dR[5] - w * dR[6] +
                          qz * dR[7] - 2.f * qy * dR[8]);
  dqn[3] = dx[6] + 2.f * (-2.f * qz * dR[0] - w * dR[1] + qx * dR[2] + w * dR[3] - 2.f * qz * dR[4] +
                          qy * dR[5] + qx * dR[6] + qy * dR[7]);
  const float pq = w * dqn[0] + qx * dqn[1] + qy * dqn[2] + qz * dqn[3];
  for (int k = 0; k < 3; k++) A.d_means[k * n + i] += dmu[k];
  for (int k = 0; k < 3; k++) A.d_log_scales[k * n + i] += dx[7 + k] * G.s[k];
  for (int k = 0; k < 4; k++) A.d_quats[k * n + i] += (dqn[k] - G.qn[k] * pq) / G.qlen;
  const float dv = dx[17] + df[6];
  A.d_vis[i] = A.accumulate ? A.d_vis[i] + dv : dv;
}

// 16 consecutive record values of row `row` for the lane's Gaussians
// base + 16 q + 0..15 (q = lane / 16): the lane's K operands of 16 matrix-core
// steps (K runs over Gaussians; A and B take the same order).
__device__ __forceinline__ void load16(const float *__restrict__ rec, int row, size_t ldn, size_t g0, float (&v)[16]) {
  const float4 *p = reinterpret_cast<const float4 *>(rec + row * ldn + g0);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const float4 t = p[k];
    v[4 * k] = t.x; v[4 * k + 1] = t.y; v[4 * k + 2] = t.z; v[4 * k + 3] = t.w;
  }
}

__device__ __forceinline__ void mma16(f32x4 &acc, const float (&a)[16], const float (&b)[16]) {
#pragma unroll
  for (int k = 0; k < 16; k++) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], b[k], acc, 0, 0, 0);
}

__device__ __forceinline__ void mma16_ones(f32x4 &acc, const float (&a)[16]) {
#pragma unroll
  for (int k = 0; k < 16; k++) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], 1.f, acc, 0, 0, 0);
}

// Weight and bias gradient of one dense layer: dz rows D0.. (OT tiles of 16
// output units), input rows A0.. (IT tiles of 16 input units).
template <int OT, int IT>
__device__ void layer_wgrad(const GmlpArgs &A, int D0, int A0, const GL &L, float *part) {
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  const size_t ldn = A.ldn;
  f32x4 acc[OT][IT], bacc[OT];
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  for (int o = 0; o < OT; o++) {
    bacc[o] = z4;
    for (int t = 0; t < IT; t++) acc[o][t] = z4;
  }
  for (size_t base = (size_t)blockIdx.x * 64; base < ldn; base += (size_t)gridDim.x * 64) {
    const size_t g0 = base + 16 * q;
    float b[IT][16];
#pragma unroll
    for (int t = 0; t < IT; t++) load16(A.act, A0 + 16 * t + r, ldn, g0, b[t]);
#pragma unroll
    for (int o = 0; o < OT; o++) {
      float a[16];
      load16(A.dz, D0 + 16 * o + r, ldn, g0, a);
#pragma unroll
      for (int t = 0; t < IT; t++) mma16(acc[o][t], a, b[t]);
      mma16_ones(bacc[o], a);
    }
  }
  // D layout: lane holds rows 4 q + j, column r
#pragma unroll
  for (int o = 0; o < OT; o++) {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int ou = 16 * o + 4 * q + j;
#pragma unroll
      for (int t = 0; t < IT; t++) part[L.w + ou * L.cols + 16 * t + r] = acc[o][t][j];
      if (r == 0) part[L.b + ou] = bacc[o][j];
    }
  }
}

__global__ __launch_bounds__(64) void gmlp_wgrad_kernel(GmlpArgs A) {
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  const size_t ldn = A.ldn;
  float *part = A.partials + (size_t)blockIdx.x * kGParams;
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  switch (blockIdx.y) {
    case 0: {  // layer 0: 42 inputs as tiles of 16 (rows 42..47 zero)
      f32x4 acc[4][3], bacc[4];
      for (int o = 0; o < 4; o++) {
        bacc[o] = z4;
        for (int t = 0; t < 3; t++) acc[o][t] = z4;
      }
      for (size_t base = (size_t)blockIdx.x * 64; base < ldn; base += (size_t)gridDim.x * 64) {
        const size_t g0 = base + 16 * q;
        float b[3][16];
        load16(A.act, kAX + r, ldn, g0, b[0]);
        load16(A.act, kAX + 16 + r, ldn, g0, b[1]);
        if (32 + r < kGIn) load16(A.act, kAX + 32 + r, ldn, g0, b[2]);
        else
          for (int k = 0; k < 16; k++) b[2][k] = 0.f;
#pragma unroll
        for (int o = 0; o < 4; o++) {
          float a[16];
          load16(A.dz, kD0 + 16 * o + r, ldn, g0, a);
#pragma unroll
          for (int t = 0; t < 3; t++) mma16(acc[o][t], a, b[t]);
          mma16_ones(bacc[o], a);
        }
      }
      for (int o = 0; o < 4; o++)
        for (int j = 0; j < 4; j++) {
          const int ou = 16 * o + 4 * q + j;
          for (int t = 0; t < 3; t++)
            if (16 * t + r < kGIn) part[kL0.w + ou * kGIn + 16 * t + r] = acc[o][t][j];
          if (r == 0) part[kL0.b + ou] = bacc[o][j];
        }
      break;
    }
    case 1: layer_wgrad<2, 4>(A, kD1, kAH1, kL1, part); break;
    case 2: layer_wgrad<2, 2>(A, kD2, kAH2, kL2, part); break;
    case 3: layer_wgrad<2, 2>(A, kDI, kAH3, kLi, part); break;
    default: {  // heads: rows 0..2 incident output (inputs e), 3..5 SSS (inputs h3)
      f32x4 ae[2], ah[2], ab;
      ab = z4;
      for (int t = 0; t < 2; t++) ae[t] = ah[t] = z4;
      for (size_t base = (size_t)blockIdx.x * 64; base < ldn; base += (size_t)gridDim.x * 64) {
        const size_t g0 = base + 16 * q;
        float a[16];
        if (r < 6) load16(A.dz, kDH + r, ldn, g0, a);
        else
          for (int k = 0; k < 16; k++) a[k] = 0.f;
        for (int t = 0; t < 2; t++) {
          float b[16];
          load16(A.act, kAE + 16 * t + r, ldn, g0, b);
          mma16(ae[t], a, b);
          load16(A.act, kAH3 + 16 * t + r, ldn, g0, b);
          mma16(ah[t], a, b);
        }
        mma16_ones(ab, a);
      }
      for (int j = 0; j < 4; j++) {
        const int ou = 4 * q + j;
        for (int t = 0; t < 2; t++) {
          if (ou < 3) part[kLl.w + ou * 32 + 16 * t + r] = ae[t][j];
          else if (ou < 6) part[kLs.w + (ou - 3) * 32 + 16 * t + r] = ah[t][j];
        }
        if (r == 0) {
          if (ou < 3) part[kLl.b + ou] = ab[j];
          else if (ou < 6) part[kLs.b + ou - 3] = ab[j];
        }
      }
      break;
    }
  }
}

}  // namespace

int gmlp_param_count() { return kGParams; }

int gmlp_wgrad_grid(int n) {
  const int chunks = (n + 63) / 64;
  return chunks < 1 ? 1 : (chunks > kGmlpMaxWaves ? kGmlpMaxWaves : chunks);
}

size_t gmlp_ldn(int n) { return (size_t)((n + 63) / 64) * 64; }
size_t gmlp_act_floats(int n) { return (size_t)kARows * gmlp_ldn(n); }
size_t gmlp_dz_floats(int n) { return (size_t)kDRows * gmlp_ldn(n); }
size_t gmlp_mask_words(int n) { return (size_t)kMaskRows * gmlp_ldn(n); }

void launch_gmlp_prep(const float *params, float *wt, hipStream_t st) {
  gmlp_prep_kernel<<<(kGParams + 255) / 256, 256, 0, st>>>(params, wt);
}

void launch_gmlp_fwd(const GmlpArgs &a, hipStream_t st) {
  if (a.n > 0) gmlp_fwd_kernel<<<(a.n + 63) / 64, 64, 0, st>>>(a);
}

void launch_gmlp_bwd(const GmlpArgs &a, hipStream_t st) {
  if (a.n > 0) gmlp_bwd_kernel<<<(int)(a.ldn / 64), 64, 0, st>>>(a);
  gmlp_wgrad_kernel<<<dim3(gmlp_wgrad_grid(a.n), 5), 64, 0, st>>>(a);
}

}  // namespace sssgs
