// losses.hip -- image loss of the training objective (Appendix "Losses"):
// L = (1 - lambda) mean|x - y| + lambda (1 - mean SSIM(x, y)), and its
// gradient with respect to the rendered image x; and the Adam update
// (Appendix "Training").
//
// SSIM uses local statistics under an 11x11 Gaussian window (sigma 1.5),
// images extended with zeros outside their border, C1 = 0.01^2, C2 = 0.03^2.
// The window is separable, so every window sum is a horizontal 11-tap pass
// followed by a vertical one over an LDS tile with a 5-pixel halo.  The
// gradient needs the adjoint of the window sums, which for this symmetric
// window is the same filter applied to the per-pixel derivative maps.
#include "launch.hpp"

namespace sssgs {

constexpr int kLT = 16;              // output tile edge
constexpr int kLR = 5;               // window radius
constexpr int kLH = kLT + 2 * kLR;   // tile edge with halo
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct SsimWin {
  float g[2 * kLR + 1];
};

// Five window sums of (x, y, x^2, y^2, xy) at every pixel of a 16x16 tile of
// channel blockIdx.z; from them SSIM and its derivatives with respect to the
// local mean of x, the local mean of x^2 and the local mean of xy, scaled by
// `wgt` (the loss weight of one pixel's SSIM).  Per-tile partial sums of SSIM
// and |x - y| go to partials[2 * tile].
__global__ __launch_bounds__(256) void ssim_stats_kernel(const float *__restrict__ x, const float *__restrict__ y,
                                                         int H, int W, SsimWin win, float wgt,
                                                         float *__restrict__ dmx, float *__restrict__ dexx,
                                                         float *__restrict__ dexy, float *__restrict__ partials) {
  __shared__ float tx[kLH][kLH + 1], ty[kLH][kLH + 1];
  __shared__ float hs[5][kLH][kLT + 1];
  __shared__ float red[2][4];
  const int t = threadIdx.x, c = blockIdx.z;
  const int x0 = blockIdx.x * kLT - kLR, y0 = blockIdx.y * kLT - kLR;
  const size_t plane = (size_t)H * W;
  const float *xc = x + c * plane, *yc = y + c * plane;
  for (int k = t; k < kLH * kLH; k += 256) {
    const int r = k / kLH, q = k % kLH, gy = y0 + r, gx = x0 + q;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    tx[r][q] = in ? xc[(size_t)gy * W + gx] : 0.f;
    ty[r][q] = in ? yc[(size_t)gy * W + gx] : 0.f;
  }
  __syncthreads();
  // horizontal pass: rows of the halo tile, the tile's 16 columns
  for (int k = t; k < kLH * kLT; k += 256) {
    const int r = k / kLT, q = k % kLT;
    float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d <= 2 * kLR; d++) {
      const float a = tx[r][q + d], b = ty[r][q + d], gw = win.g[d];
      s[0] = fmaf(gw, a, s[0]);
      s[1] = fmaf(gw, b, s[1]);
      s[2] = fmaf(gw, a * a, s[2]);
      s[3] = fmaf(gw, b * b, s[3]);
      s[4] = fmaf(gw, a * b, s[4]);
    }
#pragma unroll
    for (int m = 0; m < 5; m++) hs[m][r][q] = s[m];
  }
  __syncthreads();
  // vertical pass and the SSIM terms of pixel (r, q)
  const int r = t / kLT, q = t % kLT;
  float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int d = 0; d <= 2 * kLR; d++)
#pragma unroll
    for (int m = 0; m < 5; m++) s[m] = fmaf(win.g[d], hs[m][r + d][q], s[m]);
  const int gy = blockIdx.y * kLT + r, gx = blockIdx.x * kLT + q;
  const bool inside = gy < H && gx < W;
  float ssim = 0.f, l1 = 0.f;
  if (inside) {
    const float mx = s[0], my = s[1];
    const float a1 = 2.f * mx * my + kC1, a2 = 2.f * (s[4] - mx * my) + kC2;
    const float b1 = mx * mx + my * my + kC1, b2 = (s[2] - mx * mx) + (s[3] - my * my) + kC2;
    const float ib = 1.f / (b1 * b2);
    ssim = a1 * a2 * ib;
    const size_t pix = c * plane + (size_t)gy * W + gx;
    dmx[pix] = wgt * ((2.f * my * (a2 - a1)) * ib - ssim * (2.f * mx * (b2 - b1)) * ib);
    dexx[pix] = wgt * (-ssim / b2);
    dexy[pix] = wgt * (2.f * a1 * ib);
    l1 = fabsf(tx[r + kLR][q + kLR] - ty[r + kLR][q + kLR]);
  }
  // per-tile partial sums (fixed order: wave shuffle tree, then the 4 waves)
  float v0 = ssim, v1 = l1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v0 += __shfl_xor(v0, o, 64);
    v1 += __shfl_xor(v1, o, 64);
  }
  if ((t & 63) == 0) {
    red[0][t >> 6] = v0;
    red[1][t >> 6] = v1;
  }
  __syncthreads();
  if (t == 0) {
    const size_t tile = ((size_t)c * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partials[2 * tile] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    partials[2 * tile + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// dL/dx = W^T dmx + 2 x W^T dexx + y W^T dexy + (1 - lambda) sign(x - y) / n,
// with W^T the adjoint of the zero-extended window sum (the same symmetric
// filter applied to the derivative maps, which are zero outside the image).
__global__ __launch_bounds__(256) void ssim_grad_kernel(const float *__restrict__ x, const float *__restrict__ y,
                                                        int H, int W, SsimWin win, float l1w,
                                                        const float *__restrict__ dmx,
                                                        const float *__restrict__ dexx,
                                                        const float *__restrict__ dexy, float *__restrict__ grad) {
  __shared__ float tm[3][kLH][kLH + 1];
  __shared__ float hs[3][kLH][kLT + 1];
  const int t = threadIdx.x, c = blockIdx.z;
  const int x0 = blockIdx.x * kLT - kLR, y0 = blockIdx.y * kLT - kLR;
  const size_t plane = (size_t)H * W;
  const float *maps[3] = {dmx + c * plane, dexx + c * plane, dexy + c * plane};
  for (int k = t; k < kLH * kLH; k += 256) {
    const int r = k / kLH, q = k % kLH, gy = y0 + r, gx = x0 + q;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
#pragma unroll
    for (int m = 0; m < 3; m++) tm[m][r][q] = in ? maps[m][(size_t)gy * W + gx] : 0.f;
  }
  __syncthreads();
  for (int k = t; k < kLH * kLT; k += 256) {
    const int r = k / kLT, q = k % kLT;
#pragma unroll
    for (int m = 0; m < 3; m++) {
      float s = 0.f;
#pragma unroll
      for (int d = 0; d <= 2 * kLR; d++) s = fmaf(win.g[d], tm[m][r][q + d], s);
      hs[m][r][q] = s;
    }
  }
  __syncthreads();
  const int r = t / kLT, q = t % kLT;
  const int gy = blockIdx.y * kLT + r, gx = blockIdx.x * kLT + q;
  if (gy >= H || gx >= W) return;
  float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int d = 0; d <= 2 * kLR; d++)
#pragma unroll
    for (int m = 0; m < 3; m++) s[m] = fmaf(win.g[d], hs[m][r + d][q], s[m]);
  const size_t pix = c * plane + (size_t)gy * W + gx;
  const float xv = x[pix], yv = y[pix], dv = xv - yv;
  const float sg = dv > 0.f ? l1w : (dv < 0.f ? -l1w : 0.f);
  grad[pix] = s[0] + 2.f * xv * s[1] + yv * s[2] + sg;
}

// loss = (1 - lambda) sum|x - y| / n + lambda (1 - sum SSIM / n), summed in a fixed order.
__global__ __launch_bounds__(256) void image_loss_finish_kernel(const float *__restrict__ partials, int ntiles,
                                                                float lam, float inv_n, float *__restrict__ loss) {
  __shared__ double red[2][256];
  const int t = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int k = t; k < ntiles; k += 256) {
    s0 += (double)partials[2 * k];
    s1 += (double)partials[2 * k + 1];
  }
  red[0][t] = s0;
  red[1][t] = s1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      red[0][t] += red[0][t + o];
      red[1][t] += red[1][t + o];
    }
    __syncthreads();
  }
  if (t == 0)
    loss[0] = (float)((1.0 - lam) * red[1][0] * inv_n + lam * (1.0 - red[0][0] * inv_n));
}

size_t image_loss_workspace_bytes(int C, int H, int W) {
  const size_t plane = (size_t)H * W, tiles = (size_t)C * ((H + kLT - 1) / kLT) * ((W + kLT - 1) / kLT);
  return (3 * (size_t)C * plane + 2 * tiles) * sizeof(float);
}

void launch_image_loss(const float *x, const float *y, int C, int H, int W, float lam, void *ws, float *loss,
                       float *grad, hipStream_t st) {
  SsimWin win;
  double gs[2 * kLR + 1], tot = 0.0;
  for (int d = 0; d <= 2 * kLR; d++) {
    const double k = d - kLR;
    gs[d] = exp(-(k * k) / (2.0 * 1.5 * 1.5));
    tot += gs[d];
  }
  for (int d = 0; d <= 2 * kLR; d++) win.g[d] = (float)(gs[d] / tot);
  const size_t plane = (size_t)H * W;
  const double n = (double)C * plane;
  float *dmx = static_cast<float *>(ws), *dexx = dmx + C * plane, *dexy = dexx + C * plane;
  float *partials = dexy + C * plane;
  const dim3 grid((W + kLT - 1) / kLT, (H + kLT - 1) / kLT, C);
  ssim_stats_kernel<<<grid, 256, 0, st>>>(x, y, H, W, win, (float)(-lam / n), dmx, dexx, dexy, partials);
  image_loss_finish_kernel<<<1, 256, 0, st>>>(partials, (int)(grid.x * grid.y * grid.z), lam, (float)(1.0 / n),
                                              loss);
  if (grad)
    ssim_grad_kernel<<<grid, 256, 0, st>>>(x, y, H, W, win, (float)((1.0 - lam) / n), dmx, dexx, dexy, grad);
}

// ------------------------------------------------------------------ Adam

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v, int64_t n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
  const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t st) {
  if (n <= 0) return;
  const float c1 = (float)(1.0 / (1.0 - pow((double)b1, step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)b2, step)));
  adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

}  // namespace sssgs
