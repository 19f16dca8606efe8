"""FP64 oracle of the image loss of the training objective and of the Adam step.

TEST INFRASTRUCTURE ONLY: used by the tests; the product path never imports
this module.

Image loss (Appendix "Losses"): the rendered image is compared with the
reference by L_img = (1 - lambda) L1 + lambda (1 - SSIM) with lambda = 0.2,
where L1 is the mean absolute difference and SSIM the mean structural
similarity over pixels and channels.  The paper takes this loss from 3D
Gaussian splatting and does not restate the SSIM parameters; the reading used
here is the standard SSIM of Wang et al. (2004): local statistics under an
11x11 Gaussian window (sigma 1.5, normalised to sum 1), C1 = 0.01^2,
C2 = 0.03^2 for a data range of 1, images extended with zeros outside their
border (the window is not renormalised there).

Adam (Appendix "Training"): the paper uses Adam with its default parameters
(beta1 0.9, beta2 0.999, eps 1e-8) and bias-corrected moments.

Everything is written from the definitions, in float64, without separable
filtering or any other reordering: every local statistic is the explicit
window sum.  The gradient of SSIM is the chain rule through those sums.
"""
from __future__ import annotations

import numpy as np

WIN = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA_DSSIM = 0.2


def gaussian_window() -> np.ndarray:
    """2-D window w[a][b] = g(a) g(b), g(k) = exp(-k^2 / (2 sigma^2)) / sum, k = -5..5."""
    k = np.arange(WIN, dtype=np.float64) - WIN // 2
    g = np.exp(-(k * k) / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def _window_sum(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """out[c][i][j] = sum_{a,b} w[a][b] img[c][i + a - 5][j + b - 5], zero outside the image."""
    C, H, W = img.shape
    r = WIN // 2
    pad = np.zeros((C, H + 2 * r, W + 2 * r))
    pad[:, r:r + H, r:r + W] = img
    out = np.zeros((C, H, W))
    for a in range(WIN):
        for b in range(WIN):
            out += w[a, b] * pad[:, a:a + H, b:b + W]
    return out


def _window_adjoint(m: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of _window_sum: out[c][q] = sum_p w[p - q + 5] m[c][p] over image pixels p."""
    C, H, W = m.shape
    r = WIN // 2
    acc = np.zeros((C, H + 2 * r, W + 2 * r))
    for a in range(WIN):
        for b in range(WIN):
            acc[:, a:a + H, b:b + W] += w[a, b] * m
    return acc[:, r:r + H, r:r + W]


def ssim_map(x: np.ndarray, y: np.ndarray):
    """Per-pixel SSIM of images x, y ([C][H][W]) and the local statistics."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    w = gaussian_window()
    mx, my = _window_sum(x, w), _window_sum(y, w)
    exx, eyy, exy = _window_sum(x * x, w), _window_sum(y * y, w), _window_sum(x * y, w)
    vx, vy, cxy = exx - mx * mx, eyy - my * my, exy - mx * my
    a1, a2 = 2.0 * mx * my + C1, 2.0 * cxy + C2
    b1, b2 = mx * mx + my * my + C1, vx + vy + C2
    s = (a1 * a2) / (b1 * b2)
    return s, dict(mx=mx, my=my, exx=exx, eyy=eyy, exy=exy, a1=a1, a2=a2, b1=b1, b2=b2)


def image_loss(x: np.ndarray, y: np.ndarray, lam: float = LAMBDA_DSSIM, grad: bool = True):
    """L_img(x, y) = (1 - lam) mean|x - y| + lam (1 - mean SSIM(x, y)) and dL/dx (float64).

    sign(0) = 0 in the L1 term."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = x.size
    s, st = ssim_map(x, y)
    loss = (1.0 - lam) * np.abs(x - y).sum() / n + lam * (1.0 - s.sum() / n)
    if not grad:
        return loss, None
    w = gaussian_window()
    mx, my, a1, a2, b1, b2 = st["mx"], st["my"], st["a1"], st["a2"], st["b1"], st["b2"]
    # dS/d(local statistics of x); y is constant
    d_mx = (2.0 * my * a2 - 2.0 * my * a1) / (b1 * b2) - s * (2.0 * mx * b2 - 2.0 * mx * b1) / (b1 * b2)
    d_exx = -s / b2
    d_exy = 2.0 * a1 / (b1 * b2)
    wgt = -lam / n
    g = (_window_adjoint(wgt * d_mx, w) + 2.0 * x * _window_adjoint(wgt * d_exx, w)
         + y * _window_adjoint(wgt * d_exy, w))
    g += (1.0 - lam) * np.sign(x - y) / n
    return loss, g


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v) in float64."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
