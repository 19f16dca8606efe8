"""FP64 oracle of the ray-traced per-Gaussian light visibility (Sec. 3.2,
"Incident Light": rays traced through the Gaussians with a BVH estimate each
Gaussian's visibility of the point light).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark; it shares no code with the HIP library and uses no
acceleration structure: every Gaussian is tested against every ray (or, with
`prefilter`, every Gaussian that a plain distance bound does not exclude;
tests pin the two forms to the same bits).

What it computes, for every Gaussian i (the paper leaves the ray-Gaussian
interaction open; the reading is the one of the relightable Gaussian work the
paper follows):

* the shadow ray from the Gaussian's centre mu_i towards the light p,
  direction d = (p - mu_i) / |p - mu_i|, segment 0 < t <= |p - mu_i|;
* for every other Gaussian j, the point of the ray's line where Gaussian j is
  densest: in the whitened frame of j (y = S^-1 R^T (x - mu_j)) the ray is
  u + t w, and the densest point is t* = -(u.w)/(w.w) with squared
  Mahalanobis distance D2 = |u x w|^2 / |w|^2;
* Gaussian j occludes when t* lies on the segment and its opacity there,
  alpha_j = min(0.99, sigmoid(logit_j) exp(-D2 / 2)), reaches 1/255 (the
  compositing's cut-offs, Sec. 3.1);
* v_i = prod over occluders of (1 - alpha_j), reported as 0 when it falls
  below 1e-4 (the transmittance floor of the compositing).  The product does
  not depend on the order of the occluders and only decreases as factors are
  added, so no sort along the ray is needed and a ray may stop as soon as the
  floor is crossed.
"""
from __future__ import annotations

import numpy as np


def _rot(qn):
    w, x, y, z = qn.T
    R = np.empty((qn.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def whitening(log_scales, quats):
    """[N, 3, 3] matrices S^-1 R^T taking world offsets to the Gaussians'
    whitened frames."""
    q = np.asarray(quats, np.float64).T
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    R = _rot(qn)
    s = np.exp(np.asarray(log_scales, np.float64).T)
    return np.transpose(R, (0, 2, 1)) / s[:, :, None]


def visibility(means, log_scales, quats, opacity_logits, light_pos, margins: bool = False, receivers=None,
               prefilter: bool = False):
    """v [N] (and, with ``margins``, a per-Gaussian flag set when one of its
    decisions lies within rounding reach of a threshold: t* within 1e-6 of 0
    or of the light, alpha within 1e-6 relative of 1/255 or 0.99, the product
    within 1e-9 of the 1e-4 floor).  ``receivers``: only these Gaussians'
    rays (the others are returned as 1, unflagged).

    ``prefilter``: per ray, first drop the Gaussians that cannot reach 1/255
    anywhere on the ray's line: the whitened distance of the line from a
    centre is at least its Euclidean distance over the largest scale, so a
    Gaussian with (distance / s_max)^2 above 2 ln(255 opacity) (1 % slack)
    has alpha < 1/255 on the whole line.  Same result, far fewer Gaussians
    evaluated per ray."""
    mu_all = np.asarray(means, np.float64).T
    n = mu_all.shape[0]
    Wm_all = whitening(log_scales, quats)
    op_all = 1.0 / (1.0 + np.exp(-np.asarray(opacity_logits, np.float64)))
    smax = np.exp(np.asarray(log_scales, np.float64).max(axis=0))
    with np.errstate(divide="ignore", invalid="ignore"):
        reach2 = np.where(op_all * 255.0 > 1.0, 2.0 * np.log(np.maximum(op_all * 255.0, 1.0)), -1.0)
    P = np.asarray(light_pos, np.float64)
    v = np.ones(n)
    flag = np.zeros(n, bool)
    for i in (range(n) if receivers is None else receivers):
        dvec = P - mu_all[i]
        tmax = np.linalg.norm(dvec)
        d = dvec / tmax
        if prefilter:
            rel = mu_all - mu_all[i][None, :]
            along = rel @ d
            perp2 = np.einsum("ja,ja->j", rel, rel) - along * along
            keep = perp2 / (smax * smax) <= reach2 * 1.01 + 1e-12
            keep[i] = True
            idx = np.flatnonzero(keep)
        else:
            idx = np.arange(n)
        mu, Wm, op = mu_all[idx], Wm_all[idx], op_all[idx]
        self_j = np.flatnonzero(idx == i)
        u = np.einsum("jab,jb->ja", Wm, mu_all[i][None, :] - mu)   # whitened origin per j
        w = np.einsum("jab,b->ja", Wm, d)                            # whitened direction per j
        ww = np.einsum("ja,ja->j", w, w)
        ts = -np.einsum("ja,ja->j", u, w) / ww
        cr = np.cross(u, w)
        D2 = np.einsum("ja,ja->j", cr, cr) / ww
        araw = op * np.exp(-0.5 * D2)
        alpha = np.minimum(0.99, araw)
        hit = (ts > 0.0) & (ts <= tmax) & (alpha >= 1.0 / 255.0)
        hit[self_j] = False
        v[i] = np.prod(1.0 - alpha[hit])
        if v[i] < 1e-4:
            v[i] = 0.0
        if margins:
            near = (np.abs(ts) <= 1e-6 * (1.0 + tmax)) | (np.abs(ts - tmax) <= 1e-6 * (1.0 + tmax))
            near |= np.abs(araw * 255.0 - 1.0) <= 1e-6
            near |= np.abs(araw - 0.99) <= 1e-6
            near[self_j] = False
            prod = np.prod(1.0 - alpha[hit])
            flag[i] = bool(np.any(near & (araw >= 1.0 / 255.0 * (1 - 1e-6)))) or abs(prod - 1e-4) <= 1e-9
    return (v, flag) if margins else v
