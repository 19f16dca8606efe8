"""FP64 oracle of the per-Gaussian network (pipeline figure; Sec. 3.2 Eq. 6
evaluated "for each Gaussian"; appendix "Network").

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark.  The product path never imports this module, and
it shares no code with the HIP library.

What it computes, for every Gaussian i (numpy, float64, vectorised over i):

* the network input (appendix "Network": normal, rotation, scale, light
  direction, view direction, light distance, visibility, and a Fourier
  encoding of the position), 42 values in this order:
    n (3)      shortest rotation axis, turned toward the camera (the normal
               the R3DGS material model uses, Sec. 3.1)
    q^ (4)     unit quaternion (w, x, y, z)
    s (3)      scale exp(log_scale)
    w_in (3)   (p_light - mu) / |p_light - mu|
    w_out (3)  (c_cam - mu) / |c_cam - mu|
    d (1)      |p_light - mu|
    v (1)      visibility
    gamma (24) for k = 0..3: sin(2^k pi mu_x,y,z), then cos(2^k pi mu_x,y,z)
* the network: three trunk layers of 64, 32, 32 units, each followed by a
  Leaky-ReLU (slope 0.01); the incident-light head: one layer of 32 units with
  a Leaky-ReLU, then 3 outputs through a ReLU; the SSS head: 3 outputs through
  a sigmoid, both heads reading the trunk output.
* the eight feature planes that the compositing blends (the 18-plane
  G-buffer with F = 8): [L_in (3) | L_sss (3) | v | 1]; the composited
  constant plane is the pixel's alpha.
* the exact (almost-everywhere) derivative of all of it given the gradient of
  the feature planes: network parameters, means, log-scales, quaternions and
  visibility.

Readings where the paper is silent or garbled: the rotation enters as the
four-component unit quaternion (the printed "rotation (2)" cannot hold a 3D
rotation), so the input has 42 values rather than 16 + 24; visibility is one
scalar per Gaussian (the degree-0 term of the paper's SH visibility; the
ray-traced supervision of v is not part of this computation); the Fourier
encoding uses 4 octaves, which gives the 24 values the paper states; the
Leaky-ReLU slope is 0.01; the argmin of the scales and the sign of the normal
are piecewise constant (zero derivative).
"""
from __future__ import annotations

import numpy as np

LAYERS = ((64, 42), (32, 64), (32, 32), (32, 32), (3, 32), (3, 32))
SLOPE = 0.01
N_IN = 42
N_FEAT = 8


def param_count() -> int:
    return sum(r * c + r for r, c in LAYERS)


def unpack(params):
    """Packed vector -> [(W [rows, cols], b [rows])] per layer (float64)."""
    p = np.asarray(params, np.float64)
    out, off = [], 0
    for r, c in LAYERS:
        W = p[off:off + r * c].reshape(r, c)
        off += r * c
        b = p[off:off + r]
        off += r
        out.append((W, b))
    assert off == p.size
    return out


def _rot(qn):
    """Rotation matrices [N, 3, 3] of unit quaternions [N, 4] (w, x, y, z)."""
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


def _rot_bwd(qn, dR):
    """dL/dq^ [N, 4] of R(q^) given dL/dR [N, 3, 3], from the partial
    derivatives of the nine entries of _rot."""
    w, x, y, z = qn.T
    d = lambda i, j: dR[:, i, j]  # noqa: E731
    dw = 2 * (-z * d(0, 1) + y * d(0, 2) + z * d(1, 0) - x * d(1, 2) - y * d(2, 0) + x * d(2, 1))
    dx = 2 * (y * d(0, 1) + z * d(0, 2) + y * d(1, 0) - 2 * x * d(1, 1) - w * d(1, 2) + z * d(2, 0)
              + w * d(2, 1) - 2 * x * d(2, 2))
    dy = 2 * (-2 * y * d(0, 0) + x * d(0, 1) + w * d(0, 2) + x * d(1, 0) + z * d(1, 2) - w * d(2, 0)
              + z * d(2, 1) - 2 * y * d(2, 2))
    dz = 2 * (-2 * z * d(0, 0) - w * d(0, 1) + x * d(0, 2) + w * d(1, 0) - 2 * z * d(1, 1) + y * d(1, 2)
              + x * d(2, 0) + y * d(2, 1))
    return np.stack([dw, dx, dy, dz], axis=1)


def _unit(v):
    """(v / max(|v|, 1e-12), |v|) row-wise."""
    l = np.linalg.norm(v, axis=1)
    return v / np.maximum(l, 1e-12)[:, None], l


def inputs(means, log_scales, quats, visibility, cam_center, light_pos):
    """Network input [N, 42] and what the backward needs.  Gaussian arrays are
    structure-of-arrays ([3, N], [3, N], [4, N], [N])."""
    mu = np.asarray(means, np.float64).T
    ls = np.asarray(log_scales, np.float64).T
    q = np.asarray(quats, np.float64).T
    v = np.asarray(visibility, np.float64)
    C = np.asarray(cam_center, np.float64)
    P = np.asarray(light_pos, np.float64)
    qlen = np.linalg.norm(q, axis=1)
    qn = q / qlen[:, None]
    R = _rot(qn)
    # shortest axis: first minimum of the float32 log-scales
    kmin = np.argmin(np.asarray(log_scales, np.float32).T, axis=1)
    idx = np.arange(mu.shape[0])
    axis = R[idx, :, kmin]
    sign = np.where(np.einsum("ij,ij->i", axis, C[None, :] - mu) < 0.0, -1.0, 1.0)
    nrm = sign[:, None] * axis
    s = np.exp(ls)
    wi, dl = _unit(P[None, :] - mu)
    wo, dc = _unit(C[None, :] - mu)
    pe = []
    for k in range(4):
        arg = (2.0 ** k) * np.pi * mu
        pe += [np.sin(arg), np.cos(arg)]
    x = np.concatenate([nrm, qn, s, wi, wo, dl[:, None], v[:, None]] + pe, axis=1)
    assert x.shape[1] == N_IN
    cache = dict(mu=mu, q=q, qlen=qlen, qn=qn, kmin=kmin, sign=sign, s=s, wi=wi, dl=dl, wo=wo, dc=dc)
    return x, cache


def _lrelu(z):
    return np.where(z > 0.0, z, SLOPE * z)


def _lrelu_d(z):
    return np.where(z > 0.0, 1.0, SLOPE)


def forward(x, params):
    """Features [8, N] = [L_in | L_sss | v | 1] and the activations."""
    (W0, b0), (W1, b1), (W2, b2), (Wi, bi), (Wl, bl), (Ws, bs) = unpack(params)
    z0 = x @ W0.T + b0
    h1 = _lrelu(z0)
    z1 = h1 @ W1.T + b1
    h2 = _lrelu(z1)
    z2 = h2 @ W2.T + b2
    h3 = _lrelu(z2)
    zi = h3 @ Wi.T + bi
    e = _lrelu(zi)
    zl = e @ Wl.T + bl
    zs = h3 @ Ws.T + bs
    lin = np.maximum(zl, 0.0)
    lsss = 1.0 / (1.0 + np.exp(-zs))
    n = x.shape[0]
    feats = np.concatenate([lin, lsss, x[:, 17:18], np.ones((n, 1))], axis=1).T
    acts = dict(x=x, z0=z0, h1=h1, z1=z1, h2=h2, z2=z2, h3=h3, zi=zi, e=e, zl=zl, zs=zs, lsss=lsss)
    return feats, acts


def forward_bound(x, params):
    """Magnitude of the terms of each output's last sum [6, N]: |W| |a| + |b|
    of the output layer (the sigmoid planes times the sigmoid's slope), the
    scale of that sum's rounding error.  A diagnostic for the tolerance of an
    FP32 evaluation, not part of the method."""
    L = unpack(params)
    _, a = forward(x, params)
    bl = np.abs(a["e"]) @ np.abs(L[4][0]).T + np.abs(L[4][1])
    bs = (np.abs(a["h3"]) @ np.abs(L[5][0]).T + np.abs(L[5][1])) * a["lsss"] * (1.0 - a["lsss"])
    return np.concatenate([bl, bs], axis=1).T


def backward(dfeat, params, acts, cache, cam_center, light_pos):
    """Gradients given dL/d(features) [8, N]: dict with 'params' (packed),
    'means' [3, N], 'log_scales' [3, N], 'quats' [4, N], 'visibility' [N]."""
    (W0, b0), (W1, b1), (W2, b2), (Wi, bi), (Wl, bl), (Ws, bs) = unpack(params)
    a = acts
    df = np.asarray(dfeat, np.float64).T
    dzl = df[:, 0:3] * (a["zl"] > 0.0)
    dzs = df[:, 3:6] * a["lsss"] * (1.0 - a["lsss"])
    de = dzl @ Wl
    dzi = de * _lrelu_d(a["zi"])
    dh3 = dzi @ Wi + dzs @ Ws
    dz2 = dh3 * _lrelu_d(a["z2"])
    dh2 = dz2 @ W2
    dz1 = dh2 * _lrelu_d(a["z1"])
    dh1 = dz1 @ W1
    dz0 = dh1 * _lrelu_d(a["z0"])
    dx = dz0 @ W0
    grads = []
    for dz, inp in ((dz0, a["x"]), (dz1, a["h1"]), (dz2, a["h2"]), (dzi, a["h3"]), (dzl, a["e"]), (dzs, a["h3"])):
        grads += [(dz.T @ inp).ravel(), dz.sum(axis=0)]
    dparams = np.concatenate(grads)
    c = cache
    C = np.asarray(cam_center, np.float64)
    n = dx.shape[0]
    dn, dqn, ds = dx[:, 0:3], dx[:, 3:7].copy(), dx[:, 7:10]
    dwi, dwo, ddl, dv = dx[:, 10:13], dx[:, 13:16], dx[:, 16], dx[:, 17] + df[:, 6]
    dmu = np.zeros((n, 3))
    # w_in = u / |u|, d = |u| with u = p_light - mu
    proj = np.einsum("ij,ij->i", c["wi"], dwi)
    du = (dwi - c["wi"] * proj[:, None]) / c["dl"][:, None] + ddl[:, None] * c["wi"]
    dmu -= du
    # w_out = u / |u| with u = c_cam - mu
    proj = np.einsum("ij,ij->i", c["wo"], dwo)
    dmu -= (dwo - c["wo"] * proj[:, None]) / c["dc"][:, None]
    # Fourier encoding
    mu = c["mu"]
    for k in range(4):
        fr = (2.0 ** k) * np.pi
        dsin = dx[:, 18 + 6 * k:21 + 6 * k]
        dcos = dx[:, 21 + 6 * k:24 + 6 * k]
        dmu += dsin * fr * np.cos(fr * mu) - dcos * fr * np.sin(fr * mu)
    # normal: signed column kmin of R(q^)
    dR = np.zeros((n, 3, 3))
    dR[np.arange(n), :, c["kmin"]] = c["sign"][:, None] * dn
    dqn += _rot_bwd(c["qn"], dR)
    proj = np.einsum("ij,ij->i", c["qn"], dqn)
    dq = (dqn - c["qn"] * proj[:, None]) / c["qlen"][:, None]
    dls = ds * c["s"]
    del C
    return dict(params=dparams, means=dmu.T, log_scales=dls.T, quats=dq.T, visibility=dv)


def features(means, log_scales, quats, visibility, params, cam_center, light_pos):
    """Convenience: the feature planes [8, N] only."""
    x, _ = inputs(means, log_scales, quats, visibility, cam_center, light_pos)
    return forward(x, params)[0]


def feature_grads(means, log_scales, quats, visibility, params, cam_center, light_pos, dfeat):
    """Convenience: forward then backward for the given dL/d(features)."""
    x, cache = inputs(means, log_scales, quats, visibility, cam_center, light_pos)
    _, acts = forward(x, params)
    return backward(dfeat, params, acts, cache, cam_center, light_pos)
