"""Brute-force per-pixel renderer in float64 PyTorch (CPU), for tiny scenes.

TEST INFRASTRUCTURE ONLY.  A second, independent statement of what the FP64
oracle in ``sssgs_oracle.c`` computes, written with whole-array tensor
operations instead of per-Gaussian scalar code.  Gradients come from autograd,
so the oracle's hand-derived backward is checked against a derivative nobody
wrote by hand.

For every pixel it takes every Gaussian whose tile rectangle contains the
pixel's tile, orders them by (depth rounded to float32, index), and composites
front to back (Eq. 3 of arxiv 2408.12282), then shades the pixel (Eq. 4, 6, 7
and the per-pixel deferred shading of Sec. 3.2).  Projection follows Eq. 1-2.
"""
from __future__ import annotations

import math

import numpy as np
import torch

TILE = 16
DT = torch.float64


def _t(a):
    return torch.as_tensor(np.asarray(a, np.float64), dtype=DT)


def quat_matrix(q):
    """Rotation matrices [N,3,3] from unit quaternions q [N,4] = (w,x,y,z)."""
    w, x, y, z = q.unbind(-1)
    rows = [
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ]
    return torch.stack(rows, -2)


def sh_basis(d):
    """Real orthonormal SH, degrees 0..3, at unit directions d [...,3] -> [...,16]."""
    x, y, z = d.unbind(-1)
    pi = math.pi
    c1 = math.sqrt(3 / (4 * pi))
    c2a, c2b, c2c = math.sqrt(15 / (4 * pi)), math.sqrt(5 / (16 * pi)), math.sqrt(15 / (16 * pi))
    c3a, c3b, c3c = math.sqrt(35 / (32 * pi)), math.sqrt(105 / (4 * pi)), math.sqrt(21 / (32 * pi))
    c3d, c3e = math.sqrt(7 / (16 * pi)), math.sqrt(105 / (16 * pi))
    one = torch.ones_like(x)
    return torch.stack([
        0.5 * math.sqrt(1 / pi) * one,
        c1 * y, c1 * z, c1 * x,
        c2a * x * y, c2a * y * z, c2b * (3 * z * z - 1), c2a * x * z, c2c * (x * x - y * y),
        c3a * y * (3 * x * x - y * y), c3b * x * y * z, c3c * y * (5 * z * z - 1), c3d * z * (5 * z * z - 3),
        c3c * x * (5 * z * z - 1), c3e * z * (x * x - y * y), c3a * x * (x * x - 3 * y * y),
    ], -1)


def _normalize(v, eps=1e-12):
    n = torch.linalg.norm(v, dim=-1, keepdim=True)
    return v / torch.clamp(n, min=eps)


def _bf16(x):
    """Round to bfloat16 in the forward pass (values here are float32-exact)."""
    return x.to(torch.float32).to(torch.bfloat16).to(DT)


def _bf16_pair(x):
    """An activation as it enters a BF16 forward product: hi + lo, two bfloat16 numbers."""
    hi = _bf16(x)
    return hi + _bf16(x - hi)


def render(params: dict, cam, light, mlp=None, bf16=False, sh_degree=-1, background=None):
    """params: name -> float64 tensor (may require grad), SoA [k,N] layout.

    Returns dict(rgb [3,H,W], gbuf [C,H,W], alpha [H,W], n_contrib [H,W] (numpy),
    lists {tile: [indices]} (numpy), mean2d, conic, radius, rect).
    """
    W, H = cam.width, cam.height
    TX, TY = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    mu = params["means"].T                       # [N,3]
    n = mu.shape[0]
    Rw = _t(cam.R)
    tw = _t(cam.t)
    Cw = -(Rw.T @ tw)
    pc = mu @ Rw.T + tw                           # [N,3]
    x, y, z = pc.unbind(-1)
    s = torch.exp(params["log_scales"].T)         # [N,3]
    q = params["quats"].T
    qn = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    Rq = quat_matrix(qn)
    Sig = Rq @ torch.diag_embed(s * s) @ Rq.transpose(-1, -2)
    limx = 1.3 * (0.5 * W) / cam.fx
    limy = 1.3 * (0.5 * H) / cam.fy
    zs = torch.where(z > 0.2, z, torch.ones_like(z))
    tx = torch.clamp(x / zs, -limx, limx)
    ty = torch.clamp(y / zs, -limy, limy)
    zero = torch.zeros_like(zs)
    Jm = torch.stack([torch.stack([cam.fx / zs, zero, -cam.fx * tx / zs], -1),
                      torch.stack([zero, cam.fy / zs, -cam.fy * ty / zs], -1)], -2)  # [N,2,3]
    S2 = Jm @ Rw @ Sig @ Rw.T @ Jm.transpose(-1, -2) + 0.3 * torch.eye(2, dtype=DT)
    det = S2[:, 0, 0] * S2[:, 1, 1] - S2[:, 0, 1] * S2[:, 1, 0]
    safe = (det > 0) & (z > 0.2)
    S2s = torch.where(safe[:, None, None], S2, torch.eye(2, dtype=DT).expand_as(S2))
    conic_m = torch.linalg.inv(S2s)
    conic = torch.stack([conic_m[:, 0, 0], conic_m[:, 0, 1], conic_m[:, 1, 1]], -1)
    a_, c_ = S2s[:, 0, 0].detach().numpy(), S2s[:, 1, 1].detach().numpy()
    det_np = det.detach().numpy()
    mid = 0.5 * (a_ + c_)
    lam = mid + np.sqrt(np.maximum(0.1, mid * mid - det_np))
    radius = np.minimum(np.ceil(3.0 * np.sqrt(lam)), 1e9)
    u = cam.fx * x / zs + cam.cx
    v = cam.fy * y / zs + cam.cy
    un, vn = u.detach().numpy(), v.detach().numpy()
    rect = np.stack([
        np.clip(np.floor((un - radius) / TILE), 0, TX), np.clip(np.floor((vn - radius) / TILE), 0, TY),
        np.clip(np.floor((un + radius + TILE - 1) / TILE), 0, TX),
        np.clip(np.floor((vn + radius + TILE - 1) / TILE), 0, TY)]).astype(np.int64)
    valid = safe.numpy() & ((rect[2] - rect[0]) * (rect[3] - rect[1]) > 0)
    o = torch.sigmoid(params["opacity_logits"])
    ls = params["log_scales"].detach().numpy()
    kmin = np.argmin(ls, axis=0)                  # first minimum: lowest axis on ties
    ncol = Rq[torch.arange(n), :, torch.as_tensor(kmin)]   # column kmin -> [N,3]
    flip = torch.sign(((Cw - mu) * ncol).sum(-1)).detach()
    flip = torch.where(flip < 0, -torch.ones_like(flip), torch.ones_like(flip))
    nrm = ncol * flip[:, None]
    if sh_degree >= 0:
        dirs = _normalize(mu - Cw)
        Y = sh_basis(dirs)                                   # [N,16]
        shc = params["sh"].T.reshape(n, 16, 3)
        col = torch.clamp((Y[:, :, None] * shc).sum(1) + 0.5, min=0.0)
    else:
        col = params["albedo"].T
    feats = params["features"].T if params["features"].numel() else torch.zeros((n, 0), dtype=DT)
    ch = torch.cat([col, nrm, params["roughness"][:, None], params["metallic"][:, None],
                    params["sss"][:, None], z[:, None], feats], -1)        # [N,C]
    C = ch.shape[1]
    zkey = z.detach().numpy().astype(np.float32)

    lists = {}
    for t in range(TX * TY):
        tx_, ty_ = t % TX, t // TX
        m = valid & (rect[0] <= tx_) & (tx_ < rect[2]) & (rect[1] <= ty_) & (ty_ < rect[3])
        idx = np.nonzero(m)[0]
        order = np.lexsort((idx, zkey[idx]))
        lists[t] = idx[order]

    gbuf = torch.zeros((C, H * W), dtype=DT)
    Tfin = torch.ones(H * W, dtype=DT)
    ncontrib = np.zeros(H * W, np.int32)
    gcols = []
    tcols = []
    for py in range(H):
        for px in range(W):
            t = (py // TILE) * TX + (px // TILE)
            idx = lists[t]
            if len(idx) == 0:
                gcols.append(torch.zeros(C, dtype=DT))
                tcols.append(torch.ones((), dtype=DT))
                continue
            it = torch.as_tensor(idx)
            dx = u[it] - (px + 0.5)
            dy = v[it] - (py + 0.5)
            cn = conic[it]
            pw = -0.5 * (cn[:, 0] * dx * dx + cn[:, 2] * dy * dy) - cn[:, 1] * dx * dy
            al = torch.clamp(o[it] * torch.exp(pw), max=0.99)
            pwn, aln = pw.detach().numpy(), al.detach().numpy()
            inc = np.zeros(len(idx), bool)
            Tn = 1.0
            last = 0
            for j in range(len(idx)):
                if pwn[j] > 0 or aln[j] < 1.0 / 255.0:
                    continue
                if Tn * (1.0 - aln[j]) < 1e-4:
                    break
                inc[j] = True
                Tn *= 1.0 - aln[j]
                last = j + 1
            ncontrib[py * W + px] = last
            ae = torch.where(torch.as_tensor(inc), al, torch.zeros_like(al))
            one_m = 1.0 - ae
            Tb = torch.cat([torch.ones(1, dtype=DT), torch.cumprod(one_m, 0)[:-1]])
            wgt = Tb * ae
            gcols.append((wgt[:, None] * ch[it]).sum(0))
            tcols.append(torch.prod(one_m))
    gbuf = torch.stack(gcols, 1)          # [C, HW]
    Tfin = torch.stack(tcols)             # [HW]
    a = 1.0 - Tfin
    bg = (a < 1e-6).detach()
    a_s = torch.where(bg, torch.ones_like(a), a)
    gb = gbuf / a_s
    nraw = gb[3:6].T
    nn_ = _normalize(nraw)
    pxs = torch.arange(W, dtype=DT) + 0.5
    pys = torch.arange(H, dtype=DT) + 0.5
    vv, uu = torch.meshgrid(pys, pxs, indexing="ij")
    rc = torch.stack([(uu.reshape(-1) - cam.cx) / cam.fx, (vv.reshape(-1) - cam.cy) / cam.fy,
                      torch.ones(H * W, dtype=DT)], -1)
    ray = rc @ Rw                       # R^T rc, row form
    xw = Cw + gb[9][:, None] * ray
    wo = _normalize(Cw - xw)
    vi = _t(light.pos) - xw
    wi = _normalize(vi)
    h = _normalize(wo + wi)
    nov = (nn_ * wo).sum(-1)
    nol = (nn_ * wi).sum(-1)
    noh = (nn_ * h).sum(-1)
    voh = (wo * h).sum(-1)
    NoV = torch.clamp(nov, min=1e-4)
    NoL = torch.clamp(nol, min=1e-4)
    NoH = torch.clamp(noh, min=0.0)
    VoH = torch.clamp(voh, min=0.0)
    cosI = torch.clamp(nol, min=0.0)
    r = gb[6]
    m = gb[7]
    ag = r * r
    D = ag * ag / (math.pi * (NoH * NoH * (ag * ag - 1) + 1) ** 2)
    k = (r + 1) ** 2 / 8
    Gv = NoV / (NoV * (1 - k) + k) * NoL / (NoL * (1 - k) + k)
    b = gb[0:3].T
    F0 = 0.04 * (1 - m)[:, None] + b * m[:, None]
    Fr = F0 + (1 - F0) * ((1 - VoH) ** 5)[:, None]
    fs = D[:, None] * Fr * Gv[:, None] / (4 * NoV * NoL)[:, None]
    fd = (1 - m)[:, None] * b / math.pi
    if mlp is None:
        li2 = torch.clamp((vi * vi).sum(-1), min=1e-12)
        Lin = _t(light.intensity)[None, :] / li2[:, None]
        L = (fs + fd) * Lin * cosI[:, None]
    else:
        P = params["mlp"]
        F = C - 10
        pe = []
        for oc in range(6):
            arg = (2.0 ** oc) * math.pi * xw
            pe += [torch.sin(arg), torch.cos(arg)]
        inp = torch.cat([gb[10:10 + F].T] + pe + [wo, wi], -1)
        pad = mlp.in_pad - inp.shape[1]
        inp = torch.cat([inp, torch.zeros((inp.shape[0], pad), dtype=DT)], -1)
        off = 0
        act = _bf16_pair(inp) if bf16 else inp
        dims = [mlp.in_pad] + [mlp.width] * mlp.hidden + [mlp.out_dim]
        for l in range(mlp.hidden + 1):
            rows, cols = dims[l + 1], dims[l]
            Wl = P[off:off + rows * cols].reshape(rows, cols)
            off += rows * cols
            bl = P[off:off + rows]
            off += rows
            if bf16:
                Wl = _bf16(Wl)
            pre = act @ Wl.T + bl
            if l < mlp.hidden:
                act = torch.relu(pre)
                if bf16:
                    act = _bf16_pair(act)
            else:
                out = pre
        Lin = torch.relu(out[:, 0:3])
        Lsss = torch.sigmoid(out[:, 3:6])
        sss = gb[8][:, None]
        L = sss * Lsss + (1 - sss) * (fs + fd) * Lin * cosI[:, None]
    rgb = torch.where(bg[:, None], torch.zeros_like(L), a[:, None] * L).T
    if background is not None:  # composited over a constant colour behind the Gaussians
        rgb = rgb + _t(background)[:, None] * Tfin[None, :]
    return {
        "rgb": rgb.reshape(3, H, W), "gbuf": gbuf.reshape(C, H, W), "alpha": a.reshape(H, W),
        "n_contrib": ncontrib.reshape(H, W), "lists": lists,
        "mean2d": torch.stack([u, v]).detach().numpy(), "conic": conic.T.detach().numpy(),
        "radius": np.where(valid, radius, 0).astype(np.int64), "rect": np.where(valid[None], rect, 0),
        "valid": valid,
    }
