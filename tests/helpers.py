"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
binding and the FP64 oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

from paper_2408_12282_amd import scene

TILE = 16

# Parity tolerances shared by the GPU tests (relative L2 per output tensor or
# per parameter group unless stated).
GRAD_REL = 1e-3        # gradients, every parameter group, either network precision
FWD_REL = 1e-5         # FP32 forward images
BF16_FP64_REL = 2e-3   # BF16-network image against the FP64 network
# BF16-network image against the oracle's emulation of the same arithmetic
# (weights rounded once, activations as hi + lo pairs, FP32 accumulation):
# a pre-activation differs from the emulation's by at most the granularity of
# the pair (2^-17 of each term) plus the FP32 error of the network inputs
# (~1e-6 of the terms), about 1e-5 of the sum of its terms' magnitudes; the
# bound is three times that.
BF16_EMU_REL = 3e-5
# A pixel enters a gradient comparison only if every ReLU argument of its
# network is farther from zero than this fraction of the sum of its terms'
# magnitudes (the oracle's net_margin), the same 3x of the ~1e-5 bound above:
# closer, FP32 and FP64 may take the ReLU decision differently, which moves
# that unit's share of the gradient by O(1).
NET_MARGIN = 3e-5


def to_device(g, mlp=None, device="cuda"):
    import torch
    p = {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in g.arrays().items()}
    mp = torch.from_numpy(mlp.params).to(device) if mlp is not None else None
    return p, mp


def gpu_render(g, cam, light, mlp=None, precision="fp32", capacity=None, backward=None, want_count=True):
    """Forward (and optional backward with upstream (drgb, dgbuf, dalpha) numpy arrays) on the GPU.

    Returns a dict of numpy arrays incl. the inspected workspace regions."""
    import torch
    from paper_2408_12282_amd import sssgs as B
    prec = B.PREC_BF16 if precision == "bf16" else B.PREC_FP32
    p, mp = to_device(g, mlp)
    if capacity is None:
        capacity = max(1024, int(estimate_instances(g, cam) * 1.25) + 1024)
    view = B.View(g.n, cam.width, cam.height, g.feat_dim, mlp.width if mlp is not None else 0, capacity)
    bc, bl = B.make_camera(cam), B.make_light(light)
    mw = mlp.width if mlp is not None else 64
    rgb, gbuf, alpha, M = B.render_forward(view, p, g.sh_degree, bc, bl, mp, mw, prec, want_count=want_count)
    torch.cuda.synchronize()
    out = {"rgb": rgb.cpu().numpy(), "gbuf": gbuf.cpu().numpy(), "alpha": alpha.cpu().numpy(), "M": M}
    lay = view.layout
    T = -(-cam.width // TILE) * -(-cam.height // TILE)
    HW = cam.width * cam.height
    out["tile_ranges"] = view.region(lay.tile_ranges, 2 * T, torch.int32).view(T, 2).cpu().numpy().astype(np.int64)
    if M is not None:
        out["sorted_gauss"] = view.region(lay.sorted_gauss, M, torch.int32).cpu().numpy()
    out["t_final"] = view.region(lay.t_final, HW, torch.float32).view(cam.height, cam.width).cpu().numpy()
    out["n_contrib"] = view.region(lay.n_contrib, HW, torch.int32).view(cam.height, cam.width).cpu().numpy()
    out["radii"] = view.region(lay.radii, g.n, torch.int32).cpu().numpy()
    out["rects"] = view.region(lay.rects, 4 * g.n, torch.int16).view(g.n, 4).cpu().numpy().astype(np.int64) & 0xFFFF
    rs = lay.rec_stride
    out["records"] = view.region(lay.records, rs * g.n, torch.float32).view(g.n, rs).cpu().numpy()
    out["depth_keys"] = view.region(lay.depth_keys, g.n, torch.float32).cpu().numpy()
    out["boxes"] = view.region(lay.boxes, 4 * g.n, torch.int16).view(g.n, 4).cpu().numpy().astype(np.int64)
    if backward is not None:
        drgb, dgbuf, dalpha = backward
        t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
        grads, dmlp = B.render_backward(view, p, g.sh_degree, bc, bl, gbuf, t(drgb), t(dgbuf), t(dalpha), mp, mw,
                                        prec)
        torch.cuda.synchronize()
        out["grads"] = {k: v.cpu().numpy() for k, v in grads.items()}
        if dmlp is not None:
            out["grads"]["mlp"] = dmlp.cpu().numpy()
    out["view"] = view
    return out


def estimate_instances(g, cam) -> int:
    from oracle import oracle as O
    return O._count_instances(g, cam, {k: np.asarray(v, np.float64) for k, v in g.arrays().items()})


def rel_norm(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


def assert_close_masked(got, ref, mask_ok, rtol, name="", scale=None):
    """Element-wise |got - ref| <= rtol * scale where mask_ok.

    scale defaults to |ref| + mean|ref|; for composited values pass |ref| plus
    the oracle's sum of |terms| (the size of the rounding error of a sum)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if scale is None:
        scale = np.abs(ref) + np.abs(ref).mean()
    err = np.abs(got - ref) / np.maximum(scale, 1e-300)
    print(f"  {name}: max element error / scale = {float(np.max(np.where(mask_ok, err, 0.0))):.2e}")
    bad = (err > rtol) & mask_ok
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"{name}: {int(bad.sum())} elements off (rtol {rtol}); first {idx.tolist()}; "
                             f"got {got[tuple(idx[0])]} ref {ref[tuple(idx[0])]}")


def tile_lists_equal(gpu, ora, g_flag=None):
    """Exact comparison of per-tile Gaussian lists; returns the number of tiles compared."""
    gr, orr = gpu["tile_ranges"], ora["tile_ranges"]
    T = orr.shape[0]
    for t in range(T):
        a = gpu["sorted_gauss"][gr[t, 0]:gr[t, 1]] if gr[t, 1] > gr[t, 0] else np.zeros(0, np.int32)
        b = ora["tile_list"][orr[t, 0]:orr[t, 1]]
        if g_flag is not None and g_flag.any():
            keep_a = g_flag[a] == 0
            keep_b = g_flag[b] == 0
            a, b = a[keep_a], b[keep_b]
        if len(a) != len(b) or not np.array_equal(a, b):
            raise AssertionError(f"tile {t}: gpu {a[:10]}... ({len(a)}) vs oracle {b[:10]}... ({len(b)})")
    return T


def small_workload(cfg: int, n: int, width: int, height: int, seed: int = 0):
    """A reduced copy of workload `cfg` (same distributions, smaller N and image)."""
    w = scene.workload(cfg, seed=seed, n=n)
    cams = [scene.look_at_camera(c.center, width, height) for c in w.cameras]
    return w.gaussians, cams, w.lights, w.mlp
