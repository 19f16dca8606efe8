"""Benchmark: forward + backward of one 800x800 view with 300k Gaussians, the
deferred G-buffer, GGX shading and the residual network (BF16 on the matrix
cores vs FP32), on one MI355X.

One step = render_forward + render_backward of the whole hot path (projection,
radix binning, compositing, shading, and their backward) on inputs already
resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = 3
MPIX = 0.64
HBM_PEAK_GBS = 8000.0
# FP32 vector peak reachable here: packed FP32 is compiled out, so one FMA per
# lane per clock: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz (the 157.3
# TFLOP/s figure counts packed FMA).
FP32_VALU_TFLOPS = 78.6
BF16_MFMA_TFLOPS = 2500.0
FP32_MFMA_TFLOPS = 157.3      # dense FP32 matrix-core peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=2, help="views in the CPU oracle sample")
    ap.add_argument("--precision", choices=["both", "bf16", "fp32"], default="both")
    ap.add_argument("--no-other-workloads", action="store_true", help="skip the 100k, 8-view 500k and 1M lines")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device (a plain copy of known size, "
                         "to scale the HBM byte counters of a profiled run)")
    return ap.parse_args()


def tile_stats(view, cam):
    """Per-tile processed-record counts from the forward state (for algorithmic bytes)."""
    import torch
    lay = view.layout
    H, W = cam.height, cam.width
    nc = view.region(lay.n_contrib, H * W, torch.int32).view(H, W).to(torch.int64)
    TX, TY = -(-W // 16), -(-H // 16)
    pad = torch.zeros((TY * 16, TX * 16), dtype=torch.int64, device=nc.device)
    pad[:H, :W] = nc
    per_tile_max = pad.view(TY, 16, TX, 16).amax(dim=(1, 3))
    rg = view.region(lay.tile_ranges, 2 * TX * TY, torch.int32).view(-1, 2).to(torch.int64)
    listed = (rg[:, 1] - rg[:, 0]).clamp(min=0)
    # records a tile touches in the forward: up to the last contributor of its slowest pixel,
    # plus the Gaussian that stopped it when the list continues
    fwd = torch.minimum(per_tile_max.view(-1) + 1, listed)
    return int(per_tile_max.sum()), int(fwd.sum()), int(listed.sum())


def run_gpu(precision: str, steps: int, warmup: int):
    import torch
    from paper_2408_12282_amd import scene, sssgs as B
    w = scene.workload(WORKLOAD)
    g, cam, light, mlp = w.gaussians, w.cameras[0], w.lights[0], w.mlp
    dev = "cuda"
    p = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in g.arrays().items()}
    mp = torch.from_numpy(mlp.params).to(dev)
    prec = B.PREC_BF16 if precision == "bf16" else B.PREC_FP32
    cap = 24 * g.n
    view = B.View(g.n, cam.width, cam.height, g.feat_dim, mlp.width, cap, device=dev)
    bc, bl = B.make_camera(cam), B.make_light(light)
    _, _, _, M = B.render_forward(view, p, -1, bc, bl, mp, mlp.width, prec, want_count=True)
    drgb = torch.from_numpy(scene.upstream_weights((3, cam.height, cam.width), 1)).to(dev)
    grads = {k: torch.zeros_like(v) for k, v in p.items()}
    dmlp = torch.zeros_like(mp)

    def step():
        rgb, gbuf, alpha, _ = B.render_forward(view, p, -1, bc, bl, mp, mlp.width, prec)
        B.render_backward(view, p, -1, bc, bl, gbuf, drgb, None, None, mp, mlp.width, prec, grads, dmlp)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # timed region: exactly `steps` steps, an event between consecutive steps
    # (per-step median and percentiles), no per-stage events
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[steps]) / steps
    per_step = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    # per-stage kernel durations: HIP events recorded around every stage on the
    # stream its kernels run on, over separate steps
    B.sssgs_timing_read()
    B.sssgs_timing_enable(True)
    for _ in range(max(1, min(steps, 10))):
        step()
    torch.cuda.synchronize()
    B.sssgs_timing_enable(False)
    stages = B.sssgs_timing_read()
    extras = time_training_kernels(rgb_ref=drgb, params=p, mlp_params=mp, grads=grads, dmlp=dmlp)
    ibl = time_ibl(view, p, bc, mp, mlp.width, prec)
    gnet = time_gaussian_network(g, cam, light, drgb, steps)
    vis = time_visibility(p, bl, g.n)
    flags, m_dev = B.sssgs_workspace_status(ctypes_ptr(view), g.n, cam.width, cam.height, g.feat_dim, mlp.width,
                                            cap)
    assert flags == 0 and m_dev == M, (flags, m_dev, M)
    per_tile_last, fwd_records, listed = tile_stats(view, cam)
    return {"ms": ms, "per_step": per_step, "stages": {k: (v[0] / max(v[1], 1), v[1]) for k, v in stages.items()},
            "M": M,
            "bwd_records": per_tile_last, "fwd_records": fwd_records, "listed": listed, "n": g.n,
            "C": 10 + g.feat_dim, "HW": cam.width * cam.height, "precision": precision, "training": extras,
            "ibl": ibl, "gnet": gnet, "vis": vis}


def time_training_kernels(rgb_ref, params, mlp_params, grads, dmlp, reps: int = 10):
    """The rest of a training step, outside the headline: the image loss
    (L1 + D-SSIM, value and gradient) of an 800x800 view and one Adam update of
    every Gaussian and network parameter, timed with events on the stream."""
    import torch
    from paper_2408_12282_amd import sssgs as B
    C, H, W = rgb_ref.shape
    pred = (rgb_ref * 0.1).abs().contiguous()
    target = torch.rand_like(pred)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    B.image_loss(pred, target)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        B.image_loss(pred, target)
    t1.record()
    torch.cuda.synchronize()
    loss_ms = t0.elapsed_time(t1) / reps
    loss_bytes = 11 * C * H * W * 4
    tensors = [(v, grads[k]) for k, v in params.items()] + [(mlp_params, dmlp)]
    moments = [(torch.zeros_like(v), torch.zeros_like(v)) for v, _ in tensors]
    nparam = sum(v.numel() for v, _ in tensors)
    # Adam on copies: the benchmark's parameters stay as they are
    work = [(v.clone(), gr) for v, gr in tensors]
    torch.cuda.synchronize()
    t0.record()
    for step in range(1, reps + 1):
        for (v, gr), (m, s2) in zip(work, moments):
            B.adam_step(v, gr, m, s2, step, B.lr_schedule(step))
    t1.record()
    torch.cuda.synchronize()
    adam_ms = t0.elapsed_time(t1) / reps
    return {"image_loss": {"ms": round(loss_ms, 4), "shape": [C, H, W],
                           "gbs": round(loss_bytes / (loss_ms * 1e-3) / 1e9, 1)},
            "adam": {"ms": round(adam_ms, 4), "params": int(nparam), "launches": len(work),
                     "gbs": round(28 * nparam / (adam_ms * 1e-3) / 1e9, 1)}}


def time_ibl(view, params, cam_struct, mlp_params, mlp_width, prec, k: int = 16, reps: int = 5):
    """Image-based lighting outside the headline: the forward of the same view under
    k environment light samples (one G-buffer, k shading evaluations summed)
    against the single-light forward, timed with events on the stream."""
    import torch
    from paper_2408_12282_amd import scene, sssgs as B
    lights, weights = scene.environment_lights(k)
    bl = [B.make_light(l) for l in lights]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    res = {}
    for name, fn in (("single", lambda: B.render_forward(view, params, -1, cam_struct, bl[0], mlp_params, mlp_width,
                                                          prec)),
                     ("multi", lambda: B.render_forward_lights(view, params, -1, cam_struct, bl, weights, mlp_params,
                                                               mlp_width, prec))):
        fn()
        torch.cuda.synchronize()
        t0.record()
        for _ in range(reps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        res[name] = t0.elapsed_time(t1) / reps
    return {"lights": k, "forward_ms": round(res["multi"], 4), "single_light_forward_ms": round(res["single"], 4),
            "ms_per_added_light": round((res["multi"] - res["single"]) / (k - 1), 4),
            "workload": "300k Gaussians 800x800, environment light samples on a Fibonacci sphere"}


def time_gaussian_network(g, cam, light, drgb, steps: int):
    """The paper's per-Gaussian network (pipeline figure) outside the headline:
    the same 300k Gaussians and view, the network evaluated per Gaussian before
    rasterisation (FP32), its radiances composited into the 18-plane G-buffer
    and Eq. 7 evaluated from them; forward + backward per step, timed with
    events on the stream, then per stage."""
    import torch
    from paper_2408_12282_amd import scene, sssgs as B
    dev = "cuda"
    n = g.n
    p = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in g.arrays().items() if v is not None}
    p["features"] = torch.empty((8, n), device=dev)
    # the network's visibility input traced through the Gaussians (outside the timed step)
    vis = B.trace_visibility(p, B.make_light(light))
    gm = torch.from_numpy(scene.make_gaussian_mlp(seed=0)).to(dev)
    view = B.View(n, cam.width, cam.height, 8, 0, 24 * n, device=dev)
    bc, bl = B.make_camera(cam), B.make_light(light)
    ws = B.gaussian_mlp_workspace(n)
    grads = {k: torch.empty_like(v) for k, v in p.items()}
    dvis, dgm = torch.empty_like(vis), torch.empty_like(gm)

    def step():
        rgb, gbuf, alpha, feats, _ = B.render_gaussian_mlp_forward(view, p, bc, bl, vis, gm, ws)
        B.render_gaussian_mlp_backward(view, p, bc, bl, vis, gm, feats, gbuf, drgb, ws, grads=grads, dvis=dvis,
                                       dgmlp=dgm)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    reps = max(1, steps)
    t0.record()
    for _ in range(reps):
        step()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    B.sssgs_timing_read()
    B.sssgs_timing_enable(True)
    for _ in range(max(1, min(reps, 10))):
        step()
    torch.cuda.synchronize()
    B.sssgs_timing_enable(False)
    st = {k: v[0] / v[1] for k, v in B.sssgs_timing_read().items() if v[1] > 0}
    # multiply-adds of the network per Gaussian (42x64, 64x32, 32x32, 32x32, 32x3, 32x3); the backward
    # propagates the input gradient and forms the weight gradient (2x; it reads the forward's activations)
    flop = 2 * (42 * 64 + 64 * 32 + 32 * 32 + 32 * 32 + 32 * 3 + 32 * 3)
    roof = {}
    for name, f in (("gmlp_fwd", n * flop), ("gmlp_bwd", 2 * n * flop)):
        if st.get(name, 0) > 0:
            tf = f / (st[name] * 1e-3) / 1e12
            roof[name] = {"bound": "alu", "achieved": round(tf, 2), "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                          "frac": round(tf / FP32_VALU_TFLOPS, 4), "flop_per_launch": int(f),
                          "ms_per_launch": round(st[name], 4)}
    return {"workload": "300k Gaussians 800x800, per-Gaussian network 42->64->32->32->(32->3 | 3), FP32, "
                        "18-plane G-buffer, fwd+bwd; visibility input traced once beforehand",
            "ms_per_step": round(ms, 4), "mpix_s": round(MPIX / (ms * 1e-3), 2),
            "stages_ms": {k: round(v, 4) for k, v in st.items()}, "roofline": roof}


def time_visibility(params, light_struct, n: int, reps: int = 5):
    """Ray-traced light visibility of every Gaussian (BVH build + one shadow
    ray per Gaussian) on the same 300k Gaussians, timed with events on the
    stream."""
    import torch
    from paper_2408_12282_amd import sssgs as B
    ws = B.visibility_workspace(n)
    v = B.trace_visibility(params, light_struct, ws)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        B.trace_visibility(params, light_struct, ws)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    B.sssgs_timing_read()
    B.sssgs_timing_enable(True)
    B.trace_visibility(params, light_struct, ws)
    torch.cuda.synchronize()
    B.sssgs_timing_enable(False)
    B.sssgs_timing_read()
    return {"workload": "300k Gaussians, one shadow ray per Gaussian to the point light, BVH built per call",
            "ms": round(ms, 4), "rays_per_s": round(n / (ms * 1e-3), 1),
            "occluded_to_zero": round(float((v == 0).float().mean()), 4),
            "mean_visibility": round(float(v.mean()), 4)}


def ctypes_ptr(view):
    import ctypes as ct
    return ct.c_void_p(view.workspace.data_ptr())


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_300k_800sq_fwdbwd_bf16.md")


def measured_traffic():
    """HBM bytes per launch from the committed counter profile (FETCH_SIZE + WRITE_SIZE,
    scaled by a copy of known size), only for kernels whose source is unchanged since."""
    import hashlib
    out = {}
    if not os.path.exists(TRAFFIC_PROFILE):
        return out
    for line in open(TRAFFIC_PROFILE):
        parts = line.split()
        if len(parts) != 4 or parts[0] != "traffic":
            continue
        unchanged = True
        for item in parts[3].split(","):
            src, sha = item.split(":")
            path = os.path.join(ROOT, "paper_2408_12282_amd", "csrc", src)
            if not os.path.exists(path) or hashlib.sha256(open(path, "rb").read()).hexdigest() != sha:
                unchanged = False
        if unchanged:
            out[parts[1]] = int(parts[2])
    return out


def roofline(r):
    """Algorithmic bytes (compositing, HBM-bound model) or flops (shading network,
    matrix-core model) per launch, divided by the kernels' measured durations."""
    C = r["C"]
    in_dim, width = r.get("net") or (58, 64)
    RS = (6 + C + 3) // 4 * 4
    HW = r["HW"]
    # forward: records + index per processed instance, G-buffer + T + n_contrib written
    fwd_bytes = r["fwd_records"] * (4 * RS + 4) + HW * 4 * (C + 2)
    # backward: records + index per processed instance, dG + dT + T + n_contrib read, per-Gaussian grads written
    bwd_bytes = r["bwd_records"] * (4 * RS + 4) + HW * 4 * (C + 3) + r["n"] * 4 * (6 + C)
    # network multiply-adds per pixel (58 inputs, three hidden layers of 64, 6 outputs): forward once;
    # backward = the forward recomputed + input gradients + weight gradients (3x).  With the BF16
    # width-64 network the backward is two kernels: shading backward (recompute + input
    # gradients, 2x) and the weight-gradient kernel (1x; it recomputes what it needs on top).
    net_flop = 2 * (in_dim * width + 2 * width * width + width * 6)
    split = r["stages"].get("mlp_wgrad", (0.0, 0))[0] > 0
    out = {}
    traffic = measured_traffic()
    for name, nbytes in (("composite_fwd", fwd_bytes), ("composite_bwd", bwd_bytes)):
        t = r["stages"].get(name, (0.0, 0))[0]
        if t > 0:
            gbs = nbytes / (t * 1e-3) / 1e9
            out[name] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic.get(name), "kernel": name,
                         "bytes_per_launch": int(nbytes), "ms_per_launch": round(t, 4)}
    if not r.get("has_net", True):
        return out
    peak = BF16_MFMA_TFLOPS if r["precision"] == "bf16" else FP32_MFMA_TFLOPS
    flops = [("shade_fwd", HW * net_flop), ("shade_bwd", (2 if split else 3) * HW * net_flop)]
    if split:
        flops.append(("mlp_wgrad", HW * net_flop))
    for name, flop in flops:
        t = r["stages"].get(name, (0.0, 0))[0]
        if t > 0:
            tf = flop / (t * 1e-3) / 1e12
            out[name] = {"bound": "mfma", "achieved": round(tf, 2), "peak": peak, "unit": "TFLOP/s",
                         "frac": round(tf / peak, 4), "traffic": traffic.get(name), "kernel": name,
                         "flop_per_launch": int(flop), "ms_per_launch": round(t, 4)}
    return out


def copy_ceiling(mib: int = 1024, reps: int = 10):
    """Achievable HBM bandwidth: a device-to-device copy of `mib` MiB (read + write)."""
    import torch
    src = torch.ones(mib << 18, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    gbs = 2 * (mib << 20) / (ms * 1e-3) / 1e9
    del src, dst
    return {"gbs": round(gbs, 1), "bytes_moved": 2 * (mib << 20), "ms": round(ms, 4),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def _time_steps(step, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return ev[0].elapsed_time(ev[steps]) / steps, per


def _stage_times(step, reps: int):
    import torch
    from paper_2408_12282_amd import sssgs as B
    B.sssgs_timing_read()
    B.sssgs_timing_enable(True)
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    B.sssgs_timing_enable(False)
    return {k: (v[0] / max(v[1], 1), v[1]) for k, v in B.sssgs_timing_read().items()}


def _stats(per):
    return {"median_ms": round(float(np.median(per)), 4), "p10_ms": round(float(np.percentile(per, 10)), 4),
            "p90_ms": round(float(np.percentile(per, 90)), 4)}


def time_other_workloads(steps: int, warmup: int):
    """The other synthetic workloads (outside the headline): the 100k G-buffer
    fwd+bwd (FP32, no network, loss sum(w * G)), the 8-view 500k OLAT training
    step (BF16 network, L1 loss, gradients accumulated over the views) and the
    1M-Gaussian SH view at 1600x1200 with the width-128 BF16 network; each with
    per-step statistics, stage times and the roofline of its kernels."""
    import torch
    from paper_2408_12282_amd import scene, sssgs as B
    out = {}
    dev = "cuda"

    def setup(w, cam):
        g = w.gaussians
        p = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in g.arrays().items() if v is not None}
        mp = torch.from_numpy(w.mlp.params).to(dev) if w.mlp is not None else None
        mw = w.mlp.width if w.mlp is not None else 0
        view = B.View(g.n, cam.width, cam.height, g.feat_dim, mw, 64 * g.n, device=dev)
        return g, p, mp, mw, view

    def summarize(name, desc, ms, per, stages, view, cam, g, prec, net, mpix, extra=None):
        per_tile_last, fwd_records, listed = tile_stats(view, cam)
        r = {"stages": stages, "C": 10 + g.feat_dim, "HW": cam.width * cam.height, "n": g.n, "precision": prec,
             "fwd_records": fwd_records, "bwd_records": per_tile_last, "net": net, "has_net": net is not None}
        rl = roofline(r)
        d = {"workload": desc, "ms_per_step": round(ms, 4), "mpix_s": round(mpix / (ms * 1e-3), 2),
             "step_stats": _stats(per), "stages_ms": {k: round(v[0], 4) for k, v in stages.items() if v[1] > 0},
             "roofline": max(rl.values(), key=lambda v: v["ms_per_launch"]) if rl else None, "roofline_all": rl}
        if extra:
            d.update(extra)
        out[name] = d

    # 100k Gaussians, 800x800, G-buffer fwd + bwd, L = sum(w * G) + 0 * rgb
    w = scene.workload(2)
    cam, light = w.cameras[0], w.lights[0]
    g, p, mp, mw, view = setup(w, cam)
    bc, bl = B.make_camera(cam), B.make_light(light)
    dg = torch.from_numpy(scene.upstream_weights((10 + g.feat_dim, cam.height, cam.width), 1)).to(dev)
    zr = torch.zeros((3, cam.height, cam.width), device=dev)
    grads = {k: torch.empty_like(v) for k, v in p.items()}

    def step2():
        rgb, gbuf, alpha, _ = B.render_forward(view, p, -1, bc, bl, None, 64, B.PREC_FP32)
        B.render_backward(view, p, -1, bc, bl, gbuf, zr, dg, None, None, 64, B.PREC_FP32, grads)

    ms, per = _time_steps(step2, steps, warmup)
    summarize("gbuffer_100k_800sq", "100k Gaussians 800x800, 26-channel G-buffer fwd+bwd, FP32, loss sum(w*G)",
              ms, per, _stage_times(step2, 5), view, cam, g, "fp32", None, MPIX)
    del view, p, grads, dg
    torch.cuda.empty_cache()

    # 500k Gaussians, 8 (camera, light) views, BF16 network, L1 loss, accumulated gradients
    w = scene.workload(4)
    tw = scene.workload(4, seed=1)
    g, p, mp, mw, view = setup(w, w.cameras[0])
    tp = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in tw.gaussians.arrays().items()
          if v is not None}
    tmp = torch.from_numpy(tw.mlp.params).to(dev)
    cams = [B.make_camera(c) for c in w.cameras]
    lights = [B.make_light(l) for l in w.lights]
    # targets: the independently seeded scene rendered by this renderer (outside the timed region)
    targets = []
    for v in range(8):
        t, _, _, _ = B.render_forward(view, tp, -1, cams[v], lights[v], tmp, mw, B.PREC_BF16)
        targets.append(t.clone())
    H, W = w.cameras[0].height, w.cameras[0].width
    scale = 1.0 / (3 * H * W)
    grads = {k: torch.zeros_like(v) for k, v in p.items()}
    dmlp = torch.zeros_like(mp)
    dl = torch.empty((3, H, W), device=dev)
    loss = torch.zeros(1, device=dev)

    def step4():
        for v in range(8):
            rgb, gbuf, alpha, _ = B.render_forward(view, p, -1, cams[v], lights[v], mp, mw, B.PREC_BF16)
            B.sssgs_l1_loss(B._ptr(rgb), B._ptr(targets[v]), rgb.numel(), scale, B._ptr(loss), B._ptr(dl),
                            B._stream())
            B.render_backward(view, p, -1, cams[v], lights[v], gbuf, dl, None, None, mp, mw, B.PREC_BF16, grads,
                              dmlp, accumulate=(v > 0))

    s4 = max(2, steps // 4)
    ms, per = _time_steps(step4, s4, 1)
    summarize("olat_8view_500k_800sq", "500k Gaussians, 8 cameras on a sphere of radius 3 each with its own point "
              "light, 800x800, BF16 network, L1 loss, gradients accumulated; ms_per_step covers the 8 views",
              ms, per, _stage_times(step4, 1), view, w.cameras[7], g, "bf16", (58, 64), 8 * MPIX,
              {"ms_per_view": round(ms / 8, 4)})
    del view, p, tp, grads, targets
    torch.cuda.empty_cache()

    # 1M Gaussians, SH colour, 32 features, 1600x1200, width-128 BF16 network
    w = scene.workload(5)
    cam, light = w.cameras[0], w.lights[0]
    g, p, mp, mw, view = setup(w, cam)
    bc, bl = B.make_camera(cam), B.make_light(light)
    drgb = torch.from_numpy(scene.upstream_weights((3, cam.height, cam.width), 1)).to(dev)
    grads = {k: torch.empty_like(v) for k, v in p.items()}
    dmlp = torch.empty_like(mp)

    def step5():
        rgb, gbuf, alpha, _ = B.render_forward(view, p, 3, bc, bl, mp, mw, B.PREC_BF16)
        B.render_backward(view, p, 3, bc, bl, gbuf, drgb, None, None, mp, mw, B.PREC_BF16, grads, dmlp)

    s5 = max(3, steps // 2)
    ms, per = _time_steps(step5, s5, 2)
    summarize("sh_1m_1600x1200_w128", "1M Gaussians, degree-3 SH colour, 32 features (C = 42), 1600x1200, "
              "BF16 network 74(96)->128x3->6, fwd+bwd", ms, per, _stage_times(step5, 3), view, cam, g, "bf16",
              (74, 128), 1.92)
    del view, p, grads
    torch.cuda.empty_cache()
    return out


def cpu_baseline(views: int):
    from oracle import oracle
    from paper_2408_12282_amd import scene
    w = scene.workload(WORKLOAD)
    g, cam, light, mlp = w.gaussians, w.cameras[0], w.lights[0], w.mlp
    drgb = scene.upstream_weights((3, cam.height, cam.width), 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.render(scene.make_gaussians(100, 16, False, 0), scene.look_at_camera((0, 0, 3), 32, 32), light, mlp)
    t = time.perf_counter()
    for _ in range(views):
        oracle.render(g, cam, light, mlp, bf16=True, drgb=drgb, nthreads=threads)
    dt = (time.perf_counter() - t) / views
    # one core: the centre 400x400 quarter of the view (a quarter of the pixels)
    crop = (200, 200, 600, 600)
    t = time.perf_counter()
    oracle.render(g, cam, light, mlp, bf16=True, drgb=drgb, nthreads=1, crop=crop)
    d1 = time.perf_counter() - t
    mpix_crop = 0.16
    return {"value": round(MPIX / dt, 4), "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": f"{views} full views (300k Gaussians, 800x800, fwd+bwd, FP64 with BF16 network emulation)",
            "s_per_view": round(dt, 3),
            "one_core": {"value": round(mpix_crop / d1, 4), "unit": "Mpix/s", "cores": 1,
                         "sample": "the centre 400x400 crop of the same view, fwd+bwd", "s": round(d1, 3)}}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    res = {}
    for prec in (["bf16", "fp32"] if a.precision == "both" else [a.precision]):
        res[prec] = run_gpu(prec, a.steps, a.warmup)
    head = res.get("bf16") or res.get("fp32")
    rl = roofline(head)
    dominant = max(rl.values(), key=lambda v: v["ms_per_launch"]) if rl else None
    line = {
        "metric": "fwd+bwd ms/view & Mpix/s, 300k Gaussians 800x800 (BF16 MLP vs FP32 plain)",
        "value": round(MPIX / (head["ms"] * 1e-3), 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(head["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32; network bf16 weights x bf16 hi+lo activations, fp32 accumulate; compositing-backward "
                  "channel products bf16x3 split, fp32 accumulate") if "bf16" in res else "f32",
        "data": "synthetic",
        "config": {"workload": "300k-800sq-ggx-mlp-fwdbwd", "gaussians": head["n"], "width": 800, "height": 800,
                   "features": 16, "gbuffer_channels": head["C"], "mlp": "58(64)->64x3->6",
                   "mlp_precision": "bf16" if "bf16" in res else "fp32", "tile_instances": head["M"]},
        "roofline": dominant,
        "step_stats": _stats(head["per_step"]),
        "stages_ms": {k: round(v[0], 4) for k, v in head["stages"].items() if v[1] > 0},
    }
    if "fp32" in res and "bf16" in res:
        f = res["fp32"]
        line["fp32_plain"] = {"ms_per_step": round(f["ms"], 4), "mpix_s": round(MPIX / (f["ms"] * 1e-3), 2),
                              "stages_ms": {k: round(v[0], 4) for k, v in f["stages"].items() if v[1] > 0}}
        line["bf16_speedup_vs_fp32"] = round(f["ms"] / head["ms"], 3)
    line["roofline_all"] = rl
    line["training_kernels"] = head["training"]
    line["image_based_lighting"] = head["ibl"]
    line["per_gaussian_network"] = head["gnet"]
    line["ray_traced_visibility"] = head["vis"]
    cc = copy_ceiling()
    line["hbm_copy_ceiling"] = cc
    if dominant and dominant["unit"] == "GB/s":
        dominant["frac_of_copy_ceiling"] = round(dominant["achieved"] / cc["gbs"], 4)
    if not a.no_other_workloads:
        line["other_workloads"] = time_other_workloads(a.steps, a.warmup)
    if a.calib_copy_mib > 0:
        import torch
        src = torch.ones(a.calib_copy_mib << 18, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(a.cpu_views)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
