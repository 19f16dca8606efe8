"""Backward parity of the HIP path against the FP64 oracle's exact gradient."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_12282_amd import scene

from helpers import gpu_render, rel_norm, small_workload

pytestmark = pytest.mark.gpu

GRAD_REL = 1e-3   # per parameter group, relative L2

# The rendered function is piecewise smooth: alpha cut-offs, the transmittance
# stop and the network's ReLUs are decisions taken in floating point.  FP32 and
# FP64 can take them differently within rounding distance, and one flipped
# decision moves a gradient by O(1) of that pixel's share.  The tests therefore
# put zero upstream gradient on pixels the oracle finds within a margin of such
# a decision: alpha decisions within 1e-5 relative, and any ReLU argument of the
# network below `net_tau` (FP32: 1e-3, about 50x the FP32 error of a
# pre-activation; BF16: 5e-3, about 10x the effect of one bfloat16 rounding
# flip of an input).
NET_TAU = {"fp32": 1e-3, "bf16": 5e-3}


def _keep_mask(ora, precision=None):
    keep = ora["pix_flag"] == 0
    if precision is not None:
        keep &= ora["net_margin"] >= NET_TAU[precision]
    print(f"  pixels kept for the gradient comparison: {keep.mean():.3f}")
    return keep


def _upstream(shape_rgb, C, H, W, seed, rgb=True, gbuf=True, alpha=True):
    rng = np.random.default_rng(seed)
    drgb = rng.normal(size=shape_rgb).astype(np.float32) if rgb else np.zeros(shape_rgb, np.float32)
    dg = rng.normal(size=(C, H, W)).astype(np.float32) if gbuf else None
    da = rng.normal(size=(H, W)).astype(np.float32) if alpha else None
    return drgb, dg, da


def _compare_grads(out, ora, names, tol=GRAD_REL):
    errs = {}
    for k in names:
        ref = ora["grads"][k]
        if ref.size == 0 or not np.any(ref):
            continue
        errs[k] = rel_norm(out["grads"][k], ref)
    print("grad rel errors:", {k: f"{v:.2e}" for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if v > tol}
    assert not bad, f"gradient groups above {tol}: {bad}"
    return errs


GROUPS = ["means", "log_scales", "quats", "opacity_logits", "albedo", "roughness", "metallic", "sss", "features"]


@pytest.mark.parametrize("F,sh", [(16, False), (8, False), (0, False), (32, True)])
def test_gbuffer_backward_no_shading(F, sh):
    """G-buffer fwd+bwd with L = sum(w * G) + sum(w_a * alpha) (the 100k/800 workload, reduced;
    every channel count C = 10 + F the kernels are built for, SH colour with F = 32)."""
    g = scene.make_gaussians(5000, F, sh, seed=2)
    cam = scene.look_at_camera((0, 0, 3), 96, 96)
    light = scene.default_light()
    C = 10 + F
    drgb, dg, da = _upstream((3, 96, 96), C, 96, 96, seed=1, rgb=False)
    print(f"[gpu] gbuffer backward F={F} sh={sh}", flush=True)
    keep = _keep_mask(O.render(g, cam, light, None))
    dg, da = dg * keep, da * keep
    ora = O.render(g, cam, light, None, drgb=drgb, dgbuf=dg, dalpha=da)
    out = gpu_render(g, cam, light, None, "fp32", backward=(drgb, dg, da))
    groups = [k for k in GROUPS if (F or k != "features") and not (sh and k == "albedo")] + (["sh"] if sh else [])
    _compare_grads(out, ora, groups)


def test_shading_backward_no_network():
    w = scene.workload(1)
    g, cam, light = w.gaussians, w.cameras[0], w.lights[0]
    drgb, dg, da = _upstream((3, 128, 128), 10, 128, 128, seed=3, gbuf=False, alpha=False)
    print("[gpu] GGX backward 1k 128x128", flush=True)
    drgb = drgb * _keep_mask(O.render(g, cam, light, None))
    ora = O.render(g, cam, light, None, drgb=drgb)
    out = gpu_render(g, cam, light, None, "fp32", backward=(drgb, None, None))
    _compare_grads(out, ora, GROUPS[:-1])


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_network_backward_small(precision):
    g, cams, lights, mlp = small_workload(3, 20000, 128, 96)
    cam, light = cams[0], lights[0]
    drgb, dg, da = _upstream((3, 96, 128), 26, 96, 128, seed=4, gbuf=False, alpha=False)
    print(f"[gpu] network backward {precision}", flush=True)
    bf = precision == "bf16"
    drgb = drgb * _keep_mask(O.render(g, cam, light, mlp, bf16=bf), precision)
    ora = O.render(g, cam, light, mlp, drgb=drgb, bf16=bf)
    out = gpu_render(g, cam, light, mlp, precision, backward=(drgb, None, None))
    tol = GRAD_REL if precision == "fp32" else 1e-2
    _compare_grads(out, ora, GROUPS + ["mlp"], tol)


def test_sh_features32_width128_backward():
    """The large-scene form: SH colour, 32 features, network width 128 in BF16 (reduced size)."""
    g, cams, lights, mlp = small_workload(5, 20000, 128, 96)
    cam, light = cams[0], lights[0]
    drgb, dg, da = _upstream((3, 96, 128), 42, 96, 128, seed=5, gbuf=False, alpha=False)
    print("[gpu] SH + F32 + width 128 backward", flush=True)
    drgb = drgb * _keep_mask(O.render(g, cam, light, mlp, bf16=True), "bf16")
    ora = O.render(g, cam, light, mlp, drgb=drgb, bf16=True)
    out = gpu_render(g, cam, light, mlp, "bf16", backward=(drgb, None, None))
    groups = [k for k in GROUPS if k != "albedo"] + ["sh", "mlp"]
    _compare_grads(out, ora, groups, 1e-2)
