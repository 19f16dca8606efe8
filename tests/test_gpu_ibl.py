"""Image-based lighting (several point lights over one G-buffer) on the GPU against the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_12282_amd import scene

from helpers import BF16_EMU_REL, BF16_FP64_REL, assert_close_masked, rel_norm, small_workload, to_device

pytestmark = pytest.mark.gpu


def _gpu_lights(g, cam, lights, weights, mlp, precision):
    import torch
    from paper_2408_12282_amd import sssgs as B
    prec = B.PREC_BF16 if precision == "bf16" else B.PREC_FP32
    p, mp = to_device(g, mlp)
    view = B.View(g.n, cam.width, cam.height, g.feat_dim, mlp.width if mlp is not None else 0, 64 * g.n + 4096)
    bc = B.make_camera(cam)
    bl = [B.make_light(l) for l in lights]
    mw = mlp.width if mlp is not None else 64
    rgb, gbuf, alpha, M = B.render_forward_lights(view, p, g.sh_degree, bc, bl, weights, mp, mw, prec,
                                                  want_count=True)
    one = B.render_forward(view, p, g.sh_degree, bc, bl[0], mp, mw, prec)[0]
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), gbuf.cpu().numpy(), one.cpu().numpy()


def _masked_rel(got, ref, ok):
    m = np.broadcast_to(ok, got.shape)
    return float(np.linalg.norm((got - ref)[m]) / np.linalg.norm(ref[m]))


@pytest.mark.parametrize("k", [6, 40])
def test_environment_lighting_no_network_fp32(k):
    """k environment samples (40: more than one shading pass of 32 lights) on the
    sparse 1k-Gaussian scene.  As for one light, its sharp GGX highlights turn the
    G-buffer's FP32 rounding into rgb error in proportion to the shading's
    sensitivity, so rgb is checked element-wise against the oracle's summed
    sensitivity (1e-4, the single-light forward's element bound)."""
    w = scene.workload(1)
    g, cam = w.gaussians, w.cameras[0]
    lights, weights = scene.environment_lights(k)
    print(f"[gpu] IBL {k} lights, 1k Gaussians 128x128, no network", flush=True)
    ora = O.render_lights(g, cam, lights, weights, sens=True)
    rgb, gbuf, _ = _gpu_lights(g, cam, lights, weights, None, "fp32")
    ok = ora["pix_flag"] == 0
    assert ok.mean() > 0.99
    print(f"  rgb rel err {_masked_rel(rgb, ora['rgb'], ok):.2e} ({ok.mean():.3f} of pixels unflagged)")
    assert_close_masked(rgb, ora["rgb"], np.broadcast_to(ok, rgb.shape), 1e-4, "rgb",
                        scale=np.abs(ora["rgb"]) + ora["rgb_sens"])
    assert rel_norm(gbuf, ora["gbuf"]) < 1e-5


def test_environment_lighting_network_bf16():
    g, cams, _, mlp = small_workload(3, 20000, 128, 96)
    cam = cams[0]
    lights, weights = scene.environment_lights(5)
    print("[gpu] IBL 5 lights, 20k Gaussians 128x96, BF16 network", flush=True)
    ora = O.render_lights(g, cam, lights, weights, mlp, bf16=True)
    rgb, _, _ = _gpu_lights(g, cam, lights, weights, mlp, "bf16")
    e = rel_norm(rgb, ora["rgb"])
    print(f"  rgb rel err vs BF16 emulation {e:.2e}")
    assert e < BF16_EMU_REL
    ora64 = O.render_lights(g, cam, lights, weights, mlp, bf16=False)
    e64 = rel_norm(rgb, ora64["rgb"])
    print(f"  rgb rel err vs FP64 network {e64:.2e}")
    assert e64 < BF16_FP64_REL


def test_single_light_with_unit_weights_is_the_single_light_forward():
    """One light of weight 1 gives the single-light forward bit for bit."""
    g, cams, lights, mlp = small_workload(3, 5000, 64, 48)
    cam = cams[0]
    print("[gpu] IBL one light == forward", flush=True)
    rgb, _, one = _gpu_lights(g, cam, [lights[0]], np.ones((1, 3), np.float32), mlp, "bf16")
    assert np.array_equal(rgb.view(np.uint32), one.view(np.uint32))
