"""Forward parity of the HIP path (through the C ABI) against the FP64 oracle."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_12282_amd import scene

from helpers import assert_close_masked, gpu_render, rel_norm, small_workload, tile_lists_equal

pytestmark = pytest.mark.gpu

# Forward tolerance for FP32 compositing: per-output relative L2 error.  FP32
# accumulation over ~70 contributors with ~1 ulp per step gives ~1e-6; the
# element-wise bound is applied away from the oracle's flagged decision margins.
FWD_REL = 1e-5


def _projection_checks(g, out, ora):
    valid = ora["radius"] > 0
    np.testing.assert_array_equal(out["radii"], ora["radius"])
    np.testing.assert_array_equal(out["rects"][valid], ora["rect"].T[valid])
    rec = out["records"]
    np.testing.assert_allclose(rec[valid, 0], ora["mean2d"][0, valid], rtol=2e-7, atol=1e-4)
    np.testing.assert_allclose(rec[valid, 1], ora["mean2d"][1, valid], rtol=2e-7, atol=1e-4)
    for k in range(3):
        np.testing.assert_allclose(rec[valid, 2 + k], ora["conic"][k, valid], rtol=1e-6,
                                   atol=1e-6 * np.abs(ora["conic"][k, valid]).max())
    np.testing.assert_allclose(rec[valid, 5], ora["opacity"][valid], rtol=1e-6)
    C = 10 + g.feat_dim
    np.testing.assert_allclose(rec[valid, 6:6 + C], ora["channels"][:, valid].T, rtol=1e-6, atol=1e-6)
    # depth key: float32 rounding of the FP64 depth, bit for bit
    np.testing.assert_array_equal(out["depth_keys"][valid], ora["depth"][valid].astype(np.float32))


def _image_checks(out, ora, rtol=FWD_REL, rgb_rtol=None):
    ok = ora["pix_flag"] == 0
    assert ok.mean() > 0.99
    assert_close_masked(out["alpha"], ora["alpha"], ok, rtol, "alpha")
    assert_close_masked(out["gbuf"], ora["gbuf"], np.broadcast_to(ok, out["gbuf"].shape), rtol, "gbuf")
    np.testing.assert_array_equal(out["n_contrib"][ok], ora["n_contrib"][ok])
    assert rel_norm(out["gbuf"], ora["gbuf"]) < rtol
    assert rel_norm(out["alpha"], ora["alpha"]) < rtol
    rr = rgb_rtol if rgb_rtol is not None else rtol
    assert_close_masked(out["rgb"], ora["rgb"], np.broadcast_to(ok, out["rgb"].shape), rr, "rgb")
    assert rel_norm(out["rgb"], ora["rgb"]) < rr


def test_small_scene_no_network_1k_128():
    """The 1k-Gaussian 128x128 workload: projection, lists, G-buffer, GGX shading."""
    w = scene.workload(1)
    g, cam, light = w.gaussians, w.cameras[0], w.lights[0]
    print(f"[gpu] forward 1k 128x128 N={g.n}", flush=True)
    ora = O.render(g, cam, light, None, lists=True)
    out = gpu_render(g, cam, light)
    assert out["M"] == ora["num_instances"]
    _projection_checks(g, out, ora)
    tile_lists_equal(out, ora, ora["g_flag"])
    _image_checks(out, ora)


@pytest.mark.parametrize("W,H", [(37, 21), (100, 52), (1, 1), (17, 33)])
def test_ragged_image_sizes(W, H):
    g = scene.make_gaussians(400, 8, False, seed=W * 7 + H)
    g.log_scales += 1.0
    cam = scene.look_at_camera((0.1, -0.2, 3.0), W, H)
    light = scene.default_light()
    print(f"[gpu] ragged {W}x{H}", flush=True)
    ora = O.render(g, cam, light, None, lists=True)
    out = gpu_render(g, cam, light)
    assert out["M"] == ora["num_instances"]
    tile_lists_equal(out, ora, ora["g_flag"])
    _image_checks(out, ora)


def test_depth_ties_order_by_index():
    g = scene.make_gaussians(300, 0, False, seed=9)
    g.log_scales += 1.2
    g.means[2, :150] = np.float32(0.25)
    g.means[2, 150:] = np.float32(-0.1)
    cam = scene.look_at_camera((0, 0, 3), 64, 48)
    light = scene.default_light()
    print("[gpu] depth ties", flush=True)
    ora = O.render(g, cam, light, None, lists=True)
    out = gpu_render(g, cam, light)
    tile_lists_equal(out, ora)
    _image_checks(out, ora)


def test_empty_and_all_culled():
    light = scene.default_light()
    cam = scene.look_at_camera((0, 0, 3), 48, 40)
    print("[gpu] empty scene", flush=True)
    g0 = scene.make_gaussians(0, 0, False, seed=0)
    out = gpu_render(g0, cam, light, capacity=16)
    assert out["M"] == 0 and np.all(out["rgb"] == 0) and np.all(out["alpha"] == 0)
    g = scene.make_gaussians(50, 0, False, seed=0)
    g.means[2] = 5.0
    print("[gpu] all culled", flush=True)
    out = gpu_render(g, cam, light, capacity=16)
    assert out["M"] == 0 and np.all(out["rgb"] == 0)


def test_capacity_overflow_is_reported():
    from paper_2408_12282_amd import sssgs as B
    w = scene.workload(1)
    g, cam, light = w.gaussians, w.cameras[0], w.lights[0]
    print("[gpu] capacity overflow", flush=True)
    with pytest.raises(B.SSSGSError) as e:
        gpu_render(g, cam, light, capacity=100)
    assert e.value.status == B.ERR_CAPACITY


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_network_shading_small(precision):
    """GGX + residual network at the headline's network shape, on a reduced scene."""
    g, cams, lights, mlp = small_workload(3, 20000, 128, 96)
    cam, light = cams[0], lights[0]
    print(f"[gpu] network {precision} 20k 128x96", flush=True)
    ora = O.render(g, cam, light, mlp, lists=True, bf16=(precision == "bf16"))
    out = gpu_render(g, cam, light, mlp, precision)
    tile_lists_equal(out, ora, ora["g_flag"])
    ok = ora["pix_flag"] == 0
    assert_close_masked(out["gbuf"], ora["gbuf"], np.broadcast_to(ok, out["gbuf"].shape), FWD_REL, "gbuf")
    e = rel_norm(out["rgb"], ora["rgb"])
    print(f"rgb rel err vs oracle ({precision}): {e:.3e}")
    if precision == "fp32":
        assert e < 1e-5
    else:
        # same bfloat16 rounding on both sides; differences come from FP32 vs
        # FP64 inputs flipping a rounding now and then
        assert e < 2e-4
        ora64 = O.render(g, cam, light, mlp, bf16=False)
        e64 = rel_norm(out["rgb"], ora64["rgb"])
        print(f"rgb rel err vs FP64 network: {e64:.3e}")
        assert e64 < 2e-3


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_headline_300k_800(precision):
    """The 300k-Gaussian 800x800 view: tile lists bit-exact, images to tolerance."""
    w = scene.workload(3)
    g, cam, light, mlp = w.gaussians, w.cameras[0], w.lights[0], w.mlp
    print(f"[gpu] headline 300k 800x800 {precision}", flush=True)
    ora = O.render(g, cam, light, mlp, lists=True, bf16=(precision == "bf16"))
    out = gpu_render(g, cam, light, mlp, precision, capacity=6_000_000)
    assert out["M"] == ora["num_instances"]
    tile_lists_equal(out, ora, ora["g_flag"])
    ok = ora["pix_flag"] == 0
    assert_close_masked(out["gbuf"], ora["gbuf"], np.broadcast_to(ok, out["gbuf"].shape), FWD_REL, "gbuf")
    assert rel_norm(out["gbuf"], ora["gbuf"]) < FWD_REL
    e = rel_norm(out["rgb"], ora["rgb"])
    print(f"rgb rel err ({precision}): {e:.3e}")
    assert e < (1e-5 if precision == "fp32" else 2e-4)
