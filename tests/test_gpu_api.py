"""The boundary's options and the torch.autograd.Function, on the GPU:
deterministic gradient sums, the background colour, SSSGSRender against the
FP64 oracle's gradient and FP64 central differences, and its guards."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_12282_amd import scene

from helpers import GRAD_REL, NET_MARGIN, estimate_instances, gpu_render, rel_norm, small_workload, to_device

pytestmark = pytest.mark.gpu

GROUPS = ["means", "log_scales", "quats", "opacity_logits", "albedo", "roughness", "metallic", "sss", "features"]


def _bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_deterministic_backward_is_bit_identical(precision):
    """deterministic = 1: two backward calls give the same bits in every
    gradient group; the sums agree with the atomic form to rounding and with
    the oracle to the gradient bound."""
    import torch
    from paper_2408_12282_amd import sssgs as B
    g, cams, lights, mlp = small_workload(3, 20000, 128, 96)
    cam, light = cams[0], lights[0]
    prec = B.PREC_BF16 if precision == "bf16" else B.PREC_FP32
    print(f"[gpu] deterministic backward {precision}", flush=True)
    ora0 = O.render(g, cam, light, mlp, bf16=(precision == "bf16"))
    keep = (ora0["pix_flag"] == 0) & (ora0["net_margin"] >= NET_MARGIN)
    up = (np.random.default_rng(8).normal(size=(3, 96, 128)) * keep).astype(np.float32)
    p, mp = to_device(g, mlp)
    view = B.View(g.n, cam.width, cam.height, g.feat_dim, mlp.width, int(estimate_instances(g, cam) * 1.25) + 1024)
    bc, bl = B.make_camera(cam), B.make_light(light)
    rgb, gbuf, alpha, _ = B.render_forward(view, p, -1, bc, bl, mp, mlp.width, prec, want_count=True)
    d = torch.from_numpy(up).cuda()
    runs = []
    for det in (True, True, False):
        gr, dm = B.render_backward(view, p, -1, bc, bl, gbuf, d, None, None, mp, mlp.width, prec, deterministic=det)
        torch.cuda.synchronize()
        runs.append(({k: v.cpu().numpy() for k, v in gr.items()}, dm.cpu().numpy()))
    (a, am), (b, bm), (c, cm) = runs
    for k in GROUPS:
        assert np.array_equal(_bits(a[k]), _bits(b[k])), k
        assert rel_norm(a[k], c[k]) < 1e-5, k
    assert np.array_equal(_bits(am), _bits(bm))
    ora = O.render(g, cam, light, mlp, bf16=(precision == "bf16"), drgb=up)["grads"]
    errs = {k: rel_norm(a[k], ora[k]) for k in GROUPS}
    errs["mlp"] = rel_norm(am, ora["mlp"])
    print("grad rel errors:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v < GRAD_REL for v in errs.values()), errs


def test_background_colour():
    """rgb = a L_out + T_final b on the sparse 1k scene (most pixels see the
    background), and the gradient through T_final, against the oracle."""
    w = scene.workload(1)
    g, cam, light = w.gaussians, w.cameras[0], w.lights[0]
    bgc = (0.2, 0.5, 0.9)
    print("[gpu] background colour 1k 128x128", flush=True)
    ora = O.render(g, cam, light, None, background=bgc, sens=True)
    keep = ora["pix_flag"] == 0
    up = (np.random.default_rng(2).normal(size=(3, 128, 128)) * keep).astype(np.float32)
    import torch
    from paper_2408_12282_amd import sssgs as B
    p, _ = to_device(g)
    view = B.View(g.n, 128, 128, g.feat_dim, 0, 200_000)
    bc, bl = B.make_camera(cam), B.make_light(light)
    rgb, gbuf, alpha, _ = B.render_forward(view, p, -1, bc, bl, None, 64, B.PREC_FP32, want_count=True,
                                           background=bgc)
    gr, _ = B.render_backward(view, p, -1, bc, bl, gbuf, torch.from_numpy(up).cuda(), None, None, None, 64,
                              B.PREC_FP32, background=bgc)
    torch.cuda.synchronize()
    rgb = rgb.cpu().numpy()
    # element-wise: 1e-4 of |rgb| + the oracle's shading sensitivity (as the forward tests)
    err = np.abs(rgb - ora["rgb"]) / (np.abs(ora["rgb"]) + ora["rgb_sens"])
    print(f"  rgb max element error / scale {float(err[:, keep].max()):.2e}")
    assert float(err[:, keep].max()) < 1e-4
    empty = ora["alpha"] == 0
    assert empty.any()
    for c in range(3):
        assert np.all(rgb[c][empty] == np.float32(bgc[c]))
    og = O.render(g, cam, light, None, drgb=up, background=bgc)["grads"]
    errs = {k: rel_norm(gr[k].cpu().numpy(), og[k]) for k in GROUPS if np.any(og.get(k, 0))}
    print("grad rel errors:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v < GRAD_REL for v in errs.values()), errs


def _autograd_case():
    g = scene.make_gaussians(400, 8, False, seed=12)
    g.log_scales += 1.0
    cam = scene.look_at_camera((0.2, 0.1, 3.0), 64, 48)
    mlp = scene.make_mlp(8, 64, seed=3)
    return g, cam, scene.default_light(), mlp


def _autograd_grads(g, cam, light, mlp, precision, up, view=None):
    import torch
    from paper_2408_12282_amd import sssgs as B
    p, mp = to_device(g, mlp)
    leaves = {k: v.clone().requires_grad_(True) for k, v in p.items() if v.numel()}
    mpl = mp.clone().requires_grad_(True)
    if view is None:
        view = B.View(g.n, cam.width, cam.height, g.feat_dim, mlp.width, 400_000)
    prec = B.PREC_BF16 if precision == "bf16" else B.PREC_FP32
    rgb, gbuf, alpha = B.render(view, leaves, -1, B.make_camera(cam), B.make_light(light), mpl, mlp.width, prec)
    loss = (rgb * torch.from_numpy(up).cuda()).sum()
    torch.autograd.backward(loss)
    torch.cuda.synchronize()
    out = {k: v.grad.cpu().numpy() for k, v in leaves.items()}
    out["mlp"] = mpl.grad.cpu().numpy()
    return out, rgb.detach().cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_autograd_function_against_oracle(precision):
    g, cam, light, mlp = _autograd_case()
    bf = precision == "bf16"
    print(f"[gpu] SSSGSRender + torch.autograd.backward {precision}", flush=True)
    base = O.render(g, cam, light, mlp, bf16=bf)
    keep = (base["pix_flag"] == 0) & (base["net_margin"] >= NET_MARGIN)
    up = (np.random.default_rng(6).normal(size=(3, cam.height, cam.width)) * keep).astype(np.float32)
    gg, rgb = _autograd_grads(g, cam, light, mlp, precision, up)
    assert rel_norm(rgb, base["rgb"]) < (1e-5 if not bf else 3e-5)
    ora = O.render(g, cam, light, mlp, bf16=bf, drgb=up)["grads"]
    errs = {k: rel_norm(gg[k], ora[k]) for k in GROUPS + ["mlp"] if np.any(ora[k])}
    print("grad rel errors:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v < GRAD_REL for v in errs.values()), errs


def test_autograd_function_against_central_differences():
    """FP32 network: SSSGSRender's gradient entries against FP64 central
    differences of the oracle's loss, for sampled parameters of every group
    (samples whose decision signature changes between theta +- h are skipped)."""
    g, cam, light, mlp = _autograd_case()
    base = O.render(g, cam, light, mlp)
    keep = (base["pix_flag"] == 0) & (base["net_margin"] >= NET_MARGIN)
    up = (np.random.default_rng(9).normal(size=(3, cam.height, cam.width)) * keep).astype(np.float32)
    print("[gpu] SSSGSRender against central differences", flush=True)
    gg, _ = _autograd_grads(g, cam, light, mlp, "fp32", up)
    p64 = {k: v.astype(np.float64) for k, v in g.arrays().items()}
    p64["mlp"] = mlp.params.astype(np.float64)
    w = up.astype(np.float64)

    def loss(pp):
        o = O.render(g, cam, light, mlp, params64=pp)
        return float((o["rgb"] * w).sum()), o["signature"]

    rng = np.random.default_rng(4)
    names = [k for k in GROUPS + ["mlp"] if p64[k].size]
    checked = 0
    for trial in range(60):
        k = names[trial % len(names)]
        flat = p64[k].reshape(-1)
        # sample among entries with a sizeable gradient
        big = np.flatnonzero(np.abs(gg[k].reshape(-1)) > 1e-3 * np.abs(gg[k]).max())
        if big.size == 0:
            continue
        j = int(big[rng.integers(big.size)])
        h = 1e-6 * max(1.0, abs(flat[j]))
        pp = {kk: vv.copy() for kk, vv in p64.items()}
        pp[k].reshape(-1)[j] = flat[j] + h
        lp, sp = loss(pp)
        pp[k].reshape(-1)[j] = flat[j] - h
        lm, sm = loss(pp)
        if sp != sm:
            continue
        fd = (lp - lm) / (2 * h)
        a = float(gg[k].reshape(-1)[j])
        assert abs(a - fd) <= 1e-3 * (abs(fd) + 1e-2 * np.abs(gg[k]).max()), f"{k}[{j}]: gpu {a} fd {fd}"
        checked += 1
    print(f"  {checked} entries checked")
    assert checked >= 40


def test_autograd_guards():
    """A second forward on the same view before the backward is refused; a
    capacity overflow in the autograd forward raises ERR_CAPACITY."""
    import torch
    from paper_2408_12282_amd import sssgs as B
    g, cam, light, mlp = _autograd_case()
    p, mp = to_device(g, mlp)
    leaves = {k: v.clone().requires_grad_(True) for k, v in p.items() if v.numel()}
    view = B.View(g.n, cam.width, cam.height, g.feat_dim, mlp.width, 400_000)
    bc, bl = B.make_camera(cam), B.make_light(light)
    print("[gpu] autograd guards", flush=True)
    rgb1, _, _ = B.render(view, leaves, -1, bc, bl, mp, mlp.width, B.PREC_FP32)
    rgb2, _, _ = B.render(view, leaves, -1, bc, bl, mp, mlp.width, B.PREC_FP32)
    with pytest.raises(RuntimeError):
        rgb1.sum().backward()
    rgb2.sum().backward()  # the latest forward's backward is fine
    small = B.View(g.n, cam.width, cam.height, g.feat_dim, mlp.width, 100)
    with pytest.raises(B.SSSGSError) as e:
        B.render(small, leaves, -1, bc, bl, mp, mlp.width, B.PREC_FP32)
    assert e.value.status == B.ERR_CAPACITY
    torch.cuda.synchronize()
