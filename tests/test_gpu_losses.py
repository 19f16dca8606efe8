"""Image loss (L1 + D-SSIM) and Adam step on the GPU against the FP64 oracle."""
import numpy as np
import pytest

from oracle import losses as OL

from helpers import rel_norm

pytestmark = pytest.mark.gpu


def _pair(shape, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, size=shape).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.1, size=shape), 0, 1).astype(np.float32)
    return x, y


@pytest.mark.parametrize("shape", [(3, 96, 120), (3, 37, 53), (1, 1, 1), (2, 17, 16)])
def test_image_loss_matches_oracle(shape):
    import torch
    from paper_2408_12282_amd import sssgs as B
    x, y = _pair(shape, sum(shape))
    print(f"[gpu] image loss {shape}", flush=True)
    loss, g = B.image_loss(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    ref, gref = OL.image_loss(x, y)
    print(f"  loss {loss.item():.9g} oracle {ref:.9g}; grad rel err {rel_norm(g.cpu().numpy(), gref):.2e}")
    assert abs(loss.item() - ref) <= 1e-5 * abs(ref) + 1e-7
    gg = g.cpu().numpy()
    assert rel_norm(gg, gref) < 1e-5
    np.testing.assert_allclose(gg, gref, rtol=0, atol=1e-4 * np.abs(gref).max())


def test_image_loss_identical_images():
    import torch
    from paper_2408_12282_amd import sssgs as B
    x, _ = _pair((3, 40, 50), 3)
    t = torch.from_numpy(x).cuda()
    loss, g = B.image_loss(t, t.clone())
    torch.cuda.synchronize()
    assert abs(loss.item()) < 1e-6
    assert np.abs(g.cpu().numpy()).max() < 1e-8


def test_image_loss_full_view_800():
    """The loss on a rendered 800x800 view against a reference image (the OLAT
    training objective at its image size), value and gradient."""
    import torch
    from paper_2408_12282_amd import sssgs as B
    x, y = _pair((3, 800, 800), 11)
    print("[gpu] image loss 3x800x800", flush=True)
    loss, g = B.image_loss(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    ref, gref = OL.image_loss(x, y)
    e = rel_norm(g.cpu().numpy(), gref)
    print(f"  loss {loss.item():.9g} oracle {ref:.9g}; grad rel err {e:.2e}")
    assert abs(loss.item() - ref) <= 1e-5 * abs(ref)
    assert e < 1e-5


def test_adam_steps_match_oracle():
    import torch
    from paper_2408_12282_amd import sssgs as B
    rng = np.random.default_rng(7)
    n = 1_000_003
    p = rng.normal(size=n).astype(np.float32)
    tp = torch.from_numpy(p).cuda()
    tm = torch.zeros_like(tp)
    tv = torch.zeros_like(tp)
    pr, mr, vr = p.astype(np.float64), np.zeros(n), np.zeros(n)
    print("[gpu] adam", flush=True)
    # the C ABI takes the hyperparameters as float32: the oracle gets the same values
    f32 = lambda a: float(np.float32(a))
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        lr = B.lr_schedule(step)
        B.adam_step(tp, torch.from_numpy(g).cuda(), tm, tv, step, lr)
        pr, mr, vr = OL.adam_step(pr, g, mr, vr, step, f32(lr), f32(0.9), f32(0.999), f32(1e-8))
    torch.cuda.synchronize()
    np.testing.assert_allclose(tp.cpu().numpy(), pr, rtol=0, atol=1e-6)
    np.testing.assert_allclose(tm.cpu().numpy(), mr, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(tv.cpu().numpy(), vr, rtol=1e-5, atol=1e-9)
