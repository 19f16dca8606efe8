"""The allocation-free image loss (sssgs_image_loss_noalloc) against the
workspace form (sssgs_image_loss), through the C ABI: two calls in a row on
the same GPU, the second on a smaller image, each bit-identical to the
workspace form (the same kernels with a fixed summation order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pair(shape, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, size=shape).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.1, size=shape), 0, 1).astype(np.float32)
    return x, y


def _noalloc(x, y):
    import torch
    from paper_2408_12282_amd import sssgs as B
    C, H, W = x.shape
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    grad = torch.full(x.shape, float("nan"), dtype=torch.float32, device="cuda")
    st = B.sssgs_image_loss_noalloc(B._ptr(x), B._ptr(y), C, H, W, 0.2, B._ptr(loss), B._ptr(grad), B._stream())
    assert st == 0, B.lib().sssgs_last_error().decode()
    torch.cuda.synchronize()
    return loss.cpu().numpy(), grad.cpu().numpy()


def test_noalloc_image_loss_matches_workspace_form():
    import torch
    from paper_2408_12282_amd import sssgs as B
    for shape, seed in (((3, 800, 800), 1), ((3, 37, 53), 2)):
        x, y = _pair(shape, seed)
        xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
        print(f"[gpu] no-alloc image loss {shape}", flush=True)
        l1, g1 = _noalloc(xt, yt)
        l0, g0 = B.image_loss(xt, yt)
        torch.cuda.synchronize()
        l0, g0 = l0.cpu().numpy(), g0.cpu().numpy()
        assert np.array_equal(l1.view(np.uint32), l0.view(np.uint32)), (l1, l0)
        assert np.array_equal(g1.view(np.uint32), g0.view(np.uint32))


def test_noalloc_image_loss_rejects_images_beyond_the_scratch():
    import torch
    from paper_2408_12282_amd import sssgs as B
    x = torch.zeros((3, 1024, 1024), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    print("[gpu] no-alloc image loss, oversize", flush=True)
    st = B.sssgs_image_loss_noalloc(B._ptr(x), B._ptr(x), 3, 1024, 1024, 0.2, B._ptr(loss), None, B._stream())
    assert st == B.ERR_INVALID_ARG
