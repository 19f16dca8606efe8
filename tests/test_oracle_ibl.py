"""Pins of the oracle's image-based lighting by light samples (CPU)."""
import numpy as np

from oracle import oracle as O
from paper_2408_12282_amd import scene


def _small():
    g = scene.make_gaussians(64, 0, False, seed=3)
    cam = scene.look_at_camera((0, 0, 3), 32, 32)
    return g, cam


def test_coincident_lights_add_their_intensities():
    """Without the network, incident light is I / distance^2 (linear in I): two
    lights at one position with unit weights equal one light with I1 + I2."""
    g, cam = _small()
    p = np.array([1.5, 2.0, 2.5], np.float32)
    l1 = scene.Light(p, np.array([2.0, 3.0, 4.0], np.float32))
    l2 = scene.Light(p, np.array([5.0, 1.0, 0.5], np.float32))
    both = O.render_lights(g, cam, [l1, l2], np.ones((2, 3), np.float32))
    one = O.render(g, cam, scene.Light(p, l1.intensity + l2.intensity), None)
    assert np.abs(one["rgb"]).max() > 0
    np.testing.assert_allclose(both["rgb"], one["rgb"], rtol=1e-12, atol=1e-14)


def test_weights_scale_each_channel():
    g, cam = _small()
    light = scene.default_light()
    w = np.array([[2.0, 0.5, 3.0]], np.float32)
    out = O.render_lights(g, cam, [light], w)
    ref = O.render(g, cam, light, None)
    np.testing.assert_allclose(out["rgb"], w[0][:, None, None] * ref["rgb"], rtol=1e-15, atol=0)
    np.testing.assert_array_equal(out["gbuf"], ref["gbuf"])


def test_environment_samples_cover_the_sphere():
    """The sample weights are radiance x solid angle: a constant environment would
    give weights summing to 4 pi x radiance; here every weight is non-negative and
    the lights sit at the given radius with unit irradiance at the origin."""
    lights, w = scene.environment_lights(24, radius=30.0)
    assert w.shape == (24, 3) and (w >= 0).all()
    for l in lights:
        r = float(np.linalg.norm(l.pos))
        assert abs(r - 30.0) < 1e-3
        np.testing.assert_allclose(l.intensity / r ** 2, 1.0, rtol=1e-5)
