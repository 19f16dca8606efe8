"""Pins of the ray-traced visibility oracle (Sec. 3.2, "Incident Light")."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.spatial.transform import Rotation

from oracle import visibility as V
from paper_2408_12282_amd import scene


def _scene(centres, scales, opac, quats=None):
    n = len(centres)
    means = np.asarray(centres, np.float64).T
    log_scales = np.log(np.asarray(scales, np.float64)).T
    q = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)) if quats is None else np.asarray(quats, np.float64)
    logits = np.log(np.asarray(opac) / (1.0 - np.asarray(opac)))
    return means, log_scales, q.T, logits


def test_single_occluder_closed_form():
    """Receiver at the origin, light at (10, 0, 0), an isotropic occluder at
    (5, h, 0): the densest point is t* = 5 at Mahalanobis distance h / s."""
    s, h, o = 0.2, 0.25, 0.7
    m, ls, q, lg = _scene([[0, 0, 0], [5, h, 0]], [[0.01] * 3, [s] * 3], [0.5, o])
    v = V.visibility(m, ls, q, lg, [10.0, 0.0, 0.0])
    alpha = o * math.exp(-0.5 * (h / s) ** 2)
    assert v[0] == pytest.approx(1.0 - alpha, rel=1e-12)
    assert v[1] == 1.0        # the receiver is behind the occluder's ray origin


def test_rotated_anisotropic_occluder():
    """Scales (0.5, 0.1, 0.1) turned 90 degrees about z: the long axis lies
    along y, so an offset h along y is h / 0.5 sigmas away."""
    c = math.cos(math.pi / 4)
    m, ls, q, lg = _scene([[0, 0, 0], [5, 0.3, 0]], [[0.01] * 3, [0.5, 0.1, 0.1]], [0.5, 0.9],
                          quats=[[1, 0, 0, 0], [c, 0, 0, c]])
    v = V.visibility(m, ls, q, lg, [10.0, 0.0, 0.0])
    assert v[0] == pytest.approx(1.0 - 0.9 * math.exp(-0.5 * (0.3 / 0.5) ** 2), rel=1e-12)


def test_segment_cut_offs_and_product():
    """Occluders beyond the light or behind the origin do nothing, a faint one
    (alpha < 1/255) does nothing, a dense one clamps at 0.99, and two on the
    segment multiply."""
    cen = [[0, 0, 0], [12, 0, 0], [-3, 0, 0], [4, 0.9, 0], [6, 0, 0], [8, 0.1, 0]]
    sc = [[0.01] * 3, [0.3] * 3, [0.3] * 3, [0.2] * 3, [0.3] * 3, [0.3] * 3]
    op = [0.5, 0.99, 0.99, 0.9, 0.999, 0.5]
    m, ls, q, lg = _scene(cen, sc, op)
    v = V.visibility(m, ls, q, lg, [10.0, 0.0, 0.0])
    faint = 0.9 * math.exp(-0.5 * (0.9 / 0.2) ** 2)
    assert faint < 1 / 255
    expected = (1 - 0.99) * (1 - 0.5 * math.exp(-0.5 * (0.1 / 0.3) ** 2))
    assert v[0] == pytest.approx(expected, rel=1e-12)


def test_floor_reports_zero():
    cen = [[0, 0, 0]] + [[1 + k, 0, 0] for k in range(3)]
    m, ls, q, lg = _scene(cen, [[0.01] * 3] + [[0.3] * 3] * 3, [0.5, 0.999, 0.999, 0.999])
    v = V.visibility(m, ls, q, lg, [10.0, 0.0, 0.0])
    assert 0.01 ** 3 < 1e-4 <= 0.01 ** 2
    assert v[0] == 0.0


def test_densest_point_matches_a_numerical_line_search():
    """t* and D2 of the whitened-frame closed form against a bounded scalar
    minimisation of the Mahalanobis distance along the ray, with the
    covariance built by scipy's rotation (x, y, z, w order)."""
    g = scene.make_gaussians(6, 0, seed=8)
    g.log_scales += 2.0
    mu = g.means.T.astype(np.float64)
    P = np.array([1.7, 1.7, 1.7])
    Wm = V.whitening(g.log_scales, g.quats)
    for i in range(2):
        d = (P - mu[i]) / np.linalg.norm(P - mu[i])
        for j in range(6):
            if j == i:
                continue
            q = g.quats[:, j].astype(np.float64)
            R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
            S = np.diag(np.exp(2.0 * g.log_scales[:, j].astype(np.float64)))
            Ainv = np.linalg.inv(R @ S @ R.T)
            f = lambda t: (mu[i] + t * d - mu[j]) @ Ainv @ (mu[i] + t * d - mu[j])  # noqa: E731
            r = minimize_scalar(f, bracket=(-5, 5), tol=1e-12)
            u = Wm[j] @ (mu[i] - mu[j])
            w = Wm[j] @ d
            ts = -(u @ w) / (w @ w)
            D2 = np.cross(u, w) @ np.cross(u, w) / (w @ w)
            assert ts == pytest.approx(r.x, abs=1e-6)
            assert D2 == pytest.approx(r.fun, rel=1e-9, abs=1e-12)


def test_order_invariance():
    g = scene.make_gaussians(40, 0, seed=9)
    g.log_scales += 2.0
    P = [1.7, 1.7, 1.7]
    v = V.visibility(g.means, g.log_scales, g.quats, g.opacity_logits, P)
    perm = np.random.default_rng(0).permutation(40)
    vp = V.visibility(g.means[:, perm], g.log_scales[:, perm], g.quats[:, perm], g.opacity_logits[perm], P)
    np.testing.assert_allclose(vp, v[perm], rtol=1e-12, atol=0)
    assert (v < 1).any() and (v > 0).any()


def test_prefilter_gives_the_same_bits():
    """The per-ray distance prefilter only drops Gaussians whose alpha stays
    below 1/255 on the whole line: values and margin flags are identical."""
    g = scene.make_gaussians(3000, 0, seed=13)
    g.log_scales = (g.log_scales + 1.0).astype(np.float32)
    light = scene.default_light().pos
    args = (g.means, g.log_scales, g.quats, g.opacity_logits, light)
    recv = np.random.default_rng(2).choice(g.n, 400, replace=False)
    a, fa = V.visibility(*args, margins=True, receivers=recv)
    b, fb = V.visibility(*args, margins=True, receivers=recv, prefilter=True)
    assert np.array_equal(a, b) and np.array_equal(fa, fb)
    assert np.any((a[recv] > 0) & (a[recv] < 1))
