"""Seeded synthetic inputs for the deferred Gaussian-splatting renderer.

This module only draws random numbers and builds cameras; it holds none of the
rendering arithmetic.  Both the HIP path and the CPU oracle consume what it
produces, so it is the single place where test and benchmark inputs are made.

The paper's OLAT captures (Sec. 4, "Dataset") are not available; these scenes
stand in for them with the shapes and distributions of the five workloads:
means uniform in [-1,1]^3, log-scales N(-4, 0.5), random unit quaternions,
opacity logits N(0,1), albedo U[0,1]^3, roughness U[0.1,1], metallic U[0,1],
subsurfaceness U[0,1] (the per-Gaussian ``sss`` of Eq. 7), features N(0,0.1),
degree-3 SH colour N(0,0.1) with a zero DC term.  Gaussian arrays are
structure-of-arrays float32, shape [k, N] (one plane per component).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

TILE = 16


@dataclasses.dataclass
class Gaussians:
    means: np.ndarray            # [3, N]
    log_scales: np.ndarray       # [3, N]
    quats: np.ndarray            # [4, N]  (w, x, y, z), not necessarily unit
    opacity_logits: np.ndarray   # [N]
    albedo: np.ndarray           # [3, N]
    roughness: np.ndarray        # [N]
    metallic: np.ndarray         # [N]
    sss: np.ndarray              # [N]
    features: np.ndarray         # [F, N] (F may be 0)
    sh: Optional[np.ndarray]     # [48, N] plane k*3+c, or None

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def feat_dim(self) -> int:
        return int(self.features.shape[0])

    @property
    def sh_degree(self) -> int:
        return -1 if self.sh is None else 3

    def arrays(self):
        """Name -> array for every parameter group (sh omitted when absent)."""
        d = {k: getattr(self, k) for k in PARAM_NAMES}
        if self.sh is None:
            del d["sh"]
        return d

    def subset(self, idx) -> "Gaussians":
        return Gaussians(**{k: (None if v is None else np.ascontiguousarray(v[..., idx]))
                            for k, v in dataclasses.asdict(self).items()})


PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "albedo",
               "roughness", "metallic", "sss", "features", "sh")


@dataclasses.dataclass
class Camera:
    R: np.ndarray        # [3,3] world -> camera rotation (rows: right, down, forward)
    t: np.ndarray        # [3]   p_cam = R p + t
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def center(self) -> np.ndarray:
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


@dataclasses.dataclass
class Light:
    pos: np.ndarray        # [3]
    intensity: np.ndarray  # [3]


@dataclasses.dataclass
class MLP:
    """Residual shading network of Eq. 6, evaluated per pixel.

    ``params`` packs W0 [width, in_pad], b0 [width], then (hidden-1) blocks of
    W [width, width], b [width], then W_out [out_dim, width], b_out [out_dim];
    all row-major float32.  Columns of W0 at and beyond ``in_dim`` multiply the
    zero padding of the input vector.
    """
    in_dim: int
    width: int
    hidden: int
    out_dim: int
    params: np.ndarray

    @property
    def in_pad(self) -> int:
        return mlp_in_pad(self.in_dim)


def mlp_in_pad(in_dim: int) -> int:
    return (in_dim + 31) // 32 * 32


def mlp_in_dim(feat_dim: int) -> int:
    # blended features | Fourier encoding of position (6 octaves x sin,cos x 3) | w_out | w_in
    return feat_dim + 36 + 3 + 3


def mlp_param_count(in_dim: int, width: int, hidden: int, out_dim: int) -> int:
    p = width * mlp_in_pad(in_dim) + width
    p += (hidden - 1) * (width * width + width)
    p += out_dim * width + out_dim
    return p


def _streams(seed: int, k: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def make_gaussians(n: int, feat_dim: int = 0, sh: bool = False, seed: int = 0) -> Gaussians:
    r = _streams(seed, 10)
    f32 = np.float32
    means = r[0].uniform(-1.0, 1.0, size=(3, n)).astype(f32)
    log_scales = r[1].normal(-4.0, 0.5, size=(3, n)).astype(f32)
    q = r[2].normal(0.0, 1.0, size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    quats = q.astype(f32)
    logits = r[3].normal(0.0, 1.0, size=n).astype(f32)
    albedo = r[4].uniform(0.0, 1.0, size=(3, n)).astype(f32)
    rough = r[5].uniform(0.1, 1.0, size=n).astype(f32)
    metal = r[6].uniform(0.0, 1.0, size=n).astype(f32)
    sss = r[7].uniform(0.0, 1.0, size=n).astype(f32)
    feats = r[8].normal(0.0, 0.1, size=(feat_dim, n)).astype(f32)
    shc = None
    if sh:
        shc = r[9].normal(0.0, 0.1, size=(48, n)).astype(f32)
        shc[0:3] = 0.0
    return Gaussians(means, log_scales, quats, logits, albedo, rough, metal, sss, feats, shc)


def focal_from_fov(width: int, fov_deg: float = 50.0) -> float:
    """Pinhole focal length in pixels for a horizontal field of view."""
    return width / (2.0 * math.tan(math.radians(fov_deg) / 2.0))


def look_at_camera(position, width: int, height: int, fov_deg: float = 50.0,
                   target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> Camera:
    """Camera at ``position`` looking at ``target``; camera axes x right, y down, z forward."""
    p = np.asarray(position, np.float64)
    fwd = np.asarray(target, np.float64) - p
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32)
    t = (-(R.astype(np.float64) @ p)).astype(np.float32)
    f = focal_from_fov(width, fov_deg)
    return Camera(R, t, float(np.float32(f)), float(np.float32(f)),
                  width / 2.0, height / 2.0, int(width), int(height))


def default_light() -> Light:
    d = np.ones(3) / math.sqrt(3.0)
    return Light((3.0 * d).astype(np.float32), np.full(3, 9.0, np.float32))


def make_mlp(feat_dim: int, width: int = 64, hidden: int = 3, out_dim: int = 6, seed: int = 0) -> MLP:
    """He-normal weights N(0, 2/fan_in) with the true fan-in; zero biases; padding columns zero."""
    in_dim = mlp_in_dim(feat_dim)
    in_pad = mlp_in_pad(in_dim)
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x4D4C50]))
    chunks: List[np.ndarray] = []
    w0 = np.zeros((width, in_pad))
    w0[:, :in_dim] = rng.normal(0.0, math.sqrt(2.0 / in_dim), size=(width, in_dim))
    chunks += [w0.ravel(), np.zeros(width)]
    for _ in range(hidden - 1):
        chunks += [rng.normal(0.0, math.sqrt(2.0 / width), size=(width, width)).ravel(), np.zeros(width)]
    chunks += [rng.normal(0.0, math.sqrt(2.0 / width), size=(out_dim, width)).ravel(), np.zeros(out_dim)]
    params = np.concatenate(chunks).astype(np.float32)
    assert params.size == mlp_param_count(in_dim, width, hidden, out_dim)
    return MLP(in_dim, width, hidden, out_dim, params)


# Per-Gaussian network of the pipeline figure / appendix "Network": layer
# shapes (rows, columns) of the packed parameter vector, in order: three trunk
# layers, the incident-light head's hidden and output layers, the SSS head.
GMLP_IN = 42
GMLP_LAYERS = ((64, GMLP_IN), (32, 64), (32, 32), (32, 32), (3, 32), (3, 32))


def gmlp_param_count() -> int:
    return sum(r * c + r for r, c in GMLP_LAYERS)


def make_gaussian_mlp(seed: int = 0) -> np.ndarray:
    """Packed float32 parameters W [rows, cols] then b [rows] per layer of
    GMLP_LAYERS: He-normal weights N(0, 2/fan_in), biases N(0, 0.1)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x474D4C50]))
    chunks: List[np.ndarray] = []
    for r, c in GMLP_LAYERS:
        chunks += [rng.normal(0.0, math.sqrt(2.0 / c), size=(r, c)).ravel(), rng.normal(0.0, 0.1, size=r)]
    return np.concatenate(chunks).astype(np.float32)


def make_visibility(n: int, seed: int = 0) -> np.ndarray:
    """Per-Gaussian light visibility v, U[0, 1] float32."""
    return np.random.default_rng(np.random.SeedSequence([seed, 0x564953])).uniform(0.0, 1.0, n).astype(np.float32)


def fibonacci_cameras(k: int, radius: float, width: int, height: int, fov_deg: float = 50.0):
    """k cameras on a Fibonacci sphere of the given radius, all looking at the origin."""
    cams = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    for i in range(k):
        y = 1.0 - (2.0 * i + 1.0) / k
        rr = math.sqrt(max(0.0, 1.0 - y * y))
        phi = i * golden
        pos = radius * np.array([rr * math.cos(phi), y, rr * math.sin(phi)])
        cams.append(look_at_camera(pos, width, height, fov_deg))
    return cams


def environment_lights(k: int, radius: float = 30.0):
    """Light samples of a synthetic HDR environment for image-based lighting:
    k directions on a Fibonacci sphere, each a point light at `radius` whose
    intensity radius^2 gives unit irradiance at the origin (white light), and a
    per-channel weight = environment radiance x the sample's solid angle 4 pi / k.
    The environment (no captured maps are available) is a blue sky above the
    horizon, a brown ground below and a small warm sun.  Returns (lights, weights [k][3])."""
    golden = math.pi * (3.0 - math.sqrt(5.0))
    sun = np.array([1.0, 2.0, 0.5]) / math.sqrt(5.25)
    lights, weights = [], []
    for i in range(k):
        y = 1.0 - (2.0 * i + 1.0) / k
        rr = math.sqrt(max(0.0, 1.0 - y * y))
        phi = i * golden
        d = np.array([rr * math.cos(phi), y, rr * math.sin(phi)])
        rad = (np.array([0.3, 0.5, 0.9]) * math.sqrt(max(y, 0.0)) + np.array([0.2, 0.15, 0.1]) * max(-y, 0.0)
               + np.array([8.0, 7.0, 5.0]) * max(float(d @ sun), 0.0) ** 64)
        lights.append(Light((radius * d).astype(np.float32), np.full(3, radius * radius, np.float32)))
        weights.append((rad * 4.0 * math.pi / k).astype(np.float32))
    return lights, np.stack(weights)


@dataclasses.dataclass
class Workload:
    name: str
    gaussians: Gaussians
    cameras: List[Camera]
    lights: List[Light]
    mlp: Optional[MLP]
    backward: bool


def workload(cfg: int, seed: int = 0, n: Optional[int] = None) -> Workload:
    """The five synthetic workloads (1-based ``cfg``).  ``n`` overrides the Gaussian count."""
    if cfg == 1:
        g = make_gaussians(n or 1000, 0, False, seed)
        cams = [look_at_camera((0, 0, 3), 128, 128)]
        return Workload("1k-128sq-gbuffer-ggx-fwd", g, cams, [default_light()], None, False)
    if cfg == 2:
        g = make_gaussians(n or 100_000, 16, False, seed)
        cams = [look_at_camera((0, 0, 3), 800, 800)]
        return Workload("100k-800sq-gbuffer-fwdbwd", g, cams, [default_light()], None, True)
    if cfg == 3:
        g = make_gaussians(n or 300_000, 16, False, seed)
        cams = [look_at_camera((0, 0, 3), 800, 800)]
        return Workload("300k-800sq-ggx-mlp-fwdbwd", g, cams, [default_light()], make_mlp(16, 64, 3, 6, seed), True)
    if cfg == 4:
        g = make_gaussians(n or 500_000, 16, False, seed)
        cams = fibonacci_cameras(8, 3.0, 800, 800)
        lights = [Light(cams[(k + 1) % 8].center.astype(np.float32), np.full(3, 9.0, np.float32)) for k in range(8)]
        return Workload("500k-800sq-8view-l1-train", g, cams, lights, make_mlp(16, 64, 3, 6, seed), True)
    if cfg == 5:
        g = make_gaussians(n or 1_000_000, 32, True, seed)
        cams = [look_at_camera((0, 0, 3), 1600, 1200)]
        return Workload("1M-1600x1200-sh3-f32-mlp128-fwdbwd", g, cams, [default_light()], make_mlp(32, 128, 3, 6, seed), True)
    raise ValueError(f"unknown workload {cfg}")


def upstream_weights(shape, seed: int) -> np.ndarray:
    """Fixed N(0,1) weights w for a scalar loss L = sum(w * output)."""
    return np.random.default_rng(np.random.SeedSequence([seed, 0x57])).normal(size=shape).astype(np.float32)
