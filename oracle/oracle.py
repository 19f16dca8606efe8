"""Python front end of the FP64 CPU oracle (``sssgs_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark.  The product path never imports this module.

Inputs are the float32 arrays of ``paper_2408_12282_amd.scene``; they are
widened exactly to float64 before the oracle sees them.  See the header of
``sssgs_oracle.c`` for what is computed and which passage of the paper each
step follows.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sssgs_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CH_ALB, CH_NRM, CH_ROUGH, CH_METAL, CH_SSS, CH_DEPTH, CH_FEAT = 0, 3, 6, 7, 8, 9, 10
TILE = 16

_dp = ct.POINTER(ct.c_double)
_ip = ct.POINTER(ct.c_int32)
_lp = ct.POINTER(ct.c_int64)
_up = ct.POINTER(ct.c_uint8)
_u64p = ct.POINTER(ct.c_uint64)


class OgGauss(ct.Structure):
    _fields_ = [("n", ct.c_int), ("feat_dim", ct.c_int), ("sh_degree", ct.c_int)] + [
        (k, _dp) for k in ("means", "log_scales", "quats", "opacity_logits", "albedo", "roughness",
                           "metallic", "sss", "features", "sh")]


class OgCam(ct.Structure):
    _fields_ = [("R", ct.c_double * 9), ("t", ct.c_double * 3), ("fx", ct.c_double), ("fy", ct.c_double),
                ("cx", ct.c_double), ("cy", ct.c_double), ("width", ct.c_int), ("height", ct.c_int)]


class OgLight(ct.Structure):
    _fields_ = [("pos", ct.c_double * 3), ("intensity", ct.c_double * 3)]


class OgMlp(ct.Structure):
    _fields_ = [("in_dim", ct.c_int), ("in_pad", ct.c_int), ("width", ct.c_int), ("hidden", ct.c_int),
                ("out_dim", ct.c_int), ("bf16", ct.c_int), ("params", _dp), ("radiance_features", ct.c_int)]


class OgOut(ct.Structure):
    _fields_ = [("rgb", _dp), ("gbuf", _dp), ("alpha", _dp), ("gbuf_abs", _dp), ("net_margin", _dp),
                ("rgb_sens", _dp),
                ("n_contrib", _ip),
                ("pix_flag", _up),
                ("mean2d", _dp), ("conic", _dp), ("depth", _dp), ("opacity", _dp), ("channels", _dp),
                ("radius", _ip), ("rect", _ip), ("tiles_touched", _ip), ("g_flag", _up),
                ("tile_ranges", _lp), ("tile_list", _ip), ("list_capacity", ct.c_int64),
                ("num_instances", _lp), ("signature", _u64p)]


class OgUpstream(ct.Structure):
    _fields_ = [("drgb", _dp), ("dgbuf", _dp), ("dalpha", _dp)]


class OgGrads(ct.Structure):
    _fields_ = [(k, _dp) for k in ("means", "log_scales", "quats", "opacity_logits", "albedo", "roughness",
                                   "metallic", "sss", "features", "sh", "mlp")]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, strict IEEE: no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ct.CDLL(build())
        _lib.og_render.restype = ct.c_int
        _lib.og_render.argtypes = [ct.POINTER(OgGauss), ct.POINTER(OgCam), ct.POINTER(OgLight),
                                   ct.POINTER(OgMlp), ct.POINTER(ct.c_int), ct.POINTER(OgOut),
                                   ct.POINTER(OgUpstream), ct.POINTER(OgGrads), ct.c_int, _dp]
        _lib.og_round_bf16.restype = ct.c_double
        _lib.og_round_bf16.argtypes = [ct.c_double]
        _lib.og_brdf.restype = None
        _lib.og_brdf.argtypes = [_dp, _dp, _dp, ct.c_double, ct.c_double, ct.c_double, _dp, _dp]
        _lib.og_ggx_d.restype = ct.c_double
        _lib.og_ggx_d.argtypes = [ct.c_double, ct.c_double]
        _lib.og_sh_basis.restype = None
        _lib.og_sh_basis.argtypes = [_dp, _dp]
    return _lib


def _p(a, typ=_dp):
    return None if a is None else a.ctypes.data_as(typ)


def channels(feat_dim: int) -> int:
    return CH_FEAT + feat_dim


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def render(g, cam, light, mlp=None, bf16: bool = False, crop=None, drgb=None, dgbuf=None, dalpha=None,
           grads: bool = False, nthreads: int = 0, lists: bool = False, params64: Optional[dict] = None,
           sens: bool = False, radiance_features: bool = False, background=None):
    """Render one view (and optionally its backward) in FP64.

    ``g`` is a ``scene.Gaussians``; ``params64`` may override any of its arrays
    with float64 arrays (used by the finite-difference checks).  ``sens``
    also fills the shading-sensitivity diagnostic ``rgb_sens``.
    ``radiance_features`` (no per-pixel network): feature planes 0-2 are the
    incident light and 3-5 the SSS radiance of a per-Gaussian network, and
    Eq. 7 takes them from the composited buffers.  ``background`` (3 values,
    default black) is the colour behind the Gaussians: rgb = a L_out +
    T_final background.  Returns a dict of numpy arrays.
    """
    L = lib()
    n, F = g.n, g.feat_dim
    C = channels(F)
    H, W = cam.height, cam.width
    TX, TY = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    arr = {k: _f64(v) for k, v in g.arrays().items()}
    if params64:
        arr.update({k: _f64(v) for k, v in params64.items()})
    keep = []
    gs = OgGauss(n, F, g.sh_degree, *[_p(arr.get(k)) if arr.get(k) is not None and arr.get(k).size else None
                                      for k in ("means", "log_scales", "quats", "opacity_logits", "albedo",
                                                "roughness", "metallic", "sss", "features", "sh")])
    cs = OgCam((ct.c_double * 9)(*np.asarray(cam.R, np.float64).ravel()),
               (ct.c_double * 3)(*np.asarray(cam.t, np.float64)), cam.fx, cam.fy, cam.cx, cam.cy, W, H)
    ls = OgLight((ct.c_double * 3)(*np.asarray(light.pos, np.float64)),
                 (ct.c_double * 3)(*np.asarray(light.intensity, np.float64)))
    mp = None
    mlp_params = None
    if mlp is not None:
        mlp_params = _f64(params64["mlp"]) if (params64 and "mlp" in params64) else _f64(mlp.params)
        mp = OgMlp(mlp.in_dim, mlp.in_pad, mlp.width, mlp.hidden, mlp.out_dim, int(bf16), _p(mlp_params), 0)
    elif radiance_features:
        mp = OgMlp(0, 0, 0, 0, 0, 0, None, 1)
    o = {
        "rgb": np.zeros((3, H, W)), "gbuf": np.zeros((C, H, W)), "alpha": np.zeros((H, W)),
        "gbuf_abs": np.zeros((C, H, W)), "net_margin": np.zeros((H, W)), "rgb_sens": np.zeros((3, H, W)),
        "n_contrib": np.zeros((H, W), np.int32), "pix_flag": np.zeros((H, W), np.uint8),
        "mean2d": np.zeros((2, n)), "conic": np.zeros((3, n)), "depth": np.zeros(n), "opacity": np.zeros(n),
        "channels": np.zeros((C, n)),
        "radius": np.zeros(n, np.int32), "rect": np.zeros((4, n), np.int32),
        "tiles_touched": np.zeros(n, np.int32), "g_flag": np.zeros(n, np.uint8),
        "tile_ranges": np.zeros((TX * TY, 2), np.int64),
    }
    num = np.zeros(1, np.int64)
    sig = np.zeros(1, np.uint64)
    cap = 0
    tl = None
    if lists:
        # a first pass over rects gives M; render twice is wasteful, so size from the projection
        cap = int(_count_instances(g, cam, arr)) + 1
        tl = np.zeros(cap, np.int32)
    out = OgOut(_p(o["rgb"]), _p(o["gbuf"]), _p(o["alpha"]), _p(o["gbuf_abs"]), _p(o["net_margin"]),
                _p(o["rgb_sens"]) if sens else None,
                _p(o["n_contrib"], _ip),
                _p(o["pix_flag"], _up),
                _p(o["mean2d"]), _p(o["conic"]), _p(o["depth"]), _p(o["opacity"]), _p(o["channels"]),
                _p(o["radius"], _ip), _p(o["rect"], _ip), _p(o["tiles_touched"], _ip), _p(o["g_flag"], _up),
                _p(o["tile_ranges"], _lp), _p(tl, _ip), cap, _p(num, _lp), _p(sig, _u64p))
    upp = None
    gp = None
    gout = {}
    if drgb is not None or dgbuf is not None or dalpha is not None or grads:
        ups = [_f64(drgb), _f64(dgbuf), _f64(dalpha)]
        keep += ups
        upp = OgUpstream(*[_p(u) for u in ups])
        for k, v in arr.items():
            gout[k] = np.zeros_like(v, dtype=np.float64)
        if mlp is not None:
            gout["mlp"] = np.zeros(mlp.params.size)
        gp = OgGrads(*[_p(gout.get(k)) if gout.get(k) is not None and gout.get(k).size else None
                       for k in ("means", "log_scales", "quats", "opacity_logits", "albedo", "roughness",
                                 "metallic", "sss", "features", "sh", "mlp")])
    crop_arr = (ct.c_int * 4)(*crop) if crop is not None else None
    bg = None if background is None else np.ascontiguousarray(background, np.float64).reshape(3)
    rc = L.og_render(ct.byref(gs), ct.byref(cs), ct.byref(ls), ct.byref(mp) if mp is not None else None,
                     crop_arr, ct.byref(out), ct.byref(upp) if upp is not None else None,
                     ct.byref(gp) if gp is not None else None, int(nthreads), _p(bg))
    if rc != 0:
        raise RuntimeError(f"oracle og_render failed: {rc}")
    o["num_instances"] = int(num[0])
    o["signature"] = int(sig[0])
    if tl is not None:
        o["tile_list"] = tl[: o["num_instances"]]
    if gp is not None:
        o["grads"] = gout
    return o


def render_lights(g, cam, lights, weights, mlp=None, bf16: bool = False, nthreads: int = 0, sens: bool = False):
    """Image-based lighting by light samples (Appendix "Image Based Lighting"):
    the relit image is the sum over the samples of the single-light images,
    each scaled per channel by its weight (the environment's illumination of
    that sample).  Forward only, FP64, one full render per light.  The
    decision flags of the result combine those of every light (pix_flag: any;
    net_margin: the smallest); with ``sens`` the shading sensitivity is the
    |weight|-weighted sum of the lights' sensitivities."""
    out = None
    for light, w in zip(lights, weights):
        o = render(g, cam, light, mlp, bf16=bf16, nthreads=nthreads, sens=sens)
        w64 = np.asarray(w, np.float64)[:, None, None]
        contrib = w64 * o["rgb"]
        if out is None:
            out = dict(o)
            out["rgb"] = contrib
            out["rgb_sens"] = np.abs(w64) * o["rgb_sens"]
        else:
            out["rgb"] = out["rgb"] + contrib
            out["rgb_sens"] = out["rgb_sens"] + np.abs(w64) * o["rgb_sens"]
            out["pix_flag"] = np.maximum(out["pix_flag"], o["pix_flag"])
            out["net_margin"] = np.minimum(out["net_margin"], o["net_margin"])
    return out


def _count_instances(g, cam, arr) -> int:
    """Upper bound on the instance count: a projection-only oracle call."""
    L = lib()
    n = g.n
    tt = np.zeros(n, np.int32)
    gs = OgGauss(n, g.feat_dim, g.sh_degree, *[_p(arr.get(k)) if arr.get(k) is not None and arr.get(k).size
                                               else None for k in ("means", "log_scales", "quats",
                                                                   "opacity_logits", "albedo", "roughness",
                                                                   "metallic", "sss", "features", "sh")])
    cs = OgCam((ct.c_double * 9)(*np.asarray(cam.R, np.float64).ravel()),
               (ct.c_double * 3)(*np.asarray(cam.t, np.float64)), cam.fx, cam.fy, cam.cx, cam.cy,
               cam.width, cam.height)
    ls = OgLight((ct.c_double * 3)(0, 0, 0), (ct.c_double * 3)(0, 0, 0))
    out = OgOut()
    out.tiles_touched = _p(tt, _ip)
    crop = (ct.c_int * 4)(0, 0, 0, 0)
    rc = L.og_render(ct.byref(gs), ct.byref(cs), ct.byref(ls), None, crop, ct.byref(out), None, None, 0, None)
    if rc != 0:
        raise RuntimeError("oracle projection failed")
    return int(tt.astype(np.int64).sum())


def round_bf16(x: float) -> float:
    return lib().og_round_bf16(float(x))


def brdf(n, wo, wi, basecolor, rough, metal):
    fs = ct.c_double()
    fd = ct.c_double()
    a = [np.ascontiguousarray(v, np.float64) for v in (n, wo, wi)]
    lib().og_brdf(_p(a[0]), _p(a[1]), _p(a[2]), basecolor, rough, metal, ct.byref(fs), ct.byref(fd))
    return fs.value, fd.value


def ggx_d(noh: float, rough: float) -> float:
    return lib().og_ggx_d(noh, rough)


def sh_basis(d):
    Y = np.zeros(16)
    dd = np.ascontiguousarray(d, np.float64)
    lib().og_sh_basis(_p(dd), _p(Y))
    return Y
