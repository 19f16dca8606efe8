"""Thin Python binding of libsssgs.so (see include/sssgs.h) plus a
torch.autograd.Function around it.

Only argument marshalling happens here: every step of projection, binning,
compositing and shading runs in the library's HIP kernels.  PyTorch provides
device memory and the current HIP stream.  There is no CPU fallback: when the
library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsssgs.so")

OK, ERR_INVALID_ARG, ERR_CAPACITY, ERR_UNSUPPORTED, ERR_HIP = 0, -1, -2, -3, -4
PREC_FP32, PREC_BF16 = 0, 1
PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "albedo", "roughness", "metallic", "sss",
               "features", "sh")

_fp = ct.POINTER(ct.c_float)


class Gaussians(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("feat_dim", ct.c_int32), ("sh_degree", ct.c_int32)] + \
               [(k, ct.c_void_p) for k in PARAM_NAMES]


class GaussianGrads(ct.Structure):
    _fields_ = [(k, ct.c_void_p) for k in PARAM_NAMES]


class Camera(ct.Structure):
    _fields_ = [("R", ct.c_float * 9), ("t", ct.c_float * 3), ("fx", ct.c_float), ("fy", ct.c_float),
                ("cx", ct.c_float), ("cy", ct.c_float), ("width", ct.c_int32), ("height", ct.c_int32)]


class Light(ct.Structure):
    _fields_ = [("pos", ct.c_float * 3), ("intensity", ct.c_float * 3)]


class Mlp(ct.Structure):
    _fields_ = [("in_dim", ct.c_int32), ("width", ct.c_int32), ("hidden", ct.c_int32), ("out_dim", ct.c_int32),
                ("params", ct.c_void_p)]


class Options(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("accumulate_grads", ct.c_int32), ("radiance_features", ct.c_int32),
                ("deterministic", ct.c_int32), ("background", ct.c_float * 3)]


def make_options(precision: int, accumulate: bool = False, radiance_features: bool = False,
                 deterministic: bool = False, background=None) -> Options:
    bg = (0.0, 0.0, 0.0) if background is None else tuple(float(v) for v in background)
    return Options(int(precision), int(accumulate), int(radiance_features), int(deterministic),
                   (ct.c_float * 3)(*bg))


class Layout(ct.Structure):
    _fields_ = [("records", ct.c_size_t), ("rec_stride", ct.c_int32), ("depth_keys", ct.c_size_t),
                ("rects", ct.c_size_t), ("radii", ct.c_size_t), ("tile_ranges", ct.c_size_t),
                ("sorted_gauss", ct.c_size_t), ("t_final", ct.c_size_t),
                ("n_contrib", ct.c_size_t), ("status", ct.c_size_t), ("boxes", ct.c_size_t)]


EXPORTS = ("sssgs_mlp_param_count", "sssgs_workspace_bytes", "sssgs_render_forward", "sssgs_render_backward",
           "sssgs_l1_loss", "sssgs_workspace_status", "sssgs_workspace_layout", "sssgs_status_string",
           "sssgs_last_error", "sssgs_timing_enable", "sssgs_timing_read", "sssgs_timing_stages",
           "sssgs_timing_stage_name", "sssgs_image_loss_workspace_bytes", "sssgs_image_loss", "sssgs_adam_step",
           "sssgs_render_forward_lights", "sssgs_gaussian_mlp_param_count", "sssgs_gaussian_mlp_workspace_bytes",
           "sssgs_gaussian_mlp_forward", "sssgs_gaussian_mlp_backward", "sssgs_visibility_workspace_bytes",
           "sssgs_trace_visibility", "sssgs_image_loss_noalloc")


def load_library(path: str = LIB_PATH):
    """Load libsssgs.so and declare its signatures.  Raises if the file is absent."""
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -m paper_2408_12282_amd.build)")
    L = ct.CDLL(path)
    L.sssgs_mlp_param_count.restype = ct.c_int64
    L.sssgs_mlp_param_count.argtypes = [ct.c_int32] * 4
    L.sssgs_workspace_bytes.restype = ct.c_size_t
    L.sssgs_workspace_bytes.argtypes = [ct.c_int32] * 5 + [ct.c_int64]
    L.sssgs_render_forward.restype = ct.c_int
    L.sssgs_render_forward.argtypes = [ct.POINTER(Gaussians), ct.POINTER(Camera), ct.POINTER(Light),
                                       ct.POINTER(Mlp), ct.POINTER(Options), ct.c_void_p, ct.c_size_t, ct.c_int64,
                                       ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.POINTER(ct.c_int64), ct.c_void_p]
    L.sssgs_render_forward_lights.restype = ct.c_int
    L.sssgs_render_forward_lights.argtypes = [ct.POINTER(Gaussians), ct.POINTER(Camera), ct.POINTER(Light),
                                              ct.POINTER(ct.c_float), ct.c_int32, ct.POINTER(Mlp),
                                              ct.POINTER(Options), ct.c_void_p, ct.c_size_t, ct.c_int64,
                                              ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.POINTER(ct.c_int64),
                                              ct.c_void_p]
    L.sssgs_render_backward.restype = ct.c_int
    L.sssgs_render_backward.argtypes = [ct.POINTER(Gaussians), ct.POINTER(Camera), ct.POINTER(Light),
                                        ct.POINTER(Mlp), ct.POINTER(Options), ct.c_void_p, ct.c_size_t, ct.c_int64,
                                        ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                        ct.POINTER(GaussianGrads), ct.c_void_p, ct.c_void_p]
    L.sssgs_gaussian_mlp_param_count.restype = ct.c_int64
    L.sssgs_gaussian_mlp_param_count.argtypes = []
    L.sssgs_gaussian_mlp_workspace_bytes.restype = ct.c_size_t
    L.sssgs_gaussian_mlp_workspace_bytes.argtypes = [ct.c_int32]
    L.sssgs_gaussian_mlp_forward.restype = ct.c_int
    L.sssgs_gaussian_mlp_forward.argtypes = [ct.POINTER(Gaussians), ct.POINTER(Camera), ct.POINTER(Light),
                                             ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p,
                                             ct.c_void_p]
    L.sssgs_gaussian_mlp_backward.restype = ct.c_int
    L.sssgs_gaussian_mlp_backward.argtypes = [ct.POINTER(Gaussians), ct.POINTER(Camera), ct.POINTER(Light),
                                              ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t,
                                              ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                              ct.c_int32, ct.c_void_p]
    L.sssgs_visibility_workspace_bytes.restype = ct.c_size_t
    L.sssgs_visibility_workspace_bytes.argtypes = [ct.c_int32]
    L.sssgs_trace_visibility.restype = ct.c_int
    L.sssgs_trace_visibility.argtypes = [ct.POINTER(Gaussians), ct.POINTER(Light), ct.c_void_p, ct.c_size_t,
                                         ct.c_void_p, ct.c_void_p]
    L.sssgs_l1_loss.restype = ct.c_int
    L.sssgs_l1_loss.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_float, ct.c_void_p, ct.c_void_p,
                                ct.c_void_p]
    L.sssgs_image_loss_workspace_bytes.restype = ct.c_size_t
    L.sssgs_image_loss_workspace_bytes.argtypes = [ct.c_int32] * 3
    L.sssgs_image_loss.restype = ct.c_int
    L.sssgs_image_loss.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_float,
                                   ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_void_p, ct.c_void_p]
    L.sssgs_image_loss_noalloc.restype = ct.c_int
    L.sssgs_image_loss_noalloc.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_float,
                                           ct.c_void_p, ct.c_void_p, ct.c_void_p]
    L.sssgs_adam_step.restype = ct.c_int
    L.sssgs_adam_step.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_float,
                                  ct.c_float, ct.c_float, ct.c_float, ct.c_int32, ct.c_void_p]
    L.sssgs_workspace_status.restype = ct.c_int
    L.sssgs_workspace_status.argtypes = [ct.c_void_p] + [ct.c_int32] * 5 + [ct.c_int64, ct.c_void_p,
                                                                           ct.POINTER(ct.c_int32),
                                                                           ct.POINTER(ct.c_int64)]
    L.sssgs_workspace_layout.restype = ct.c_int
    L.sssgs_workspace_layout.argtypes = [ct.c_int32] * 5 + [ct.c_int64, ct.POINTER(Layout)]
    L.sssgs_status_string.restype = ct.c_char_p
    L.sssgs_status_string.argtypes = [ct.c_int]
    L.sssgs_last_error.restype = ct.c_char_p
    L.sssgs_last_error.argtypes = []
    L.sssgs_timing_enable.restype = ct.c_int
    L.sssgs_timing_enable.argtypes = [ct.c_int32]
    L.sssgs_timing_read.restype = ct.c_int
    L.sssgs_timing_read.argtypes = [ct.c_int32, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int32),
                                    ct.POINTER(ct.c_int32)]
    L.sssgs_timing_stages.restype = ct.c_int32
    L.sssgs_timing_stages.argtypes = []
    L.sssgs_timing_stage_name.restype = ct.c_char_p
    L.sssgs_timing_stage_name.argtypes = [ct.c_int32]
    return L


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class SSSGSError(RuntimeError):
    def __init__(self, status: int):
        L = lib()
        super().__init__(f"{L.sssgs_status_string(status).decode()}: {L.sssgs_last_error().decode()}")
        self.status = status


def _check(status: int):
    if status != OK:
        raise SSSGSError(status)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_contiguous() and t.dtype == torch.float32, "float32 contiguous tensors expected"
    return ct.c_void_p(t.data_ptr())


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ same-name C entry points

def sssgs_mlp_param_count(in_dim, width, hidden=3, out_dim=6) -> int:
    return int(lib().sssgs_mlp_param_count(in_dim, width, hidden, out_dim))


def sssgs_workspace_bytes(n, width, height, feat_dim, mlp_width, instance_capacity) -> int:
    return int(lib().sssgs_workspace_bytes(n, width, height, feat_dim, mlp_width, instance_capacity))


def sssgs_workspace_layout(n, width, height, feat_dim, mlp_width, instance_capacity) -> Layout:
    lay = Layout()
    _check(lib().sssgs_workspace_layout(n, width, height, feat_dim, mlp_width, instance_capacity, ct.byref(lay)))
    return lay


def sssgs_render_forward(g, cam, light, mlp, opt, workspace, ws_bytes, capacity, out_rgb, out_gbuffer, out_alpha,
                         want_count=False, stream=None):
    cnt = ct.c_int64(0)
    st = lib().sssgs_render_forward(ct.byref(g), ct.byref(cam), ct.byref(light), ct.byref(mlp) if mlp else None,
                                    ct.byref(opt), workspace, ws_bytes, capacity, out_rgb, out_gbuffer, out_alpha,
                                    ct.byref(cnt) if want_count else None, stream)
    return st, int(cnt.value)


def sssgs_render_forward_lights(g, cam, lights, weights, mlp, opt, workspace, ws_bytes, capacity, out_rgb,
                                out_gbuffer, out_alpha, want_count=False, stream=None):
    """lights: sequence of Light structures; weights: [len(lights)][3] floats (host)."""
    k = len(lights)
    arr = (Light * k)(*lights)
    w = (ct.c_float * (3 * k))(*[float(v) for row in weights for v in row])
    cnt = ct.c_int64(0)
    st = lib().sssgs_render_forward_lights(ct.byref(g), ct.byref(cam), arr, w, k, ct.byref(mlp) if mlp else None,
                                           ct.byref(opt), workspace, ws_bytes, capacity, out_rgb, out_gbuffer,
                                           out_alpha, ct.byref(cnt) if want_count else None, stream)
    return st, int(cnt.value)


def sssgs_render_backward(g, cam, light, mlp, opt, workspace, ws_bytes, capacity, gbuffer, drgb, dgbuf, dalpha,
                          grads, dmlp, stream=None):
    return lib().sssgs_render_backward(ct.byref(g), ct.byref(cam), ct.byref(light), ct.byref(mlp) if mlp else None,
                                       ct.byref(opt), workspace, ws_bytes, capacity, gbuffer, drgb, dgbuf, dalpha,
                                       ct.byref(grads), dmlp, stream)


def sssgs_l1_loss(pred, target, count, scale, loss_out, grad, stream=None):
    return lib().sssgs_l1_loss(pred, target, count, scale, loss_out, grad, stream)


def sssgs_image_loss_workspace_bytes(channels, height, width) -> int:
    return int(lib().sssgs_image_loss_workspace_bytes(channels, height, width))


def sssgs_image_loss(pred, target, channels, height, width, lambda_dssim, workspace, ws_bytes, loss_out, grad,
                     stream=None):
    return lib().sssgs_image_loss(pred, target, channels, height, width, lambda_dssim, workspace, ws_bytes,
                                  loss_out, grad, stream)


def sssgs_image_loss_noalloc(pred, target, channels, height, width, lambda_dssim, loss_out, grad, stream=None):
    return lib().sssgs_image_loss_noalloc(pred, target, channels, height, width, lambda_dssim, loss_out, grad,
                                          stream)


def sssgs_adam_step(param, grad, m, v, count, lr, beta1, beta2, eps, step, stream=None):
    return lib().sssgs_adam_step(param, grad, m, v, count, lr, beta1, beta2, eps, step, stream)


def image_loss(pred: torch.Tensor, target: torch.Tensor, lambda_dssim: float = 0.2, want_grad: bool = True):
    """(1 - lambda) L1 + lambda (1 - SSIM) of [C][H][W] float32 device images; returns (loss[1], dL/dpred)."""
    C, H, W = pred.shape
    nb = sssgs_image_loss_workspace_bytes(C, H, W)
    ws = torch.empty(nb, dtype=torch.uint8, device=pred.device)
    loss = torch.empty(1, dtype=torch.float32, device=pred.device)
    grad = torch.empty_like(pred) if want_grad else None
    _check(sssgs_image_loss(_ptr(pred), _ptr(target), C, H, W, lambda_dssim, ct.c_void_p(ws.data_ptr()), nb,
                            _ptr(loss), _ptr(grad), _stream()))
    return loss, grad


def adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """In-place Adam update of a float32 device tensor (moments m, v of the same shape)."""
    _check(sssgs_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(), lr, beta1, beta2, eps, step,
                           _stream()))


def lr_schedule(step: int, base: float = 1e-3, gamma: float = 0.99, every: int = 1000) -> float:
    """Learning rate of the network at a step: base lr 0.001 decayed by 0.99 every 1000 steps
    (Appendix "Training")."""
    return base * gamma ** (step // every)


def sssgs_workspace_status(workspace, n, width, height, feat_dim, mlp_width, capacity, stream=None):
    flags = ct.c_int32(0)
    num = ct.c_int64(0)
    _check(lib().sssgs_workspace_status(workspace, n, width, height, feat_dim, mlp_width, capacity, stream,
                                        ct.byref(flags), ct.byref(num)))
    return int(flags.value), int(num.value)


def sssgs_timing_enable(on: bool):
    _check(lib().sssgs_timing_enable(int(bool(on))))


def sssgs_timing_read() -> dict:
    """Stage name -> (summed ms, launches) of the calls timed since the last read."""
    L = lib()
    k = L.sssgs_timing_stages()
    ms = (ct.c_double * k)()
    cnt = (ct.c_int32 * k)()
    ns = ct.c_int32(0)
    _check(L.sssgs_timing_read(k, ms, cnt, ct.byref(ns)))
    return {L.sssgs_timing_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(ns.value)}


def sssgs_timing_stages() -> int:
    return int(lib().sssgs_timing_stages())


def sssgs_timing_stage_name(k: int) -> str:
    return lib().sssgs_timing_stage_name(k).decode()


# ------------------------------------------------------------------ helpers

def make_camera(cam) -> Camera:
    """From scene.Camera (numpy R, t, intrinsics)."""
    return Camera((ct.c_float * 9)(*[float(v) for v in cam.R.reshape(-1)]),
                  (ct.c_float * 3)(*[float(v) for v in cam.t.reshape(-1)]),
                  float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy), int(cam.width), int(cam.height))


def make_light(light) -> Light:
    return Light((ct.c_float * 3)(*[float(v) for v in light.pos]),
                 (ct.c_float * 3)(*[float(v) for v in light.intensity]))


def gaussians_struct(params: dict, feat_dim: int, sh_degree: int) -> Gaussians:
    n = int(params["means"].shape[1])
    return Gaussians(n, feat_dim, sh_degree, *[_ptr(params.get(k)) if params.get(k) is not None
                                               and params[k].numel() else None for k in PARAM_NAMES])


def grads_struct(grads: dict) -> GaussianGrads:
    return GaussianGrads(*[_ptr(grads.get(k)) if grads.get(k) is not None and grads[k].numel() else None
                           for k in PARAM_NAMES])


class View:
    """Everything one view needs on the device: workspace and output buffers."""

    def __init__(self, n: int, width: int, height: int, feat_dim: int, mlp_width: int, capacity: int,
                 device="cuda"):
        self.n, self.width, self.height, self.feat_dim, self.mlp_width = n, width, height, feat_dim, mlp_width
        self.capacity = int(capacity)
        self.C = 10 + feat_dim
        self.ws_bytes = sssgs_workspace_bytes(n, width, height, feat_dim, mlp_width, self.capacity)
        if self.ws_bytes == 0:
            raise SSSGSError(ERR_INVALID_ARG)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.layout = sssgs_workspace_layout(n, width, height, feat_dim, mlp_width, self.capacity)
        # forward calls on this workspace so far: a backward must follow the
        # forward whose state the workspace holds (SSSGSRender checks it)
        self.generation = 0

    def region(self, offset: int, count: int, dtype=torch.int32) -> torch.Tensor:
        """A typed view of `count` elements of the workspace at byte `offset`."""
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return self.workspace[offset:offset + nbytes].view(dtype)


def render_forward(view: View, params: dict, sh_degree: int, cam: Camera, light: Light, mlp_params=None,
                   mlp_width: int = 64, precision: int = PREC_BF16, want_count: bool = False,
                   radiance_features: bool = False, background=None):
    """One forward call.  Returns (rgb [3,H,W], gbuf [C,H,W], alpha [H,W], M or None).
    ``radiance_features``: Eq. 7 takes its radiances from feature planes 0-5
    (the outputs of the per-Gaussian network).  ``background``: colour behind
    the Gaussians (default black)."""
    dev = params["means"].device
    H, W = view.height, view.width
    rgb = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    gbuf = torch.empty((view.C, H, W), dtype=torch.float32, device=dev)
    alpha = torch.empty((H, W), dtype=torch.float32, device=dev)
    g = gaussians_struct(params, view.feat_dim, sh_degree)
    m = None
    if mlp_params is not None:
        m = Mlp(view.feat_dim + 42, mlp_width, 3, 6, _ptr(mlp_params))
    opt = make_options(precision, radiance_features=radiance_features, background=background)
    view.generation += 1
    st, cnt = sssgs_render_forward(g, cam, light, m, opt, ct.c_void_p(view.workspace.data_ptr()), view.ws_bytes,
                                   view.capacity, _ptr(rgb), _ptr(gbuf), _ptr(alpha), want_count, _stream())
    _check(st)
    return rgb, gbuf, alpha, (cnt if want_count else None)


def render_forward_lights(view: View, params: dict, sh_degree: int, cam: Camera, lights, weights, mlp_params=None,
                          mlp_width: int = 64, precision: int = PREC_BF16, want_count: bool = False):
    """Forward under several point lights: rgb = sum_k weights[k] * rgb(lights[k]) over one G-buffer.
    Returns (rgb [3,H,W], gbuf [C,H,W], alpha [H,W], M or None)."""
    dev = params["means"].device
    H, W = view.height, view.width
    rgb = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    gbuf = torch.empty((view.C, H, W), dtype=torch.float32, device=dev)
    alpha = torch.empty((H, W), dtype=torch.float32, device=dev)
    g = gaussians_struct(params, view.feat_dim, sh_degree)
    m = Mlp(view.feat_dim + 42, mlp_width, 3, 6, _ptr(mlp_params)) if mlp_params is not None else None
    opt = make_options(precision)
    view.generation += 1
    st, cnt = sssgs_render_forward_lights(g, cam, list(lights), weights, m, opt,
                                          ct.c_void_p(view.workspace.data_ptr()), view.ws_bytes, view.capacity,
                                          _ptr(rgb), _ptr(gbuf), _ptr(alpha), want_count, _stream())
    _check(st)
    return rgb, gbuf, alpha, (cnt if want_count else None)


def render_backward(view: View, params: dict, sh_degree: int, cam: Camera, light: Light, gbuf, drgb, dgbuf=None,
                    dalpha=None, mlp_params=None, mlp_width: int = 64, precision: int = PREC_BF16,
                    grads: Optional[dict] = None, dmlp: Optional[torch.Tensor] = None, accumulate: bool = False,
                    radiance_features: bool = False, deterministic: bool = False, background=None):
    dev = params["means"].device
    if grads is None:
        grads = {k: torch.zeros_like(v) for k, v in params.items() if v is not None}
    if mlp_params is not None and dmlp is None:
        dmlp = torch.zeros_like(mlp_params)
    g = gaussians_struct(params, view.feat_dim, sh_degree)
    m = Mlp(view.feat_dim + 42, mlp_width, 3, 6, _ptr(mlp_params)) if mlp_params is not None else None
    opt = make_options(precision, accumulate, radiance_features, deterministic, background)
    gs = grads_struct(grads)
    st = sssgs_render_backward(g, cam, light, m, opt, ct.c_void_p(view.workspace.data_ptr()), view.ws_bytes,
                               view.capacity, _ptr(gbuf), _ptr(drgb.contiguous()),
                               _ptr(dgbuf.contiguous()) if dgbuf is not None else None,
                               _ptr(dalpha.contiguous()) if dalpha is not None else None, gs,
                               _ptr(dmlp) if dmlp is not None else None, _stream())
    _check(st)
    del dev
    return grads, dmlp


class SSSGSRender(torch.autograd.Function):
    """(rgb, gbuffer, alpha) = render(Gaussian parameters, network parameters).

    Differentiable w.r.t. every Gaussian parameter tensor and the packed
    network parameters.  ``ctx_args`` = (view, sh_degree, Camera, Light,
    mlp_width, precision, deterministic, background).  The forward reads the
    instance count back (one wait on the stream) and raises SSSGSError
    (ERR_CAPACITY) when the view's capacity is too small.  The backward uses
    the state the forward left in the view's workspace: it raises if another
    forward ran on the same view in between.
    """

    @staticmethod
    def forward(ctx, ctx_args, mlp_params, *tensors):
        view, sh_degree, cam, light, mlp_width, precision, deterministic, background = ctx_args
        params = {k: (t if t is not None and t.numel() else None) for k, t in zip(PARAM_NAMES, tensors)}
        rgb, gbuf, alpha, _ = render_forward(view, params, sh_degree, cam, light, mlp_params, mlp_width, precision,
                                             want_count=True, background=background)
        ctx.ctx_args = ctx_args
        ctx.generation = view.generation
        ctx.save_for_backward(gbuf, mlp_params if mlp_params is not None else torch.empty(0), *[
            t if t is not None else torch.empty(0) for t in tensors])
        ctx.has_mlp = mlp_params is not None
        return rgb, gbuf, alpha

    @staticmethod
    def backward(ctx, drgb, dgbuf, dalpha):
        view, sh_degree, cam, light, mlp_width, precision, deterministic, background = ctx.ctx_args
        if view.generation != ctx.generation:
            raise RuntimeError("SSSGSRender: another forward ran on this view before the backward; "
                               "use one View per forward whose backward is pending")
        saved = ctx.saved_tensors
        gbuf = saved[0]
        mlp_params = saved[1] if ctx.has_mlp else None
        params = {k: (t if t.numel() else None) for k, t in zip(PARAM_NAMES, saved[2:])}
        drgb = drgb if drgb is not None else torch.zeros((3, view.height, view.width), device=gbuf.device)
        grads, dmlp = render_backward(view, params, sh_degree, cam, light, gbuf, drgb.contiguous(),
                                      dgbuf.contiguous() if dgbuf is not None else None,
                                      dalpha.contiguous() if dalpha is not None else None, mlp_params, mlp_width,
                                      precision, deterministic=deterministic, background=background)
        out = [grads.get(k) if params.get(k) is not None else None for k in PARAM_NAMES]
        return (None, dmlp, *out)


def render(view: View, params: dict, sh_degree: int, cam: Camera, light: Light, mlp_params=None,
           mlp_width: int = 64, precision: int = PREC_BF16, deterministic: bool = False, background=None):
    """Differentiable render (torch.autograd): returns (rgb, gbuffer, alpha)."""
    tensors: Sequence = [params.get(k) for k in PARAM_NAMES]
    bg = None if background is None else tuple(float(v) for v in background)
    return SSSGSRender.apply((view, sh_degree, cam, light, mlp_width, precision, bool(deterministic), bg),
                             mlp_params, *tensors)


# ----------------------------------------------------------------- per-Gaussian network

def gaussian_mlp_param_count() -> int:
    return int(lib().sssgs_gaussian_mlp_param_count())


def gaussian_mlp_workspace(n: int, device="cuda") -> torch.Tensor:
    nb = int(lib().sssgs_gaussian_mlp_workspace_bytes(int(n)))
    return torch.empty(nb, dtype=torch.uint8, device=device)


def gaussian_mlp_forward(params: dict, cam: Camera, light: Light, visibility: torch.Tensor, gmlp: torch.Tensor,
                         workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Feature planes [8, N] = incident light | SSS radiance | visibility | 1 of
    the per-Gaussian network (see include/sssgs.h).  A backward needs the
    records this call leaves in ``workspace``: pass the same workspace to
    both."""
    n = int(params["means"].shape[1])
    if workspace is None:
        workspace = gaussian_mlp_workspace(n, params["means"].device)
    feats = torch.empty((8, n), dtype=torch.float32, device=params["means"].device)
    g = gaussians_struct(params, 0, -1)
    _check(lib().sssgs_gaussian_mlp_forward(ct.byref(g), ct.byref(cam), ct.byref(light), _ptr(visibility),
                                            _ptr(gmlp), ct.c_void_p(workspace.data_ptr()), workspace.numel(),
                                            _ptr(feats), _stream()))
    return feats


def gaussian_mlp_backward(params: dict, cam: Camera, light: Light, visibility: torch.Tensor, gmlp: torch.Tensor,
                          dfeat: torch.Tensor, grads: dict, dvis: torch.Tensor, dgmlp: torch.Tensor,
                          workspace: torch.Tensor, accumulate: bool = False):
    """Adds the network's share to grads['means'|'log_scales'|'quats'];
    writes (or adds) dvis and dgmlp.  ``workspace`` is the one the forward
    of the same inputs used."""
    g = gaussians_struct(params, 0, -1)
    _check(lib().sssgs_gaussian_mlp_backward(ct.byref(g), ct.byref(cam), ct.byref(light), _ptr(visibility),
                                             _ptr(gmlp), _ptr(dfeat.contiguous()), ct.c_void_p(workspace.data_ptr()),
                                             workspace.numel(), _ptr(grads["means"]), _ptr(grads["log_scales"]),
                                             _ptr(grads["quats"]), _ptr(dvis), _ptr(dgmlp), int(accumulate),
                                             _stream()))


def render_gaussian_mlp_forward(view: View, params: dict, cam: Camera, light: Light, visibility: torch.Tensor,
                                gmlp: torch.Tensor, workspace: torch.Tensor, want_count: bool = False):
    """Per-Gaussian network -> projection and compositing of the 18-plane
    G-buffer -> Eq. 7 from the composited radiances.  ``view`` has feat_dim 8
    and no per-pixel network; ``workspace`` (gaussian_mlp_workspace) keeps the
    network's records for the backward.  Returns (rgb, gbuf, alpha, features,
    M or None)."""
    feats = gaussian_mlp_forward(params, cam, light, visibility, gmlp, workspace)
    p = dict(params, features=feats)
    rgb, gbuf, alpha, cnt = render_forward(view, p, -1, cam, light, None, 64, PREC_FP32, want_count,
                                           radiance_features=True)
    return rgb, gbuf, alpha, feats, cnt


def render_gaussian_mlp_backward(view: View, params: dict, cam: Camera, light: Light, visibility: torch.Tensor,
                                 gmlp: torch.Tensor, feats: torch.Tensor, gbuf, drgb, workspace: torch.Tensor,
                                 dgbuf=None, dalpha=None, grads: Optional[dict] = None,
                                 dvis: Optional[torch.Tensor] = None, dgmlp: Optional[torch.Tensor] = None):
    """Gradients of every Gaussian parameter (dict), of the visibility and of
    the network parameters (all overwritten; pass buffers to reuse them)."""
    p = dict(params, features=feats)
    if grads is None:
        grads = {k: torch.empty_like(v) for k, v in p.items() if v is not None}
    else:
        grads = dict(grads)
        grads.setdefault("features", torch.empty_like(feats))
    render_backward(view, p, -1, cam, light, gbuf, drgb, dgbuf, dalpha, None, 64, PREC_FP32, grads=grads,
                    radiance_features=True)
    dvis = torch.empty_like(visibility) if dvis is None else dvis
    dgmlp = torch.empty_like(gmlp) if dgmlp is None else dgmlp
    gaussian_mlp_backward(params, cam, light, visibility, gmlp, grads["features"], grads, dvis, dgmlp, workspace)
    dfeat = grads.pop("features")
    return grads, dvis, dgmlp, dfeat


# ----------------------------------------------------------------- ray-traced visibility

def visibility_workspace(n: int, device="cuda") -> torch.Tensor:
    nb = int(lib().sssgs_visibility_workspace_bytes(int(n)))
    return torch.empty(nb, dtype=torch.uint8, device=device)


def trace_visibility(params: dict, light: Light, workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Each Gaussian's visibility of the light [N] by ray tracing through the
    other Gaussians (see include/sssgs.h); usable as the per-Gaussian
    network's visibility input."""
    n = int(params["means"].shape[1])
    if workspace is None:
        workspace = visibility_workspace(n, params["means"].device)
    vis = torch.empty(n, dtype=torch.float32, device=params["means"].device)
    g = gaussians_struct(params, 0, -1)
    _check(lib().sssgs_trace_visibility(ct.byref(g), ct.byref(light), ct.c_void_p(workspace.data_ptr()),
                                        workspace.numel(), _ptr(vis), _stream()))
    return vis
