"""Gaussian Wave Splatting hot path on MI355X (gfx950): thin Python binding of libgws.

The library (``include/gws.h``) does every step of the path on the GPU: per-Gaussian
preprocessing, the depth / support-radius sort, binning into frequency tiles, the
order-invariant spectrum accumulation of Eq. 12, the inverse 2D transform, and the
adjoint.  This module only marshals arguments: torch supplies device memory and the
stream, and the raw pointers go through ctypes.  If ``libgws.so`` has not been built the
import of the binding fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import threading
from typing import Dict, Optional, Sequence

__all__ = ["LIB_PATH", "GwsError", "Problem", "Context", "load_library", "render", "GaussianWaveSplat",
           "render_tilted", "TiltedGaussianWaveSplat", "TILTED_PARAMS",
           "STATUS", "XFORM_FFT_FP32", "XFORM_DFT_BF16X3", "check_gaussians", "check_tensor", "check_offsets"]

# The in-tree build; GWS_LIBRARY names another build of the same library (e.g. to compare two).
LIB_PATH = os.environ.get("GWS_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgws.so")

XFORM_FFT_FP32 = 0
XFORM_DFT_BF16X3 = 1
BLEND_OIT = 0
BLEND_EXACT = 1
MAX_LAMBDA = 4
FS_PHASE_INPUT = 1
FS_HALF_BAND = 2
FS_COMPLEX_OUTPUT = 4

STATUS = {0: "GWS_OK", -1: "GWS_ERR_INVALID_ARG", -2: "GWS_ERR_SHAPE", -3: "GWS_ERR_UNSUPPORTED",
          -4: "GWS_ERR_WORKSPACE", -5: "GWS_ERR_NO_DEVICE", -6: "GWS_ERR_HIP", -7: "GWS_ERR_OOM"}


class GwsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("pitch_x", ctypes.c_double),
                ("pitch_y", ctypes.c_double), ("n_lambda", ctypes.c_int32),
                ("lambdas", ctypes.c_double * MAX_LAMBDA), ("blend", ctypes.c_int32), ("xform", ctypes.c_int32),
                ("eps_support", ctypes.c_double), ("phase_mode", ctypes.c_int32), ("tile_config", ctypes.c_int32),
                ("ref_nu_x", ctypes.c_double), ("ref_nu_y", ctypes.c_double)]


_fp = ctypes.c_void_p


class _Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, _fp) for k in (
        "mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity", "amplitude", "phase")]


TILTED_PARAMS = ("mean_x", "mean_y", "depth", "quat_w", "quat_x", "quat_y", "quat_z", "scale_u", "scale_v",
                 "opacity", "amplitude", "phase")


class _TiltedGaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, _fp) for k in TILTED_PARAMS]


class _TiltedGrads(ctypes.Structure):
    _fields_ = [(k, _fp) for k in TILTED_PARAMS]


class _Output(ctypes.Structure):
    _fields_ = [("field", _fp), ("spectrum", _fp)]


class _Grads(ctypes.Structure):
    _fields_ = [(k, _fp) for k in ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity",
                                   "amplitude", "phase")]


class _Stats(ctypes.Structure):
    _fields_ = [("n_input", ctypes.c_int64), ("n_culled", ctypes.c_int64), ("n_tiles", ctypes.c_int64),
                ("n_items", ctypes.c_int64), ("chunk", ctypes.c_int64), ("n_pairs_evaluated", ctypes.c_int64),
                ("n_candidates", ctypes.c_int64), ("tile_config", ctypes.c_int32), ("graph_replayed", ctypes.c_int32),
                ("n_window_clamped", ctypes.c_int64)]


class _View(ctypes.Structure):
    _fields_ = [("world_to_view", ctypes.c_double * 12), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("near", ctypes.c_double),
                ("ray_to_holo", ctypes.c_double * 6), ("depth_scale", ctypes.c_double),
                ("depth_offset", ctypes.c_double), ("sh_degree", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _WorldGaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in ("mean", "quat", "scale", "opacity_sh")]


PLANE_FIELDS = ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity")


class _PlaneGaussians(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in PLANE_FIELDS]


class _Peaks(ctypes.Structure):
    _fields_ = [("trans_ops_per_s", ctypes.c_double), ("valu_ops_per_s", ctypes.c_double),
                ("hbm_bytes_per_s", ctypes.c_double)]


PARAMS = ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity", "amplitude", "phase")

# exported symbol -> (restype, argtypes)
_SIGNATURES = {
    "gws_abi_version": (ctypes.c_int, []),
    "gws_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gws_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    "gws_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "gws_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "gws_check_problem": (ctypes.c_int, [ctypes.POINTER(_Problem)]),
    "gws_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "gws_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.POINTER(_Gaussians),
                                   ctypes.POINTER(_Output), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gws_forward_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.POINTER(_Gaussians),
                                           ctypes.POINTER(_Output), ctypes.c_void_p]),
    "gws_workspace_size_tilted": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int64,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "gws_forward_tilted": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.POINTER(_TiltedGaussians),
                                          ctypes.POINTER(_Output), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gws_backward_tilted": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem),
                                           ctypes.POINTER(_TiltedGaussians), ctypes.c_void_p,
                                           ctypes.POINTER(_TiltedGrads), ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p]),
    "gws_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.POINTER(_Gaussians),
                                    ctypes.c_void_p, ctypes.POINTER(_Grads), ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p]),
    "gws_workspace_size_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t)]),
    "gws_forward_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_Gaussians),
                                           ctypes.POINTER(_Output), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gws_backward_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_Gaussians),
                                            ctypes.c_void_p, ctypes.POINTER(_Grads), ctypes.c_void_p,
                                            ctypes.c_size_t, ctypes.c_void_p]),
    "gws_dft_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "gws_dft2d": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                 ctypes.c_void_p]),
    "gws_tile_config_count": (ctypes.c_int, []),
    "gws_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int64, ctypes.c_char_p,
                                    ctypes.c_void_p]),
    "gws_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Stats)]),
    "gws_measure_peaks": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Peaks), ctypes.c_void_p]),
    "gws_l2_workspace_size": (ctypes.c_size_t, []),
    "gws_l2_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]),
    "gws_holographics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_View), ctypes.POINTER(_WorldGaussians),
                                        ctypes.POINTER(_PlaneGaussians), ctypes.c_void_p]),
    "gws_dpac_workspace_size": (ctypes.c_size_t, [ctypes.c_int32]),
    "gws_dpac_encode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p]),
    "gws_focal_stack_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_int32,
                                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "gws_focal_stack": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Problem), ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gws_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "gws_read_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]),
}

STAGES = ("prep_sort", "bin", "accumulate", "reduce", "xform_inverse", "xform_forward", "dtable", "adjoint",
          "grad_final", "loss", "dpac", "focal_stack", "holographics")

_lib = None
_lib_lock = threading.Lock()


def load_library(path: str = LIB_PATH):
    """Load libgws.so and declare every entry point.  Raises if it has not been built."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(path):
                raise ImportError("libgws.so is not built (%s); run python -m paper_2505_06582_amd.build" % path)
            lib = ctypes.CDLL(path)
            for name, (res, args) in _SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


@dataclasses.dataclass
class Problem:
    """Mirror of gws_problem."""

    nx: int
    ny: int
    pitch_x: float = 8e-6
    pitch_y: float = 8e-6
    lambdas: Sequence[float] = (520e-9,)
    xform: int = XFORM_FFT_FP32
    eps_support: float = 0.0
    phase_mode: int = 0
    tile_config: int = 0
    blend: int = BLEND_OIT
    ref_nu: Sequence[float] = (0.0, 0.0)  # reference plane wave's transverse frequency (cycles/m)

    @staticmethod
    def from_grid(grid, **kw) -> "Problem":
        kw.setdefault("ref_nu", tuple(getattr(grid, "ref_nu", (0.0, 0.0))))
        return Problem(nx=grid.nx, ny=grid.ny, pitch_x=grid.px, pitch_y=grid.py, lambdas=tuple(grid.lambdas), **kw)

    @property
    def n_lambda(self) -> int:
        return len(self.lambdas)

    def _c(self) -> _Problem:
        p = _Problem()
        p.nx, p.ny, p.pitch_x, p.pitch_y = self.nx, self.ny, self.pitch_x, self.pitch_y
        p.n_lambda = len(self.lambdas)
        for i in range(MAX_LAMBDA):
            p.lambdas[i] = float(self.lambdas[i]) if i < len(self.lambdas) else 0.0
        p.blend, p.xform, p.eps_support = self.blend, self.xform, self.eps_support
        p.phase_mode, p.tile_config = self.phase_mode, self.tile_config
        p.ref_nu_x, p.ref_nu_y = float(self.ref_nu[0]), float(self.ref_nu[1])
        return p


def _check(status: int, ctx_handle=None):
    if status != 0:
        lib = load_library()
        msg = lib.gws_last_error(ctx_handle)
        raise GwsError(status, (msg or b"").decode(errors="replace"))


def _torch():
    import torch  # imported lazily so the ABI tests run without touching torch.cuda
    return torch


def check_gaussians(g: Dict[str, "object"], n_lambda: int, params=PARAMS) -> int:
    """Number of Gaussians n after checking the sizes of the parameter tensors: every field
    holds n elements, amplitude n_lambda * n, laid out channel-major ([n_lambda][n]).  The
    kernels index these arrays by n alone, so a mis-sized tensor would be read out of bounds;
    raises ValueError before anything reaches the library."""
    missing = [k for k in params if k not in g or g[k] is None]
    if missing:
        raise ValueError("missing Gaussian parameters: %s" % ", ".join(missing))
    n = int(g["mean_x"].numel())
    for k in params:
        t = g[k]
        if k == "amplitude":
            ok = (t.dim() == 1 and t.numel() == n_lambda * n) or (t.dim() == 2 and tuple(t.shape) == (n_lambda, n))
            if not ok:
                raise ValueError("amplitude must have shape (%d, %d) (n_lambda, n) or %d elements, got %s"
                                 % (n_lambda, n, n_lambda * n, tuple(t.shape)))
        elif t.numel() != n:
            raise ValueError("%s has %d elements, mean_x has %d" % (k, t.numel(), n))
    return n


def check_tensor(t, name: str, shape, dtype_name: str):
    """Shape, dtype and contiguity of a tensor handed to the library (ValueError); the device is
    checked when its address is taken."""
    torch = _torch()
    if t is None:
        raise ValueError("%s is required" % name)
    if tuple(t.shape) != tuple(int(v) for v in shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if t.dtype != getattr(torch, dtype_name):
        raise ValueError("%s must be %s, got %s" % (name, dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _dptr(t) -> int:
    """Device address of a tensor going to the library; host tensors are rejected."""
    if not t.is_cuda:
        raise ValueError("a %s tensor of shape %s is on the host; the library takes CUDA tensors"
                         % (t.dtype, tuple(t.shape)))
    return t.data_ptr()


def check_offsets(offsets, n: int):
    """CSR scene offsets: n_scenes + 1 non-decreasing entries from 0 to n, 1..64 scenes."""
    offs = [int(v) for v in offsets]
    if len(offs) < 2 or len(offs) > 65 or offs[0] != 0 or offs[-1] != n or any(
            b < a for a, b in zip(offs, offs[1:])):
        raise ValueError("offsets must be 2..65 non-decreasing entries from 0 to n = %d, got %s" % (n, offs))
    return offs


def _gaussians_struct(g: Dict[str, "object"], n_lambda: int) -> _Gaussians:
    n = check_gaussians(g, n_lambda)
    s = _Gaussians()
    s.n = n
    for k in PARAMS:
        t = g[k]
        if n > 0 and not (t.dtype == _torch().float32 and t.is_contiguous()):
            raise ValueError("%s must be a contiguous float32 tensor" % k)
        setattr(s, k, _dptr(t) if n > 0 else None)
    return s


def _tilted_struct(g: Dict[str, "object"], n_lambda: int) -> _TiltedGaussians:
    n = check_gaussians(g, n_lambda, TILTED_PARAMS)
    s = _TiltedGaussians()
    s.n = n
    for k in TILTED_PARAMS:
        t = g[k]
        if n > 0 and not (t.dtype == _torch().float32 and t.is_contiguous()):
            raise ValueError("%s must be a contiguous float32 tensor" % k)
        setattr(s, k, _dptr(t) if n > 0 else None)
    return s


def _grads_struct(grads: Dict[str, "object"], g: Dict[str, "object"], n: int) -> _Grads:
    """Gradient outputs: each the shape of its parameter, float32 CUDA, contiguous; depth may be None."""
    keys = [k for k in PARAMS if not (k == "depth" and grads.get(k) is None)]
    if n > 0:
        for k in keys:
            check_tensor(grads.get(k), "grad " + k, tuple(g[k].shape), "float32")
    gr = _Grads()
    for k in PARAMS:
        setattr(gr, k, _dptr(grads[k]) if (n > 0 and k in keys) else None)
    return gr


class Context:
    """A libgws context on one device, with a cached workspace."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.lib = load_library()
        self.device = device
        h = ctypes.c_void_p()
        _check(self.lib.gws_create(ctypes.byref(h), device))
        self.handle = h
        self._ws = None
        self.torch_device = torch.device("cuda", device)

    def close(self):
        if self.handle:
            self.lib.gws_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(_torch().cuda.current_stream(self.device).cuda_stream)

    def workspace(self, nbytes: int):
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.torch_device)
        return self._ws

    def workspace_size(self, prob: Problem, n: int) -> int:
        sz = ctypes.c_size_t()
        _check(self.lib.gws_workspace_size(self.handle, ctypes.byref(prob._c()), n, ctypes.byref(sz)), self.handle)
        return sz.value

    def forward(self, prob: Problem, g: Dict[str, "object"], want_spectrum: bool = False, out=None):
        """Field (n_lambda, ny, nx) complex64 (and the DFT-ready spectrum if asked)."""
        torch = _torch()
        n = check_gaussians(g, prob.n_lambda)
        shape = (prob.n_lambda, prob.ny, prob.nx)
        field = out if out is not None else torch.empty(shape, dtype=torch.complex64, device=self.torch_device)
        check_tensor(field, "out", shape, "complex64")
        gs = _gaussians_struct(g, prob.n_lambda)
        spec = torch.empty_like(field) if want_spectrum else None
        o = _Output()
        o.field = _dptr(field)
        o.spectrum = _dptr(spec) if spec is not None else None
        ws = self.workspace(self.workspace_size(prob, n))
        _check(self.lib.gws_forward(self.handle, ctypes.byref(prob._c()), ctypes.byref(gs), ctypes.byref(o),
                                    ctypes.c_void_p(_dptr(ws)), ws.numel(), self._stream()), self.handle)
        return (field, spec) if want_spectrum else field

    def forward_noalloc(self, prob: Problem, g: Dict[str, "object"], out):
        """forward() for callers that cannot allocate device memory: the library works in its own
        per-device scratch array, the caller passes the output field (n_lambda, ny, nx) complex64.
        The plan for this grid must exist (an earlier forward() with the same shape and tiling)."""
        n = check_gaussians(g, prob.n_lambda)
        check_tensor(out, "out", (prob.n_lambda, prob.ny, prob.nx), "complex64")
        gs = _gaussians_struct(g, prob.n_lambda)
        o = _Output()
        o.field = _dptr(out)
        o.spectrum = None
        _check(self.lib.gws_forward_noalloc(self.handle, ctypes.byref(prob._c()), ctypes.byref(gs), ctypes.byref(o),
                                            self._stream()), self.handle)
        return out

    def workspace_size_tilted(self, prob: Problem, n: int) -> int:
        sz = ctypes.c_size_t()
        _check(self.lib.gws_workspace_size_tilted(self.handle, ctypes.byref(prob._c()), n, ctypes.byref(sz)),
               self.handle)
        return sz.value

    def forward_tilted(self, prob: Problem, g: Dict[str, "object"], want_spectrum: bool = False, out=None):
        """Field (n_lambda, ny, nx) complex64 of tilted Gaussians (fields TILTED_PARAMS), and the
        DFT-ready spectrum if asked."""
        torch = _torch()
        n = check_gaussians(g, prob.n_lambda, TILTED_PARAMS)
        shape = (prob.n_lambda, prob.ny, prob.nx)
        field = out if out is not None else torch.empty(shape, dtype=torch.complex64, device=self.torch_device)
        check_tensor(field, "out", shape, "complex64")
        gs = _tilted_struct(g, prob.n_lambda)
        spec = torch.empty_like(field) if want_spectrum else None
        o = _Output()
        o.field = _dptr(field)
        o.spectrum = _dptr(spec) if spec is not None else None
        ws = self.workspace(self.workspace_size_tilted(prob, n))
        _check(self.lib.gws_forward_tilted(self.handle, ctypes.byref(prob._c()), ctypes.byref(gs), ctypes.byref(o),
                                           ctypes.c_void_p(_dptr(ws)), ws.numel(), self._stream()), self.handle)
        return (field, spec) if want_spectrum else field

    def backward_tilted(self, prob: Problem, g: Dict[str, "object"], grad_field, out=None) -> dict:
        """Gradients of every tilted-Gaussian parameter (TILTED_PARAMS) given grad_field =
        dL/dRe u + j dL/dIm u, complex64 (n_lambda, ny, nx)."""
        torch = _torch()
        n = check_gaussians(g, prob.n_lambda, TILTED_PARAMS)
        check_tensor(grad_field, "grad_field", (prob.n_lambda, prob.ny, prob.nx), "complex64")
        grads = dict(out) if out is not None else {}
        for k in TILTED_PARAMS:   # every size checked before any address is taken
            if grads.get(k) is None:
                grads[k] = torch.empty_like(g[k])
            elif n > 0:
                check_tensor(grads[k], "grad " + k, tuple(g[k].shape), "float32")
        gs = _tilted_struct(g, prob.n_lambda)
        gr = _TiltedGrads()
        for k in TILTED_PARAMS:
            setattr(gr, k, _dptr(grads[k]) if n > 0 else None)
        ws = self.workspace(self.workspace_size_tilted(prob, n))
        _check(self.lib.gws_backward_tilted(self.handle, ctypes.byref(prob._c()), ctypes.byref(gs),
                                            ctypes.c_void_p(_dptr(grad_field)), ctypes.byref(gr),
                                            ctypes.c_void_p(_dptr(ws)), ws.numel(), self._stream()), self.handle)
        return grads

    def backward(self, prob: Problem, g: Dict[str, "object"], grad_field, want_depth: bool = True, out=None):
        """dL/d(parameter) for every Gaussian, given dL/dRe u + j dL/dIm u."""
        torch = _torch()
        n = check_gaussians(g, prob.n_lambda)
        grad_field = grad_field.to(torch.complex64).contiguous()
        check_tensor(grad_field, "grad_field", (prob.n_lambda, prob.ny, prob.nx), "complex64")
        grads = dict(out) if out is not None else {k: torch.empty_like(g[k]) for k in PARAMS}
        if not want_depth:
            grads["depth"] = None
        elif grads.get("depth") is None:
            grads["depth"] = torch.empty_like(g["depth"])
        gr = _grads_struct(grads, g, n)
        gs = _gaussians_struct(g, prob.n_lambda)
        if n == 0:
            return grads
        ws = self.workspace(self.workspace_size(prob, n))
        _check(self.lib.gws_backward(self.handle, ctypes.byref(prob._c()), ctypes.byref(gs),
                                     ctypes.c_void_p(_dptr(grad_field)), ctypes.byref(gr),
                                     ctypes.c_void_p(_dptr(ws)), ws.numel(), self._stream()), self.handle)
        return grads

    def workspace_size_batched(self, prob: Problem, offsets) -> int:
        offs = (ctypes.c_int64 * len(offsets))(*[int(v) for v in offsets])
        sz = ctypes.c_size_t()
        _check(self.lib.gws_workspace_size_batched(self.handle, ctypes.byref(prob._c()), len(offsets) - 1, offs,
                                                   ctypes.byref(sz)), self.handle)
        return sz.value

    def forward_batched(self, prob: Problem, g: Dict[str, "object"], offsets, out=None, want_spectrum: bool = False,
                        spectrum=None):
        """Fields of several scenes (Gaussians [offsets[s], offsets[s+1]) each), shape (S, C, ny, nx)
        (and their DFT-ready spectra, same shape, if asked).

        The first call for a given set of pointers and offsets captures the launch sequence
        into a hipGraph (on a non-default stream); later calls replay it."""
        torch = _torch()
        offsets = check_offsets(offsets, check_gaussians(g, prob.n_lambda))
        S = len(offsets) - 1
        shape = (S, prob.n_lambda, prob.ny, prob.nx)
        field = out if out is not None else torch.empty(shape, dtype=torch.complex64, device=self.torch_device)
        check_tensor(field, "out", shape, "complex64")
        if want_spectrum and spectrum is None:
            spectrum = torch.empty_like(field)
        if spectrum is not None:
            check_tensor(spectrum, "spectrum", shape, "complex64")
        gs = _gaussians_struct(g, prob.n_lambda)
        o = _Output()
        o.field = _dptr(field)
        o.spectrum = _dptr(spectrum) if spectrum is not None else None
        offs = (ctypes.c_int64 * (S + 1))(*offsets)
        need = self.workspace_size_batched(prob, offsets)
        ws = self._batch_ws(need)
        _check(self.lib.gws_forward_batched(self.handle, ctypes.byref(prob._c()), S, offs, ctypes.byref(gs),
                                            ctypes.byref(o), ctypes.c_void_p(_dptr(ws)), ws.numel(),
                                            self._stream()), self.handle)
        return (field, spectrum) if spectrum is not None else field

    def backward_batched(self, prob: Problem, g: Dict[str, "object"], offsets, grad_fields, want_depth: bool = True,
                         out=None):
        """Gradients of every Gaussian of the batch, given (S, C, ny, nx) field gradients."""
        torch = _torch()
        n = check_gaussians(g, prob.n_lambda)
        offsets = check_offsets(offsets, n)
        S = len(offsets) - 1
        check_tensor(grad_fields, "grad_fields", (S, prob.n_lambda, prob.ny, prob.nx), "complex64")
        grads = dict(out) if out is not None else {k: torch.empty_like(g[k]) for k in PARAMS}
        if not want_depth:
            grads["depth"] = None
        elif grads.get("depth") is None:
            grads["depth"] = torch.empty_like(g["depth"])
        gr = _grads_struct(grads, g, n)
        gs = _gaussians_struct(g, prob.n_lambda)
        offs = (ctypes.c_int64 * (S + 1))(*offsets)
        ws = self._batch_ws(self.workspace_size_batched(prob, offsets))
        _check(self.lib.gws_backward_batched(self.handle, ctypes.byref(prob._c()), S, offs, ctypes.byref(gs),
                                             ctypes.c_void_p(_dptr(grad_fields)), ctypes.byref(gr),
                                             ctypes.c_void_p(_dptr(ws)), ws.numel(), self._stream()), self.handle)
        return grads

    def _batch_ws(self, nbytes: int):
        # the batched workspace is part of the captured graph's key: keep it stable
        torch = _torch()
        if getattr(self, "_bws", None) is None or self._bws.numel() < nbytes:
            self._bws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.torch_device)
        return self._bws

    def autotune(self, prob: Problem, n_hint: int, cache_path: Optional[str] = None):
        """Time every tiling on n_hint synthetic Gaussians; later calls of this shape use the fastest."""
        _check(self.lib.gws_autotune(self.handle, ctypes.byref(prob._c()), int(n_hint),
                                     cache_path.encode() if cache_path else None, self._stream()), self.handle)

    def dft2d(self, x, direction: int, xform: int = XFORM_FFT_FP32, out=None):
        """Unnormalised 2D DFT of (batch, ny, nx) complex64: exp(+j..) for direction +1."""
        torch = _torch()
        x = x.to(torch.complex64).contiguous()
        if x.dim() != 3:
            raise ValueError("x must have shape (batch, ny, nx), got %s" % (tuple(x.shape),))
        b, ny, nx = x.shape
        out = out if out is not None else torch.empty_like(x)
        check_tensor(x, "x", (b, ny, nx), "complex64")
        check_tensor(out, "out", (b, ny, nx), "complex64")
        sz = ctypes.c_size_t()
        _check(self.lib.gws_dft_workspace_size(self.handle, nx, ny, b, xform, ctypes.byref(sz)), self.handle)
        ws = self.workspace(sz.value) if sz.value else None
        _check(self.lib.gws_dft2d(self.handle, nx, ny, b, direction, xform, ctypes.c_void_p(_dptr(x)),
                                  ctypes.c_void_p(_dptr(out)), ctypes.c_void_p(_dptr(ws) if ws is not None else 0),
                                  ws.numel() if ws is not None else 0, self._stream()), self.handle)
        return out

    def l2_loss_grad(self, field, target, grad=None, loss=None):
        """loss = sum |u - t|^2 (float64 device scalar) and grad = 2 (u - t), in the library."""
        torch = _torch()
        n = field.numel()
        shape = tuple(field.shape)
        check_tensor(field, "field", shape, "complex64")
        check_tensor(target, "target", shape, "complex64")
        if grad is None:
            grad = torch.empty_like(field)
        check_tensor(grad, "grad", shape, "complex64")
        if loss is None:
            loss = torch.empty((), dtype=torch.float64, device=self.torch_device)
        check_tensor(loss, "loss", (), "float64")
        if getattr(self, "_l2ws", None) is None:
            self._l2ws = torch.empty(int(self.lib.gws_l2_workspace_size()), dtype=torch.uint8, device=self.torch_device)
        _check(self.lib.gws_l2_loss_grad(self.handle, n, ctypes.c_void_p(_dptr(field)),
                                         ctypes.c_void_p(_dptr(target)), ctypes.c_void_p(_dptr(grad)),
                                         ctypes.c_void_p(_dptr(loss)), ctypes.c_void_p(_dptr(self._l2ws)),
                                         self._l2ws.numel(), self._stream()), self.handle)
        return loss, grad

    def holographics(self, view: dict, world: Dict[str, "object"], out=None) -> dict:
        """World-space Gaussians (mean [n, 3], quat [n, 4], scale [n, 3], opacity_sh [n, K]
        float32 device tensors) to hologram-space in-plane Gaussians (dict of [n] tensors)."""
        torch = _torch()
        n = int(world["mean"].shape[0])
        deg = int(view["sh_degree"])
        # a degree outside 0..3 is left to the library, which rejects it before reading anything
        sh_cols = (deg + 1) ** 2 if 0 <= deg <= 3 else int(world["opacity_sh"].shape[-1])
        for k, cols in (("mean", 3), ("quat", 4), ("scale", 3), ("opacity_sh", sh_cols)):
            check_tensor(world.get(k), k, (n, cols), "float32")
        v = _View()
        for i, x in enumerate(view["world_to_view"]):
            v.world_to_view[i] = float(x)
        for i, x in enumerate(view["ray_to_holo"]):
            v.ray_to_holo[i] = float(x)
        for k in ("fx", "fy", "cx", "cy", "near", "depth_scale", "depth_offset"):
            setattr(v, k, float(view[k]))
        v.sh_degree = int(view["sh_degree"])
        w = _WorldGaussians(n, *[ctypes.c_void_p(_dptr(world[k])) for k in ("mean", "quat", "scale", "opacity_sh")])
        if out is None:
            out = {k: torch.empty(n, dtype=torch.float32, device=world["mean"].device) for k in PLANE_FIELDS}
        for k in PLANE_FIELDS:
            check_tensor(out.get(k), "out " + k, (n,), "float32")
        pg = _PlaneGaussians(*[ctypes.c_void_p(_dptr(out[k])) for k in PLANE_FIELDS])
        _check(self.lib.gws_holographics(self.handle, ctypes.byref(v), ctypes.byref(w), ctypes.byref(pg),
                                         self._stream()), self.handle)
        return out

    def dpac_encode(self, field, a_max: Optional[float] = None, out=None):
        """Double-phase coding of a (C, ny, nx) complex64 field into a float32 phase-only
        pattern of the same shape; a_max None takes each channel's largest |u|."""
        torch = _torch()
        if field.dim() != 3:
            raise ValueError("field must have shape (C, ny, nx), got %s" % (tuple(field.shape),))
        C, ny, nx = field.shape
        check_tensor(field, "field", (C, ny, nx), "complex64")
        out = out if out is not None else torch.empty((C, ny, nx), dtype=torch.float32, device=field.device)
        check_tensor(out, "out", (C, ny, nx), "float32")
        am = 0.0 if a_max is None else float(a_max)
        if getattr(self, "_dpacws", None) is None:
            self._dpacws = torch.empty(int(self.lib.gws_dpac_workspace_size(4)), dtype=torch.uint8,
                                       device=self.torch_device)
        _check(self.lib.gws_dpac_encode(self.handle, nx, ny, C, ctypes.c_void_p(_dptr(field)), am,
                                        ctypes.c_void_p(_dptr(out)), ctypes.c_void_p(_dptr(self._dpacws)),
                                        self._dpacws.numel(), self._stream()), self.handle)
        return out

    def focal_stack(self, prob: Problem, inp, depths, phase_input: bool = False, half_band: bool = False,
                    complex_output: bool = False, out=None):
        """(K, C, ny, nx) intensities |P(u; d_k)|^2 (float32) or fields (complex64) of a
        (C, ny, nx) field, or of the phase-only pattern e^{jP} with phase_input."""
        torch = _torch()
        flags = (FS_PHASE_INPUT if phase_input else 0) | (FS_HALF_BAND if half_band else 0) | \
            (FS_COMPLEX_OUTPUT if complex_output else 0)
        K = len(depths)
        shape = (K, prob.n_lambda, prob.ny, prob.nx)
        check_tensor(inp, "inp", (prob.n_lambda, prob.ny, prob.nx), "float32" if phase_input else "complex64")
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64 if complex_output else torch.float32,
                              device=inp.device)
        check_tensor(out, "out", shape, "complex64" if complex_output else "float32")
        dep = (ctypes.c_double * max(K, 1))(*[float(d) for d in depths])
        pc = prob._c()
        sz = ctypes.c_size_t()
        _check(self.lib.gws_focal_stack_workspace_size(self.handle, ctypes.byref(pc), K, flags, ctypes.byref(sz)),
               self.handle)
        ws = self.workspace(sz.value)
        _check(self.lib.gws_focal_stack(self.handle, ctypes.byref(pc), ctypes.c_void_p(_dptr(inp)), K, dep,
                                        flags, ctypes.c_void_p(_dptr(out)), ctypes.c_void_p(_dptr(ws)),
                                        ws.numel(), self._stream()), self.handle)
        return out

    def set_profiling(self, on: bool):
        _check(self.lib.gws_set_profiling(self.handle, 1 if on else 0), self.handle)

    def read_profile(self) -> dict:
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        _check(self.lib.gws_read_profile(self.handle, ms, cnt), self.handle)
        return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}

    def stats(self) -> dict:
        s = _Stats()
        _check(self.lib.gws_get_stats(self.handle, ctypes.byref(s)), self.handle)
        return {f: getattr(s, f) for f, _ in _Stats._fields_}

    def measure_peaks(self) -> dict:
        """Measured roofline denominators of this device (gws_measure_peaks)."""
        p = _Peaks()
        _check(self.lib.gws_measure_peaks(self.handle, ctypes.byref(p), self._stream()), self.handle)
        return {f: getattr(p, f) for f, _ in _Peaks._fields_}


_ctx_cache: Dict[int, Context] = {}


def context(device: int = 0) -> Context:
    if device not in _ctx_cache:
        _ctx_cache[device] = Context(device)
    return _ctx_cache[device]


class GaussianWaveSplat:
    """torch.autograd.Function wrapper: field = GWS(params); backward through gws_backward."""

    _fn = None

    @classmethod
    def function(cls):
        if cls._fn is None:
            torch = _torch()

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(fctx, prob, mean_x, mean_y, depth, cov_xx, cov_xy, cov_yy, opacity, amplitude, phase):
                    g = dict(mean_x=mean_x, mean_y=mean_y, depth=depth, cov_xx=cov_xx, cov_xy=cov_xy, cov_yy=cov_yy,
                             opacity=opacity, amplitude=amplitude, phase=phase)
                    g = {k: v.detach().contiguous() for k, v in g.items()}
                    if prob.n_lambda > 3 and prob.blend == BLEND_OIT and fctx.needs_input_grad[3]:
                        # refused by the library's backward: say so now, not at loss.backward()
                        raise ValueError("the order-invariant adjoint takes the depth gradient for at most 3 "
                                         "wavelengths; detach depth or use fewer wavelengths")
                    fctx.prob = prob
                    fctx.save_for_backward(*[g[k] for k in PARAMS])
                    return context(mean_x.device.index or 0).forward(prob, g)

                @staticmethod
                def backward(fctx, grad_field):
                    saved = dict(zip(PARAMS, fctx.saved_tensors))
                    dev = saved["mean_x"].device.index or 0
                    grads = context(dev).backward(fctx.prob, saved, grad_field,
                                                  want_depth=fctx.needs_input_grad[3])
                    return (None,) + tuple(grads[k] if fctx.needs_input_grad[i + 1] else None
                                           for i, k in enumerate(PARAMS))

            cls._fn = _F
        return cls._fn


def render(prob: Problem, mean_x, mean_y, depth, cov_xx, cov_xy, cov_yy, opacity, amplitude, phase):
    """Differentiable field of the Gaussians at the SLM plane, (n_lambda, ny, nx) complex64."""
    return GaussianWaveSplat.function().apply(prob, mean_x, mean_y, depth, cov_xx, cov_xy, cov_yy, opacity,
                                              amplitude, phase)


class TiltedGaussianWaveSplat:
    """torch.autograd.Function wrapper for tilted Gaussians: field = gws_forward_tilted(params);
    backward through gws_backward_tilted (every parameter's gradient is computed in one call)."""

    _fn = None

    @classmethod
    def function(cls):
        if cls._fn is None:
            torch = _torch()

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(fctx, prob, *params):
                    g = {k: v.detach().contiguous() for k, v in zip(TILTED_PARAMS, params)}
                    fctx.prob = prob
                    fctx.save_for_backward(*[g[k] for k in TILTED_PARAMS])
                    return context(params[0].device.index or 0).forward_tilted(prob, g)

                @staticmethod
                def backward(fctx, grad_field):
                    saved = dict(zip(TILTED_PARAMS, fctx.saved_tensors))
                    dev = saved["mean_x"].device.index or 0
                    grads = context(dev).backward_tilted(fctx.prob, saved, grad_field.contiguous())
                    return (None,) + tuple(grads[k] if fctx.needs_input_grad[i + 1] else None
                                           for i, k in enumerate(TILTED_PARAMS))

            cls._fn = _F
        return cls._fn


def render_tilted(prob: Problem, mean_x, mean_y, depth, quat_w, quat_x, quat_y, quat_z, scale_u, scale_v, opacity,
                  amplitude, phase):
    """Differentiable field of tilted Gaussians (fields TILTED_PARAMS) at the SLM plane,
    (n_lambda, ny, nx) complex64."""
    return TiltedGaussianWaveSplat.function().apply(prob, mean_x, mean_y, depth, quat_w, quat_x, quat_y, quat_z,
                                                    scale_u, scale_v, opacity, amplitude, phase)
