"""FP64 CPU oracle for the Gaussian Wave Splatting hot path (order-invariant variant).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by
the CPU-baseline leg of ``bench.py``.  The product library never imports, links or calls
anything here, and nothing here touches the GPU library: the two share no code.

The oracle evaluates, in float64 and with no culling, blocking or reordering beyond the
definitions:

* O1  the closed-form angular spectrum of each in-plane 2D Gaussian (Sec. 4.1, Eq. 10;
      Fourier pair of Eq. 7 in ordinary frequency; det J = 1, det S = sqrt(det Sigma)),
      shifted by the transverse frequency nu_r of the reference plane wave that
      illuminates every Gaussian (Sec. 4.1): g_i(nu - nu_r),
* O2  the angular-spectrum transfer function H(nu, d) = exp(j 2 pi d sqrt(1/l^2 - |nu|^2))
      inside the propagating band, 0 outside (Eq. 3-4), applied at d = -z_i (Eq. 5, 12),
* O3  the order-invariant sum of Eq. 12 over Gaussians taken front to back (descending
      depth, ties by input index), as Alg. 1 accumulates them,
* O4  one centred inverse DFT to the SLM plane (Alg. 1, last step):
      u_c[n] = 1/(Nx Ny px py) sum_m U_c(nu_m) exp(+j 2 pi nu_m . x_n),  x_n = (n - N//2) p,
      written as two dense DFT matrices whose phases are reduced exactly in integers,
* O5  the adjoint: the spectrum-domain gradient (the conjugate transpose of O4 applied to
      the field gradient) contracted with the analytic derivative of every term of Eq. 12.

The sums O1-O3 and O5 run in ``gws_oracle.c`` (plain C, OpenMP over frequencies or over
Gaussians); the transforms O4 are numpy matrix products.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gws_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# Mutation testing of the pins compiles a deliberately broken copy of the C source.
if os.environ.get("GWS_ORACLE_SRC"):
    _SRC = os.environ["GWS_ORACLE_SRC"]
    _LIB_PATH = _SRC + ".so"
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (no fast-math, so libm stays exact)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            dp = ctypes.POINTER(ctypes.c_double)
            i32p = ctypes.POINTER(ctypes.c_int32)
            i64p = ctypes.POINTER(ctypes.c_int64)
            lib.oracle_spectrum.argtypes = [ctypes.c_int64] + [dp] * 9 + [
                ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp,
                ctypes.c_double, ctypes.c_double, ctypes.c_int64, i32p, i32p, dp]
            lib.oracle_spectrum.restype = None
            lib.oracle_param_grads.argtypes = [ctypes.c_int64] + [dp] * 9 + [
                ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp,
                ctypes.c_double, ctypes.c_double, dp, ctypes.c_int64, i64p, dp]
            lib.oracle_param_grads.restype = None
            _lib = lib
    return _lib


def _ptr(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _scene_f64(scene):
    """Promote the float32 scene exactly to float64, in the argument order of the C code."""
    return [_f64(scene.mean_x), _f64(scene.mean_y), _f64(scene.depth), _f64(scene.cov_xx),
            _f64(scene.cov_xy), _f64(scene.cov_yy), _f64(scene.opacity),
            _f64(np.reshape(scene.amplitude, (-1, scene.n))), _f64(scene.phase)]


def _ref_nu(grid):
    """Transverse frequency (cycles/m) of the reference plane wave, (0, 0) when the grid has none."""
    r = getattr(grid, "ref_nu", (0.0, 0.0))
    return float(r[0]), float(r[1])


def depth_order(scene) -> np.ndarray:
    """Front-to-back order: descending depth (the viewer sits at +z), ties by input index."""
    return np.argsort(-np.asarray(scene.depth, dtype=np.float64), kind="stable")


def signed_freq_index(n: int) -> np.ndarray:
    """m' for FFT-order index m: m if 2m < n else m - n (numpy ``fftfreq`` order)."""
    m = np.arange(n)
    return np.where(2 * m < n, m, m - n)


def spectrum(scene, grid, freq_mx=None, freq_my=None, ordered: bool = True) -> np.ndarray:
    """Eq. 12 angular spectrum U_c(nu_m) (physical units, no DFT scaling).

    With no frequency list, returns the full grid, shape (n_lambda, ny, nx) indexed by
    FFT-order (m_y, m_x).  With lists of FFT-order indices, returns (n_lambda, len).
    """
    lib = _load()
    s = scene.subset(depth_order(scene)) if ordered else scene
    full = freq_mx is None
    if full:
        my, mx = np.meshgrid(np.arange(grid.ny, dtype=np.int32), np.arange(grid.nx, dtype=np.int32),
                             indexing="ij")
        freq_mx, freq_my = mx.ravel(), my.ravel()
    freq_mx = np.ascontiguousarray(freq_mx, dtype=np.int32)
    freq_my = np.ascontiguousarray(freq_my, dtype=np.int32)
    lam = _f64(grid.lambdas)
    out = np.zeros((grid.n_lambda, freq_mx.size, 2), dtype=np.float64)
    args = _scene_f64(s)
    lib.oracle_spectrum(s.n, *[_ptr(a) for a in args], grid.nx, grid.ny, grid.px, grid.py,
                        grid.n_lambda, _ptr(lam), *_ref_nu(grid), freq_mx.size, _ptr(freq_mx, ctypes.c_int32),
                        _ptr(freq_my, ctypes.c_int32), _ptr(out))
    u = out[..., 0] + 1j * out[..., 1]
    if full:
        u = u.reshape(grid.n_lambda, grid.ny, grid.nx)
    return u


def dft_matrix(n: int) -> np.ndarray:
    """E[n_idx, m] = exp(+j 2 pi nu_m x_n) with nu_m x_n = m' (n - N//2) / N, reduced exactly."""
    k = np.outer(np.arange(n) - n // 2, signed_freq_index(n))  # integer phase numerators
    return np.exp(2j * math.pi * (np.mod(k, n) / n))


def field_from_spectrum(U: np.ndarray, grid) -> np.ndarray:
    """O4: centred inverse DFT of a full spectrum (n_lambda, ny, nx) to the SLM field."""
    Ey, Ex = dft_matrix(grid.ny), dft_matrix(grid.nx)
    scale = 1.0 / (grid.nx * grid.ny * grid.px * grid.py)
    return np.stack([scale * (Ey @ U[c] @ Ex.T) for c in range(U.shape[0])])


def spectrum_grad_from_field_grad(G: np.ndarray, grid) -> np.ndarray:
    """Adjoint of O4: dL/dU (torch's complex convention) from dL/du, same scale."""
    Ey, Ex = dft_matrix(grid.ny), dft_matrix(grid.nx)
    scale = 1.0 / (grid.nx * grid.ny * grid.px * grid.py)
    G = np.asarray(G, dtype=np.complex128)
    return np.stack([scale * (Ey.conj().T @ G[c] @ Ex.conj()) for c in range(G.shape[0])])


def forward(scene, grid) -> np.ndarray:
    """The hot path: complex field at the SLM, shape (n_lambda, ny, nx), row-major, x fastest."""
    return field_from_spectrum(spectrum(scene, grid), grid)


def loss_and_field_grad(u: np.ndarray, target: np.ndarray):
    """L = sum |u - t|^2 and its gradient dL/dRe u + j dL/dIm u = 2 (u - t)."""
    d = np.asarray(u, dtype=np.complex128) - np.asarray(target, dtype=np.complex128)
    return float(np.sum(np.abs(d) ** 2)), 2.0 * d


PARAM_NAMES = ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity", "phase")


def param_grads_from_spectrum_grad(scene, grid, gs: np.ndarray, sel=None) -> dict:
    """O5: dL/d(parameter) for the Gaussians in ``sel`` (all if None), given dL/dU."""
    lib = _load()
    sel = np.arange(scene.n, dtype=np.int64) if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    gs = np.ascontiguousarray(gs, dtype=np.complex128)
    assert gs.shape == (grid.n_lambda, grid.ny, grid.nx)
    gsv = gs.view(np.float64)
    lam = _f64(grid.lambdas)
    stride = 9 + grid.n_lambda
    out = np.zeros((sel.size, stride), dtype=np.float64)
    args = _scene_f64(scene)
    lib.oracle_param_grads(scene.n, *[_ptr(a) for a in args], grid.nx, grid.ny, grid.px, grid.py,
                           grid.n_lambda, _ptr(lam), *_ref_nu(grid), _ptr(gsv), sel.size,
                           _ptr(sel, ctypes.c_int64), _ptr(out))
    res = {name: out[:, k].copy() for k, name in enumerate(PARAM_NAMES)}
    res["amplitude"] = out[:, 9:].T.copy()
    return res


def backward(scene, grid, field_grad: np.ndarray, sel=None) -> dict:
    """Gradients of a loss with respect to every Gaussian parameter, given dL/du."""
    gs = spectrum_grad_from_field_grad(field_grad, grid)
    return param_grads_from_spectrum_grad(scene, grid, gs, sel)


def rel_l2(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2 (float64)."""
    x = np.asarray(x, dtype=np.complex128 if np.iscomplexobj(x) or np.iscomplexobj(ref) else np.float64)
    ref = np.asarray(ref, dtype=x.dtype)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((x - ref).ravel()) / (den if den > 0 else 1.0))
