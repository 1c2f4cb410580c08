"""FP64 CPU oracle for exact alpha wave blending (Sec. 4, Eq. 5-6; supplement Alg. 2).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/`` and never by
the product library, with which it shares no code.

Exact blending replaces the order-invariant sum of Eq. 12 by the global transmittance map of
alpha wave blending.  Following Alg. 2, the Gaussians are taken front to back (descending
depth, ties by input index, the same order as the order-invariant oracle) and for each
Gaussian k:

  1. u_k, the Gaussian's own wavefront on its plane: the centred inverse DFT of its angular
     spectrum (Eq. 10, unit colour and opacity, no propagation) times e^{j phi_k};
  2. the masked wavefront T u_k is taken back to the frequency domain (the exact inverse of
     the centred inverse DFT), propagated to the SLM by H(nu, -z_k) (Eq. 4, the same sign
     reading as Eq. 12) and added, times colour a_{k,c} and opacity o_k, to the spectrum;
  3. alpha_k = o_k |u_k|, set to zero where it does not exceed t_eps = 1/255;
  4. T <- T (1 - alpha_k).

One centred inverse DFT of the accumulated spectrum gives the SLM field.  With T = 1 every
step reduces to Eq. 12.  The disk-based variant (binarised alpha) is not part of this path.

The transforms are numpy's FP64 FFT with the centring x_n = (n - N//2) p applied as an
exactly reduced phase factor per frequency, so any grid size works.
"""
from __future__ import annotations

import math

import numpy as np

from . import depth_order, signed_freq_index, spectrum

T_EPS = 1.0 / 255.0


def _centre_factor(n: int) -> np.ndarray:
    """f_m = exp(+j 2 pi m' (N//2) / N), the phase that moves the DFT origin to pixel N//2."""
    k = np.mod(signed_freq_index(n) * (n // 2), n)
    return np.exp(2j * math.pi * k / n)


def field_from_spectrum_fft(U: np.ndarray, grid) -> np.ndarray:
    """u[n] = 1/(Nx Ny px py) sum_m U[m] exp(+j 2 pi nu_m . x_n), for (..., ny, nx) spectra."""
    fy, fx = _centre_factor(grid.ny), _centre_factor(grid.nx)
    V = U * np.conj(fy)[:, None] * np.conj(fx)[None, :]
    return np.fft.ifft2(V, axes=(-2, -1)) / (grid.px * grid.py)


def spectrum_from_field_fft(u: np.ndarray, grid) -> np.ndarray:
    """The exact inverse of field_from_spectrum_fft: px py sum_n u[n] exp(-j 2 pi nu_m . x_n)."""
    fy, fx = _centre_factor(grid.ny), _centre_factor(grid.nx)
    return grid.px * grid.py * np.fft.fft2(u, axes=(-2, -1)) * fy[:, None] * fx[None, :]


def transfer(grid, lam: float, d: float) -> np.ndarray:
    """H(nu, d) = exp(j 2 pi d sqrt(1/lam^2 - |nu|^2)) for |nu| < 1/lam, else 0 (Eq. 4)."""
    nux = signed_freq_index(grid.nx) / (grid.nx * grid.px)
    nuy = signed_freq_index(grid.ny) / (grid.ny * grid.py)
    nu2 = nuy[:, None] ** 2 + nux[None, :] ** 2
    w2 = 1.0 / lam ** 2 - nu2
    prop = w2 > 0.0
    ph = d * np.sqrt(np.where(prop, w2, 0.0))           # revolutions
    return np.where(prop, np.exp(2j * math.pi * np.mod(ph, 1.0)), 0.0)


def own_wavefront(scene, k: int, grid) -> np.ndarray:
    """u_k: the k-th Gaussian's wavefront on its own plane, e^{j phi_k} times its profile,
    from its closed-form angular spectrum with unit colour and opacity and z = 0."""
    one = scene.subset([k]).copy()
    one.depth[:] = 0.0
    one.opacity[:] = 1.0
    one.amplitude[:] = 1.0
    g1 = type(grid)(grid.nx, grid.ny, grid.px, grid.py, (grid.lambdas[0],))
    return field_from_spectrum_fft(spectrum(one, g1, ordered=False)[0], grid)


def exact_spectrum(scene, grid, t_eps: float = T_EPS, return_transmittance: bool = False):
    """Alg. 2 in the frequency domain: the accumulated SLM spectrum (n_lambda, ny, nx)."""
    order = depth_order(scene)
    U = np.zeros((grid.n_lambda, grid.ny, grid.nx), dtype=np.complex128)
    T = np.ones((grid.ny, grid.nx), dtype=np.float64)
    for k in order:
        u = own_wavefront(scene, int(k), grid)
        S = spectrum_from_field_fft(T * u, grid)
        o = float(scene.opacity[k])
        z = float(scene.depth[k])
        for c in range(grid.n_lambda):
            a = float(np.reshape(scene.amplitude, (-1, scene.n))[c, k])
            U[c] += a * o * transfer(grid, grid.lambdas[c], -z) * S
        alpha = o * np.abs(u)
        alpha = np.where(alpha > t_eps, alpha, 0.0)
        T = T * (1.0 - alpha)
    return (U, T) if return_transmittance else U


def exact_forward(scene, grid, t_eps: float = T_EPS) -> np.ndarray:
    """Exact alpha wave blending: the SLM field (n_lambda, ny, nx)."""
    return field_from_spectrum_fft(exact_spectrum(scene, grid, t_eps), grid)
