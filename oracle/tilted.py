"""FP64 CPU oracle for tilted 2D Gaussians (Sec. 4.1, Eq. 8-10; supplement, the derivation of
the Gaussian's angular spectrum: translation, rotation and scaling steps).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/`` and never by
the product library, with which it shares no code.

A tilted Gaussian i is the canonical Gaussian exp(-|x_c|^2 / 2) of the plane z_c = 0 placed in
hologram space by x = R_i S_i x_c + mu_i, with S_i = diag(s_u, s_v, 0), R_i the rotation of the
unit quaternion (w, x, y, z) and mu_i = (mean_x, mean_y, depth).  Its angular spectrum on the
plane z = depth (parallel to the SLM, through the centre) follows the paper's three steps:

  * scaling (affine theorem): on its own plane the disk has the 2D spectrum
      G_o(k_ox, k_oy) = 2 pi s_u s_v exp(-2 pi^2 (s_u^2 k_ox^2 + s_v^2 k_oy^2));
  * rotation (the tilted-plane remap): the plane wave of wave vector k = (nu_x, nu_y, k_z),
    k_z = sqrt(1/lambda^2 - |nu|^2), is the plane wave k_o = R^{-1} k = R^T k of the disk's
    frame, and the change of integration variables from (k_ox, k_oy) to (nu_x, nu_y) on the
    sphere |k| = 1/lambda has the Jacobian det J = k_oz / k_z, so
      G_t(nu) = |det J| G_o(k_ox, k_oy);
  * translation: the transverse offset (mean_x, mean_y) multiplies by exp(-j 2 pi nu . mu_xy).

Readings (the paper is silent on them):
  T1  |det J|, not det J: R and R diag(1, -1, -1) (also R diag(-1, 1, -1)) describe the same
      disk, since the canonical profile is even in x_c and y_c; they differ only in the sign of
      k_oz.  A disk radiates to both sides of its plane, and the side facing the SLM is the one
      whose waves reach it, so the magnitude is taken.  At grazing waves (k_oz = 0) the term
      vanishes, continuously.
  T2  Evanescent frequencies (|nu| >= 1/lambda) carry nothing, as in the transfer function.
  T3  The exponent uses the same 2 pi^2 (ordinary frequency) convention as the in-plane
      spectrum, and the transform sign of the in-plane oracle (exp(-j 2 pi nu . mu)), so a
      rotation about z alone gives exactly the in-plane Gaussian with Sigma = R S^2 R^T.
  T4  No reference-wave shift: tilted Gaussians are defined for on-axis illumination only.

The wave is then carried to the SLM by H(nu, -depth) and weighted by a_c o e^{j phi}, and the
Gaussians are summed (order-invariant, Eq. 12); the field is the centred inverse DFT of the
in-plane oracle (O4).
"""
from __future__ import annotations

import math

import numpy as np

from . import field_from_spectrum, signed_freq_index
from .holographics import quat_to_matrix

TILTED_FIELDS = ("mean_x", "mean_y", "depth", "quat_w", "quat_x", "quat_y", "quat_z", "scale_u", "scale_v",
                 "opacity", "amplitude", "phase")


def rotation(scene, i: int) -> np.ndarray:
    """R_i from the (normalised) quaternion of Gaussian i."""
    q = [float(scene.quat_w[i]), float(scene.quat_x[i]), float(scene.quat_y[i]), float(scene.quat_z[i])]
    return quat_to_matrix(q)


def object_spectrum(su: float, sv: float, kox, koy):
    """G_o: the disk's spectrum on its own plane (scaling step, affine theorem)."""
    return 2.0 * math.pi * su * sv * np.exp(-2.0 * math.pi ** 2 * (su * su * kox * kox + sv * sv * koy * koy))


def gaussian_spectrum(R: np.ndarray, su: float, sv: float, nux, nuy, lam: float):
    """G_t(nu): one tilted Gaussian's spectrum on the plane through its centre parallel to the
    SLM (rotation step), before the transverse ramp.  0 where evanescent (T2)."""
    nux = np.asarray(nux, dtype=np.float64)
    nuy = np.asarray(nuy, dtype=np.float64)
    inv_l = 1.0 / lam
    w2 = inv_l * inv_l - (nux * nux + nuy * nuy)
    prop = w2 > 0.0
    kz = np.sqrt(np.where(prop, w2, 1.0))
    # k_o = R^T k, component by component (column j of R dotted with k)
    kox = R[0, 0] * nux + R[1, 0] * nuy + R[2, 0] * kz
    koy = R[0, 1] * nux + R[1, 1] * nuy + R[2, 1] * kz
    koz = R[0, 2] * nux + R[1, 2] * nuy + R[2, 2] * kz
    detj = np.abs(koz) / kz                                                   # T1
    return np.where(prop, detj * object_spectrum(su, sv, kox, koy), 0.0)


def spectrum(scene, grid, freq_mx=None, freq_my=None) -> np.ndarray:
    """Order-invariant angular spectrum U_c(nu_m) of tilted Gaussians at the SLM (physical
    units).  Full grid (n_lambda, ny, nx) in FFT-order indices, or (n_lambda, len) at the given
    FFT-order index lists."""
    if tuple(getattr(grid, "ref_nu", (0.0, 0.0))) != (0.0, 0.0):
        raise ValueError("tilted Gaussians are defined for on-axis illumination only")   # T4
    full = freq_mx is None
    if full:
        my, mx = np.meshgrid(np.arange(grid.ny), np.arange(grid.nx), indexing="ij")
        freq_mx, freq_my = mx.ravel(), my.ravel()
    nux = signed_freq_index(grid.nx)[np.asarray(freq_mx)] / (grid.nx * grid.px)
    nuy = signed_freq_index(grid.ny)[np.asarray(freq_my)] / (grid.ny * grid.py)
    nu2 = nux * nux + nuy * nuy
    out = np.zeros((grid.n_lambda, nux.size), dtype=np.complex128)
    for i in range(scene.n):
        R = rotation(scene, i)
        su, sv = float(scene.scale_u[i]), float(scene.scale_v[i])
        mx_, my_, z = float(scene.mean_x[i]), float(scene.mean_y[i]), float(scene.depth[i])
        ramp = np.exp(-2j * math.pi * (nux * mx_ + nuy * my_))
        for c, lam in enumerate(grid.lambdas):
            inv_l = 1.0 / lam
            w2 = inv_l * inv_l - nu2
            kz = np.sqrt(np.where(w2 > 0.0, w2, 0.0))
            H = np.where(w2 > 0.0, np.exp(2j * math.pi * (-z) * kz), 0.0)   # H(nu, -z), Eq. 3-4
            a = float(scene.amplitude[c, i]) * float(scene.opacity[i])
            out[c] += a * np.exp(1j * float(scene.phase[i])) * gaussian_spectrum(R, su, sv, nux, nuy, lam) * ramp * H
    if full:
        out = out.reshape(grid.n_lambda, grid.ny, grid.nx)
    return out


def forward(scene, grid) -> np.ndarray:
    """Field of tilted Gaussians at the SLM, (n_lambda, ny, nx)."""
    return field_from_spectrum(spectrum(scene, grid), grid)
