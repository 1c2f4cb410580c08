"""FP64 gradient oracle for tilted Gaussians: the field of oracle/tilted.py written again with
float64 PyTorch CPU ops and differentiated in reverse mode.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/`` and never by
the product library, with which it shares no code.

The forward follows the same steps as oracle/tilted.py (Sec. 4.1, Eq. 8-10; the supplement's
scaling, rotation and translation steps; readings T1-T4): R from the normalised quaternion,
k_o = R^T k, the spectrum |k_oz / k_z| 2 pi s_u s_v exp(-2 pi^2 (s_u^2 k_ox^2 + s_v^2 k_oy^2))
on the plane through the centre, the ramp exp(-j 2 pi nu . mu_xy), H(nu, -depth), the weight
a_c o e^{j phi}, the order-invariant sum (Eq. 12) and the centred inverse DFT (O4).  For a real
loss L of the field with G = dL/dRe u + j dL/dIm u, the gradient of every parameter is
d/dt Re <G, u(t)>, taken by autograd; at a grazing wave (k_oz = 0) the derivative of |k_oz| is
taken as 0 (a set of measure zero on the lattice).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import dft_matrix, signed_freq_index

PARAMS = ("mean_x", "mean_y", "depth", "quat_w", "quat_x", "quat_y", "quat_z", "scale_u", "scale_v", "opacity",
          "amplitude", "phase")


def _rotation(qw, qx, qy, qz):
    """[n][3][3] rotation matrices of the quaternions, normalised first."""
    nrm = torch.sqrt(qw * qw + qx * qx + qy * qy + qz * qz)
    w, x, y, z = qw / nrm, qx / nrm, qy / nrm, qz / nrm
    r0 = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1)
    r1 = torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1)
    r2 = torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)
    return torch.stack([r0, r1, r2], -2)


def field(params: dict, grid) -> torch.Tensor:
    """Complex128 field (n_lambda, ny, nx) of the tilted Gaussians in ``params`` (float64 tensors)."""
    sx = torch.from_numpy(signed_freq_index(grid.nx).astype(np.float64)) / (grid.nx * grid.px)
    sy = torch.from_numpy(signed_freq_index(grid.ny).astype(np.float64)) / (grid.ny * grid.py)
    nuy, nux = torch.meshgrid(sy, sx, indexing="ij")             # [ny][nx], FFT-order indices
    nu2 = nux * nux + nuy * nuy
    R = _rotation(params["quat_w"], params["quat_x"], params["quat_y"], params["quat_z"])   # [n][3][3]
    su, sv = params["scale_u"], params["scale_v"]
    mx, my, z = params["mean_x"], params["mean_y"], params["depth"]
    ph, o = params["phase"], params["opacity"]
    ramp = torch.exp(-2j * math.pi * (nux[None] * mx[:, None, None] + nuy[None] * my[:, None, None]))
    U = []
    for c, lam in enumerate(grid.lambdas):
        inv_l = 1.0 / lam
        w2 = inv_l * inv_l - nu2
        prop = w2 > 0
        kz = torch.sqrt(torch.where(prop, w2, torch.ones_like(w2)))
        # k_o = R^T k: column j of R dotted with k = (nu_x, nu_y, k_z)
        kox = R[:, 0, 0, None, None] * nux + R[:, 1, 0, None, None] * nuy + R[:, 2, 0, None, None] * kz
        koy = R[:, 0, 1, None, None] * nux + R[:, 1, 1, None, None] * nuy + R[:, 2, 1, None, None] * kz
        koz = R[:, 0, 2, None, None] * nux + R[:, 1, 2, None, None] * nuy + R[:, 2, 2, None, None] * kz
        g = (2 * math.pi * (su * sv)[:, None, None]
             * torch.exp(-2 * math.pi ** 2 * (su[:, None, None] ** 2 * kox ** 2 + sv[:, None, None] ** 2 * koy ** 2))
             * torch.abs(koz) / kz)
        H = torch.exp(2j * math.pi * (-z[:, None, None]) * kz)
        a = params["amplitude"][c] * o
        term = (a * torch.exp(1j * ph))[:, None, None] * g * ramp * H
        U.append(torch.where(prop[None], term, torch.zeros_like(term)).sum(0))
    Usum = torch.stack(U)                                           # [C][ny][nx]
    Ey = torch.from_numpy(dft_matrix(grid.ny))
    Ex = torch.from_numpy(dft_matrix(grid.nx))
    scale = 1.0 / (grid.nx * grid.ny * grid.px * grid.py)
    return scale * (Ey @ Usum @ Ex.T)


def backward(scene, grid, field_grad) -> dict:
    """dL/d(parameter) for every Gaussian (float64 numpy, amplitude [n_lambda][n]), given
    G = dL/dRe u + j dL/dIm u of shape (n_lambda, ny, nx)."""
    if tuple(getattr(grid, "ref_nu", (0.0, 0.0))) != (0.0, 0.0):
        raise ValueError("tilted Gaussians are defined for on-axis illumination only")
    params = {k: torch.tensor(np.asarray(getattr(scene, k), dtype=np.float64), requires_grad=True) for k in PARAMS}
    u = field(params, grid)
    G = torch.from_numpy(np.asarray(field_grad, dtype=np.complex128))
    # Re <G, u> = sum Re(G) Re(u) + Im(G) Im(u): its gradient is dL/dt by the chain rule
    lin = (G.real * u.real + G.imag * u.imag).sum()
    lin.backward()
    return {k: params[k].grad.numpy().copy() for k in PARAMS}
