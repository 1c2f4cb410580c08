"""FP64 gradients of a field loss through exact alpha wave blending (Eq. 5-6, Alg. 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The forward steps of oracle/exact.py are written again with plain PyTorch CPU ops in
float64 / complex128 -- the closed-form angular spectrum of Eq. 10, the centred inverse and
forward DFTs (torch.fft with the exactly reduced centring phase), the mask by the
transmittance map, H(nu, -z) of Eq. 4, alpha = o |u| with the 1/255 threshold, and the
front-to-back update of the map -- and reverse-mode differentiation of that chain gives the
gradient with respect to every Gaussian parameter.  The threshold is a step function: its
derivative is taken as zero, i.e. the kept/dropped decision is held fixed.

Parameters follow the library's convention: mean_x, mean_y (m), depth (m), cov_xx, cov_xy,
cov_yy (m^2; cov_xy one parameter filling both off-diagonal entries), opacity, amplitude
(n_lambda, n), phase (rad).
"""
from __future__ import annotations

import math
import types

import numpy as np
import torch

from . import depth_order, signed_freq_index

T_EPS = 1.0 / 255.0
PARAMS = ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity", "amplitude", "phase")


def _centre(n: int) -> torch.Tensor:
    k = np.mod(signed_freq_index(n) * (n // 2), n)
    return torch.from_numpy(np.exp(2j * math.pi * k / n))


def _grid_freqs(grid):
    nux = torch.from_numpy(signed_freq_index(grid.nx) / (grid.nx * grid.px))
    nuy = torch.from_numpy(signed_freq_index(grid.ny) / (grid.ny * grid.py))
    return nux[None, :], nuy[:, None]


def exact_field_torch(p: dict, grid, t_eps: float = T_EPS) -> torch.Tensor:
    """The exact-blending SLM field (n_lambda, ny, nx) from float64 parameter tensors."""
    n = p["mean_x"].shape[0]
    order = depth_order(types.SimpleNamespace(depth=p["depth"].detach().numpy()))
    nux, nuy = _grid_freqs(grid)
    fy, fx = _centre(grid.ny), _centre(grid.nx)
    area = grid.px * grid.py
    C = grid.n_lambda
    nu2 = nux ** 2 + nuy ** 2
    U = [torch.zeros((grid.ny, grid.nx), dtype=torch.complex128) for _ in range(C)]
    T = torch.ones((grid.ny, grid.nx), dtype=torch.float64)
    for k in order:
        k = int(k)
        sxx, sxy, syy = p["cov_xx"][k], p["cov_xy"][k], p["cov_yy"][k]
        det = sxx * syy - sxy * sxy
        # Eq. 10 (in-plane, unit colour and opacity): 2 pi sqrt(det) exp(-2 pi^2 nu^T S nu) e^{-j 2 pi nu.mu}
        quad = sxx * nux ** 2 + 2.0 * sxy * nux * nuy + syy * nuy ** 2
        ramp = nux * p["mean_x"][k] + nuy * p["mean_y"][k]
        spec = 2.0 * math.pi * torch.sqrt(det) * torch.exp(-2.0 * math.pi ** 2 * quad) * \
            torch.exp(-2j * math.pi * ramp) * torch.exp(1j * p["phase"][k])
        # u_k = centred inverse DFT: 1/(Nx Ny px py) sum_m spec e^{+j 2 pi nu.x}
        u = torch.fft.ifft2(spec * torch.conj(fy)[:, None] * torch.conj(fx)[None, :]) / area
        S = area * torch.fft.fft2(T * u) * fy[:, None] * fx[None, :]
        for c in range(C):
            lam = grid.lambdas[c]
            w2 = 1.0 / lam ** 2 - nu2
            prop = w2 > 0.0
            W = torch.sqrt(torch.where(prop, w2, torch.zeros_like(w2)))
            H = torch.where(prop, torch.exp(-2j * math.pi * p["depth"][k] * W), torch.zeros((), dtype=torch.complex128))
            U[c] = U[c] + p["amplitude"][c, k] * p["opacity"][k] * H * S
        alpha = p["opacity"][k] * torch.abs(u)
        keep = (alpha > t_eps).detach()
        T = T * (1.0 - torch.where(keep, alpha, torch.zeros_like(alpha)))
    out = []
    for c in range(C):
        out.append(torch.fft.ifft2(U[c] * torch.conj(fy)[:, None] * torch.conj(fx)[None, :]) / area)
    return torch.stack(out)


def exact_loss_grads(scene, grid, target: np.ndarray, t_eps: float = T_EPS):
    """L = sum |u - t|^2 for the exact-blending field u, and dL/d(parameter) for every
    parameter; returns (L, field, grads as float64 numpy arrays)."""
    p = {}
    for k in PARAMS:
        v = np.asarray(getattr(scene, k), dtype=np.float64)
        if k == "amplitude":
            v = np.reshape(v, (-1, scene.n))
        p[k] = torch.tensor(v, dtype=torch.float64, requires_grad=True)
    u = exact_field_torch(p, grid, t_eps)
    t = torch.from_numpy(np.asarray(target, dtype=np.complex128))
    loss = torch.sum(torch.abs(u - t) ** 2)
    loss.backward()
    grads = {k: p[k].grad.numpy().copy() for k in PARAMS}
    return float(loss.detach()), u.detach().numpy(), grads
