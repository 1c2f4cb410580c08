"""Helpers shared by the GPU tests: move seeded scenes to the device, map oracle spectra to
the library's DFT-ready layout, and compare."""
import numpy as np

import paper_2505_06582_amd as gws


def scene_to_torch(scene, device="cuda"):
    import torch
    out = {}
    for k, v in scene.fields().items():
        out[k] = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(device)
    return out


def dft_ready(U_phys, grid):
    """Oracle spectrum U(nu_m) -> U (-1)^(m_x'+m_y') / (nx ny px py), the library's spectrum layout."""
    import oracle
    sx = oracle.signed_freq_index(grid.nx)
    sy = oracle.signed_freq_index(grid.ny)
    sign = np.where(((sy[:, None] + sx[None, :]) % 2) == 0, 1.0, -1.0)
    return U_phys * sign / (grid.nx * grid.ny * grid.px * grid.py)


def to_numpy(t):
    return t.detach().cpu().numpy()


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.complex128 if np.iscomplexobj(x) or np.iscomplexobj(ref) else np.float64)
    ref = np.asarray(ref, dtype=x.dtype)
    d = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((x - ref).ravel()) / (d if d > 0 else 1.0))


def problem(grid, **kw):
    return gws.Problem.from_grid(grid, **kw)
