"""FP64 CPU oracle for the holographics transform (supplement, Holographics pipeline; Sec. 4
view-dependent opacity): world-space Gaussians and a camera to the in-plane hologram-space
Gaussians that the order-invariant and exact splatting paths take.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/`` and never by
the product library, with which it shares no code.

Steps, in the supplement's order, per Gaussian:
  1. model transform: the canonical Gaussian mapped by x_w = R_w S_w x_c + mu_w, with R_w from
     the unit quaternion (w, x, y, z) and S_w = diag(scale), so Sigma_w = R_w S_w S_w^T R_w^T;
  2. view transform W = [R_v | t] to view space, where the camera looks along -z;
  3. projective mapping Pi to ray space (pinhole: Pi(p) = (f_x p_x / -p_z + c_x,
     f_y p_y / -p_z + c_y)) and its local affine approximation, the Jacobian J of Pi at
     W mu_w (EWA splatting): Sigma_r = J R_v Sigma_w R_v^T J^T, mu_r = Pi(W mu_w);
  4. lift to 3D: mu_r is augmented with the view-space depth (W mu_w)_z; Sigma_r is
     eigen-decomposed into R' S'^2 R'^T and re-embedded with zero rotation about x and y and
     zero z-scale;
  5. hologram transform T (3 x 3 plus translation) to hologram space.  Only transforms that
     keep the SLM plane and the depth axis apart are taken (an in-plane 2 x 2 part and an
     affine depth map), so every Gaussian stays an in-plane Gaussian at one depth;
  6. view-dependent opacity o = SH(o_coeffs, d): real spherical harmonics of degree <= 3 (the
     Condon-Shortley phase kept, coefficient k = l^2 + l + m), d the unit direction from the
     camera centre to mu_w, clamped to [0, 1].  Gaussians closer than `near` in front of the
     camera are culled: opacity 0 and a zero covariance.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import sph_harm_y


def quat_to_matrix(q) -> np.ndarray:
    """Rotation matrix of the quaternion (w, x, y, z), normalised first."""
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def real_sh(deg: int, d) -> np.ndarray:
    """Real spherical harmonics Y_k(d), k = l^2 + l + m, l <= deg, from scipy's complex ones
    (Condon-Shortley phase kept): m < 0: sqrt(2) Im Y_l^|m|; m = 0: Y_l^0; m > 0: sqrt(2) Re Y_l^m."""
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0])
    out = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            y = complex(sph_harm_y(l, abs(m), theta, phi))
            out.append(math.sqrt(2.0) * y.imag if m < 0 else (y.real if m == 0 else math.sqrt(2.0) * y.real))
    return np.array(out)


def project(p, cam) -> np.ndarray:
    """Pi: view space to ray space (pinhole, camera looking along -z)."""
    return np.array([cam["fx"] * p[0] / -p[2] + cam["cx"], cam["fy"] * p[1] / -p[2] + cam["cy"]])


def project_jacobian(p, cam) -> np.ndarray:
    """J = dPi/dp at p (2 x 3)."""
    iz = 1.0 / -p[2]
    return np.array([[cam["fx"] * iz, 0.0, cam["fx"] * p[0] * iz * iz],
                     [0.0, cam["fy"] * iz, cam["fy"] * p[1] * iz * iz]])


def camera_parts(cam):
    V = np.asarray(cam["world_to_view"], dtype=np.float64).reshape(3, 4)
    Rv, t = V[:, :3], V[:, 3]
    H = np.asarray(cam["ray_to_holo"], dtype=np.float64).reshape(2, 3)
    T = np.array([[H[0, 0], H[0, 1], 0.0], [H[1, 0], H[1, 1], 0.0], [0.0, 0.0, cam["depth_scale"]]])
    tt = np.array([H[0, 2], H[1, 2], cam["depth_offset"]])
    return Rv, t, T, tt


def transform_one(mean, quat, scale, sh, cam) -> dict:
    """Hologram-space in-plane Gaussian (metres) and its view-dependent opacity."""
    Rv, t, T, tt = camera_parts(cam)
    mu_w = np.asarray(mean, dtype=np.float64)
    # 1. model transform
    M = quat_to_matrix(quat) @ np.diag(np.asarray(scale, dtype=np.float64))
    Sigma_w = M @ M.T
    # 2. view transform
    p = Rv @ mu_w + t
    if -p[2] < cam["near"]:
        return dict(mean_x=0.0, mean_y=0.0, depth=0.0, cov_xx=0.0, cov_xy=0.0, cov_yy=0.0, opacity=0.0)
    # 3. projective mapping and its Jacobian
    J = project_jacobian(p, cam)
    Sigma_r = J @ Rv @ Sigma_w @ Rv.T @ J.T
    # 4. lift: eigen-decomposition, zero x/y rotation, zero z-scale
    evals, evecs = np.linalg.eigh(Sigma_r)
    R3 = np.eye(3)
    R3[:2, :2] = evecs
    S3 = np.zeros((3, 3))
    S3[0, 0], S3[1, 1] = np.sqrt(np.maximum(evals, 0.0))
    Sigma_v = R3 @ S3 @ S3.T @ R3.T
    mu_v = np.concatenate([project(p, cam), [p[2]]])
    # 5. hologram transform
    Sigma_h = T @ Sigma_v @ T.T
    mu_h = T @ mu_v + tt
    # 6. view-dependent opacity
    centre = -Rv.T @ t
    deg = int(cam["sh_degree"])
    o = float(np.dot(np.asarray(sh, dtype=np.float64)[:(deg + 1) ** 2], real_sh(deg, mu_w - centre)))
    return dict(mean_x=mu_h[0], mean_y=mu_h[1], depth=mu_h[2], cov_xx=Sigma_h[0, 0], cov_xy=Sigma_h[0, 1],
                cov_yy=Sigma_h[1, 1], opacity=min(max(o, 0.0), 1.0))


OUTPUTS = ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity")


def transform(world: dict, cam: dict) -> dict:
    """All Gaussians of `world` (mean [n, 3], quat [n, 4], scale [n, 3], opacity_sh [n, K])."""
    n = len(world["mean"])
    out = {k: np.zeros(n) for k in OUTPUTS}
    for i in range(n):
        r = transform_one(world["mean"][i], world["quat"][i], world["scale"][i], world["opacity_sh"][i], cam)
        for k in OUTPUTS:
            out[k][i] = r[k]
    return out
