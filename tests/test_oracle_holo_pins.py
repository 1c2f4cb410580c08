"""Pins of the holographics oracle (oracle/holographics.py).

Each compares the oracle with an independent route:
  * the quaternion rotation against scipy's Rotation;
  * the projection Jacobian against central differences of the projection;
  * the projected covariance against the sample covariance of points drawn from the 3D
    Gaussian and projected exactly (perspective, no linearisation);
  * a Gaussian on the optical axis, facing the camera, against the closed form (f sigma / d)^2;
  * the spherical-harmonic basis against orthonormality on the sphere (quadrature) and the
    signs of the degree-1 functions;
  * culling behind the near plane, and the hologram transform's scaling and offsets.
"""
import math

import numpy as np
from scipy.spatial.transform import Rotation

import oracle.holographics as hg

CAM = dict(world_to_view=[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], fx=1000.0, fy=900.0, cx=960.0, cy=540.0, near=0.1,
           ray_to_holo=[8e-6, 0, -960 * 8e-6, 0, 8e-6, -540 * 8e-6], depth_scale=0.01, depth_offset=0.02,
           sh_degree=3)


def rotated_camera(seed):
    rng = np.random.default_rng(seed)
    R = Rotation.from_rotvec(rng.normal(0, 0.3, 3)).as_matrix()
    t = rng.normal(0, 0.5, 3)
    cam = dict(CAM)
    cam["world_to_view"] = np.concatenate([R, t[:, None]], axis=1).ravel().tolist()
    return cam, R, t


def test_quaternion_matches_scipy():
    rng = np.random.default_rng(1)
    for _ in range(20):
        q = rng.normal(size=4) * 3.0          # not normalised: the oracle normalises
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()   # scipy takes (x, y, z, w)
        assert np.max(np.abs(hg.quat_to_matrix(q) - ref)) < 1e-14


def test_jacobian_is_derivative_of_projection():
    rng = np.random.default_rng(2)
    for _ in range(20):
        p = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), -rng.uniform(0.5, 3)])
        J = hg.project_jacobian(p, CAM)
        h = 1e-6
        num = np.stack([(hg.project(p + h * e, CAM) - hg.project(p - h * e, CAM)) / (2 * h) for e in np.eye(3)], axis=1)
        assert np.max(np.abs(J - num)) < 1e-5 * np.max(np.abs(J))


def test_projected_covariance_matches_projected_samples():
    # a small Gaussian far from the camera: the perspective nonlinearity is O((sigma / depth)^2)
    cam, Rv, t = rotated_camera(3)
    rng = np.random.default_rng(4)
    p_view = np.array([0.3, -0.2, -2.5])
    mu = Rv.T @ (p_view - t)
    q = rng.normal(size=4)
    s = np.array([4e-3, 2e-3, 1e-3])
    out = hg.transform_one(mu, q, s, np.r_[1.0, np.zeros(15)], cam)
    M = hg.quat_to_matrix(q) @ np.diag(s)
    N = 400000
    xw = mu[None, :] + rng.standard_normal((N, 3)) @ M.T
    pv = xw @ Rv.T + t
    uv = np.stack([cam["fx"] * pv[:, 0] / -pv[:, 2] + cam["cx"], cam["fy"] * pv[:, 1] / -pv[:, 2] + cam["cy"]], 1)
    A = np.asarray(cam["ray_to_holo"]).reshape(2, 3)[:, :2]
    C = A @ np.cov(uv.T) @ A.T
    got = np.array([[out["cov_xx"], out["cov_xy"]], [out["cov_xy"], out["cov_yy"]]])
    # Monte-Carlo error of a covariance estimate ~ sqrt(2 / N) relative
    assert np.max(np.abs(got - C)) < 0.01 * np.max(np.abs(C))
    mean_h = A @ uv.mean(axis=0) + np.asarray(cam["ray_to_holo"]).reshape(2, 3)[:, 2]
    assert abs(out["mean_x"] - mean_h[0]) < 0.01 * math.sqrt(C[0, 0])
    assert abs(out["mean_y"] - mean_h[1]) < 0.01 * math.sqrt(C[1, 1])


def test_on_axis_facing_gaussian_closed_form():
    d, sx, sy = 2.0, 3e-3, 1e-3
    out = hg.transform_one([0, 0, -d], [1, 0, 0, 0], [sx, sy, 0.0], np.r_[0.9 / 0.28209479177387814, np.zeros(15)], CAM)
    p = 8e-6
    assert abs(out["cov_xx"] - (CAM["fx"] * sx / d * p) ** 2) < 1e-12 * out["cov_xx"]
    assert abs(out["cov_yy"] - (CAM["fy"] * sy / d * p) ** 2) < 1e-12 * out["cov_yy"]
    assert abs(out["cov_xy"]) < 1e-25
    assert abs(out["mean_x"]) < 1e-18 and abs(out["mean_y"]) < 1e-18     # principal point -> SLM centre
    assert abs(out["depth"] - (0.01 * -d + 0.02)) < 1e-15
    assert abs(out["opacity"] - 0.9) < 1e-12                              # constant (degree-0) opacity


def test_sh_basis_is_orthonormal_with_the_stated_signs():
    # Gauss-Legendre in cos(theta) x uniform phi integrates products of degree <= 6 exactly
    xg, wg = np.polynomial.legendre.leggauss(12)
    nph = 24
    G = np.zeros((16, 16))
    for ct, w in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for j in range(nph):
            ph = 2 * math.pi * j / nph
            y = hg.real_sh(3, [st * math.cos(ph), st * math.sin(ph), ct])
            G += w * (2 * math.pi / nph) * np.outer(y, y)
    assert np.max(np.abs(G - np.eye(16))) < 1e-12
    c1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(hg.real_sh(1, [1, 0, 0])[1:], [0, 0, -c1])
    assert np.allclose(hg.real_sh(1, [0, 1, 0])[1:], [-c1, 0, 0])
    assert np.allclose(hg.real_sh(1, [0, 0, 1])[1:], [0, c1, 0])


def test_view_dependent_opacity_follows_the_direction():
    # a degree-1 term along +x: seen from -x (direction +x) the opacity rises, from +x it falls
    sh = np.zeros(16)
    sh[0] = 0.5 / 0.28209479177387814
    sh[3] = -0.3 / math.sqrt(3 / (4 * math.pi))       # times Y_1^1 = -c1 x: +0.3 x
    cam = dict(CAM)
    o_plus = hg.transform_one([1.0, 0, -2.0], [1, 0, 0, 0], [1e-3, 1e-3, 0], sh, cam)["opacity"]
    o_minus = hg.transform_one([-1.0, 0, -2.0], [1, 0, 0, 0], [1e-3, 1e-3, 0], sh, cam)["opacity"]
    dx = 1 / math.sqrt(5)
    assert abs(o_plus - (0.5 + 0.3 * dx)) < 1e-12
    assert abs(o_minus - (0.5 - 0.3 * dx)) < 1e-12


def test_near_plane_culls_and_opacity_clamps():
    assert hg.transform_one([0, 0, 0.5], [1, 0, 0, 0], [1e-3] * 3, np.ones(16), CAM)["opacity"] == 0.0
    assert hg.transform_one([0, 0, -0.05], [1, 0, 0, 0], [1e-3] * 3, np.ones(16), CAM)["opacity"] == 0.0
    big = np.r_[10.0, np.zeros(15)]
    assert hg.transform_one([0, 0, -2], [1, 0, 0, 0], [1e-3] * 3, big, CAM)["opacity"] == 1.0
    assert hg.transform_one([0, 0, -2], [1, 0, 0, 0], [1e-3] * 3, -big, CAM)["opacity"] == 0.0


def test_camera_motion_is_rigid():
    # moving the camera and the scene together leaves every output unchanged
    cam, Rv, t = rotated_camera(6)
    rng = np.random.default_rng(7)
    for _ in range(5):
        p = np.array([rng.uniform(-.5, .5), rng.uniform(-.3, .3), -rng.uniform(1, 3)])
        q = rng.normal(size=4)
        s = rng.uniform(1e-3, 5e-3, 3)
        sh = rng.normal(0, 0.2, 16)
        sh[0] = 1.5
        a = hg.transform_one(p, q, s, sh, CAM)
        # the same Gaussian in world coordinates seen by the moved camera
        Rq = Rotation.from_matrix(Rv.T).as_quat()                 # world rotation = Rv^T * local
        qw = Rotation.from_quat([Rq[0], Rq[1], Rq[2], Rq[3]]) * Rotation.from_quat([q[1], q[2], q[3], q[0]])
        xyzw = qw.as_quat()
        b = hg.transform_one(Rv.T @ (p - t), [xyzw[3], xyzw[0], xyzw[1], xyzw[2]], s, sh, cam)
        for k in ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy"):
            assert abs(a[k] - b[k]) <= 1e-9 * max(abs(a[k]), 1e-12), k
        # the view direction rotates with the camera, so SH opacity is not invariant unless
        # the coefficients rotate too; the degree-0 part alone is
        sh0 = np.r_[sh[0], np.zeros(15)]
        assert abs(hg.transform_one(p, q, s, sh0, CAM)["opacity"] -
                   hg.transform_one(Rv.T @ (p - t), [xyzw[3], xyzw[0], xyzw[1], xyzw[2]], s, sh0, cam)["opacity"]) < 1e-12
