"""Seeded synthetic scene generator shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the wave-splatting method itself: it only draws
random in-plane 2D Gaussians (position, depth, covariance built from two scales and a
rotation, opacity, per-channel amplitude, phase) and random target fields, in the
shapes and distributions of the synthetic workloads.  Everything is drawn in float64
with ``numpy.random.Generator(PCG64(seed))`` and cast to float32, so both sides of a
parity check see bit-identical inputs.

Draw order (vectorised, one array per quantity): mean_x, mean_y, depth, s_u, s_v,
theta, opacity, amplitude[c] for c in wavelength order, phase.  The covariance is
Sigma = R(theta) diag(s_u^2, s_v^2) R(theta)^T with the scales in metres, formed in
float64 and cast.  An optional "far" subset (the 1M-Gaussian precision workload)
replaces mean and depth of a random 5% of the Gaussians after the main draw.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

__all__ = ["Grid", "Scene", "TiltedScene", "make_scene", "make_tilted_scene", "make_target", "WORKLOADS",
           "workload"]


@dataclasses.dataclass(frozen=True)
class Grid:
    """Hologram sampling grid: ``ny`` rows by ``nx`` columns at pitch (``px``, ``py``) metres."""

    nx: int
    ny: int
    px: float = 8e-6
    py: float = 8e-6
    lambdas: tuple = (520e-9,)
    # transverse frequency (cycles/m along x, y) of the illuminating reference plane wave,
    # the same for every wavelength; (0, 0) is on-axis illumination
    ref_nu: tuple = (0.0, 0.0)

    @property
    def n_lambda(self) -> int:
        return len(self.lambdas)


@dataclasses.dataclass
class Scene:
    """Structure-of-arrays float32 Gaussians; ``amplitude`` has shape (n_lambda, n)."""

    mean_x: np.ndarray
    mean_y: np.ndarray
    depth: np.ndarray
    cov_xx: np.ndarray
    cov_xy: np.ndarray
    cov_yy: np.ndarray
    opacity: np.ndarray
    amplitude: np.ndarray
    phase: np.ndarray

    @property
    def n(self) -> int:
        return int(self.mean_x.shape[0])

    def fields(self):
        return dict(mean_x=self.mean_x, mean_y=self.mean_y, depth=self.depth,
                    cov_xx=self.cov_xx, cov_xy=self.cov_xy, cov_yy=self.cov_yy,
                    opacity=self.opacity, amplitude=self.amplitude, phase=self.phase)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(**{k: (v[:, idx] if k == "amplitude" else v[idx]) for k, v in self.fields().items()})

    def copy(self) -> "Scene":
        return Scene(**{k: v.copy() for k, v in self.fields().items()})

    @staticmethod
    def concat(scenes: Sequence["Scene"]) -> "Scene":
        out = {}
        for k in scenes[0].fields():
            axis = 1 if k == "amplitude" else 0
            out[k] = np.ascontiguousarray(np.concatenate([getattr(s, k) for s in scenes], axis=axis))
        return Scene(**out)


def make_scene(n: int, grid: Grid, seed: int, depth_range=(-5e-3, 5e-3),
               sigma_px=(2.0, 20.0), opacity_range=(0.1, 1.0),
               far_fraction: float = 0.0, far_depth=(20e-3, 50e-3)) -> Scene:
    """Draw ``n`` random in-plane Gaussians over the field of ``grid``.

    Means are uniform over [-W/2, W/2) x [-H/2, H/2) with W = nx*px, H = ny*py (the
    field is centred on the SLM centre); standard deviations are uniform in
    ``sigma_px`` pixels per principal axis, rotation uniform in [0, pi), opacity and
    per-channel amplitude uniform, phase uniform in [0, 2 pi).  With
    ``far_fraction`` > 0 that fraction of Gaussians is moved to the outer band
    (|x| in [0.4, 0.5) W or |y| in [0.4, 0.5) H) at depths uniform in ``far_depth``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    W, H = grid.nx * grid.px, grid.ny * grid.py
    mean_x = rng.uniform(-W / 2, W / 2, n)
    mean_y = rng.uniform(-H / 2, H / 2, n)
    depth = rng.uniform(depth_range[0], depth_range[1], n)
    s_u = rng.uniform(sigma_px[0], sigma_px[1], n) * grid.px
    s_v = rng.uniform(sigma_px[0], sigma_px[1], n) * grid.py
    theta = rng.uniform(0.0, math.pi, n)
    opacity = rng.uniform(opacity_range[0], opacity_range[1], n)
    amplitude = np.stack([rng.uniform(0.0, 1.0, n) for _ in range(grid.n_lambda)])
    phase = rng.uniform(0.0, 2.0 * math.pi, n)
    if far_fraction > 0.0:
        n_far = int(round(far_fraction * n))
        sel = rng.choice(n, size=n_far, replace=False)
        # outer band: pick an axis, put that coordinate in the band, the other one uniform
        axis_x = rng.uniform(0.0, 1.0, n_far) < 0.5
        band = rng.uniform(0.4, 0.5, n_far) * np.where(rng.uniform(0.0, 1.0, n_far) < 0.5, -1.0, 1.0)
        other = rng.uniform(-0.5, 0.5, n_far)
        mean_x[sel] = np.where(axis_x, band * W, other * W)
        mean_y[sel] = np.where(axis_x, other * H, band * H)
        depth[sel] = rng.uniform(far_depth[0], far_depth[1], n_far)
    c, s = np.cos(theta), np.sin(theta)
    cov_xx = c * c * s_u ** 2 + s * s * s_v ** 2
    cov_xy = c * s * (s_u ** 2 - s_v ** 2)
    cov_yy = s * s * s_u ** 2 + c * c * s_v ** 2
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(mean_x=f32(mean_x), mean_y=f32(mean_y), depth=f32(depth),
                 cov_xx=f32(cov_xx), cov_xy=f32(cov_xy), cov_yy=f32(cov_yy),
                 opacity=f32(opacity), amplitude=f32(amplitude), phase=f32(phase))


@dataclasses.dataclass
class TiltedScene:
    """Structure-of-arrays float32 tilted 2D Gaussians: centre (mean_x, mean_y, depth), unit
    quaternion (w, x, y, z) of the rotation that places the Gaussian's plane, the two in-plane
    scales (metres), opacity, per-channel amplitude (n_lambda, n) and phase."""

    mean_x: np.ndarray
    mean_y: np.ndarray
    depth: np.ndarray
    quat_w: np.ndarray
    quat_x: np.ndarray
    quat_y: np.ndarray
    quat_z: np.ndarray
    scale_u: np.ndarray
    scale_v: np.ndarray
    opacity: np.ndarray
    amplitude: np.ndarray
    phase: np.ndarray

    @property
    def n(self) -> int:
        return int(self.mean_x.shape[0])

    def fields(self):
        return {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}

    def subset(self, idx) -> "TiltedScene":
        idx = np.asarray(idx)
        return TiltedScene(**{k: (v[:, idx] if k == "amplitude" else v[idx]) for k, v in self.fields().items()})

    def copy(self) -> "TiltedScene":
        return TiltedScene(**{k: v.copy() for k, v in self.fields().items()})


def make_tilted_scene(n: int, grid: Grid, seed: int, depth_range=(-5e-3, 5e-3), sigma_px=(2.0, 20.0),
                      opacity_range=(0.1, 1.0), tilt_max_deg: float = 2.0) -> TiltedScene:
    """Draw ``n`` random tilted Gaussians: as ``make_scene`` for position, depth, scales,
    in-plane angle theta, opacity, amplitude and phase, then a tilt: its axis at angle psi
    uniform in [0, 2 pi) in the SLM plane and its angle uniform in [0, ``tilt_max_deg``].
    The rotation is the tilt applied after the in-plane rotation, q = q_tilt * q_z(theta)
    (Hamilton product), stored as a float32 quaternion (w, x, y, z).

    Draw order: mean_x, mean_y, depth, s_u, s_v, theta, psi, tilt, opacity, amplitude[c],
    phase."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W, H = grid.nx * grid.px, grid.ny * grid.py
    mean_x = rng.uniform(-W / 2, W / 2, n)
    mean_y = rng.uniform(-H / 2, H / 2, n)
    depth = rng.uniform(depth_range[0], depth_range[1], n)
    s_u = rng.uniform(sigma_px[0], sigma_px[1], n) * grid.px
    s_v = rng.uniform(sigma_px[0], sigma_px[1], n) * grid.py
    theta = rng.uniform(0.0, math.pi, n)
    psi = rng.uniform(0.0, 2.0 * math.pi, n)
    tilt = np.radians(rng.uniform(0.0, tilt_max_deg, n))
    opacity = rng.uniform(opacity_range[0], opacity_range[1], n)
    amplitude = np.stack([rng.uniform(0.0, 1.0, n) for _ in range(grid.n_lambda)])
    phase = rng.uniform(0.0, 2.0 * math.pi, n)
    # q_tilt = (cos t/2, cos psi sin t/2, sin psi sin t/2, 0), q_z = (cos th/2, 0, 0, sin th/2)
    a0, ax, ay = np.cos(tilt / 2), np.cos(psi) * np.sin(tilt / 2), np.sin(psi) * np.sin(tilt / 2)
    b0, bz = np.cos(theta / 2), np.sin(theta / 2)
    qw, qx, qy, qz = a0 * b0, ax * b0 + ay * bz, ay * b0 - ax * bz, a0 * bz
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return TiltedScene(mean_x=f32(mean_x), mean_y=f32(mean_y), depth=f32(depth), quat_w=f32(qw), quat_x=f32(qx),
                       quat_y=f32(qy), quat_z=f32(qz), scale_u=f32(s_u), scale_v=f32(s_v), opacity=f32(opacity),
                       amplitude=f32(amplitude), phase=f32(phase))


def make_target(grid: Grid, seed: int) -> np.ndarray:
    """i.i.d. circular complex normal CN(0, 1) target field, shape (n_lambda, ny, nx), complex64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (grid.n_lambda, grid.ny, grid.nx)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return ((re + 1j * im) / math.sqrt(2.0)).astype(np.complex64)


RGB = (638e-9, 520e-9, 450e-9)

# The five synthetic workloads: (n, grid, depth range, seed, extras)
WORKLOADS = {
    "small": dict(n=64, grid=Grid(256, 256, 8e-6, 8e-6, (520e-9,)), depth_range=(-5e-3, 5e-3), seed=1001),
    "fwd10k": dict(n=10_000, grid=Grid(1920, 1080, 8e-6, 8e-6, RGB), depth_range=(-10e-3, 10e-3), seed=1002),
    "fwdbwd100k": dict(n=100_000, grid=Grid(1920, 1080, 8e-6, 8e-6, RGB), depth_range=(-10e-3, 10e-3), seed=1003),
    "precision1m": dict(n=1_000_000, grid=Grid(3840, 2160, 8e-6, 8e-6, RGB), depth_range=(-10e-3, 10e-3),
                        seed=1004, far_fraction=0.05),
}


def workload(name: str):
    """Return (scene, grid) for a named workload."""
    w = dict(WORKLOADS[name])
    grid = w.pop("grid")
    n = w.pop("n")
    seed = w.pop("seed")
    return make_scene(n, grid, seed, **w), grid


def batched_counts(n_scenes: int = 16, seed: int = 5000, lo: float = 1e3, hi: float = 5e5):
    """Gaussian counts log-uniform in [lo, hi] for the multi-scene batched workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(round(math.exp(v))) for v in rng.uniform(math.log(lo), math.log(hi), n_scenes)]


# ---- world-space scenes for the holographics transform ----------------------------------

def make_camera(seed: int, nx: int = 1920, ny: int = 1080, pitch: float = 8e-6, sh_degree: int = 3,
                depth_range=(-10e-3, 10e-3), near_far=(1.0, 3.0)) -> dict:
    """A pinhole camera with a random pose (world_to_view = [R | t], rows, R from a random
    rotation vector of ~0.3 rad, t ~ N(0, 0.5 m)), focal lengths 1000 / 1000 px and the
    principal point at the image centre; ray-space pixels map to SLM metres with the principal
    point at the SLM centre, and view distances near_far map linearly onto depth_range (the
    nearest to the largest depth, i.e. closest to the viewer)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rv = rng.normal(0.0, 0.3, 3)
    t = rng.normal(0.0, 0.5, 3)
    ang = float(np.linalg.norm(rv))
    k = rv / ang
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    R = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)
    d0, d1 = near_far
    z0, z1 = depth_range
    # z_h = a * z_view + b with z_view = -d1 -> z0 and z_view = -d0 -> z1
    a = (z1 - z0) / (d1 - d0)
    b = z1 + a * d0
    return dict(world_to_view=np.concatenate([R, t[:, None]], axis=1).ravel().tolist(), fx=1000.0, fy=1000.0,
                cx=nx / 2.0, cy=ny / 2.0, near=0.1,
                ray_to_holo=[pitch, 0.0, -nx / 2.0 * pitch, 0.0, pitch, -ny / 2.0 * pitch],
                depth_scale=a, depth_offset=b, sh_degree=sh_degree)


def make_world_scene(n: int, cam: dict, seed: int, nx: int = 1920, ny: int = 1080, near_far=(1.0, 3.0),
                     sigma_px=(2.0, 20.0), sh_degree: int = 3, flat: bool = True) -> dict:
    """n world-space Gaussians inside the camera's view: view-space positions uniform over
    the image and over the distance range, taken back to world space through the camera pose;
    random unnormalised quaternions (w, x, y, z); scales giving 2-20 px on the image (third
    scale 0 for flat 2D Gaussians); opacity SH coefficients with the degree-0 term giving
    0.1-1 and small higher-order terms.  Draw order: u, v, distance, quaternion, scales, SH."""
    rng = np.random.Generator(np.random.PCG64(seed))
    V = np.asarray(cam["world_to_view"], dtype=np.float64).reshape(3, 4)
    R, t = V[:, :3], V[:, 3]
    u = rng.uniform(0, nx, n)
    v = rng.uniform(0, ny, n)
    dist = rng.uniform(near_far[0], near_far[1], n)
    p = np.stack([(u - cam["cx"]) / cam["fx"] * dist, (v - cam["cy"]) / cam["fy"] * dist, -dist], axis=1)
    mean = (p - t[None, :]) @ R            # R^T (p - t), row-wise
    quat = rng.normal(size=(n, 4))
    s = rng.uniform(sigma_px[0], sigma_px[1], (n, 3)) * (dist / cam["fx"])[:, None]
    if flat:
        s[:, 2] = 0.0
    K = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.05, (n, K))
    sh[:, 0] = rng.uniform(0.1, 1.0, n) / 0.28209479177387814
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(mean=f32(mean), quat=f32(quat), scale=f32(s), opacity_sh=f32(sh))
