"""Pins of the exact alpha wave blending oracle (Sec. 4, Eq. 5-6; supplement Alg. 2).

Each compares the oracle with an independent route:
  * below the alpha threshold the transmittance stays 1 and exact blending is Eq. 12 (the
    order-invariant oracle, itself pinned in test_oracle_pins.py);
  * with no propagation and no phase the paper's alpha wave blending reduces to ray-based
    alpha compositing, which is evaluated here pixel by pixel in space;
  * Gaussians sharing one depth z0 give the z = 0 result propagated by -z0 (independent
    numpy angular-spectrum propagation);
  * one Gaussian, or Gaussians too far apart to occlude one another, are unaffected.
"""
import math

import numpy as np
import pytest

import gwsgen
import oracle
import oracle.exact as ex
from gwsgen import Grid, Scene

T_EPS = 1.0 / 255.0


def small_scene(n, grid, seed, depth_range=(-1e-3, 1e-3), o_range=(0.3, 1.0)):
    s = gwsgen.make_scene(n, grid, seed, depth_range=depth_range)
    rng = np.random.default_rng(seed + 77)
    s.opacity[:] = rng.uniform(*o_range, n).astype(np.float32)
    # cluster the means so the Gaussians overlap and occlude one another
    w, h = grid.nx * grid.px, grid.ny * grid.py
    s.mean_x[:] = (rng.uniform(-0.15, 0.15, n) * w).astype(np.float32)
    s.mean_y[:] = (rng.uniform(-0.15, 0.15, n) * h).astype(np.float32)
    return s


def periodised_profile(scene, i, grid, periods=1):
    """exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)) sampled at x_n = (n - N//2) p, periodised."""
    x = (np.arange(grid.nx) - grid.nx // 2) * grid.px
    y = (np.arange(grid.ny) - grid.ny // 2) * grid.py
    X, Y = np.meshgrid(x, y)
    sxx, sxy, syy = float(scene.cov_xx[i]), float(scene.cov_xy[i]), float(scene.cov_yy[i])
    det = sxx * syy - sxy * sxy
    ixx, ixy, iyy = syy / det, -sxy / det, sxx / det
    W, H = grid.nx * grid.px, grid.ny * grid.py
    g = np.zeros((grid.ny, grid.nx))
    for kx in range(-periods, periods + 1):
        for ky in range(-periods, periods + 1):
            dx = X - float(scene.mean_x[i]) - kx * W
            dy = Y - float(scene.mean_y[i]) - ky * H
            g += np.exp(-0.5 * (ixx * dx * dx + 2 * ixy * dx * dy + iyy * dy * dy))
    return g


def ray_alpha_composite(scene, grid, c):
    """Front-to-back alpha compositing in space (the ray-based counterpart of Eq. 5-6):
    C(x) = sum_k a_k o_k g_k(x) e^{j phi_k} prod_{j in front of k} (1 - alpha_j(x)),
    alpha_j = o_j g_j, dropped where it does not exceed 1/255; front = larger depth."""
    order = sorted(range(scene.n), key=lambda k: (-float(scene.depth[k]), k))
    T = np.ones((grid.ny, grid.nx))
    out = np.zeros((grid.ny, grid.nx), dtype=np.complex128)
    amp = np.reshape(scene.amplitude, (-1, scene.n))
    for k in order:
        g = periodised_profile(scene, k, grid)
        o = float(scene.opacity[k])
        out += float(amp[c, k]) * o * np.exp(1j * float(scene.phase[k])) * T * g
        a = o * g
        T = T * (1.0 - np.where(a > T_EPS, a, 0.0))
    return out


def asm(u, grid, lam, d):
    """u propagated by d with numpy's FFT and the textbook transfer function."""
    fx = np.fft.fftfreq(grid.nx, grid.px)
    fy = np.fft.fftfreq(grid.ny, grid.py)
    FX, FY = np.meshgrid(fx, fy)
    w = 1.0 / lam ** 2 - FX ** 2 - FY ** 2
    Hf = np.where(w > 0, np.exp(2j * np.pi * d * np.sqrt(np.maximum(w, 0.0))), 0.0)
    return np.fft.ifft2(np.fft.fft2(u) * Hf)


GRID = Grid(64, 48, 8e-6, 8e-6, (520e-9, 638e-9))


def test_below_threshold_is_order_invariant_sum():
    s = small_scene(12, GRID, 11)
    s.opacity[:] = np.float32(0.9 * T_EPS)     # every alpha <= 1/255: T stays 1
    U = ex.exact_spectrum(s, GRID)
    ref = oracle.spectrum(s, GRID)
    assert oracle.rel_l2(U, ref) < 1e-11


def test_transmittance_stays_one_below_threshold():
    s = small_scene(6, GRID, 12)
    s.opacity[:] = np.float32(0.5 * T_EPS)
    _, T = ex.exact_spectrum(s, GRID, return_transmittance=True)
    assert np.all(T == 1.0)


def test_no_propagation_no_phase_is_ray_alpha_compositing():
    s = small_scene(10, GRID, 13)
    s.phase[:] = 0.0
    # distinct but negligible depths fix the front-to-back order without propagating:
    # the largest phase 2 pi z / lambda is below 1e-4 rad
    s.depth[:] = (np.arange(s.n)[::-1] * 1e-12).astype(np.float32)
    rng = np.random.default_rng(5)
    s.depth[:] = s.depth[rng.permutation(s.n)]
    u = ex.exact_forward(s, GRID)
    for c in range(GRID.n_lambda):
        ref = ray_alpha_composite(s, GRID, c)
        err = oracle.rel_l2(u[c], ref)
        assert err < 2e-4, err
    # and it is not the order-invariant sum
    assert oracle.rel_l2(u, oracle.forward(s, GRID)) > 1e-2


def test_phase_rides_on_each_term():
    s = small_scene(6, GRID, 14)
    s.depth[:] = (np.arange(s.n) * 1e-12).astype(np.float32)
    u = ex.exact_forward(s, GRID)
    for c in range(GRID.n_lambda):
        assert oracle.rel_l2(u[c], ray_alpha_composite(s, GRID, c)) < 2e-4


def test_common_depth_is_propagated_z0_result():
    s0 = small_scene(8, GRID, 15)
    s0.depth[:] = 0.0
    z0 = 2.5e-3
    s1 = s0.copy()
    s1.depth[:] = np.float32(z0)
    u0 = ex.exact_forward(s0, GRID)
    u1 = ex.exact_forward(s1, GRID)
    for c, lam in enumerate(GRID.lambdas):
        ref = asm(u0[c], GRID, lam, -float(np.float32(z0)))
        assert oracle.rel_l2(u1[c], ref) < 1e-10


def test_single_gaussian_equals_order_invariant_sum():
    s = small_scene(1, GRID, 16, o_range=(1.0, 1.0))
    assert oracle.rel_l2(ex.exact_spectrum(s, GRID), oracle.spectrum(s, GRID)) < 1e-11


def test_far_apart_gaussians_do_not_occlude():
    g = Grid(128, 64, 8e-6, 8e-6, (520e-9,))
    s = small_scene(2, g, 17, o_range=(1.0, 1.0))
    s.cov_xx[:] = np.float32((2.5 * 8e-6) ** 2)
    s.cov_yy[:] = np.float32((2.5 * 8e-6) ** 2)
    s.cov_xy[:] = 0.0
    s.mean_x[:] = np.array([-30 * 8e-6, 30 * 8e-6], dtype=np.float32)
    s.mean_y[:] = 0.0
    s.depth[:] = np.array([1e-3, -1e-3], dtype=np.float32)
    # 60 px apart at sigma 2.5 px: the front alpha is below 1/255 wherever the back field
    # exceeds 1e-40, so T = 1 on the back Gaussian's support
    assert oracle.rel_l2(ex.exact_spectrum(s, g), oracle.spectrum(s, g)) < 1e-11


def test_front_to_back_order_matters():
    s = small_scene(2, GRID, 18, o_range=(0.9, 0.9))
    s.mean_x[:] = 0.0
    s.mean_y[:] = 0.0
    s.depth[:] = np.array([1e-3, -1e-3], dtype=np.float32)
    r = s.copy()
    r.depth[:] = np.array([-1e-3, 1e-3], dtype=np.float32)
    assert oracle.rel_l2(ex.exact_forward(s, GRID), ex.exact_forward(r, GRID)) > 1e-2
