"""Pins of the exact-blending gradient oracle (reverse-mode differentiation of Alg. 2 in
float64 PyTorch): its field is the numpy oracle's, its gradients are central differences of
the numpy oracle's loss, and below the alpha threshold they are the order-invariant oracle's
analytic gradients (test_oracle_pins.py pins those)."""
import numpy as np
import pytest

import gwsgen
import oracle
import oracle.exact as ex
import oracle.exact_grad as eg
from gwsgen import Grid

GRID = Grid(32, 24, 8e-6, 8e-6, (520e-9, 638e-9))


def tiny_scene(n, seed, o_range=(0.4, 1.0)):
    s = gwsgen.make_scene(n, GRID, seed, depth_range=(-2e-3, 2e-3))
    rng = np.random.default_rng(seed + 3)
    su, sv = rng.uniform(1.5, 3.0, n), rng.uniform(1.5, 3.0, n)
    th = rng.uniform(0, np.pi, n)
    c, sn = np.cos(th), np.sin(th)
    p2 = GRID.px * GRID.py
    s.cov_xx[:] = ((c * c * su * su + sn * sn * sv * sv) * p2).astype(np.float32)
    s.cov_xy[:] = ((c * sn * (su * su - sv * sv)) * p2).astype(np.float32)
    s.cov_yy[:] = ((sn * sn * su * su + c * c * sv * sv) * p2).astype(np.float32)
    s.mean_x[:] = (rng.uniform(-3, 3, n) * GRID.px).astype(np.float32)
    s.mean_y[:] = (rng.uniform(-3, 3, n) * GRID.py).astype(np.float32)
    s.opacity[:] = rng.uniform(*o_range, n).astype(np.float32)
    return s


def numpy_loss(scene, target):
    u = ex.exact_forward(scene, GRID)
    return float(np.sum(np.abs(u - target) ** 2))


def test_field_is_the_numpy_oracle_field():
    s = tiny_scene(5, 301)
    t = gwsgen.make_target(GRID, 302)
    _, u, _ = eg.exact_loss_grads(s, GRID, t)
    assert oracle.rel_l2(u, ex.exact_forward(s, GRID)) < 1e-12


@pytest.mark.parametrize("param", eg.PARAMS)
def test_gradients_are_central_differences(param):
    s = tiny_scene(4, 303)
    t = gwsgen.make_target(GRID, 304) * 0.3
    _, _, grads = eg.exact_loss_grads(s, GRID, t)
    base = {k: np.asarray(getattr(s, k), dtype=np.float64).copy() for k in eg.PARAMS}
    # depth steps turn the propagation phase 2 pi z sqrt(1/l^2 - nu^2) by up to 2 pi h / l, so they
    # stay well below a wavelength
    scale = {"mean_x": GRID.px, "mean_y": GRID.py, "depth": 1e-5, "cov_xx": 4 * GRID.px ** 2,
             "cov_xy": 4 * GRID.px ** 2, "cov_yy": 4 * GRID.px ** 2, "opacity": 1.0, "amplitude": 1.0,
             "phase": 1.0}[param]
    h = 1e-5 * scale
    g_ad = np.asarray(grads[param])
    flat = g_ad.reshape(-1)
    for i in range(flat.size):
        vals = []
        for sgn in (1, -1):
            sc = s.copy()
            for k in eg.PARAMS:          # float64 copies so the step is not rounded to float32
                setattr(sc, k, base[k].copy())
            arr = getattr(sc, param).reshape(-1)
            arr[i] += sgn * h
            vals.append(numpy_loss(sc, t))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - flat[i]) <= 1e-5 * (abs(fd) + abs(flat[i])) + 1e-9 / scale, (param, i, fd, flat[i])


def test_below_threshold_gradients_are_order_invariant_gradients():
    s = tiny_scene(6, 305, o_range=(0.5 / 255, 0.9 / 255))
    t = gwsgen.make_target(GRID, 306) * 1e-3
    _, u, grads = eg.exact_loss_grads(s, GRID, t)
    _, G = oracle.loss_and_field_grad(u, t)
    ref = oracle.backward(s, GRID, G)
    for k in eg.PARAMS:
        err = oracle.rel_l2(np.asarray(grads[k]), np.asarray(ref[k]))
        assert err < 1e-9, (k, err)
