"""Pins of the tilted-Gaussian gradient oracle (oracle/tilted_grad.py).

  * its float64 torch field equals the numpy tilted oracle's field (1e-12);
  * every parameter's gradient of L = Re <G, u> equals fourth-order central differences of the
    numpy oracle's L (strong tilts on a fine grid, two wavelengths, depth and offsets);
  * for rotations about z alone, the gradients of mean, depth, phase, opacity and amplitude equal
    the in-plane C oracle's analytic ones, and the scale gradients equal the chain rule of its
    covariance gradients through Sigma = R diag(s_u^2, s_v^2) R^T.
"""
import math

import numpy as np

import gwsgen
import oracle
import oracle.tilted as otl
import oracle.tilted_grad as otg


def rng_field(grid, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal((grid.n_lambda, grid.ny, grid.nx)) + 1j * r.standard_normal((grid.n_lambda, grid.ny, grid.nx))


def loss(scene, grid, G):
    u = otl.forward(scene, grid)
    return float(np.sum(G.real * u.real + G.imag * u.imag))


def f64(scene):
    s = scene.copy()
    for k, v in s.fields().items():
        setattr(s, k, np.asarray(v, dtype=np.float64).copy())
    return s


def test_torch_field_equals_numpy_oracle():
    grid = gwsgen.Grid(40, 36, 1e-6, 1e-6, (520e-9, 633e-9))
    sc = f64(gwsgen.make_tilted_scene(6, grid, 51, depth_range=(-20e-6, 20e-6), sigma_px=(1.5, 4.0), tilt_max_deg=25.0))
    import torch
    p = {k: torch.tensor(getattr(sc, k)) for k in otg.PARAMS}
    a = otg.field(p, grid).numpy()
    b = otl.forward(sc, grid)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_gradients_match_finite_differences():
    grid = gwsgen.Grid(32, 28, 1e-6, 1e-6, (520e-9, 633e-9))
    sc = f64(gwsgen.make_tilted_scene(3, grid, 52, depth_range=(-15e-6, 15e-6), sigma_px=(1.5, 3.0), tilt_max_deg=30.0))
    G = rng_field(grid, 53)
    got = otg.backward(sc, grid, G)
    steps = {"mean_x": 1e-8, "mean_y": 1e-8, "depth": 2e-9, "quat_w": 1e-5, "quat_x": 1e-5, "quat_y": 1e-5,
             "quat_z": 1e-5, "scale_u": 1e-9, "scale_v": 1e-9, "opacity": 1e-4, "amplitude": 1e-4, "phase": 1e-4}
    for name, h in steps.items():
        for i in range(sc.n):
            cs = [0] if name != "amplitude" else [0, 1]
            for c in cs:
                def at(delta):
                    s2 = sc.copy()
                    arr = getattr(s2, name)
                    if name == "amplitude":
                        arr[c, i] += delta
                    else:
                        arr[i] += delta
                    return loss(s2, grid, G)
                fd = (8 * (at(h) - at(-h)) - (at(2 * h) - at(-2 * h))) / (12 * h)
                g = got[name][c, i] if name == "amplitude" else got[name][i]
                scale = max(abs(fd), 1e-3 * max(abs(v) for v in np.ravel(got[name])))
                assert abs(g - fd) <= 1e-5 * scale, (name, i, c, g, fd)


def test_rotation_about_z_matches_in_plane_gradients():
    grid = gwsgen.Grid(48, 40, 8e-6, 8e-6, gwsgen.RGB)
    rng = np.random.default_rng(54)
    n = 5
    W, H = grid.nx * grid.px, grid.ny * grid.py
    th = rng.uniform(-math.pi, math.pi, n)
    su, sv = rng.uniform(1.5, 5, n) * 8e-6, rng.uniform(1.5, 5, n) * 8e-6
    sc = gwsgen.TiltedScene(mean_x=rng.uniform(-W / 2, W / 2, n), mean_y=rng.uniform(-H / 2, H / 2, n),
                            depth=rng.uniform(-5e-3, 5e-3, n), quat_w=np.cos(th / 2), quat_x=np.zeros(n),
                            quat_y=np.zeros(n), quat_z=np.sin(th / 2), scale_u=su, scale_v=sv,
                            opacity=rng.uniform(0.1, 1, n), amplitude=rng.uniform(0, 1, (3, n)),
                            phase=rng.uniform(0, 2 * math.pi, n))
    c, s = np.cos(th), np.sin(th)
    ip = gwsgen.Scene(mean_x=sc.mean_x, mean_y=sc.mean_y, depth=sc.depth, cov_xx=c * c * su ** 2 + s * s * sv ** 2,
                      cov_xy=c * s * (su ** 2 - sv ** 2), cov_yy=s * s * su ** 2 + c * c * sv ** 2,
                      opacity=sc.opacity, amplitude=sc.amplitude, phase=sc.phase)
    G = rng_field(grid, 55)
    got = otg.backward(sc, grid, G)
    ref = oracle.backward(ip, grid, G)
    for k in ("mean_x", "mean_y", "depth", "phase", "opacity"):
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-8 * np.max(np.abs(ref[k])), k
    assert np.max(np.abs(got["amplitude"] - ref["amplitude"])) <= 1e-8 * np.max(np.abs(ref["amplitude"]))
    # scales: dL/ds_u = 2 s_u r1^T G_S r1 with G_S = [[g_xx, g_xy / 2], [g_xy / 2, g_yy]]
    for i in range(n):
        GS = np.array([[ref["cov_xx"][i], ref["cov_xy"][i] / 2], [ref["cov_xy"][i] / 2, ref["cov_yy"][i]]])
        r1, r2 = np.array([c[i], s[i]]), np.array([-s[i], c[i]])
        for name, sgm, r in (("scale_u", su[i], r1), ("scale_v", sv[i], r2)):
            want = 2 * sgm * r @ GS @ r
            assert abs(got[name][i] - want) <= 1e-8 * max(abs(want), 1e-30), (name, i)
