"""Pins of the tilted-Gaussian oracle (oracle/tilted.py).

Each compares the oracle with a route that does not use its remap:
  * a rotation about z alone is an in-plane Gaussian: the tilted oracle must equal the in-plane
    C oracle (Eq. 10) with Sigma = R S^2 R^T, to rounding, over depths, phases, amplitudes and
    three wavelengths;
  * brute force: the field of one strongly tilted Gaussian, written as the superposition of the
    plane waves of the disk's own frame (its 2D spectrum integrated over (k_ox, k_oy) by the
    trapezoid rule, each wave carried to SLM pixels by exp(j 2 pi k . (x - mu)) with k = R k_o),
    against the oracle's field at sampled pixels: no remap and no Jacobian are involved, so a
    transposed rotation, a dropped, inverted or misplaced det J, a swapped scale or a sign slip
    of the ramp or the propagation all show;
  * the same disk described by R and by R diag(1, -1, -1) (the quaternion times (0, 1, 0, 0))
    gives the same spectrum (reading T1);
  * evanescent frequencies carry nothing, and a reference-wave shift is refused.
"""
import math

import numpy as np
import pytest

import gwsgen
import oracle
import oracle.tilted as tl


def tilted_from(mean, depth, quats, su, sv, opacity, amplitude, phase):
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    q = np.asarray(quats, dtype=np.float64)
    return gwsgen.TiltedScene(mean_x=f(mean[:, 0]), mean_y=f(mean[:, 1]), depth=f(depth), quat_w=f(q[:, 0]),
                              quat_x=f(q[:, 1]), quat_y=f(q[:, 2]), quat_z=f(q[:, 3]), scale_u=f(su), scale_v=f(sv),
                              opacity=f(opacity), amplitude=f(amplitude), phase=f(phase))


def test_rotation_about_z_is_the_in_plane_gaussian():
    grid = gwsgen.Grid(48, 40, 8e-6, 8e-6, gwsgen.RGB)
    rng = np.random.default_rng(11)
    n = 7
    W, H = grid.nx * grid.px, grid.ny * grid.py
    mean = np.stack([rng.uniform(-W / 2, W / 2, n), rng.uniform(-H / 2, H / 2, n)], axis=1)
    depth = rng.uniform(-8e-3, 8e-3, n)
    su, sv = rng.uniform(1.5, 6, n) * 8e-6, rng.uniform(1.5, 6, n) * 8e-6
    th = rng.uniform(-math.pi, math.pi, n)
    quats = np.stack([np.cos(th / 2), 0 * th, 0 * th, np.sin(th / 2)], axis=1)
    opacity, phase = rng.uniform(0.1, 1, n), rng.uniform(0, 2 * math.pi, n)
    amplitude = rng.uniform(0, 1, (3, n))
    ts = tilted_from(mean, depth, quats, su, sv, opacity, amplitude, phase)
    c, s = np.cos(th), np.sin(th)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    ip = gwsgen.Scene(mean_x=f(mean[:, 0]), mean_y=f(mean[:, 1]), depth=f(depth),
                      cov_xx=f(c * c * su ** 2 + s * s * sv ** 2), cov_xy=f(c * s * (su ** 2 - sv ** 2)),
                      cov_yy=f(s * s * su ** 2 + c * c * sv ** 2), opacity=f(opacity), amplitude=f(amplitude),
                      phase=f(phase))
    got = tl.spectrum(ts, grid)
    ref = oracle.spectrum(ip, grid, ordered=False)
    # rounding only: the phases reach 2 pi z / lambda ~ 1e5 rad, whose FP64 ulp is ~1e-11 rad
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def plane_wave_field(R, su, sv, mean3, lam, pts, a=1.0, phi=0.0, nsig=9.0, h=1.0e4):
    """u(x) = a e^{j phi} sum over the disk-frame plane waves: the 2D Gaussian spectrum on the
    disk's own plane (Fourier pair of the canonical Gaussian) at (k_ox, k_oy), the wave vector
    k = R k_o with k_oz = +sqrt(1/lambda^2 - k_ox^2 - k_oy^2), trapezoid rule in (k_ox, k_oy)."""
    Lu, Lv = nsig / (2 * math.pi * su), nsig / (2 * math.pi * sv)
    ku = np.arange(-Lu, Lu + h / 2, h)
    kv = np.arange(-Lv, Lv + h / 2, h)
    KU, KV = np.meshgrid(ku, kv, indexing="ij")
    KU, KV = KU.ravel(), KV.ravel()
    KW = np.sqrt(1.0 / lam ** 2 - KU ** 2 - KV ** 2)
    G = 2 * math.pi * su * sv * np.exp(-0.5 * (2 * math.pi) ** 2 * (su ** 2 * KU ** 2 + sv ** 2 * KV ** 2))
    K = R @ np.stack([KU, KV, KW])                       # hologram-frame wave vectors
    assert np.all(K[2] > 0)                              # every wave heads for the SLM side
    d = pts - mean3[None, :]                             # pixel minus centre, 3D
    out = np.empty(len(pts), dtype=np.complex128)
    for i in range(len(pts)):
        out[i] = np.sum(G * np.exp(2j * math.pi * (d[i] @ K))) * h * h
    return a * np.exp(1j * phi) * out


@pytest.mark.parametrize("case", [0, 1])
def test_field_matches_plane_wave_superposition(case):
    # a fine grid whose band holds the whole propagating disk of 1/lambda, so a 20-28 degree
    # tilt keeps the Gaussian's spectrum inside it
    lam = (500e-9, 633e-9)
    grid = gwsgen.Grid(160, 144, 0.2e-6, 0.2e-6, lam)
    rng = np.random.default_rng(20 + case)
    tilt, psi, th = math.radians(20 + 8 * case), rng.uniform(0, 2 * math.pi), rng.uniform(0, math.pi)
    qt = np.array([math.cos(tilt / 2), math.cos(psi) * math.sin(tilt / 2), math.sin(psi) * math.sin(tilt / 2), 0])
    qz = np.array([math.cos(th / 2), 0, 0, math.sin(th / 2)])
    # Hamilton product qt * qz
    q = np.array([qt[0] * qz[0] - qt[3] * qz[3], qt[1] * qz[0] + qt[2] * qz[3], qt[2] * qz[0] - qt[1] * qz[3],
                  qt[0] * qz[3] + qt[3] * qz[0]])
    su, sv = 1.7e-6, 2.2e-6
    mean = np.array([[0.8e-6, -1.1e-6]])
    depth = np.array([2.5e-6 if case == 0 else -3.0e-6])
    amp = np.array([[0.7], [0.4]])
    ts = tilted_from(mean, depth, q[None, :], [su], [sv], [0.9], amp, [1.3])
    u = tl.forward(ts, grid)
    R = oracle.holographics.quat_to_matrix(q)
    py_, px_ = np.meshgrid(np.arange(grid.ny), np.arange(grid.nx), indexing="ij")
    sel = rng.choice(grid.nx * grid.ny, 160, replace=False)
    # half of the samples near the centre, where the field is large
    r2 = ((px_.ravel() - grid.nx // 2) * grid.px - mean[0, 0]) ** 2 + ((py_.ravel() - grid.ny // 2) * grid.py
                                                                       - mean[0, 1]) ** 2
    near = np.argsort(r2)[:2000]
    sel = np.concatenate([sel, rng.choice(near, 160, replace=False)])
    pts = np.stack([(px_.ravel()[sel] - grid.nx // 2) * grid.px, (py_.ravel()[sel] - grid.ny // 2) * grid.py,
                    np.zeros(sel.size)], axis=1)
    mean3 = np.array([mean[0, 0], mean[0, 1], depth[0]])
    for c, l in enumerate(lam):
        ref = plane_wave_field(R, su, sv, mean3, l, pts, a=amp[c, 0] * 0.9, phi=1.3)
        got = u[c].ravel()[sel]
        scale = np.max(np.abs(u[c]))
        assert scale > 0.1 * np.max(np.abs(ref))
        err = np.max(np.abs(got - ref)) / scale
        assert err < 1e-9, (c, err)


def test_flipped_description_of_the_same_disk():
    grid = gwsgen.Grid(40, 36, 2e-6, 2e-6, (520e-9, 450e-9))
    sc = gwsgen.make_tilted_scene(5, grid, 31, sigma_px=(1.0, 3.0), tilt_max_deg=25.0)
    fl = sc.copy()
    # q * (0, 1, 0, 0): R -> R diag(1, -1, -1)
    w, x, y, z = (sc.quat_w.astype(np.float64), sc.quat_x.astype(np.float64), sc.quat_y.astype(np.float64),
                  sc.quat_z.astype(np.float64))
    fl.quat_w, fl.quat_x, fl.quat_y, fl.quat_z = -x, w, z, -y
    a, b = tl.spectrum(sc, grid), tl.spectrum(fl, grid)
    assert np.max(np.abs(a)) > 0
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_evanescent_band_and_reference_wave():
    # pitch below lambda / 2: the grid's corners are evanescent
    grid = gwsgen.Grid(32, 32, 0.2e-6, 0.2e-6, (520e-9,))
    sc = gwsgen.make_tilted_scene(3, grid, 41, sigma_px=(0.5, 1.0), tilt_max_deg=30.0)
    U = tl.spectrum(sc, grid)
    mx = oracle.signed_freq_index(grid.nx) / (grid.nx * grid.px)
    my = oracle.signed_freq_index(grid.ny) / (grid.ny * grid.py)
    ev = (my[:, None] ** 2 + mx[None, :] ** 2) >= (1 / 520e-9) ** 2
    assert ev.any() and (~ev).any()
    assert np.all(U[0][ev] == 0) and np.any(U[0][~ev] != 0)
    with pytest.raises(ValueError):
        tl.spectrum(sc, gwsgen.Grid(32, 32, 8e-6, 8e-6, (520e-9,), ref_nu=(1000.0, 0.0)))
