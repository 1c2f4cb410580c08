"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these retype the oracle's formula: each compares it with an independent route
(spatial sampling + numpy FFT, a closed form, an identity of the DFT, finite
differences) chosen so that a plausible slip in the oracle -- a dropped 2 pi, a wrong
sign of the ramp or of the propagation, a transposed axis, a missing sqrt(det Sigma),
a wrong centring -- fails at least one of them.
"""
import math

import numpy as np
import pytest

import gwsgen
import oracle
from gwsgen import Grid, Scene


def one_gaussian(mx, my, z, sxx, sxy, syy, o=1.0, a=(1.0,), phi=0.0, dtype=np.float64):
    arr = lambda v: np.array([v], dtype=dtype)
    return Scene(mean_x=arr(mx), mean_y=arr(my), depth=arr(z), cov_xx=arr(sxx), cov_xy=arr(sxy),
                 cov_yy=arr(syy), opacity=arr(o), amplitude=np.array([[v] for v in a], dtype=dtype),
                 phase=arr(phi))


def cov_from(su_px, sv_px, theta, p):
    c, s = math.cos(theta), math.sin(theta)
    su, sv = su_px * p, sv_px * p
    return c * c * su ** 2 + s * s * sv ** 2, c * s * (su ** 2 - sv ** 2), s * s * su ** 2 + c * c * sv ** 2


def spatial_gaussian(scene, grid, c, periods=2):
    """Sample a_c o e^{j phi} exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)) on the grid, periodised.  With a
    reference plane wave (grid.ref_nu, on the frequency lattice so that it is periodic on the
    grid) the samples are multiplied by exp(+j 2 pi nu_r . x), x measured from the SLM centre."""
    nx, ny, px, py = grid.nx, grid.ny, grid.px, grid.py
    x = (np.arange(nx) - nx // 2) * px
    y = (np.arange(ny) - ny // 2) * py
    X, Y = np.meshgrid(x, y)
    tilt = np.exp(2j * math.pi * (grid.ref_nu[0] * X + grid.ref_nu[1] * Y))
    out = np.zeros((ny, nx), dtype=np.complex128)
    W, H = nx * px, ny * py
    for i in range(scene.n):
        sxx, sxy, syy = float(scene.cov_xx[i]), float(scene.cov_xy[i]), float(scene.cov_yy[i])
        det = sxx * syy - sxy * sxy
        ixx, ixy, iyy = syy / det, -sxy / det, sxx / det
        amp = float(scene.amplitude[c][i]) * float(scene.opacity[i]) * np.exp(1j * float(scene.phase[i]))
        for kx in range(-periods, periods + 1):
            for ky in range(-periods, periods + 1):
                dx = X - float(scene.mean_x[i]) - kx * W
                dy = Y - float(scene.mean_y[i]) - ky * H
                out += amp * np.exp(-0.5 * (ixx * dx * dx + 2 * ixy * dx * dy + iyy * dy * dy))
    return out * tilt


def freq_grid(grid):
    nux = oracle.signed_freq_index(grid.nx) / (grid.nx * grid.px)
    nuy = oracle.signed_freq_index(grid.ny) / (grid.ny * grid.py)
    return np.meshgrid(nux, nuy)


def asm_propagate(u, grid, lam, d):
    """FFT-based angular spectrum method P(u; d) with numpy's FFT (independent of the oracle)."""
    NX, NY = freq_grid(grid)
    w2 = 1.0 / lam ** 2 - NX ** 2 - NY ** 2
    H = np.where(w2 > 0, np.exp(2j * math.pi * d * np.sqrt(np.maximum(w2, 0.0))), 0.0)
    return np.fft.fftshift(np.fft.ifft2(np.fft.fft2(np.fft.ifftshift(u)) * H))


def brute_force_field(scene, grid):
    """P1: spatial samples -> numpy FFT -> H(nu, -z_i) per Gaussian -> inverse FFT."""
    out = np.zeros((grid.n_lambda, grid.ny, grid.nx), dtype=np.complex128)
    for c, lam in enumerate(grid.lambdas):
        for i in range(scene.n):
            g = spatial_gaussian(scene.subset([i]), grid, c)
            out[c] += asm_propagate(g, grid, lam, -float(scene.depth[i]))
    return out


def test_p1_brute_force_tiny_grids():
    rng = np.random.default_rng(7)
    for (nx, ny) in [(64, 48), (40, 56), (45, 33)]:
        grid = Grid(nx, ny, 8e-6, 6e-6, (638e-9, 450e-9))
        n = 4
        sxx, sxy, syy = zip(*[cov_from(rng.uniform(2.5, 5), rng.uniform(2.5, 5), rng.uniform(0, math.pi), 7e-6)
                              for _ in range(n)])
        scene = Scene(mean_x=rng.uniform(-0.3, 0.3, n) * nx * grid.px, mean_y=rng.uniform(-0.3, 0.3, n) * ny * grid.py,
                      depth=rng.uniform(-3e-3, 3e-3, n), cov_xx=np.array(sxx), cov_xy=np.array(sxy),
                      cov_yy=np.array(syy), opacity=rng.uniform(0.1, 1, n), amplitude=rng.uniform(0, 1, (2, n)),
                      phase=rng.uniform(0, 2 * math.pi, n))
        u = oracle.forward(scene, grid)
        ref = brute_force_field(scene, grid)
        assert oracle.rel_l2(u, ref) < 1e-9, (nx, ny, oracle.rel_l2(u, ref))


def test_p8_zero_depth_is_sampled_gaussian_peak_at_mean():
    """z = 0, phi = 0: the field is the sampled Gaussian (Eq. 7 pair); its peak a*o sits at mu."""
    grid = Grid(96, 80, 8e-6, 8e-6, (520e-9,))
    sxx, sxy, syy = cov_from(4.0, 2.5, 0.6, 8e-6)
    scene = one_gaussian(3 * 8e-6, -2 * 8e-6, 0.0, sxx, sxy, syy, o=0.7, a=(0.5,))
    u = oracle.forward(scene, grid)[0]
    ref = spatial_gaussian(scene, grid, 0)
    assert oracle.rel_l2(u, ref) < 1e-12
    iy, ix = np.unravel_index(np.argmax(np.abs(u)), u.shape)
    assert (ix - grid.nx // 2, iy - grid.ny // 2) == (3, -2)
    assert abs(u[iy, ix] - 0.35) < 1e-12
    assert np.max(np.abs(u.imag)) < 1e-12 * np.max(np.abs(u))


def test_p2_translation_is_cyclic_shift_and_linear_phase():
    grid = Grid(64, 48, 8e-6, 8e-6, (520e-9, 450e-9))
    sxx, sxy, syy = cov_from(3.0, 5.0, 1.1, 8e-6)
    base = one_gaussian(1.3e-5, -2.1e-5, 2.5e-3, sxx, sxy, syy, o=0.8, a=(0.9, 0.4), phi=1.0)
    shifted = base.copy()
    shifted.mean_x += 5 * grid.px
    shifted.mean_y -= 3 * grid.py
    u0, u1 = oracle.forward(base, grid), oracle.forward(shifted, grid)
    assert np.max(np.abs(u1 - np.roll(u0, (-3, 5), axis=(1, 2)))) < 1e-11 * np.max(np.abs(u0))
    # sub-pixel shift: the spectrum picks up exactly exp(-j 2 pi nu . delta)
    d = (0.37 * grid.px, -1.61 * grid.py)
    sub = base.copy()
    sub.mean_x += d[0]
    sub.mean_y += d[1]
    NX, NY = freq_grid(grid)
    U0, U1 = oracle.spectrum(base, grid), oracle.spectrum(sub, grid)
    assert oracle.rel_l2(U1, U0 * np.exp(-2j * math.pi * (NX * d[0] + NY * d[1]))) < 1e-10


def test_p3_propagate_back_by_depth_gives_in_focus_gaussian():
    grid = Grid(128, 96, 8e-6, 8e-6, (638e-9, 520e-9))
    sxx, sxy, syy = cov_from(4.0, 6.0, 0.3, 8e-6)
    z = 4e-3
    at_z = one_gaussian(-1e-4, 5e-5, z, sxx, sxy, syy, o=0.9, a=(0.6, 1.0), phi=0.4)
    at_0 = at_z.copy()
    at_0.depth[:] = 0.0
    u_z, u_0 = oracle.forward(at_z, grid), oracle.forward(at_0, grid)
    for c, lam in enumerate(grid.lambdas):
        assert oracle.rel_l2(asm_propagate(u_z[c], grid, lam, +z), u_0[c]) < 1e-10
        assert oracle.rel_l2(asm_propagate(asm_propagate(u_z[c], grid, lam, z), grid, lam, -z), u_z[c]) < 1e-10
    # the field at the SLM of a Gaussian at depth z is not the in-focus one
    assert oracle.rel_l2(u_z[0], u_0[0]) > 0.1


def test_p4_parseval_and_closed_form_energy():
    grid = Grid(160, 128, 8e-6, 8e-6, (520e-9,))
    sxx, sxy, syy = cov_from(3.0, 4.5, 2.0, 8e-6)
    scene = one_gaussian(2e-5, 1e-5, -6e-3, sxx, sxy, syy, o=0.6, a=(0.8,), phi=2.0)
    U = oracle.spectrum(scene, grid)
    u = oracle.forward(scene, grid)
    e_space = np.sum(np.abs(u) ** 2) * grid.px * grid.py
    e_freq = np.sum(np.abs(U) ** 2) / (grid.nx * grid.px * grid.ny * grid.py)
    assert abs(e_space / e_freq - 1) < 1e-12
    det = sxx * syy - sxy * sxy
    closed = (0.6 * 0.8) ** 2 * math.pi * math.sqrt(det)
    assert abs(e_space / closed - 1) < 1e-12


def test_p5_zero_opacity_and_zero_amplitude_contribute_nothing():
    s, g = gwsgen.workload("small")
    s = s.subset(np.arange(12))
    g = Grid(64, 64, g.px, g.py, (520e-9, 638e-9))
    s.amplitude = np.vstack([s.amplitude, s.amplitude[::-1] * 0.5]).astype(np.float32)
    u = oracle.forward(s, g)
    extra = s.subset(np.concatenate([np.arange(12), [3, 5]]))
    extra.opacity[12] = 0.0
    extra.amplitude[:, 13] = 0.0
    u2 = oracle.forward(extra, g)
    assert np.array_equal(u, u2)


def test_p6_fresnel_gaussian_beam_closed_form():
    """An isotropic Gaussian at depth z reaches the SLM as a Gaussian beam propagated by -z."""
    grid = Grid(256, 256, 8e-6, 8e-6, (520e-9,))
    lam, sig, z = 520e-9, 10 * 8e-6, 3e-3
    scene = one_gaussian(0.0, 0.0, z, sig ** 2, 0.0, sig ** 2, o=0.5, a=(0.8,), phi=0.3)
    u = oracle.forward(scene, grid)[0]
    x = (np.arange(grid.nx) - grid.nx // 2) * grid.px
    X, Y = np.meshgrid(x, x)
    Q = sig ** 2 - 1j * lam * z / (2 * math.pi)
    ref = 0.4 * np.exp(1j * 0.3) * np.exp(-2j * math.pi * z / lam) * (sig ** 2 / Q) * np.exp(-(X ** 2 + Y ** 2) / (2 * Q))
    assert oracle.rel_l2(u, ref) < 1e-7
    # the opposite propagation sign is far off
    ref_wrong = np.conj(ref * np.exp(-1j * 0.3)) * np.exp(1j * 0.3)
    assert oracle.rel_l2(u, ref_wrong) > 1e-2


def test_p7_superposition_scaling_and_permutation():
    s, g = gwsgen.workload("small")
    s = s.subset(np.arange(10))
    g = Grid(64, 48, g.px, g.py, (520e-9,))
    a, b = s.subset(np.arange(6)), s.subset(np.arange(6, 10))
    u, ua, ub = oracle.forward(s, g), oracle.forward(a, g), oracle.forward(b, g)
    assert oracle.rel_l2(ua + ub, u) < 1e-11
    perm = np.random.default_rng(1).permutation(10)
    assert oracle.rel_l2(oracle.forward(s.subset(perm), g), u) < 1e-11
    # amplitude and phase act linearly
    t = s.copy().subset(np.arange(10))
    t.amplitude = (t.amplitude.astype(np.float64) * 2.0)
    t.phase = t.phase.astype(np.float64) + 0.5
    assert oracle.rel_l2(oracle.forward(t, g), 2.0 * np.exp(0.5j) * u) < 1e-11


def test_p9_transform_identities():
    grid = Grid(30, 20, 8e-6, 5e-6, (520e-9,))
    # delta in the spectrum -> plane wave with the documented centring
    U = np.zeros((1, grid.ny, grid.nx), dtype=np.complex128)
    U[0, 3, grid.nx - 4] = 1.0  # m_y' = 3, m_x' = -4
    u = oracle.field_from_spectrum(U, grid)[0]
    n_x = np.arange(grid.nx) - grid.nx // 2
    n_y = np.arange(grid.ny) - grid.ny // 2
    plane = np.exp(2j * math.pi * (np.outer(3 * n_y, np.ones(grid.nx)) / grid.ny - 4 * n_x[None, :] / grid.nx))
    assert np.max(np.abs(u * grid.nx * grid.ny * grid.px * grid.py - plane)) < 1e-12
    # agrees with numpy's FFT with explicit shifts
    rng = np.random.default_rng(3)
    U = rng.standard_normal((2, grid.ny, grid.nx)) + 1j * rng.standard_normal((2, grid.ny, grid.nx))
    g2 = Grid(30, 20, 8e-6, 5e-6, (520e-9, 450e-9))
    u = oracle.field_from_spectrum(U, g2)
    ref = np.fft.fftshift(np.fft.ifft2(U), axes=(1, 2)) / (g2.px * g2.py)
    assert oracle.rel_l2(u, ref) < 1e-13
    # the adjoint is the conjugate transpose: <A x, y> = <x, A^H y>
    G = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    lhs = np.vdot(G, oracle.field_from_spectrum(U, g2))
    rhs = np.vdot(oracle.spectrum_grad_from_field_grad(G, g2), U)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _single_fields(scene, grid):
    return [oracle.forward(scene.subset([i]), grid) for i in range(scene.n)]


def test_p10_gradients_match_central_differences():
    rng = np.random.default_rng(11)
    grid = Grid(48, 40, 8e-6, 8e-6, (638e-9, 450e-9))
    n = 3
    sxx, sxy, syy = zip(*[cov_from(rng.uniform(2.5, 5), rng.uniform(2.5, 5), rng.uniform(0, math.pi), 8e-6)
                          for _ in range(n)])
    scene = Scene(mean_x=rng.uniform(-0.2, 0.2, n) * grid.nx * grid.px, mean_y=rng.uniform(-0.2, 0.2, n) * grid.ny * grid.py,
                  depth=rng.uniform(-3e-3, 3e-3, n), cov_xx=np.array(sxx), cov_xy=np.array(sxy), cov_yy=np.array(syy),
                  opacity=rng.uniform(0.2, 1, n), amplitude=rng.uniform(0.2, 1, (2, n)), phase=rng.uniform(0, 6, n))
    target = gwsgen.make_target(grid, 99).astype(np.complex128) * 0.05
    fields = _single_fields(scene, grid)
    u = sum(fields)
    _, G = oracle.loss_and_field_grad(u, target)
    grads = oracle.backward(scene, grid, G)

    def loss_with(i, name, c, value):
        s = scene.subset([i])
        if name == "amplitude":
            s.amplitude[c, 0] = value
        else:
            getattr(s, name)[0] = value
        ui = oracle.forward(s, grid)
        return oracle.loss_and_field_grad(u - fields[i] + ui, target)[0]

    for i in range(n):
        for name in ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity", "phase", "amplitude"):
            for c in (range(grid.n_lambda) if name == "amplitude" else [0]):
                v = float(scene.amplitude[c, i]) if name == "amplitude" else float(getattr(scene, name)[i])
                # depth moves the phase by 2 pi / lambda ~ 1e7 rad per metre: keep k h small
                scale = {"mean_x": 8e-6, "mean_y": 8e-6, "depth": 1e-5}.get(name, abs(v) if v != 0 else 1.0)
                # fourth-order central difference: truncation ~ (k h)^4, while a larger h keeps
                # the ~1e-11 rad FP64 rounding noise of the large propagation phase negligible
                h = 1e-4 * scale
                fd = (8 * (loss_with(i, name, c, v + h) - loss_with(i, name, c, v - h))
                      - (loss_with(i, name, c, v + 2 * h) - loss_with(i, name, c, v - 2 * h))) / (12 * h)
                an = grads[name][c, i] if name == "amplitude" else grads[name][i]
                assert abs(fd - an) <= 1e-6 * abs(an), (i, name, c, fd, an)


def test_p11_evanescent_band_is_zero():
    """Eq. 4: H vanishes for |nu| >= 1/lambda; at a 0.2 um pitch the grid reaches past it."""
    grid = Grid(32, 32, 2e-7, 2e-7, (520e-9,))
    sxx, sxy, syy = cov_from(1.0, 1.0, 0.0, 2e-7)
    scene = one_gaussian(0.0, 0.0, 1e-6, sxx, sxy, syy)
    U = oracle.spectrum(scene, grid)[0]
    NX, NY = freq_grid(grid)
    outside = NX ** 2 + NY ** 2 >= (1 / 520e-9) ** 2
    assert outside.sum() > 100 and (~outside).sum() > 100
    assert np.all(U[outside] == 0)
    assert np.all(np.abs(U[~outside]) > 0)


def test_oracle_matches_its_committed_checksums():
    """Regression of the oracle against values it wrote itself (tests/golden/make_golden.py)."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "small_field_checksums.json")))
    scene, grid = gwsgen.workload("small")
    u = oracle.forward(scene, grid)[0]
    assert abs(np.linalg.norm(u) / ref["norm_l2"] - 1) < 1e-12
    for k, (re, im) in ref["pixels"].items():
        iy, ix = map(int, k.split(","))
        assert abs(u[iy, ix] - complex(re, im)) < 1e-12 * ref["norm_l2"]


# ---- the reference plane wave (Sec. 4.1): every Gaussian is illuminated by a plane wave of
# transverse frequency nu_r, which shifts its angular spectrum by nu_r; the transfer function
# H keeps the full frequency.  Pinned by spatial sampling, the modulation theorem and the
# tilted Gaussian-beam closed form.


def _lattice_ref(grid, sx, sy):
    return (sx / (grid.nx * grid.px), sy / (grid.ny * grid.py))


def test_r1_reference_wave_brute_force():
    """Spatial samples times exp(j 2 pi nu_r.x) -> numpy FFT -> H(nu, -z) -> inverse FFT."""
    rng = np.random.default_rng(17)
    for (nx, ny, sx, sy) in [(64, 48, 3, -2), (40, 56, -5, 4)]:
        base = Grid(nx, ny, 8e-6, 6e-6, (638e-9, 450e-9))
        grid = Grid(nx, ny, 8e-6, 6e-6, (638e-9, 450e-9), ref_nu=_lattice_ref(base, sx, sy))
        n = 3
        sxx, sxy, syy = zip(*[cov_from(rng.uniform(2.5, 5), rng.uniform(2.5, 5), rng.uniform(0, math.pi), 7e-6)
                              for _ in range(n)])
        scene = Scene(mean_x=rng.uniform(-0.3, 0.3, n) * nx * grid.px, mean_y=rng.uniform(-0.3, 0.3, n) * ny * grid.py,
                      depth=rng.uniform(-3e-3, 3e-3, n), cov_xx=np.array(sxx), cov_xy=np.array(sxy),
                      cov_yy=np.array(syy), opacity=rng.uniform(0.1, 1, n), amplitude=rng.uniform(0, 1, (2, n)),
                      phase=rng.uniform(0, 2 * math.pi, n))
        u = oracle.forward(scene, grid)
        ref = brute_force_field(scene, grid)
        assert oracle.rel_l2(u, ref) < 1e-9, (nx, ny, oracle.rel_l2(u, ref))
        # and it is not the on-axis field
        assert oracle.rel_l2(u, oracle.forward(scene, base)) > 0.5


def test_r2_reference_wave_at_zero_depth_is_modulation():
    """z = 0: the field is the on-axis field times the plane wave exp(j 2 pi nu_r.x_n)."""
    base = Grid(96, 80, 8e-6, 8e-6, (520e-9, 638e-9))
    grid = Grid(96, 80, 8e-6, 8e-6, (520e-9, 638e-9), ref_nu=_lattice_ref(base, 7, -4))
    sxx, sxy, syy = cov_from(4.0, 2.5, 0.6, 8e-6)
    scene = one_gaussian(3.3e-5, -2.1e-5, 0.0, sxx, sxy, syy, o=0.7, a=(0.5, 0.9), phi=0.8)
    x = (np.arange(grid.nx) - grid.nx // 2) * grid.px
    y = (np.arange(grid.ny) - grid.ny // 2) * grid.py
    X, Y = np.meshgrid(x, y)
    plane = np.exp(2j * math.pi * (grid.ref_nu[0] * X + grid.ref_nu[1] * Y))
    assert oracle.rel_l2(oracle.forward(scene, grid), oracle.forward(scene, base) * plane) < 1e-12


def test_r3_reference_wave_tilted_gaussian_beam():
    """Fresnel closed form of a tilted Gaussian beam: an isotropic Gaussian at depth z under a
    plane wave of transverse frequency nu_r reaches the SLM as
    exp(j 2 pi nu_r.x) exp(j pi lambda z |nu_r|^2) u_0(x + lambda z nu_r),
    u_0 the on-axis beam (the walk-off lambda z nu_r is the beam travelling along the tilt)."""
    base = Grid(256, 256, 8e-6, 8e-6, (520e-9,))
    grid = Grid(256, 256, 8e-6, 8e-6, (520e-9,), ref_nu=_lattice_ref(base, 5, -3))
    lam, sig, z = 520e-9, 10 * 8e-6, 3e-3
    rx, ry = grid.ref_nu
    scene = one_gaussian(0.0, 0.0, z, sig ** 2, 0.0, sig ** 2, o=0.5, a=(0.8,), phi=0.3)
    u = oracle.forward(scene, grid)[0]
    x = (np.arange(grid.nx) - grid.nx // 2) * grid.px
    X, Y = np.meshgrid(x, x)
    Q = sig ** 2 - 1j * lam * z / (2 * math.pi)

    def beam(x0, y0):
        return (0.4 * np.exp(1j * 0.3) * np.exp(-2j * math.pi * z / lam) * (sig ** 2 / Q)
                * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * Q)))

    tilt = np.exp(2j * math.pi * (rx * X + ry * Y)) * np.exp(1j * math.pi * lam * z * (rx * rx + ry * ry))
    ref = tilt * beam(-lam * z * rx, -lam * z * ry)
    assert oracle.rel_l2(u, ref) < 5e-7  # non-paraxial residual ~1.4e-7 at this tilt and depth
    # walk-off the other way, or none (the transfer function shifted with the spectrum), are far off
    assert oracle.rel_l2(u, tilt * beam(lam * z * rx, lam * z * ry)) > 1e-2
    assert oracle.rel_l2(u, np.exp(2j * math.pi * (rx * X + ry * Y)) * beam(0.0, 0.0)) > 1e-2


def test_r4_reference_wave_gradients_match_central_differences():
    rng = np.random.default_rng(23)
    base = Grid(48, 40, 8e-6, 8e-6, (638e-9, 450e-9))
    grid = Grid(48, 40, 8e-6, 8e-6, (638e-9, 450e-9), ref_nu=(2.7 / (48 * 8e-6), -1.9 / (40 * 8e-6)))
    n = 2
    sxx, sxy, syy = zip(*[cov_from(rng.uniform(2.5, 5), rng.uniform(2.5, 5), rng.uniform(0, math.pi), 8e-6)
                          for _ in range(n)])
    scene = Scene(mean_x=rng.uniform(-0.2, 0.2, n) * grid.nx * grid.px, mean_y=rng.uniform(-0.2, 0.2, n) * grid.ny * grid.py,
                  depth=rng.uniform(-3e-3, 3e-3, n), cov_xx=np.array(sxx), cov_xy=np.array(sxy), cov_yy=np.array(syy),
                  opacity=rng.uniform(0.2, 1, n), amplitude=rng.uniform(0.2, 1, (2, n)), phase=rng.uniform(0, 6, n))
    target = gwsgen.make_target(base, 98).astype(np.complex128) * 0.05
    fields = _single_fields(scene, grid)
    u = sum(fields)
    _, G = oracle.loss_and_field_grad(u, target)
    grads = oracle.backward(scene, grid, G)

    def loss_with(i, name, value):
        s = scene.subset([i])
        getattr(s, name)[0] = value
        return oracle.loss_and_field_grad(u - fields[i] + oracle.forward(s, grid), target)[0]

    for i in range(n):
        for name in ("mean_x", "mean_y", "cov_xx", "cov_xy", "cov_yy", "depth"):
            v = float(getattr(scene, name)[i])
            scale = {"mean_x": 8e-6, "mean_y": 8e-6, "depth": 1e-5}.get(name, abs(v))
            h = 1e-4 * scale
            fd = (8 * (loss_with(i, name, v + h) - loss_with(i, name, v - h))
                  - (loss_with(i, name, v + 2 * h) - loss_with(i, name, v - 2 * h))) / (12 * h)
            an = grads[name][i]
            assert abs(fd - an) <= 1e-6 * abs(an), (i, name, fd, an)
