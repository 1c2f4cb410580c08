"""Pins of the display oracle (oracle/display.py): double-phase amplitude coding and
angular-spectrum focal stacks.

Each compares the oracle with something it does not compute itself:
  * the two double phases average back to the field (a trigonometric identity the encoding
    must satisfy, checked by summing phasors);
  * a uniform field's interlaced pattern has exactly two spectral lines, at DC and at the
    Nyquist corner, with closed-form values;
  * the half-band filter passes a band-limited field unchanged and removes it once it is
    moved to the Nyquist corner;
  * propagation by d then -d is the identity, keeps the energy of every plane, and matches
    the Fresnel closed form of a Gaussian beam;
  * the focal plane at depth z of a hologram made (by the order-invariant oracle) from
    Gaussians at depth z equals the hologram of the same Gaussians at depth 0.
"""
import math

import numpy as np

import gwsgen
import oracle
import oracle.display as dp
from gwsgen import Grid

GRID = Grid(96, 64, 8e-6, 8e-6, (638e-9, 520e-9))


def random_field(grid, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    shape = (grid.n_lambda, grid.ny, grid.nx)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def test_double_phases_average_to_the_field():
    u = random_field(GRID, 1)
    pm, pp = dp.dpac_phases(u)
    am = dp.channel_amax(u)
    rec = am[:, None, None] * 0.5 * (np.exp(1j * pm) + np.exp(1j * pp))
    assert np.max(np.abs(rec - u)) < 1e-13 * np.max(np.abs(u))
    # with an a_max above every amplitude the identity still holds
    pm, pp = dp.dpac_phases(u, a_max=3.0 * am.max())
    rec = 3.0 * am.max() * 0.5 * (np.exp(1j * pm) + np.exp(1j * pp))
    assert np.max(np.abs(rec - u)) < 1e-13 * np.max(np.abs(u))


def test_uniform_field_has_two_spectral_lines():
    g = Grid(32, 24, 8e-6, 8e-6, (520e-9,))
    r, phi, amax = 0.37, 1.1, 2.0
    u = np.full((1, g.ny, g.nx), r * amax * np.exp(1j * phi))
    P = dp.dpac_encode(u, a_max=amax)
    S = np.fft.fft2(np.exp(1j * P[0]))
    M = g.nx * g.ny
    dc = M * r * np.exp(1j * phi)
    # e^{jP} = e^{j phi} (cos t - j sin t (-1)^(x+y)), t = arccos r: the corner line is
    # -j M e^{j phi} sqrt(1 - r^2) with P- on the even pixels
    corner = -1j * M * np.exp(1j * phi) * math.sqrt(1.0 - r * r)
    assert abs(S[0, 0] - dc) < 1e-11 * M
    assert abs(S[g.ny // 2, g.nx // 2] - corner) < 1e-11 * M
    S[0, 0] = 0.0
    S[g.ny // 2, g.nx // 2] = 0.0
    assert np.max(np.abs(S)) < 1e-11 * M


def test_full_amplitude_pixel_gets_equal_phases():
    u = random_field(GRID, 2)
    pm, pp = dp.dpac_phases(u)
    for c in range(GRID.n_lambda):
        i = np.unravel_index(np.argmax(np.abs(u[c])), u[c].shape)
        assert abs(pm[c][i] - pp[c][i]) < 1e-7      # arccos(1) = 0 up to the rounding of |u| / max |u|
        assert abs(pm[c][i] - np.angle(u[c][i])) < 1e-7


def test_filter_passes_band_limited_field_and_removes_the_corner():
    u = random_field(GRID, 3)
    spec = np.fft.fft2(u, axes=(-2, -1))
    mx = np.abs(np.fft.fftfreq(GRID.nx) * GRID.nx) * 4 < GRID.nx
    my = np.abs(np.fft.fftfreq(GRID.ny) * GRID.ny) * 4 < GRID.ny
    spec *= (my[:, None] & mx[None, :])
    bl = np.fft.ifft2(spec, axes=(-2, -1))
    out = dp.propagate(bl, GRID, 0.0, half_band=True)
    assert oracle.rel_l2(out, bl) < 1e-14
    # (-1)^(n_x + n_y), (-1)^n_x and (-1)^n_y move the band by half the grid along both
    # axes, along x and along y: every copy lies outside the filter
    sx = (-1.0) ** np.arange(GRID.nx)
    sy = (-1.0) ** np.arange(GRID.ny)
    for sign in (np.where(dp.checkerboard(GRID.ny, GRID.nx), 1.0, -1.0), np.outer(np.ones(GRID.ny), sx),
                 np.outer(sy, np.ones(GRID.nx))):
        out = dp.propagate(bl * sign[None], GRID, 0.0, half_band=True)
        assert np.max(np.abs(out)) < 1e-14 * np.max(np.abs(bl))


def test_filtered_dpac_of_uniform_field_is_the_field():
    g = Grid(32, 24, 8e-6, 8e-6, (520e-9,))
    u = np.full((1, g.ny, g.nx), 0.6 * np.exp(-0.4j))
    P = dp.dpac_encode(u, a_max=1.0)
    st = dp.focal_stack(P, g, [0.0], phase_input=True, half_band=True, complex_output=True)
    assert np.max(np.abs(st[0] - u)) < 1e-14


def test_propagation_round_trip_and_energy():
    u = random_field(GRID, 4)
    for d in (1e-3, -4e-3, 2.5e-2):
        v = dp.propagate(u, GRID, d)
        assert oracle.rel_l2(dp.propagate(v, GRID, -d), u) < 1e-12
        st = dp.focal_stack(u, GRID, [d])
        e0 = np.sum(np.abs(u) ** 2, axis=(-2, -1))
        assert np.max(np.abs(np.sum(st[0], axis=(-2, -1)) - e0) / e0) < 1e-12


def test_gaussian_beam_closed_form():
    # isotropic sigma = 8 px on a 256 px field (32 sigma): wrap and aliasing are negligible,
    # and the non-paraxial phase at the spectral width is ~1e-8 rad
    g = Grid(256, 256, 8e-6, 8e-6, (520e-9,))
    sig = 8 * 8e-6
    x = (np.arange(g.nx) - g.nx // 2) * g.px
    y = (np.arange(g.ny) - g.ny // 2) * g.py
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    u0 = np.exp(-r2 / (2 * sig * sig))[None].astype(np.complex128)
    lam = g.lambdas[0]
    for d in (3e-3, -2e-3):
        Q = sig * sig + 1j * lam * d / (2 * math.pi)
        ref = np.exp(2j * math.pi * math.fmod(d / lam, 1.0)) * (sig * sig / Q) * np.exp(-r2 / (2 * Q))
        got = dp.focal_stack(u0, g, [d], complex_output=True)[0, 0]
        assert oracle.rel_l2(got, ref) < 1e-7


def test_focal_plane_refocuses_the_gaussian_hologram():
    g = Grid(128, 96, 8e-6, 8e-6, (638e-9, 450e-9))
    s0 = gwsgen.make_scene(12, g, 31)
    s0.depth[:] = 0.0
    z0 = 4e-3
    s1 = s0.copy()
    s1.depth[:] = np.float32(z0)
    u0 = oracle.forward(s0, g)
    u1 = oracle.forward(s1, g)
    st = dp.focal_stack(u1, g, [float(np.float32(z0)), 0.0], complex_output=True)
    assert oracle.rel_l2(st[0], u0) < 1e-10
    assert oracle.rel_l2(st[1], u1) < 1e-13


def test_phase_input_is_the_unit_phasor_field():
    rng = np.random.default_rng(5)
    P = rng.uniform(-2 * math.pi, 2 * math.pi, (GRID.n_lambda, GRID.ny, GRID.nx))
    a = dp.focal_stack(P, GRID, [1e-3, -1e-3], phase_input=True, half_band=True)
    b = dp.focal_stack(np.exp(1j * P), GRID, [1e-3, -1e-3], half_band=True)
    assert oracle.rel_l2(a, b) < 1e-14
    # a phase-only field carries unit intensity in the plane of the SLM
    c = dp.focal_stack(P, GRID, [0.0], phase_input=True)
    assert np.max(np.abs(c - 1.0)) < 1e-12


def test_zero_field_and_empty_stack():
    u = np.zeros((2, 8, 8), dtype=np.complex128)
    pm, pp = dp.dpac_phases(u)
    assert np.all(pm == -math.pi / 2) and np.all(pp == math.pi / 2)
    g = Grid(8, 8, 8e-6, 8e-6, (638e-9, 520e-9))
    assert dp.focal_stack(u, g, []).shape == (0, 2, 8, 8)
