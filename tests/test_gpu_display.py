"""GPU parity of the display-side entry points -- double-phase amplitude coding and
angular-spectrum focal stacks -- through the C ABI against the FP64 oracle in
oracle/display.py, on seeded fields."""
import math
import sys

import numpy as np
import pytest

import gwsgen
import oracle
import oracle.display as dp
from gwsgen import Grid
from gpu_util import problem, rel_l2, scene_to_torch, to_numpy

pytestmark = pytest.mark.gpu

# Focal-stack planes in FP32 (FFT of the field, FP32 product with H whose phase is reduced in
# FP64, FP32 inverse FFT): relative L2 per plane, the same bar as the hologram itself.
TOL_FIELD = 1e-5
# Double-phase coding: atan2 and the |u| / a_max ratio in FP32 contribute a few ulp; arccos
# amplifies an error dr of the ratio by 1 / sqrt(1 - r^2) (unbounded at r = 1), so each phase is
# held to 2e-6 rad plus what a ratio error of DR does to arccos at that pixel.
TOL_PHASE = 2e-6
DR = 1e-6


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def phase_bound(u, a_max=None):
    """Per-pixel tolerance of a double phase: TOL_PHASE + the change of arccos(r) under a
    ratio error of DR."""
    a = np.abs(u.astype(np.complex128))
    am = dp.channel_amax(u) if a_max is None else np.full(u.shape[0], float(a_max))
    r = np.clip(a / np.where(am > 0, am, 1.0)[:, None, None], 0.0, 1.0)
    r = np.where((am > 0)[:, None, None], r, 0.0)
    t = np.arccos(r)
    dev = np.maximum(np.abs(np.arccos(np.clip(r + DR, 0, 1)) - t), np.abs(np.arccos(np.clip(r - DR, 0, 1)) - t))
    return TOL_PHASE + dev


@pytest.mark.parametrize("nx,ny,lams,seed,a_max", [
    (96, 64, (638e-9, 520e-9), 3101, None),
    (251, 129, gwsgen.RGB, 3102, None),               # odd row and column counts for the checkerboard
    (64, 48, (520e-9,), 3103, 5.0),                   # a_max above every amplitude
    (64, 48, (520e-9,), 3104, 0.5),                   # a_max below most amplitudes: ratios clip to 1
])
def test_dpac_matches_oracle(ctx, nx, ny, lams, seed, a_max):
    g = Grid(nx, ny, 8e-6, 8e-6, lams)
    log("dpac %dx%dx%d a_max=%s" % (nx, ny, len(lams), a_max))
    u = gwsgen.make_target(g, seed)
    got = to_numpy(ctx.dpac_encode(cuda(u), a_max=a_max)).astype(np.float64)
    ref = dp.dpac_encode(u.astype(np.complex128), a_max=a_max)
    err = dp.phase_distance(got, ref)
    bound = phase_bound(u, a_max)
    log("  max phase error %.3g rad, worst error/bound %.3g" % (err.max(), (err / bound).max()))
    assert np.all(err <= bound)
    if a_max is None:
        # each channel's peak pixel has ratio exactly 1: both phases equal arg u
        for c in range(len(lams)):
            i = np.unravel_index(np.argmax(np.abs(u[c])), u[c].shape)
            assert dp.phase_distance(got[c][i], np.angle(u[c][i].astype(np.complex128))) < TOL_PHASE


def test_dpac_zero_field(ctx):
    u = np.zeros((2, 32, 48), dtype=np.complex64)
    got = to_numpy(ctx.dpac_encode(cuda(u)))
    even = dp.checkerboard(32, 48)
    want = np.where(even, -math.pi / 2, math.pi / 2)
    assert np.max(np.abs(got - want[None])) < 1e-6


@pytest.mark.parametrize("nx,ny,lams,depths,flags,seed", [
    (96, 64, (638e-9, 520e-9), (-4e-3, 0.0, 2.5e-3, 1e-2), "", 3201),
    (240, 200, (450e-9,), (5e-2, -3e-2), "complex", 3202),                  # |z| / lambda ~ 1e5 rev
    (120, 80, gwsgen.RGB, (1e-3, -7e-3), "phase half_band", 3203),
    (64, 48, (520e-9,), tuple(np.linspace(-2e-2, 2e-2, 40)), "", 3204),    # two launches of planes
])
def test_focal_stack_matches_oracle(ctx, nx, ny, lams, depths, flags, seed):
    g = Grid(nx, ny, 8e-6, 8e-6, lams)
    log("focal stack %dx%dx%d planes=%d flags=%r" % (nx, ny, len(lams), len(depths), flags))
    phase_in = "phase" in flags
    if phase_in:
        rng = np.random.default_rng(seed)
        inp = rng.uniform(-2 * math.pi, 2 * math.pi, (len(lams), ny, nx)).astype(np.float32)
    else:
        inp = gwsgen.make_target(g, seed)
    got = to_numpy(ctx.focal_stack(problem(g), cuda(inp), depths, phase_input=phase_in,
                                   half_band="half_band" in flags, complex_output="complex" in flags))
    ref = dp.focal_stack(inp, g, depths, phase_input=phase_in, half_band="half_band" in flags,
                         complex_output="complex" in flags)
    assert got.shape == ref.shape
    worst = max(rel_l2(got[k], ref[k]) for k in range(len(depths)))
    log("  worst plane rel L2 %.3g" % worst)
    assert worst < TOL_FIELD


def test_focal_stack_full_size(ctx):
    g = Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    depths = (-1e-2, 0.0, 3e-3, 2e-2)
    log("focal stack 1080x1920x3, 4 planes")
    u = gwsgen.make_target(g, 3301)
    got = to_numpy(ctx.focal_stack(problem(g), cuda(u), depths))
    ref = dp.focal_stack(u, g, depths)
    worst = max(rel_l2(got[k], ref[k]) for k in range(len(depths)))
    log("  worst plane rel L2 %.3g" % worst)
    assert worst < TOL_FIELD


def test_gpu_hologram_refocuses_in_its_plane(ctx):
    """The library's hologram of Gaussians at one depth z0, taken by the library's focal stack
    to z0, is the oracle's hologram of the same Gaussians at depth 0."""
    g = Grid(128, 96, 8e-6, 8e-6, (638e-9, 450e-9))
    s = gwsgen.make_scene(16, g, 3401)
    z0 = np.float32(4e-3)
    s.depth[:] = z0
    s0 = s.copy()
    s0.depth[:] = 0.0
    u = ctx.forward(problem(g), scene_to_torch(s))
    got = to_numpy(ctx.focal_stack(problem(g), u, [float(z0)], complex_output=True))[0]
    err = rel_l2(got, oracle.forward(s0, g))
    log("refocus rel L2 %.3g" % err)
    assert err < TOL_FIELD


def test_dpac_then_filtered_focal_stack(ctx):
    """The whole display chain on the GPU (coding, e^{jP}, half-band filter, propagation)
    against the oracle's chain from the same seeded field."""
    g = Grid(160, 120, 8e-6, 8e-6, gwsgen.RGB)
    s = gwsgen.make_scene(24, g, 3501)
    u = oracle.forward(s, g).astype(np.complex64)
    depths = (float(np.float32(2e-3)), -1e-3)
    P = ctx.dpac_encode(cuda(u))
    got = to_numpy(ctx.focal_stack(problem(g), P, depths, phase_input=True, half_band=True))
    ref = dp.focal_stack(dp.dpac_encode(u.astype(np.complex128)), g, depths, phase_input=True, half_band=True)
    worst = max(rel_l2(got[k], ref[k]) for k in range(len(depths)))
    log("dpac + filtered focal stack worst rel L2 %.3g" % worst)
    assert worst < TOL_FIELD


def test_focal_stack_no_planes_and_bad_width(ctx):
    import paper_2505_06582_amd as gws
    g = Grid(64, 48, 8e-6, 8e-6, (520e-9,))
    u = cuda(gwsgen.make_target(g, 3601))
    assert ctx.focal_stack(problem(g), u, []).shape == (0, 1, 48, 64)
    wide = Grid(5000, 16, 8e-6, 8e-6, (520e-9,))
    with pytest.raises(gws.GwsError):  # the library's width limit (GWS_ERR_SHAPE), not the binding's checks
        ctx.focal_stack(problem(wide), cuda(gwsgen.make_target(wide, 3602)), [0.0])


def test_four_wavelengths(ctx):
    """The display calls take up to four wavelengths (the problem's maximum)."""
    lams = (638e-9, 560e-9, 520e-9, 450e-9)
    g = Grid(80, 64, 8e-6, 8e-6, lams)
    u = gwsgen.make_target(g, 3701)
    got = to_numpy(ctx.dpac_encode(cuda(u))).astype(np.float64)
    assert np.all(dp.phase_distance(got, dp.dpac_encode(u.astype(np.complex128))) <= phase_bound(u))
    depths = (3e-3, -6e-3)
    st = to_numpy(ctx.focal_stack(problem(g), cuda(u), depths))
    ref = dp.focal_stack(u, g, depths)
    worst = max(rel_l2(st[k], ref[k]) for k in range(len(depths)))
    log("four wavelengths: focal stack worst rel L2 %.3g" % worst)
    assert worst < TOL_FIELD
