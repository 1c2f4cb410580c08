"""GPU parity of the forward path (through the C ABI) against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

import gwsgen
import oracle
from gwsgen import Grid
from gpu_util import dft_ready, problem, rel_l2, scene_to_torch, to_numpy

pytestmark = pytest.mark.gpu

# FP32 forward tolerance: relative L2 of the field against FP64 (the hot path's stated bound)
TOL_FWD = 1e-5


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# Row lengths cover every elements-per-thread bound of the row pass (<= 512, 1024, 2048, 4096,
# 8192) and column lengths both LDS budgets of the column pass (80 KB slabs of 8..4 columns,
# 160 KB slabs down to one column at 8000).
@pytest.mark.parametrize("ny,nx,batch", [(256, 256, 1), (40, 48, 2), (1080, 1920, 3), (90, 160, 1), (1000, 1000, 1),
                                         (2160, 3840, 1), (16, 8000, 2), (8000, 16, 1)])
def test_fft_matches_numpy_both_directions(ctx, ny, nx, batch):
    import torch
    log("fft %dx%d batch %d" % (ny, nx, batch))
    g = Grid(nx, ny, 8e-6, 8e-6, (520e-9,) * batch)
    x = gwsgen.make_target(g, 77)
    xt = torch.from_numpy(x).cuda()
    inv = to_numpy(ctx.dft2d(xt, +1))
    fwd = to_numpy(ctx.dft2d(xt, -1))
    xd = x.astype(np.complex128)
    assert rel_l2(inv, np.fft.ifft2(xd) * (nx * ny)) < 2e-6
    assert rel_l2(fwd, np.fft.fft2(xd)) < 2e-6


def _sizes_235(lo, hi):
    out = []
    for n in range(lo, hi + 1, 2):
        m = n
        for f in (2, 3, 5):
            while m % f == 0:
                m //= f
        if m == 1:
            out.append(n)
    return out


def test_fft_every_length(ctx):
    """Every even length 16..8192 with factors 2, 3, 5 as a row length and as a column length:
    each radix order and each LDS layout the plans choose, in both directions."""
    import torch
    sizes = _sizes_235(16, 8192)
    worst = 0.0
    for n in sizes:
        for ny, nx in ((16, n), (n, 16)):
            x = gwsgen.make_target(Grid(nx, ny, 8e-6, 8e-6, (520e-9,)), 1000 + n)
            xt = torch.from_numpy(x).cuda()
            xd = x.astype(np.complex128)
            e1 = rel_l2(to_numpy(ctx.dft2d(xt, +1)), np.fft.ifft2(xd) * (nx * ny))
            e2 = rel_l2(to_numpy(ctx.dft2d(xt, -1)), np.fft.fft2(xd))
            worst = max(worst, e1, e2)
            assert e1 < 2e-6 and e2 < 2e-6, (ny, nx, e1, e2)
    log("fft: %d lengths as rows and columns, worst rel L2 %.3g" % (len(sizes), worst))


def run_forward(ctx, scene, grid, **kw):
    f, s = ctx.forward(problem(grid, **kw), scene_to_torch(scene), want_spectrum=True)
    return to_numpy(f), to_numpy(s)


def test_forward_small_workload(ctx):
    log("forward small")
    scene, grid = gwsgen.workload("small")
    field, spec = run_forward(ctx, scene, grid)
    ref = oracle.forward(scene, grid)
    U = oracle.spectrum(scene, grid)
    e_field, e_spec = rel_l2(field, ref), rel_l2(spec, dft_ready(U, grid))
    log("small: field rel %.3e spectrum rel %.3e" % (e_field, e_spec))
    assert e_spec < TOL_FWD
    assert e_field < TOL_FWD


@pytest.mark.parametrize("nx,ny,n,seed", [(96, 80, 300, 11), (160, 90, 500, 12), (48, 40, 40, 13)])
def test_forward_ragged_three_wavelengths(ctx, nx, ny, n, seed):
    log("forward ragged %dx%d n=%d" % (nx, ny, n))
    grid = Grid(nx, ny, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(n, grid, seed, depth_range=(-10e-3, 10e-3))
    field, spec = run_forward(ctx, scene, grid)
    ref = oracle.forward(scene, grid)
    e = rel_l2(field, ref)
    log("  rel %.3e" % e)
    assert e < TOL_FWD
    for c in range(3):
        assert rel_l2(field[c], ref[c]) < TOL_FWD


def test_forward_medium_many_tiles(ctx):
    log("forward medium")
    grid = Grid(480, 270, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(1500, grid, 21, depth_range=(-10e-3, 10e-3))
    field, spec = run_forward(ctx, scene, grid)
    ref = oracle.forward(scene, grid)
    e = rel_l2(field, ref)
    log("  rel %.3e" % e)
    assert e < TOL_FWD


def test_forward_empty_and_all_culled(ctx):
    import torch
    log("forward empty / culled")
    grid = Grid(64, 64, 8e-6, 8e-6, (520e-9, 638e-9))
    scene = gwsgen.make_scene(0, grid, 1)
    field, spec = run_forward(ctx, scene, grid)
    assert np.all(field == 0) and np.all(spec == 0)
    scene = gwsgen.make_scene(50, grid, 2)
    scene.opacity[:] = 0.0
    field, spec = run_forward(ctx, scene, grid)
    assert np.all(field == 0)
    st = ctx.stats()
    assert st["n_culled"] == 50


def test_forward_zero_opacity_gaussian_changes_nothing_bitwise(ctx):
    log("forward zero-opacity bitwise")
    grid = Grid(128, 96, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(120, grid, 5, depth_range=(-10e-3, 10e-3))
    extra = scene.subset(np.concatenate([np.arange(120), [7, 9]]))
    extra.opacity[120] = 0.0
    extra.amplitude[:, 121] = 0.0
    f1, _ = run_forward(ctx, scene, grid)
    f2, _ = run_forward(ctx, extra, grid)
    assert np.array_equal(f1, f2)


def test_forward_is_deterministic(ctx):
    log("forward determinism")
    scene, grid = gwsgen.workload("small")
    f1, _ = run_forward(ctx, scene, grid)
    f2, _ = run_forward(ctx, scene, grid)
    assert np.array_equal(f1, f2)


def test_forward_extreme_sizes_and_depths(ctx):
    """Very small and very large Gaussians, large depths and means outside the field."""
    log("forward extremes")
    grid = Grid(128, 128, 8e-6, 8e-6, (638e-9, 450e-9))
    s = gwsgen.make_scene(60, grid, 31, depth_range=(-50e-3, 50e-3), sigma_px=(0.7, 60.0))
    s.mean_x[:10] += np.float32(3 * grid.nx * grid.px)
    field, _ = run_forward(ctx, s, grid)
    ref = oracle.forward(s, grid)
    e = rel_l2(field, ref)
    log("  rel %.3e" % e)
    assert e < TOL_FWD


def test_forward_evanescent_band(ctx):
    """At a 0.25 um pitch part of the grid lies beyond 1/lambda: H = 0 there (Eq. 4)."""
    log("forward evanescent")
    grid = Grid(64, 64, 2.5e-7, 2.5e-7, (520e-9, 638e-9))
    s = gwsgen.make_scene(20, grid, 41, depth_range=(-2e-6, 2e-6), sigma_px=(1.0, 3.0))
    field, spec = run_forward(ctx, s, grid)
    ref = oracle.forward(s, grid)
    U = dft_ready(oracle.spectrum(s, grid), grid)
    assert np.all(spec[U == 0] == 0)
    assert rel_l2(field, ref) < TOL_FWD


# split-bf16 matrix-core DFT: each FP32 operand = bf16 hi + bf16 lo, three products per real
# product, FP32 accumulation; measured error against FP64 is ~1e-5 relative L2, asserted below 1e-4
TOL_BF16 = 1e-4


@pytest.mark.parametrize("ny,nx,batch", [(256, 256, 1), (40, 48, 2), (1080, 1920, 3)])
def test_dft_bf16x3_matches_numpy(ctx, ny, nx, batch):
    import torch
    import paper_2505_06582_amd as gws
    log("bf16x3 dft %dx%d batch %d" % (ny, nx, batch))
    g = Grid(nx, ny, 8e-6, 8e-6, (520e-9,) * batch)
    x = gwsgen.make_target(g, 78)
    xt = torch.from_numpy(x).cuda()
    inv = to_numpy(ctx.dft2d(xt, +1, xform=gws.XFORM_DFT_BF16X3))
    fwd = to_numpy(ctx.dft2d(xt, -1, xform=gws.XFORM_DFT_BF16X3))
    xd = x.astype(np.complex128)
    e_inv = rel_l2(inv, np.fft.ifft2(xd) * (nx * ny))
    e_fwd = rel_l2(fwd, np.fft.fft2(xd))
    log("  rel L2 inverse %.3e forward %.3e" % (e_inv, e_fwd))
    assert e_inv < TOL_BF16 and e_fwd < TOL_BF16


def test_forward_with_bf16x3_transform(ctx):
    import paper_2505_06582_amd as gws
    log("forward bf16x3")
    grid = Grid(160, 90, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(400, grid, 81, depth_range=(-10e-3, 10e-3))
    field, spec = run_forward(ctx, scene, grid, xform=gws.XFORM_DFT_BF16X3)
    ref = oracle.forward(scene, grid)
    e = rel_l2(field, ref)
    log("  rel %.3e" % e)
    assert e < TOL_BF16


@pytest.mark.parametrize("cfg", list(range(1, 10)))
def test_forward_every_tiling(ctx, cfg):
    log("forward tiling %d" % cfg)
    grid = Grid(160, 90, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(300, grid, 100 + cfg, depth_range=(-10e-3, 10e-3))
    field, spec = run_forward(ctx, scene, grid, tile_config=cfg)
    assert ctx.stats()["tile_config"] == cfg
    e = rel_l2(field, oracle.forward(scene, grid))
    log("  rel %.3e" % e)
    assert e < TOL_FWD
