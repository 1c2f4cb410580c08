"""GPU parity of the adjoint (through the C ABI) against the FP64 oracle gradient."""
import numpy as np
import pytest

import gwsgen
import oracle
from gwsgen import Grid
from gpu_util import problem, rel_l2, scene_to_torch, to_numpy

pytestmark = pytest.mark.gpu

# normwise relative L2 per parameter group against the FP64 oracle gradient
TOL_GRAD = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


def check_grads(ctx, scene, grid, seed, tol=TOL_GRAD, want_depth=True):
    import torch
    G = gwsgen.make_target(grid, seed)
    got = ctx.backward(problem(grid), scene_to_torch(scene), torch.from_numpy(G).cuda(), want_depth=want_depth)
    ref = oracle.backward(scene, grid, G.astype(np.complex128))
    errs = {}
    names = ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity", "phase", "amplitude")
    for k in names if want_depth else [n for n in names if n != "depth"]:
        errs[k] = rel_l2(to_numpy(got[k]), ref[k])
    print({k: "%.2e" % v for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < tol, (k, v)


def test_backward_small_workload(ctx):
    scene, grid = gwsgen.workload("small")
    check_grads(ctx, scene, grid, 501)


def test_backward_without_depth_gradient(ctx):
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(100, grid, 63, depth_range=(-10e-3, 10e-3))
    check_grads(ctx, scene, grid, 64, want_depth=False)


@pytest.mark.parametrize("nx,ny,n,seed", [(96, 80, 150, 61), (48, 40, 30, 62)])
def test_backward_ragged_three_wavelengths(ctx, nx, ny, n, seed):
    grid = Grid(nx, ny, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(n, grid, seed, depth_range=(-10e-3, 10e-3))
    check_grads(ctx, scene, grid, seed + 1000)


def test_backward_zero_opacity_and_amplitude_still_get_gradients(ctx):
    grid = Grid(64, 64, 8e-6, 8e-6, (520e-9, 450e-9))
    scene = gwsgen.make_scene(20, grid, 71, depth_range=(-5e-3, 5e-3))
    scene.opacity[3] = 0.0
    scene.amplitude[:, 5] = 0.0
    check_grads(ctx, scene, grid, 72)


def test_backward_is_deterministic(ctx):
    import torch
    scene, grid = gwsgen.workload("small")
    G = torch.from_numpy(gwsgen.make_target(grid, 3)).cuda()
    a = ctx.backward(problem(grid), scene_to_torch(scene), G)
    b = ctx.backward(problem(grid), scene_to_torch(scene), G)
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_backward_with_bf16x3_transform(ctx):
    import torch
    import paper_2505_06582_amd as gws
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(80, grid, 91, depth_range=(-10e-3, 10e-3))
    G = gwsgen.make_target(grid, 92)
    got = ctx.backward(problem(grid, xform=gws.XFORM_DFT_BF16X3), scene_to_torch(scene), torch.from_numpy(G).cuda())
    ref = oracle.backward(scene, grid, G.astype(np.complex128))
    for k in ref:
        e = rel_l2(to_numpy(got[k]), ref[k])
        assert e < 1e-3, (k, e)


@pytest.mark.parametrize("cfg", list(range(1, 10)))
@pytest.mark.parametrize("want_depth", [True, False])
def test_backward_every_tiling(ctx, cfg, want_depth):
    import torch
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(60, grid, 200 + cfg, depth_range=(-10e-3, 10e-3))
    G = gwsgen.make_target(grid, 300 + cfg)
    got = ctx.backward(problem(grid, tile_config=cfg), scene_to_torch(scene), torch.from_numpy(G).cuda(),
                       want_depth=want_depth)
    ref = oracle.backward(scene, grid, G.astype(np.complex128))
    for k in ref:
        if k == "depth" and not want_depth:
            continue
        e = rel_l2(to_numpy(got[k]), ref[k])
        assert e < TOL_GRAD, (cfg, k, e)


FOUR = (638e-9, 520e-9, 450e-9, 405e-9)


def test_backward_four_wavelengths(ctx):
    """Four colour channels (the most the problem takes), without the depth gradient: every
    other parameter group against the oracle."""
    grid = Grid(96, 80, 8e-6, 8e-6, FOUR)
    scene = gwsgen.make_scene(90, grid, 411, depth_range=(-10e-3, 10e-3))
    check_grads(ctx, scene, grid, 412, want_depth=False)


@pytest.mark.skip(reason="four wavelengths with the depth gradient hung on the GPU in an earlier build of the "
                         "adjoint (108 KB of LDS per work-group) and the cause is not shown; the library "
                         "returns GWS_ERR_UNSUPPORTED for it")
def test_backward_four_wavelengths_with_depth(ctx):
    grid = Grid(96, 80, 8e-6, 8e-6, FOUR)
    scene = gwsgen.make_scene(90, grid, 411, depth_range=(-10e-3, 10e-3))
    check_grads(ctx, scene, grid, 412, want_depth=True)


def test_backward_four_wavelengths_depth_is_refused(ctx):
    import torch
    import paper_2505_06582_amd as gws
    grid = Grid(32, 32, 8e-6, 8e-6, FOUR)
    scene = gwsgen.make_scene(4, grid, 413)
    G = torch.from_numpy(gwsgen.make_target(grid, 414)).cuda()
    with pytest.raises(gws.GwsError):
        ctx.backward(problem(grid), scene_to_torch(scene), G, want_depth=True)


def test_backward_many_chunks_and_regions(ctx):
    """1500 Gaussians: several work-group chunks of sorted Gaussians, each over many frequency
    regions and tile ranges, with a ragged last chunk."""
    grid = Grid(256, 240, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(1500, grid, 421, depth_range=(-10e-3, 10e-3))
    check_grads(ctx, scene, grid, 422)
