"""Reference plane-wave illumination (Sec. 4.1: the angular spectrum shifted by k_r) on the GPU
against the FP64 oracle: forward field and every gradient, for shifts on and between frequency
bins, and one reaching towards the band edge.  With nu_r = 0 the path is the on-axis one,
bitwise."""
import dataclasses

import numpy as np
import pytest

import gwsgen
import oracle
from gwsgen import Grid
from gpu_util import problem, rel_l2, scene_to_torch, to_numpy

pytestmark = pytest.mark.gpu

TOL_FWD = 1e-5
TOL_GRAD = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


def log(msg):
    print(msg, flush=True)


def shifted(grid, mx, my):
    """The grid with a reference wave whose support centre is (mx, my) in frequency-index units."""
    return dataclasses.replace(grid, ref_nu=(mx / (grid.nx * grid.px), my / (grid.ny * grid.py)))


CASES = [
    ((96, 80, 160, 801), (23.37, -11.6)),   # between bins
    ((96, 80, 120, 802), (-17.0, 9.0)),     # on bins
    ((160, 90, 200, 803), (61.2, 30.9)),    # towards the band edge: supports wrap off the grid
    ((48, 40, 40, 804), (-3.5, 0.25)),
]


@pytest.mark.parametrize("shape,mr", CASES)
def test_refwave_forward_matches_oracle(ctx, shape, mr):
    nx, ny, n, seed = shape
    grid = shifted(Grid(nx, ny, 8e-6, 8e-6, gwsgen.RGB), *mr)
    scene = gwsgen.make_scene(n, grid, seed, depth_range=(-10e-3, 10e-3))
    u = to_numpy(ctx.forward(problem(grid), scene_to_torch(scene)))
    e = rel_l2(u, oracle.forward(scene, grid))
    log("refwave forward %dx%d m_r=%s: rel L2 %.3e" % (nx, ny, mr, e))
    assert e < TOL_FWD


@pytest.mark.parametrize("shape,mr", CASES[:3])
@pytest.mark.parametrize("want_depth", [True, False])
def test_refwave_backward_matches_oracle(ctx, shape, mr, want_depth):
    import torch
    nx, ny, n, seed = shape
    grid = shifted(Grid(nx, ny, 8e-6, 8e-6, gwsgen.RGB), *mr)
    scene = gwsgen.make_scene(n, grid, seed, depth_range=(-10e-3, 10e-3))
    G = gwsgen.make_target(grid, seed + 50)
    got = ctx.backward(problem(grid), scene_to_torch(scene), torch.from_numpy(G).cuda(), want_depth=want_depth)
    ref = oracle.backward(scene, grid, G.astype(np.complex128))
    errs = {k: rel_l2(to_numpy(got[k]), ref[k]) for k in ref if want_depth or k != "depth"}
    log("refwave backward %dx%d m_r=%s: %s" % (nx, ny, mr, {k: "%.2e" % v for k, v in errs.items()}))
    for k, v in errs.items():
        assert v < TOL_GRAD, (k, v)


def test_refwave_zero_is_the_on_axis_path_bitwise(ctx):
    import torch
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(150, grid, 805, depth_range=(-10e-3, 10e-3))
    g = scene_to_torch(scene)
    a = ctx.forward(problem(grid), g)
    b = ctx.forward(problem(grid, ref_nu=(0.0, 0.0)), g)
    assert torch.equal(a, b)


def test_refwave_exact_blend_and_out_of_band_are_refused(ctx):
    import torch
    import paper_2505_06582_amd as gws
    grid = Grid(32, 32, 8e-6, 8e-6, (520e-9,))
    scene = gwsgen.make_scene(4, grid, 806)
    g = scene_to_torch(scene)
    with pytest.raises(gws.GwsError):
        ctx.forward(problem(grid, blend=gws.BLEND_EXACT, ref_nu=(1000.0, 0.0)), g)
    with pytest.raises(gws.GwsError):
        ctx.forward(problem(grid, ref_nu=(0.6 / grid.px, 0.0)), g)
