"""The allocation-free forward (gws_forward_noalloc, through the C ABI) against gws_forward on
the same inputs: two calls in a row on one context, the second with fewer Gaussians and a
smaller grid than the first, so the shared scratch holds the first call's contents when the
second starts.  Both run the same kernels, so the fields must agree bitwise; the oracle bar
(relative L2 1e-5) is checked too."""
import numpy as np
import pytest

import gwsgen
import oracle
from gwsgen import Grid
from gpu_util import problem, rel_l2, scene_to_torch, to_numpy

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def test_noalloc_forward_matches_forward_twice():
    import torch
    import paper_2505_06582_amd as gws
    ctx = gws.context(0)
    cases = [(Grid(192, 160, 8e-6, 8e-6, gwsgen.RGB), 900, 7101), (Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB), 120, 7102)]
    for grid, n, seed in cases:
        log("noalloc forward: %d Gaussians at %dx%dx%d" % (n, grid.nx, grid.ny, grid.n_lambda))
        scene = gwsgen.make_scene(n, grid, seed, depth_range=(-10e-3, 10e-3))
        prob = problem(grid)
        g = scene_to_torch(scene)
        ref = ctx.forward(prob, g)  # builds the plan for this shape
        out = torch.full_like(ref, complex(np.nan, np.nan))
        got = ctx.forward_noalloc(prob, g, out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref), "noalloc field differs from gws_forward"
        e = rel_l2(to_numpy(got), oracle.forward(scene, grid))
        log("  bitwise equal to gws_forward; rel L2 vs oracle %.3e" % e)
        assert e < 1e-5


def test_noalloc_refuses_without_plan_and_beyond_scratch():
    import torch
    import paper_2505_06582_amd as gws
    ctx = gws.Context(0)  # a context of its own: no plan built yet, whatever ran before
    grid = Grid(80, 64, 8e-6, 8e-6, (520e-9,))
    scene = gwsgen.make_scene(10, grid, 7103)
    out = torch.empty((1, 64, 80), dtype=torch.complex64, device="cuda")
    with pytest.raises(gws.GwsError) as ei:
        ctx.forward_noalloc(problem(grid), scene_to_torch(scene), out)
    assert ei.value.status == -3  # GWS_ERR_UNSUPPORTED
    big = Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(20000, big, 7104, depth_range=(-10e-3, 10e-3))
    g = scene_to_torch(scene)
    ctx.forward(problem(big), scene_to_torch(scene.subset(np.arange(10))))  # plan exists
    out = torch.empty((3, 1080, 1920), dtype=torch.complex64, device="cuda")
    with pytest.raises(gws.GwsError) as ei:
        ctx.forward_noalloc(problem(big), g, out)
    assert ei.value.status == -4  # GWS_ERR_WORKSPACE
    log("  refused: %s" % ei.value)
