"""Batched scenes in one persistent launch, captured in a hipGraph, and the autotuner."""
import os

import numpy as np
import pytest

import gwsgen
import oracle
from gwsgen import Grid
from gpu_util import problem, rel_l2, scene_to_torch, to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


def batch(grid, counts, seed):
    scenes = [gwsgen.make_scene(n, grid, seed + i, depth_range=(-10e-3, 10e-3)) for i, n in enumerate(counts)]
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return scenes, gwsgen.Scene.concat(scenes), offsets


def test_batched_forward_equals_sequential_and_graph_replays(ctx):
    import torch
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    counts = [120, 7, 300, 0, 45]
    scenes, cat, offsets = batch(grid, counts, 400)
    prob = problem(grid)
    seq = [to_numpy(ctx.forward(prob, scene_to_torch(sc))) for sc in scenes]
    st = torch.cuda.Stream()
    g = scene_to_torch(cat)
    out = torch.empty((len(counts), 3, grid.ny, grid.nx), dtype=torch.complex64, device="cuda")
    with torch.cuda.stream(st):
        for rep in range(4):
            ctx.forward_batched(prob, g, offsets, out=out)
            st.synchronize()
            replayed = ctx.stats()["graph_replayed"]
            assert replayed == (1 if rep > 0 else 0)
            got = to_numpy(out)
            for i in range(len(counts)):
                assert np.array_equal(got[i], seq[i]), (rep, i)
            # eager work between replays
            out.zero_()
            torch.cuda.synchronize()
    # the replayed graph reads the current Gaussian values
    cat2 = cat.copy()
    cat2.phase = (cat2.phase + np.float32(0.7)).astype(np.float32)
    g2 = scene_to_torch(cat2)
    for k in g:
        g[k].copy_(g2[k])
    with torch.cuda.stream(st):
        ctx.forward_batched(prob, g, offsets, out=out)
        st.synchronize()
    assert ctx.stats()["graph_replayed"] == 1
    got = to_numpy(out)
    for i, n in enumerate(counts):
        sub = cat2.subset(np.arange(offsets[i], offsets[i + 1]))
        ref = oracle.forward(sub, grid) if n else np.zeros((3, grid.ny, grid.nx))
        assert rel_l2(got[i], ref) < 1e-5 if n else np.all(got[i] == 0)


def test_batched_backward_equals_sequential(ctx):
    import torch
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    counts = [60, 150, 3]
    scenes, cat, offsets = batch(grid, counts, 500)
    prob = problem(grid)
    G = np.stack([gwsgen.make_target(grid, 600 + i) for i in range(len(counts))])
    seq = [ctx.backward(prob, scene_to_torch(sc), torch.from_numpy(G[i]).cuda()) for i, sc in enumerate(scenes)]
    seq = [{k: to_numpy(v) for k, v in d.items()} for d in seq]
    st = torch.cuda.Stream()
    g = scene_to_torch(cat)
    Gt = torch.from_numpy(G).cuda()
    with torch.cuda.stream(st):
        for rep in range(3):
            got = ctx.backward_batched(prob, g, offsets, Gt)
            st.synchronize()
            for k in got:
                v = to_numpy(got[k])
                for i in range(len(counts)):
                    a, b = offsets[i], offsets[i + 1]
                    ref = seq[i][k][..., :] if k != "amplitude" else seq[i][k]
                    part = v[:, a:b] if k == "amplitude" else v[a:b]
                    assert np.array_equal(part, ref), (rep, k, i)
            torch.cuda.synchronize()


def test_autotune_picks_a_tiling_and_results_stay_exact(ctx, tmp_path):
    import torch
    import paper_2505_06582_amd as gws
    grid = Grid(160, 90, 8e-6, 8e-6, gwsgen.RGB)
    prob = problem(grid)
    cache = str(tmp_path / "tune.jsonl")
    ctx.autotune(prob, 2000, cache)
    text = open(cache).read()
    assert '"nx": 160' in text and '"tile_config"' in text
    scene = gwsgen.make_scene(2000, grid, 700, depth_range=(-10e-3, 10e-3))
    field = to_numpy(ctx.forward(prob, scene_to_torch(scene)))
    cfg = ctx.stats()["tile_config"]
    assert 1 <= cfg <= 9
    assert rel_l2(field, oracle.forward(scene, grid)) < 1e-5
    # a new context picks the choice up from the cache file
    os.environ["GWS_TUNE_CACHE"] = cache
    try:
        c2 = gws.Context(0)
        c2.forward(prob, scene_to_torch(scene))
        assert c2.stats()["tile_config"] == cfg
        c2.close()
    finally:
        del os.environ["GWS_TUNE_CACHE"]
