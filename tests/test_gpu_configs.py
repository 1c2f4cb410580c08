"""Parity at the full sizes of the plain 10k-Gaussian forward and of the 16-scene batched
workload (both 1080 x 1920 x 3 wavelengths), in the launch configuration the benchmark uses.

Outputs the FP64 oracle can compute one by one are compared element by element:
  - the whole field of a few hundred Gaussians of the 10k workload's distributions;
  - spectrum entries sampled by radius band (the multi-chunk tiles around DC, three rings,
    and the band next to Nyquist), each an exact sum over every Gaussian of the scene, with
    the whole-grid relative L2 estimated from the band-weighted samples;
  - the transform stage separately: the GPU field against an FP64 inverse DFT of the GPU's
    own spectrum.  By Parseval the field's relative error equals the spectrum's, so the two
    bound the whole path's error;
  - gradients of sampled Gaussians against the oracle's dense FP64 gradient.
Batched calls (one persistent launch per kernel, replayed from a captured graph) must equal
one call per scene bitwise."""
import numpy as np
import pytest

import gwsgen
import oracle
from gpu_util import check_spectrum_and_transform, problem, rel_l2, scene_to_torch, to_numpy

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


def test_fwd10k_whole_field_of_300_gaussians(ctx):
    """Every pixel of the 1080 x 1920 x 3 field of 300 Gaussians of the 10k workload."""
    scene, grid = gwsgen.workload("fwd10k")
    sub = scene.subset(np.arange(300))
    log("fwd10k subset: whole field of 300 Gaussians at 1080x1920x3")
    field = to_numpy(ctx.forward(problem(grid), scene_to_torch(sub)))
    ref = oracle.forward(sub, grid)
    for c in range(3):
        log("  channel %d rel L2 %.3e" % (c, rel_l2(field[c], ref[c])))
    e = rel_l2(field, ref)
    peak = np.max(np.abs(ref))
    log("  whole field rel L2 %.3e, max |error| / max |field| %.3e" % (e, np.max(np.abs(field - ref)) / peak))
    assert e < 1e-5


def test_fwd10k_full_scene_sampled_by_band(ctx):
    """The full 10k-Gaussian scene: spectrum samples in every radius band, and the transform."""
    scene, grid = gwsgen.workload("fwd10k")
    log("fwd10k: 10k Gaussians at 1080x1920x3")
    field, spec = ctx.forward(problem(grid), scene_to_torch(scene), want_spectrum=True)
    check_spectrum_and_transform(scene, grid, to_numpy(field), to_numpy(spec), 1024, 21, "fwd10k")


def test_autotune_at_full_size(tmp_path):
    """The autotuner at 1080 x 1920 x 3 with the 10k workload: it records its timings under this
    grid's key, a new context takes the recorded choice from the cache file, the forward under
    that choice meets the oracle on band-sampled spectrum entries, and both contexts give the
    same field bit for bit."""
    import os
    import paper_2505_06582_amd as gws
    scene, grid = gwsgen.workload("fwd10k")
    prob = problem(grid)
    cache = str(tmp_path / "tune.jsonl")
    t = gws.Context(0)
    try:
        t.autotune(prob, scene.n, cache)
        text = open(cache).read()
        log("autotune at 1080x1920x3, 10k Gaussians: %s" % text.strip()[-300:])
        assert '"nx": 1920' in text and '"ny": 1080' in text and '"tile_config"' in text
        g = scene_to_torch(scene)
        field, spec = t.forward(prob, g, want_spectrum=True)
        cfg = t.stats()["tile_config"]
        assert 1 <= cfg <= 9
        check_spectrum_and_transform(scene, grid, to_numpy(field), to_numpy(spec), 512, 23, "fwd10k tuned")
        os.environ["GWS_TUNE_CACHE"] = cache
        try:
            c2 = gws.Context(0)
            f2 = c2.forward(prob, g)
            assert c2.stats()["tile_config"] == cfg
            assert np.array_equal(to_numpy(f2), to_numpy(field))
            c2.close()
        finally:
            del os.environ["GWS_TUNE_CACHE"]
    finally:
        t.close()


@pytest.fixture(scope="module")
def batched16():
    counts = gwsgen.batched_counts(16)
    grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    scenes = [gwsgen.make_scene(n, grid, 5000 + i, depth_range=(-10e-3, 10e-3)) for i, n in enumerate(counts)]
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return grid, counts, scenes, gwsgen.Scene.concat(scenes), offsets


def test_batched16_full_size_forward(ctx, batched16):
    import torch
    grid, counts, scenes, cat, offsets = batched16
    log("batched16 forward: %d scenes, %d Gaussians, counts %s" % (len(counts), cat.n, counts))
    prob = problem(grid)
    g = scene_to_torch(cat)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        fields, specs = ctx.forward_batched(prob, g, offsets, want_spectrum=True)
        ctx.forward_batched(prob, g, offsets, out=fields, spectrum=specs)
        st.synchronize()
        assert ctx.stats()["graph_replayed"] == 1
    for i, sc in enumerate(scenes):
        f, s = ctx.forward(prob, scene_to_torch(sc), want_spectrum=True)
        st_i = ctx.stats()
        assert torch.equal(f, fields[i]) and torch.equal(s, specs[i]), i
        log("  scene %2d: %6d Gaussians, %d items, chunk %d: batched == one call (bitwise)"
            % (i, counts[i], st_i["n_items"], st_i["chunk"]))
    for i in (int(np.argmin(counts)), int(np.argmax(counts))):
        check_spectrum_and_transform(scenes[i], grid, to_numpy(fields[i]), to_numpy(specs[i]), 512, 50 + i,
                                     "scene %d (%d Gaussians)" % (i, counts[i]))


def test_batched16_full_size_backward(ctx, batched16):
    import torch
    grid, counts, scenes, cat, offsets = batched16
    log("batched16 backward: %d scenes, %d Gaussians" % (len(counts), cat.n))
    prob = problem(grid)
    g = scene_to_torch(cat)
    G = np.stack([gwsgen.make_target(grid, 6000 + i) for i in range(len(counts))])
    Gt = torch.from_numpy(G).cuda()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        got = ctx.backward_batched(prob, g, offsets, Gt)
        got = ctx.backward_batched(prob, g, offsets, Gt, out=got)
        st.synchronize()
        assert ctx.stats()["graph_replayed"] == 1
    for i, sc in enumerate(scenes):
        a, b = int(offsets[i]), int(offsets[i + 1])
        one = ctx.backward(prob, scene_to_torch(sc), Gt[i])
        for k, v in one.items():
            part = got[k][:, a:b] if k == "amplitude" else got[k][a:b]
            assert torch.equal(part, v), (i, k)
    log("  batched gradients == one call per scene (bitwise), every parameter")
    host = {k: to_numpy(v) for k, v in got.items()}
    for i in (int(np.argmin(counts)), int(np.argmax(counts))):
        a, b = int(offsets[i]), int(offsets[i + 1])
        sel = np.random.default_rng(70 + i).choice(b - a, 24, replace=False)
        gs = oracle.spectrum_grad_from_field_grad(G[i].astype(np.complex128), grid)
        ref = oracle.param_grads_from_spectrum_grad(scenes[i], grid, gs, sel)
        for k in ("mean_x", "mean_y", "depth", "cov_xx", "cov_xy", "cov_yy", "opacity", "phase", "amplitude"):
            v = host[k][:, a:b][:, sel] if k == "amplitude" else host[k][a:b][sel]
            e = rel_l2(v, ref[k])
            log("  scene %d (%d Gaussians) %-9s rel L2 vs oracle %.3e" % (i, counts[i], k, e))
            assert e < 1e-4, (i, k, e)
