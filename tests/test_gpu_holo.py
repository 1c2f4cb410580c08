"""GPU parity of the holographics transform (gws_holographics) against the FP64 oracle in
oracle/holographics.py, and its composition with the order-invariant forward."""
import sys

import numpy as np
import pytest

import gwsgen
import oracle
import oracle.holographics as hg
from gwsgen import Grid, Scene
from gpu_util import problem, rel_l2, scene_to_torch, to_numpy

pytestmark = pytest.mark.gpu

# The kernel computes in FP64 from the same FP32 inputs and rounds each output to FP32 once:
# per output, |gpu - oracle| <= TOL_REL * (|oracle| + the field's scale).
TOL_REL = 2e-6


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def world_to_torch(w):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in w.items()}


def compare(got, ref):
    for k in hg.OUTPUTS:
        g = to_numpy(got[k]).astype(np.float64)
        r = ref[k]
        scale = np.max(np.abs(r)) if k != "opacity" else 1.0
        err = np.max(np.abs(g - r) / (np.abs(r) + scale))
        log("  %-8s max rel err %.3g" % (k, err))
        assert err < TOL_REL, k


@pytest.mark.parametrize("n,sh_degree,flat,seed", [
    (3000, 3, True, 4101),      # flat 2D Gaussians, degree-3 opacity
    (1000, 1, False, 4102),     # full 3D scales
    (777, 0, True, 4103),       # constant opacity, ragged count
])
def test_holographics_matches_oracle(ctx, n, sh_degree, flat, seed):
    log("holographics n=%d sh_degree=%d flat=%s" % (n, sh_degree, flat))
    cam = gwsgen.make_camera(seed, sh_degree=sh_degree)
    w = gwsgen.make_world_scene(n, cam, seed + 1, sh_degree=sh_degree, flat=flat)
    got = ctx.holographics(cam, world_to_torch(w))
    compare(got, hg.transform(w, cam))


def test_holographics_culls_behind_the_near_plane(ctx):
    cam = gwsgen.make_camera(4201)
    w = gwsgen.make_world_scene(256, cam, 4202)
    # push a third of the Gaussians behind the camera and a third inside the near distance
    V = np.asarray(cam["world_to_view"]).reshape(3, 4)
    R, t = V[:, :3], V[:, 3]
    p = w["mean"].astype(np.float64) @ R.T + t
    p[::3, 2] = -p[::3, 2]
    p[1::3, 2] = -0.05
    w["mean"] = np.ascontiguousarray(((p - t) @ R).astype(np.float32))
    got = ctx.holographics(cam, world_to_torch(w))
    ref = hg.transform(w, cam)
    culled = ref["opacity"] == 0.0
    assert culled.sum() >= 170
    for k in ("opacity", "cov_xx", "cov_yy", "cov_xy"):
        assert np.all(to_numpy(got[k])[culled] == 0.0), k
    compare(got, ref)


def test_holographics_empty_and_bad_degree(ctx):
    import torch
    import paper_2505_06582_amd as gws
    cam = gwsgen.make_camera(4301)
    w = world_to_torch(gwsgen.make_world_scene(0, cam, 4302))
    out = ctx.holographics(cam, w)
    assert all(v.numel() == 0 for v in out.values())
    bad = dict(cam)
    bad["sh_degree"] = 4
    with pytest.raises(gws.GwsError):
        ctx.holographics(bad, world_to_torch(gwsgen.make_world_scene(4, cam, 4303)))


def plane_scene(out, n, grid, seed):
    """A Scene with the transform's outputs and seeded amplitudes and phases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    amp = rng.uniform(0, 1, (grid.n_lambda, n)).astype(np.float32)
    ph = rng.uniform(0, 2 * np.pi, n).astype(np.float32)
    f = {k: np.asarray(out[k], dtype=np.float32) for k in hg.OUTPUTS}
    return Scene(mean_x=f["mean_x"], mean_y=f["mean_y"], depth=f["depth"], cov_xx=f["cov_xx"], cov_xy=f["cov_xy"],
                 cov_yy=f["cov_yy"], opacity=f["opacity"], amplitude=amp, phase=ph)


def test_world_scene_hologram(ctx):
    """World-space Gaussians to a hologram: the library's forward on the oracle's transform
    outputs matches the oracle's forward to the forward's own tolerance, and the whole GPU
    chain (transform + forward) agrees with it up to the FP32 rounding of the transform's
    outputs (means of ~5 mm rounded to 4e-10 m shift phases by up to 2 pi nu 4e-10 at the
    spectral widths, ~1e-5 rad)."""
    grid = Grid(384, 256, 8e-6, 8e-6, gwsgen.RGB)
    cam = gwsgen.make_camera(4401, nx=384, ny=256, depth_range=(-5e-3, 5e-3))
    w = gwsgen.make_world_scene(300, cam, 4402, nx=384, ny=256)
    ref_t = hg.transform(w, cam)
    s_ref = plane_scene(ref_t, 300, grid, 4403)
    u_ref = oracle.forward(s_ref, grid)
    u1 = to_numpy(ctx.forward(problem(grid), scene_to_torch(s_ref)))
    e1 = rel_l2(u1, u_ref)
    got_t = ctx.holographics(cam, world_to_torch(w))
    s_gpu = scene_to_torch(s_ref)
    for k in hg.OUTPUTS:
        s_gpu[k] = got_t[k]
    e2 = rel_l2(to_numpy(ctx.forward(problem(grid), s_gpu)), u_ref)
    log("world scene: forward on oracle transform rel L2 %.3g; GPU chain %.3g" % (e1, e2))
    assert e1 < 1e-5
    assert e2 < 1e-4
