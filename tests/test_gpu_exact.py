"""GPU parity of exact alpha wave blending (Eq. 5-6, Alg. 2) through the C ABI against the
FP64 oracle in oracle/exact.py."""
import sys

import numpy as np
import pytest

import gwsgen
import oracle
import oracle.exact as ex
from gwsgen import Grid
from gpu_util import problem, rel_l2, scene_to_torch, to_numpy

pytestmark = pytest.mark.gpu

# FP32 tolerance for exact blending (relative L2 of the field), the same bar as the FP32
# order-invariant path: the transmittance is a product of FP32 factors and the profile is
# truncated at eps = 1e-7 of its peak (measured 4e-7 .. 2e-6).  The 1/255 alpha decision is
# taken in FP32 on the GPU and in FP64 by the oracle; at a pixel within rounding of the
# threshold both are correct, which test_exact_alpha_straddling_the_threshold covers with a
# bound of its own (these seeded scenes have no such pixel).
TOL_EXACT = 1e-5


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def clustered_scene(n, grid, seed, spread=0.3, o_range=(0.2, 1.0), depth_range=(-5e-3, 5e-3)):
    """Seeded Gaussians with the workloads' shapes, centred in a fraction of the field so that
    they overlap and occlude one another."""
    s = gwsgen.make_scene(n, grid, seed, depth_range=depth_range)
    rng = np.random.default_rng(seed + 1)
    # standard deviations up to a tenth of the grid, so that one periodic image of each
    # profile is all that reaches the field (the kernel's window is at most half the grid)
    smax = min(20.0, min(grid.nx, grid.ny) / 10.0)
    su, sv = rng.uniform(2.0, smax, n), rng.uniform(2.0, smax, n)
    th = rng.uniform(0.0, np.pi, n)
    c, sn = np.cos(th), np.sin(th)
    p2 = grid.px * grid.py
    s.cov_xx[:] = ((c * c * su * su + sn * sn * sv * sv) * p2).astype(np.float32)
    s.cov_xy[:] = ((c * sn * (su * su - sv * sv)) * p2).astype(np.float32)
    s.cov_yy[:] = ((sn * sn * su * su + c * c * sv * sv) * p2).astype(np.float32)
    w, h = grid.nx * grid.px, grid.ny * grid.py
    s.mean_x[:] = (rng.uniform(-spread / 2, spread / 2, n) * w).astype(np.float32)
    s.mean_y[:] = (rng.uniform(-spread / 2, spread / 2, n) * h).astype(np.float32)
    s.opacity[:] = rng.uniform(*o_range, n).astype(np.float32)
    return s


def gpu_exact(ctx, scene, grid, **kw):
    import paper_2505_06582_amd as gws
    prob = problem(grid, blend=gws.BLEND_EXACT, **kw)
    return to_numpy(ctx.forward(prob, scene_to_torch(scene)))


@pytest.mark.parametrize("n,grid,seed", [
    (32, Grid(64, 48, 8e-6, 8e-6, (520e-9, 638e-9)), 2101),          # one batch
    (200, Grid(256, 256, 8e-6, 8e-6, gwsgen.RGB), 2102),              # four batches, 3 wavelengths
    (65, Grid(240, 200, 8e-6, 8e-6, (450e-9,)), 2103),                # ragged batch, non-square grid
])
def test_exact_matches_oracle(ctx, n, grid, seed):
    log("exact parity n=%d grid=%dx%dx%d seed=%d" % (n, grid.nx, grid.ny, grid.n_lambda, seed))
    s = clustered_scene(n, grid, seed)
    u = gpu_exact(ctx, s, grid)
    ref = ex.exact_forward(s, grid)
    err = rel_l2(u, ref)
    log("  rel L2 %.3g" % err)
    assert err < TOL_EXACT
    # the occlusion is real: the order-invariant sum differs by far more than the tolerance
    assert rel_l2(oracle.forward(s, grid), ref) > 100 * TOL_EXACT


def test_exact_wraps_around_the_grid_edge(ctx):
    grid = Grid(128, 96, 8e-6, 8e-6, (520e-9,))
    s = clustered_scene(24, grid, 2104)
    # put the cluster on the corner so every window wraps in both axes
    s.mean_x[:] = (s.mean_x + np.float32(0.5 * grid.nx * grid.px)).astype(np.float32)
    s.mean_y[:] = (s.mean_y + np.float32(0.5 * grid.ny * grid.py)).astype(np.float32)
    err = rel_l2(gpu_exact(ctx, s, grid), ex.exact_forward(s, grid))
    log("exact wrap rel L2 %.3g" % err)
    assert err < TOL_EXACT


def test_exact_below_threshold_equals_gpu_order_invariant(ctx):
    grid = Grid(192, 160, 8e-6, 8e-6, gwsgen.RGB)
    s = clustered_scene(40, grid, 2105, o_range=(0.5 / 255, 0.9 / 255))
    u_exact = gpu_exact(ctx, s, grid)
    u_oit = to_numpy(ctx.forward(problem(grid), scene_to_torch(s)))
    err = rel_l2(u_exact, u_oit)
    log("exact vs OIT below threshold rel L2 %.3g" % err)
    assert err < 1e-5


def test_exact_empty_and_zero_opacity(ctx):
    grid = Grid(64, 64, 8e-6, 8e-6, (520e-9,))
    s = clustered_scene(8, grid, 2106)
    s.opacity[:] = 0.0
    assert np.all(gpu_exact(ctx, s, grid) == 0)
    empty = s.subset(np.arange(0))
    assert np.all(gpu_exact(ctx, empty, grid) == 0)


def test_exact_counts_culled_and_clamped_windows(ctx):
    """Invalid Gaussians are skipped and counted; a Gaussian whose eps-window reaches past half
    the grid is counted as clamped (its profile is cut at nx/2 - 1, ny/2 - 1 pixels)."""
    import paper_2505_06582_amd as gws
    grid = Grid(64, 48, 8e-6, 8e-6, (520e-9,))
    s = clustered_scene(12, grid, 2111)
    # every other Gaussian isotropic with sigma 2.5 px: window ceil(2.5 sqrt(2 ln 1e7)) = 15 px,
    # inside the 31 x 23 px half-grid, so only the two wide ones below are clamped
    s.cov_xx[:] = s.cov_yy[:] = np.float32(6.25 * 64e-12)
    s.cov_xy[:] = np.float32(0.0)
    s.cov_xy[0] = np.float32(2.0 * np.sqrt(float(s.cov_xx[0]) * float(s.cov_yy[0])))  # not positive definite
    s.mean_x[1] = np.float32(np.nan)
    wide = (4, 9)
    for i in wide:   # sigma 10 px: window 10 sqrt(2 ln 1e7) = 57 px > 31 and 23
        s.cov_xx[i], s.cov_xy[i], s.cov_yy[i] = np.float32(100 * 64e-12), np.float32(0.0), np.float32(100 * 64e-12)
    prob = problem(grid, blend=gws.BLEND_EXACT)
    ctx.forward(prob, scene_to_torch(s))
    st = ctx.stats()
    log("exact stats: culled %d, clamped %d" % (st["n_culled"], st["n_window_clamped"]))
    assert st["n_culled"] == 2 and st["n_window_clamped"] == len(wide)
    G = gwsgen.make_target(grid, 2112)
    import torch
    ctx.backward(prob, scene_to_torch(s), torch.from_numpy(G).cuda())
    st = ctx.stats()
    assert st["n_culled"] == 2 and st["n_window_clamped"] == len(wide)
    ctx.forward(problem(grid), scene_to_torch(s))
    assert ctx.stats()["n_window_clamped"] == 0


def test_exact_alpha_straddling_the_threshold(ctx):
    """Front Gaussians whose alpha equals 1/255 to FP32 rounding on whole rings of pixels
    (isotropic, centred on a pixel, opacity exp(r^2 / 2 sigma^2) / 255 for an integer r^2), over a
    Gaussian behind them.  At those pixels either decision is a correct reading (the GPU takes
    it in FP32, the oracle in FP64), so the GPU field must lie within the FP32 tolerance of the
    oracle plus the distance between the oracle with the threshold moved down and up by 1e-5
    (which brackets every mix of decisions at pixels within 1e-5 of it)."""
    grid = Grid(128, 96, 8e-6, 8e-6, (520e-9,))
    p = grid.px
    front = [((0, 0), 3.0, 25), ((-14, 8), 2.5, 13), ((12, -9), 4.0, 50), ((9, 11), 3.5, 34)]
    n = len(front) + 1
    s = clustered_scene(n, grid, 2113)
    for i, ((cx, cy), sig, r2) in enumerate(front):
        s.mean_x[i], s.mean_y[i] = np.float32(cx * p), np.float32(cy * p)
        s.cov_xx[i] = s.cov_yy[i] = np.float32(sig * sig * p * p)
        s.cov_xy[i] = np.float32(0.0)
        s.opacity[i] = np.float32(np.exp(r2 / (2 * sig * sig)) / 255.0)
        s.depth[i] = np.float32(1e-3 + 1e-4 * i)
    s.mean_x[-1], s.mean_y[-1] = np.float32(0.0), np.float32(0.0)
    # sigma 6 px: window ceil(6 sqrt(2 ln 1e7)) = 35 px, inside the 63 x 47 px half-grid
    s.cov_xx[-1] = s.cov_yy[-1] = np.float32(36 * p * p)
    s.cov_xy[-1] = np.float32(0.0)
    s.opacity[-1] = np.float32(0.8)
    s.depth[-1] = np.float32(-2e-3)
    u = gpu_exact(ctx, s, grid)
    assert ctx.stats()["n_window_clamped"] == 0
    mid = ex.exact_forward(s, grid)
    lo = ex.exact_forward(s, grid, t_eps=ex.T_EPS * (1 - 1e-5))
    hi = ex.exact_forward(s, grid, t_eps=ex.T_EPS * (1 + 1e-5))
    spread = rel_l2(lo, hi)
    err = rel_l2(u, mid)
    log("straddling scene: oracle spread (threshold -/+ 1e-5) %.3e, GPU vs oracle %.3e, vs lower %.3e, "
        "vs upper %.3e" % (spread, err, rel_l2(u, lo), rel_l2(u, hi)))
    assert spread > 1e-6        # the scene does sit on the threshold
    assert err <= TOL_EXACT + spread


def test_exact_full_size_grid(ctx):
    grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    s = clustered_scene(40, grid, 2107, spread=0.05, depth_range=(-10e-3, 10e-3))
    log("exact 1080x1920x3, 40 Gaussians")
    u = gpu_exact(ctx, s, grid)
    ref = ex.exact_forward(s, grid)
    err = rel_l2(u, ref)
    log("  rel L2 %.3g" % err)
    assert err < TOL_EXACT


def test_exact_batched_equals_one_call_per_scene(ctx):
    """Batched exact blending (scenes of 30, 0, 70 and 5 Gaussians) gives each scene's own
    exact forward and backward, and the forward matches the oracle per scene."""
    import torch
    import paper_2505_06582_amd as gws
    grid = Grid(96, 80, 8e-6, 8e-6, (638e-9, 520e-9))
    parts = [clustered_scene(n, grid, 2108 + i) for i, n in enumerate((30, 0, 70, 5))]
    offs = np.cumsum([0] + [p.n for p in parts]).tolist()
    allg = gwsgen.Scene.concat(parts)
    prob = problem(grid, blend=gws.BLEND_EXACT)
    tg = scene_to_torch(allg)
    fb = to_numpy(ctx.forward_batched(prob, tg, offs))
    M = grid.n_lambda * grid.ny * grid.nx
    G = np.stack([gwsgen.make_target(grid, 2120 + i) * 0.05 for i in range(len(parts))])
    gb = ctx.backward_batched(prob, tg, offs, torch.from_numpy(G.astype(np.complex64)).cuda(), want_depth=True)
    for i, p in enumerate(parts):
        one = to_numpy(ctx.forward(prob, scene_to_torch(p)))
        assert np.array_equal(fb[i], one), i
        assert rel_l2(fb[i], ex.exact_forward(p, grid)) < TOL_EXACT or p.n == 0
        if p.n == 0:
            assert np.all(fb[i] == 0)
            continue
        g1 = ctx.backward(prob, scene_to_torch(p), torch.from_numpy(G[i].astype(np.complex64)).cuda(),
                          want_depth=True)
        for k in g1:
            a = to_numpy(gb[k])
            a = a[:, offs[i]:offs[i + 1]] if a.ndim == 2 else a[offs[i]:offs[i + 1]]
            assert np.array_equal(a, to_numpy(g1[k])), (i, k)
    log("batched exact == per-scene calls (forward and backward), %d scenes" % len(parts))


# Gradients through exact blending: per parameter group, normwise relative L2 against the FP64
# reverse-mode oracle (itself pinned to central differences), the same bar as the
# order-invariant adjoint.
TOL_EXACT_GRAD = 1e-4


@pytest.mark.parametrize("n,grid,seed", [
    (24, Grid(64, 48, 8e-6, 8e-6, (520e-9, 638e-9)), 2201),          # one batch, 2 wavelengths
    (100, Grid(128, 96, 8e-6, 8e-6, gwsgen.RGB), 2202),               # two batches, 3 wavelengths
    (65, Grid(96, 80, 8e-6, 8e-6, (450e-9,)), 2203),                  # ragged second batch
    (40, Grid(64, 48, 8e-6, 8e-6, (638e-9, 520e-9, 450e-9, 405e-9)), 2205),  # four wavelengths
])
def test_exact_backward_matches_oracle(ctx, n, grid, seed):
    import torch
    import paper_2505_06582_amd as gws
    import oracle.exact_grad as eg
    log("exact backward n=%d grid=%dx%dx%d" % (n, grid.nx, grid.ny, grid.n_lambda))
    s = clustered_scene(n, grid, seed)
    t = gwsgen.make_target(grid, seed + 50) * 0.05
    _, u, ref = eg.exact_loss_grads(s, grid, t)
    G = torch.from_numpy((2.0 * (u - t)).astype(np.complex64)).cuda()
    prob = problem(grid, blend=gws.BLEND_EXACT)
    got = ctx.backward(prob, scene_to_torch(s), G, want_depth=True)
    for k in eg.PARAMS:
        err = rel_l2(to_numpy(got[k]).astype(np.float64), np.asarray(ref[k]))
        log("  %-10s rel L2 %.3g" % (k, err))
        assert err < TOL_EXACT_GRAD, k


def test_exact_backward_wraps_around_the_grid_edge(ctx):
    """Gradients when every window wraps around both grid edges, over two batches: the
    windowed transforms load and store only the windows' (wrapped) columns and rows."""
    import torch
    import paper_2505_06582_amd as gws
    import oracle.exact_grad as eg
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    s = clustered_scene(70, grid, 2204)
    s.mean_x[:] = (s.mean_x + np.float32(0.5 * grid.nx * grid.px)).astype(np.float32)
    s.mean_y[:] = (s.mean_y + np.float32(0.5 * grid.ny * grid.py)).astype(np.float32)
    t = gwsgen.make_target(grid, 2254) * 0.05
    _, u, ref = eg.exact_loss_grads(s, grid, t)
    G = torch.from_numpy((2.0 * (u - t)).astype(np.complex64)).cuda()
    got = ctx.backward(problem(grid, blend=gws.BLEND_EXACT), scene_to_torch(s), G, want_depth=True)
    for k in eg.PARAMS:
        err = rel_l2(to_numpy(got[k]).astype(np.float64), np.asarray(ref[k]))
        log("  wrap %-10s rel L2 %.3g" % (k, err))
        assert err < TOL_EXACT_GRAD, k


@pytest.mark.parametrize("blend", ["oit", "exact"])
def test_render_autograd_matches_oracle(ctx, blend):
    """The torch.autograd.Function path (render + loss.backward) for both blending models."""
    import torch
    import paper_2505_06582_amd as gws
    import oracle.exact_grad as eg
    grid = Grid(64, 48, 8e-6, 8e-6, (520e-9, 638e-9))
    s = clustered_scene(20, grid, 2301)
    t = gwsgen.make_target(grid, 2302) * 0.05
    prob = problem(grid, blend=gws.BLEND_EXACT if blend == "exact" else gws.BLEND_OIT)
    params = {k: v.clone().requires_grad_(True) for k, v in scene_to_torch(s).items()}
    u = gws.render(prob, *[params[k] for k in eg.PARAMS])
    loss = torch.sum(torch.abs(u - torch.from_numpy(t.astype(np.complex64)).cuda()) ** 2)
    loss.backward()
    if blend == "exact":
        _, _, ref = eg.exact_loss_grads(s, grid, t)
    else:
        uo = oracle.forward(s, grid)
        _, G = oracle.loss_and_field_grad(uo, t)
        ref = oracle.backward(s, grid, G)
    for k in eg.PARAMS:
        err = rel_l2(to_numpy(params[k].grad).astype(np.float64), np.asarray(ref[k]))
        log("  render/%s %-10s rel L2 %.3g" % (blend, k, err))
        assert err < TOL_EXACT_GRAD, k


def test_exact_backward_full_size_grid(ctx):
    """Gradients at the benchmark's shape (1080 x 1920, three wavelengths) and launch
    configuration, against the FP64 oracle: 17 Gaussians, so eight packed pairs and one
    Gaussian alone in its image in the adjoint's inverse transforms."""
    import torch
    import paper_2505_06582_amd as gws
    import oracle.exact_grad as eg
    grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    s = clustered_scene(17, grid, 2301, spread=0.05, depth_range=(-10e-3, 10e-3))
    t = gwsgen.make_target(grid, 2351) * 0.05
    _, u, ref = eg.exact_loss_grads(s, grid, t)
    G = torch.from_numpy((2.0 * (u - t)).astype(np.complex64)).cuda()
    del u
    got = ctx.backward(problem(grid, blend=gws.BLEND_EXACT), scene_to_torch(s), G, want_depth=True)
    for k in eg.PARAMS:
        err = rel_l2(to_numpy(got[k]).astype(np.float64), np.asarray(ref[k]))
        log("  full-size %-10s rel L2 %.3g" % (k, err))
        assert err < TOL_EXACT_GRAD, k
