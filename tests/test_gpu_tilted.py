"""Tilted Gaussians (Sec. 4.1, Eq. 8-10) on the GPU against the FP64 oracle (oracle/tilted.py):
field and spectrum on small grids (one to three wavelengths, ragged tile edges, tilts of a few
degrees at the workloads' 8 um pitch, and 20-28 degree tilts on fine grids whose band reaches
the evanescent edge), edge cases (no Gaussians, culled ones, a flipped description of the same
disk, a rotation about z alone against the in-plane path), determinism, and the 100k-Gaussian
1080 x 1920 x 3 workload on sampled frequencies; the adjoint against the float64 autograd oracle
(oracle/tilted_grad.py) on the same kinds of grids, with culled and zero-opacity Gaussians, and
for sampled Gaussians of the 100k workload."""
import dataclasses

import numpy as np
import pytest

import gwsgen
import oracle
import oracle.tilted as otl
import oracle.tilted_grad as otg
from gwsgen import Grid
from gpu_util import dft_ready, problem, rel_l2, scene_to_torch, stratified_freqs, to_numpy

pytestmark = pytest.mark.gpu

TOL = 1e-5
FOUR = (638e-9, 520e-9, 450e-9, 405e-9)


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


def log(msg):
    print(msg, flush=True)


CASES = [
    # (nx, ny, pitch, lambdas, n, seed, sigma_px, tilt_max_deg)
    (96, 80, 8e-6, gwsgen.RGB, 200, 901, (2.0, 20.0), 2.0),
    (160, 90, 8e-6, gwsgen.RGB, 300, 902, (2.0, 20.0), 2.0),
    (48, 40, 8e-6, (520e-9,), 60, 903, (1.0, 6.0), 3.0),
    (128, 96, 1e-6, (520e-9, 450e-9), 120, 904, (1.0, 4.0), 25.0),
    (64, 72, 0.25e-6, (633e-9,), 80, 905, (2.0, 6.0), 28.0),   # band past 1/lambda: evanescent corners
    (64, 48, 8e-6, FOUR, 60, 906, (2.0, 20.0), 2.0),             # four wavelengths (the problem's maximum)
    (64, 48, 8e-6, (520e-9,), 20000, 907, (2.0, 20.0), 2.0),     # tiles' Gaussians in two parts
]


@pytest.mark.parametrize("case", CASES, ids=["%dx%d-%dl-t%g" % (c[0], c[1], len(c[3]), c[7]) for c in CASES])
def test_tilted_forward_matches_oracle(ctx, case):
    nx, ny, pitch, lams, n, seed, sig, tilt = case
    grid = Grid(nx, ny, pitch, pitch, lams)
    scene = gwsgen.make_tilted_scene(n, grid, seed, depth_range=(-10e-3, 10e-3), sigma_px=sig, tilt_max_deg=tilt)
    u, s = ctx.forward_tilted(problem(grid), scene_to_torch(scene), want_spectrum=True)
    U = otl.spectrum(scene, grid)
    es = rel_l2(to_numpy(s), dft_ready(U, grid))
    eu = rel_l2(to_numpy(u), oracle.field_from_spectrum(U, grid))
    st = ctx.stats()
    log("tilted %dx%d pitch %g C=%d tilt<=%g: spectrum %.3e field %.3e (pairs %d, staged %d)"
        % (nx, ny, pitch, len(lams), tilt, es, eu, st["n_pairs_evaluated"], st["n_candidates"]))
    assert es < TOL and eu < TOL


def test_tilted_split_bf16_transform(ctx):
    import paper_2505_06582_amd as gws
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_tilted_scene(150, grid, 906, depth_range=(-10e-3, 10e-3))
    u = to_numpy(ctx.forward_tilted(problem(grid, xform=gws.XFORM_DFT_BF16X3), scene_to_torch(scene)))
    e = rel_l2(u, otl.forward(scene, grid))
    log("tilted split-bf16 transform: %.3e" % e)
    assert e < 1e-4


def test_tilted_empty_and_culled(ctx):
    import torch
    grid = Grid(64, 48, 8e-6, 8e-6, gwsgen.RGB)
    sc = gwsgen.make_tilted_scene(12, grid, 907)
    # no Gaussians: a zero field
    empty = {k: (v[:, :0] if k == "amplitude" else v[:0]) for k, v in scene_to_torch(sc).items()}
    u = ctx.forward_tilted(problem(grid), empty)
    assert torch.count_nonzero(u).item() == 0
    # every Gaussian invalid in a different way: all culled, zero field, counted
    bad = sc.copy()
    bad.opacity[0] = 0.0
    bad.scale_u[1] = 0.0
    bad.scale_v[2] = -1e-5
    bad.quat_w[3] = bad.quat_x[3] = bad.quat_y[3] = bad.quat_z[3] = 0.0
    bad.mean_x[4] = np.nan
    bad.amplitude[:, 5] = 0.0
    bad.phase[6] = np.inf
    bad.depth[7] = np.nan
    bad.quat_y[8] = np.inf
    bad.amplitude[1, 9] = np.nan
    bad.scale_v[10] = np.nan
    bad.opacity[11] = np.nan
    u = ctx.forward_tilted(problem(grid), scene_to_torch(bad))
    assert torch.count_nonzero(u).item() == 0
    assert ctx.stats()["n_culled"] == 12
    # culled Gaussians among valid ones change nothing
    keep = np.arange(12) % 3 == 0
    mix = sc.copy()
    for i in np.flatnonzero(~keep):
        mix.opacity[i] = 0.0
    a = to_numpy(ctx.forward_tilted(problem(grid), scene_to_torch(mix)))
    b = to_numpy(ctx.forward_tilted(problem(grid), scene_to_torch(sc.subset(np.flatnonzero(keep)))))
    assert np.array_equal(a, b)


def test_tilted_flipped_description_and_determinism(ctx):
    grid = Grid(96, 80, 2e-6, 2e-6, (520e-9, 450e-9))
    sc = gwsgen.make_tilted_scene(100, grid, 908, sigma_px=(1.0, 5.0), tilt_max_deg=20.0)
    fl = sc.copy()
    w, x, y, z = sc.quat_w.copy(), sc.quat_x.copy(), sc.quat_y.copy(), sc.quat_z.copy()
    fl.quat_w, fl.quat_x, fl.quat_y, fl.quat_z = -x, w, z, -y   # R -> R diag(1, -1, -1)
    g = scene_to_torch(sc)
    a = to_numpy(ctx.forward_tilted(problem(grid), g))
    a2 = to_numpy(ctx.forward_tilted(problem(grid), g))
    b = to_numpy(ctx.forward_tilted(problem(grid), scene_to_torch(fl)))
    assert np.array_equal(a, a2)
    e = rel_l2(b, a)
    log("tilted flipped description: %.3e" % e)
    assert e < 2e-6


def test_rotation_about_z_matches_in_plane_path(ctx):
    grid = Grid(160, 90, 8e-6, 8e-6, gwsgen.RGB)
    sc = gwsgen.make_tilted_scene(300, grid, 909, depth_range=(-10e-3, 10e-3), tilt_max_deg=0.0)
    # the in-plane Gaussians with Sigma = R S^2 R^T for the same float32 scales and rotation
    R = np.stack([oracle.holographics.quat_to_matrix([sc.quat_w[i], sc.quat_x[i], sc.quat_y[i], sc.quat_z[i]])
                  for i in range(sc.n)])
    su, sv = sc.scale_u.astype(np.float64), sc.scale_v.astype(np.float64)
    cxx = R[:, 0, 0] ** 2 * su ** 2 + R[:, 0, 1] ** 2 * sv ** 2
    cxy = R[:, 0, 0] * R[:, 1, 0] * su ** 2 + R[:, 0, 1] * R[:, 1, 1] * sv ** 2
    cyy = R[:, 1, 0] ** 2 * su ** 2 + R[:, 1, 1] ** 2 * sv ** 2
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    ip = gwsgen.Scene(mean_x=sc.mean_x, mean_y=sc.mean_y, depth=sc.depth, cov_xx=f(cxx), cov_xy=f(cxy),
                      cov_yy=f(cyy), opacity=sc.opacity, amplitude=sc.amplitude, phase=sc.phase)
    a = to_numpy(ctx.forward_tilted(problem(grid), scene_to_torch(sc)))
    b = to_numpy(ctx.forward(problem(grid), scene_to_torch(ip)))
    e = rel_l2(a, b)
    log("tilted path with tilt 0 vs in-plane path: %.3e" % e)
    assert e < 1e-5


def test_tilted_refuses_exact_blend_and_reference_wave(ctx):
    import paper_2505_06582_amd as gws
    grid = Grid(64, 48, 8e-6, 8e-6, (520e-9,))
    g = scene_to_torch(gwsgen.make_tilted_scene(4, grid, 910))
    with pytest.raises(gws.GwsError):
        ctx.forward_tilted(problem(grid, blend=gws.BLEND_EXACT), g)
    with pytest.raises(gws.GwsError):
        ctx.forward_tilted(problem(dataclasses.replace(grid, ref_nu=(100.0, 0.0))), g)


def test_tilted_workload_100k_sampled(ctx):
    """The bench's tilted workload (100k Gaussians, tilts up to 2 degrees, 1080 x 1920 x 3) in the
    launch configuration the bench times, on frequencies sampled by radius band."""
    nx, ny = 1920, 1080
    grid = Grid(nx, ny, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_tilted_scene(100_000, grid, 1005, depth_range=(-10e-3, 10e-3), tilt_max_deg=2.0)
    u, s = ctx.forward_tilted(problem(grid), scene_to_torch(scene), want_spectrum=True)
    mx, my, band, w = stratified_freqs(grid, 120, 911)
    log("tilted 100k: oracle at %d sampled frequencies" % mx.size)
    U = otl.spectrum(scene, grid, mx, my)
    sxf = oracle.signed_freq_index(nx)[mx]
    syf = oracle.signed_freq_index(ny)[my]
    ref = U * np.where((sxf + syf) % 2 == 0, 1.0, -1.0) / (nx * ny * grid.px * grid.py)
    got = to_numpy(s)[:, my, mx]
    e = rel_l2(got, ref)
    log("tilted 100k sampled spectrum: rel L2 %.3e" % e)
    assert e < TOL
    assert np.all(np.isfinite(to_numpy(u)))
    # eight parts per tile, added in part order: the same field again, bit for bit
    u2 = ctx.forward_tilted(problem(grid), scene_to_torch(scene))
    assert np.array_equal(to_numpy(u), to_numpy(u2))


# ---- adjoint -------------------------------------------------------------------------------

GRAD_TOL = 1e-4
BWD_CASES = [
    (96, 80, 8e-6, gwsgen.RGB, 40, 921, (2.0, 20.0), 2.0),
    (48, 40, 8e-6, (520e-9,), 20, 922, (1.0, 6.0), 3.0),
    (128, 96, 1e-6, (520e-9, 450e-9), 24, 923, (1.0, 4.0), 25.0),
    (64, 72, 0.25e-6, (633e-9,), 16, 924, (2.0, 6.0), 28.0),
    (64, 48, 8e-6, FOUR, 16, 930, (2.0, 20.0), 2.0),
]


def grads_rel(got, ref, names):
    out = {}
    for k in names:
        g = np.asarray(got[k], dtype=np.float64).ravel()
        r = np.asarray(ref[k], dtype=np.float64).ravel()
        out[k] = float(np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300))
    return out


@pytest.mark.parametrize("case", BWD_CASES, ids=["%dx%d-%dl-t%g" % (c[0], c[1], len(c[3]), c[7]) for c in BWD_CASES])
def test_tilted_backward_matches_oracle(ctx, case):
    import torch
    nx, ny, pitch, lams, n, seed, sig, tilt = case
    grid = Grid(nx, ny, pitch, pitch, lams)
    scene = gwsgen.make_tilted_scene(n, grid, seed, depth_range=(-10e-3, 10e-3), sigma_px=sig, tilt_max_deg=tilt)
    G = gwsgen.make_target(grid, seed + 1)
    got = ctx.backward_tilted(problem(grid), scene_to_torch(scene), torch.from_numpy(G).cuda())
    got = {k: to_numpy(v) for k, v in got.items()}
    ref = otg.backward(scene, grid, G)
    e = grads_rel(got, ref, otg.PARAMS)
    log("tilted backward %dx%d pitch %g C=%d tilt<=%g: %s" % (nx, ny, pitch, len(lams), tilt,
                                                             {k: "%.2e" % v for k, v in e.items()}))
    assert max(e.values()) < GRAD_TOL, e


def test_tilted_backward_split_bf16_transform(ctx):
    """The adjoint with the split-bf16 MFMA DFT taking the field gradient to Gs."""
    import torch
    import paper_2505_06582_amd as gws
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_tilted_scene(30, grid, 931, depth_range=(-10e-3, 10e-3))
    G = gwsgen.make_target(grid, 932)
    got = ctx.backward_tilted(problem(grid, xform=gws.XFORM_DFT_BF16X3), scene_to_torch(scene),
                              torch.from_numpy(G).cuda())
    got = {k: to_numpy(v) for k, v in got.items()}
    e = grads_rel(got, otg.backward(scene, grid, G), otg.PARAMS)
    log("tilted backward, split-bf16 transform: %s" % {k: "%.2e" % v for k, v in e.items()})
    assert max(e.values()) < GRAD_TOL, e


def test_render_tilted_autograd(ctx):
    """The torch.autograd.Function path (render_tilted + loss.backward) against the float64
    autograd oracle of the same loss, and bitwise against a direct backward_tilted call."""
    import torch
    import paper_2505_06582_amd as gws
    grid = Grid(64, 48, 8e-6, 8e-6, (520e-9, 638e-9))
    scene = gwsgen.make_tilted_scene(12, grid, 933, depth_range=(-5e-3, 5e-3), tilt_max_deg=10.0)
    t = gwsgen.make_target(grid, 934)   # a random target: no cancellation in the loss's gradient
    prob = problem(grid)
    params = {k: v.clone().requires_grad_(True) for k, v in scene_to_torch(scene).items()}
    u = gws.render_tilted(prob, *[params[k] for k in gws.TILTED_PARAMS])
    tt = torch.from_numpy(t.astype(np.complex64)).cuda()
    r = u - tt
    loss = torch.sum(r.real ** 2 + r.imag ** 2)   # its field gradient is exactly 2 (u - t)
    loss.backward()
    # the same step by hand: dL/dRe u + j dL/dIm u = 2 (u - t)
    direct = ctx.backward_tilted(prob, scene_to_torch(scene), (2 * (u.detach() - tt)).contiguous())
    for k in gws.TILTED_PARAMS:
        assert torch.equal(params[k].grad, direct[k]), k
    # the oracle's gradient for the same field gradient (the loss's own cancellations would
    # otherwise magnify the FP32 field's rounding)
    G = 2 * (to_numpy(u.detach()).astype(np.complex128) - t.astype(np.complex64).astype(np.complex128))
    e = grads_rel({k: to_numpy(params[k].grad) for k in gws.TILTED_PARAMS}, otg.backward(scene, grid, G), otg.PARAMS)
    log("render_tilted autograd: %s" % {k: "%.2e" % v for k, v in e.items()})
    assert max(e.values()) < GRAD_TOL, e


def test_tilted_backward_culled_zero_opacity_and_determinism(ctx):
    import torch
    grid = Grid(64, 48, 8e-6, 8e-6, gwsgen.RGB)
    sc = gwsgen.make_tilted_scene(10, grid, 925, tilt_max_deg=2.0)
    sc.opacity[0] = 0.0            # kept by the adjoint: its opacity gradient is not zero
    sc.scale_u[1] = 0.0            # culled: zeros
    sc.mean_x[2] = np.nan          # culled: zeros
    G = gwsgen.make_target(grid, 926)
    Gt = torch.from_numpy(G).cuda()
    g = scene_to_torch(sc)
    a = {k: to_numpy(v) for k, v in ctx.backward_tilted(problem(grid), g, Gt).items()}
    b = {k: to_numpy(v) for k, v in ctx.backward_tilted(problem(grid), g, Gt).items()}
    for k in otg.PARAMS:
        assert np.array_equal(a[k], b[k]), k
    for k in otg.PARAMS:
        v = a[k][:, 1:3] if k == "amplitude" else a[k][1:3]
        assert np.all(v == 0), k
    good = np.array([0] + list(range(3, 10)))
    ref = otg.backward(sc.subset(good), grid, G)
    got = {k: (a[k][:, good] if k == "amplitude" else a[k][good]) for k in otg.PARAMS}
    e = grads_rel(got, ref, otg.PARAMS)
    log("tilted backward with culled and zero-opacity Gaussians: %s" % {k: "%.2e" % v for k, v in e.items()})
    assert max(e.values()) < GRAD_TOL, e
    assert abs(a["opacity"][0]) > 0


def test_tilted_fp32_phase_mode(ctx):
    """phase_mode 1 (the carrier and ramp bases formed in FP32 instead of FP64): on a grid whose
    phases stay small it still meets the oracle, forward and backward, and differs from the FP64
    bases only by FP32 rounding."""
    import torch
    grid = Grid(96, 80, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_tilted_scene(40, grid, 928, depth_range=(-2e-3, 2e-3), tilt_max_deg=2.0)
    g = scene_to_torch(scene)
    u1 = to_numpy(ctx.forward_tilted(problem(grid, phase_mode=1), g))
    u0 = to_numpy(ctx.forward_tilted(problem(grid), g))
    ref = otl.forward(scene, grid)
    e1, e01 = rel_l2(u1, ref), rel_l2(u1, u0)
    G = gwsgen.make_target(grid, 929)
    got = {k: to_numpy(v) for k, v in ctx.backward_tilted(problem(grid, phase_mode=1), g,
                                                          torch.from_numpy(G).cuda()).items()}
    eg = grads_rel(got, otg.backward(scene, grid, G), otg.PARAMS)
    log("tilted phase_mode 1: field rel L2 %.2e (vs FP64 bases %.2e), gradients %s"
        % (e1, e01, {k: "%.2e" % v for k, v in eg.items()}))
    assert e1 < 1e-4 and e01 < 1e-4
    assert max(eg.values()) < 1e-3, eg


def test_tilted_backward_workload_100k_sampled(ctx):
    """Gradients of the tilted100k workload in the launch configuration the bench times, checked
    for eight Gaussians -- the narrowest and the widest, the most tilted, the deepest, and four
    drawn at random (each Gaussian's gradient depends only on its own term and the given field
    gradient, so the oracle computes it alone)."""
    import torch
    grid = Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_tilted_scene(100_000, grid, 1005, depth_range=(-10e-3, 10e-3), tilt_max_deg=2.0)
    G = gwsgen.make_target(grid, 1006)
    got = ctx.backward_tilted(problem(grid), scene_to_torch(scene), torch.from_numpy(G).cuda())
    got = {k: to_numpy(v) for k, v in got.items()}
    rng = np.random.default_rng(927)
    smin = np.minimum(scene.scale_u, scene.scale_v)
    smax = np.maximum(scene.scale_u, scene.scale_v)
    tilt = scene.quat_x.astype(np.float64) ** 2 + scene.quat_y.astype(np.float64) ** 2
    picks = [int(np.argmin(smin)), int(np.argmax(smax)), int(np.argmax(tilt)), int(np.argmax(np.abs(scene.depth)))]
    picks += [int(i) for i in rng.choice(scene.n, 4, replace=False)]
    refs = []
    for i in picks:
        log("tilted 100k backward: oracle for Gaussian %d" % i)
        refs.append(otg.backward(scene.subset([i]), grid, G))
    for k in otg.PARAMS:
        g = np.stack([np.ravel(got[k][:, i] if k == "amplitude" else got[k][i]) for i in picks])
        r = np.stack([np.ravel(ref[k]) for ref in refs])
        e = rel_l2(g, r)
        log("  %-9s rel L2 over the sample %.3e" % (k, e))
        # over the sample, and componentwise with an absolute floor of 1e-4 x the sample's norm
        assert e < 1e-4, (k, e)
        assert np.all(np.abs(g - r) <= 1e-3 * np.abs(r) + 1e-4 * np.linalg.norm(r)), (k, g, r)
