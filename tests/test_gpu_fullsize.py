"""Parity at the full benchmark size (100k Gaussians, 1080x1920, 3 wavelengths), in the
launch configuration bench.py times, on outputs the FP64 oracle can compute one by one:
spectrum entries sampled by radius band (each an exact sum over all 100k Gaussians), the
transform stage against an FP64 inverse DFT of the GPU spectrum, and the gradients of 32
sampled Gaussians (each an exact dense sum over the whole grid) checked against the oracle
gradient and against FP64 central differences.  Also the 1M-Gaussian 2160x3840 precision
workload."""
import math
import sys

import numpy as np
import pytest

import gwsgen
import oracle
from gpu_util import (check_spectrum_and_transform, oracle_dft_ready, physical_spectrum, problem, rel_l2,
                      scene_to_torch, stratified_errors, stratified_freqs, to_numpy)

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2505_06582_amd as gws
    assert torch.cuda.is_available()
    return gws.context(0)


@pytest.fixture(scope="module")
def bench_scene():
    return gwsgen.workload("fwdbwd100k")


def test_fullsize_forward_sampled_by_band(ctx, bench_scene):
    """Spectrum entries sampled in every radius band (the multi-chunk tiles around DC, three
    rings and the band next to Nyquist), each an exact FP64 sum over all 100k Gaussians, and
    the GPU field against an FP64 inverse DFT of the GPU spectrum."""
    scene, grid = bench_scene
    log("full-size forward: 100k Gaussians 1080x1920x3")
    field, spec = ctx.forward(problem(grid), scene_to_torch(scene), want_spectrum=True)
    st = ctx.stats()
    log("  %d work items, chunk %d" % (st["n_items"], st["chunk"]))
    check_spectrum_and_transform(scene, grid, to_numpy(field), to_numpy(spec), 1024, 31, "fwdbwd100k")


def test_fullsize_backward_32_sampled_gaussians(ctx, bench_scene):
    import torch
    scene, grid = bench_scene
    log("full-size backward: 32 sampled Gaussians of 100k")
    G = gwsgen.make_target(grid, 2003)
    got = ctx.backward(problem(grid), scene_to_torch(scene), torch.from_numpy(G).cuda(), want_depth=False)
    got = {k: to_numpy(v) for k, v in got.items() if v is not None}
    sel = np.random.default_rng(7).choice(scene.n, 32, replace=False)
    gs = oracle.spectrum_grad_from_field_grad(G.astype(np.complex128), grid)
    ref = oracle.param_grads_from_spectrum_grad(scene, grid, gs, sel)
    for k in ("mean_x", "mean_y", "cov_xx", "cov_xy", "cov_yy", "opacity", "phase", "amplitude"):
        g = got[k][:, sel] if k == "amplitude" else got[k][sel]
        e = rel_l2(g, ref[k])
        log("  %-9s rel L2 vs oracle gradient %.3e" % (k, e))
        assert e < 1e-4, (k, e)
    # FP64 central differences of the linear functional Re<G, u(theta)> for each sampled
    # Gaussian, in the spectrum domain (exactly equal by the adjoint identity)
    def functional(s1):
        U = oracle.spectrum(s1, grid)
        return float(np.real(np.vdot(gs, U)))
    checks = 0
    for j, i in enumerate(sel[:8]):
        base = scene.subset([i])
        base = gwsgen.Scene(**{k: v.astype(np.float64) for k, v in base.fields().items()})
        for k, scale in (("mean_x", 8e-6), ("cov_xx", None), ("cov_xy", None), ("opacity", None), ("phase", 1.0)):
            v = float(getattr(base, k)[0])
            h = 1e-4 * (scale if scale else max(abs(v), 1e-14))
            plus, minus = base.copy(), base.copy()
            getattr(plus, k)[0] = v + h
            getattr(minus, k)[0] = v - h
            fd = (functional(plus) - functional(minus)) / (2 * h)
            gpu = float(got[k][i])
            # componentwise 1e-3, with an absolute floor of 1e-4 x the norm of the group over the sample
            norm = float(np.linalg.norm(got[k][sel]))
            assert abs(gpu - fd) <= 1e-3 * abs(fd) + 1e-4 * norm, (k, i, gpu, fd)
            checks += 1
    log("  %d FD checks passed" % checks)


def test_precision_workload_1m_gaussians_sampled(ctx):
    """1M Gaussians at 2160x3840x3 with 5% far off-axis at 20-50 mm: sampled spectrum entries
    against exact FP64 sums; the plain-FP32 phase base (phase_mode 1) is shown to be worse."""
    scene, grid = gwsgen.workload("precision1m")
    log("precision workload: 1M Gaussians 2160x3840x3")
    g = scene_to_torch(scene)
    field, spec = ctx.forward(problem(grid), g, want_spectrum=True)
    field, spec = to_numpy(field), to_numpy(spec)
    mx, my, band, w = stratified_freqs(grid, 256, 41)
    sx = oracle.signed_freq_index(grid.nx)[mx]
    sy = oracle.signed_freq_index(grid.ny)[my]
    ref = oracle_dft_ready(scene, grid, mx, my)
    e, per, plain = stratified_errors(spec[:, my, mx], ref, band, w)
    log("  all 1M: spectrum rel L2 (band-weighted estimate) %.3e; relative L2 within each band %s"
        % (e, {k: "%.2e" % v for k, v in plain.items()}))
    assert all(v < 1.0 for v in per.values()), (plain, per)
    e_xf = rel_l2(field, oracle.field_from_spectrum(physical_spectrum(spec, grid), grid))
    log("  transform stage rel L2 %.3e" % e_xf)
    assert e_xf < 2e-6
    del field
    # the far subset alone
    far = np.flatnonzero(np.abs(scene.depth) > 15e-3)
    sub = scene.subset(far)
    _, spec_far = ctx.forward(problem(grid), scene_to_torch(sub), want_spectrum=True)
    _, spec_far32 = ctx.forward(problem(grid, phase_mode=1), scene_to_torch(sub), want_spectrum=True)
    ref_f = oracle_dft_ready(sub, grid, mx, my)
    e_far = rel_l2(to_numpy(spec_far)[:, my, mx], ref_f)
    e_far32 = rel_l2(to_numpy(spec_far32)[:, my, mx], ref_f)
    # away from DC (|m'| > 400 index units) the phase ramp m'.r reaches hundreds of revolutions
    hi = np.flatnonzero(np.hypot(sx, sy) > 400)
    e_hi = rel_l2(to_numpy(spec_far)[:, my[hi], mx[hi]], ref_f[:, hi])
    e_hi32 = rel_l2(to_numpy(spec_far32)[:, my[hi], mx[hi]], ref_f[:, hi])
    log("  sampled rel L2: all %.3e, far subset %.3e (FP32 base %.3e); far subset at |m'| > 400: %.3e "
        "(FP32 base %.3e, %d samples)" % (e, e_far, e_far32, e_hi, e_hi32, hi.size))
    assert e < 1e-5 and e_far < 1e-5 and e_hi < 1e-5
    assert e_hi32 > 10 * e_hi
