"""CPU-only tests of the binding's argument checks: every tensor handed to the library is
checked against the problem's sizes before any C call, since the kernels index the raw
pointers by the problem's sizes alone.  The Context used here has no library handle, so a
check that let a bad argument through would fail with AttributeError instead of ValueError."""
import numpy as np
import pytest
import torch

import gwsgen
import paper_2505_06582_amd as gws


def cpu_scene(n=5, C=3):
    grid = gwsgen.Grid(32, 16, 8e-6, 8e-6, gwsgen.RGB[:C])
    sc = gwsgen.make_scene(n, grid, 3, depth_range=(-1e-3, 1e-3))
    return grid, {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in sc.fields().items()}


def shell():
    """A Context with no device and no library: any call that reaches the C side raises AttributeError."""
    ctx = object.__new__(gws.Context)
    ctx.lib = None
    ctx.handle = None
    ctx.device = 0
    ctx._ws = None
    ctx.torch_device = torch.device("cpu")
    return ctx


def test_check_gaussians_sizes():
    grid, g = cpu_scene()
    assert gws.check_gaussians(g, 3) == 5
    bad = dict(g)
    bad["mean_y"] = torch.zeros(6)
    with pytest.raises(ValueError, match="mean_y"):
        gws.check_gaussians(bad, 3)
    bad = dict(g)
    bad["amplitude"] = g["amplitude"].t().contiguous()  # (n, C) instead of (C, n)
    with pytest.raises(ValueError, match="amplitude"):
        gws.check_gaussians(bad, 3)
    bad = dict(g)
    bad["amplitude"] = torch.zeros(2 * 5)
    with pytest.raises(ValueError, match="amplitude"):
        gws.check_gaussians(bad, 3)
    # a flat channel-major amplitude of n_lambda * n elements is accepted
    ok = dict(g)
    ok["amplitude"] = g["amplitude"].reshape(-1)
    assert gws.check_gaussians(ok, 3) == 5
    bad = dict(g)
    del bad["phase"]
    with pytest.raises(ValueError, match="phase"):
        gws.check_gaussians(bad, 3)


def test_check_tensor_shape_dtype_layout_device():
    t = torch.zeros((3, 4, 5), dtype=torch.complex64)
    with pytest.raises(ValueError, match="shape"):
        gws.check_tensor(t, "out", (3, 4, 6), "complex64")
    with pytest.raises(ValueError, match="complex64"):
        gws.check_tensor(t.real.contiguous(), "out", (3, 4, 5), "complex64")
    with pytest.raises(ValueError, match="contiguous"):
        gws.check_tensor(t.transpose(1, 2), "out", (3, 5, 4), "complex64")
    assert gws.check_tensor(t, "out", (3, 4, 5), "complex64") is t
    with pytest.raises(ValueError, match="CUDA"):
        gws._dptr(t)
    with pytest.raises(ValueError, match="required"):
        gws.check_tensor(None, "out", (3, 4, 5), "complex64")


def test_check_offsets():
    assert gws.check_offsets(np.array([0, 2, 5]), 5) == [0, 2, 5]
    for bad in ([0, 3, 2, 5], [1, 5], [0, 4], [0], list(range(0, 67))):
        with pytest.raises(ValueError):
            gws.check_offsets(bad, bad[-1] if bad[-1] != 4 else 5)


def test_forward_and_backward_reject_bad_sizes_before_the_library():
    grid, g = cpu_scene()
    prob = gws.Problem.from_grid(grid)
    ctx = shell()
    bad = dict(g)
    bad["cov_xy"] = torch.zeros(4)
    with pytest.raises(ValueError, match="cov_xy"):
        ctx.forward(prob, bad)
    with pytest.raises(ValueError, match="cov_xy"):
        ctx.backward(prob, bad, torch.zeros((3, grid.ny, grid.nx), dtype=torch.complex64))
    with pytest.raises(ValueError, match="out"):
        ctx.forward(prob, g, out=torch.zeros((3, grid.ny, grid.nx + 2), dtype=torch.complex64))
    with pytest.raises(ValueError, match="grad_field"):
        ctx.backward(prob, g, torch.zeros((2, grid.ny, grid.nx), dtype=torch.complex64))
    # gradient outputs must match their parameters
    G = torch.zeros((3, grid.ny, grid.nx), dtype=torch.complex64)
    out = {k: torch.zeros_like(v) for k, v in g.items()}
    out["amplitude"] = torch.zeros(5)
    with pytest.raises(ValueError, match="grad amplitude"):
        ctx.backward(prob, g, G, out=out)
    # right sizes on host memory: still rejected before any C call
    with pytest.raises(ValueError, match="CUDA"):
        ctx.forward(prob, g)


def test_batched_calls_reject_bad_offsets_and_shapes():
    grid, g = cpu_scene(n=6)
    prob = gws.Problem.from_grid(grid)
    ctx = shell()
    with pytest.raises(ValueError, match="offsets"):
        ctx.forward_batched(prob, g, [0, 2, 7])
    with pytest.raises(ValueError, match="out"):
        ctx.forward_batched(prob, g, [0, 2, 6], out=torch.zeros((3, 3, grid.ny, grid.nx), dtype=torch.complex64))
    with pytest.raises(ValueError, match="grad_fields"):
        ctx.backward_batched(prob, g, [0, 2, 6], torch.zeros((3, 3, grid.ny, grid.nx), dtype=torch.complex64))


def test_other_entry_points_reject_bad_shapes():
    grid, _ = cpu_scene()
    prob = gws.Problem.from_grid(grid)
    ctx = shell()
    f = torch.zeros((3, grid.ny, grid.nx), dtype=torch.complex64)
    with pytest.raises(ValueError, match="target"):
        ctx.l2_loss_grad(f, torch.zeros((3, grid.ny, grid.nx - 2), dtype=torch.complex64))
    with pytest.raises(ValueError, match="out"):
        ctx.dpac_encode(f, out=torch.zeros((3, grid.ny, grid.nx), dtype=torch.complex64))
    with pytest.raises(ValueError, match="inp"):
        ctx.focal_stack(prob, f, [0.0], phase_input=True)
    with pytest.raises(ValueError, match="out"):
        ctx.dft2d(f, +1, out=torch.zeros((3, grid.ny, grid.nx), dtype=torch.complex128))
    n = 4
    world = {"mean": torch.zeros((n, 3)), "quat": torch.zeros((n, 4)), "scale": torch.zeros((n, 3)),
             "opacity_sh": torch.zeros((n, 9))}
    view = dict(gwsgen.make_camera(1), sh_degree=3)
    with pytest.raises(ValueError, match="opacity_sh"):
        ctx.holographics(view, world)


def test_render_refuses_four_wavelength_depth_gradient_at_forward_time():
    # the library's order-invariant adjoint takes the depth gradient for at most three
    # wavelengths; render() says so when the graph is built, before any device work
    import torch
    prob = gws.Problem(64, 48, lambdas=(638e-9, 520e-9, 450e-9, 405e-9))
    p = lambda: torch.zeros(3, requires_grad=True)
    with pytest.raises(ValueError, match="depth gradient"):
        gws.render(prob, p(), p(), p(), p(), p(), p(), p(), torch.zeros(4, 3, requires_grad=True), p())


def test_tilted_calls_reject_bad_sizes_before_the_library():
    grid = gwsgen.Grid(32, 16, 8e-6, 8e-6, gwsgen.RGB)
    sc = gwsgen.make_tilted_scene(5, grid, 4)
    g = {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in sc.fields().items()}
    prob = gws.Problem.from_grid(grid)
    ctx = shell()
    bad = dict(g)
    bad["quat_z"] = torch.zeros(4)
    with pytest.raises(ValueError, match="quat_z"):
        ctx.forward_tilted(prob, bad)
    missing = {k: v for k, v in g.items() if k != "scale_v"}
    with pytest.raises(ValueError, match="scale_v"):
        ctx.forward_tilted(prob, missing)
    with pytest.raises(ValueError, match="out"):
        ctx.forward_tilted(prob, g, out=torch.zeros((3, grid.ny, grid.nx + 2), dtype=torch.complex64))
    with pytest.raises(ValueError, match="grad_field"):
        ctx.backward_tilted(prob, g, torch.zeros((2, grid.ny, grid.nx), dtype=torch.complex64))
    G = torch.zeros((3, grid.ny, grid.nx), dtype=torch.complex64)
    out = {k: torch.zeros_like(v) for k, v in g.items()}
    out["amplitude"] = torch.zeros(5)
    with pytest.raises(ValueError, match="amplitude"):
        ctx.backward_tilted(prob, g, G, out=out)
    with pytest.raises(ValueError, match="CUDA"):
        ctx.forward_tilted(prob, g)


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr)
