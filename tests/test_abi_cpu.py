"""The C-ABI library builds, loads and exports every entry point of include/gws.h, and its
host-side validation returns the documented codes -- all without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2505_06582_amd as gws

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gws.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gws_[a-z0-9_]+)\s*\(", text)))


def test_header_compiles_as_c_and_cxx(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "gws.h"\nint main(void){gws_problem p; gws_stats s; (void)p; (void)s; return GWS_ABI_VERSION == 4 ? 0 : 1;}\n')
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I", os.path.dirname(HEADER), str(src)])
    subprocess.check_call(["g++", "-std=c++17", "-Wall", "-Werror", "-fsyntax-only", "-x", "c++", "-I",
                           os.path.dirname(HEADER), str(src)])


def test_library_exports_every_declared_symbol():
    lib = gws.load_library()
    syms = declared_symbols()
    assert len(syms) >= 17
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    assert set(syms) == set(gws._SIGNATURES), set(syms) ^ set(gws._SIGNATURES)
    out = subprocess.check_output(["nm", "-D", "--defined-only", gws.LIB_PATH], text=True)
    exported = set(re.findall(r"\bT (gws_[a-z0-9_]+)", out))
    assert set(syms) <= exported


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gws.h"\nint main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n",'
                   ' sizeof(gws_problem), offsetof(gws_problem, eps_support), offsetof(gws_problem, tile_config),'
                   ' sizeof(gws_gaussians), sizeof(gws_output), sizeof(gws_grads), sizeof(gws_stats)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)], text=True).split()]
    want = [ctypes.sizeof(gws._Problem), gws._Problem.eps_support.offset, gws._Problem.tile_config.offset,
            ctypes.sizeof(gws._Gaussians), ctypes.sizeof(gws._Output), ctypes.sizeof(gws._Grads),
            ctypes.sizeof(gws._Stats)]
    assert got == want


def test_holographics_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "szh.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gws.h"\nint main(void){printf("%zu %zu %zu %zu %zu\\n",'
                   ' sizeof(gws_view), offsetof(gws_view, ray_to_holo), offsetof(gws_view, sh_degree),'
                   ' sizeof(gws_world_gaussians), sizeof(gws_plane_gaussians)); return 0;}\n')
    exe = tmp_path / "szh"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)], text=True).split()]
    want = [ctypes.sizeof(gws._View), gws._View.ray_to_holo.offset, gws._View.sh_degree.offset,
            ctypes.sizeof(gws._WorldGaussians), ctypes.sizeof(gws._PlaneGaussians)]
    assert got == want


def test_tilted_struct_layout_and_workspace_on_the_host(tmp_path):
    src = tmp_path / "szt.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gws.h"\nint main(void){printf("%zu %zu %zu\\n",'
                   ' sizeof(gws_tilted_gaussians), offsetof(gws_tilted_gaussians, quat_w),'
                   ' offsetof(gws_tilted_gaussians, phase)); return 0;}\n')
    exe = tmp_path / "szt"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)], text=True).split()]
    assert got == [ctypes.sizeof(gws._TiltedGaussians), gws._TiltedGaussians.quat_w.offset,
                   gws._TiltedGaussians.phase.offset]
    lib = gws.load_library()
    prob = gws.Problem(1920, 1080, lambdas=(638e-9, 520e-9, 450e-9))._c()
    sz, sz2 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.gws_workspace_size_tilted(None, ctypes.byref(prob), 1000, ctypes.byref(sz)) == 0
    assert lib.gws_workspace_size_tilted(None, ctypes.byref(prob), 100000, ctypes.byref(sz2)) == 0
    spec = 3 * 1920 * 1080 * 8
    assert spec + 1000 * 112 <= sz.value < spec + 1000 * 112 + 8192
    # each area rounded to 256 bytes; at 100000 Gaussians 8 partial spectra (a tile's Gaussians in
    # 8 parts, one per 8192) join the workspace
    assert 99000 * 112 - 1024 + 8 * spec <= sz2.value - sz.value < 99000 * 112 + 8 * spec + 8192
    assert lib.gws_workspace_size_tilted(None, ctypes.byref(prob), -1, ctypes.byref(sz)) == -1
    bad = gws.Problem(1921, 1080)._c()
    assert lib.gws_workspace_size_tilted(None, ctypes.byref(bad), 10, ctypes.byref(sz)) != 0
    assert lib.gws_forward_tilted(None, ctypes.byref(prob), None, None, None, 0, None) == -1
    assert lib.gws_backward_tilted(None, ctypes.byref(prob), None, None, None, None, 0, None) == -1


def test_holographics_validates_on_the_host():
    lib = gws.load_library()
    v = gws._View()
    v.fx = v.fy = 1000.0
    v.sh_degree = 3
    w = gws._WorldGaussians(0)
    pg = gws._PlaneGaussians()
    assert lib.gws_holographics(None, ctypes.byref(v), ctypes.byref(w), ctypes.byref(pg), None) == -1


def _check(prob):
    lib = gws.load_library()
    return lib.gws_check_problem(ctypes.byref(prob._c()))


def test_problem_validation_codes():
    lib = gws.load_library()
    assert lib.gws_abi_version() == 4
    ok = gws.Problem(1920, 1080, lambdas=(638e-9, 520e-9, 450e-9))
    assert _check(ok) == 0
    assert _check(gws.Problem(1921, 1080)) == -2          # odd
    assert _check(gws.Problem(1022, 1080)) == -2          # factor 7 * 73
    assert _check(gws.Problem(8, 1080)) == -2             # too small
    assert _check(gws.Problem(256, 256, pitch_x=0.0)) == -1
    assert _check(gws.Problem(256, 256, lambdas=())) == -1
    assert _check(gws.Problem(256, 256, lambdas=(1e-6,) * 5)) == -1
    assert _check(gws.Problem(256, 256, lambdas=(-5e-7,))) == -1
    assert _check(gws.Problem(256, 256, eps_support=0.5)) == -1
    assert _check(gws.Problem(256, 256, xform=7)) == -1
    assert _check(gws.Problem(256, 256, blend=gws.BLEND_EXACT)) == 0
    assert _check(gws.Problem(256, 256, blend=5)) == -1
    assert lib.gws_check_problem(None) == -1
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.gws_status_string(code)


def test_workspace_size_is_host_only_and_grows_with_n():
    lib = gws.load_library()
    prob = gws.Problem(1920, 1080, lambdas=(638e-9, 520e-9, 450e-9))._c()
    sizes = []
    for n in (0, 64, 10_000, 100_000):
        sz = ctypes.c_size_t()
        assert lib.gws_workspace_size(None, ctypes.byref(prob), n, ctypes.byref(sz)) == 0
        sizes.append(sz.value)
    assert sizes == sorted(sizes) and sizes[0] > 0
    sz = ctypes.c_size_t()
    assert lib.gws_workspace_size(None, ctypes.byref(prob), -1, ctypes.byref(sz)) == -1
    assert lib.gws_workspace_size(None, ctypes.byref(prob), 10, None) == -1


def test_exact_blending_workspace_sizes():
    lib = gws.load_library()
    prob = gws.Problem(1920, 1080, lambdas=(638e-9, 520e-9, 450e-9), blend=gws.BLEND_EXACT)._c()
    sz = ctypes.c_size_t()
    assert lib.gws_workspace_size(None, ctypes.byref(prob), 1000, ctypes.byref(sz)) == 0
    # one batch of 64 Gaussians in 32 full-grid complex64 images (two Gaussians each)
    # dominates; the adjoint packs its images the same way and needs no second set
    M = 1920 * 1080
    assert 32 * M * 8 <= sz.value < 64 * M * 8
    single = sz.value
    # batched exact blending runs scene after scene: the workspace of the largest scene
    offs = (ctypes.c_int64 * 4)(0, 1000, 1000, 1600)
    assert lib.gws_workspace_size_batched(None, ctypes.byref(prob), 3, offs, ctypes.byref(sz)) == 0
    assert sz.value == single


def test_dft_workspace_query_validates_shape_and_batch():
    lib = gws.load_library()
    sz = ctypes.c_size_t()
    assert lib.gws_dft_workspace_size(None, 1920, 1080, 3, 0, ctypes.byref(sz)) == 0 and sz.value == 0
    assert lib.gws_dft_workspace_size(None, 1920, 1080, 3, 1, ctypes.byref(sz)) == 0 and sz.value > 0
    assert lib.gws_dft_workspace_size(None, 1920, 1080, 0, 0, ctypes.byref(sz)) == -1
    assert lib.gws_dft_workspace_size(None, 1921, 1080, 1, 0, ctypes.byref(sz)) == -2   # odd
    assert lib.gws_dft_workspace_size(None, 1920, 1078, 1, 0, ctypes.byref(sz)) == -2   # factor 7
    # the whole batch's rows (and column slabs) must fit a 32-bit grid
    assert lib.gws_dft_workspace_size(None, 1920, 1080, (1 << 31) // 1920 + 1, 0, ctypes.byref(sz)) == -2
    assert lib.gws_dft_workspace_size(None, 1920, 1080, (1 << 31) // 1920, 0, ctypes.byref(sz)) == 0


def test_entry_points_reject_bad_arguments_without_a_device():
    lib = gws.load_library()
    h = ctypes.c_void_p()
    st = lib.gws_create(ctypes.byref(h), 0)
    if st == 0:
        lib.gws_destroy(h)
        pytest.skip("a gfx950 device is present")
    assert st == -5
    assert lib.gws_last_error(None)
    assert lib.gws_create(None, 0) == -1
    prob = gws.Problem(256, 256)._c()
    assert lib.gws_forward(None, ctypes.byref(prob), None, None, None, 0, None) == -1
    assert lib.gws_backward(None, ctypes.byref(prob), None, None, None, None, 0, None) == -1
    assert lib.gws_dft2d(None, 256, 256, 1, 1, 0, None, None, None, 0, None) == -1
    assert lib.gws_destroy(None) == 0


def test_display_entry_points_validate_on_the_host():
    lib = gws.load_library()
    assert lib.gws_dpac_workspace_size(3) >= 3 * 4 and lib.gws_dpac_workspace_size(3) % 256 == 0
    prob = gws.Problem(1920, 1080, lambdas=(638e-9, 520e-9, 450e-9))._c()
    sz = ctypes.c_size_t()
    img = 1920 * 1080 * 3 * 8
    # intensity output: the spectrum plus one complex plane buffer per plane (up to 32 per launch)
    assert lib.gws_focal_stack_workspace_size(None, ctypes.byref(prob), 8, 0, ctypes.byref(sz)) == 0
    assert sz.value >= 9 * img
    assert lib.gws_focal_stack_workspace_size(None, ctypes.byref(prob), 100, 0, ctypes.byref(sz)) == 0
    assert img * 33 <= sz.value < img * 34
    # complex output: the planes are the output itself
    assert lib.gws_focal_stack_workspace_size(None, ctypes.byref(prob), 8, gws.FS_COMPLEX_OUTPUT,
                                              ctypes.byref(sz)) == 0
    assert img <= sz.value < 2 * img
    assert lib.gws_focal_stack_workspace_size(None, ctypes.byref(prob), -1, 0, ctypes.byref(sz)) == -1
    assert lib.gws_focal_stack_workspace_size(None, ctypes.byref(prob), 1, 64, ctypes.byref(sz)) == -1
    wide = gws.Problem(8000, 64, lambdas=(520e-9,))._c()
    assert lib.gws_focal_stack_workspace_size(None, ctypes.byref(wide), 1, 0, ctypes.byref(sz)) == -2
    assert lib.gws_dpac_encode(None, 64, 64, 1, None, 0.0, None, None, 0, None) == -1
    assert lib.gws_focal_stack(None, ctypes.byref(prob), None, 1, None, 0, None, None, 0, None) == -1
