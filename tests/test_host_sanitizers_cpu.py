"""AddressSanitizer + UndefinedBehaviorSanitizer on host code, without a GPU:

* the C oracle (oracle/gws_oracle.c) built with gcc and both sanitizers, driven by
  tests/sanitize/oracle_driver.c (spectrum on a small odd grid, gradients of selected Gaussians);
* the host code of libgws: every csrc/*.hip compiled by hipcc with the sanitizers on the host
  side only (each flag behind -Xarch_host; the gfx950 code is built as usual), linked with
  tests/sanitize/lib_driver.c, which calls every host-only entry point with valid and invalid
  arguments.

Both must exit 0, print OK, and report nothing (UBSan aborts on the first finding:
-fno-sanitize-recover=all).  Leak checking is off: the HIP runtime keeps allocations until exit.
"""
import concurrent.futures
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2505_06582_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def run_clean(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "OK" in r.stdout, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", os.path.join(HERE, "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "gws_oracle.c"), "-lm", "-o", exe])
    run_clean(exe)


HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc") and shutil.which("hipcc") is None,
                    reason="hipcc is not installed")
def test_library_host_code_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = ([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
                "-Xclang", "-packed-fp32-ops"] + HOST_SAN + ["-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj])
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "lib_driver")
    r = subprocess.run([hipcc, "-O1", "-g"] + HOST_SAN + ["-I", INCLUDE, "-x", "c", os.path.join(HERE, "lib_driver.c"),
                                                          "-x", "none"] + objs + ["-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    run_clean(exe)
