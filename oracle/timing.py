"""Host timing of the FP64 oracle (the CPU baseline beside the GPU numbers).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: used by ``bench.py``'s CPU-baseline
leg and run by hand for the full-size timings; the product library never imports it.

Two measurements, both of the oracle exactly as the parity tests use it (dense: every
Gaussian at every requested frequency, no culling):

* ``sampled``: the order-invariant sum (Eq. 12) at a random sample of frequencies x every
  Gaussian x every wavelength, one dense centred DFT of the grid, and the dense gradients of a
  random sample of Gaussians; extrapolated to one forward + backward hologram of the workload
  (frequencies and gradient Gaussians scale linearly; the transform runs 2 x n_lambda times);
* ``full``: the whole forward (the spectrum at every frequency, then the inverse transform),
  timed end to end.

    python -m oracle.timing --workload fwd10k --mode full
    OMP_NUM_THREADS=1 python -m oracle.timing --workload fwdbwd100k --mode sampled --freqs 256 --grads 8

Prints one JSON line with the host's CPU model and the threads used.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def host_info() -> dict:
    """CPU model, logical CPUs of the host, the CPUs this process may use, and the thread count
    the oracle's OpenMP loops run with (OMP_NUM_THREADS when set, else every allowed CPU)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = allowed
    if os.environ.get("OMP_NUM_THREADS"):
        threads = min(allowed, int(os.environ["OMP_NUM_THREADS"]))
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "allowed_cpus": allowed, "threads": threads}


def sampled(scene, grid, n_freq: int, n_grad: int, seed: int = 4242) -> dict:
    """Time the oracle on a bounded sample and extrapolate to one fwd+bwd hologram (seconds)."""
    import gwsgen
    import oracle
    rng = np.random.default_rng(seed)
    M = grid.nx * grid.ny
    mx = rng.integers(0, grid.nx, n_freq).astype(np.int32)
    my = rng.integers(0, grid.ny, n_freq).astype(np.int32)
    t0 = time.perf_counter()
    oracle.spectrum(scene, grid, mx, my)
    t_fwd = time.perf_counter() - t0
    g1 = gwsgen.Grid(grid.nx, grid.ny, grid.px, grid.py, (grid.lambdas[0],))
    G1 = gwsgen.make_target(g1, 3).astype(np.complex128)
    t0 = time.perf_counter()
    gs1 = oracle.spectrum_grad_from_field_grad(G1, g1)
    t_xf = time.perf_counter() - t0
    sel = rng.choice(scene.n, n_grad, replace=False)
    gs = np.repeat(gs1, grid.n_lambda, axis=0)
    t0 = time.perf_counter()
    oracle.param_grads_from_spectrum_grad(scene, grid, gs, sel)
    t_bwd = time.perf_counter() - t0
    full = t_fwd * M / n_freq + t_bwd * scene.n / n_grad + 2 * grid.n_lambda * t_xf
    evals = 2.0 * scene.n * M * grid.n_lambda   # dense Gaussian.freq-px evaluations, forward + backward
    return {"mode": "sampled", "freqs": n_freq, "grad_gaussians": n_grad, "t_fwd_sample_s": t_fwd,
            "t_transform_s": t_xf, "t_bwd_sample_s": t_bwd, "extrapolated_s_per_hologram": full,
            "holograms_per_s": 1.0 / full, "dense_evals_per_s": evals / full}


def full_forward(scene, grid) -> dict:
    """Time the oracle's whole forward (every frequency, then the inverse transform)."""
    import oracle
    t0 = time.perf_counter()
    U = oracle.spectrum(scene, grid)
    t_spec = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.field_from_spectrum(U, grid)
    t_xf = time.perf_counter() - t0
    evals = float(scene.n) * grid.nx * grid.ny * grid.n_lambda
    return {"mode": "full", "t_spectrum_s": t_spec, "t_transform_s": t_xf, "t_forward_s": t_spec + t_xf,
            "dense_evals_per_s": evals / t_spec}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="fwdbwd100k", help="a gwsgen workload, or batched16:<scene>")
    ap.add_argument("--mode", choices=("sampled", "full"), default="sampled")
    ap.add_argument("--freqs", type=int, default=4096)
    ap.add_argument("--grads", type=int, default=640)
    args = ap.parse_args()
    import gwsgen
    if args.workload.startswith("batched16:"):
        i = int(args.workload.split(":")[1])
        n = gwsgen.batched_counts(16)[i]
        grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
        scene = gwsgen.make_scene(n, grid, 5000 + i, depth_range=(-10e-3, 10e-3))
    else:
        scene, grid = gwsgen.workload(args.workload)
    out = {"workload": args.workload, "gaussians": scene.n, "ny": grid.ny, "nx": grid.nx,
           "n_lambda": grid.n_lambda}
    out.update(host_info())
    if args.mode == "sampled":
        out.update(sampled(scene, grid, min(args.freqs, grid.nx * grid.ny), min(args.grads, scene.n)))
    else:
        out.update(full_forward(scene, grid))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
