#!/usr/bin/env python3
"""Throughput of the Gaussian Wave Splatting hot path on one MI355X.

Workload: 100,000 random in-plane Gaussians, 1080 x 1920 hologram, 3 wavelengths
(638 / 520 / 450 nm), 8 um pitch.  One step = forward (preprocess, sort, bin, spectrum
accumulation, inverse FFT) + L2 loss against a random complex target + backward
(forward FFT of the field gradient, adjoint accumulation, chain rule): parameters on the
device to gradients on the device, every step in the HIP library.

Prints one JSON line: holograms/s (fwd+bwd steps per second; gradients with respect to mean, covariance,
opacity, amplitude and phase) with the roofline of the
dominant kernel measured by HIP events on the library's stream, and the FP64 CPU oracle
timed on a bounded sample on this host.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "holograms/s @1080x1920x3λ,100k Gaussians fwd+bwd; Gaussian·freq-px evals/s"
# Transcendental peak of MI355X from unit counts and clock: a SIMD issues a wave64 v_exp_f32,
# v_sin_f32 or v_cos_f32 in two quad-cycles (8 clocks, no dual issue), i.e. 8 lanes per clock:
# 256 CUs x 4 SIMDs x 8 lanes x 2.4 GHz = 19.66 T ops/s.  Plain FP32 VALU ops take one
# quad-cycle and two can issue together (256 x 4 x 32 x 2.4 GHz = 78.6 T ops/s, 157.3 TFLOP/s FMA).
PEAK_TRANS = 256 * 4 * 8 * 2.4e9
PEAK_HBM = 8.0e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def ellipse_support_points(scene, grid, eps=1e-7):
    """Algorithmic work: lattice frequencies inside each Gaussian's eps-support ellipse (area)."""
    import numpy as np
    tau = math.log(1.0 / eps)
    Wx, Wy = grid.nx * grid.px, grid.ny * grid.py
    sxx = scene.cov_xx.astype(np.float64)
    sxy = scene.cov_xy.astype(np.float64)
    syy = scene.cov_yy.astype(np.float64)
    # exponent 2 pi^2 nu^T S nu <= tau; in index units nu = m / W
    a = 2 * math.pi ** 2 * sxx / Wx ** 2
    b = 2 * math.pi ** 2 * sxy / (Wx * Wy)
    c = 2 * math.pi ** 2 * syy / Wy ** 2
    valid = (sxx > 0) & (sxx * syy - sxy * sxy > 0) & (scene.opacity != 0)
    area = np.where(valid, math.pi * tau / np.sqrt(np.maximum(a * c - b * b, 1e-300)), 0.0)
    return float(np.minimum(area, grid.nx * grid.ny).sum())


def cpu_baseline(scene, grid, workload):
    """The FP64 oracle timed on this host on a bounded sample, extrapolated to one fwd+bwd
    hologram: on every allowed core (in this process) and on one core (a child process with one
    OpenMP and one BLAS thread, on a smaller sample).  About 20 s of host time."""
    import subprocess
    import oracle.timing as ot
    allc = ot.sampled(scene, grid, 4096, 640)
    info = ot.host_info()
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    one = None
    try:
        r = subprocess.run([sys.executable, "-m", "oracle.timing", "--workload", workload, "--mode", "sampled",
                            "--freqs", "256", "--grads", "16"], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=300)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
        else:
            log("bench: single-core oracle run failed: %s" % r.stderr[-500:])
    except (subprocess.TimeoutExpired, ValueError) as e:
        log("bench: single-core oracle run failed: %s" % e)
    out = {
        "value": allc["holograms_per_s"], "unit": "holograms/s", "cores": info["threads"], "kind": "oracle",
        "cpu_model": info["cpu_model"], "host_cpus": info["host_cpus"], "allowed_cpus": info["allowed_cpus"],
        "dense_evals_per_s": allc["dense_evals_per_s"],
        "sample": ("FP64 C/OpenMP oracle (dense: every Gaussian at every frequency): Eq. 12 at %d random "
                   "frequencies x %d Gaussians x %d wavelengths (%.1f s), one dense centred DFT of %dx%d "
                   "(%.1f s, x%d for inverse+adjoint per wavelength), dense gradients of %d random Gaussians "
                   "over the full grid (%.1f s); extrapolated to the full fwd+bwd hologram = %.0f s"
                   % (allc["freqs"], scene.n, grid.n_lambda, allc["t_fwd_sample_s"], grid.ny, grid.nx,
                      allc["t_transform_s"], 2 * grid.n_lambda, allc["grad_gaussians"], allc["t_bwd_sample_s"],
                      allc["extrapolated_s_per_hologram"])),
    }
    if one is not None:
        out["single_core"] = {"value": one["holograms_per_s"], "unit": "holograms/s", "cores": one["threads"],
                              "dense_evals_per_s": one["dense_evals_per_s"],
                              "sample": "%d frequencies, gradients of %d Gaussians; extrapolated %.0f s per hologram"
                                        % (one["freqs"], one["grad_gaussians"], one["extrapolated_s_per_hologram"])}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fwdbwd100k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile-config", type=int, default=0, help="0: tuned/default tiling; k: explicit tiling k")
    ap.add_argument("--phase-mode", type=int, default=0,
                    help="0: exact phase bases (the product setting); 1: plain FP32 bases (precision study)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy 1 GiB device-to-device 3 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X; sharding a hologram "
              "or a batch across GPUs is not implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws

    if args.copy_calibration and args.workload != "fwdbwd100k":
        copy_calibration()
    if args.workload == "batched16":
        return bench_batched(args)
    if args.workload == "exact1k":
        return bench_exact(args)
    if args.workload == "paper15k":
        return bench_paper(args)
    if args.workload == "holo100k":
        return bench_holo(args)
    if args.workload == "focal8":
        return bench_focal(args)
    if args.workload == "precision1m":
        return bench_precision(args)
    if args.workload == "fwd10k":
        return bench_fwd10k(args)
    if args.workload == "tilted100k":
        return bench_tilted(args)
    if args.workload == "sizes":
        return bench_sizes(args)
    log("bench: generating workload %s" % args.workload)
    scene, grid = gwsgen.workload(args.workload)
    target = gwsgen.make_target(grid, 2003)
    prob = gws.Problem.from_grid(grid, tile_config=args.tile_config, phase_mode=args.phase_mode)
    ctx = gws.context(0)
    dev = torch.device("cuda", 0)
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.fields().items()}
    t = torch.from_numpy(target).to(dev)
    field = torch.empty((grid.n_lambda, grid.ny, grid.nx), dtype=torch.complex64, device=dev)
    G = torch.empty_like(field)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    grads = {k: torch.empty_like(v) for k, v in g.items()}

    def step():
        ctx.forward(prob, g, out=field)
        ctx.l2_loss_grad(field, t, grad=G, loss=loss)
        ctx.backward(prob, g, G, out=grads, want_depth=False)

    # counts of the evaluated work (deterministic for the scene)
    log("bench: counting work")
    ctx.forward(prob, g, out=field)
    st_f = ctx.stats()
    ctx.l2_loss_grad(field, t, grad=G, loss=loss)
    ctx.backward(prob, g, G, out=grads, want_depth=False)
    st_b = ctx.stats()
    torch.cuda.synchronize()

    peaks = ctx.measure_peaks()
    log("bench: measured peaks %s" % {k: "%.3g" % v for k, v in peaks.items()})

    log("bench: warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.read_profile()
    ctx.set_profiling(True)
    log("bench: timing %d steps" % args.steps)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    evs[0].record()
    for i in range(args.steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = evs[0].elapsed_time(evs[-1]) / args.steps
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    ms_median = per_step[len(per_step) // 2] if len(per_step) % 2 else 0.5 * (per_step[len(per_step) // 2 - 1] + per_step[len(per_step) // 2])
    ctx.set_profiling(False)
    prof = ctx.read_profile()
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}
    log("bench: %.3f ms/step (wall %.3f ms/step); stages %s" % (
        ms_step, 1e3 * wall / args.steps, {k: round(v, 3) for k, v in stage_ms.items()}))

    C = grid.n_lambda
    M = grid.nx * grid.ny
    support = ellipse_support_points(scene, grid)          # (Gaussian, frequency) pairs inside eps-support
    evals_alg = support * C                                # Gaussian.freq-px evaluations per pass
    trans_per_pair = 1 + 2 * C                             # one exp2, a sin and a cos per wavelength
    fwd_pairs_eval = st_f["n_pairs_evaluated"]             # (Gaussian, frequency) pairs evaluated
    bwd_pairs_eval = st_b["n_pairs_evaluated"]
    kern = {}
    t_acc = stage_ms["accumulate"] * 1e-3
    t_adj = stage_ms["adjoint"] * 1e-3
    if t_acc > 0:
        kern["accumulate"] = {
            "ms": stage_ms["accumulate"], "bound": "alu",
            "achieved": support * trans_per_pair / t_acc / 1e12, "peak": PEAK_TRANS / 1e12, "unit": "TOP/s",
            "frac": support * trans_per_pair / t_acc / PEAK_TRANS,
            "evaluated_frac": fwd_pairs_eval * trans_per_pair / t_acc / PEAK_TRANS,
            "evaluated_over_support": fwd_pairs_eval / support}
    if t_adj > 0:
        kern["adjoint"] = {
            "ms": stage_ms["adjoint"], "bound": "alu",
            "achieved": support * trans_per_pair / t_adj / 1e12, "peak": PEAK_TRANS / 1e12, "unit": "TOP/s",
            "frac": support * trans_per_pair / t_adj / PEAK_TRANS,
            "evaluated_frac": bwd_pairs_eval * trans_per_pair / t_adj / PEAK_TRANS,
            "evaluated_over_support": bwd_pairs_eval / support}
    for name in ("xform_inverse", "xform_forward"):
        if stage_ms[name] > 0:
            # algorithmic bytes: one read + one write of C x M complex64 (any 2D transform must
            # move that much); the two-pass design (rows, then columns) moves twice as much
            bytes_alg = 2 * C * M * 8
            t = stage_ms[name] * 1e-3
            kern[name] = {"ms": stage_ms[name], "bound": "hbm", "achieved": bytes_alg / t / 1e9,
                          "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": bytes_alg / t / PEAK_HBM,
                          "algorithmic_bytes": bytes_alg, "two_pass_bytes": 2 * bytes_alg,
                          "two_pass_GB_per_s": 2 * bytes_alg / t / 1e9}
    for name, k in kern.items():
        meas = peaks["trans_ops_per_s"] / 1e12 if k["bound"] == "alu" else peaks["hbm_bytes_per_s"] / 1e9
        k["peak_measured"] = meas
        k["frac_of_measured"] = k["achieved"] / meas
    dom = max(("accumulate", "adjoint"), key=lambda k: stage_ms[k])
    d = kern[dom]
    roofline = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
                "frac": d["frac"], "traffic": None, "kernel": dom,
                "peak_measured": d["peak_measured"], "frac_of_measured": d["frac_of_measured"],
                "work_per_launch": "%.4g transcendental ops (= %.4g (Gaussian, frequency) pairs inside the "
                                   "1e-7 support x (1 exp2 + 2 x %d sin/cos))" % (support * trans_per_pair, support, C)}

    value = 1e3 / ms_step
    out = {
        "metric": METRIC, "value": value, "unit": "holograms/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "ms_per_step_median": ms_median,
        "ms_per_step_min": per_step[0], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%d random in-plane Gaussians, %dx%d hologram, %d wavelengths (638/520/450 nm), "
                               "8 um pitch, forward + L2 loss + backward" % (scene.n, grid.ny, grid.nx, C),
                   "gaussians": scene.n, "ny": grid.ny, "nx": grid.nx, "n_lambda": C, "eps_support": 1e-7,
                   "tile_config": st_b["tile_config"],
                   "parallelism": "single GPU"},
        "evals_per_s": 2 * evals_alg / (ms_step * 1e-3),
        "evals_per_s_note": "Gaussian.freq-px evaluations inside the eps-support, forward + backward, per second",
        "dense_equiv_evals_per_s": 2 * scene.n * M * C / (ms_step * 1e-3),
        "stage_ms": stage_ms,
        "kernels": kern,
        "measured_peaks": peaks,
        "roofline": roofline,
    }
    tr = traffic_from_profiles(dom)
    if tr is not None:
        roofline["traffic"] = tr
    if args.copy_calibration:
        copy_calibration()
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(scene, grid, args.workload)
    print(json.dumps(out), flush=True)


def copy_calibration(nbytes=1 << 30, reps=3):
    """Plain device-to-device copies of known size for scaling the HBM byte counters."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()


# Sources whose change invalidates a kernel's stored counter readings: the kernel itself, the
# binning that orders its work items, and the shared record layouts.
TRAFFIC_SOURCES = {
    "adjoint": ("k_adjoint.hip", "k_prep.hip", "gws_internal.h"),
    "accumulate": ("k_accum.hip", "k_prep.hip", "gws_internal.h"),
}


def source_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2505_06582_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary,
    or None when there is none or a source that shapes the kernel's traffic changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_fwdbwd100k.json" % kernel)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_sha256_16") != source_digest(kernel):
        return None
    return d["bytes_per_launch"]


def bench_batched(args):
    """16 scenes with log-uniform Gaussian counts in [1e3, 5e5], 1080x1920x3 each, fwd + loss + bwd:
    one batched call pair (persistent launches, hipGraph replay) against 16 sequential calls."""
    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws
    counts = gwsgen.batched_counts(16)
    grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    log("bench batched16: counts %s (total %d)" % (counts, sum(counts)))
    scenes = [gwsgen.make_scene(n, grid, 5000 + i, depth_range=(-10e-3, 10e-3)) for i, n in enumerate(counts)]
    cat = gwsgen.Scene.concat(scenes)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    S, C, M = len(counts), grid.n_lambda, grid.nx * grid.ny
    ctx = gws.context(0)
    prob = gws.Problem.from_grid(grid, tile_config=args.tile_config)
    dev = torch.device("cuda", 0)
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in cat.fields().items()}
    gs = [{k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in sc.fields().items()} for sc in scenes]
    target = torch.from_numpy(np.stack([gwsgen.make_target(grid, 6000 + i) for i in range(S)])).to(dev)
    fields = torch.empty((S, C, grid.ny, grid.nx), dtype=torch.complex64, device=dev)
    G = torch.empty_like(fields)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    grads = {k: torch.empty_like(v) for k, v in g.items()}
    sgrads = [{k: torch.empty_like(v) for k, v in gi.items()} for gi in gs]
    stream = torch.cuda.Stream()

    def step_batched():
        ctx.forward_batched(prob, g, offsets, out=fields)
        ctx.l2_loss_grad(fields, target, grad=G, loss=loss)
        ctx.backward_batched(prob, g, offsets, G, want_depth=False, out=grads)

    def step_sequential():
        for i in range(S):
            ctx.forward(prob, gs[i], out=fields[i])
            ctx.l2_loss_grad(fields[i], target[i], grad=G[i], loss=loss)
            ctx.backward(prob, gs[i], G[i], out=sgrads[i], want_depth=False)

    res = {}
    with torch.cuda.stream(stream):
        for name, fn in (("batched", step_batched), ("sequential", step_sequential)):
            for _ in range(max(1, args.warmup)):
                fn()
            stream.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                fn()
            e1.record(stream)
            stream.synchronize()
            res[name] = e0.elapsed_time(e1) / args.steps
            log("bench batched16: %s %.2f ms per 16-scene step" % (name, res[name]))
            if name == "batched":
                replayed = ctx.stats()["graph_replayed"]  # the last batched call replayed its graph
    out = {"metric": "holograms/s, 16 scenes (Gaussians log-uniform in [1e3, 5e5]) at 1080x1920x3 fwd+bwd",
           "value": 1e3 * S / res["batched"], "unit": "holograms/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["batched"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batched16", "scenes": S, "counts": counts, "ny": grid.ny, "nx": grid.nx,
                      "n_lambda": C},
           "sequential_ms_per_step": res["sequential"], "sequential_holograms_per_s": 1e3 * S / res["sequential"],
           "speedup_vs_sequential": res["sequential"] / res["batched"], "graph_replayed": replayed}
    print(json.dumps(out), flush=True)


def bench_exact(args):
    """Exact alpha wave blending (Eq. 5-6) forward: 1000 Gaussians of the 100k workload's
    distributions at 1080x1920x3, against the order-invariant forward of the same scene."""
    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws
    grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_scene(1000, grid, 1005, depth_range=(-10e-3, 10e-3))
    ctx = gws.context(0)
    dev = torch.device("cuda", 0)
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.fields().items()}
    field = torch.empty((grid.n_lambda, grid.ny, grid.nx), dtype=torch.complex64, device=dev)
    res = {}
    for name, blend in (("exact", gws.BLEND_EXACT), ("order_invariant", gws.BLEND_OIT)):
        prob = gws.Problem.from_grid(grid, blend=blend)
        for _ in range(max(1, args.warmup)):
            ctx.forward(prob, g, out=field)
        torch.cuda.synchronize()
        ctx.read_profile()
        ctx.set_profiling(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            ctx.forward(prob, g, out=field)
        e1.record()
        torch.cuda.synchronize()
        ctx.set_profiling(False)
        prof = ctx.read_profile()
        res[name] = {"ms_per_forward": e0.elapsed_time(e1) / args.steps,
                     "stage_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}}
        log("bench exact1k: %s %.2f ms per forward" % (name, res[name]["ms_per_forward"]))
    # the training step: exact forward, L2 loss and its gradient, exact backward
    prob = gws.Problem.from_grid(grid, blend=gws.BLEND_EXACT)
    target = torch.from_numpy(gwsgen.make_target(grid, 1006)).to(dev)
    G = torch.empty_like(field)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    grads = {k: torch.empty_like(v) for k, v in g.items()}

    def step():
        ctx.forward(prob, g, out=field)
        ctx.l2_loss_grad(field, target, grad=G, loss=loss)
        ctx.backward(prob, g, G, out=grads, want_depth=False)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    res["exact_fwd_bwd_ms"] = e0.elapsed_time(e1) / args.steps
    log("bench exact1k: exact forward + loss + backward %.2f ms per step" % res["exact_fwd_bwd_ms"])
    M, C = grid.nx * grid.ny, grid.n_lambda
    t = res["exact"]["stage_ms"]["accumulate"] * 1e-3
    # per Gaussian, the least the FFT route must move: two Gaussians' real masked profiles
    # share one complex image, whose full spectrum the transform writes once and the splat
    # reads once (8 M bytes per pair each way): 8 M bytes per Gaussian (the window strips the
    # transform also moves are left out)
    bytes_alg = scene.n * 8.0 * M
    out = {"metric": "exact-blending forward holograms/s, 1000 Gaussians at 1080x1920x3",
           "value": 1e3 / res["exact"]["ms_per_forward"], "unit": "holograms/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["exact"]["ms_per_forward"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "exact1k", "gaussians": scene.n, "ny": grid.ny, "nx": grid.nx, "n_lambda": C},
           "variants": res,
           "roofline": {"bound": "hbm", "achieved": bytes_alg / t / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                        "frac": bytes_alg / t / PEAK_HBM, "traffic": None, "kernel": "exact mask + FFT + splat",
                        "work_per_launch": "8 x M bytes per Gaussian (a pair's packed spectrum written once and read once)"}}
    print(json.dumps(out), flush=True)


# The paper's Table 3: runtimes for 15k Gaussians (its GPU and precision unstated).
PAPER_TABLE3_S = {(1280, 1024): {"fast": 6.84, "exact": 180.0}, (2000, 2000): {"fast": 18.06, "exact": 470.0}}


def bench_paper(args):
    """The paper's runtime shapes (Table 3): 15k Gaussians of the 1080x1920 workloads'
    distributions at 1024x1280 and 2000x2000, one wavelength (520 nm); the order-invariant
    (fast) and exact forwards, each against the paper's reported seconds (context: another
    GPU, unnamed)."""
    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws
    ctx = gws.context(0)
    dev = torch.device("cuda", 0)
    res = {}
    for (nx, ny), seed in (((1280, 1024), 1011), ((2000, 2000), 1012)):
        grid = gwsgen.Grid(nx, ny, 8e-6, 8e-6, (520e-9,))
        scene = gwsgen.make_scene(15000, grid, seed, depth_range=(-10e-3, 10e-3))
        g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.fields().items()}
        field = torch.empty((1, ny, nx), dtype=torch.complex64, device=dev)
        key = "%dx%d" % (ny, nx)
        res[key] = {}
        for name, blend, steps in (("fast", gws.BLEND_OIT, args.steps), ("exact", gws.BLEND_EXACT, max(1, args.steps // 4))):
            prob = gws.Problem.from_grid(grid, blend=blend)
            for _ in range(max(1, args.warmup)):
                ctx.forward(prob, g, out=field)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                ctx.forward(prob, g, out=field)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            paper = PAPER_TABLE3_S[(nx, ny)][name]
            res[key][name] = {"ms": ms, "paper_s": paper, "paper_over_ours": paper / (ms * 1e-3)}
            log("bench paper15k %s %s: %.3f ms (paper: %.2f s)" % (key, name, ms, paper))
    t = res["1024x1280"]["fast"]["ms"]
    out = {"metric": "fast-GWS forward holograms/s, 15k Gaussians at 1024x1280, one wavelength (the paper's Table 3 shape)",
           "value": 1e3 / t, "unit": "holograms/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": t, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": (1e3 / t) / (1.0 / PAPER_TABLE3_S[(1280, 1024)]["fast"]), "dtype": "f32",
           "data": "synthetic", "config": {"workload": "paper15k", "gaussians": 15000, "n_lambda": 1,
                                           "shapes": ["1024x1280", "2000x2000"]},
           "runs": res,
           "note": "vs_baseline divides by the paper's 6.84 s on an unnamed GPU: context, not a like-for-like target"}
    print(json.dumps(out), flush=True)


def bench_holo(args):
    """World space to hologram: 100k flat world-space Gaussians with degree-3 opacity seen by
    a random camera, the holographics transform, then the order-invariant forward at
    1080x1920x3."""
    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws
    grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    n = 100_000
    cam = gwsgen.make_camera(1008)
    w = gwsgen.make_world_scene(n, cam, 1009)
    ctx = gws.context(0)
    dev = torch.device("cuda", 0)
    wt = {k: torch.from_numpy(v).to(dev) for k, v in w.items()}
    rng = np.random.Generator(np.random.PCG64(1010))
    g = {"amplitude": torch.from_numpy(rng.uniform(0, 1, (3, n)).astype(np.float32)).to(dev),
         "phase": torch.from_numpy(rng.uniform(0, 2 * np.pi, n).astype(np.float32)).to(dev)}
    plane = ctx.holographics(cam, wt)
    g.update(plane)
    prob = gws.Problem.from_grid(grid)
    field = torch.empty((3, grid.ny, grid.nx), dtype=torch.complex64, device=dev)

    def step():
        ctx.holographics(cam, wt, out=plane)
        ctx.forward(prob, g, out=field)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    ctx.read_profile()
    ctx.set_profiling(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    prof = ctx.read_profile()
    ms = e0.elapsed_time(e1) / args.steps
    st = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items() if v[1]}
    log("bench holo100k: %.3f ms per step; stages %s" % (ms, {k: round(v, 4) for k, v in st.items()}))
    # per Gaussian: mean 12 B, quaternion 16 B, scales 12 B, 16 SH coefficients 64 B read,
    # seven 4-byte outputs written
    b_holo = n * (12.0 + 16.0 + 12.0 + 64.0 + 28.0)
    t_holo = st["holographics"] * 1e-3
    out = {"metric": "world-space scene to hologram (holographics transform + order-invariant forward) per second, "
                     "100k Gaussians at 1080x1920x3",
           "value": 1e3 / ms, "unit": "holograms/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": "holo100k", "gaussians": n, "ny": grid.ny, "nx": grid.nx,
                                           "n_lambda": 3, "sh_degree": 3},
           "stage_ms": st,
           "holographics_roofline": {"bound": "hbm", "achieved": b_holo / t_holo / 1e9, "peak": PEAK_HBM / 1e9,
                                     "unit": "GB/s", "frac": b_holo / t_holo / PEAK_HBM,
                                     "work_per_launch": "132 bytes per Gaussian"}}
    print(json.dumps(out), flush=True)


def bench_focal(args):
    """Display chain at 1080x1920x3: double-phase coding of a hologram-sized field, then the
    half-band-filtered focal stack of the phase-only pattern at 8 planes (-10 .. 10 mm)."""
    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws
    grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    K = 8
    depths = [float(d) for d in np.linspace(-10e-3, 10e-3, K)]
    ctx = gws.context(0)
    dev = torch.device("cuda", 0)
    prob = gws.Problem.from_grid(grid)
    u = torch.from_numpy(gwsgen.make_target(grid, 1007)).to(dev)
    C, M = grid.n_lambda, grid.nx * grid.ny
    P = torch.empty((C, grid.ny, grid.nx), dtype=torch.float32, device=dev)
    stack = torch.empty((K, C, grid.ny, grid.nx), dtype=torch.float32, device=dev)

    def step():
        ctx.dpac_encode(u, out=P)
        ctx.focal_stack(prob, P, depths, phase_input=True, half_band=True, out=stack)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    ctx.read_profile()
    ctx.set_profiling(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    prof = ctx.read_profile()
    ms = e0.elapsed_time(e1) / args.steps
    st = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items() if v[1]}
    log("bench focal8: %.3f ms per step; stages %s" % (ms, {k: round(v, 4) for k, v in st.items()}))
    # algorithmic bytes: the coding reads the field (8 B) and writes the pattern (4 B); the
    # stack reads the pattern once (4 B) and writes K intensity planes (4 B each)
    b_dpac, b_focal = 12.0 * C * M, (4.0 + 4.0 * K) * C * M
    t_focal = st["focal_stack"] * 1e-3
    out = {"metric": "display chain (double-phase coding + 8-plane filtered focal stack) per second, 1080x1920x3",
           "value": 1e3 / ms, "unit": "stacks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "focal8", "planes": K, "depths_m": depths, "ny": grid.ny, "nx": grid.nx,
                      "n_lambda": C},
           "stage_ms": st,
           "dpac_roofline": {"bound": "hbm", "achieved": b_dpac / (st["dpac"] * 1e-3) / 1e9,
                             "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                             "frac": b_dpac / (st["dpac"] * 1e-3) / PEAK_HBM},
           "roofline": {"bound": "hbm", "achieved": b_focal / t_focal / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                        "frac": b_focal / t_focal / PEAK_HBM, "traffic": None,
                        "kernel": "focal stack (e^{jP}, forward FFT, per-plane transfer + inverse FFT, |u|^2)",
                        "work_per_launch": "(4 + 4 K) bytes per pixel and wavelength"}}
    print(json.dumps(out), flush=True)


def bench_sizes(args):
    """Throughput against scene size: the fwdbwd100k distributions (1080x1920x3, depths
    U(-10, 10) mm) at 1k ... 1M Gaussians; per size the forward alone and the training step
    (forward, L2 loss, backward without the depth gradient), and the work inside the supports."""
    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws
    grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    ctx = gws.context(0)
    dev = torch.device("cuda", 0)
    prob = gws.Problem.from_grid(grid, tile_config=args.tile_config)
    target = torch.from_numpy(gwsgen.make_target(grid, 2003)).to(dev)
    field = torch.empty((grid.n_lambda, grid.ny, grid.nx), dtype=torch.complex64, device=dev)
    G = torch.empty_like(field)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for j, n in enumerate((1_000, 3_000, 10_000, 30_000, 100_000, 300_000, 1_000_000)):
        scene = gwsgen.make_scene(n, grid, 1100 + j, depth_range=(-10e-3, 10e-3))
        g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.fields().items()}
        grads = {k: torch.empty_like(v) for k, v in g.items()}
        steps = max(2, min(args.steps, int(2e6 // n)))

        def fwd():
            ctx.forward(prob, g, out=field)

        def step():
            ctx.forward(prob, g, out=field)
            ctx.l2_loss_grad(field, target, grad=G, loss=loss)
            ctx.backward(prob, g, G, out=grads, want_depth=False)

        out = {"gaussians": n, "steps": steps}
        for name, fn in (("forward", fwd), ("fwd_bwd", step)):
            for _ in range(max(1, args.warmup)):
                fn()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            out[name + "_ms"] = e0.elapsed_time(e1) / steps
        pairs = ellipse_support_points(scene, grid)
        out["support_pairs"] = pairs
        out["fwd_bwd_pairs_per_s"] = 2 * pairs / (out["fwd_bwd_ms"] * 1e-3)
        log("bench sizes: %7d Gaussians: forward %.3f ms, fwd+bwd %.3f ms, %.3g support pairs"
            % (n, out["forward_ms"], out["fwd_bwd_ms"], pairs))
        rows.append(out)
        del g, grads
    big = rows[-1]
    print(json.dumps({"metric": "holograms/s against scene size, 1080x1920x3 fwd+bwd",
                      "value": 1e3 / big["fwd_bwd_ms"], "unit": "holograms/s (at 1M Gaussians)", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": big["fwd_bwd_ms"],
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                      "data": "synthetic", "config": {"workload": "sizes: 1k-1M Gaussians, 1080x1920x3"},
                      "sizes": rows}), flush=True)


def bench_fwd10k(args):
    """The plain forward: 10k Gaussians at 1080x1920x3 (preprocess, sort, bin, accumulate, inverse FFT)."""
    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws
    scene, grid = gwsgen.workload("fwd10k")
    ctx = gws.context(0)
    dev = torch.device("cuda", 0)
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.fields().items()}
    field = torch.empty((grid.n_lambda, grid.ny, grid.nx), dtype=torch.complex64, device=dev)
    prob = gws.Problem.from_grid(grid, tile_config=args.tile_config)
    for _ in range(max(1, args.warmup)):
        ctx.forward(prob, g, out=field)
    torch.cuda.synchronize()
    ctx.read_profile()
    ctx.set_profiling(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        ctx.forward(prob, g, out=field)
    e1.record()
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    prof = ctx.read_profile()
    ms = e0.elapsed_time(e1) / args.steps
    st = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items() if v[1]}
    C = grid.n_lambda
    support = ellipse_support_points(scene, grid)
    t_acc = st["accumulate"] * 1e-3
    log("bench fwd10k: %.3f ms per forward; stages %s" % (ms, {k: round(v, 4) for k, v in st.items()}))
    out = {"metric": "forward holograms/s, 10k Gaussians at 1080x1920x3", "value": 1e3 / ms, "unit": "holograms/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "fwd10k", "gaussians": scene.n, "ny": grid.ny, "nx": grid.nx, "n_lambda": C},
           "stage_ms": st,
           "roofline": {"bound": "alu", "achieved": support * (1 + 2 * C) / t_acc / 1e12, "peak": PEAK_TRANS / 1e12,
                        "unit": "TOP/s", "frac": support * (1 + 2 * C) / t_acc / PEAK_TRANS, "traffic": None,
                        "kernel": "accumulate"}}
    print(json.dumps(out), flush=True)


def tilted_support_triples(scene, grid, step=8, chunk=2048):
    """(Gaussian, frequency, wavelength) triples strictly inside the eps-support of tilted
    Gaussians (Gaussian factor >= 1e-7 of its peak, propagating frequency), estimated on the
    regular sub-lattice of every step-th row and column of the grid (x step^2).  The coverage
    is a smooth function of frequency, so the sub-lattice sum is accurate to well under 1 %.
    Float64 on the GPU (torch), arithmetic of the definition; measurement only."""
    import numpy as np
    import torch

    dev = torch.device("cuda", 0)
    K2 = 2.0 * math.pi ** 2 / math.log(2.0)
    tau2 = math.log2(1e7)
    mx = torch.arange(-(grid.nx // 2), grid.nx // 2, step, dtype=torch.float64, device=dev) / (grid.nx * grid.px)
    my = torch.arange(-(grid.ny // 2), grid.ny // 2, step, dtype=torch.float64, device=dev) / (grid.ny * grid.py)
    NY, NX = torch.meshgrid(my, mx, indexing="ij")
    nux, nuy = NX.reshape(-1), NY.reshape(-1)
    q = np.stack([scene.quat_w, scene.quat_x, scene.quat_y, scene.quat_z]).astype(np.float64)
    w, x, y, z = q / np.linalg.norm(q, axis=0)
    # rotation matrices of the unit quaternions, [n][3][3]
    R = np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                  np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                  np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)
    Rt = torch.from_numpy(np.ascontiguousarray(R)).to(dev)
    su = torch.from_numpy(scene.scale_u.astype(np.float64)).to(dev)
    sv = torch.from_numpy(scene.scale_v.astype(np.float64)).to(dev)
    total = 0.0
    for lam in grid.lambdas:
        w2 = 1.0 / lam ** 2 - (nux * nux + nuy * nuy)
        prop = w2 > 0
        kz = torch.sqrt(torch.clamp(w2, min=0.0))
        for a in range(0, scene.n, chunk):
            r = Rt[a:a + chunk]
            kox = r[:, 0, 0, None] * nux + r[:, 1, 0, None] * nuy + r[:, 2, 0, None] * kz
            koy = r[:, 0, 1, None] * nux + r[:, 1, 1, None] * nuy + r[:, 2, 1, None] * kz
            q = K2 * ((su[a:a + chunk, None] * kox) ** 2 + (sv[a:a + chunk, None] * koy) ** 2)
            total += float(((q < tau2) & prop).sum().item())
    return total * step * step


def bench_tilted(args):
    """100k tilted Gaussians (tilts up to 2 degrees about random in-plane axes, the fwd100k
    distributions otherwise) at 1080x1920x3: forward (records, accumulation, inverse FFT), then
    the training step (forward, L2 loss, backward)."""
    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws
    grid = gwsgen.Grid(1920, 1080, 8e-6, 8e-6, gwsgen.RGB)
    scene = gwsgen.make_tilted_scene(100_000, grid, 1005, depth_range=(-10e-3, 10e-3), tilt_max_deg=2.0)
    ctx = gws.context(0)
    dev = torch.device("cuda", 0)
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.fields().items()}
    field = torch.empty((grid.n_lambda, grid.ny, grid.nx), dtype=torch.complex64, device=dev)
    prob = gws.Problem.from_grid(grid)
    for _ in range(max(1, args.warmup)):
        ctx.forward_tilted(prob, g, out=field)
    torch.cuda.synchronize()
    ctx.read_profile()
    ctx.set_profiling(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        ctx.forward_tilted(prob, g, out=field)
    e1.record()
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    prof = ctx.read_profile()
    st = ctx.stats()
    ms = e0.elapsed_time(e1) / args.steps
    stage = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items() if v[1]}
    # the training step: forward, L2 loss and its field gradient, backward (every gradient)
    target = torch.from_numpy(gwsgen.make_target(grid, 2005)).to(dev)
    G = torch.empty_like(field)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    grads = {k: torch.empty_like(v) for k, v in g.items()}

    def train_step():
        ctx.forward_tilted(prob, g, out=field)
        ctx.l2_loss_grad(field, target, G, loss)
        ctx.backward_tilted(prob, g, G, out=grads)

    for _ in range(max(1, args.warmup)):
        train_step()
    torch.cuda.synchronize()
    ctx.read_profile()
    ctx.set_profiling(True)
    e0.record()
    for _ in range(args.steps):
        train_step()
    e1.record()
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    prof_b = ctx.read_profile()
    st_b = ctx.stats()
    ms_fb = e0.elapsed_time(e1) / args.steps
    stage_fb = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof_b.items() if v[1]}
    C = grid.n_lambda
    triples = tilted_support_triples(scene, grid)
    evaluated = float(st["n_pairs_evaluated"])   # (Gaussian, frequency, wavelength) triples
    t_acc = stage["accumulate"] * 1e-3
    log("bench tilted100k: %.3f ms per forward; stages %s; support triples %.4g, evaluated %.4g"
        % (ms, {k: round(v, 4) for k, v in stage.items()}, triples, evaluated))
    out = {"metric": "forward holograms/s, 100k tilted Gaussians at 1080x1920x3", "value": 1e3 / ms,
           "unit": "holograms/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "tilted100k: 100k tilted Gaussians (tilt U(0, 2) deg about a random in-plane axis), "
                                  "1080x1920x3, 8 um pitch, forward", "gaussians": scene.n, "ny": grid.ny,
                      "nx": grid.nx, "n_lambda": C},
           "stage_ms": stage,
           "roofline": {"bound": "alu", "achieved": 3 * triples / t_acc / 1e12, "peak": PEAK_TRANS / 1e12,
                        "unit": "TOP/s", "frac": 3 * triples / t_acc / PEAK_TRANS, "traffic": None,
                        "kernel": "tilted accumulate",
                        "work_per_launch": "%.4g transcendental ops (= %.4g (Gaussian, frequency, wavelength) triples "
                                           "inside the 1e-7 support x (1 exp2 + 1 sin + 1 cos))" % (3 * triples, triples),
                        "evaluated_frac": 3 * evaluated / t_acc / PEAK_TRANS,
                        "evaluated_over_support": evaluated / triples},
           "fwd_bwd": {"ms_per_step": ms_fb, "holograms_per_s": 1e3 / ms_fb, "stage_ms": stage_fb,
                       "adjoint_roofline": {
                           "bound": "alu", "achieved": 3 * triples / (stage_fb["adjoint"] * 1e-3) / 1e12,
                           "peak": PEAK_TRANS / 1e12, "unit": "TOP/s",
                           "frac": 3 * triples / (stage_fb["adjoint"] * 1e-3) / PEAK_TRANS,
                           "evaluated_over_support": float(st_b["n_pairs_evaluated"]) / triples},
                       "note": "forward + L2 loss + backward (every parameter's gradient); the backward "
                               "synchronises once to size its partial-sum buffer"}}
    log("bench tilted100k: fwd+bwd %.3f ms; stages %s" % (ms_fb, {k: round(v, 4) for k, v in stage_fb.items()}))
    print(json.dumps(out), flush=True)


def bench_precision(args):
    """1M Gaussians at 2160x3840x3 (5% far off-axis at 20-50 mm): forward with the FP32 FFT and
    with the split-bf16 MFMA DFT; the transform kernels' rooflines."""
    import numpy as np
    import torch

    import gwsgen
    import paper_2505_06582_amd as gws
    scene, grid = gwsgen.workload("precision1m")
    ctx = gws.context(0)
    dev = torch.device("cuda", 0)
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in scene.fields().items()}
    field = torch.empty((grid.n_lambda, grid.ny, grid.nx), dtype=torch.complex64, device=dev)
    res = {}
    # the FP32 FFT and the split-bf16 DFT with exact phase bases, then the FFT path with plain
    # FP32 phase bases (what the exact bases cost in the accumulation)
    runs = (("fft_fp32", gws.XFORM_FFT_FP32, 0), ("dft_bf16x3", gws.XFORM_DFT_BF16X3, 0),
            ("fft_fp32_fp32_phase_base", gws.XFORM_FFT_FP32, 1))
    for name, xf, pm in runs:
        prob = gws.Problem.from_grid(grid, xform=xf, tile_config=args.tile_config, phase_mode=pm)
        for _ in range(max(1, args.warmup)):
            ctx.forward(prob, g, out=field)
        torch.cuda.synchronize()
        ctx.read_profile()
        ctx.set_profiling(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            ctx.forward(prob, g, out=field)
        e1.record()
        torch.cuda.synchronize()
        ctx.set_profiling(False)
        prof = ctx.read_profile()
        res[name] = {"ms_per_forward": e0.elapsed_time(e1) / args.steps,
                     "stage_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}}
        log("bench precision1m: %s %.2f ms per forward" % (name, res[name]["ms_per_forward"]))
    C, M, nx, ny = grid.n_lambda, grid.nx * grid.ny, grid.nx, grid.ny
    # error of each transform against an FP64 inverse DFT of the same (GPU) spectrum
    errs = {}
    for name, xf in (("fft_fp32", gws.XFORM_FFT_FP32), ("dft_bf16x3", gws.XFORM_DFT_BF16X3)):
        prob = gws.Problem.from_grid(grid, xform=xf, tile_config=args.tile_config)
        f, sp = ctx.forward(prob, g, want_spectrum=True)
        torch.cuda.synchronize()
        if name == "fft_fp32":
            s64 = sp.cpu().numpy().astype(np.complex128)
            ref = np.fft.ifft2(s64) * (nx * ny)
            del s64
        got = f.cpu().numpy().astype(np.complex128)
        errs[name] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        del got, f, sp
        log("bench precision1m: %s transform rel L2 vs FP64 inverse DFT of the same spectrum %.3e" % (name, errs[name]))
    del ref
    for name in errs:
        res[name]["transform_rel_l2_vs_fp64"] = errs[name]
    t_fft = res["fft_fp32"]["stage_ms"]["xform_inverse"] * 1e-3
    t_dft = res["dft_bf16x3"]["stage_ms"]["xform_inverse"] * 1e-3
    flops = C * 24.0 * (ny * nx * nx + nx * ny * ny)   # two complex GEMMs, 3 bf16 products each
    out = {"metric": "forward holograms/s, 1M Gaussians at 2160x3840x3 (5% far off-axis at 20-50 mm)",
           "value": 1e3 / res["fft_fp32"]["ms_per_forward"], "unit": "holograms/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["fft_fp32"]["ms_per_forward"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "precision1m", "gaussians": scene.n, "ny": ny, "nx": nx, "n_lambda": C},
           "variants": res,
           "accumulate_ms_by_phase_base": {"exact_fp64": res["fft_fp32"]["stage_ms"]["accumulate"],
                                            "plain_fp32": res["fft_fp32_fp32_phase_base"]["stage_ms"]["accumulate"]},
           "transform_roofline": {
               "fft_fp32": {"bound": "hbm", "achieved": 2 * C * M * 8 / t_fft / 1e9, "peak": 8000.0, "unit": "GB/s",
                            "frac": 2 * C * M * 8 / t_fft / 8e12, "algorithmic_bytes": 2 * C * M * 8,
                            "two_pass_bytes": 4 * C * M * 8},
               "dft_bf16x3": {"bound": "mfma", "achieved": flops / t_dft / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                              "frac": flops / t_dft / 2.5e15}}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
