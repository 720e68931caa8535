#!/usr/bin/env python3
"""AMG-PCG time-to-1e-8 on one MI355X.

A step is one pass of the whole hot path on one synthetic system: amg_setup
(strength, aggregation, Galerkin, colouring, FP32 copies, coarse Cholesky),
pcg_solve to relative residual 1e-8 (FP32 V-cycle inside FP64 flexible CG),
and amg_free.  The workload is the heterogeneous 256^3 system: cell
permeability K = exp(2 g') with g' a 2x2x2 box-filtered N(0,1) field
(seed 1), 7-point cell-centred finite volumes with harmonic faces, RHS
uniform[-1,1], x0 = 0.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AMG-PCG time-to-1e-8 & HBM GB/s at 256^3; solves/s + p99 latency (stream)"
HBM_PEAK_GBS = 8000.0
SWEEP_SOURCE = os.path.join(ROOT, "paper_1209_0960_amd", "csrc", "kernels_solve.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweep_hetero256.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(SWEEP_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    --pmc summary, or None when the kernel changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(sample_n: int, full_n: int):
    """The oracle (single thread) on the same recipe at sample_n^3, scaled by
    unknowns to full_n^3."""
    import oracle as O
    from paper_1209_0960_amd import problems as P

    s = P.lognormal(sample_n, seed=1)
    t0 = time.perf_counter()
    H = O.Hierarchy(s.rowptr, s.colind, s.vals, vcycle_fp32=1)
    t1 = time.perf_counter()
    out = H.pcg(s.b, rtol=1e-8)
    t2 = time.perf_counter()
    H.close()
    sec = t2 - t0
    scale = (full_n / sample_n) ** 3
    return {
        "value": 1.0 / (sec * scale),
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle setup+FCG(FP32 V-cycle) to 1e-8 on the same lognormal recipe at {sample_n}^3 "
                   f"({s.n} unknowns, seed 1): setup {t1 - t0:.2f} s, solve {t2 - t1:.2f} s, "
                   f"{out['iterations']} iterations; time scaled by unknowns x{scale:.0f} to {full_n}^3"),
        "sample_seconds": sec,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--cpu-sample-n", type=int, default=96)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain-FP64 comparison solves")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is not part of this "
              "build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1209_0960_amd import amg as A
    from paper_1209_0960_amd import problems as P

    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "repeats": 3}), flush=True)
        return
    A.lib()
    n = args.n
    t = time.perf_counter()
    s = P.lognormal(n, seed=1)
    log(f"workload lognormal {n}^3: n={s.n} nnz={s.nnz} generated in {time.perf_counter() - t:.1f} s")
    rp, ci, v, b = A.to_device(s)
    torch.cuda.synchronize()

    def step(fp32: bool, x=None, rtol=1e-8):
        h = A.Hierarchy(rp, ci, v, vcycle_fp32=1 if fp32 else 0)
        x, r = h.solve(b, x, rtol=rtol)
        levels = h.levels
        h.close()
        return x, r, levels

    for w in range(args.warmup):
        _, r, _ = step(True)
        log(f"warmup {w}: setup {r.setup_ms:.1f} ms solve {r.solve_ms:.1f} ms it={r.iterations}")

    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        x_mixed, r, levels = step(True)
        infos.append(r)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    for r in infos:
        log(f"timed step: setup {r.setup_ms:.1f} ms solve {r.solve_ms:.1f} ms it={r.iterations} "
            f"true_rel_res={r.true_rel_residual:.2e}")
    # Per-kernel HIP-event timing of the dominant kernel: one more step of the
    # same workload with event timing on (iterations launched individually, the
    # kernels are the ones the graph replays).
    A.set_kernel_timing([A.KIND_SWEEP])
    A.reset_kernel_timing()
    _, rt, _ = step(True)
    A.set_kernel_timing(False)
    sweep_ms, sweep_launches, sweep_bytes = A.kernel_timing(A.KIND_SWEEP)
    log(f"event-timed step: solve {rt.solve_ms:.1f} ms, {sweep_launches} sweep launches")

    extra = {}
    if not args.no_compare:
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        x_plain, rp64, _ = step(False)
        torch.cuda.synchronize()
        c1 = time.perf_counter()
        x_ref, rref, _ = step(False, rtol=1e-12)
        err = float(torch.linalg.norm(x_mixed - x_ref) / torch.linalg.norm(x_ref))
        err_plain = float(torch.linalg.norm(x_plain - x_ref) / torch.linalg.norm(x_ref))
        extra = {
            "plain_fp64": {"ms": (c1 - c0) * 1e3, "setup_ms": rp64.setup_ms, "solve_ms": rp64.solve_ms,
                           "iterations": rp64.iterations, "fp64_solution_error": err_plain},
            "mixed_fp64_solution_error": err,
            "speedup_mixed_vs_plain_fp64": (c1 - c0) * 1e3 / ms_per_step,
        }

    avg_launch_ms = sweep_ms / max(sweep_launches, 1)
    bytes_per_launch = sweep_bytes / max(sweep_launches, 1)
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9 if sweep_launches else None
    traffic = traffic_per_launch()
    last = infos[-1]
    out = {
        "metric": METRIC,
        "value": 1e3 / ms_per_step,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 CG + f32 V-cycle",
        "data": "synthetic",
        "config": {
            "workload": f"lognormal-K 7-point CCFV {n}^3 (sigma^2=4, 2x2x2 box filter, seed 1), "
                        f"FP32 V(1,1) MC-SGS in FP64 flexible CG to rtol 1e-8",
            "unknowns": s.n, "nnz": s.nnz, "levels": levels, "iterations": last.iterations,
            "setup_ms": last.setup_ms, "solve_ms": last.solve_ms, "time_to_1e8_ms": ms_per_step,
            "true_rel_residual": last.true_rel_residual, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_gs_sell<float> (one level-0 colour pass of the Gauss-Seidel smoother, SELL-64)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic,
            "method": "HIP events on the launch stream around every level-0 colour pass of one extra step "
                      "of the same workload after the timed steps",
            "launches": sweep_launches,
            "avg_launch_us": avg_launch_ms * 1e3,
            "algorithmic_bytes_per_launch": bytes_per_launch,
        },
    }
    out["config"].update(extra)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
