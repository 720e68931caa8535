#!/usr/bin/env python3
"""AMG-PCG time-to-1e-8 on one MI355X.

A step is one pass of the whole hot path on one synthetic system: amg_setup
(strength, aggregation, Galerkin, colouring, coarse Cholesky), pcg_solve to
relative residual 1e-8 with the plain FP64 method (FP64 V(1,1) cycle inside
FP64 CG, the paper's precision; multicolour symmetric Gauss-Seidel on level
0, the tile-ordered multicolour form of the paper's hybrid smoother on the
coarser levels), and amg_free.  The workload is the heterogeneous 256^3 system: cell permeability
K = exp(2 g') with g' a 2x2x2 box-filtered N(0,1) field (seed 1), 7-point
cell-centred finite volumes with harmonic faces, RHS uniform[-1,1], x0 = 0.
Inputs are resident in HBM before timing starts.

More sections go into the same line: config.mixed (the same steps with the
FP32 V-cycle inside FP64 flexible CG, timed the same way, with the speedup
and both FP64 solution errors), config.c1 (32^3 Poisson: time, iterations,
levels, launches per iteration), config.c2 (128^3 heterogeneous: plain
against mixed), "paper_solver" in config (BiCGSTAB, the paper's Krylov
method, with multicolour and hybrid SGS on the same system; BiCGSTAB
iteration counts on the paper's Laplace, manufactured Poisson and
jump-coefficient problems beside its published counts), "large" (layered
512^3, per-kernel GB/s and the FP64 solution error against a 1e-12
reference), "batched" (64 uneven systems with 4 right-hand sides each,
amg_setup_batched + pcg_solve_batched against a loop of single solves) and
"serving" (a request stream served with continuous batching against serial
plain-FP64 solves, with p50/p99 latency) and "block" (point-based AMG on a
3-component coupled system against the scalar hierarchy of the same matrix).

Prints one JSON line.  --gpus above 1 is refused: the library runs on one GPU.
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
# Smoothing of the headline method: multicolour SGS on level 0, the hybrid
# smoother of Sec. 3.2 with each tile's rows in colour order on levels >= 1
# (one launch per sweep there instead of two per colour).
HEAD = {"coarse_smoother": 3, "coarse_from": 1}
HEAD_TEXT = "V(1,1): MC-SGS on level 0, tile-ordered MC-SGS (hybrid, Sec. 3.2, 128-row tiles) on levels >= 1"
HBM_PEAK_GBS = 8000.0
SWEEP_SOURCE = os.path.join(ROOT, "paper_1209_0960_amd", "csrc", "kernels_solve.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gs_fp64_hetero256.json")
ROOFLINE_KERNEL = "kb_gs<double, 1, true>"


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
    if t.get("kernel_source_sha256_16") != kernel_hash() or t.get("kernel_name") != ROOFLINE_KERNEL:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(sample_n: int):
    """The oracle (plain single-threaded C++, FP64 throughout) measured on the
    configuration-2 recipe (lognormal sigma^2 = 4, 2x2x2 box filter, seed 1)
    at sample_n^3 with the headline's method (FP64 V(1,1) cycle with the
    headline's smoothers, in PCG to 1e-8), the calling thread pinned to one
    host core.  Measured, not
    scaled: the value is that workload's solves/s."""
    import oracle as O
    from paper_1209_0960_amd import problems as P

    s = P.lognormal(sample_n, seed=1)
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        H = O.Hierarchy(s.rowptr, s.colind, s.vals, **HEAD)
        t1 = time.perf_counter()
        out = H.pcg(s.b, rtol=1e-8)
        t2 = time.perf_counter()
        levels = H.levels
        H.close()
    finally:
        os.sched_setaffinity(0, set(allowed))
    sec = t2 - t0
    return {
        "value": 1.0 / sec,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle setup + FP64 PCG (FP64 {HEAD_TEXT}) to 1e-8 on the configuration-2 recipe at "
                   f"{sample_n}^3 ({s.n} unknowns, lognormal sigma^2=4, seed 1), one thread pinned to core {core}: "
                   f"TB {t1 - t0:.2f} s, TS {t2 - t1:.2f} s, {out['iterations']} iterations, {levels} levels; "
                   f"measured at this size, not scaled"),
        "unknowns": s.n, "setup_s": t1 - t0, "solve_s": t2 - t1, "iterations": out["iterations"],
        "levels": levels, "unknowns_per_s": s.n / sec, "true_rel_residual": out["true_rel_residual"],
        "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "pinned_core": core,
    }


def batched_section(A, P, nsys: int, nrhs: int = 4, seed: int = 3):
    """64 uneven lognormal systems x 4 right-hand sides, FP32 V-cycle in FP64
    flexible CG to 1e-8: amg_setup_batched + pcg_solve_batched with the
    autotuned tile / cycle / right-hand-side-interleave variants (tuning timed
    apart), the same with default parameters, and a loop of amg_setup +
    pcg_solve per system and right-hand side (default parameters)."""
    import torch

    from paper_1209_0960_amd import autotune as AT

    t = time.perf_counter()
    systems = P.batched_systems(nsys, seed=seed, nrhs=nrhs)
    gen = time.perf_counter() - t
    dev = [(torch.from_numpy(s.rowptr).cuda(), torch.from_numpy(s.colind).cuda(), torch.from_numpy(s.vals).cuda(),
            torch.from_numpy(s.b.reshape(-1)).cuda()) for s in systems]
    rows = sum(s.n for s in systems)
    common = {"vcycle_fp32": 1}

    def loop():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ts = 0.0
        infos = []
        for d, s in zip(dev, systems):
            a = time.perf_counter()
            h = A.Hierarchy(*d[:3], **common)
            ts += time.perf_counter() - a
            n = s.n
            for k in range(nrhs):
                x, r = h.solve(d[3][k * n:(k + 1) * n].contiguous(), rtol=1e-8, maxit=500)
                infos.append(r)
            h.close()
        torch.cuda.synchronize()
        return ts, time.perf_counter() - t0 - ts, infos

    AT.run_batched(dev, lambda i: {}, nrhs, nrhs, **common)  # warm-up (allocator pool, code objects)
    table = AT.tune(dev, nrhs, **common)
    ts, tv, tinf, tst, _ = AT.run_batched(dev, AT.params_from(table, dev), nrhs, table["R"], **common)
    ds, dv, dinf, dst, _ = AT.run_batched(dev, lambda i: {}, nrhs, nrhs, **common)
    ls, lv, linf = loop()
    its = [i["iterations"] for inf in tinf for i in inf]
    classes = {str(k): v for k, v in table.items() if isinstance(k, int)}
    return {
        "workload": f"{nsys} lognormal systems, edges from {{16,24,32,48,64}} (seed {seed}), sigma^2=2, 4^3 box "
                    f"filter, {nrhs} right-hand sides each; FP32 V-cycle in FP64 flexible CG to 1e-8",
        "unknowns": rows, "solves": nsys * nrhs, "generation_s": gen,
        "batched_ms": (ts + tv) * 1e3, "batched_setup_ms": ts * 1e3, "batched_solve_ms": tv * 1e3,
        "batched_default_ms": (ds + dv) * 1e3, "batched_default_setup_ms": ds * 1e3,
        "batched_default_solve_ms": dv * 1e3,
        "loop_ms": (ls + lv) * 1e3, "loop_setup_ms": ls * 1e3, "loop_solve_ms": lv * 1e3,
        "speedup_batched_vs_loop": (ls + lv) / (ts + tv),
        "unknown_rhs_per_s_batched": rows * nrhs / (ts + tv),
        "autotune": {"per_class_rows": classes, "rhs_interleave": table["R"],
                     "rhs_interleave_ms": {str(k): v for k, v in table["R_ms"].items()},
                     "tuning_s": table["tuning_s"],
                     "variants": "tile_rows in {64,128,256,512} x tail_rows in {0, 8192, 2^30 (whole cycle in "
                                 "one workgroup)} x coarse smoother {MC-SGS, tile-ordered MC-SGS from level 1} "
                                 "per size class (every timed variant in variants_ms), then the level-0 SpMV "
                                 "layout (SELL-64 or CSR with lanes per row); right-hand sides per entry in "
                                 "{4,2,1}"},
        "iterations_max": max(its), "iterations_mean": float(sum(its)) / len(its),
        "all_converged": tst == A.OK and dst == A.OK and all(i["converged"] for inf in tinf for i in inf)
                         and all(r.converged for r in linf),
        "worst_true_rel_residual": max(i["true_rel_residual"] for inf in tinf for i in inf),
    }


def serving_section(A, P, seconds: float, rate: float):
    """Request stream (Poisson arrivals at `rate` for `seconds`, edges U{32..256},
    sigma^2 U[0,4], 30% reuse; fields generated on the device): continuous
    batching (FP32 V-cycle, flexible CG) against serial plain-FP64 solves."""
    import torch
    from paper_1209_0960_amd import serve as S

    trace = P.serving_trace(rate=rate, seconds=seconds, seed=4)
    reqs, gen_s = S.requests_from_trace(trace)
    srv = S.Server(cap_bytes=200e9, max_entries=32, setup_workers=2, vcycle_fp32=1, **HEAD)
    try:
        recs = srv.run(reqs)
        stats = dict(srv.stats)
    finally:
        srv.close()
    base, bstats, _ = S.serve_serial(reqs, vcycle_fp32=0, **HEAD)
    # a point below capacity: the latency of service rather than of queueing
    low_rate, low_seconds = rate / 10.0, 5.0 * seconds
    del reqs
    A.release_cached_memory()
    torch.cuda.empty_cache()
    ltrace = P.serving_trace(rate=low_rate, seconds=low_seconds, seed=5)
    lreqs, _ = S.requests_from_trace(ltrace)
    lsrv = S.Server(cap_bytes=200e9, max_entries=32, setup_workers=2, vcycle_fp32=1, **HEAD)
    try:
        lrecs = lsrv.run(lreqs)
        lstats = dict(lsrv.stats)
    finally:
        lsrv.close()
    del lreqs
    lsm = S.summarise(lrecs, **lstats)
    unknowns = sum(r.n for r in recs)
    A.release_cached_memory()
    torch.cuda.empty_cache()
    sm, sb = S.summarise(recs, **stats), S.summarise(base, **bstats)
    ok = all(r.status == A.OK for r in recs) and all(r.status == A.OK for r in base)
    return {
        "workload": f"{len(trace)} requests: Poisson arrivals at {rate:g}/s over {seconds:g} s (seed 4), edge U{{32..256}}, "
                    f"sigma^2 U[0,4], 30% reuse of a resident matrix with a new right-hand side, rtol 1e-8",
        "unknowns": unknowns, "generation_s": gen_s, "all_converged": ok,
        "served": {"solves_per_s": sm.solves_per_s, "p50_ms": sm.p50_ms, "p99_ms": sm.p99_ms,
                   "makespan_s": sm.makespan_s, "hits": sm.hits, "setups": sm.setups, "evictions": sm.evictions,
                   "max_running": sm.max_running, "peak_reserved_bytes": sm.peak_reserved_bytes,
                   "policy": f"continuous batching (32 slots), FP32 cycle ({HEAD_TEXT}) + FP64 flexible CG, "
                             "admission by estimated HBM footprint under 200 GB, LRU hierarchy cache"},
        "serial_fp64": {"solves_per_s": sb.solves_per_s, "p50_ms": sb.p50_ms, "p99_ms": sb.p99_ms,
                        "makespan_s": sb.makespan_s, "hits": sb.hits, "setups": sb.setups},
        "throughput_ratio": sm.solves_per_s / sb.solves_per_s,
        "p99_ratio": sb.p99_ms / sm.p99_ms,
        "below_capacity": {"workload": f"{len(ltrace)} requests: Poisson arrivals at {low_rate:g}/s over "
                                       f"{low_seconds:g} s (seed 5), same request recipe",
                           "solves_per_s": lsm.solves_per_s, "p50_ms": lsm.p50_ms, "p99_ms": lsm.p99_ms,
                           "makespan_s": lsm.makespan_s, "max_running": lsm.max_running,
                           "all_converged": all(r.status == A.OK for r in lrecs)},
    }


def block_section(A, P, n: int = 96, bs: int = 3, seed: int = 6):
    """Point-based AMG for systems (Sec. 4.2): the 3-component coupled
    lognormal diffusion system on n^3 cells (problems.coupled), FP64 PCG to
    1e-8 with the block hierarchy (node graph with row-sum norm weights,
    P (x) I, block Gauss-Seidel) against the scalar hierarchy of the same
    matrix; the FP32 block cycle in flexible CG; the level-0 block pass rate
    from HIP events."""
    import numpy as np
    import torch

    t = time.perf_counter()
    s = P.coupled(n, bs=bs, seed=seed)
    gen = time.perf_counter() - t
    rp, ci, v, b = A.to_device(s)
    out = {"workload": f"{bs}-component coupled lognormal diffusion {n}^3 cells (sigma^2=2, face couplings "
                       f"I + v v^T, seed {seed}), FP64 PCG to 1e-8",
           "unknowns": s.n, "nnz": s.nnz, "generation_s": gen}
    for key, kw in (("block_fp64", dict(block_size=bs)), ("scalar_fp64", dict()),
                    ("block_fp32_vcycle", dict(block_size=bs, vcycle_fp32=1))):
        ts = []
        for _ in range(4):
            torch.cuda.synchronize()
            a = time.perf_counter()
            h = A.Hierarchy(rp, ci, v, **kw)
            x, r = h.solve(b, rtol=1e-8, maxit=500)
            lev = h.levels
            h.close()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - a) * 1e3)
        out[key] = {"time_to_1e8_ms": float(np.median(ts[1:])), "setup_ms": r.setup_ms, "solve_ms": r.solve_ms,
                    "iterations": r.iterations, "levels": lev, "true_rel_residual": r.true_rel_residual}
        log(f"block section {key}: {out[key]}")
    out["speedup_block_vs_scalar"] = out["scalar_fp64"]["time_to_1e8_ms"] / out["block_fp64"]["time_to_1e8_ms"]
    h = A.Hierarchy(rp, ci, v, block_size=bs)
    A.set_kernel_timing([A.KIND_SWEEP])
    A.reset_kernel_timing()
    h.solve(b, rtol=1e-8, maxit=500)
    A.set_kernel_timing(False)
    h.close()
    ms, cnt, by = A.kernel_timing(A.KIND_SWEEP)
    out["kb_bgs_level0"] = {"launches": cnt, "avg_us": ms * 1e3 / max(cnt, 1),
                            "algorithmic_bytes_per_launch": by / max(cnt, 1),
                            "GB/s": by / max(ms * 1e-3, 1e-12) / 1e9,
                            "bytes": "entries 12 B, b, x read and written, diagonal and 3 values of the inverse "
                                     "block per row"}
    del rp, ci, v, b
    torch.cuda.empty_cache()
    return out


def large_section(A, P, n: int = 512, seed: int = 2):
    """Layered 512^3 (contrast ~1e6): FP64 operator, FP32 hierarchy and
    smoother in flexible CG to 1e-8; per-kernel-class GB/s from HIP events of
    one more solve; FP64 solution error against a plain-FP64 PCG solve to
    1e-12 on the same GPU.  The field and right-hand side are drawn on the
    host (default_rng(seed)), the operator is assembled on the device."""
    import torch

    t = time.perf_counter()
    K, b_lex, _ = P.layered_field_and_rhs(n, seed)
    Kt = torch.from_numpy(K).cuda()
    del K
    rp, ci, v, order = P.ccfv7_torch(Kt)
    del Kt
    b = torch.from_numpy(b_lex).cuda()[order].contiguous()
    del b_lex, order
    torch.cuda.synchronize()
    gen = time.perf_counter() - t
    out = {"workload": f"layered K {n}^3 (u_z ~ U[-3,3] per 4-cell z-layer times lognormal sigma=1, seed {seed}), "
                       f"FP32 cycle ({HEAD_TEXT}) in FP64 flexible CG to 1e-8",
           "unknowns": rp.numel() - 1, "nnz": ci.numel(), "generation_s": gen}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = A.Hierarchy(rp, ci, v, vcycle_fp32=1, **HEAD)
    x, r = h.solve(b, rtol=1e-8, maxit=500)
    torch.cuda.synchronize()
    out.update(time_to_1e8_ms=(time.perf_counter() - t0) * 1e3, setup_ms=r.setup_ms, solve_ms=r.solve_ms,
               iterations=r.iterations, levels=h.levels, true_rel_residual=r.true_rel_residual,
               hierarchy_bytes=h.bytes)
    A.set_kernel_timing(True)
    A.reset_kernel_timing()
    h.solve(b, rtol=1e-8, maxit=500)
    A.set_kernel_timing(False)
    names = {A.KIND_SPMV_F64: "spmv_f64_level0", A.KIND_SWEEP: "gs_colour_pass_level0",
             A.KIND_RESTRICT: "residual_restrict_level0", A.KIND_PROLONG: "prolong_level0",
             A.KIND_CG_VEC: "cg_vectors", A.KIND_COARSE_LEVELS: "levels_1_and_below", A.KIND_OTHER: "fills_level0"}
    out["kernel_gbs"] = {}
    for k, nm in names.items():
        ms, cnt, by = A.kernel_timing(k)
        if cnt:
            out["kernel_gbs"][nm] = {"GB/s": by / (ms * 1e-3) / 1e9, "launches": cnt, "ms": ms}
    h.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h64 = A.Hierarchy(rp, ci, v, vcycle_fp32=0, **HEAD)
    x64, r64 = h64.solve(b, rtol=1e-8, maxit=500)
    torch.cuda.synchronize()
    out["plain_fp64"] = {"time_to_1e8_ms": (time.perf_counter() - t0) * 1e3, "iterations": r64.iterations}
    xr, rr = h64.solve(b, rtol=1e-12, maxit=1000, raise_on_error=False)
    h64.close()
    nr = float(torch.linalg.norm(xr))
    out["fp64_solution_error_mixed"] = float(torch.linalg.norm(x - xr)) / nr
    out["fp64_solution_error_plain"] = float(torch.linalg.norm(x64 - xr)) / nr
    out["reference"] = {"rtol": 1e-12, "iterations": rr.iterations, "status": int(rr.status),
                        "true_rel_residual": rr.true_rel_residual}
    out["speedup_mixed_vs_plain_fp64"] = out["plain_fp64"]["time_to_1e8_ms"] / out["time_to_1e8_ms"]
    del rp, ci, v, b, x, x64, xr
    torch.cuda.empty_cache()
    return out


def mcsgs_all_levels(A, args, rp, ci, v, b, timed, infos, ms_per_step):
    """The headline method with the multicolour smoother on every level,
    timed like the headline, and the event-timed time of all launches of
    levels >= 1 per V-cycle for both smoothings (one more solve each)."""
    _, cinfos, per_mc, ms_mc, _ = timed(False, "plain-fp64-mcsgs-all-levels", smoothing={})
    coarse = {}
    for key, sm in (("headline", HEAD), ("mcsgs_all_levels", {})):
        hc = A.Hierarchy(rp, ci, v, vcycle_fp32=0, **sm)
        A.set_kernel_timing([A.KIND_COARSE_LEVELS])
        A.reset_kernel_timing()
        _, rc = hc.solve(b)
        A.set_kernel_timing(False)
        hc.close()
        cms, cl, _ = A.kernel_timing(A.KIND_COARSE_LEVELS)
        coarse[key] = {"ms_per_vcycle": cms / max(rc.iterations, 1), "launches_per_vcycle": cl / max(rc.iterations, 1)}
    lc = cinfos[-1]
    mcsgs_all = {"method": "V(1,1) MC-SGS on every level, plain FP64 PCG to 1e-8", "ms_per_step": ms_mc,
                 "step_ms_min": min(per_mc), "step_ms_max": max(per_mc), "setup_ms": lc.setup_ms,
                 "solve_ms": lc.solve_ms, "iterations": lc.iterations, "true_rel_residual": lc.true_rel_residual,
                 "headline_speedup": ms_mc / ms_per_step,
                 "headline_solve_speedup": lc.solve_ms / infos[-1].solve_ms,
                 "coarse_levels_event_timed": coarse}
    log(f"mcsgs on all levels: {ms_mc:.1f} ms/step (solve {lc.solve_ms:.1f} ms, it={lc.iterations}); "
        f"coarse levels per V-cycle {coarse}")
    return mcsgs_all


def extra_sections(args, A, P, torch, step, timed, x_plain, ms_per_step):
    """config.mixed (FP32 cycle, timed like the headline), config.c1 (32^3
    Poisson) and config.c2 (128^3 heterogeneous, plain against mixed)."""
    import numpy as np

    # The FP32 V-cycle inside FP64 flexible CG, timed the same way.
    x_mixed, minfos, per_mixed, ms_mixed, _ = timed(True, "mixed")
    extra = {}
    x_ref, rref, _ = step(False, rtol=1e-12)
    nref = torch.linalg.norm(x_ref)
    err_mixed = float(torch.linalg.norm(x_mixed - x_ref) / nref)
    err_plain = float(torch.linalg.norm(x_plain - x_ref) / nref)
    lm = minfos[-1]
    extra["mixed"] = {
        "method": f"FP32 cycle ({HEAD_TEXT}; FP32 values, vectors and accumulation on levels above the "
                  "coarsest) inside FP64 flexible CG (Polak-Ribiere beta), to 1e-8",
        "ms_per_step": ms_mixed, "solves_per_s": 1e3 / ms_mixed, "steps": args.steps, "warmup": args.warmup,
        "step_ms_min": min(per_mixed), "step_ms_max": max(per_mixed),
        "setup_ms": lm.setup_ms, "solve_ms": lm.solve_ms, "iterations": lm.iterations,
        "true_rel_residual": lm.true_rel_residual, "fp64_solution_error": err_mixed,
        "speedup_vs_plain_fp64": ms_per_step / ms_mixed,
    }
    extra["plain_fp64_solution_error"] = err_plain
    extra["reference_solve"] = {"rtol": 1e-12, "iterations": rref.iterations,
                                "true_rel_residual": rref.true_rel_residual}

    # Configuration 1: 32^3 Poisson (K = 1), seed 0, plain FP64: time to
    # 1e-8 (median of five), iterations, levels and solve-phase launches per
    # iteration (counted by the library's launch timers).
    s1 = P.poisson(32, seed=0)
    d1 = A.to_device(s1)
    t1s = []
    for _ in range(6):
        torch.cuda.synchronize()
        a = time.perf_counter()
        _, r1, lev1 = step(False, system=d1)
        torch.cuda.synchronize()
        t1s.append((time.perf_counter() - a) * 1e3)
    h1 = A.Hierarchy(*d1[:3], vcycle_fp32=0, **HEAD)
    A.set_kernel_timing(True)
    A.reset_kernel_timing()
    _, r1t = h1.solve(d1[3])
    A.set_kernel_timing(False)
    h1.close()
    launches = sum(A.kernel_timing(k)[1] for k in range(7))
    extra["c1"] = {"workload": "Poisson K=1 32^3 (32768 unknowns, 223232 nnz), b U[-1,1] seed 0, plain FP64 "
                               f"PCG to 1e-8, {HEAD_TEXT}",
                   "time_to_1e8_ms": float(np.median(t1s[1:])), "setup_ms": r1.setup_ms, "solve_ms": r1.solve_ms,
                   "iterations": r1.iterations, "levels": lev1, "true_rel_residual": r1.true_rel_residual,
                   "solve_launches_per_iteration": launches / max(r1t.iterations, 1)}
    log(f"c1: {extra['c1']}")
    del d1

    # Configuration 2: 128^3 heterogeneous (sigma^2 = 4, seed 1), plain FP64
    # against the FP32 cycle, both to 1e-8 (median of three after one warm-up).
    s2 = P.lognormal(128, seed=1)
    d2 = A.to_device(s2)
    c2 = {"workload": "lognormal K 128^3 (sigma^2=4, 2x2x2 box filter, seed 1), 2.1M unknowns"}
    xs2 = {}
    for fp32, key in ((False, "plain_fp64"), (True, "mixed")):
        ts2 = []
        for _ in range(4):
            torch.cuda.synchronize()
            a = time.perf_counter()
            x2, r2, lev2 = step(fp32, system=d2)
            torch.cuda.synchronize()
            ts2.append((time.perf_counter() - a) * 1e3)
        xs2[key] = x2
        c2[key] = {"time_to_1e8_ms": float(np.median(ts2[1:])), "setup_ms": r2.setup_ms, "solve_ms": r2.solve_ms,
                   "iterations": r2.iterations, "levels": lev2, "true_rel_residual": r2.true_rel_residual}
    x2r, _, _ = step(False, rtol=1e-12, system=d2)
    for key in xs2:
        c2[key]["fp64_solution_error"] = float(torch.linalg.norm(xs2[key] - x2r) / torch.linalg.norm(x2r))
    c2["speedup_mixed_vs_plain_fp64"] = c2["plain_fp64"]["time_to_1e8_ms"] / c2["mixed"]["time_to_1e8_ms"]
    extra["c2"] = c2
    log(f"c2: {c2}")
    del d2, xs2, x2r

    return extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--cpu-sample-n", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-systems", type=int, default=64, help="systems of the batched section (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=1.0, help="length of the request stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="request arrival rate (per s)")
    ap.add_argument("--large-n", type=int, default=512, help="edge of the layered large section (0: skip)")
    ap.add_argument("--block-n", type=int, default=96, help="edge of the point-based (block) AMG section (0: skip)")
    ap.add_argument("--no-bicgstab", action="store_true",
                    help="skip the BiCGSTAB / hybrid-smoother solves of the headline system")
    ap.add_argument("--only-headline", action="store_true",
                    help="run the headline steps and the event-timed step only (for profiler runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is not implemented",
              file=sys.stderr)
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

    def step(fp32: bool, x=None, rtol=1e-8, system=None, smoothing=HEAD):
        srp, sci, sv, sb = system if system is not None else (rp, ci, v, b)
        h = A.Hierarchy(srp, sci, sv, vcycle_fp32=1 if fp32 else 0, **smoothing)
        x, r = h.solve(sb, x, rtol=rtol)
        levels = h.levels
        h.close()
        return x, r, levels

    def timed(fp32: bool, label: str, smoothing=HEAD):
        """args.warmup untimed steps, then args.steps steps between two device
        synchronisations; per-step wall times give the spread."""
        for w in range(args.warmup):
            _, r, _ = step(fp32, smoothing=smoothing)
            log(f"{label} warmup {w}: setup {r.setup_ms:.1f} ms solve {r.solve_ms:.1f} ms it={r.iterations}")
        infos, per = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            a = time.perf_counter()
            x, r, levels = step(fp32, smoothing=smoothing)
            per.append((time.perf_counter() - a) * 1e3)
            infos.append(r)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        for r in infos:
            log(f"{label} timed step: setup {r.setup_ms:.1f} ms solve {r.solve_ms:.1f} ms it={r.iterations} "
                f"true_rel_res={r.true_rel_residual:.2e}")
        return x, infos, per, ms, levels

    # Headline: the plain FP64 method.
    x_plain, infos, per_plain, ms_per_step, levels = timed(False, "plain-fp64")

    # Per-kernel HIP-event timing of the dominant kernel, the level-0 colour
    # pass of the FP64 smoother: one more plain step with event timing on
    # (iterations launched individually; they are the kernels the timed steps
    # ran).  Algorithmic bytes of a level-0 colour pass by the survey's
    # count: 12 B per stored entry of the colour's rows (value + column) and
    # 28 B per row (row pointer, b, x read, x written).
    h = A.Hierarchy(rp, ci, v, vcycle_fp32=0, **HEAD)
    col0 = np.zeros(s.n, np.int32)
    A._check(A.lib().amg_copy_level(h.h, 0, None, col0.ctypes.data_as(A.C.c_void_p), None, None, None, None, None))
    rows_c = np.bincount(col0)
    nnz_c = np.bincount(col0, weights=np.diff(s.rowptr).astype(np.float64))
    A.set_kernel_timing([A.KIND_SWEEP])
    A.reset_kernel_timing()
    _, rt = h.solve(b)
    A.set_kernel_timing(False)
    h.close()
    sweep_ms, sweep_launches, sweep_bytes = A.kernel_timing(A.KIND_SWEEP)

    log(f"event-timed step: solve {rt.solve_ms:.1f} ms, {sweep_launches} sweep launches, colours {rows_c.tolist()}")
    # the kb_gs passes of a V(1,1) cycle on two colours: pre colour 1, post colours 0, 1, 0
    survey_pass = [12.0 * nnz_c[c] + 28.0 * rows_c[c] for c in range(len(rows_c))]
    survey_bytes = float(np.mean(survey_pass)) if len(rows_c) == 2 else float(12.0 * s.nnz + 28.0 * s.n) / len(rows_c)

    # The same method with the multicolour smoother on every level, timed
    # the same way, and the event-timed time of all launches of levels >= 1
    # per V-cycle for both (one more solve each); not in profiler runs.
    mcsgs_all = None
    if not args.only_headline:
        mcsgs_all = mcsgs_all_levels(A, args, rp, ci, v, b, timed, infos, ms_per_step)

    extra = {"step_ms_min": min(per_plain), "step_ms_max": max(per_plain)}
    if args.only_headline:
        args.no_bicgstab, args.large_n, args.batched_systems, args.serve_seconds = True, 0, 0, 0
        args.block_n = 0
        args.no_cpu_baseline = True
    else:
        extra.update(extra_sections(args, A, P, torch, step, timed, x_plain, ms_per_step))

    # The oracle's CPU baseline runs on one pinned host core in a thread of
    # its own while the remaining sections use the GPU (the oracle is a C
    # call that releases the interpreter lock).
    cpu_thread = None
    if not args.no_cpu_baseline:
        import threading

        log(f"cpu baseline: oracle at {args.cpu_sample_n}^3 on one pinned core, alongside the GPU sections ...")
        cpu_res = {}

        def cpu_job():
            try:
                cpu_res["out"] = cpu_baseline(args.cpu_sample_n)
            except Exception as e:  # reported in the line instead of a baseline
                cpu_res["error"] = repr(e)
            log("cpu baseline: done")

        cpu_thread = threading.Thread(target=cpu_job, daemon=True)
        cpu_thread.start()

    if not args.no_bicgstab:
        # The paper's outer solver (Sec. 5): BiCGSTAB, two V-cycles per
        # iteration, same hierarchy parameters, both V-cycle precisions.
        # With the hybrid smoother (Sec. 3.2; block-Jacobi over the tiles) it
        # is the paper's own solver configuration; CG with it for comparison.
        bic = {}
        # (smoother, FP32 cycle, method, the headline's coarse-level smoothing)
        runs = [(0, 1, "bicgstab", False), (0, 0, "bicgstab", False), (2, 1, "bicgstab", False),
                (2, 0, "bicgstab", False), (2, 1, "cg", False), (0, 0, "bicgstab", True)]
        for smoother, fp32, method, head in runs:
            torch.cuda.synchronize()
            q0 = time.perf_counter()
            h = A.Hierarchy(rp, ci, v, vcycle_fp32=fp32, smoother=smoother, **(HEAD if head else {}))
            xb, rb = h.solve(b, rtol=1e-8, method=method)
            h.close()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - q0) * 1e3
            key = ("bicgstab" if method == "bicgstab" else "cg") + ("_hybrid_sgs" if smoother == 2 else "_mcsgs") + \
                ("_tile_mcsgs_coarse" if head else "") + ("_fp32_vcycle" if fp32 else "_fp64_vcycle")
            bic[key] = {
                "time_to_1e8_ms": ms, "setup_ms": rb.setup_ms, "solve_ms": rb.solve_ms,
                "iterations": rb.iterations, "half_step_exit": bool(rb.half_step),
                "ms_per_iteration": rb.solve_ms / max(rb.iterations, 1), "true_rel_residual": rb.true_rel_residual,
                "status": A.STATUS[rb.status]}
            log(f"{key}: {ms:.1f} ms (setup {rb.setup_ms:.1f}, solve {rb.solve_ms:.1f}), "
                f"it={rb.iterations} half={rb.half_step} true_rel_res={rb.true_rel_residual:.2e}")
        extra["paper_solver"] = bic
        # Iteration counts on the paper's Laplace problem (K = 1), the
        # setting of its Table 1 (80^3 on one process: 5 levels, It = 8) and
        # Table 4 (256^3 on one process: It = 6), BiCGSTAB with the
        # multicolour, hybrid and tile-ordered smoothers; the hybrid blocks
        # also larger on level 0 and smaller on the coarse levels.
        lap = {}
        for m in (80, 256):
            sl = P.poisson(m)
            lrp, lci, lv, lb = A.to_device(sl)
            # (smoother, aggregation tiles, smoothing blocks above level 1, from level 1)
            for smoother, tiles, stile, ctile in ((0, 128, 0, 0), (2, 128, 0, 0), (0, 1024, 0, 0), (2, 128, 256, 0),
                                                  (2, 128, 128, 64), (2, 128, 256, 64), (3, 128, 0, 0)):
                torch.cuda.synchronize()
                q0 = time.perf_counter()
                h = A.Hierarchy(lrp, lci, lv, smoother=smoother, tile_rows=tiles, smooth_tile_rows=stile,
                                coarse_smooth_tile_rows=ctile)
                _, rl = h.solve(lb, rtol=1e-8, method="bicgstab")
                lev = h.levels
                h.close()
                torch.cuda.synchronize()
                tag = {0: 'mcsgs', 2: 'hybrid_sgs', 3: 'tile_mcsgs'}[smoother]
                tag += "" if tiles == 128 else f"_tiles{tiles}"
                tag += f"_blocks{stile}" if stile else ""
                tag += f"_coarse_blocks{ctile}" if ctile else ""
                lap[f"{m}^3_{tag}"] = {
                    "levels": lev, "iterations": rl.iterations, "half_step_exit": bool(rl.half_step),
                    "time_to_1e8_ms": (time.perf_counter() - q0) * 1e3, "setup_ms": rl.setup_ms,
                    "solve_ms": rl.solve_ms, "true_rel_residual": rl.true_rel_residual}
            del lrp, lci, lv, lb
        lap["paper_one_process"] = {"80^3": {"levels": 5, "iterations": 8}, "256^3": {"iterations": 6}}
        log("laplace: " + ", ".join(f"{k} it={v['iterations']} lev={v['levels']}" for k, v in lap.items()
                                    if "levels" in v and "iterations" in v and k != "paper_one_process"))
        bic["laplace_bicgstab_fp64_vcycle"] = lap
        # The paper's other workloads at its one-process sizes: the
        # manufactured Poisson problem at 190^3 (Table 3: 5 levels, It = 8;
        # solution error against exp(-|x|^2)) and the jump-coefficient cube at
        # 80^3 (Table 6: 5 levels, It = 9).
        wl = {}
        sm, um = P.manufactured(190)
        sj = P.jump_cube(80)
        for name, sysw in (("manufactured_190^3", sm), ("jump_cube_80^3", sj)):
            wrp, wci, wv, wb = A.to_device(sysw)
            for smoother in (0, 2):
                torch.cuda.synchronize()
                q0 = time.perf_counter()
                h = A.Hierarchy(wrp, wci, wv, smoother=smoother)
                xw, rw = h.solve(wb, rtol=1e-8, method="bicgstab")
                lev = h.levels
                h.close()
                torch.cuda.synchronize()
                rec = {"levels": lev, "iterations": rw.iterations, "time_to_1e8_ms": (time.perf_counter() - q0) * 1e3,
                       "setup_ms": rw.setup_ms, "solve_ms": rw.solve_ms, "true_rel_residual": rw.true_rel_residual}
                if sysw is sm:
                    rec["max_error_vs_exact"] = float((xw.cpu() - torch.from_numpy(um)).abs().max())
                wl[f"{name}_{'hybrid_sgs' if smoother == 2 else 'mcsgs'}"] = rec
            del wrp, wci, wv, wb
        wl["paper_one_process"] = {"manufactured_190^3": {"levels": 5, "iterations": 8},
                                   "jump_cube_80^3": {"levels": 5, "iterations": 9}}
        log("workloads: " + ", ".join(f"{k} it={v['iterations']} lev={v['levels']}" for k, v in wl.items()
                                      if k != "paper_one_process"))
        bic["paper_workloads_bicgstab_fp64_vcycle"] = wl

    avg_launch_ms = sweep_ms / max(sweep_launches, 1)
    sell_bytes = sweep_bytes / max(sweep_launches, 1)
    achieved = survey_bytes / (avg_launch_ms * 1e-3) / 1e9 if sweep_launches else None
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"lognormal-K 7-point CCFV {n}^3 (sigma^2=4, 2x2x2 box filter, seed 1), plain FP64: "
                        f"{HEAD_TEXT}, in PCG to rtol 1e-8 (setup + solve + free per step)",
            "unknowns": s.n, "nnz": s.nnz, "levels": levels, "iterations": last.iterations,
            "setup_ms": last.setup_ms, "solve_ms": last.solve_ms, "time_to_1e8_ms": ms_per_step,
            "true_rel_residual": last.true_rel_residual, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "kb_gs<double, 1, true> (one level-0 colour pass of the FP64 Gauss-Seidel smoother, SELL-64)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic,
            "method": "HIP events on the launch stream around every level-0 colour pass of one extra plain "
                      "FP64 solve of the same system after the timed steps; achieved = algorithmic bytes per "
                      "pass (12 B per stored entry of the colour's rows + 28 B per row) / average duration",
            "launches": sweep_launches,
            "avg_launch_us": avg_launch_ms * 1e3,
            "algorithmic_bytes_per_launch": survey_bytes,
            "sell_bytes_per_launch": sell_bytes,
            "sell_frac": (sell_bytes / (avg_launch_ms * 1e-3) / 1e9) / HBM_PEAK_GBS if sweep_launches else None,
            "colour_rows": rows_c.tolist(), "colour_entries": [int(x) for x in nnz_c],
        },
    }
    out["config"].update(extra)
    if mcsgs_all is not None:
        out["config"]["mcsgs_all_levels"] = mcsgs_all
    if args.block_n > 0:
        log(f"block section (coupled 3-component {args.block_n}^3) ...")
        out["block"] = block_section(A, P, args.block_n)
    if args.large_n > 0:
        log(f"large section (layered {args.large_n}^3) ...")
        out["large"] = large_section(A, P, args.large_n)
        log(f"large: {out['large']['time_to_1e8_ms']:.0f} ms, {out['large']['iterations']} iterations, "
            f"FP64 error {out['large']['fp64_solution_error_mixed']:.2e}")
    if args.batched_systems > 0:
        log("batched section ...")
        out["batched"] = batched_section(A, P, args.batched_systems)
        log(f"batched: {out['batched']['batched_ms']:.0f} ms vs loop {out['batched']['loop_ms']:.0f} ms")
    if args.serve_seconds > 0:
        A.release_cached_memory()
        torch.cuda.empty_cache()
        log("serving section ...")
        out["serving"] = serving_section(A, P, args.serve_seconds, args.serve_rate)
        log(f"serving: {out['serving']['served']['solves_per_s']:.1f} solves/s p99 "
            f"{out['serving']['served']['p99_ms']:.0f} ms vs serial {out['serving']['serial_fp64']['solves_per_s']:.1f}"
            f" solves/s p99 {out['serving']['serial_fp64']['p99_ms']:.0f} ms")
    if cpu_thread is not None:
        if cpu_thread.is_alive():
            log("waiting for the cpu baseline ...")
        cpu_thread.join()
        out["cpu_baseline"] = cpu_res.get("out") or {"error": cpu_res.get("error")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
