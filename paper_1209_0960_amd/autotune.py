"""Autotuner for batched solves of many uneven systems.

Three launch/layout variants are chosen by measurement on the GPU:

* tile variant, per size class: `tile_rows`, the rows of a decoupled
  aggregation tile (Alg. 4's unit of independent aggregation; it sets the
  setup's parallelism and per-tile latency, and the hierarchy it builds);
* cycle variant, per size class: `tail_rows`, below which a system's levels
  are cycled by one workgroup instead of one launch per colour pass, and the
  coarse-level smoother (the multicolour smoother on every level, or the
  tile-ordered multicolour smoother from level 1 on);
* SpMV variant, per size class: `spmv_format`, the layout of CG's level-0
  product (SELL-64 slices with one lane per row, or CSR with a group of lanes
  per row); per batch: R, the right-hand sides interleaved in one entry
  (R > 1 reads every matrix once for R products; R = 1 gives R entries per
  system and more independent work).

`tail_rows` = 2^30 cycles every level of a system by one workgroup (the
whole V-cycle of an entry in one launch per leg).

A size class is the rows of a system.  For each class the candidates are
timed on a sample of the batch's own systems (batched setup plus batched
solve, best of `reps`); R is then timed on the whole batch with the chosen
per-class parameters.  The table maps class -> parameters and is reusable.
"""
from __future__ import annotations

import itertools
import time
from collections import defaultdict

import torch

from . import amg as A

TILES = (64, 128, 256, 512)
TAILS = (0, 8192, 1 << 30)
COARSE = ({}, {"coarse_smoother": A.SMOOTHER_TILE_MCSGS, "coarse_from": 1})
SPMV = (0, 1)
RHS = (4, 2, 1)


def _variant_name(tile, tail, coarse):
    return f"tile_rows={tile},tail_rows={tail},coarse={'tile_mcsgs' if coarse else 'mcsgs'}"


def _sync():
    torch.cuda.synchronize()


def run_batched(systems, params_of, nrhs: int, R: int, rtol: float = 1e-8, maxit: int = 500, **common):
    """Batched setup (one amg_setup_batched per parameter group) and one
    pcg_solve_batched over all systems with R right-hand sides per entry.
    systems: list of (rowptr, colind, vals, b) with b holding nrhs * n values.
    params_of(i) -> dict of per-system parameters.  Returns (setup_s, solve_s,
    infos per system and right-hand side, hierarchies closed)."""
    if nrhs % R:
        raise ValueError("R must divide the right-hand sides per system")
    groups = defaultdict(list)
    for i in range(len(systems)):
        groups[tuple(sorted(params_of(i).items()))].append(i)
    _sync()
    t0 = time.perf_counter()
    hs = [None] * len(systems)
    for key, idx in groups.items():
        made = A.Hierarchy.batched([systems[i][:3] for i in idx], **dict(key), **common)
        for i, h in zip(idx, made):
            hs[i] = h
    _sync()
    t1 = time.perf_counter()
    handles, bs, xs, who = [], [], [], []
    for i, (rp, ci, v, b) in enumerate(systems):
        n = rp.numel() - 1
        for j in range(nrhs // R):
            handles.append(hs[i].h)
            bs.append(b[j * R * n:(j + 1) * R * n])
            xs.append(torch.zeros(R * n, dtype=torch.float64, device=b.device))
            who.append(i)
    st, infos = A.pcg_solve_batched(handles, bs, xs, nrhs=R, rtol=rtol, maxit=maxit)
    _sync()
    t2 = time.perf_counter()
    for h in hs:
        h.close()
    per = defaultdict(list)
    for i, inf in zip(who, infos):
        per[i].extend(inf)
    return t1 - t0, t2 - t1, [per[i] for i in range(len(systems))], st, xs


def tune(systems, nrhs: int, sample: int = 4, reps: int = 2, **common) -> dict:
    """Table {rows: {"tile_rows", "tail_rows", "coarse", "spmv_format", "ms",
    "variants_ms"}} per size class (every timed variant kept), plus {"R": best
    interleave, "R_ms": {R: ms}} for the whole batch."""
    by_class = defaultdict(list)
    for i, s in enumerate(systems):
        by_class[s[0].numel() - 1].append(i)
    table = {}
    t_start = time.perf_counter()
    for rows, idx in sorted(by_class.items()):
        pick = [systems[i] for i in idx[:sample]]
        best = None
        variants = {}
        for tile, tail, coarse in itertools.product(TILES, TAILS, COARSE):
            ms = float("inf")
            for _ in range(reps):
                try:
                    a, b, _, st, _ = run_batched(pick, lambda i: {"tile_rows": tile, "tail_rows": tail, **coarse},
                                                 nrhs, nrhs, **common)
                except A.AMGError:  # e.g. a tile graph larger than the LDS
                    break
                if st == A.OK:
                    ms = min(ms, (a + b) * 1e3)
            variants[_variant_name(tile, tail, coarse)] = ms
            if best is None or ms < best[3]:
                best = (tile, tail, coarse, ms)
        fmt, fms = 0, best[3]
        for f in SPMV[1:]:  # the SpMV layout with the chosen tile and cycle variants
            ms = float("inf")
            for _ in range(reps):
                a, b, _, st, _ = run_batched(pick, lambda i: {"tile_rows": best[0], "tail_rows": best[1], **best[2],
                                                              "spmv_format": f}, nrhs, nrhs, **common)
                if st == A.OK:
                    ms = min(ms, (a + b) * 1e3)
            variants[_variant_name(best[0], best[1], best[2]) + f",spmv_format={f}"] = ms
            if ms < fms:
                fmt, fms = f, ms
        table[rows] = {"tile_rows": best[0], "tail_rows": best[1], "coarse": dict(best[2]), "spmv_format": fmt,
                       "ms": fms, "variants_ms": variants}

    params_of = params_from(table, systems)

    rms = {}
    for R in RHS:
        if nrhs % R:
            continue
        a, b, _, st, _ = run_batched(systems, params_of, nrhs, R, **common)
        rms[R] = (a + b) * 1e3 if st == A.OK else float("inf")
    table["R"] = min(rms, key=rms.get)
    table["R_ms"] = rms
    table["tuning_s"] = time.perf_counter() - t_start
    return table


def params_from(table: dict, systems) -> callable:
    def params_of(i):
        c = table[systems[i][0].numel() - 1]
        return {"tile_rows": c["tile_rows"], "tail_rows": c["tail_rows"], "spmv_format": c.get("spmv_format", 0),
                **c.get("coarse", {})}
    return params_of
