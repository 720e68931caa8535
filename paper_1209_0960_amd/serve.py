"""Serving loop: a stream of solve requests with continuous batching.

Requests (a matrix key, a right-hand side, an arrival time) are admitted in
arrival order as memory and batch slots allow:

* hierarchies stay on the device in an LRU cache keyed by matrix; a request
  whose matrix is cached skips the setup (a "hit"), otherwise its hierarchy is
  built by amg_setup on a background host thread with its own stream, so
  setups overlap the running solves on the device;
* admission is by device-memory footprint (amg_estimate_bytes): the cached
  hierarchies, the solve contexts of running requests and the setup peaks of
  running setups stay under `cap_bytes`; idle hierarchies are evicted least
  recently used first;
* admitted solves join the running batch (amg_batch_submit) between two
  iterations and leave it when converged; every step advances all of them by
  one CG iteration in shared launches (amg_batch_step).

An entry's arithmetic does not depend on the others, so each result equals
that of pcg_solve on the same hierarchy alone, bit for bit.  Latency is
completion time minus scheduled arrival time.
"""
from __future__ import annotations

import collections
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import amg as A
from . import problems as P


@dataclass
class Request:
    id: int
    t: float          # scheduled arrival (s from the start of the run)
    matrix: int       # key of the matrix (requests with one key share a hierarchy)
    rowptr: torch.Tensor
    colind: torch.Tensor
    vals: torch.Tensor
    b: torch.Tensor


@dataclass
class Record:
    id: int
    matrix: int
    n: int
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    status: int = -1
    iterations: int = 0
    true_rel_residual: float = float("nan")
    hit: bool = False
    setup_ms: float = 0.0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class Summary:
    requests: int
    makespan_s: float
    solves_per_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    hits: int
    setups: int
    evictions: int
    peak_reserved_bytes: int
    max_running: int
    extra: dict = field(default_factory=dict)


def summarise(records: list, **extra) -> Summary:
    lat = np.array([r.latency for r in records]) * 1e3
    makespan = max(r.done for r in records)
    return Summary(len(records), makespan, len(records) / makespan, float(np.percentile(lat, 50)),
                   float(np.percentile(lat, 99)), float(lat.mean()), sum(r.hit for r in records),
                   extra.pop("setups", 0), extra.pop("evictions", 0), extra.pop("peak", 0),
                   extra.pop("max_running", 0), extra)


class Server:
    """Continuous-batching request loop over the native engine."""

    def __init__(self, cap_bytes: float = 200e9, max_entries: int = 32, rtol: float = 1e-8, maxit: int = 500,
                 setup_workers: int = 2, use_graphs: bool = True, keep_solutions: bool = False, **params):
        self.params = dict(params)
        self.p = A.default_params(**params)
        self.cap = float(cap_bytes)
        self.rtol, self.maxit = rtol, maxit
        self.batch = A.Batch(nrhs=1, max_entries=max_entries, use_graphs=use_graphs)
        self.max_entries = max_entries
        self.cache: collections.OrderedDict = collections.OrderedDict()  # key -> Hierarchy (LRU first)
        self.hbytes: dict = {}
        self.inuse = collections.Counter()
        self.pool = ThreadPoolExecutor(max_workers=setup_workers)
        self.workers = setup_workers
        self.streams = [torch.cuda.Stream() for _ in range(setup_workers)]
        self.free_streams = list(range(setup_workers))
        self.keep = keep_solutions
        self.solutions: dict = {}
        self.setups = self.evictions = 0

    # ---------------------------------------------------------------- memory
    def _resident(self) -> float:
        return sum(self.hbytes.values()) + self.reserved

    def _make_room(self, need: float) -> bool:
        """Evict idle hierarchies (LRU first) until `need` more bytes fit."""
        while self._resident() + need > self.cap:
            victim = next((k for k in self.cache if self.inuse[k] == 0), None)
            if victim is None:
                return False
            self.cache.pop(victim).close()
            self.hbytes.pop(victim)
            self.evictions += 1
        return True

    def _build(self, req: Request, stream_idx: int):
        s = self.streams[stream_idx]
        t = time.perf_counter()
        h = A.Hierarchy(req.rowptr, req.colind, req.vals, stream=s, **self.params)
        return h, (time.perf_counter() - t) * 1e3

    # ---------------------------------------------------------------- loop
    def run(self, requests: list) -> list:
        reqs = sorted(requests, key=lambda r: r.t)
        rec = {r.id: Record(r.id, r.matrix, r.rowptr.numel() - 1, r.t) for r in reqs}
        arriving = collections.deque(reqs)
        queue: list = []
        building: dict = {}       # key -> (future, reserved bytes, stream index, request id)
        built_by: dict = {}       # key -> request whose arrival triggered the latest setup
        running: dict = {}        # id -> (request, x, reserved bytes)
        self.reserved = 0.0
        peak = 0.0
        max_running = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while arriving or queue or running or building:
            now = time.perf_counter() - t0
            while arriving and arriving[0].t <= now:
                queue.append(arriving.popleft())
            # finished setups enter the cache
            for key in [k for k, v in building.items() if v[0].done()]:
                fut, res, si, rid = building.pop(key)
                h, ms = fut.result()
                self.reserved -= res
                self.free_streams.append(si)
                self.cache[key] = h
                self.hbytes[key] = h.bytes
                rec[rid].setup_ms = ms
            # admission in arrival order; setups start in arrival order
            setup_blocked = False
            for r in list(queue):
                key = r.matrix
                n, nnz = r.rowptr.numel() - 1, r.colind.numel()
                est = A.estimate_bytes(n, nnz, self.p)
                if key in self.cache:
                    if len(running) >= self.max_entries:
                        continue
                    self.inuse[key] += 1  # pinned: room is made by evicting others
                    if not self._make_room(est["context"]):
                        self.inuse[key] -= 1
                        continue
                    self.cache.move_to_end(key)
                    x = torch.zeros_like(r.b)
                    self.batch.submit(self.cache[key], r.b, x, self.rtol, self.maxit, tag=r.id)
                    self.reserved += est["context"]
                    running[r.id] = (r, x, est["context"])
                    rec[r.id].admitted = time.perf_counter() - t0
                    rec[r.id].hit = built_by.get(key) != r.id
                    queue.remove(r)
                elif key not in building and not setup_blocked:
                    if not self.free_streams or not self._make_room(est["setup_peak"]):
                        setup_blocked = True
                        continue
                    si = self.free_streams.pop()
                    self.reserved += est["setup_peak"]
                    building[key] = (self.pool.submit(self._build, r, si), est["setup_peak"], si, r.id)
                    built_by[key] = r.id
                    self.setups += 1
            peak = max(peak, self._resident())
            max_running = max(max_running, len(running))
            if running:
                self.batch.step(1)
                for tag, st, info in self.batch.poll():
                    r, x, res = running.pop(tag)
                    self.reserved -= res
                    self.inuse[r.matrix] -= 1
                    R = rec[tag]
                    R.done = time.perf_counter() - t0
                    R.status, R.iterations = st, info[0]["iterations"]
                    R.true_rel_residual = info[0]["true_rel_residual"]
                    if self.keep:
                        self.solutions[tag] = x
            elif queue and not building and not arriving and not self.cache:
                raise RuntimeError("request cannot be admitted: cap_bytes below its setup footprint")
            else:  # idle: wait for the next arrival or a setup to finish
                nxt = arriving[0].t - (time.perf_counter() - t0) if arriving else 0.0005
                time.sleep(min(max(nxt, 0.0), 0.0005))
        self.stats = dict(setups=self.setups, evictions=self.evictions, peak=int(peak), max_running=max_running)
        return [rec[r.id] for r in reqs]

    def close(self):
        self.pool.shutdown(wait=True)
        for h in self.cache.values():
            h.close()
        self.cache.clear()
        self.hbytes.clear()
        self.batch.close()


def serve_serial(requests: list, cap_bytes: float = 200e9, rtol: float = 1e-8, maxit: int = 500,
                 keep_solutions: bool = False, **params) -> tuple:
    """Baseline: the same requests served one at a time in arrival order with
    pcg_solve, hierarchies cached (LRU under cap_bytes)."""
    reqs = sorted(requests, key=lambda r: r.t)
    cache: collections.OrderedDict = collections.OrderedDict()
    nb: dict = {}
    rec = []
    sols = {}
    setups = evictions = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        wait = r.t - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        R = Record(r.id, r.matrix, r.rowptr.numel() - 1, r.t)
        R.admitted = time.perf_counter() - t0
        if r.matrix in cache:
            cache.move_to_end(r.matrix)
            R.hit = True
        else:
            while cache and sum(nb.values()) > cap_bytes:
                k, h = cache.popitem(last=False)
                h.close()
                nb.pop(k)
                evictions += 1
            t = time.perf_counter()
            h = A.Hierarchy(r.rowptr, r.colind, r.vals, **params)
            R.setup_ms = (time.perf_counter() - t) * 1e3
            cache[r.matrix] = h
            nb[r.matrix] = h.bytes
            setups += 1
        x, res = cache[r.matrix].solve(r.b, rtol=rtol, maxit=maxit, raise_on_error=False)
        torch.cuda.synchronize()
        R.done = time.perf_counter() - t0
        R.status, R.iterations, R.true_rel_residual = res.status, res.iterations, res.true_rel_residual
        if keep_solutions:
            sols[r.id] = x
        rec.append(R)
    for h in cache.values():
        h.close()
    return rec, dict(setups=setups, evictions=evictions), sols


def requests_from_trace(trace: list, device: str = "cuda") -> tuple:
    """Device inputs of a request stream (problems.serving_trace): a request
    that introduces a matrix draws its lognormal field and then its right-hand
    side from its own generator; a reusing request draws only its right-hand
    side and shares the arrays of its target.  Returns (requests, seconds)."""
    mats: dict = {}
    out = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r in trace:
        g = torch.Generator(device=device).manual_seed(r["seed"])
        e = r["edge"]
        if r["matrix"] == r["id"]:
            rp, ci, v, b = P.lognormal_torch(e, r["sigma2"], g)
            mats[r["id"]] = (rp, ci, v)
        else:
            rp, ci, v = mats[r["matrix"]]
            b = P.rhs_torch(P.morton_order_torch(e, e, e, device), g)
        out.append(Request(r["id"], r["t"], r["matrix"], rp, ci, v, b[0].contiguous()))
    torch.cuda.synchronize()
    return out, time.perf_counter() - t
