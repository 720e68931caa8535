"""Serving loop: every served result equals the solve of the same system alone.

Requests of a short stream (problems.serving_trace recipe, small edges) arrive
while others run, join the batch between iterations, share hierarchies
(reuse), and -- with a small memory cap -- evict and rebuild hierarchies.  A
hierarchy built again from the same matrix is identical (setup is
deterministic), so each served x is compared bit for bit with pcg_solve on a
freshly built hierarchy.
"""
import numpy as np
import pytest
import torch

from paper_1209_0960_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    from paper_1209_0960_amd import amg, serve
    amg.lib()
    return amg, serve


def check_against_alone(A, reqs, recs, sols, **params):
    for r, R in zip(sorted(reqs, key=lambda q: q.t), recs):
        assert R.id == r.id and R.status == A.OK, (R.id, R.status)
        with A.Hierarchy(r.rowptr, r.colind, r.vals, **params) as h:
            x, res = h.solve(r.b, rtol=1e-8, maxit=500)
        assert res.iterations == R.iterations, r.id
        assert torch.equal(sols[r.id], x), r.id
        assert res.true_rel_residual == R.true_rel_residual


def test_served_results_equal_alone(mods):
    A, S = mods
    trace = P.serving_trace(rate=400.0, seconds=0.06, seed=7, edges=(8, 24), reuse=0.4)
    assert len(trace) >= 10 and any(t["matrix"] != t["id"] for t in trace)
    reqs, _ = S.requests_from_trace(trace)
    srv = S.Server(cap_bytes=4e9, max_entries=4, setup_workers=2, keep_solutions=True, vcycle_fp32=1)
    try:
        recs = srv.run(reqs)
        assert srv.stats["max_running"] >= 2  # requests overlapped on the device
    finally:
        srv.close()
    sm = S.summarise(recs, **srv.stats)
    assert sm.requests == len(trace) and sm.p99_ms >= sm.p50_ms > 0
    check_against_alone(A, reqs, recs, srv.solutions, vcycle_fp32=1)


def test_small_cap_evicts_and_rebuilds(mods):
    A, S = mods
    trace = P.serving_trace(rate=300.0, seconds=0.05, seed=9, edges=(16, 24), reuse=0.5)
    reqs, _ = S.requests_from_trace(trace)
    big = max(A.estimate_bytes(r.rowptr.numel() - 1, r.colind.numel(), A.default_params(vcycle_fp32=1))["setup_peak"]
              for r in reqs)
    srv = S.Server(cap_bytes=1.3 * big, max_entries=2, setup_workers=1, keep_solutions=True, vcycle_fp32=1)
    try:
        recs = srv.run(reqs)
        assert srv.stats["evictions"] > 0
        assert srv.stats["peak"] <= 1.3 * big
    finally:
        srv.close()
    check_against_alone(A, reqs, recs, srv.solutions, vcycle_fp32=1)


def test_serial_baseline_matches_alone(mods):
    A, S = mods
    trace = P.serving_trace(rate=400.0, seconds=0.03, seed=11, edges=(8, 16), reuse=0.4)
    reqs, _ = S.requests_from_trace(trace)
    recs, stats, sols = S.serve_serial(reqs, keep_solutions=True, vcycle_fp32=0)
    assert stats["setups"] == len({r.matrix for r in reqs})
    check_against_alone(A, reqs, recs, sols, vcycle_fp32=0)
