"""GPU paths that the main parity file does not reach, each against the CPU
oracle through the C ABI:

* flexible CG (Polak-Ribiere beta) with a non-symmetric FP64 cycle (one
  pre-smoothing step, no post-smoothing): every iterate within 1e-10;
* pcg_solve_batched with four right-hand sides per system (FP64 cycle):
  every right-hand side against the oracle's PCG;
* a served request trace (FP32 cycle, continuous batching) against the
  oracle's flexible CG with its FP32 cycle;
* host-forced statuses: an allocator hook that runs out after k bytes
  (AMG_ERR_OUT_OF_MEMORY, NULL handle, every byte returned), a matrix that
  does not coarsen (AMG_ERR_COARSENING_STALLED and the 0.9 guard, as the
  oracle), an indefinite matrix that breaks CG down (AMG_ERR_BREAKDOWN at the
  oracle's iteration);
* amg_free while a preconditioner application is still queued on another
  stream.
"""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

import oracle as O
from paper_1209_0960_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    from paper_1209_0960_amd import amg
    amg.lib()
    return amg


def rel(a, b):
    """Larger of ||a - b|| / ||b|| and max|a - b| / max|b|."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = a - b
    nrm = np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300)
    ele = np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)
    return float(max(nrm, ele))


def tdev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def compare_levels(hg, ho, tag):
    assert hg.levels == ho.levels, (tag, hg.levels, ho.levels)
    for l in range(ho.levels):
        g, o = hg.level(l), ho.level(l)
        assert g["n"] == o.n and np.array_equal(g["rowptr"], o.rowptr) and np.array_equal(g["colind"], o.colind)
        assert np.array_equal(g["vals"].view(np.int64), o.vals.view(np.int64)), (tag, l)
        assert np.array_equal(g["colour"], o.colour), (tag, l)
        if l < ho.levels - 1:
            assert np.array_equal(g["agg"], o.agg), (tag, l)


# ---------------------------------------------------------------- flexible CG
@pytest.mark.parametrize("name,maker", [("hetero_24", lambda: P.lognormal(24)),
                                        ("jump_20", lambda: P.jump_cube(20))])
def test_fcg_fp64_nonsymmetric_cycle_iterates(A, name, maker):
    """FCG with the Polak-Ribiere beta z.(r - r_old)/rho and a cycle with one
    pre- and no post-smoothing step (not symmetric, so the beta of PCG would
    give other iterates): every FP64 iterate within 1e-10 of the oracle."""
    s = maker()
    rp, ci, v, b = tdev(s.rowptr, s.colind, s.vals, s.b)
    kw = dict(flexible=1, pre_sweeps=1, post_sweeps=0)
    maxit = 200
    with A.Hierarchy(rp, ci, v, **kw) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, **kw)
        hist = torch.zeros((maxit + 1) * s.n, dtype=torch.float64, device="cuda")
        x, r = hg.solve(b, rtol=1e-8, maxit=maxit, iter_hist=hist)
        o = ho.pcg(s.b, rtol=1e-8, maxit=maxit, keep_iterates=True)
        assert r.status == A.OK and o["status"] == O.OK
        assert abs(r.iterations - o["iterations"]) <= 1
        k = min(r.iterations, o["iterations"])
        H = hist.cpu().numpy().reshape(maxit + 1, s.n)
        for it in range(1, k + 1):
            assert rel(H[it], o["iterates"][it]) <= 1e-10, (name, it)
        # the PCG beta on the same cycle gives different iterates
        op = O.Hierarchy(s.rowptr, s.colind, s.vals, flexible=0, pre_sweeps=1, post_sweeps=0).pcg(
            s.b, rtol=1e-8, maxit=maxit, keep_iterates=True)
        kk = min(k, op["iterations"])
        assert max(rel(op["iterates"][i], o["iterates"][i]) for i in range(1, kk + 1)) > 1e-6


# ---------------------------------------------------------------- batched
def test_batched_four_rhs_against_oracle(A):
    """pcg_solve_batched, FP64 cycle, 4 right-hand sides per system: each
    right-hand side's solution and iteration count against the oracle's PCG
    (iterations within one, x within 1e-10 when the counts agree)."""
    rng = np.random.default_rng(21)
    nrhs = 4
    syss = []
    for n in (12, 20, 9, 16):
        K = P.field_lognormal(rng, n, 2.0, 2, np.sqrt(8.0))
        rp, ci, v, order = P.ccfv7(K)
        B = np.ascontiguousarray(rng.uniform(-1.0, 1.0, (nrhs, n ** 3))[:, order])
        syss.append((rp, ci, v, B))
    hs, bs, xs = [], [], []
    for rp, ci, v, B in syss:
        trp, tci, tv, tB = tdev(rp, ci, v, B)
        hs.append(A.Hierarchy(trp, tci, tv, vcycle_fp32=0))
        bs.append(tB.reshape(-1).clone())
        xs.append(torch.zeros_like(bs[-1]))
    try:
        st, infos = A.pcg_solve_batched([h.h for h in hs], bs, xs, nrhs=nrhs, rtol=1e-8, maxit=200)
        assert st == A.OK
        for si, (rp, ci, v, B) in enumerate(syss):
            n = B.shape[1]
            ho = O.Hierarchy(rp, ci, v)
            xg = xs[si].cpu().numpy()
            for k in range(nrhs):
                o = ho.pcg(B[k], rtol=1e-8, maxit=200)
                assert o["status"] == O.OK
                it = infos[si][k]["iterations"]
                assert abs(it - o["iterations"]) <= 1, (si, k)
                tol = 1e-10 if it == o["iterations"] else 1e-6
                assert rel(xg[k * n:(k + 1) * n], o["x"]) <= tol, (si, k)
    finally:
        for h in hs:
            h.close()


# ---------------------------------------------------------------- serving
def test_served_trace_against_oracle(A):
    """A short request stream served with continuous batching (FP32 V-cycle in
    FP64 flexible CG): each result against the oracle's FCG with its FP32
    cycle on the same system (iterations within two, x within 1e-6)."""
    from paper_1209_0960_amd import serve as S
    trace = P.serving_trace(rate=400.0, seconds=0.04, seed=17, edges=(8, 20), reuse=0.4)
    reqs, _ = S.requests_from_trace(trace)
    srv = S.Server(cap_bytes=4e9, max_entries=4, setup_workers=2, keep_solutions=True, vcycle_fp32=1)
    try:
        recs = srv.run(reqs)
    finally:
        srv.close()
    by_id = {r.id: r for r in reqs}
    assert len(recs) == len(reqs) >= 5
    for R in recs:
        r = by_id[R.id]
        assert R.status == A.OK
        ho = O.Hierarchy(r.rowptr.cpu().numpy(), r.colind.cpu().numpy(), r.vals.cpu().numpy(), vcycle_fp32=1)
        o = ho.pcg(r.b.cpu().numpy(), rtol=1e-8)
        assert o["status"] == O.OK
        assert abs(R.iterations - o["iterations"]) <= 2, R.id
        assert rel(srv.solutions[R.id].cpu().numpy(), o["x"]) <= 1e-6, R.id


# ---------------------------------------------------------------- out of memory
class CountingHook:
    """Allocator hook over torch's caching allocator that returns NULL once the
    bytes handed out in total would exceed `limit`; it records every live
    block so that leaks show."""

    def __init__(self, A):
        self.limit = float("inf")
        self.total = 0
        self.live = {}
        self.refused = 0

        def alloc(size, stream, ctx):
            if self.total + size > self.limit:
                self.refused += 1
                return None
            p = torch.cuda.caching_allocator_alloc(size, 0, stream or 0)
            self.total += size
            self.live[p] = size
            return p

        def free(ptr, stream, ctx):
            if ptr in self.live:
                del self.live[ptr]
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = A.ALLOC_FN(alloc)
        self.free_fn = A.FREE_FN(free)


def test_out_of_memory_from_allocator_hook(A):
    s = P.lognormal(20, seed=2)
    rp, ci, v, b = tdev(s.rowptr, s.colind, s.vals, s.b)
    with A.Hierarchy(rp, ci, v) as h:
        xref, rref = h.solve(b)
    torch.cuda.synchronize()
    hook = CountingHook(A)
    A.set_allocator(hook.alloc_fn, hook.free_fn)
    try:
        base = torch.cuda.memory_allocated()
        with A.Hierarchy(rp, ci, v) as h:
            need = hook.total
            assert h.levels >= 2
        assert not hook.live
        for frac in (0.0, 0.05, 0.2, 0.5, 0.8, 0.97):
            hook.total, hook.limit, hook.refused = 0, int(frac * need), 0
            out = C.c_void_p(12345)
            p = A.default_params()
            csr = A.CSR(s.n, s.nnz, C.c_void_p(rp.data_ptr()), C.c_void_p(ci.data_ptr()), C.c_void_p(v.data_ptr()))
            st = A.lib().amg_setup(C.byref(csr), C.byref(p), None, C.byref(out))
            torch.cuda.synchronize()
            assert st == A.ERR_OUT_OF_MEMORY, (frac, st)
            assert out.value is None, frac
            assert hook.refused >= 1 and not hook.live, (frac, len(hook.live))
            assert torch.cuda.memory_allocated() == base, frac
        # the solve context: setup fits, the first solve's vectors do not
        hook.total, hook.limit = 0, float("inf")
        h = A.Hierarchy(rp, ci, v)
        try:
            hook.limit = hook.total
            x = torch.zeros_like(b)
            r = A.pcg_solve(h.h, b, x, raise_on_error=False)
            assert r.status == A.ERR_OUT_OF_MEMORY
            hook.limit = float("inf")
            x, r = h.solve(b)
            assert r.status == A.OK and r.iterations == rref.iterations
            assert torch.equal(x, xref)
            del x
        finally:
            h.close()
        torch.cuda.synchronize()
        assert not hook.live
        assert torch.cuda.memory_allocated() == base
    finally:
        A.set_allocator(None, None)


# ---------------------------------------------------------------- coarsening stop
def chain_pairs(m, s):
    """A chain of 2m + s rows with weak positive couplings +0.01 between
    neighbours, except inside the first m pairs (2i, 2i+1), which are coupled
    by -1 (diagonal 2.5).  The other s rows (diagonal 3) are isolated
    (positive couplings are never strong).  Each pair becomes one aggregate,
    each isolated row a singleton (no adjacent aggregate is shared by two
    isolated rows): m + s aggregates.  On the next level every row is
    isolated.  Diagonally dominant, hence SPD; no row is without couplings."""
    n = 2 * m + s
    rows, cols, vals = [], [], []
    for i in range(n):
        rows.append(i)
        cols.append(i)
        vals.append(2.5 if i < 2 * m else 3.0)
    for i in range(n - 1):
        c = -1.0 if (i < 2 * m and i % 2 == 0) else 0.01
        rows += [i, i + 1]
        cols += [i + 1, i]
        vals += [c, c]
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    M.sort_indices()
    return M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64), M


@pytest.mark.parametrize("m,s,levels", [(100, 800, 2), (99, 802, 1), (300, 400, 2)])
def test_stall_guard_like_oracle(A, m, s, levels):
    """900 of 1000 aggregates keeps the level (0.9 n is not exceeded), 901
    does not; the hierarchy, the coarsest factor's solve and CG agree with the
    oracle."""
    rp, ci, v, M = chain_pairs(m, s)
    ho = O.Hierarchy(rp, ci, v)
    assert ho.levels == levels
    trp, tci, tv = tdev(rp, ci, v)
    b = np.random.default_rng(m).uniform(-1, 1, rp.shape[0] - 1)
    with A.Hierarchy(trp, tci, tv) as hg:
        compare_levels(hg, ho, (m, s))
        x, r = hg.solve(torch.from_numpy(b).cuda())
        o = ho.pcg(b)
        assert r.status == A.OK and o["status"] == O.OK and abs(r.iterations - o["iterations"]) <= 1
        assert rel(x.cpu().numpy(), spla.spsolve(M.tocsc(), b)) <= 1e-7


def test_coarsening_stalled_status(A):
    """4097 isolated rows: nothing coarsens and the coarsest level would have
    more than 4096 rows -> AMG_ERR_COARSENING_STALLED on both sides; 4096
    rows are factorised and solved directly."""
    rp, ci, v, _ = chain_pairs(0, 4097)
    with pytest.raises(O.OracleError) as e:
        O.Hierarchy(rp, ci, v)
    assert e.value.status == O.STALLED
    with pytest.raises(A.AMGError) as e:
        A.Hierarchy(*tdev(rp, ci, v))
    assert e.value.status == A.ERR_COARSENING_STALLED
    rp, ci, v, M = chain_pairs(0, 4096)
    b = np.random.default_rng(1).uniform(-1, 1, 4096)
    with A.Hierarchy(*tdev(rp, ci, v)) as hg:
        assert hg.levels == 1
        x, r = hg.solve(torch.from_numpy(b).cuda())
        assert r.iterations == 1
        assert rel(x.cpu().numpy(), spla.spsolve(M.tocsc(), b)) <= 1e-12


# ---------------------------------------------------------------- breakdown
BREAKDOWN = [  # (c, pre, post, b): the oracle pins give the iteration (numpy PCG with the dense cycle)
    (5.0, 1, 1, [1.0, 0.0, -1.0, 0.0]),
    (5.0, 1, 1, [0.0872, 0.8701, 0.6317, -0.9945]),
    (5.5, 1, 0, [-1.0, 0.9, -0.4, -0.4]),
    (5.5, 1, 0, [-0.2, 0.3, -0.3, -0.6]),
    (5.5, 1, 0, [0.0, 0.4, 0.2, -0.9]),
]


@pytest.mark.parametrize("c,pre,post,b", BREAKDOWN)
def test_breakdown_status_like_oracle(A, c, pre, post, b):
    """Symmetric, positive diagonal, indefinite; SPD Galerkin matrix: CG stops
    with AMG_ERR_BREAKDOWN at the oracle's iteration, x the oracle's."""
    M = np.diag([4.0] * 4)
    M[0, 1] = M[1, 0] = M[2, 3] = M[3, 2] = -1.0
    M[0, 2] = M[2, 0] = c
    S = sp.csr_matrix(M)
    S.sort_indices()
    rp, ci, v = S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64)
    kw = dict(coarse_max=2, tile_rows=64, flexible=0, pre_sweeps=pre, post_sweeps=post)
    ho = O.Hierarchy(rp, ci, v, **kw)
    o = ho.pcg(np.array(b), maxit=50)
    assert o["status"] == O.BREAKDOWN
    with A.Hierarchy(*tdev(rp, ci, v), **kw) as hg:
        compare_levels(hg, ho, c)
        x = torch.zeros(4, dtype=torch.float64, device="cuda")
        r = A.pcg_solve(hg.h, torch.tensor(b, dtype=torch.float64, device="cuda"), x, maxit=50,
                        raise_on_error=False)
        assert r.status == A.ERR_BREAKDOWN
        assert r.iterations == o["iterations"]
        assert rel(x.cpu().numpy(), o["x"]) <= 1e-12 or np.abs(o["x"]).max() == 0.0 == np.abs(x.cpu().numpy()).max()


# ---------------------------------------------------------------- free vs apply
def test_free_waits_for_queued_precond_apply(A):
    """amg_precond_apply is asynchronous on the caller's stream.  Freeing the
    hierarchy while the application still waits behind other work on that
    stream, then building and using another hierarchy (which takes the freed
    blocks), must leave the queued application's output intact."""
    s = P.lognormal(24, seed=3)
    rp, ci, v, b = tdev(s.rowptr, s.colind, s.vals, s.b)
    with A.Hierarchy(rp, ci, v) as h:
        zref = h.precond(b)
    torch.cuda.synchronize()
    s2 = P.lognormal(24, seed=4)
    rp2, ci2, v2, b2 = tdev(s2.rowptr, s2.colind, s2.vals, s2.b)
    busy = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    h = A.Hierarchy(rp, ci, v)
    with torch.cuda.stream(side):
        for _ in range(40):
            busy.mul_(1.0)  # keeps the application queued
        z = h.precond(b)
    h.close()
    with A.Hierarchy(rp2, ci2, v2) as h2:
        for _ in range(3):
            h2.precond(b2)
            h2.solve(b2)
    side.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(z, zref)


# ---------------------------------------------------------------- SpMV layout
def test_csr_outer_product_against_oracle_and_in_batches(A):
    """spmv_format 1: CG's level-0 product reads the CSR form with a group of
    lanes per row.  Every FP64 iterate within 1e-10 of the oracle; a batch
    mixing both layouts gives each entry its solve alone bit for bit."""
    s = P.lognormal(24, seed=12)
    rp, ci, v, b = tdev(s.rowptr, s.colind, s.vals, s.b)
    maxit = 200
    ho = O.Hierarchy(s.rowptr, s.colind, s.vals)
    o = ho.pcg(s.b, rtol=1e-8, maxit=maxit, keep_iterates=True)
    with A.Hierarchy(rp, ci, v, spmv_format=1) as hc, A.Hierarchy(rp, ci, v) as hs:
        hist = torch.zeros((maxit + 1) * s.n, dtype=torch.float64, device="cuda")
        x, r = hc.solve(b, rtol=1e-8, maxit=maxit, iter_hist=hist)
        assert r.status == A.OK and abs(r.iterations - o["iterations"]) <= 1
        H = hist.cpu().numpy().reshape(maxit + 1, s.n)
        for it in range(1, min(r.iterations, o["iterations"]) + 1):
            assert rel(H[it], o["iterates"][it]) <= 1e-10, it
        xs_alone, rs_alone = hs.solve(b, rtol=1e-8, maxit=maxit)
        bs = [b.clone(), b.clone()]
        xs = [torch.zeros_like(b), torch.zeros_like(b)]
        st, infos = A.pcg_solve_batched([hc.h, hs.h], bs, xs, nrhs=1, rtol=1e-8, maxit=maxit)
        assert st == A.OK
        assert torch.equal(xs[0], x) and infos[0][0]["iterations"] == r.iterations
        assert torch.equal(xs[1], xs_alone) and infos[1][0]["iterations"] == rs_alone.iterations


def test_release_cached_memory(A):
    """The cached free blocks go back to the device; later setups allocate
    anew and give the same results."""
    s = P.lognormal(32, seed=13)
    rp, ci, v, b = tdev(s.rowptr, s.colind, s.vals, s.b)
    with A.Hierarchy(rp, ci, v) as h:
        x1, r1 = h.solve(b)
    free0 = torch.cuda.mem_get_info()[0]
    A.release_cached_memory()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 > free0  # the hierarchy's and solve context's blocks were returned
    with A.Hierarchy(rp, ci, v) as h:
        x2, r2 = h.solve(b)
    assert torch.equal(x1, x2) and r1.iterations == r2.iterations
