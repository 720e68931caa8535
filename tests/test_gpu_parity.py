"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Integer setup outputs (strong flags, isolated flags, aggregates, colours,
coarse sparsity) and the Galerkin values (ordered sums) must be bit-exact on
every level; the V-cycle output and every PCG iterate in FP64 must agree to
1e-10 relative with iteration counts within one; the FP32 V-cycle inside FP64
flexible CG must reach the FP64 true residual 1e-8.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1209_0960_amd import problems as P

pytestmark = pytest.mark.gpu

CASES = {
    "k1_20": lambda: P.poisson(20),                       # 8000 rows: 15 full tiles + a 320-row tail
    "hetero_24": lambda: P.lognormal(24),                 # sigma^2 = 4 lognormal, 27 tiles
    "jump_20": lambda: P.jump_cube(20),                   # coefficient jumps 1e3 / 1e-2
    "layered_16": lambda: P.layered(16),                  # contrast ~1e6
    "box_13x17x11": lambda: P.poisson(0, shape=(13, 17, 11)),  # non-cubic, ragged Morton order
    "hetero_32_s0": lambda: P.lognormal(32, seed=0),
}


@pytest.fixture(scope="module")
def A():
    from paper_1209_0960_amd import amg
    amg.lib()
    return amg


def dev(sys):
    from paper_1209_0960_amd import amg
    return amg.to_device(sys)


_SYS = {}


def system(name):
    if name not in _SYS:
        _SYS[name] = CASES[name]()
    return _SYS[name]


def compare_levels(hg, ho, name):
    assert hg.levels == ho.levels, (name, hg.levels, ho.levels)
    for l in range(ho.levels):
        g = hg.level(l)
        o = ho.level(l)
        assert g["n"] == o.n and g["nnz"] == o.nnz, (name, l)
        assert np.array_equal(g["rowptr"], o.rowptr), (name, l, "rowptr")
        assert np.array_equal(g["colind"], o.colind), (name, l, "colind")
        assert np.array_equal(g["vals"].view(np.int64), o.vals.view(np.int64)), (name, l, "vals not bit-exact")
        assert g["ncolours"] == o.ncol and np.array_equal(g["colour"], o.colour), (name, l, "colour")
        if l < ho.levels - 1:
            assert np.array_equal(g["strong"], o.strong), (name, l, "strong")
            assert np.array_equal(g["iso"], o.iso), (name, l, "iso")
            assert np.array_equal(g["agg"], o.agg), (name, l, "agg")


@pytest.mark.parametrize("name", list(CASES))
def test_setup_bit_exact(A, name):
    s = system(name)
    rp, ci, v, b = dev(s)
    with A.Hierarchy(rp, ci, v, keep_setup_data=1) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals)
        compare_levels(hg, ho, name)


@pytest.mark.parametrize("params", [dict(tile_rows=64), dict(tile_rows=1000, agg_min=4, agg_max=6, agg_diameter=2),
                                    dict(strength_threshold=0.25, colour_seed=7), dict(smoother=2),
                                    dict(smoother=2, tile_rows=200)])
def test_setup_bit_exact_other_parameters(A, params):
    s = system("hetero_24")
    rp, ci, v, b = dev(s)
    with A.Hierarchy(rp, ci, v, keep_setup_data=1, **params) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, **params)
        compare_levels(hg, ho, str(params))


def rel(a, b):
    """Larger of the norm-wise relative difference ||a - b|| / ||b|| and the
    element-wise one max|a - b| / max|b|: a bound on it bounds both, so an
    error confined to a few rows cannot hide in the norm."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = a - b
    nrm = np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300)
    ele = np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)
    return float(max(nrm, ele))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("smoother", [0, 1, 2])
def test_vcycle_fp64_parity(A, name, smoother):
    s = system(name)
    rp, ci, v, b = dev(s)
    with A.Hierarchy(rp, ci, v, smoother=smoother) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, smoother=smoother)
        z = hg.precond(b)
        torch.cuda.synchronize()
        assert rel(z.cpu().numpy(), ho.vcycle(s.b)) <= 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_pcg_fp64_iterates(A, name):
    s = system(name)
    rp, ci, v, b = dev(s)
    maxit = 200
    with A.Hierarchy(rp, ci, v) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals)
        hist = torch.zeros((maxit + 1) * s.n, dtype=torch.float64, device="cuda")
        x, r = hg.solve(b, rtol=1e-8, maxit=maxit, iter_hist=hist)
        o = ho.pcg(s.b, rtol=1e-8, maxit=maxit, keep_iterates=True)
        assert r.status == A.OK and o["status"] == O.OK
        assert abs(r.iterations - o["iterations"]) <= 1
        k = min(r.iterations, o["iterations"])
        H = hist.cpu().numpy().reshape(maxit + 1, s.n)
        for it in range(1, k + 1):
            assert rel(H[it], o["iterates"][it]) <= 1e-10, (name, it)
        assert np.allclose(r.res_hist[:k + 1], o["res_hist"][:k + 1], rtol=1e-8, atol=0)
        assert r.true_rel_residual <= 1.01e-8


@pytest.mark.parametrize("name", ["k1_20", "hetero_24", "layered_16"])
def test_fcg_fp32_vcycle(A, name):
    s = system(name)
    rp, ci, v, b = dev(s)
    with A.Hierarchy(rp, ci, v, vcycle_fp32=1) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, vcycle_fp32=1)
        z = hg.precond(b)
        torch.cuda.synchronize()
        assert rel(z.cpu().numpy(), ho.vcycle(s.b)) <= 1e-5
        x, r = hg.solve(b, rtol=1e-8)
        o = ho.pcg(s.b, rtol=1e-8)
        assert r.status == A.OK
        assert abs(r.iterations - o["iterations"]) <= 2
        assert r.true_rel_residual <= 1.5e-8
        # FP64 solution error against the plain FP64 method solved to 1e-12
        with A.Hierarchy(rp, ci, v) as h64:
            xr, _ = h64.solve(b, rtol=1e-12)
        err = rel(x.cpu().numpy(), xr.cpu().numpy())
        assert err <= 1e-6


def test_single_level_is_direct_solve(A):
    s = P.lognormal(6, seed=4)
    rp, ci, v, b = dev(s)
    with A.Hierarchy(rp, ci, v) as hg:
        assert hg.levels == 1
        x, r = hg.solve(b)
        assert r.iterations == 1 and r.true_rel_residual <= 1e-12


@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 3, 3), (4, 4, 4), (13, 5, 1), (13, 10, 1), (10, 10, 5), (10, 10, 10),
                                   (16, 16, 16)])
def test_dense_coarse_inverse(A, shape):
    """One-level hierarchies (coarse_max >= n): the preconditioner is the
    dense inverse (blocked Cholesky of 64 x 64 blocks, then the inverse of the
    factor), so z = A^-1 b for sizes at, below and across the block edges."""
    nx, ny, nz = shape
    K = np.exp(0.5 * np.random.default_rng(3).standard_normal((nz, ny, nx)))  # mild contrast: well conditioned
    s = P.from_field(K, seed=3)
    rp, ci, v, b = dev(s)
    with A.Hierarchy(rp, ci, v, coarse_max=s.n) as hg:
        assert hg.levels == 1
        z = hg.precond(b)
        torch.cuda.synchronize()
        Ad = np.zeros((s.n, s.n))
        for i in range(s.n):
            Ad[i, s.colind[s.rowptr[i]:s.rowptr[i + 1]]] = s.vals[s.rowptr[i]:s.rowptr[i + 1]]
        ref = np.linalg.solve(Ad, s.b)
        assert rel(z.cpu().numpy(), ref) <= 1e-12, shape


def test_setup_deterministic(A):
    s = system("hetero_32_s0")
    rp, ci, v, b = dev(s)
    levs = []
    for _ in range(3):
        with A.Hierarchy(rp, ci, v, keep_setup_data=1) as hg:
            levs.append([hg.level(l) for l in range(hg.levels)])
    for run in levs[1:]:
        for a, c in zip(levs[0], run):
            for k in ("agg", "colour", "rowptr", "colind", "vals", "strong", "iso"):
                if a[k] is not None:
                    assert np.array_equal(a[k], c[k]), k


def test_error_paths(A):
    s = P.poisson(6)
    rp, ci, v, b = dev(s)

    def status(rp_, ci_, v_, **kw):
        try:
            h = A.Hierarchy(rp_, ci_, v_, **kw)
            h.close()
            return A.OK
        except A.AMGError as e:
            return e.status

    ci2 = ci.clone()
    ci2[1], ci2[2] = ci[2].item(), ci[1].item()
    assert status(rp, ci2, v) == A.ERR_INVALID_ARG
    v2 = v.clone()
    v2[0] = -1.0
    assert status(rp, ci, v2) == A.ERR_BAD_DIAGONAL
    v3 = v.clone()
    v3[1] = -0.5
    assert status(rp, ci, v3) == A.ERR_NOT_SYMMETRIC
    assert status(rp, ci, v3, check_symmetry=0) == A.OK
    v4 = v.clone()
    v4[3] = float("nan")
    assert status(rp, ci, v4) == A.ERR_INVALID_ARG
    ci5 = ci.clone()
    ci5[-1] = s.n + 5
    assert status(rp, ci5, v) == A.ERR_INVALID_ARG
    assert status(rp, ci, v, agg_max=40) == A.ERR_UNSUPPORTED
    # indefinite matrix: the coarsest Cholesky fails (oracle reports the same)
    vv = s.vals.copy()
    rows = np.repeat(np.arange(s.n), np.diff(s.rowptr))
    vv[(rows == 0) & (s.colind != 0)] *= 50
    vv[(s.colind == 0) & (rows != 0)] *= 50
    assert status(rp, ci, torch.from_numpy(vv).cuda()) == A.ERR_NOT_SPD
    with pytest.raises(O.OracleError):
        O.Hierarchy(s.rowptr, s.colind, vv)


def spoke_matrix(tiles=2100, T=64):
    """SPD chain (tridiagonal 4, -1) with row 0 also coupled to the first row
    of each of `tiles` - 1 other T-row tiles: row 0's tile has more
    neighbour tiles than the multicolour colouring's tile graph holds."""
    n = tiles * T
    spokes = np.arange(T, n, T)
    rows = [np.arange(n), np.arange(1, n), np.arange(n - 1), np.zeros(len(spokes), int), spokes]
    cols = [np.arange(n), np.arange(n - 1), np.arange(1, n), spokes, np.zeros(len(spokes), int)]
    vals = [np.full(n, 4.0), np.full(n - 1, -1.0), np.full(n - 1, -1.0), np.full(len(spokes), -0.5),
            np.full(len(spokes), -0.5)]
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    v[(r == 0) & (c == 0)] += 0.5 * len(spokes)  # diagonally dominant rows: SPD
    v[(r == c) & (r % T == 0) & (r > 0)] = 4.5
    o = np.lexsort((c, r))
    r, c, v = r[o], c[o], v[o]
    d = np.r_[0, np.cumsum(np.bincount(r, minlength=n))].astype(np.int32)
    return d, c.astype(np.int32), v, n


def test_failure_in_the_colouring_thread(A):
    """Level 0's multicolour colouring fails (row 0's tile has more than 2048
    neighbour tiles) while the coarsening goes on beside it: the setup
    reports UNSUPPORTED, in a single setup (colouring on its own host thread)
    and in a batch (colouring inline); the hybrid smoother, which needs no
    such colouring, sets up the same matrix; a later setup works."""
    d, c, v, n = spoke_matrix()
    rp, ci, vv = (torch.from_numpy(d).cuda(), torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())
    with pytest.raises(A.AMGError) as e:
        A.Hierarchy(rp, ci, vv, colour_tile_rows=64)
    assert e.value.status == A.ERR_UNSUPPORTED and "neighbour tiles" in str(e.value)
    with pytest.raises(A.AMGError) as e:
        A.Hierarchy.batched([(rp, ci, vv), (rp, ci, vv)], colour_tile_rows=64)
    assert e.value.status == A.ERR_UNSUPPORTED
    with A.Hierarchy(rp, ci, vv, colour_tile_rows=64, smoother=2) as h:
        assert h.levels >= 2
    s = P.poisson(12)
    rp2, ci2, v2, b2 = dev(s)
    with A.Hierarchy(rp2, ci2, v2) as h:
        x, r = h.solve(b2, rtol=1e-8)
        assert r.status == A.OK


def test_not_converged_keeps_last_iterate(A):
    s = system("hetero_24")
    rp, ci, v, b = dev(s)
    with A.Hierarchy(rp, ci, v) as hg:
        x, r = hg.solve(b, rtol=1e-14, maxit=3)
        assert r.status == A.ERR_NOT_CONVERGED and r.iterations == 3
        o = O.Hierarchy(s.rowptr, s.colind, s.vals).pcg(s.b, rtol=1e-14, maxit=3)
        assert o["status"] == O.NOT_CONVERGED
        assert rel(x.cpu().numpy(), o["x"]) <= 1e-10


@pytest.mark.parametrize("fp32", [0, 1])
def test_graph_replays_match_eager(A, fp32):
    """Each CG iteration replayed from a captured HIP graph gives bit-identical
    iterates to the eager launches, over repeated solves on one hierarchy with
    eager work in between."""
    s = system("hetero_24")
    rp, ci, v, b = dev(s)
    maxit = 100
    runs = []
    for graphs in (0, 1):
        with A.Hierarchy(rp, ci, v, use_graphs=graphs, vcycle_fp32=fp32) as h:
            hists = []
            for rep in range(3):
                hist = torch.zeros((maxit + 1) * s.n, dtype=torch.float64, device="cuda")
                x, r = h.solve(b, maxit=maxit, iter_hist=hist)
                assert r.status == A.OK
                z = h.precond(b)  # eager work between replays
                torch.cuda.synchronize()
                hists.append((hist.cpu().numpy()[:(r.iterations + 1) * s.n], x.cpu().numpy(), z.cpu().numpy()))
            runs.append(hists)
    ref = runs[0][0]
    for hists in runs:
        for h in hists:
            for a, c in zip(h, ref):
                assert np.array_equal(a, c)


@pytest.mark.parametrize("fp32", [0, 1])
def test_vcycle_hybrid_large_tiles(A, fp32):
    """Hybrid smoother with 1024-row tiles: a tile's couplings no longer fit
    the 64 KiB LDS staging (coarse levels, and level 0 in FP64), so those
    sweeps run with the iterate alone in LDS; FP32 level 0 still stages
    everything.  Both paths against the oracle."""
    s = system("hetero_24")
    rp, ci, v, b = dev(s)
    with A.Hierarchy(rp, ci, v, smoother=2, tile_rows=1024, vcycle_fp32=fp32) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, smoother=2, tile_rows=1024, vcycle_fp32=fp32)
        z = hg.precond(b)
        torch.cuda.synchronize()
        assert rel(z.cpu().numpy(), ho.vcycle(s.b)) <= (1e-5 if fp32 else 1e-12)


@pytest.mark.parametrize("fp32", [0, 1])
def test_user_stream_ordering_is_exact(A, fp32):
    """Calls run after the caller's earlier work on its stream and leave their
    results ready on it: a right-hand side still being produced on a busy side
    stream is waited for, and the solution is consumed there at once.
    Doubling b is exact in floating point, so x(2b) = 2 x(b) bit for bit (CG,
    BiCGSTAB, the preconditioner)."""
    s = system("hetero_24")
    rp, ci, v, b = dev(s)
    busy = torch.ones(1 << 24, device="cuda", dtype=torch.float64)
    side = torch.cuda.Stream()
    with A.Hierarchy(rp, ci, v, vcycle_fp32=fp32) as h:
        refs = {m: h.solve(b, method=m)[0] for m in ("cg", "bicgstab")}
        zref = h.precond(b)
        torch.cuda.synchronize()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for m in ("cg", "bicgstab"):
                for _ in range(20):
                    busy.mul_(1.0)  # work ahead of the right-hand side on this stream
                x2, _ = h.solve(b * 2.0, method=m)
                assert torch.equal(x2 * 0.5, refs[m]), m
            for _ in range(20):
                busy.mul_(1.0)
            z2 = h.precond(b * 2.0) * 0.5
        side.synchronize()
        assert torch.equal(z2, zref)
