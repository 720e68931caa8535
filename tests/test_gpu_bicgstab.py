"""GPU parity of BiCGSTAB (the paper's outer solver, Sec. 5) against the oracle.

The FP64 iterates x_k must agree with the oracle's to 1e-10 relative, the bar
of the CG iterates: each V-cycle application agrees to about 1e-13 (different
summation orders), two applications per iteration, and over the iterations
compared the recurrences amplify that by less than 1e3.  The residual ratios ||r_k||/||r_0|| agree to 1e-12
absolute.  Iteration counts agree within one; a half-step
exit agrees when the counts do.  The FP32 V-cycle must reach the FP64 true
residual bound; the one-level hierarchy (exact preconditioner) stops at the
first half step.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle as O
from paper_1209_0960_amd import problems as P

pytestmark = pytest.mark.gpu

CASES = {
    "k1_20": lambda: P.poisson(20),
    "hetero_24": lambda: P.lognormal(24),
    "jump_20": lambda: P.jump_cube(20),
    "layered_16": lambda: P.layered(16),
    "box_13x17x11": lambda: P.poisson(0, shape=(13, 17, 11)),
}
_SYS = {}


def system(name):
    if name not in _SYS:
        _SYS[name] = CASES[name]()
    return _SYS[name]


@pytest.fixture(scope="module")
def A():
    from paper_1209_0960_amd import amg
    amg.lib()
    return amg


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


def true_res(s, x):
    M = sp.csr_matrix((s.vals, s.colind, s.rowptr), shape=(s.n, s.n))
    return np.linalg.norm(s.b - M @ x) / np.linalg.norm(s.b)


@pytest.mark.parametrize("name", list(CASES))
def test_bicgstab_fp64_iterates(A, name):
    s = system(name)
    rp, ci, v, b = A.to_device(s)
    maxit = 100
    with A.Hierarchy(rp, ci, v) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals)
        hist = torch.zeros((maxit + 1) * s.n, dtype=torch.float64, device="cuda")
        x, r = hg.solve(b, rtol=1e-8, maxit=maxit, iter_hist=hist, method="bicgstab")
        o = ho.bicgstab(s.b, rtol=1e-8, maxit=maxit, keep_iterates=True)
        assert r.status == A.OK and o["status"] == O.OK, (r.status, o["status"])
        assert abs(r.iterations - o["iterations"]) <= 1
        if r.iterations == o["iterations"]:
            assert r.half_step == o["half"]
        k = min(r.iterations, o["iterations"])
        H = hist.cpu().numpy().reshape(maxit + 1, s.n)
        assert np.array_equal(H[0], np.zeros(s.n))
        worst = max(rel(H[it], o["iterates"][it]) for it in range(1, k + 1))
        print(f"{name}: {r.iterations} iterations (oracle {o['iterations']}), half {r.half_step}, "
              f"max iterate difference {worst:.2e}")
        assert worst <= 1e-10
        # residual ratios: rounding-level agreement in units of ||r_0|| (they
        # fall by cancellation, so their relative difference grows as they do)
        assert np.allclose(r.res_hist[:k + 1], o["res_hist"][:k + 1], rtol=1e-5, atol=1e-12)
        xs = x.cpu().numpy()
        assert true_res(s, xs) <= 1.01e-8
        assert abs(true_res(s, xs) - r.true_rel_residual) <= 1e-3 * r.true_rel_residual + 1e-14
        assert rel(xs, o["x"]) <= 1e-6


@pytest.mark.parametrize("name", ["k1_20", "hetero_24", "layered_16"])
def test_bicgstab_fp32_vcycle(A, name):
    s = system(name)
    rp, ci, v, b = A.to_device(s)
    with A.Hierarchy(rp, ci, v, vcycle_fp32=1) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, vcycle_fp32=1)
        x, r = hg.solve(b, rtol=1e-8, method="bicgstab")
        o = ho.bicgstab(s.b, rtol=1e-8)
        assert r.status == A.OK and o["status"] == O.OK
        assert abs(r.iterations - o["iterations"]) <= 2
        xs = x.cpu().numpy()
        assert true_res(s, xs) <= 1.5e-8
        assert rel(xs, o["x"]) <= 1e-6


def test_bicgstab_single_level_stops_at_half_step(A):
    s = P.lognormal(6, seed=4)
    rp, ci, v, b = A.to_device(s)
    with A.Hierarchy(rp, ci, v) as hg:
        assert hg.levels == 1
        x, r = hg.solve(b, rtol=1e-10, method="bicgstab")
        assert r.status == A.OK and r.iterations == 1 and r.half_step == 1
        assert r.true_rel_residual <= 1e-12


def test_bicgstab_trivial_and_error_cases(A):
    s = P.poisson(12)
    rp, ci, v, b = A.to_device(s)
    with A.Hierarchy(rp, ci, v) as hg:
        z = torch.zeros_like(b)
        x, r = hg.solve(z, method="bicgstab")
        assert r.status == A.OK and r.iterations == 0 and not x.any().item()
        x0 = torch.full_like(b, 0.5)
        x, r = hg.solve(b, x=x0.clone(), maxit=0, method="bicgstab", raise_on_error=False)
        assert r.status == A.ERR_NOT_CONVERGED and r.iterations == 0
        assert torch.equal(x, x0)
        st = A.lib().bicgstab_solve(hg.h, A._ptr(b), A._ptr(x), 1e-8, -1, None, None, None, None, None)
        assert st == A.ERR_INVALID_ARG
        # a capped run keeps the last iterate, and the oracle's agrees with it
        x, r = hg.solve(b, maxit=2, method="bicgstab", raise_on_error=False)
        o = O.Hierarchy(s.rowptr, s.colind, s.vals).bicgstab(s.b, maxit=2)
        assert r.status == A.ERR_NOT_CONVERGED and o["status"] == O.NOT_CONVERGED and r.iterations == 2
        assert rel(x.cpu().numpy(), o["x"]) <= 1e-10


def test_bicgstab_interleaved_with_cg_is_deterministic(A):
    """The solvers share the hierarchy's solve context: results do not depend
    on what ran before (bit for bit)."""
    s = system("hetero_24")
    rp, ci, v, b = A.to_device(s)
    with A.Hierarchy(rp, ci, v) as hg:
        x1, r1 = hg.solve(b, method="bicgstab")
        xc, rc = hg.solve(b)
        z = hg.precond(b)
        x2, r2 = hg.solve(b, method="bicgstab")
        xc2, _ = hg.solve(b)
        torch.cuda.synchronize()
        assert torch.equal(x1, x2) and r1.iterations == r2.iterations
        assert torch.equal(xc, xc2)
        assert rc.status == A.OK and r1.status == A.OK


def test_bicgstab_fullsize_128_true_residual(A):
    """The 128^3 lognormal system (sigma^2 = 4) at its benchmark size, both
    V-cycle precisions: true FP64 residual from an independent CPU product."""
    s = P.lognormal(128, seed=1)
    rp, ci, v, b = A.to_device(s)
    for fp32 in (0, 1):
        with A.Hierarchy(rp, ci, v, vcycle_fp32=fp32) as hg:
            x, r = hg.solve(b, rtol=1e-8, method="bicgstab")
            assert r.status == A.OK
            res = true_res(s, x.cpu().numpy())
            print(f"128^3 fp32={fp32}: {r.iterations} iterations, half {r.half_step}, true residual {res:.3e}")
            assert res <= 1.5e-8
            assert abs(res - r.true_rel_residual) <= 1e-3 * res + 1e-14


@pytest.mark.parametrize("name", ["hetero_24", "jump_20", "box_13x17x11"])
@pytest.mark.parametrize("T", [128, 200])
def test_bicgstab_hybrid_sgs_fp64_iterates(A, name, T):
    """The paper's own configuration (Sec. 5): BiCGSTAB with one V-cycle of
    hybrid symmetric Gauss-Seidel smoothing (block-Jacobi over tiles of T
    rows, ragged when T = 200), iterates against the oracle's."""
    s = system(name)
    rp, ci, v, b = A.to_device(s)
    maxit = 100
    with A.Hierarchy(rp, ci, v, smoother=2, tile_rows=T) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, smoother=2, tile_rows=T)
        hist = torch.zeros((maxit + 1) * s.n, dtype=torch.float64, device="cuda")
        x, r = hg.solve(b, rtol=1e-8, maxit=maxit, iter_hist=hist, method="bicgstab")
        o = ho.bicgstab(s.b, rtol=1e-8, maxit=maxit, keep_iterates=True)
        assert r.status == A.OK and o["status"] == O.OK
        assert abs(r.iterations - o["iterations"]) <= 1
        k = min(r.iterations, o["iterations"])
        H = hist.cpu().numpy().reshape(maxit + 1, s.n)
        worst = max(rel(H[it], o["iterates"][it]) for it in range(1, k + 1))
        print(f"{name} T={T}: {r.iterations} iterations (oracle {o['iterations']}), max iterate difference "
              f"{worst:.2e}")
        assert worst <= 1e-10
        assert true_res(s, x.cpu().numpy()) <= 1.01e-8


@pytest.mark.parametrize("name", ["hetero_24", "k1_20"])
@pytest.mark.parametrize("kw", [dict(smoother=2, smooth_tile_rows=256, coarse_smooth_tile_rows=64),
                                dict(smoother=3), dict(coarse_smoother=3, coarse_from=1)],
                         ids=["hybrid_blocks256_64", "tile_mcsgs", "headline_smoothing"])
def test_bicgstab_smoothing_variants_fp64_iterates(A, name, kw):
    """BiCGSTAB with the hybrid smoother on blocks of their own size (256
    rows on level 0, 64 below), with the tile-ordered multicolour smoother on
    every level, and with the headline's smoothing: iterates against the
    oracle's."""
    s = system(name)
    rp, ci, v, b = A.to_device(s)
    maxit = 100
    with A.Hierarchy(rp, ci, v, **kw) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, **kw)
        hist = torch.zeros((maxit + 1) * s.n, dtype=torch.float64, device="cuda")
        x, r = hg.solve(b, rtol=1e-8, maxit=maxit, iter_hist=hist, method="bicgstab")
        o = ho.bicgstab(s.b, rtol=1e-8, maxit=maxit, keep_iterates=True)
        assert r.status == A.OK and o["status"] == O.OK
        assert abs(r.iterations - o["iterations"]) <= 1
        k = min(r.iterations, o["iterations"])
        H = hist.cpu().numpy().reshape(maxit + 1, s.n)
        worst = max(rel(H[it], o["iterates"][it]) for it in range(1, k + 1))
        assert worst <= 1e-10, (name, kw, worst)
        assert true_res(s, x.cpu().numpy()) <= 1.01e-8


def test_hybrid_sgs_fp32_vcycle_and_cg(A):
    s = system("hetero_24")
    rp, ci, v, b = A.to_device(s)
    with A.Hierarchy(rp, ci, v, smoother=2, vcycle_fp32=1) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, smoother=2, vcycle_fp32=1)
        z = hg.precond(b)
        torch.cuda.synchronize()
        assert rel(z.cpu().numpy(), ho.vcycle(s.b)) <= 1e-5
        for method, oracle_run in (("cg", ho.pcg), ("bicgstab", ho.bicgstab)):
            x, r = hg.solve(b, rtol=1e-8, method=method)
            o = oracle_run(s.b, rtol=1e-8)
            assert r.status == A.OK and abs(r.iterations - o["iterations"]) <= 2, method
            assert true_res(s, x.cpu().numpy()) <= 1.5e-8


@pytest.mark.parametrize("smoother", [0, 2])
def test_manufactured_poisson_solution_error(A, smoother):
    """The paper's manufactured Poisson problem (consistent pair, non-zero
    Dirichlet data) at 48^3 with BiCGSTAB: the AMG solution to rtol 1e-10 is
    the discrete solution (against a CPU direct solve of the same system at
    24^3, where that is cheap) and its error against exp(-|x|^2) is O(h^2):
    the 24^3 -> 48^3 ratio is about 4."""
    import scipy.sparse.linalg as sla

    errs = []
    for n in (24, 48):
        s, u = P.manufactured(n)
        rp, ci, v, b = A.to_device(s)
        with A.Hierarchy(rp, ci, v, smoother=smoother) as h:
            x, r = h.solve(b, rtol=1e-10, method="bicgstab")
        assert r.status == A.OK
        xs = x.cpu().numpy()
        if n == 24:
            M = sp.csr_matrix((s.vals, s.colind, s.rowptr), shape=(s.n, s.n))
            xd = sla.spsolve(M.tocsc(), s.b)
            assert rel(xs, xd) <= 1e-9
        errs.append(np.abs(xs - u).max())
    assert 3.6 < errs[0] / errs[1] < 4.4, errs


def test_jump_cube_80_paper_regime(A):
    """The paper's jump-coefficient problem at 80^3 (its Table 6 one-process
    size): BiCGSTAB with both smoothers reaches the true FP64 residual bound
    from an independent product."""
    s = P.jump_cube(80)
    rp, ci, v, b = A.to_device(s)
    for smoother in (0, 2):
        with A.Hierarchy(rp, ci, v, smoother=smoother) as h:
            x, r = h.solve(b, rtol=1e-8, method="bicgstab")
            print(f"jump 80^3 smoother={smoother}: {h.levels} levels, {r.iterations} iterations")
        assert r.status == A.OK
        assert true_res(s, x.cpu().numpy()) <= 1.01e-8
