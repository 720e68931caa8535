"""Point-based (block) AMG on the GPU against the oracle (Sec. 4.2): a
3-component coupled 7-point diffusion system in scalar form with whole 3x3
blocks.  Node-graph strength flags, aggregates, colours and the coarse
sparsity bit for bit, Galerkin values bit for bit (the same ordered sums of
the expanded prolongation), the block V-cycle within 1e-12, every FP64 PCG
iterate within 1e-10 with iterations within one, the FP32 cycle in flexible
CG to the FP64 bound, batched and fixed-scratch applications, input errors.
"""
import numpy as np
import pytest
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
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = a - b
    return float(max(np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300),
                     np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)))


def tdev(s):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (s.rowptr, s.colind, s.vals, s.b)]


CASES = {
    "coupled3_12": lambda: P.coupled(12, bs=3, seed=6),   # 5184 unknowns: tiles of 128 nodes, ragged tail
    "coupled3_16": lambda: P.coupled(16, bs=3, seed=7),
    "coupled2_14": lambda: P.coupled(14, bs=2, seed=8),   # slices of 64 rows hold 32 nodes
    "coupled4_10": lambda: P.coupled(10, bs=4, seed=9),
}
_S = {}


def system(name):
    if name not in _S:
        _S[name] = CASES[name]()
    return _S[name]


def bs_of(name):
    return int(name[7])


@pytest.mark.parametrize("name", list(CASES))
def test_block_setup_bit_exact(A, name):
    s = system(name)
    bs = bs_of(name)
    rp, ci, v, b = tdev(s)
    kw = dict(block_size=bs, coarse_max=60 * bs)
    with A.Hierarchy(rp, ci, v, keep_setup_data=1, **kw) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, **kw)
        assert hg.levels == ho.levels >= 2
        for l in range(ho.levels):
            g, o = hg.level(l), ho.level(l)
            assert np.array_equal(g["rowptr"], o.rowptr) and np.array_equal(g["colind"], o.colind), l
            assert np.array_equal(g["vals"].view(np.int64), o.vals.view(np.int64)), l
            assert g["ncolours"] == o.ncol and np.array_equal(g["colour"], o.colour), l
            if l < ho.levels - 1:
                assert np.array_equal(g["strong"], o.strong) and np.array_equal(g["iso"], o.iso), l
                assert np.array_equal(g["agg"], o.agg), l


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("fp32", [0, 1])
def test_block_vcycle_parity(A, name, fp32):
    s = system(name)
    bs = bs_of(name)
    rp, ci, v, b = tdev(s)
    kw = dict(block_size=bs, coarse_max=60 * bs, vcycle_fp32=fp32)
    with A.Hierarchy(rp, ci, v, **kw) as hg:
        ho = O.Hierarchy(s.rowptr, s.colind, s.vals, **kw)
        z = hg.precond(b)
        zn = torch.empty_like(b)
        A.amg_precond_apply_noalloc(hg.h, b, zn)
        torch.cuda.synchronize()
        assert rel(z.cpu().numpy(), ho.vcycle(s.b)) <= (1e-5 if fp32 else 1e-12)
        assert torch.equal(z, zn)


@pytest.mark.parametrize("name", list(CASES))
def test_block_pcg_fp64_iterates(A, name):
    s = system(name)
    bs = bs_of(name)
    rp, ci, v, b = tdev(s)
    kw = dict(block_size=bs, coarse_max=60 * bs)
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
        assert r.true_rel_residual <= 1.01e-8
        # the scalar treatment of the same system needs more iterations
        with A.Hierarchy(rp, ci, v, coarse_max=60 * bs) as hs:
            _, rs = hs.solve(b, rtol=1e-8, maxit=maxit)
        assert rs.iterations > r.iterations


def test_block_fcg_fp32_and_batched(A):
    s = system("coupled3_16")
    rp, ci, v, b = tdev(s)
    kw = dict(block_size=3, coarse_max=180)
    with A.Hierarchy(rp, ci, v, vcycle_fp32=1, **kw) as h32, A.Hierarchy(rp, ci, v, **kw) as h64:
        x32, r32 = h32.solve(b, rtol=1e-8)
        assert r32.status == A.OK and r32.true_rel_residual <= 1.5e-8
        xr, _ = h64.solve(b, rtol=1e-12)
        assert rel(x32.cpu().numpy(), xr.cpu().numpy()) <= 1e-6
        # batched: two right-hand sides of this system and one alone agree bit for bit
        B2 = torch.stack([b, b.flip(0).contiguous()]).reshape(-1).contiguous()
        X2 = torch.zeros_like(B2)
        st, infos = A.pcg_solve_batched([h64.h], [B2], [X2], nrhs=2, rtol=1e-8, maxit=200)
        assert st == A.OK
        xa, ra = h64.solve(b, rtol=1e-8)
        assert torch.equal(X2[:s.n], xa) and infos[0][0]["iterations"] == ra.iterations


def test_block_input_errors(A):
    s = system("coupled3_12")
    rp, ci, v, b = tdev(s)

    def status(**kw):
        try:
            A.Hierarchy(rp, ci, v, **kw).close()
            return A.OK
        except A.AMGError as e:
            return e.status

    assert status(block_size=4) == A.ERR_INVALID_ARG      # 5184 rows, but blocks of 3 are stored
    assert status(block_size=5) == A.ERR_UNSUPPORTED
    assert status(block_size=3, smoother=1) == A.ERR_UNSUPPORTED
    assert status(block_size=3, tail_rows=1000) == A.ERR_UNSUPPORTED
    assert status(block_size=3, coarse_smoother=3) == A.ERR_UNSUPPORTED
    # one entry of the first node's first row removed: no longer whole blocks
    rp2 = rp.clone()
    rp2[1:] -= 1
    keep = torch.ones(ci.numel(), dtype=torch.bool, device="cuda")
    keep[1] = False
    with pytest.raises(A.AMGError) as e:
        A.Hierarchy(rp2, ci[keep].contiguous(), v[keep].contiguous(), block_size=3, check_symmetry=0)
    assert e.value.status in (A.ERR_INVALID_ARG, A.ERR_NOT_SYMMETRIC)
