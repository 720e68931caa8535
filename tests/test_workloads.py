"""Workload generators (host and device twins) and the request stream."""
import numpy as np
import pytest
import torch

from paper_1209_0960_amd import problems as P


@pytest.mark.parametrize("shape", [(5, 6, 7), (8, 8, 8), (3, 9, 4), (16, 16, 16)])
def test_ccfv7_torch_equals_host_assembly(shape):
    rng = np.random.default_rng(sum(shape))
    K = np.exp(2.0 * rng.standard_normal(shape))
    host = P.ccfv7(K)
    dev = P.ccfv7_torch(torch.from_numpy(K))
    for a, b in zip(host, dev):
        assert np.array_equal(a, b.numpy())


def test_lognormal_torch_shapes_and_symmetry():
    g = torch.Generator().manual_seed(3)
    rp, ci, v, b = P.lognormal_torch(12, 2.0, g, nrhs=2)
    n = 12 ** 3
    assert rp.numel() == n + 1 and ci.numel() == P.nnz_7pt(12, 12, 12) and b.shape == (2, n)
    import scipy.sparse as sp
    M = sp.csr_matrix((v.numpy(), ci.numpy(), rp.numpy()), shape=(n, n))
    assert abs(M - M.T).max() == 0.0
    assert np.all(M.diagonal() > 0) and float(b.abs().max()) <= 1.0


def test_serving_trace_recipe():
    tr = P.serving_trace(rate=200.0, seconds=2.0, seed=4)
    assert tr == P.serving_trace(rate=200.0, seconds=2.0, seed=4)
    t = np.array([r["t"] for r in tr])
    assert np.all(np.diff(t) > 0) and t[-1] < 2.0
    assert 300 < len(tr) < 500  # Poisson(400)
    assert all(32 <= r["edge"] <= 256 and 0.0 <= r["sigma2"] <= 4.0 for r in tr)
    reuse = [r for r in tr if r["matrix"] != r["id"]]
    assert 0.2 < len(reuse) / len(tr) < 0.4
    for r in reuse:
        j = tr[r["matrix"]]
        assert j["matrix"] == j["id"] and j["id"] < r["id"]
        assert (r["edge"], r["sigma2"]) == (j["edge"], j["sigma2"])
    assert len({r["seed"] for r in tr}) == len(tr)


def test_manufactured_poisson_converges_second_order():
    """The manufactured problem (consistent pair u = exp(-|x|^2),
    f = (6 - 4|x|^2) exp(-|x|^2), Dirichlet data u): the exact discrete solution
    approaches u at the cell centres as O(h^2), so halving h divides the
    largest error by about 4 (a wrong source sign, boundary weight or face
    centre breaks the ratio)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    errs = []
    for n in (8, 16):
        s, u = P.manufactured(n)
        A = sp.csr_matrix((s.vals, s.colind, s.rowptr), shape=(s.n, s.n))
        x = sla.spsolve(A.tocsc(), s.b)
        errs.append(np.abs(x - u).max())
    assert errs[1] < 1e-3
    assert 3.6 < errs[0] / errs[1] < 4.4
