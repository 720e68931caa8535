"""Batched and continuously batched solves against solves of each system alone.

Every entry of a batch runs the same kernels as pcg_solve with its own split
of rows into blocks, so its iterates are bit-identical to the solve alone:
checked for pcg_solve_batched with one and with four right-hand sides per
system, for the continuous-batching interface with entries joining and
leaving at different steps (including two entries of one hierarchy), and for
amg_setup_batched against amg_setup.  Alone-solves are pinned to the oracle
by the parity tests; here the check is exact equality.
"""
import numpy as np
import pytest
import torch

from paper_1209_0960_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    from paper_1209_0960_amd import amg
    amg.lib()
    return amg


def systems(nrhs=1, seed=11):
    """Uneven sizes: one-level (5^3 = 125 rows), small and multi-level systems."""
    rng = np.random.default_rng(seed)
    out = []
    for n in (5, 12, 20, 9, 24, 16):
        K = P.field_lognormal(rng, n, 2.0, 2, np.sqrt(8.0))
        rp, ci, v, order = P.ccfv7(K)
        B = rng.uniform(-1.0, 1.0, (nrhs, n ** 3))[:, order]
        out.append((rp, ci, v, np.ascontiguousarray(B)))
    return out


def dev(sysl):
    return [(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(v).cuda(),
             torch.from_numpy(B).cuda()) for rp, ci, v, B in sysl]


def alone(A, h, b):
    x = torch.zeros_like(b)
    x, r = h.solve(b, x, rtol=1e-8, maxit=200)
    return x, r


@pytest.mark.parametrize("fp32", [1, 0])
def test_batched_one_rhs_bit_identical(A, fp32):
    d = dev(systems(1))
    hs = [A.Hierarchy(rp, ci, v, vcycle_fp32=fp32) for rp, ci, v, _ in d]
    bs = [B.reshape(-1).clone() for *_, B in d]
    xs = [torch.zeros_like(b) for b in bs]
    st, infos = A.pcg_solve_batched([h.h for h in hs], bs, xs, nrhs=1, rtol=1e-8, maxit=200)
    assert st == A.OK
    for k, (h, b, x) in enumerate(zip(hs, bs, xs)):
        xa, r = alone(A, h, b)
        assert infos[k][0]["iterations"] == r.iterations, k
        assert torch.equal(x, xa), k
        assert infos[k][0]["true_rel_residual"] == r.true_rel_residual
        assert infos[k][0]["levels"] == h.levels
    for h in hs:
        h.close()


@pytest.mark.parametrize("nrhs", [2, 4])
def test_batched_multi_rhs_matches_each_rhs_alone(A, nrhs):
    d = dev(systems(nrhs, seed=12))
    hs = [A.Hierarchy(rp, ci, v, vcycle_fp32=1) for rp, ci, v, _ in d]
    bs = [B.reshape(-1).clone() for *_, B in d]
    xs = [torch.zeros_like(b) for b in bs]
    st, infos = A.pcg_solve_batched([h.h for h in hs], bs, xs, nrhs=nrhs, rtol=1e-8, maxit=200)
    assert st == A.OK
    for s, (h, (*_, B)) in enumerate(zip(hs, d)):
        n = B.shape[1]
        for k in range(nrhs):
            xa, r = alone(A, h, B[k].contiguous())
            assert infos[s][k]["iterations"] == r.iterations, (s, k)
            assert torch.equal(xs[s][k * n:(k + 1) * n], xa), (s, k)
    for h in hs:
        h.close()


def test_continuous_batching_join_and_leave(A):
    """Entries join at different steps, one hierarchy serves two entries at
    once, finished entries leave and their slots are reused."""
    d = dev(systems(1, seed=13))
    hs = [A.Hierarchy(rp, ci, v, vcycle_fp32=1) for rp, ci, v, _ in d]
    reqs = [(0, 0), (1, 0), (2, 3), (0, 5), (3, 5), (4, 9), (5, 12), (2, 20)]  # (system, join step)
    rng = np.random.default_rng(5)
    rhs = []
    for sidx, _ in reqs:
        n = hs[sidx].n
        rhs.append(torch.from_numpy(rng.uniform(-1, 1, n)).cuda())
    outs = [torch.zeros_like(b) for b in rhs]
    done = {}
    with A.Batch(nrhs=1, max_entries=4) as bt:
        pend = list(enumerate(reqs))
        step = 0
        while pend or bt.active:
            while pend and pend[0][1][1] <= step and bt.active < 4:
                i, (sidx, _) = pend.pop(0)
                bt.submit(hs[sidx], rhs[i], outs[i], rtol=1e-8, maxit=200, tag=i)
            bt.step(1)
            for tag, st, info in bt.poll():
                done[tag] = (st, info[0])
            step += 1
            assert step < 2000
    assert sorted(done) == list(range(len(reqs)))
    for i, (sidx, _) in enumerate(reqs):
        xa, r = alone(A, hs[sidx], rhs[i])
        st, info = done[i]
        assert st == A.OK
        assert info["iterations"] == r.iterations, i
        assert torch.equal(outs[i], xa), i
    for h in hs:
        h.close()


def test_setup_batched_equals_setup(A):
    d = dev(systems(1, seed=14))
    hb = A.Hierarchy.batched([(rp, ci, v) for rp, ci, v, _ in d], vcycle_fp32=0)
    for (rp, ci, v, _), h in zip(d, hb):
        with A.Hierarchy(rp, ci, v, vcycle_fp32=0) as ha:
            assert ha.levels == h.levels
            for l in range(ha.levels):
                a, b = ha.level(l), h.level(l)
                for key in ("agg", "colour", "rowptr", "colind", "vals"):
                    if a[key] is None:
                        assert b[key] is None
                    else:
                        assert np.array_equal(a[key], b[key]), (l, key)
        h.close()


def test_batch_errors(A):
    d = dev(systems(1, seed=15))
    h32 = A.Hierarchy(*d[1][:3], vcycle_fp32=1)
    h64 = A.Hierarchy(*d[2][:3], vcycle_fp32=0)
    b1 = d[1][3].reshape(-1).clone()
    b2 = d[2][3].reshape(-1).clone()
    with pytest.raises(A.AMGError) as e:
        A.pcg_solve_batched([h32.h, h64.h], [b1, b2], [torch.zeros_like(b1), torch.zeros_like(b2)])
    assert e.value.status == A.ERR_INVALID_ARG
    with pytest.raises(A.AMGError) as e:
        A.pcg_solve_batched([h32.h], [b1.repeat(3)], [torch.zeros(3 * b1.numel(), dtype=torch.float64,
                                                                   device="cuda")], nrhs=3)
    assert e.value.status == A.ERR_UNSUPPORTED
    with A.Batch(nrhs=1, max_entries=1) as bt:
        x1 = torch.zeros_like(b1)
        bt.submit(h32, b1, x1)
        with pytest.raises(A.AMGError) as e:
            bt.submit(h32, b1, torch.zeros_like(b1))
        assert e.value.status == A.ERR_INVALID_ARG
        while bt.active:
            bt.step(1)
            bt.poll()
    h32.close()
    h64.close()


def test_precond_after_solve_matches_fresh(A):
    """amg_precond_apply shares the solve context with pcg_solve: the product
    is the same before and after a solve."""
    d = dev(systems(1, seed=16))
    rp, ci, v, B = d[4]
    with A.Hierarchy(rp, ci, v, vcycle_fp32=1) as h:
        r = B.reshape(-1).clone()
        z1 = h.precond(r)
        torch.cuda.synchronize()
        h.solve(r)
        z2 = h.precond(r)
        torch.cuda.synchronize()
        assert torch.equal(z1, z2)


@pytest.mark.parametrize("fp32,pre,post,smoother", [(1, 1, 1, 0), (0, 1, 1, 0), (1, 2, 2, 0), (1, 0, 1, 0),
                                                    (1, 1, 0, 0), (1, 1, 1, 1), (1, 1, 1, 2), (0, 1, 1, 2),
                                                    (1, 2, 2, 2), (1, 0, 1, 2), (0, 1, 1, 3), (1, 1, 1, (0, 3, 1)),
                                                    (0, 2, 2, (0, 3, 2)), (0, 1, 1, (2, 0, 1))])
def test_tail_bit_identical(A, fp32, pre, post, smoother):
    """Levels cycled by one workgroup per entry (tail_rows: below that many
    rows; the coarsest solve stays a many-block launch) give the same bits as
    one launch per step: single solves, preconditioner applications, and
    batches with four right-hand sides per system.  The tail fills, forms the
    residual and prolongs every row, so this also checks the launch path's
    shortcuts (colour-0 rows skipped, residual from the last pre-smoothing
    pass) for several sweep counts and every smoother."""
    d = dev(systems(4, seed=5))
    ref = None
    kw = dict(vcycle_fp32=fp32, pre_sweeps=pre, post_sweeps=post, smoother=smoother)
    if isinstance(smoother, tuple):  # (smoother, coarse_smoother, coarse_from)
        kw.update(smoother=smoother[0], coarse_smoother=smoother[1], coarse_from=smoother[2])
    if pre + post == 0 or (fp32 == 0 and smoother == 1):
        pytest.skip("not a symmetric positive definite preconditioner")
    for tail in (0, 600, 1 << 30):
        hs = [A.Hierarchy(rp, ci, v, tail_rows=tail, **kw) for rp, ci, v, _ in d]
        try:
            out = []
            for h, (*_, B) in zip(hs, d):
                b = B[0].contiguous()
                x, r = alone(A, h, b)
                out.append((r.iterations, x.cpu().numpy(), h.precond(b).cpu().numpy()))
            bs = [B.reshape(-1).clone() for *_, B in d]
            xs = [torch.zeros_like(b) for b in bs]
            st, infos = A.pcg_solve_batched([h.h for h in hs], bs, xs, nrhs=4, rtol=1e-8, maxit=200)
            assert st == A.OK
            out.append(([i["iterations"] for inf in infos for i in inf], [x.cpu().numpy() for x in xs]))
        finally:
            for h in hs:
                h.close()
        if ref is None:
            ref = out
            continue
        for k, (a, c) in enumerate(zip(ref[:-1], out[:-1])):
            assert a[0] == c[0], (tail, k)
            assert np.array_equal(a[1], c[1]) and np.array_equal(a[2], c[2]), (tail, k)
        assert ref[-1][0] == out[-1][0], tail
        for a, c in zip(ref[-1][1], out[-1][1]):
            assert np.array_equal(a, c), tail
