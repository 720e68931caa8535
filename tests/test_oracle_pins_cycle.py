"""Pins of the oracle's multilevel cycle, smoothers, coarsening stop and CG
breakdown against facts fixed by the paper and by linear algebra.

* The V-cycle of Sec. 2 is rebuilt densely in numpy with the paper's own
  scaling of the coarse operators, A_{l+1} = (1/omega) P_l^T A_l P_l (Sec. 2.1),
  no factor at prolongation, and textbook smoothers; the oracle stores P^T A P
  unscaled and damps the prolongated correction by omega on every level.  The
  two must give the same cycle on three and more levels.
* Without smoothing, three levels give the closed form
  omega^2 Q (Q^T A Q)^-1 Q^T with Q = P_0 P_1.
* One l1-Jacobi sweep on a 3x3 matrix with a positive off-diagonal is
  compared with a value derived by hand.
* The coarsening stop (a level that shrinks by less than 10 % ends the
  hierarchy; a coarsest level above 4096 rows is an error) on matrices whose
  aggregation is known by construction.
* A positive-diagonal, symmetric, indefinite matrix whose Galerkin coarse
  matrix is SPD drives CG into breakdown; a numpy CG with the dense cycle
  operator must break down at the same iteration.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_1209_0960_amd import problems as P


def dense(rp, ci, v):
    n = rp.shape[0] - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()


def prolongation(agg, nc):
    Pm = np.zeros((agg.shape[0], nc))
    Pm[np.arange(agg.shape[0]), agg] = 1.0
    return Pm


# ------------------------------------------------------------ dense paper cycle
def sgs_dense(A, order):
    """Textbook symmetric Gauss-Seidel in the given row order: a forward sweep
    x += (D + L)^-1 (b - A x) then a backward sweep x += (D + U)^-1 (b - A x),
    with L and U the strict triangles of A permuted to that order."""
    Ap = A[np.ix_(order, order)]
    Lo = np.tril(Ap)
    Up = np.triu(Ap)

    def apply(b, x):
        bp, xp = b[order], x[order]
        xp = xp + np.linalg.solve(Lo, bp - Ap @ xp)
        xp = xp + np.linalg.solve(Up, bp - Ap @ xp)
        out = np.empty_like(x)
        out[order] = xp
        return out
    return apply


def l1_jacobi_dense(A):
    """l1-Jacobi (Baker, Falgout, Kolev, Yang 2011): x += (b - A x) / d with
    d_i the sum of |a_ij| over the row."""
    d = np.abs(A).sum(axis=1)

    def apply(b, x):
        return x + (b - A @ x) / d
    return apply


def tile_order(n, T, colour=None):
    """Rows tile by tile (tiles of T consecutive rows, in order); inside a
    tile natural order, or (colour, row) order given colours."""
    if colour is None:
        return np.arange(n)
    return np.lexsort((np.arange(n), colour, np.arange(n) // T))


def hybrid_dense(A, T, colour=None):
    """Block-Jacobi over row tiles of T with one symmetric Gauss-Seidel step
    inside each block (Sec. 3.2), the rows of a tile swept in natural order
    or, with colours, in (colour, row) order: in that order,
    x += M^-1 (b - A x), M = (D + L_B) D^-1 (D + U_B), L_B / U_B the strict
    triangles of the tile-block-diagonal part of A."""
    n = A.shape[0]
    o = tile_order(n, T, colour)
    Ap = A[np.ix_(o, o)]
    tile = np.arange(n)[o] // T
    B = np.where(tile[:, None] == tile[None, :], Ap, 0.0)
    D = np.diag(np.diag(Ap))
    M = (D + np.tril(B, -1)) @ np.linalg.inv(D) @ (D + np.triu(B, 1))

    def apply(b, x):
        out = np.empty_like(x)
        out[o] = x[o] + np.linalg.solve(M, b[o] - Ap @ x[o])
        return out
    return apply


def paper_cycle(H, A0, omega, smoother, pre, post, tile_rows):
    """Dense V-cycle of Sec. 2 with the paper's coarse operators
    A_{l+1} = (1/omega) P_l^T A_l P_l and x_l += P_l x_{l+1}.  Only the
    aggregates and the colours of each level are taken from the hierarchy
    (both are pinned on their own); every operator is formed here.
    smoother: one smoother for every level, or a list with one per level
    (0 MC-SGS, 1 l1-Jacobi, 2 hybrid SGS, 3 hybrid SGS in colour order);
    tile_rows: the hybrid blocks' rows, one for every level or one per level."""
    L = H.levels
    sms = smoother if isinstance(smoother, (list, tuple)) else [smoother] * L
    Ts = tile_rows if isinstance(tile_rows, (list, tuple)) else [tile_rows] * L
    As, Ps, smooths = [A0], [], []
    for l in range(L - 1):
        lv = H.level(l)
        Pm = prolongation(lv.agg, H.level(l + 1).n)
        Ps.append(Pm)
        As.append((Pm.T @ As[l] @ Pm) / omega)
    for l in range(L - 1):
        A = As[l]
        lv = H.level(l)
        if sms[l] == 0:
            order = np.lexsort((np.arange(lv.n), lv.colour))  # colour, then row
            smooths.append(sgs_dense(A, order))
        elif sms[l] == 1:
            smooths.append(l1_jacobi_dense(A))
        elif sms[l] == 2:
            smooths.append(hybrid_dense(A, Ts[l]))
        else:
            smooths.append(hybrid_dense(A, Ts[l], lv.colour))

    def cycle(l, b):
        if l == L - 1:
            return np.linalg.solve(As[l], b)
        x = np.zeros_like(b)
        for _ in range(pre):
            x = smooths[l](b, x)
        xc = cycle(l + 1, Ps[l].T @ (b - As[l] @ x))
        x = x + Ps[l] @ xc
        for _ in range(post):
            x = smooths[l](b, x)
        return x
    return lambda b: cycle(0, b), As


CYCLE_CASES = [
    # (smoother, omega, pre, post)
    (0, 1.6, 1, 1), (0, 1.0, 1, 1), (0, 1.6, 2, 1), (0, 1.6, 1, 0), (0, 1.6, 0, 2),
    (1, 1.6, 1, 1), (1, 1.0, 2, 2), (1, 1.6, 0, 1),
    (2, 1.6, 1, 1), (2, 1.0, 1, 0),
    (3, 1.6, 1, 1), (3, 1.0, 0, 1),
]


@pytest.mark.parametrize("smoother,omega,pre,post", CYCLE_CASES)
def test_vcycle_equals_paper_cycle_with_scaled_coarse_operators(smoother, omega, pre, post):
    """Four levels of a lognormal 12^3 problem (64-row tiles): the oracle's
    cycle on every right-hand side equals the dense cycle of Sec. 2 built from
    A_{l+1} = (1/omega) P^T A_l P (Sec. 2.1)."""
    s = P.lognormal(12, seed=7)
    T = 64
    H = O.Hierarchy(s.rowptr, s.colind, s.vals, coarse_max=8, omega=omega, smoother=smoother,
                    pre_sweeps=pre, post_sweeps=post, tile_rows=T, colour_tile_rows=64)
    assert H.levels >= 4, H.levels
    A0 = dense(s.rowptr, s.colind, s.vals)
    ref, _ = paper_cycle(H, A0, omega, smoother, pre, post, T)
    rng = np.random.default_rng(11)
    for _ in range(4):
        b = rng.uniform(-1, 1, s.n)
        z = H.vcycle(b)
        zr = ref(b)
        assert np.abs(z - zr).max() <= 1e-11 * np.abs(zr).max()


@pytest.mark.parametrize("omega", [1.0, 1.6])
def test_three_level_coarse_correction_closed_form(omega):
    """With no smoothing, three levels give x = omega^2 Q (Q^T A Q)^-1 Q^T b,
    Q = P_0 P_1: the paper's A_2 = (1/omega^2) Q^T A Q inverted and prolongated
    twice without damping."""
    s = P.lognormal(10, seed=3)
    H = O.Hierarchy(s.rowptr, s.colind, s.vals, coarse_max=30, omega=omega, pre_sweeps=0, post_sweeps=0,
                    tile_rows=64)
    assert H.levels == 3, H.levels
    A = dense(s.rowptr, s.colind, s.vals)
    Q = prolongation(H.level(0).agg, H.level(1).n) @ prolongation(H.level(1).agg, H.level(2).n)
    Bref = omega ** 2 * Q @ np.linalg.solve(Q.T @ A @ Q, Q.T)
    B = np.column_stack([H.vcycle(e) for e in np.eye(s.n)])
    assert np.abs(B - Bref).max() <= 1e-10 * np.abs(Bref).max()


# One smoother on the first levels, another from coarse_from on.  An index
# mistake (from coarse_from + 1, or from coarse_from - 1) changes one level's
# smoother, and with it the cycle.
PER_LEVEL_CASES = [
    # (smoother, coarse_smoother, coarse_from)
    (0, 3, 1), (0, 3, 2), (0, 3, 3), (0, 1, 2), (0, 2, 1), (2, 0, 2), (3, 0, 1),
]


@pytest.mark.parametrize("smoother,coarse,start", PER_LEVEL_CASES)
def test_vcycle_per_level_smoothers_equal_paper_cycle(smoother, coarse, start):
    """Four or more levels of a lognormal 12^3 problem (64-row tiles) with
    `smoother` on levels 0..start-1 and `coarse` from level `start` on: the
    oracle's cycle equals the dense cycle of Sec. 2 with those smoothers."""
    s = P.lognormal(12, seed=7)
    T = 64
    H = O.Hierarchy(s.rowptr, s.colind, s.vals, coarse_max=8, smoother=smoother, coarse_smoother=coarse,
                    coarse_from=start, tile_rows=T, colour_tile_rows=64)
    assert H.levels >= 4, H.levels
    sms = [smoother if l < start else coarse for l in range(H.levels)]
    for l in range(H.levels - 1):  # the tile order needs the level's colouring
        assert (H.level(l).ncol > 1) == (sms[l] in (0, 1, 3)), (l, sms[l], H.level(l).ncol)
    A0 = dense(s.rowptr, s.colind, s.vals)
    ref, _ = paper_cycle(H, A0, 1.6, sms, 1, 1, T)
    rng = np.random.default_rng(12)
    for _ in range(3):
        b = rng.uniform(-1, 1, s.n)
        zr = ref(b)
        assert np.abs(H.vcycle(b) - zr).max() <= 1e-11 * np.abs(zr).max()


def first_fit_tile_colours(L, T):
    """Row by row in ascending order, the smallest colour that no earlier row
    of the same T-row tile coupled to it holds (brute force)."""
    c = np.empty(L.n, np.int64)
    for i in range(L.n):
        lo = i - i % T
        nb = L.colind[L.rowptr[i]:L.rowptr[i + 1]]
        used = set(c[nb[(nb >= lo) & (nb < i)]].tolist())
        c[i] = min(set(range(len(used) + 1)) - used)
    return c


# Smoothing tiles of their own size: `stile` rows on the levels above
# coarse_from, `ctile` from it on (0: tile_rows, and the finer levels' size).
# The sizes neither divide nor are multiples of the 64-row aggregation tiles,
# so a block size taken from the wrong parameter, or switched at the wrong
# level, changes the cycle.
SMOOTH_TILE_CASES = [
    # (smoother, coarse_smoother, coarse_from, smooth_tile_rows, coarse_smooth_tile_rows)
    (2, -1, 1, 200, 0), (2, -1, 2, 96, 16), (3, -1, 2, 0, 24), (0, 3, 1, 0, 40), (3, 2, 2, 300, 50),
    (2, 3, 1, 48, 0),
]


@pytest.mark.parametrize("smoother,coarse,start,stile,ctile", SMOOTH_TILE_CASES)
def test_vcycle_smoothing_tiles_equal_paper_cycle(smoother, coarse, start, stile, ctile):
    """Hybrid blocks of a size of their own (Sec. 3.2 with blocks that are
    not the aggregation tiles): aggregation is that of 64-row tiles whatever
    the blocks; tile-ordered levels are coloured first-fit per block; the
    cycle equals the dense cycle of Sec. 2 with hybrid blocks of those
    sizes."""
    s = P.lognormal(12, seed=7)
    kw = dict(coarse_max=8, smoother=smoother, coarse_smoother=coarse, coarse_from=start, tile_rows=64,
              colour_tile_rows=64)
    H = O.Hierarchy(s.rowptr, s.colind, s.vals, smooth_tile_rows=stile, coarse_smooth_tile_rows=ctile, **kw)
    H0 = O.Hierarchy(s.rowptr, s.colind, s.vals, **kw)
    assert H.levels == H0.levels >= 4
    sms = [coarse if coarse >= 0 and l >= start else smoother for l in range(H.levels)]
    Ts = [ctile if ctile and l >= start else (stile or 64) for l in range(H.levels)]
    for l in range(H.levels - 1):
        assert np.array_equal(H.level(l).agg, H0.level(l).agg), l
        if sms[l] == 3:
            assert np.array_equal(H.level(l).colour, first_fit_tile_colours(H.level(l), Ts[l])), l
    A0 = dense(s.rowptr, s.colind, s.vals)
    ref, _ = paper_cycle(H, A0, 1.6, sms, 1, 1, Ts)
    rng = np.random.default_rng(13)
    for _ in range(3):
        b = rng.uniform(-1, 1, s.n)
        zr = ref(b)
        assert np.abs(H.vcycle(b) - zr).max() <= 1e-11 * np.abs(zr).max()


def test_per_level_smoother_input_errors():
    """Smoother ids outside 0..3, a coarse smoother below -1 and a start level
    below 1 are rejected; point-based levels take the multicolour smoother on
    every level."""
    s = P.lognormal(6, seed=1)
    for kw in (dict(smoother=4), dict(smoother=-1), dict(coarse_smoother=4), dict(coarse_smoother=-2),
               dict(coarse_smoother=3, coarse_from=0), dict(coarse_smooth_tile_rows=64, coarse_from=0),
               dict(smooth_tile_rows=-1), dict(coarse_smooth_tile_rows=-64)):
        with pytest.raises(O.OracleError) as e:
            O.Hierarchy(s.rowptr, s.colind, s.vals, **kw)
        assert e.value.status == O.INVALID, kw
    O.Hierarchy(s.rowptr, s.colind, s.vals, coarse_smoother=-1, coarse_from=0)  # unused start level


# ------------------------------------------------------------------ l1-Jacobi
def test_l1_jacobi_sweep_hand_derived():
    """A = [[4, 1, -2], [1, 5, 0], [-2, 0, 6]] (one positive off-diagonal),
    x = (1, -1, 2), b = (0, 3, 1).  A x = (-1, -4, 10), b - A x = (1, 7, -9),
    row sums of |a_ij|: d = (7, 6, 8).  One sweep: x + (b - A x) / d =
    (1 + 1/7, -1 + 7/6, 2 - 9/8) = (8/7, 1/6, 7/8).  (With d_i = a_ii the
    result would be (1.25, 0.4, 0.5).)"""
    rp = np.array([0, 3, 5, 7], np.int32)
    ci = np.array([0, 1, 2, 0, 1, 0, 2], np.int32)
    v = np.array([4.0, 1.0, -2.0, 1.0, 5.0, -2.0, 6.0])
    H = O.Hierarchy(rp, ci, v, smoother=1)
    x = H.smooth(0, np.array([0.0, 3.0, 1.0]), np.array([1.0, -1.0, 2.0]))
    expect = np.array([8 / 7, 1 / 6, 7 / 8])
    assert np.abs(x - expect).max() <= 4e-16
    xf = H.smooth(0, np.array([0.0, 3.0, 1.0]), np.array([1.0, -1.0, 2.0]), fp32=True)
    assert np.abs(xf - expect).max() <= 4e-7


def test_l1_jacobi_converges_where_jacobi_diverges():
    """For SPD A, D_l1 - A is weakly diagonally dominant with a non-negative
    diagonal, hence positive semi-definite, so the l1 sweep is A-norm
    contracting.  On a matrix with large positive off-diagonals plain Jacobi
    (d_i = a_ii) has an error operator with spectral radius above one."""
    rng = np.random.default_rng(5)
    n = 12
    M = rng.uniform(0.2, 1.0, (n, n))
    A = (M + M.T) / 2
    np.fill_diagonal(A, 0.0)
    A = A + np.diag(A.sum(axis=1) * 0.6)
    A = A + (-np.linalg.eigvalsh(A).min() + 0.5) * np.eye(n)  # SPD, off-diagonals positive
    Dj = np.diag(np.diag(A))
    assert np.abs(np.linalg.eigvals(np.eye(n) - np.linalg.solve(Dj, A))).max() > 1.0
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    H = O.Hierarchy(rp, ci, A.ravel().copy(), smoother=1)
    E = np.column_stack([H.smooth(0, np.zeros(n), e) for e in np.eye(n)])  # error operator
    assert np.abs(np.linalg.eigvals(E)).max() < 1.0
    d = np.abs(A).sum(axis=1)
    assert np.abs(E - (np.eye(n) - A / d[:, None])).max() <= 1e-15


# ------------------------------------------------------------- coarsening stop
def pairs_and_singletons(m, s):
    """m pairs of rows (2i, 2i+1) coupled as [[2, -1], [-1, 2]] followed by s
    uncoupled rows with diagonal 3.  Each pair is two-way strong and becomes one
    aggregate (no other candidates); each uncoupled row is isolated and stays a
    singleton (no adjacent aggregate): m + s aggregates of 2m + s rows.  The
    Galerkin matrix of a pair is the 1x1 matrix 2 with no coupling."""
    rp, ci, v = [0], [], []
    for i in range(m):
        a, b = 2 * i, 2 * i + 1
        ci += [a, b, a, b]
        v += [2.0, -1.0, -1.0, 2.0]
        rp += [rp[-1] + 2, rp[-1] + 4]
    for k in range(s):
        ci.append(2 * m + k)
        v.append(3.0)
        rp.append(rp[-1] + 1)
    return np.array(rp, np.int32), np.array(ci, np.int32), np.array(v)


def test_coarsening_continues_at_exactly_nine_tenths():
    """n = 1000 rows, 900 aggregates: 900 is not above 0.9 n, so the level is
    kept; the next level (900 isolated rows, 900 singletons) does not shrink
    and becomes the coarsest."""
    H = O.Hierarchy(*pairs_and_singletons(100, 800))
    assert H.levels == 2 and H.level(1).n == 900
    assert H.level(0).agg.max() == 899


def test_coarsening_stops_above_nine_tenths():
    """n = 1000 rows, 901 aggregates: the level would shrink by less than 10 %,
    so level 0 itself is the coarsest (1000 <= 4096 rows: factorised)."""
    H = O.Hierarchy(*pairs_and_singletons(99, 802))
    assert H.levels == 1 and H.level(0).n == 1000


def test_coarsest_factor_of_stalled_level_is_its_cholesky():
    """The stalled level of 1000 rows is factorised exactly: L L^T = A."""
    rp, ci, v = pairs_and_singletons(99, 802)
    H = O.Hierarchy(rp, ci, v)
    Lf = H.coarse_factor()
    A = dense(rp, ci, v)
    assert np.abs(Lf @ Lf.T - A).max() <= 1e-14


def test_stalled_above_4096_rows():
    """A diagonal matrix does not coarsen (all rows isolated singletons); with
    4097 rows the coarsest level would exceed 4096 rows: COARSENING_STALLED."""
    n = 4097
    with pytest.raises(O.OracleError) as e:
        O.Hierarchy(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 3.0))
    assert e.value.status == O.STALLED


def test_stalled_level_of_4096_rows_is_factorised():
    """4096 rows is the largest coarsest level: the diagonal matrix is kept as
    one level and factorised (diagonal factor sqrt(3))."""
    n = 4096
    H = O.Hierarchy(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 3.0))
    assert H.levels == 1
    L = H.coarse_factor()
    assert np.array_equal(np.diag(L), np.full(n, np.sqrt(3.0)))


def test_max_levels_ends_the_hierarchy():
    """max_levels caps the hierarchy even while levels still shrink."""
    s = P.poisson(12)
    full = O.Hierarchy(s.rowptr, s.colind, s.vals, coarse_max=8, tile_rows=64)
    assert full.levels >= 3
    capped = O.Hierarchy(s.rowptr, s.colind, s.vals, coarse_max=8, tile_rows=64, max_levels=2)
    assert capped.levels == 2 and capped.level(1).n == full.level(1).n


# --------------------------------------------------------------- CG breakdown
def indefinite_pairs(c=5.0, across=(0, 2)):
    """Four rows: pairs (0, 1) and (2, 3) coupled by -1 (two-way strong, one
    aggregate each), diagonal 4, and one weak positive coupling c between the
    rows `across`.  For c = 5 across (0, 2) A is symmetric with a positive
    diagonal but indefinite (v = (1, 0, -1, 0): v^T A v = 8 - 2c < 0); its
    Galerkin matrix [[6, c], [c, 6]] is SPD for c < 6, so the coarsest
    factorisation succeeds."""
    A = np.diag([4.0] * 4)
    A[0, 1] = A[1, 0] = A[2, 3] = A[3, 2] = -1.0
    i, j = across
    A[i, j] = A[j, i] = c
    rp, ci, v = [0], [], []
    for r in range(4):
        for k in range(4):
            if A[r, k] != 0:
                ci.append(k)
                v.append(A[r, k])
        rp.append(len(ci))
    return A, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v)


def numpy_pcg_breakdown(A, B, b, maxit):
    """Textbook PCG with preconditioner matrix B; returns the iteration count at
    which r.z <= 0 or p.Ap <= 0 first occurs, and which one."""
    r = b.copy()
    z = B @ r
    p = z.copy()
    rho = r @ z
    if not rho > 0:
        return 0, "rz"
    x = np.zeros_like(b)
    for k in range(1, maxit + 1):
        q = A @ p
        pq = p @ q
        if not pq > 0:
            return k - 1, "pq"
        a = rho / pq
        x = x + a * p
        r = r - a * q
        z = B @ r
        rz = r @ z
        if not rz > 0:
            return k, "rz"
        p = z + (rz / rho) * p
        rho = rz
    return None, None


BREAKDOWN_CASES = [
    # (c, across, pre, post, b, (iteration, kind) from the numpy CG)
    (5.0, (0, 2), 1, 1, [1.0, 0.0, -1.0, 0.0], (0, "pq")),
    (5.0, (0, 2), 1, 1, [0.0872, 0.8701, 0.6317, -0.9945], (1, "pq")),
    (5.0, (0, 2), 1, 1, [1.0, 1.0, 1.0, 1.0], (0, "pq")),
    (5.5, (0, 2), 1, 0, [-1.0, 0.9, -0.4, -0.4], (0, "rz")),
    (5.5, (0, 2), 1, 0, [-0.2, 0.3, -0.3, -0.6], (4, "pq")),
    (5.5, (0, 2), 1, 0, [0.0, 0.4, 0.2, -0.9], (6, "pq")),
]


@pytest.mark.parametrize("c,across,pre,post,b,expect", BREAKDOWN_CASES)
def test_cg_breakdown_on_indefinite_matrix(c, across, pre, post, b, expect):
    """PCG with the oracle's cycle breaks down exactly where a numpy PCG with
    the dense paper cycle (an SPD-looking but indefinite A) finds r.z <= 0 or
    p.Ap <= 0; x0 = 0."""
    A, rp, ci, v = indefinite_pairs(c, across)
    assert np.linalg.eigvalsh(A).min() < 0
    assert O.validate(rp, ci, v) == O.OK
    H = O.Hierarchy(rp, ci, v, coarse_max=2, tile_rows=64, flexible=0, pre_sweeps=pre, post_sweeps=post)
    assert H.levels == 2 and H.level(0).agg.tolist() == [0, 0, 1, 1]
    cyc, _ = paper_cycle(H, A, 1.6, 0, pre, post, 64)
    B = np.column_stack([cyc(e) for e in np.eye(4)])
    Bo = np.column_stack([H.vcycle(e) for e in np.eye(4)])
    assert np.abs(B - Bo).max() <= 1e-12 * np.abs(B).max()
    b = np.array(b)
    assert numpy_pcg_breakdown(A, B, b, 50) == expect
    out = H.pcg(b, maxit=50)
    assert out["status"] == O.BREAKDOWN and out["iterations"] == expect[0]
