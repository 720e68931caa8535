"""Seeded synthetic workloads: 7-point cell-centred finite-volume diffusion
matrices on structured boxes, their coefficient fields and right-hand sides.

This module holds no part of the multigrid method: it only discretises the
model problem -div(K grad u) = f (the SPD sign convention of the paper's model
problem, Sec. 2, eqs. (model) and (ls)) so that both the CPU oracle and the GPU
path receive the same CSR arrays.

Discretisation (lowest-order cell-centred finite volumes on an nx*ny*nz box):
  * interior face between cells a and b: transmissibility t = 2 Ka Kb / (Ka + Kb)
    (harmonic average of the two cell coefficients);
  * boundary face: homogeneous Dirichlet at distance h/2, t = 2 K_cell;
  * A_ii = sum of the six face values (fixed order -x,+x,-y,+y,-z,+z),
    A_ij = -t for the shared face; the common factor h is dropped so that
    K == 1 yields integer entries.

Row order: Morton (bit-interleaved x, y, z with x in the lowest bit), so that
512 consecutive rows of a box whose edges are multiples of 8 form an 8^3 cube.
For edges that are not powers of two the Morton codes are sorted and compacted.
Random draws are always taken in lexicographic cell order (x fastest) and then
permuted, so fields and right-hand sides do not depend on the row order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class CSRSystem:
    """A CSR matrix (int32 row pointers / columns, float64 values) plus a RHS."""

    rowptr: np.ndarray
    colind: np.ndarray
    vals: np.ndarray
    b: np.ndarray
    shape: tuple  # (nx, ny, nz)
    order: np.ndarray  # order[r] = lexicographic cell index of row r

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])


def morton_order(nx: int, ny: int, nz: int) -> np.ndarray:
    """Return order[r] = lexicographic index (x fastest) of the r-th Morton cell."""
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.int64), np.arange(ny, dtype=np.int64),
                          np.arange(nx, dtype=np.int64), indexing="ij")
    x = x.ravel(); y = y.ravel(); z = z.ravel()
    code = np.zeros(x.shape, dtype=np.int64)
    bits = max(1, int(math.ceil(math.log2(max(nx, ny, nz, 2)))))
    for b in range(bits):
        code |= ((x >> b) & 1) << (3 * b)
        code |= ((y >> b) & 1) << (3 * b + 1)
        code |= ((z >> b) & 1) << (3 * b + 2)
    n = nx * ny * nz
    if nx == ny == nz and (nx & (nx - 1)) == 0:
        order = np.empty(n, dtype=np.int64)
        order[code] = np.arange(n, dtype=np.int64)
        return order
    return np.argsort(code, kind="stable")


def ccfv7(K: np.ndarray) -> tuple:
    """Assemble the 7-point CCFV operator for a coefficient field K[z, y, x].

    Returns (rowptr, colind, vals, order) in Morton row order with ascending
    columns in every row and the diagonal stored.
    """
    K = np.ascontiguousarray(K, dtype=np.float64)
    nz, ny, nx = K.shape
    n = nx * ny * nz

    def harm(a, b):
        return 2.0 * a * b / (a + b)

    # face values per direction, shape of the cell array, boundary faces 2K
    txm = np.empty_like(K); txp = np.empty_like(K)
    tym = np.empty_like(K); typ = np.empty_like(K)
    tzm = np.empty_like(K); tzp = np.empty_like(K)
    fx = harm(K[:, :, :-1], K[:, :, 1:])
    txp[:, :, :-1] = fx; txp[:, :, -1] = 2.0 * K[:, :, -1]
    txm[:, :, 1:] = fx; txm[:, :, 0] = 2.0 * K[:, :, 0]
    fy = harm(K[:, :-1, :], K[:, 1:, :])
    typ[:, :-1, :] = fy; typ[:, -1, :] = 2.0 * K[:, -1, :]
    tym[:, 1:, :] = fy; tym[:, 0, :] = 2.0 * K[:, 0, :]
    fz = harm(K[:-1, :, :], K[1:, :, :])
    tzp[:-1, :, :] = fz; tzp[-1, :, :] = 2.0 * K[-1, :, :]
    tzm[1:, :, :] = fz; tzm[0, :, :] = 2.0 * K[0, :, :]
    del fx, fy, fz
    diag = txm + txp
    diag += tym
    diag += typ
    diag += tzm
    diag += tzp

    order = morton_order(nx, ny, nz)
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n, dtype=np.int64)

    z, y, x = np.unravel_index(order, (nz, ny, nx))
    sentinel = n
    cols = np.full((n, 7), sentinel, dtype=np.int64)
    vals = np.zeros((n, 7), dtype=np.float64)
    rows = np.arange(n, dtype=np.int64)
    cols[:, 0] = rows
    vals[:, 0] = diag.ravel()[order]
    del diag
    lex = order
    stride = {"x": 1, "y": nx, "z": nx * ny}
    slot = 1
    for axis, coord, ext, tm, tp in (("x", x, nx, txm, txp), ("y", y, ny, tym, typ),
                                     ("z", z, nz, tzm, tzp)):
        s = stride[axis]
        lo = coord > 0
        cols[lo, slot] = inv[lex[lo] - s]
        vals[lo, slot] = -tm.ravel()[lex[lo]]
        slot += 1
        hi = coord < ext - 1
        cols[hi, slot] = inv[lex[hi] + s]
        vals[hi, slot] = -tp.ravel()[lex[hi]]
        slot += 1
    del x, y, z, inv
    perm = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, perm, axis=1)
    vals = np.take_along_axis(vals, perm, axis=1)
    del perm
    valid = cols < sentinel
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cols[valid].astype(np.int32)
    v = vals[valid]
    return rowptr.astype(np.int32), colind, np.ascontiguousarray(v), order


def field_constant(n: int, shape=None) -> np.ndarray:
    nx, ny, nz = shape if shape is not None else (n, n, n)
    return np.ones((nz, ny, nx), dtype=np.float64)


def field_lognormal(rng: np.random.Generator, n: int, sigma2: float, window: int,
                    divisor: float) -> np.ndarray:
    """K = exp(sigma * g') with g' a window-summed white noise field.

    g ~ N(0,1) i.i.d. on (n+window-1)^3 points (lexicographic draw, x fastest);
    g'[z,y,x] = (sum of the window^3 block starting at [z,y,x]) / divisor.
    """
    m = n + window - 1
    g = rng.standard_normal(m * m * m).reshape(m, m, m)
    gs = np.zeros((n, n, n), dtype=np.float64)
    for dz in range(window):
        for dy in range(window):
            for dx in range(window):
                gs += g[dz:dz + n, dy:dy + n, dx:dx + n]
    gs /= divisor
    return np.exp(math.sqrt(sigma2) * gs)


def field_layered(rng: np.random.Generator, n: int, layer: int = 4) -> np.ndarray:
    """K = 10^{u_z} * exp(eps): u_z ~ U[-3,3] per z-layer of `layer` cells, eps ~ N(0,1)."""
    nl = (n + layer - 1) // layer
    u = rng.uniform(-3.0, 3.0, nl)
    eps = rng.standard_normal(n * n * n).reshape(n, n, n)
    zlayer = np.arange(n) // layer
    return (10.0 ** u[zlayer])[:, None, None] * np.exp(eps)


def field_jump_cube(n: int) -> np.ndarray:
    """Coefficient of the jump problem: k = 1e3 in a centred cube of width 0.8,
    k = 1e-2 in the eight corner cubes of width 0.1, k = 1 elsewhere (cell centres)."""
    c = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    K = np.ones((n, n, n))
    inner = (np.abs(X - 0.5) < 0.4) & (np.abs(Y - 0.5) < 0.4) & (np.abs(Z - 0.5) < 0.4)
    K[inner] = 1e3

    def corner(v):
        return (v < 0.1) | (v > 0.9)

    K[corner(X) & corner(Y) & corner(Z)] = 1e-2
    return K


def _rhs(rng: np.random.Generator, order: np.ndarray) -> np.ndarray:
    b_lex = rng.uniform(-1.0, 1.0, order.shape[0])
    return np.ascontiguousarray(b_lex[order])


def poisson(n: int, seed: int = 0, shape=None) -> CSRSystem:
    """K == 1 on an n^3 (or nx*ny*nz) box; b ~ U[-1,1] from default_rng(seed)."""
    nx, ny, nz = shape if shape is not None else (n, n, n)
    K = field_constant(n, (nx, ny, nz))
    rowptr, colind, vals, order = ccfv7(K)
    rng = np.random.default_rng(seed)
    return CSRSystem(rowptr, colind, vals, _rhs(rng, order), (nx, ny, nz), order)


def lognormal(n: int, seed: int = 1, sigma2: float = 4.0, window: int = 2,
              divisor: float = math.sqrt(8.0)) -> CSRSystem:
    """Heterogeneous lognormal K (defaults: sigma^2 = 4, normalised 2x2x2 box filter)."""
    rng = np.random.default_rng(seed)
    K = field_lognormal(rng, n, sigma2, window, divisor)
    rowptr, colind, vals, order = ccfv7(K)
    return CSRSystem(rowptr, colind, vals, _rhs(rng, order), (n, n, n), order)


def layered(n: int, seed: int = 2) -> CSRSystem:
    """Layered lognormal K with contrast about 1e6."""
    rng = np.random.default_rng(seed)
    K = field_layered(rng, n)
    rowptr, colind, vals, order = ccfv7(K)
    return CSRSystem(rowptr, colind, vals, _rhs(rng, order), (n, n, n), order)


def jump_cube(n: int, seed: int = 5) -> CSRSystem:
    K = field_jump_cube(n)
    rowptr, colind, vals, order = ccfv7(K)
    rng = np.random.default_rng(seed)
    return CSRSystem(rowptr, colind, vals, _rhs(rng, order), (n, n, n), order)


def manufactured_exact(x, y, z) -> np.ndarray:
    """u = exp(-|x|^2) of the manufactured Poisson problem."""
    return np.exp(-(x * x + y * y + z * z))


def manufactured(n: int) -> tuple:
    """The Poisson problem with a known solution of the paper's helics3a runs
    (Sec. 5): -Laplace u = f in (0,1)^3, u = g on the boundary.  The printed
    pair is inconsistent (for u = exp(|x|), -Laplace u = -(1 + 2/|x|) exp(|x|)),
    so the consistent pair u = exp(-|x|^2), f = (6 - 4|x|^2) exp(-|x|^2) is
    used, with g = u.  K = 1 gives the matrix of `poisson`; with the dropped
    factor h, row i reads sum_faces t (u_i - u_j) = h^2 f(x_i) + 2 g(c) summed
    over the centres c of its boundary faces (Dirichlet data at distance h/2).
    Returns (system, exact u at the cell centres in row order); the
    discrete solution converges to it as O(h^2)."""
    h = 1.0 / n
    K = field_constant(n, (n, n, n))
    rowptr, colind, vals, order = ccfv7(K)
    c = (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r2 = X * X + Y * Y + Z * Z
    b = h * h * (6.0 - 4.0 * r2) * np.exp(-r2)
    # one term per boundary face (corner and edge cells have several)
    b[:, :, 0] += 2.0 * manufactured_exact(0.0, Y[:, :, 0], Z[:, :, 0])
    b[:, :, -1] += 2.0 * manufactured_exact(1.0, Y[:, :, -1], Z[:, :, -1])
    b[:, 0, :] += 2.0 * manufactured_exact(X[:, 0, :], 0.0, Z[:, 0, :])
    b[:, -1, :] += 2.0 * manufactured_exact(X[:, -1, :], 1.0, Z[:, -1, :])
    b[0, :, :] += 2.0 * manufactured_exact(X[0, :, :], Y[0, :, :], 0.0)
    b[-1, :, :] += 2.0 * manufactured_exact(X[-1, :, :], Y[-1, :, :], 1.0)
    u = manufactured_exact(X, Y, Z)
    sysm = CSRSystem(rowptr, colind, vals, np.ascontiguousarray(b.ravel()[order]), (n, n, n), order)
    return sysm, np.ascontiguousarray(u.ravel()[order])


def block_expand(rowptr, colind, blocks: np.ndarray) -> tuple:
    """Scalar form of a block matrix with bs x bs blocks: node i's unknowns
    are rows i*bs .. i*bs+bs-1 (node-major), every stored block is stored in
    full, columns ascend in every row.  blocks[k] is the block of node entry k
    (row-major, shape (nnzb, bs, bs))."""
    nb = rowptr.shape[0] - 1
    bs = blocks.shape[1]
    cnt = np.diff(rowptr).astype(np.int64)
    nrow = nb * bs
    rp = np.zeros(nrow + 1, np.int64)
    rp[1:] = np.cumsum(np.repeat(cnt * bs, bs))
    node_of_entry = np.repeat(np.arange(nb), cnt)
    # scalar entry (i*bs + c, colind[k]*bs + d) at rp[i*bs + c] + (k - rowptr[i]) * bs + d
    k = np.arange(colind.shape[0])
    pos_in_row = (k - rowptr[node_of_entry]) * bs
    ci = np.empty(rp[-1], np.int64)
    v = np.empty(rp[-1], np.float64)
    for c in range(bs):
        base = rp[node_of_entry * bs + c] + pos_in_row
        for d in range(bs):
            ci[base + d] = colind * bs + d
            v[base + d] = blocks[:, c, d]
    return rp.astype(np.int32), ci.astype(np.int32), v


def coupled(n: int, bs: int = 3, seed: int = 6, sigma2: float = 2.0) -> CSRSystem:
    """A bs-component coupled diffusion system on n^3 cells (point-based AMG
    workload): A = sum over interior faces f = (i, j) of
    t_f (e_i - e_j)(e_i - e_j)^T (x) C_f plus, for every boundary face of cell
    i, 2 K_i e_i e_i^T (x) I, with t_f the harmonic face transmissibility of a
    lognormal K (sigma^2, 2x2x2 box filter) and C_f = I + v_f v_f^T a face
    coupling with v_f ~ U[0,1]^bs.  SPD; off-diagonal blocks -t_f C_f have
    only negative entries, diagonal blocks are dense.  Returned in scalar form,
    node-major (unknown c of cell-row i is row i*bs + c), cells in Morton order.
    Draws from default_rng(seed): the field, then v for the x-, y- and z-faces
    (one vector per cell and axis, lexicographic order), then b."""
    rng = np.random.default_rng(seed)
    K = field_lognormal(rng, n, sigma2, 2, math.sqrt(8.0))
    rowptr, colind, vals, order = ccfv7(K)
    nc = n * n * n
    V = [rng.uniform(0.0, 1.0, (nc, bs)) for _ in range(3)]  # faces to the +x, +y, +z neighbour
    nb = rowptr.shape[0] - 1
    rows = np.repeat(np.arange(nb), np.diff(rowptr))
    off = colind != rows
    lex_i = order[rows]
    lex_j = order[colind]
    d = np.abs(lex_j - lex_i)
    low = np.minimum(lex_i, lex_j)
    axis = np.where(d == 1, 0, np.where(d == n, 1, 2))
    I = np.eye(bs)
    blocks = np.zeros((colind.shape[0], bs, bs))
    ko = np.nonzero(off)[0]
    v = np.stack(V)[axis[ko], low[ko]]
    C = I[None, :, :] + v[:, :, None] * v[:, None, :]
    t = -vals[ko]  # transmissibility of the face
    blocks[ko] = -t[:, None, None] * C
    # diagonal block: couplings of the faces plus the boundary faces (identity)
    kd = np.nonzero(~off)[0]
    face_sum = np.zeros((nb, bs, bs))
    np.add.at(face_sum, rows[ko], t[:, None, None] * C)
    tsum = np.zeros(nb)
    np.add.at(tsum, rows[ko], t)
    bnd = vals[kd] - tsum  # boundary faces 2 K of every cell (diagonal entry minus interior faces)
    blocks[kd] = face_sum + bnd[:, None, None] * I[None, :, :]
    rp, ci, vv = block_expand(rowptr, colind, blocks)
    b = rng.uniform(-1.0, 1.0, (nc, bs))[order].reshape(-1)
    return CSRSystem(rp, ci, vv, np.ascontiguousarray(b), (n, n, n), order)


def from_field(K: np.ndarray, seed: int = 0) -> CSRSystem:
    nz, ny, nx = K.shape
    rowptr, colind, vals, order = ccfv7(K)
    rng = np.random.default_rng(seed)
    return CSRSystem(rowptr, colind, vals, _rhs(rng, order), (nx, ny, nz), order)


def batched_systems(count: int = 64, seed: int = 3, edges=(16, 24, 32, 48, 64),
                    nrhs: int = 4, sigma2: float = 2.0) -> list:
    """Independent lognormal systems with edges drawn from `edges` (4^3 window / 8)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(edges), size=count)
    out = []
    for n in ns:
        n = int(n)
        K = field_lognormal(rng, n, sigma2, 4, 8.0)
        rowptr, colind, vals, order = ccfv7(K)
        B = rng.uniform(-1.0, 1.0, (nrhs, n * n * n))[:, order]
        out.append(CSRSystem(rowptr, colind, vals, np.ascontiguousarray(B), (n, n, n), order))
    return out


def nnz_7pt(nx: int, ny: int, nz: int) -> int:
    """Stored entries of the 7-point operator with eliminated Dirichlet boundaries."""
    return nx * ny * nz + 2 * ((nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1))


# ---------------------------------------------------------------- device generation
# The same discretisation with torch tensor operations, for workloads too large
# to generate on the host (a request stream).  ccfv7_torch(K) on a float64
# tensor returns exactly the arrays of ccfv7(K.numpy()) (same face formulas and
# summation order, same Morton order), on K's device.

def morton_order_torch(nx: int, ny: int, nz: int, device) -> "torch.Tensor":
    import torch
    z, y, x = torch.meshgrid(torch.arange(nz, device=device), torch.arange(ny, device=device),
                             torch.arange(nx, device=device), indexing="ij")
    x = x.reshape(-1); y = y.reshape(-1); z = z.reshape(-1)
    code = torch.zeros_like(x)
    bits = max(1, int(math.ceil(math.log2(max(nx, ny, nz, 2)))))
    for b in range(bits):
        code |= ((x >> b) & 1) << (3 * b)
        code |= ((y >> b) & 1) << (3 * b + 1)
        code |= ((z >> b) & 1) << (3 * b + 2)
    return torch.argsort(code, stable=True)


def ccfv7_torch(K) -> tuple:
    """Device twin of ccfv7: (rowptr int32, colind int32, vals float64, order int64)."""
    import torch
    K = K.to(torch.float64).contiguous()
    nz, ny, nx = K.shape
    n = nx * ny * nz
    dev = K.device

    def harm(a, b):
        return 2.0 * a * b / (a + b)

    txm = torch.empty_like(K); txp = torch.empty_like(K)
    tym = torch.empty_like(K); typ = torch.empty_like(K)
    tzm = torch.empty_like(K); tzp = torch.empty_like(K)
    fx = harm(K[:, :, :-1], K[:, :, 1:])
    txp[:, :, :-1] = fx; txp[:, :, -1] = 2.0 * K[:, :, -1]
    txm[:, :, 1:] = fx; txm[:, :, 0] = 2.0 * K[:, :, 0]
    fy = harm(K[:, :-1, :], K[:, 1:, :])
    typ[:, :-1, :] = fy; typ[:, -1, :] = 2.0 * K[:, -1, :]
    tym[:, 1:, :] = fy; tym[:, 0, :] = 2.0 * K[:, 0, :]
    fz = harm(K[:-1, :, :], K[1:, :, :])
    tzp[:-1, :, :] = fz; tzp[-1, :, :] = 2.0 * K[-1, :, :]
    tzm[1:, :, :] = fz; tzm[0, :, :] = 2.0 * K[0, :, :]
    del fx, fy, fz
    diag = txm + txp
    diag += tym
    diag += typ
    diag += tzm
    diag += tzp
    order = morton_order_torch(nx, ny, nz, dev)
    inv = torch.empty(n, dtype=torch.int64, device=dev)
    inv[order] = torch.arange(n, dtype=torch.int64, device=dev)
    x = order % nx
    y = (order // nx) % ny
    z = order // (nx * ny)
    cols = torch.full((n, 7), n, dtype=torch.int64, device=dev)
    vals = torch.zeros((n, 7), dtype=torch.float64, device=dev)
    cols[:, 0] = torch.arange(n, dtype=torch.int64, device=dev)
    vals[:, 0] = diag.reshape(-1)[order]
    del diag
    slot = 1
    for s, coord, ext, tm, tp in ((1, x, nx, txm, txp), (nx, y, ny, tym, typ), (nx * ny, z, nz, tzm, tzp)):
        lo = coord > 0
        cols[lo, slot] = inv[order[lo] - s]
        vals[lo, slot] = -tm.reshape(-1)[order[lo]]
        slot += 1
        hi = coord < ext - 1
        cols[hi, slot] = inv[order[hi] + s]
        vals[hi, slot] = -tp.reshape(-1)[order[hi]]
        slot += 1
    del x, y, z, inv, txm, txp, tym, typ, tzm, tzp
    cols, perm = torch.sort(cols, dim=1, stable=True)
    vals = torch.gather(vals, 1, perm)
    del perm
    valid = cols < n
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    rowptr[1:] = torch.cumsum(valid.sum(dim=1), 0)
    colind = cols[valid].to(torch.int32)
    v = vals[valid].contiguous()
    return rowptr.to(torch.int32), colind, v, order


def lognormal_torch(edge: int, sigma2: float, generator, window: int = 2, divisor: float = math.sqrt(8.0),
                    nrhs: int = 1):
    """Lognormal K (g ~ N(0,1) on (edge+window-1)^3, window sum / divisor,
    K = exp(sigma g')) and nrhs right-hand sides U[-1,1], drawn on the
    generator's device in that order; returns (rowptr, colind, vals, b) with b
    of shape (nrhs, edge^3) in row order."""
    import torch
    dev = generator.device
    n = edge
    m = n + window - 1
    g = torch.randn((m, m, m), generator=generator, device=dev, dtype=torch.float64)
    gs = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    for dz in range(window):
        for dy in range(window):
            for dx in range(window):
                gs += g[dz:dz + n, dy:dy + n, dx:dx + n]
    del g
    gs /= divisor
    K = torch.exp(math.sqrt(sigma2) * gs)
    del gs
    rp, ci, v, order = ccfv7_torch(K)
    del K
    b = rhs_torch(order, generator, nrhs)
    return rp, ci, v, b


def rhs_torch(order, generator, nrhs: int = 1):
    """nrhs right-hand sides U[-1,1] drawn in lexicographic cell order, returned in row order."""
    import torch
    n = order.numel()
    b = torch.rand((nrhs, n), generator=generator, device=order.device, dtype=torch.float64) * 2.0 - 1.0
    return b[:, order].contiguous()


def serving_trace(rate: float = 200.0, seconds: float = 60.0, seed: int = 4, edges=(32, 256),
                  sigma2=(0.0, 4.0), reuse: float = 0.3) -> list:
    """Request stream: Poisson arrivals (exponential gaps of mean 1/rate) until
    `seconds`; per request, in this order: edge ~ U{edges}, sigma^2 ~ U[sigma2],
    reuse ~ Bernoulli(reuse) and, when reusing, a target drawn uniformly from
    the earlier requests that introduced a new matrix (the request then solves
    that matrix with a new right-hand side).  Request i draws its own field
    and right-hand side from the stream seeded by SeedSequence([seed, i])."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out, news = [], []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        i = len(out)
        edge = int(rng.integers(edges[0], edges[1] + 1))
        s2 = float(rng.uniform(sigma2[0], sigma2[1]))
        hit = bool(rng.random() < reuse)
        if hit and news:
            j = news[int(rng.integers(len(news)))]
            edge, s2, matrix = out[j]["edge"], out[j]["sigma2"], j
        else:
            matrix = i
            news.append(i)
        seed_i = int(np.random.SeedSequence([seed, i]).generate_state(1)[0])
        out.append(dict(id=i, t=t, edge=edge, sigma2=s2, matrix=matrix, seed=seed_i))
    return out


# ---------------------------------------------------------------- large layered workload
def layered_field_and_rhs(n: int, seed: int = 2):
    """Layered field K[z, y, x] (field_layered recipe) and b_lex ~ U[-1,1] in
    lexicographic order, drawn in that order from default_rng(seed); returns
    (K, b_lex, rng) with rng positioned after the draws."""
    rng = np.random.default_rng(seed)
    K = field_layered(rng, n)
    b_lex = rng.uniform(-1.0, 1.0, n * n * n)
    return K, b_lex, rng


def layered_subsampled(n_full: int = 512, seed: int = 2) -> CSRSystem:
    """The (n_full/2)^3 system of the field sampled at even cells,
    K_sub[k, j, i] = K[2k, 2j, 2i], with its own b drawn from the same
    generator after the full-size field and right-hand side."""
    K, _, rng = layered_field_and_rhs(n_full, seed)
    Ks = np.ascontiguousarray(K[::2, ::2, ::2])
    del K
    rowptr, colind, vals, order = ccfv7(Ks)
    m = n_full // 2
    b = rng.uniform(-1.0, 1.0, m * m * m)[order]
    return CSRSystem(rowptr, colind, vals, np.ascontiguousarray(b), (m, m, m), order)
