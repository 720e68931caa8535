"""CPU oracle of the aggregation AMG-PCG: ctypes shim over liboracle.so.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this package.  The product library never does.

Every function takes plain numpy arrays (int32 CSR, float64 values) and follows
the paper's definitions; the C source states the reading used for each step.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_LIB = None

I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
U8P = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")

# status codes of the oracle
OK, INVALID, BAD_DIAGONAL, NOT_SYMMETRIC, NOT_SPD, STALLED, BREAKDOWN, NOT_CONVERGED = 0, 1, 2, 3, 4, 5, 7, 8


class Params(C.Structure):
    _fields_ = [("strength_threshold", C.c_double), ("isolated_threshold", C.c_double),
                ("agg_min", C.c_int), ("agg_max", C.c_int), ("agg_diameter", C.c_int),
                ("omega", C.c_double), ("coarse_max", C.c_int), ("max_levels", C.c_int),
                ("tile_rows", C.c_int), ("smoother", C.c_int), ("pre_sweeps", C.c_int),
                ("post_sweeps", C.c_int), ("vcycle_fp32", C.c_int), ("flexible", C.c_int),
                ("colour_seed", C.c_uint32), ("check_symmetry", C.c_int), ("colour_tile_rows", C.c_int),
                ("block_size", C.c_int), ("coarse_smoother", C.c_int), ("coarse_from", C.c_int),
                ("smooth_tile_rows", C.c_int), ("coarse_smooth_tile_rows", C.c_int)]


def default_params(**kw) -> Params:
    p = Params(strength_threshold=0.08, isolated_threshold=1e-5, agg_min=8, agg_max=12,
               agg_diameter=3, omega=1.6, coarse_max=500, max_levels=25, tile_rows=128,
               smoother=0, pre_sweeps=1, post_sweeps=1, vcycle_fp32=0, flexible=-1,
               colour_seed=0, check_symmetry=1, colour_tile_rows=128, block_size=1,
               coarse_smoother=-1, coarse_from=1, smooth_tile_rows=0, coarse_smooth_tile_rows=0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        src = _build.SRC
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        L = C.CDLL(path)
        L.orc_validate.restype = C.c_int
        L.orc_validate.argtypes = [C.c_int, C.c_int, I32P, I32P, F64P, C.c_int]
        L.orc_strength.restype = None
        L.orc_strength.argtypes = [C.c_int, C.c_int, I32P, I32P, F64P, C.c_int, C.c_double, C.c_double, U8P, U8P]
        L.orc_aggregate.restype = C.c_int
        L.orc_aggregate.argtypes = [C.c_int, C.c_int, I32P, I32P, U8P, U8P, C.c_int, C.c_int, C.c_int, C.c_int,
                                    I32P, I32P]
        L.orc_aggregate_tiles.restype = None
        L.orc_aggregate_tiles.argtypes = [C.c_int, C.c_int, I32P, I32P, U8P, U8P, C.c_int, C.c_int, C.c_int,
                                          C.c_int, C.c_int, I32P, I32P, I32P]
        L.orc_galerkin.restype = C.c_int
        L.orc_galerkin.argtypes = [C.c_int, C.c_int, I32P, I32P, F64P, I32P, C.c_int, I32P, C.c_void_p,
                                   C.c_void_p]
        L.orc_colour.restype = C.c_int
        L.orc_colour.argtypes = [C.c_int, C.c_int, I32P, I32P, C.c_int, C.c_uint32, I32P]
        L.orc_fmix32.restype = C.c_uint32
        L.orc_fmix32.argtypes = [C.c_uint32]
        L.orc_cholesky.restype = C.c_int
        L.orc_cholesky.argtypes = [C.c_int, F64P, F64P]
        L.orc_mcsgs.restype = None
        L.orc_mcsgs.argtypes = [C.c_int, C.c_int, I32P, I32P, F64P, I32P, C.c_int, F64P, F64P]
        L.orc_hybrid_sgs.restype = None
        L.orc_hybrid_sgs.argtypes = [C.c_int, C.c_int, I32P, I32P, F64P, C.c_int, F64P, F64P, C.c_void_p]
        L.orc_setup.restype = C.c_void_p
        L.orc_setup.argtypes = [C.c_int, C.c_int, I32P, I32P, F64P, C.POINTER(Params), C.POINTER(C.c_int)]
        L.orc_free.restype = None
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_num_levels.restype = C.c_int
        L.orc_num_levels.argtypes = [C.c_void_p]
        L.orc_level_info.restype = None
        L.orc_level_info.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int)]
        L.orc_copy_level.restype = None
        L.orc_copy_level.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 7
        L.orc_coarse_factor.restype = None
        L.orc_coarse_factor.argtypes = [C.c_void_p, F64P]
        L.orc_vcycle.restype = None
        L.orc_vcycle.argtypes = [C.c_void_p, F64P, F64P]
        L.orc_smooth.restype = None
        L.orc_smooth.argtypes = [C.c_void_p, C.c_int, C.c_int, F64P, F64P]
        L.orc_pcg.restype = C.c_int
        L.orc_pcg.argtypes = [C.c_void_p, F64P, F64P, C.c_double, C.c_int, C.POINTER(C.c_int), C.c_void_p,
                              C.c_void_p, C.POINTER(C.c_double)]
        L.orc_bicgstab.restype = C.c_int
        L.orc_bicgstab.argtypes = [C.c_void_p, F64P, F64P, C.c_double, C.c_int, C.POINTER(C.c_int),
                                   C.POINTER(C.c_int), C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
        L.orc_bicgstab_plain.restype = C.c_int
        L.orc_bicgstab_plain.argtypes = [C.c_int, C.c_int, I32P, I32P, F64P, F64P, F64P, C.c_double, C.c_int,
                                         C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_void_p, C.c_void_p,
                                         C.POINTER(C.c_double)]
        _LIB = L
    return _LIB


def _csr(rowptr, colind, vals=None):
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.float64)
    return rp, ci, v


def validate(rowptr, colind, vals, check_symmetry=True) -> int:
    rp, ci, v = _csr(rowptr, colind, vals)
    return lib().orc_validate(rp.shape[0] - 1, ci.shape[0], rp, ci, v, int(check_symmetry))


def strength(rowptr, colind, vals, tile_rows=128, delta=0.08, beta=1e-5):
    """Strong flag per stored entry and isolated flag per row (Sec. 2.1)."""
    rp, ci, v = _csr(rowptr, colind, vals)
    n, nnz = rp.shape[0] - 1, ci.shape[0]
    strong = np.zeros(nnz, np.uint8)
    iso = np.zeros(n, np.uint8)
    lib().orc_strength(n, nnz, rp, ci, v, tile_rows, delta, beta, strong, iso)
    return strong, iso


def aggregate(rowptr, colind, strong, iso, tile_rows=128, smin=8, smax=12, dmax=3):
    """Global aggregate id per row, number of aggregates, per-tile counts (Alg. 1-4)."""
    rp, ci, _ = _csr(rowptr, colind)
    n, nnz = rp.shape[0] - 1, ci.shape[0]
    agg = np.zeros(n, np.int32)
    tc = np.zeros((n + tile_rows - 1) // tile_rows, np.int32)
    nc = lib().orc_aggregate(n, nnz, rp, ci, np.ascontiguousarray(strong, np.uint8),
                             np.ascontiguousarray(iso, np.uint8), tile_rows, smin, smax, dmax, agg, tc)
    return agg, nc, tc


def aggregate_tiles(rowptr, colind, strong, iso, tiles, tile_rows=128, smin=8, smax=12, dmax=3):
    """Tile-local aggregate ids for the rows of the given tiles (others -1) and their counts."""
    rp, ci, _ = _csr(rowptr, colind)
    n, nnz = rp.shape[0] - 1, ci.shape[0]
    tiles = np.ascontiguousarray(tiles, np.int32)
    loc = np.full(n, -1, np.int32)
    cnt = np.zeros(tiles.shape[0], np.int32)
    lib().orc_aggregate_tiles(n, nnz, rp, ci, np.ascontiguousarray(strong, np.uint8),
                              np.ascontiguousarray(iso, np.uint8), tile_rows, smin, smax, dmax,
                              tiles.shape[0], tiles, loc, cnt)
    return loc, cnt


def galerkin(rowptr, colind, vals, agg, nc):
    """Coarse CSR of P^T A P with the ordered summation (Sec. 2.1)."""
    rp, ci, v = _csr(rowptr, colind, vals)
    n, nnz = rp.shape[0] - 1, ci.shape[0]
    a = np.ascontiguousarray(agg, np.int32)
    cptr = np.zeros(nc + 1, np.int32)
    L = lib()
    cnnz = L.orc_galerkin(n, nnz, rp, ci, v, a, nc, cptr, None, None)
    ccol = np.zeros(cnnz, np.int32)
    cval = np.zeros(cnnz, np.float64)
    L.orc_galerkin(n, nnz, rp, ci, v, a, nc, cptr, ccol.ctypes.data, cval.ctypes.data)
    return cptr, ccol, cval


def colour(rowptr, colind, seed=0, tile_rows=128):
    """Tile-ordered greedy colouring: colour per row and number of colours."""
    rp, ci, _ = _csr(rowptr, colind)
    n = rp.shape[0] - 1
    c = np.zeros(n, np.int32)
    k = lib().orc_colour(n, ci.shape[0], rp, ci, tile_rows, seed & 0xFFFFFFFF, c)
    return c, k


def fmix32(h: int) -> int:
    return int(lib().orc_fmix32(h & 0xFFFFFFFF))


def cholesky(A: np.ndarray):
    A = np.ascontiguousarray(A, np.float64)
    n = A.shape[0]
    L = np.zeros_like(A)
    st = lib().orc_cholesky(n, A.ravel(), L.ravel())
    return st, L.reshape(n, n)


def mcsgs(rowptr, colind, vals, col, ncol, b, x):
    rp, ci, v = _csr(rowptr, colind, vals)
    x = np.ascontiguousarray(x, np.float64).copy()
    lib().orc_mcsgs(rp.shape[0] - 1, ci.shape[0], rp, ci, v, np.ascontiguousarray(col, np.int32), ncol,
                    np.ascontiguousarray(b, np.float64), x)
    return x


def hybrid_sgs(rowptr, colind, vals, tile_rows, b, x, colour=None):
    """One hybrid SGS step (block-Jacobi over tiles of tile_rows rows, SGS
    inside); with `colour`, each tile's rows are swept in (colour, row) order."""
    rp, ci, v = _csr(rowptr, colind, vals)
    x = np.ascontiguousarray(x, np.float64).copy()
    col = None if colour is None else np.ascontiguousarray(colour, np.int32)
    lib().orc_hybrid_sgs(rp.shape[0] - 1, ci.shape[0], rp, ci, v, tile_rows, np.ascontiguousarray(b, np.float64), x,
                         None if col is None else col.ctypes.data)
    return x


@dataclass
class LevelData:
    n: int
    nnz: int
    ncol: int
    rowptr: np.ndarray
    colind: np.ndarray
    vals: np.ndarray
    agg: np.ndarray | None
    colour: np.ndarray
    strong: np.ndarray | None
    iso: np.ndarray | None


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


class Hierarchy:
    """Oracle AMG hierarchy: setup, V-cycle, PCG/FCG."""

    def __init__(self, rowptr, colind, vals, **params):
        rp, ci, v = _csr(rowptr, colind, vals)
        self.params = default_params(**params)
        st = C.c_int(0)
        self._h = lib().orc_setup(rp.shape[0] - 1, ci.shape[0], rp, ci, v, C.byref(self.params), C.byref(st))
        if not self._h:
            raise OracleError(st.value)
        self.n = rp.shape[0] - 1

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def levels(self) -> int:
        return lib().orc_num_levels(self._h)

    def level(self, l: int) -> LevelData:
        n, nnz, nc = C.c_int(), C.c_int(), C.c_int()
        lib().orc_level_info(self._h, l, C.byref(n), C.byref(nnz), C.byref(nc))
        n, nnz = n.value, nnz.value
        last = l == self.levels - 1
        agg = None if last else np.zeros(n, np.int32)
        col = np.zeros(n, np.int32)
        rp = np.zeros(n + 1, np.int32)
        ci = np.zeros(nnz, np.int32)
        v = np.zeros(nnz, np.float64)
        bs = max(1, int(self.params.block_size))
        strong = None if last else np.zeros(nnz // (bs * bs), np.uint8)  # node graph when bs > 1
        iso = None if last else np.zeros(n // bs, np.uint8)

        def p(a):
            return None if a is None else a.ctypes.data

        lib().orc_copy_level(self._h, l, p(agg), p(col), p(rp), p(ci), p(v), p(strong), p(iso))
        return LevelData(n, nnz, nc.value, rp, ci, v, agg, col, strong, iso)

    def coarse_factor(self) -> np.ndarray:
        nL = self.level(self.levels - 1).n
        L = np.zeros(nL * nL, np.float64)
        lib().orc_coarse_factor(self._h, L)
        return L.reshape(nL, nL)

    def vcycle(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros(self.n, np.float64)
        lib().orc_vcycle(self._h, np.ascontiguousarray(r, np.float64), z)
        return z

    def smooth(self, l: int, b: np.ndarray, x: np.ndarray, fp32: bool = False) -> np.ndarray:
        """One application of level l's smoother to a copy of x."""
        x = np.ascontiguousarray(x, np.float64).copy()
        lib().orc_smooth(self._h, l, int(fp32), np.ascontiguousarray(b, np.float64), x)
        return x

    def pcg(self, b, x0=None, rtol=1e-8, maxit=1000, keep_iterates=False):
        n = self.n
        x = np.zeros(n) if x0 is None else np.array(x0, np.float64)
        res = np.zeros(maxit + 1, np.float64)
        hist = np.zeros((maxit + 1) * n, np.float64) if keep_iterates else None
        it = C.c_int(0)
        tr = C.c_double(0.0)
        st = lib().orc_pcg(self._h, np.ascontiguousarray(b, np.float64), x, rtol, maxit, C.byref(it),
                           res.ctypes.data, None if hist is None else hist.ctypes.data, C.byref(tr))
        k = it.value
        out = dict(status=st, x=x, iterations=k, res_hist=res[:k + 1], true_rel_residual=tr.value)
        if hist is not None:
            out["iterates"] = hist[:(k + 1) * n].reshape(k + 1, n)
        return out

    def bicgstab(self, b, x0=None, rtol=1e-8, maxit=1000, keep_iterates=False):
        """BiCGSTAB preconditioned by one V-cycle (Sec. 5); see _bicgstab_result."""
        def call(x, res, hist, it, half, tr):
            return lib().orc_bicgstab(self._h, np.ascontiguousarray(b, np.float64), x, rtol, maxit, C.byref(it),
                                      C.byref(half), res, hist, C.byref(tr))
        return _bicgstab_result(call, self.n, x0, maxit, keep_iterates)


def _bicgstab_result(call, n, x0, maxit, keep_iterates):
    """Runs an oracle BiCGSTAB; iterations k stopped in (half = 1: at the half
    step, x = x_{k-1} + alpha M p), res_hist[0..k], iterates x_0..x_k."""
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64)
    res = np.zeros(maxit + 1, np.float64)
    hist = np.zeros((maxit + 1) * n, np.float64) if keep_iterates else None
    it, half, tr = C.c_int(0), C.c_int(0), C.c_double(0.0)
    st = call(x, res.ctypes.data, None if hist is None else hist.ctypes.data, it, half, tr)
    k = it.value
    out = dict(status=st, x=x, iterations=k, half=half.value, res_hist=res[:k + 1], true_rel_residual=tr.value)
    if hist is not None:
        out["iterates"] = hist[:(k + 1) * n].reshape(k + 1, n)
    return out


def bicgstab_plain(rowptr, colind, vals, b, x0=None, rtol=1e-8, maxit=1000, keep_iterates=False):
    """Unpreconditioned BiCGSTAB on any square CSR matrix (the iteration alone)."""
    rp, ci, v = _csr(rowptr, colind, vals)
    n = rp.shape[0] - 1

    def call(x, res, hist, it, half, tr):
        return lib().orc_bicgstab_plain(n, ci.shape[0], rp, ci, v, np.ascontiguousarray(b, np.float64), x, rtol,
                                        maxit, C.byref(it), C.byref(half), res, hist, C.byref(tr))
    return _bicgstab_result(call, n, x0, maxit, keep_iterates)
