"""ctypes binding of the C interface declared in include/amg.h.

Argument marshalling only: every step of setup and solve runs in the HIP
library libamg_mi355x.so.  PyTorch supplies device memory (tensors) and the
stream; the functions keep the C names (amg_setup, amg_precond_apply,
pcg_solve, amg_free).  The library must be built (python -m
paper_1209_0960_amd.build); a missing library raises instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch  # loaded first so that the library binds to torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamg_mi355x.so")

OK = 0
STATUS = {0: "AMG_OK", 1: "AMG_ERR_INVALID_ARG", 2: "AMG_ERR_BAD_DIAGONAL", 3: "AMG_ERR_NOT_SYMMETRIC",
          4: "AMG_ERR_NOT_SPD", 5: "AMG_ERR_COARSENING_STALLED", 6: "AMG_ERR_OUT_OF_MEMORY",
          7: "AMG_ERR_BREAKDOWN", 8: "AMG_ERR_NOT_CONVERGED", 9: "AMG_ERR_HIP", 10: "AMG_ERR_UNSUPPORTED"}
ERR_INVALID_ARG, ERR_BAD_DIAGONAL, ERR_NOT_SYMMETRIC, ERR_NOT_SPD = 1, 2, 3, 4
ERR_COARSENING_STALLED, ERR_OUT_OF_MEMORY, ERR_BREAKDOWN, ERR_NOT_CONVERGED = 5, 6, 7, 8
ERR_HIP, ERR_UNSUPPORTED = 9, 10
SMOOTHER_MCSGS, SMOOTHER_L1_JACOBI, SMOOTHER_HYBRID_SGS, SMOOTHER_TILE_MCSGS = 0, 1, 2, 3
KIND_SPMV_F64, KIND_SWEEP, KIND_RESTRICT, KIND_PROLONG, KIND_CG_VEC, KIND_COARSE_LEVELS, KIND_OTHER = range(7)


class AMGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("strength_threshold", C.c_double), ("isolated_threshold", C.c_double),
                ("agg_min", C.c_int32), ("agg_max", C.c_int32), ("agg_diameter", C.c_int32),
                ("omega", C.c_double), ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
                ("tile_rows", C.c_int32), ("smoother", C.c_int32), ("pre_sweeps", C.c_int32),
                ("post_sweeps", C.c_int32), ("vcycle_fp32", C.c_int32), ("flexible", C.c_int32),
                ("colour_seed", C.c_uint32), ("check_symmetry", C.c_int32), ("keep_setup_data", C.c_int32),
                ("use_graphs", C.c_int32), ("tail_rows", C.c_int32),
                ("colour_tile_rows", C.c_int32), ("block_size", C.c_int32), ("spmv_format", C.c_int32),
                ("coarse_smoother", C.c_int32), ("coarse_from", C.c_int32),
                ("smooth_tile_rows", C.c_int32), ("coarse_smooth_tile_rows", C.c_int32)]


class CSR(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("vals", C.c_void_p)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("levels", C.c_int32),
                ("rel_residual", C.c_double), ("true_rel_residual", C.c_double), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

_LIB = None


def lib():
    """Load libamg_mi355x.so (raises if it was not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run python -m paper_1209_0960_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, i32, st = C.c_void_p, C.c_int32, C.c_int
        L.amg_default_params.restype = st
        L.amg_default_params.argtypes = [C.POINTER(Params)]
        L.amg_setup.restype = st
        L.amg_setup.argtypes = [C.POINTER(CSR), C.POINTER(Params), vp, C.POINTER(vp)]
        L.amg_precond_apply.restype = st
        L.amg_precond_apply.argtypes = [vp, vp, vp, vp]
        L.amg_precond_apply_noalloc.restype = st
        L.amg_precond_apply_noalloc.argtypes = [vp, vp, vp, vp]
        L.pcg_solve.restype = st
        L.pcg_solve.argtypes = [vp, vp, vp, C.c_double, i32, C.POINTER(SolveInfo), vp, vp, vp]
        L.bicgstab_solve.restype = st
        L.bicgstab_solve.argtypes = [vp, vp, vp, C.c_double, i32, C.POINTER(SolveInfo), C.POINTER(i32), vp, vp,
                                     vp]
        L.amg_free.restype = None
        L.amg_free.argtypes = [vp]
        L.amg_status_string.restype = C.c_char_p
        L.amg_status_string.argtypes = [st]
        L.amg_last_error.restype = C.c_char_p
        L.amg_last_error.argtypes = []
        L.amg_release_cached_memory.restype = st
        L.amg_release_cached_memory.argtypes = []
        L.amg_set_allocator.restype = st
        L.amg_set_allocator.argtypes = [vp, vp, vp]
        L.amg_hierarchy_bytes.restype = st
        L.amg_hierarchy_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.amg_num_levels.restype = st
        L.amg_num_levels.argtypes = [vp, C.POINTER(i32)]
        L.amg_level_info.restype = st
        L.amg_level_info.argtypes = [vp, i32] + [C.POINTER(i32)] * 4
        L.amg_copy_level.restype = st
        L.amg_copy_level.argtypes = [vp, i32] + [vp] * 7
        L.amg_set_kernel_timing.restype = st
        L.amg_set_kernel_timing.argtypes = [i32]
        L.amg_get_kernel_timing.restype = st
        L.amg_get_kernel_timing.argtypes = [i32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                            C.POINTER(C.c_double)]
        L.amg_reset_kernel_timing.restype = st
        L.amg_reset_kernel_timing.argtypes = []
        L.amg_setup_batched.restype = st
        L.amg_setup_batched.argtypes = [C.POINTER(CSR), i32, C.POINTER(Params), vp, C.POINTER(vp)]
        L.pcg_solve_batched.restype = st
        L.pcg_solve_batched.argtypes = [C.POINTER(vp), i32, i32, C.POINTER(vp), C.POINTER(vp), C.c_double, i32,
                                        C.POINTER(SolveInfo), vp]
        L.amg_estimate_bytes.restype = st
        L.amg_estimate_bytes.argtypes = [i32, i32, C.POINTER(Params), i32] + [C.POINTER(C.c_size_t)] * 3
        L.amg_batch_create.restype = st
        L.amg_batch_create.argtypes = [i32, i32, i32, C.POINTER(vp)]
        L.amg_batch_submit.restype = st
        L.amg_batch_submit.argtypes = [vp, vp, vp, vp, C.c_double, i32, C.c_int64, vp]
        L.amg_batch_step.restype = st
        L.amg_batch_step.argtypes = [vp, i32]
        L.amg_batch_poll.restype = st
        L.amg_batch_poll.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(SolveInfo), i32,
                                     C.POINTER(i32)]
        L.amg_batch_active.restype = st
        L.amg_batch_active.argtypes = [vp, C.POINTER(i32)]
        L.amg_batch_bytes.restype = st
        L.amg_batch_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.amg_batch_free.restype = None
        L.amg_batch_free.argtypes = [vp]
        _LIB = L
    return _LIB


def _check(status: int):
    if status != OK:
        raise AMGError(status, lib().amg_last_error().decode())


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def default_params(**kw) -> Params:
    p = Params()
    _check(lib().amg_default_params(C.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def amg_setup(rowptr: torch.Tensor, colind: torch.Tensor, vals: torch.Tensor, params: Params | None = None,
              stream=None) -> C.c_void_p:
    """amg_setup on device CSR tensors (int32, int32, float64); returns the handle."""
    if rowptr.dtype != torch.int32 or colind.dtype != torch.int32 or vals.dtype != torch.float64:
        raise TypeError("CSR must be int32/int32/float64")
    A = CSR(rowptr.numel() - 1, colind.numel(), _ptr(rowptr), _ptr(colind), _ptr(vals))
    p = params if params is not None else default_params()
    h = C.c_void_p()
    _check(lib().amg_setup(C.byref(A), C.byref(p), _stream(stream), C.byref(h)))
    return h


def _csr(rowptr, colind, vals) -> CSR:
    if rowptr.dtype != torch.int32 or colind.dtype != torch.int32 or vals.dtype != torch.float64:
        raise TypeError("CSR must be int32/int32/float64")
    return CSR(rowptr.numel() - 1, colind.numel(), _ptr(rowptr), _ptr(colind), _ptr(vals))


def amg_setup_batched(systems, params: Params | None = None, stream=None) -> list:
    """amg_setup_batched over a list of (rowptr, colind, vals) device tensors; returns the handles."""
    arr = (CSR * len(systems))(*[_csr(*s) for s in systems])
    out = (C.c_void_p * len(systems))()
    p = params if params is not None else default_params()
    _check(lib().amg_setup_batched(arr, len(systems), C.byref(p), _stream(stream), out))
    return [C.c_void_p(h) for h in out]


def pcg_solve_batched(handles, bs, xs, nrhs: int = 1, rtol: float = 1e-8, maxit: int = 1000, stream=None):
    """pcg_solve_batched: bs[s], xs[s] hold nrhs * n_s values (right-hand side k
    at k * n_s).  Returns (status, list of nsys lists of nrhs info dicts)."""
    ns = len(handles)
    hs = (C.c_void_p * ns)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    bp = (C.c_void_p * ns)(*[b.data_ptr() for b in bs])
    xp = (C.c_void_p * ns)(*[x.data_ptr() for x in xs])
    for t in list(bs) + list(xs):
        _ptr(t)
    info = (SolveInfo * (ns * nrhs))()
    st = lib().pcg_solve_batched(hs, ns, nrhs, bp, xp, rtol, maxit, info, _stream(stream))
    if st not in (OK, ERR_NOT_CONVERGED):
        _check(st)
    return st, [[_info_dict(info[s * nrhs + k]) for k in range(nrhs)] for s in range(ns)]


def estimate_bytes(n: int, nnz: int, params: Params | None = None, nrhs: int = 1) -> dict:
    """amg_estimate_bytes: dict(setup_peak, hierarchy, context) in bytes."""
    p = params if params is not None else default_params()
    a, b, c = C.c_size_t(), C.c_size_t(), C.c_size_t()
    _check(lib().amg_estimate_bytes(n, nnz, C.byref(p), nrhs, C.byref(a), C.byref(b), C.byref(c)))
    return dict(setup_peak=a.value, hierarchy=b.value, context=c.value)


def _info_dict(i: SolveInfo) -> dict:
    return dict(iterations=i.iterations, converged=bool(i.converged), levels=i.levels, rel_residual=i.rel_residual,
                true_rel_residual=i.true_rel_residual, setup_ms=i.setup_ms, solve_ms=i.solve_ms)


class Batch:
    """Continuous batching of CG solves (amg_batch_*): submit, step, poll."""

    def __init__(self, nrhs: int = 1, max_entries: int = 64, use_graphs: bool = True):
        self.nrhs = nrhs
        self.b = C.c_void_p()
        _check(lib().amg_batch_create(nrhs, max_entries, 1 if use_graphs else 0, C.byref(self.b)))

    def submit(self, h, rhs: torch.Tensor, x: torch.Tensor, rtol=1e-8, maxit=1000, tag=0, stream=None):
        hh = h.h if isinstance(h, Hierarchy) else h
        _check(lib().amg_batch_submit(self.b, hh, _ptr(rhs), _ptr(x), rtol, maxit, tag, _stream(stream)))

    def step(self, iterations: int = 1):
        _check(lib().amg_batch_step(self.b, iterations))

    def poll(self, cap: int = 256) -> list:
        tags = (C.c_int64 * cap)()
        sts = (C.c_int * cap)()
        info = (SolveInfo * (cap * self.nrhs))()
        cnt = C.c_int32()
        _check(lib().amg_batch_poll(self.b, tags, sts, info, cap, C.byref(cnt)))
        return [(tags[i], sts[i], [_info_dict(info[i * self.nrhs + k]) for k in range(self.nrhs)])
                for i in range(cnt.value)]

    @property
    def active(self) -> int:
        a = C.c_int32()
        _check(lib().amg_batch_active(self.b, C.byref(a)))
        return a.value

    @property
    def bytes(self) -> int:
        v = C.c_size_t()
        _check(lib().amg_batch_bytes(self.b, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "b", None):
            try:
                lib().amg_batch_free(self.b)
            except TypeError:
                pass
            self.b = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def amg_precond_apply(h, r: torch.Tensor, z: torch.Tensor, stream=None):
    _check(lib().amg_precond_apply(h, _ptr(r), _ptr(z), _stream(stream)))


def amg_precond_apply_noalloc(h, r: torch.Tensor, z: torch.Tensor, stream=None):
    _check(lib().amg_precond_apply_noalloc(h, _ptr(r), _ptr(z), _stream(stream)))


@dataclass
class SolveResult:
    status: int
    iterations: int
    converged: bool
    levels: int
    rel_residual: float
    true_rel_residual: float
    setup_ms: float
    solve_ms: float
    res_hist: np.ndarray
    half_step: int = 0  # BiCGSTAB: stopped at the half step of the last iteration


def pcg_solve(h, b: torch.Tensor, x: torch.Tensor, rtol: float = 1e-8, maxit: int = 1000,
              iter_hist: torch.Tensor | None = None, stream=None, raise_on_error: bool = True) -> SolveResult:
    """pcg_solve: x holds x0 on entry and the solution on return."""
    info = SolveInfo()
    res = np.zeros(maxit + 1, np.float64)
    st = lib().pcg_solve(h, _ptr(b), _ptr(x), rtol, maxit, C.byref(info), res.ctypes.data_as(C.c_void_p),
                         _ptr(iter_hist), _stream(stream))
    if st not in (OK, ERR_NOT_CONVERGED) and raise_on_error:
        _check(st)
    k = info.iterations
    return SolveResult(st, k, bool(info.converged), info.levels, info.rel_residual, info.true_rel_residual,
                       info.setup_ms, info.solve_ms, res[:k + 1].copy())


def bicgstab_solve(h, b: torch.Tensor, x: torch.Tensor, rtol: float = 1e-8, maxit: int = 1000,
                   iter_hist: torch.Tensor | None = None, stream=None, raise_on_error: bool = True):
    """bicgstab_solve: x holds x0 on entry and the solution on return."""
    info = SolveInfo()
    half = C.c_int32(0)
    res = np.zeros(maxit + 1, np.float64)
    st = lib().bicgstab_solve(h, _ptr(b), _ptr(x), rtol, maxit, C.byref(info), C.byref(half),
                              res.ctypes.data_as(C.c_void_p), _ptr(iter_hist), _stream(stream))
    if st not in (OK, ERR_NOT_CONVERGED) and raise_on_error:
        _check(st)
    k = info.iterations
    return SolveResult(st, k, bool(info.converged), info.levels, info.rel_residual, info.true_rel_residual,
                       info.setup_ms, info.solve_ms, res[:k + 1].copy(), half.value)


def amg_free(h):
    if h:
        lib().amg_free(h)


def set_allocator(alloc, free, ctx=None):
    """Install ctypes callbacks (ALLOC_FN/FREE_FN) or None to restore the default."""
    _check(lib().amg_set_allocator(C.cast(alloc, C.c_void_p) if alloc else None,
                                   C.cast(free, C.c_void_p) if free else None, ctx))


def release_cached_memory():
    """amg_release_cached_memory: hand the library's cached free blocks back to the device."""
    _check(lib().amg_release_cached_memory())


def set_kernel_timing(kinds=True):
    """kinds: True (all), False (none) or an iterable of KIND_* values."""
    if kinds is True:
        mask = -1
    elif kinds is False or kinds is None:
        mask = 0
    else:
        mask = 0
        for k in kinds:
            mask |= 1 << k
    _check(lib().amg_set_kernel_timing(mask))


def reset_kernel_timing():
    _check(lib().amg_reset_kernel_timing())


def kernel_timing(kind: int):
    ms, n, by = C.c_double(), C.c_int64(), C.c_double()
    _check(lib().amg_get_kernel_timing(kind, C.byref(ms), C.byref(n), C.byref(by)))
    return ms.value, n.value, by.value


class Hierarchy:
    """Owning wrapper of an amg_hierarchy handle."""

    def __init__(self, rowptr, colind, vals, stream=None, **params):
        self.params = default_params(**params)
        self.n = rowptr.numel() - 1
        self.h = amg_setup(rowptr, colind, vals, self.params, stream)

    @classmethod
    def batched(cls, systems, stream=None, **params) -> list:
        """amg_setup_batched over [(rowptr, colind, vals), ...]."""
        p = default_params(**params)
        hs = amg_setup_batched(systems, p, stream)
        out = []
        for (rp, _, _), h in zip(systems, hs):
            o = cls.__new__(cls)
            o.params, o.n, o.h = p, rp.numel() - 1, h
            out.append(o)
        return out

    def close(self):
        if getattr(self, "h", None):
            try:
                amg_free(self.h)
            except TypeError:  # interpreter shutdown: module globals already cleared
                pass
            self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def levels(self) -> int:
        k = C.c_int32()
        _check(lib().amg_num_levels(self.h, C.byref(k)))
        return k.value

    @property
    def bytes(self) -> int:
        b = C.c_size_t()
        _check(lib().amg_hierarchy_bytes(self.h, C.byref(b)))
        return b.value

    def level_info(self, l: int):
        n, nnz, nc, nn = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().amg_level_info(self.h, l, C.byref(n), C.byref(nnz), C.byref(nc), C.byref(nn)))
        return dict(n=n.value, nnz=nnz.value, ncolours=nc.value, n_next=nn.value)

    def level(self, l: int) -> dict:
        """Host copies of level l (agg, colour, CSR, strong/iso when kept)."""
        info = self.level_info(l)
        n, nnz = info["n"], info["nnz"]
        out = dict(info)
        out["agg"] = np.zeros(n, np.int32) if info["n_next"] > 0 else None
        out["colour"] = np.zeros(n, np.int32)
        out["rowptr"] = np.zeros(n + 1, np.int32)
        out["colind"] = np.zeros(nnz, np.int32)
        out["vals"] = np.zeros(nnz, np.float64)
        keep = bool(self.params.keep_setup_data) and info["n_next"] > 0
        bs = max(1, int(self.params.block_size))  # node graph flags on point-based levels
        out["strong"] = np.zeros(nnz // (bs * bs), np.uint8) if keep else None
        out["iso"] = np.zeros(n // bs, np.uint8) if keep else None

        def p(a):
            return None if a is None else a.ctypes.data_as(C.c_void_p)

        _check(lib().amg_copy_level(self.h, l, p(out["agg"]), p(out["colour"]), p(out["rowptr"]),
                                    p(out["colind"]), p(out["vals"]), p(out["strong"]), p(out["iso"])))
        return out

    def precond(self, r: torch.Tensor, z: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if z is None:
            z = torch.empty_like(r)
        amg_precond_apply(self.h, r, z, stream)
        return z

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, rtol=1e-8, maxit=1000, iter_hist=None,
              stream=None, raise_on_error=True, method="cg") -> tuple:
        """method "cg": pcg_solve; "bicgstab": bicgstab_solve."""
        if x is None:
            x = torch.zeros_like(b)
        if method == "bicgstab":
            return x, bicgstab_solve(self.h, b, x, rtol, maxit, iter_hist, stream, raise_on_error)
        if method != "cg":
            raise ValueError(f"unknown method {method!r}")
        r = pcg_solve(self.h, b, x, rtol, maxit, iter_hist, stream, raise_on_error)
        return x, r


def to_device(system, device="cuda"):
    """Copy a problems.CSRSystem to device tensors (rowptr, colind, vals, b)."""
    return (torch.from_numpy(system.rowptr).to(device), torch.from_numpy(system.colind).to(device),
            torch.from_numpy(system.vals).to(device), torch.from_numpy(np.ascontiguousarray(system.b)).to(device))
