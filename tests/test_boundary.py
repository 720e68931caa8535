"""CPU checks of the C-ABI boundary: the built library loads and exports every
function include/amg.h declares (no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amg.h")
LIB = os.path.join(ROOT, "paper_1209_0960_amd", "libamg_mi355x.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"AMG_API\s+[\w\s\*]+?\b(\w+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared()
    for fn in ("amg_setup", "amg_precond_apply", "pcg_solve", "bicgstab_solve", "amg_free"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("HIP library not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_params_struct_matches_header_defaults():
    """amg_default_params runs on the host only: compare with the documented defaults."""
    if not os.path.exists(LIB):
        pytest.skip("HIP library not built")
    from paper_1209_0960_amd import amg as A
    p = A.default_params()
    assert (p.strength_threshold, p.isolated_threshold, p.agg_min, p.agg_max, p.agg_diameter) == (0.08, 1e-5, 8, 12, 3)
    assert (p.omega, p.coarse_max, p.max_levels, p.tile_rows) == (1.6, 500, 25, 128)
    assert (p.smoother, p.pre_sweeps, p.post_sweeps, p.vcycle_fp32, p.flexible) == (0, 1, 1, 0, -1)
    assert p.use_graphs == 1
    assert p.tail_rows == 0
    assert ctypes.sizeof(A.Params) == 120  # 3 doubles + 22 int32 fields (4 bytes of padding before omega), 8-byte aligned
    assert p.block_size == 1
    assert (p.coarse_smoother, p.coarse_from) == (-1, 1)
    assert (p.smooth_tile_rows, p.coarse_smooth_tile_rows) == (0, 0)


def test_header_compiles_as_c_and_matches_ctypes_layout(tmp_path):
    """The public header is plain C; the binding's structs have its layout."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "amg.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(amg_params), sizeof(amg_solve_info),'
                   ' sizeof(amg_csr), offsetof(amg_params, use_graphs), offsetof(amg_params, coarse_smooth_tile_rows));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    sizes = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    from paper_1209_0960_amd import amg as A
    assert sizes == [ctypes.sizeof(A.Params), ctypes.sizeof(A.SolveInfo), ctypes.sizeof(A.CSR),
                     A.Params.use_graphs.offset, A.Params.coarse_smooth_tile_rows.offset]


def test_bicgstab_and_hybrid_host_checks():
    """Host-only paths of the new calls: bicgstab_solve rejects a NULL
    hierarchy and bad arguments before touching the device; the footprint
    estimate counts the hybrid smoother's per-row steps."""
    if not os.path.exists(LIB):
        pytest.skip("HIP library not built")
    from paper_1209_0960_amd import amg as A
    L = A.lib()
    assert L.bicgstab_solve(None, None, None, 1e-8, 10, None, None, None, None, None) == A.ERR_INVALID_ARG
    p = A.default_params()
    sizes = []
    for smoother in (A.SMOOTHER_MCSGS, A.SMOOTHER_HYBRID_SGS):
        p.smoother = smoother
        hier = ctypes.c_size_t(0)
        assert L.amg_estimate_bytes(1000000, 7000000, ctypes.byref(p), 1, None, ctypes.byref(hier), None) == A.OK
        sizes.append(hier.value)
    assert sizes[1] > sizes[0]
