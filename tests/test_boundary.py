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
    for fn in ("amg_setup", "amg_precond_apply", "pcg_solve", "amg_free"):
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
    assert (p.omega, p.coarse_max, p.max_levels, p.tile_rows) == (1.6, 500, 25, 512)
    assert (p.smoother, p.pre_sweeps, p.post_sweeps, p.vcycle_fp32, p.flexible) == (0, 1, 1, 0, -1)
    assert ctypes.sizeof(A.Params) == 88
