"""The C-ABI library loads on the host and exports every entry point that
include/za.h declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "za.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(za_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("za_rhs", "za_rhs_fluxes", "za_step", "za_solve", "za_ctx_create", "za_ctx_destroy",
                 "za_server_create", "za_server_submit", "za_server_poll", "za_server_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2603_26272_amd import za
    lib = ctypes.CDLL(za.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(za.EXPORTED) >= set(declared_functions())


def test_host_only_calls():
    """Calls that need no device: sizes and status strings."""
    from paper_2603_26272_amd import za
    from paper_2603_26272_amd.problem import Problem
    P = Problem(dim=2, nx=100, ny=50)
    assert za.state_count(P) == 4 * 100 * 50
    assert za.workspace_bytes(P) >= 3 * 4 * 100 * 50 * 8
    assert za.state_count(Problem(dim=3)) == 0
    assert za.status_str(0) == "ok" and za.status_str(4).startswith("non-finite")
