"""The C-ABI library loads and exports every entry point include/ep.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "ep.h")).read()
    return re.findall(r"EP_API\s+[\w\s\*]+?\b(ep_\w+)\s*\(", src)


def test_header_declares_the_boundary():
    names = set(declared())
    for core in ("ep_create_grid", "ep_set_conductivity_fibres", "ep_step",
                 "ep_solve_elliptic", "ep_read_state"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2302_12519_amd import ep
    lib = ctypes.CDLL(ep.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    from paper_2302_12519_amd import ep
    assert ep.lib.ep_status_string(0) == b"EP_OK"
    assert ep.lib.ep_status_string(4) == b"EP_ERR_NOCONV"
    # NULL arguments are rejected before any device work
    assert ep.lib.ep_create_grid(None, None) == ep.EP_ERR_ARG
    assert ep.lib.ep_step(None, 1, None) == ep.EP_ERR_ARG
