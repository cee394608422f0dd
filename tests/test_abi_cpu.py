"""CPU-side checks of the C-ABI library: it loads, exports every entry point that
include/fdw.h declares, and its pure host-side validation rejects bad problems (no GPU
calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdw.h")
LIB = os.path.join(ROOT, "paper_2005_11931_amd", "_lib", "libfdw.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fdw_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2005_11931_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fdw_init", "fdw_set_coeff", "fdw_step_n", "fdw_adjoint", "fdw_energy"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    import importlib

    fdw = importlib.import_module("paper_2005_11931_amd.fdw")
    assert sorted(fdw.EXPORTED) == _declared()


def test_host_validation(lib):
    from paper_2005_11931_amd import fdw

    ws = lib.fdw_workspace_bytes
    ws.restype = ctypes.c_size_t
    ws.argtypes = [ctypes.POINTER(fdw.fdw_problem), ctypes.c_int32]
    good = fdw.problem(64, 48, 1e-3, 100, fdw.FDW_F32)
    assert ws(ctypes.byref(good), 1) > 0
    for bad in (
        fdw.problem(2, 48, 1e-3, 100),            # nx < 3
        fdw.fdw_problem(64, 48, -1, 1, -1, 1, 0.0, 0.0, 1, 0),    # tau = 0
        fdw.fdw_problem(64, 48, -1, 1, -1, 1, 1e-3, 0.10005, 1, 0),  # T/tau not an integer
        fdw.fdw_problem(64, 48, 1, -1, -1, 1, 1e-3, 0.1, 1, 0),   # x1 < x0
        fdw.fdw_problem(64, 48, -1, 1, -1, 1, 1e-3, 0.1, 7, 0),   # bad dtype
    ):
        assert ws(ctypes.byref(bad), 1) == 0
    # a family mixing storage types holds one child context per type: the sum of their workspaces
    p32, p64 = fdw.problem(64, 48, 1e-3, 10, fdw.FDW_F32), fdw.problem(64, 48, 1e-3, 10, fdw.FDW_F64)
    mixed = (fdw.fdw_problem * 2)(p32, p64)
    align = lambda b: (b + 255) // 256 * 256
    assert ws(mixed, 2) == align(ws(ctypes.byref(p32), 1)) + align(ws(ctypes.byref(p64), 1))
    bad_mixed = (fdw.fdw_problem * 2)(p32, fdw.fdw_problem(64, 48, -1, 1, -1, 1, 1e-3, 0.01, 7, 0))
    assert ws(bad_mixed, 2) == 0
    # init rejects NULL arguments before touching the device
    out = ctypes.c_void_p()
    lib.fdw_init.restype = ctypes.c_int
    assert lib.fdw_init(None, 1, None, 0, None, None, None, ctypes.byref(out)) == fdw.FDW_EINVAL
    lib.fdw_status_string.restype = ctypes.c_char_p
    assert lib.fdw_status_string(fdw.FDW_ECFL) == b"time step above the stability bound"
