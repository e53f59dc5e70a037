"""CPU-side checks of the C-ABI library: it loads and exports every symbol
include/shiftsolve.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shiftsolve.h")
LIB = os.path.join(ROOT, "paper_1708_06290_amd", "libshiftsolve.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(shs_[a-z_]+)\s*\(", text)))


def _lib():
    if not os.path.exists(LIB):
        pytest.skip("libshiftsolve.so not built")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("shs_reduce", "shs_solve", "shs_solve_workspace", "shs_apply_q", "shs_get_reduced",
                 "shs_info", "shs_destroy", "shs_strerror", "shs_abi_version"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (shs_[a-z_]+)\b", out))
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)


def test_host_only_calls():
    lib = _lib()
    lib.shs_abi_version.restype = ctypes.c_int
    assert lib.shs_abi_version() == 2
    lib.shs_strerror.restype = ctypes.c_char_p
    assert lib.shs_strerror(0) == b"success"
    assert lib.shs_strerror(-3) == b"invalid argument"
    assert lib.shs_strerror(7) == b"cancelled"
    # argument validation happens before any device work
    lib.shs_reduce.restype = ctypes.c_int
    h = ctypes.c_void_p()
    rc = lib.shs_reduce(ctypes.c_int64(1), ctypes.c_int64(1), ctypes.c_int64(1), None, ctypes.c_int64(1),
                        None, ctypes.c_int64(1), None, ctypes.c_int64(1), None, None, ctypes.byref(h))
    assert rc == -1
    rc = lib.shs_reduce(ctypes.c_int64(10), ctypes.c_int64(17), ctypes.c_int64(1), None, ctypes.c_int64(10),
                        None, ctypes.c_int64(10), None, ctypes.c_int64(1), None, None, ctypes.byref(h))
    assert rc == -2
    lib.shs_info.restype = ctypes.c_int
    assert lib.shs_info(None, None) == -1


def test_binding_names_match_the_abi():
    import paper_1708_06290_amd as ss
    for name in ("shs_reduce", "shs_solve", "shs_solve_workspace", "shs_apply_q", "shs_get_reduced",
                 "shs_info", "shs_destroy"):
        assert callable(getattr(ss, name))


@pytest.mark.parametrize("n,m,p", [(10000, 8, 8), (16384, 10, 10), (4096, 4, 4), (1000, 8, 8), (8192, 16, 16),
                                   (1024, 1, 1), (777, 5, 2), (70, 1, 2), (129, 3, 0), (17, 16, 3)])
def test_reduction_launch_plan_stays_in_bounds(n, m, p):
    """Every GEMM launch of the blocked reduction (grid, split-K partials,
    operand extents against the buffers shs_reduce allocates) is checked on
    the host, at the full sizes the benchmark and tests reduce."""
    lib = _lib()
    lib.shs_reduce_check_plan.restype = ctypes.c_int
    lib.shs_reduce_check_plan.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_char_p, ctypes.c_int64]
    launches = ctypes.c_int64()
    msg = ctypes.create_string_buffer(256)
    rc = lib.shs_reduce_check_plan(n, m, p, ctypes.byref(launches), msg, 256)
    assert rc == 0, msg.value.decode()
    assert launches.value > 0 or n - m - 1 <= 0   # no column needs a reflector
