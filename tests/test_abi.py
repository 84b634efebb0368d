"""The C-ABI library loads on the CPU and exports every declared entry point."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastperm.h")
LIB = os.path.join(ROOT, "paper_2602_00898_amd", "libfastperm.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\*]+\s+)+\**(fp_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2602_00898_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = declared()
    for n in ("fp_version", "fp_create", "fp_destroy", "fp_query", "fp_order", "fp_last_error",
              "fp_options_default", "fp_status_str"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_host_only_calls(lib):
    lib.fp_version.restype = ctypes.c_int
    assert lib.fp_version() == 2
    lib.fp_status_str.restype = ctypes.c_char_p
    assert lib.fp_status_str(0) == b"ok"
    from paper_2602_00898_amd.fastperm import Options
    o = Options()
    lib.fp_options_default(ctypes.byref(o))
    assert o.patch_size == 512 and o.nd_level == -1 and o.block_size == 1 and o.lloyd_iters == 1
    assert o.flags == 2  # FP_FLAG_VALIDATE
    # sizing calls need no device memory: the supernode workspace grows with n
    ws = ctypes.c_size_t()
    assert lib.fp_supernodes_query(ctypes.c_int64(1000), ctypes.byref(ws)) == 0 and ws.value > 0
    assert lib.fp_supernodes_query(ctypes.c_int64(-1), ctypes.byref(ws)) == 1
