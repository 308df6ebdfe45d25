"""The C-ABI library loads without a GPU and exports every function that
include/stag.h declares; argument checks that precede any device work behave
as documented."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stag.h")
LIB = os.path.join(ROOT, "paper_1710_09178_amd", "libstag.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stag_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1710_09178_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (stag_\w+)", out))
    assert set(names) <= exported


def test_create_rejects_bad_dims_before_touching_the_gpu(lib):
    lib.stag_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    for dims in [(4, 4, 4, 3), (4, 0, 4, 4), (1, 4, 4, 4)]:
        arr = (ctypes.c_int * 4)(*dims)
        assert lib.stag_create(ctypes.byref(h), arr, None) == -1
        assert b"even" in lib.stag_last_error(None)
    assert lib.stag_create(None, (ctypes.c_int * 4)(4, 4, 4, 4), None) == -1


def test_null_handle_calls_are_rejected(lib):
    assert lib.stag_dslash(None, None, None, 1) == -1
    assert lib.stag_destroy(None) == 0
    assert lib.stag_field_bytes(None, 0) == 0
