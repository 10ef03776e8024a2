"""The C-ABI library loads and exports every symbol the header declares (CPU).

No compute call is made here: that needs the GPU.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmm.h")
LIB = os.path.join(ROOT, "paper_1505_07570_amd", "librmm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(rmm_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_paper_calls():
    names = declared_functions()
    for required in ("rmm_sketch", "rmm_rsvd", "rmm_sketched_lsr", "rmm_plain_lsr",
                     "rmm_sketch_hashes", "rmm_sketch_signs", "rmm_srht_indices",
                     "rmm_gaussian", "rmm_create", "rmm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("librmm.so not built")
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_strerror_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("librmm.so not built")
    L = ctypes.CDLL(LIB)
    L.rmm_strerror.restype = ctypes.c_char_p
    L.rmm_strerror.argtypes = [ctypes.c_int]
    assert L.rmm_strerror(0) == b"ok"
    assert L.rmm_strerror(-1) == b"invalid argument"
    assert L.rmm_strerror(-2) == b"workspace too small"


def test_null_handle_is_rejected_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("librmm.so not built")
    L = ctypes.CDLL(LIB)
    L.rmm_sketch.restype = ctypes.c_int
    assert L.rmm_set_stream(None, None) == -1
    assert L.rmm_set_workspace(None, None, ctypes.c_size_t(0)) == -1
