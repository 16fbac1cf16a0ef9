"""The C-ABI library loads and exports every function include/gsn.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "gsn.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("gs_build_graph", "gs_count_3pcf", "gs_count_4pcf_parity", "gs_create",
                     "gs_destroy", "gs_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2607_06604_amd as gsn
    lib = ctypes.CDLL(gsn.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(gsn.EXPORTS) == _declared()


def test_strerror_without_device():
    import paper_2607_06604_amd as gsn
    lib = gsn.load()
    assert lib.gs_strerror(0) == b"ok"
    assert lib.gs_strerror(gsn.GS_EINVAL) == b"invalid argument"
    assert lib.gs_strerror(-12345) == b"unknown status"


def test_null_arguments_rejected_without_device():
    import paper_2607_06604_amd as gsn
    lib = gsn.load()
    assert lib.gs_destroy(None) == gsn.GS_EINVAL
    assert lib.gs_graph_free(None) == gsn.GS_EINVAL
    assert lib.gs_graph_info(None, None) == gsn.GS_EINVAL
    assert lib.gs_create(None, 0, 0, None) == gsn.GS_EINVAL
