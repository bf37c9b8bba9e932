"""CPU-only checks of the C ABI library: it loads and exports every symbol
include/bsmm.h declares.  No compute call is made (no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_1705_10218_amd import bsmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "bsmm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bsmm_[a-z_]+)\s*\(", txt)))


def test_header_lists_the_abi():
    names = _declared()
    assert "bsmm_multiply" in names and "bsmm_block_norms" in names and "bsmm_filter" in names
    assert "bsmm_mat_create" in names
    assert set(names) == set(bsmm.SYMBOLS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(bsmm.LIB_PATH):
        pytest.fail("libbsmm.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(bsmm.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_device():
    L = bsmm.lib()
    assert bsmm.status_string(0) == "BSMM_OK"
    assert bsmm.status_string(5) == "BSMM_ERR_OUT_OF_MEMORY"
    assert L.bsmm_last_error() is not None
