"""C-ABI checks that need no GPU: the library loads, exports every function
include/hbi.h declares, and rejects bad arguments before any device call."""
import ctypes
import os
import re

import pytest

from _hbi_util import ROOT, ensure_built
from paper_2210_02698_amd import _lib

HEADER = os.path.join(ROOT, "include", "hbi.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hbi_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    ensure_built()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(n for n, _, _ in _lib.SIGNATURES) == names


def test_null_context_is_an_argument_error(lib):
    null = ctypes.c_void_p()
    assert lib.hbi_build(null, 1e-7, 0) == _lib.HBI_ERR_ARG
    assert lib.hbi_apply(null, None, None, 1, 1) == _lib.HBI_ERR_ARG
    assert lib.hbi_apply_adjoint(null, None, None, 1, 1) == _lib.HBI_ERR_ARG
    assert lib.hbi_load_tables(null, None) == _lib.HBI_ERR_ARG
    assert lib.hbi_load_tables_from(null, null, 1.0) == _lib.HBI_ERR_ARG
    assert lib.hbi_set_inclusion(null, 0, None, None, None) == _lib.HBI_ERR_ARG
    assert lib.hbi_set_build_opts(null, None) == _lib.HBI_ERR_ARG
    assert lib.hbi_entries(null, None, 0, None, 0, None) == _lib.HBI_ERR_ARG
    assert lib.hbi_get_info(null, None, 0) == _lib.HBI_ERR_ARG
    assert lib.hbi_set_stream(null, None) == _lib.HBI_ERR_ARG
    assert lib.hbi_set_profiling(null, 1) == _lib.HBI_ERR_ARG
    assert lib.hbi_get_profile(null, None, 0) == _lib.HBI_ERR_ARG
    assert lib.hbi_last_error(null) == b"ctx is NULL"
    assert lib.hbi_destroy(null) == _lib.HBI_OK


def test_create_rejects_null_out(lib):
    assert lib.hbi_create(0, None, None) == _lib.HBI_ERR_ARG
    assert b"out" in lib.hbi_last_error(None)


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="not found"):
        _lib._lib = None
        try:
            _lib.load(str(tmp_path / "nope.so"))
        finally:
            _lib._lib = None
