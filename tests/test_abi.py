"""C ABI checks that need no GPU: the library loads, exports every call the
header declares, the Python constants equal the header's, and argument errors
come back as codes (no compute call is made)."""
import ctypes
import os
import re

import pytest

import paper_2208_11469_amd as pg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "probgraph.h")


def _header_text():
    with open(HEADER) as f:
        return f.read()


def _declared_functions():
    text = re.sub(r"/\*.*?\*/", "", _header_text(), flags=re.S)
    return sorted(set(re.findall(r"\b(pg_[a-z0-9_]+)\s*\(", text)))


def _defines():
    out = {}
    for name, val in re.findall(r"#define\s+(PG_[A-Z0-9_]+)\s+\(?(-?\d+)u?\)?", _header_text()):
        out[name] = int(val)
    return out


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pg.LIB_PATH):
        pytest.fail("libprobgraph.so is not built (run __graft_entry__.build())")
    return pg.load()


def test_every_declared_function_is_exported(lib):
    declared = _declared_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in probgraph.h but not exported"
    assert sorted(pg.EXPORTED) == declared


def test_python_constants_match_header():
    for name, val in _defines().items():
        assert getattr(pg, name) == val, name


def test_version_and_error_strings(lib):
    assert "gfx950" in pg.pg_version()
    assert isinstance(pg.pg_last_error(), str)


def test_null_arguments_are_rejected_without_a_device(lib):
    h = ctypes.c_void_p()
    assert lib.pg_ctx_create(0, None) == pg.PG_E_INVALID
    assert lib.pg_ctx_destroy(None) == pg.PG_E_INVALID
    assert lib.pg_graph_create(None, 4, 0, None, None, 0, None, ctypes.byref(h)) == pg.PG_E_INVALID
    assert lib.pg_graph_destroy(None) == pg.PG_E_INVALID
    assert lib.pg_build_sketches(None, None, pg.PG_BF, 256, 1, 1, None, ctypes.byref(h)) == pg.PG_E_INVALID
    assert lib.pg_tc(None, None, pg.PG_EST_BF_AND, None, None) == pg.PG_E_INVALID
    assert lib.pg_sketches_destroy(None) == pg.PG_E_INVALID
    assert "NULL" in pg.pg_last_error() or "null" in pg.pg_last_error().lower()


def test_no_gpu_context_creation_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = lib.pg_ctx_create(0, ctypes.byref(h))
    assert rc in (pg.PG_E_INVALID, pg.PG_E_DEVICE)
    assert not h.value
