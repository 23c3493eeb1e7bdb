"""The C-ABI library loads and exports every symbol the header declares.

No compute call is made here (this runs without a GPU); the argument checks
that reject NULL or invalid arguments before touching the device are
exercised through the binding."""

import ctypes as C
import os
import re

import pytest

import paper_2106_03172_amd as pkg
from paper_2106_03172_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "svr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(svr_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    return pkg.lib()


def test_every_declared_symbol_is_exported(L):
    decl = _declared()
    assert len(decl) >= 25
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(binding.EXPORTED)


def test_version(L):
    assert L.svr_version() >= 10000


def test_null_arguments_are_rejected(L):
    h = C.c_void_p()
    assert L.svr_build_system_matrix(None, 1, 0, None, None, C.byref(h)) == binding.SVR_EINVAL
    assert b"NULL" in L.svr_last_error()
    assert L.svr_matrix_info(None, None, None) == binding.SVR_EINVAL
    assert L.svr_serve_create(None, C.byref(h)) == binding.SVR_EINVAL
    assert L.svr_osem_epoch(None, None, 0, None) == binding.SVR_EINVAL
    L.svr_matrix_destroy(None)
    L.svr_recon_destroy(None)
    L.svr_serve_destroy(None)


def test_invalid_geometry_is_rejected(L):
    h = C.c_void_p()
    for g in (binding.svr_geometry(0, 4, 1.0, 4, 5, 1.0, 3.14),
              binding.svr_geometry(4, 4, -1.0, 4, 5, 1.0, 3.14),
              binding.svr_geometry(4, 4, 1.0, 4, 5, float("nan"), 3.14)):
        assert L.svr_build_system_matrix(C.byref(g), 1, 0, None, None, C.byref(h)) == binding.SVR_EINVAL
    g = binding.svr_geometry(4, 4, 1.0, 4, 5, 1.0, 3.14)
    assert L.svr_build_system_matrix(C.byref(g), 5, 0, None, None, C.byref(h)) == binding.SVR_EINVAL
    assert L.svr_build_system_matrix(C.byref(g), 0, 0, None, None, C.byref(h)) == binding.SVR_EINVAL
    assert L.svr_build_system_matrix(C.byref(g), 2, 7, None, None, C.byref(h)) == binding.SVR_EINVAL


def test_serve_config_is_validated(L):
    h = C.c_void_p()
    cfg = binding.svr_serve_config(0, 1, 1)
    assert L.svr_serve_create(C.byref(cfg), C.byref(h)) == binding.SVR_EINVAL
    cfg = binding.svr_serve_config(1 << 30, 0, 1)
    assert L.svr_serve_create(C.byref(cfg), C.byref(h)) == binding.SVR_EINVAL
