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
    assert L.svr_serve_stats(None, None) == binding.SVR_EINVAL
    n = C.c_int32(7)
    assert L.svr_serve_done(None, None, 0, C.byref(n)) == binding.SVR_EINVAL
    assert L.svr_serve_trim(None, 1, 0) == binding.SVR_EINVAL
    assert L.svr_osem_epoch(None, None, 0, None) == binding.SVR_EINVAL
    L.svr_matrix_destroy(None)
    L.svr_recon_destroy(None)
    L.svr_serve_destroy(None)


def test_invalid_server_config_is_rejected(L):
    """svr_serve_create checks its configuration before it touches a device:
    budget, slots, streams, and the 0/1 switches batch and share_matrices."""
    h = C.c_void_p()
    good = dict(mem_budget_bytes=1 << 30, max_slots=2, n_streams=1, batch=1, share_matrices=1)
    for field, bad in [("mem_budget_bytes", 0), ("max_slots", 0), ("n_streams", 0), ("batch", 2),
                       ("share_matrices", 2), ("share_matrices", -1)]:
        cfg = binding.svr_serve_config(**dict(good, **{field: bad}))
        assert L.svr_serve_create(C.byref(cfg), C.byref(h)) == binding.SVR_EINVAL, field
        assert h.value is None
        assert L.svr_last_error()


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


def test_binding_rejects_mismatched_sizes_before_any_call():
    """The wrappers check that the tensors they pass hold the sizes the
    library will read and write (S*N, S*M), so a short buffer raises in Python
    instead of reaching the device; no library call is made here."""
    import numpy as np
    import torch
    from types import SimpleNamespace

    A = object.__new__(pkg.SystemMatrix)
    A.M, A.N, A.h = 12, 9, None
    with pytest.raises(ValueError):
        A.project(torch.zeros(10))                      # not a multiple of N
    with pytest.raises(ValueError):
        A.project(torch.zeros(18), y=torch.zeros(12))   # 2 slices need 24 outputs
    with pytest.raises(ValueError):
        A.backproject(torch.zeros(0))
    with pytest.raises(ValueError):
        A.backproject(torch.zeros(12), x=torch.zeros(8))
    with pytest.raises(ValueError):
        pkg.Recon(A, np.zeros(24), np.zeros(12), np.ones(18), pkg.params("svrem"))
    with pytest.raises(ValueError):
        pkg.Recon(A, np.zeros(12), np.zeros(12), np.ones(18), pkg.params("svrem"))
    S = object.__new__(pkg.Server)
    S.h, S._keep = None, {}
    geom = SimpleNamespace(nx=3, ny=3, pixel_mm=1.0, n_views=3, n_bins=4, bin_mm=1.0)
    with pytest.raises(ValueError):
        S.submit(geom, 1, np.zeros(11), np.zeros(12), pkg.params("svrem"), 1, 0)
    with pytest.raises(ValueError):
        S.submit(geom, 1, np.zeros(12), np.zeros(13), pkg.params("svrem"), 1, 0)
    S.h = None
    A.h = None


def test_host_phases_carry_roctx_ranges():
    """Matrix build, epoch calls, anchors, projector calls and serving ticks
    push named roctx ranges, so the library imports the roctx entry points."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None or not os.path.exists(binding.LIB_PATH):
        pytest.skip("nm or library not available")
    syms = subprocess.run([nm, "-D", "--undefined-only", binding.LIB_PATH], capture_output=True, text=True,
                          check=True).stdout
    assert "roctxRangePushA" in syms and "roctxRangePop" in syms
