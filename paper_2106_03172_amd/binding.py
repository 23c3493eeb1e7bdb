"""Thin ctypes binding of the C ABI in ``include/svr.h``.

Argument marshalling only: every step of the reconstruction runs in the HIP
library.  PyTorch supplies device memory (tensors) and the HIP stream
(``torch.cuda.current_stream()``).  If the built library is missing this
module raises instead of falling back to anything else.

The functions keep the C names (``svr_build_system_matrix``,
``svr_project``, ...); ``SystemMatrix`` and ``Recon`` wrap the handles.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SVR_LIBRARY", os.path.join(_HERE, "_lib", "libsvr.so"))

SVR_OK, SVR_PENDING, SVR_EINVAL, SVR_ENOMEM, SVR_EDEVICE = 0, 1, -1, -2, -3
SVR_ENOTFOUND, SVR_ENUMERIC, SVR_ECANCELLED = -4, -5, -6
SVR_W_F32, SVR_W_F16, SVR_W_BF16 = 0, 1, 2
SVR_W_INDEX32 = 0x100
ALGO = dict(osem=0, svrem=1, svrg=2, saga=3, sga=4, bsrem=5, sem=6, sagaem=7)
PEN = dict(quadratic=0, huber=1, logcosh=2, hyperbola=3)
PRECOND = dict(full_frozen=0, subset_frozen=1, iterate=2)
FLAG_RESET_SHAT_AT_ANCHOR, FLAG_AXIAL_PENALTY, FLAG_PERSISTENT_EPOCH, FLAG_MODIFIED_LL = 1, 2, 4, 8


class SvrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"svr error {code}: {msg}")
        self.code = code


class svr_geometry(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("pixel_mm", C.c_double),
                ("n_views", C.c_int32), ("n_bins", C.c_int32), ("bin_mm", C.c_double),
                ("arc_rad", C.c_double)]


class svr_matrix_info_t(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("bytes", C.c_int64), ("n_subsets", C.c_int32),
                ("n_rows", C.c_int32), ("n_pixels", C.c_int32), ("max_row_nnz", C.c_int32),
                ("max_col_nnz", C.c_int32), ("wtype", C.c_int32), ("index_bytes", C.c_int32)]


class svr_params(C.Structure):
    _fields_ = [("algo", C.c_int32), ("alpha", C.c_double), ("eta", C.c_int32),
                ("beta", C.c_double), ("penalty", C.c_int32), ("delta", C.c_double),
                ("precond", C.c_int32), ("flags", C.c_int32), ("decay", C.c_double),
                ("ll_eps", C.c_double)]


class svr_recon_info_t(C.Structure):
    _fields_ = [("k", C.c_int64), ("n_snapshots", C.c_int64), ("n_subsets", C.c_int32),
                ("n_slices", C.c_int32), ("n_pixels", C.c_int32), ("n_rows", C.c_int32),
                ("state_bytes", C.c_int64)]


class svr_kernel_times_t(C.Structure):
    _fields_ = [("launches", C.c_int64 * 6), ("total_ms", C.c_double * 6)]


class svr_tuning_t(C.Structure):
    _fields_ = [("fwd_pairs_per_wave", C.c_int32), ("bp_rows_per_group", C.c_int32),
                ("fwd_pair_rows", C.c_int32), ("fwd_us", C.c_double), ("bp_us", C.c_double),
                ("fwd_natural_order", C.c_int32), ("subset_fwd_batch", C.c_int32), ("subset_bp_batch", C.c_int32)]


class svr_serve_config(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_int64), ("max_slots", C.c_int32), ("n_streams", C.c_int32),
                ("batch", C.c_int32), ("share_matrices", C.c_int32)]


class svr_serve_request(C.Structure):
    _fields_ = [("geom", svr_geometry), ("n_subsets", C.c_int32), ("wtype", C.c_int32),
                ("params", svr_params), ("epochs", C.c_int32), ("order_seed", C.c_uint64),
                ("g_host", C.POINTER(C.c_float)), ("w_host", C.POINTER(C.c_float)),
                ("f0_value", C.c_float)]


class svr_serve_stats_t(C.Structure):
    _fields_ = [("queued", C.c_int32), ("resident", C.c_int32), ("max_slots", C.c_int32),
                ("done_unpolled", C.c_int32), ("used_bytes", C.c_int64), ("mem_budget_bytes", C.c_int64),
                ("ticks", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64), ("epochs", C.c_int64),
                ("cached_bytes", C.c_int64), ("block_reuses", C.c_int64), ("matrix_reuses", C.c_int64)]


class svr_serve_result(C.Structure):
    _fields_ = [("f_host", C.POINTER(C.c_float)), ("phi", C.c_double), ("queue_ms", C.c_double),
                ("run_ms", C.c_double), ("status", C.c_int32)]


_lib = None
_VP, _I32, _I64 = C.c_void_p, C.c_int32, C.c_int64
_SIGS = {
    "svr_last_error": ([], C.c_char_p),
    "svr_version": ([], C.c_int),
    "svr_build_system_matrix": ([C.POINTER(svr_geometry), _I32, _I32, _VP, _VP, C.POINTER(_VP)], C.c_int),
    "svr_matrix_info": ([_VP, C.POINTER(svr_matrix_info_t), _VP], C.c_int),
    "svr_matrix_export": ([_VP, _I32, _VP, _VP, _VP], C.c_int),
    "svr_sensitivity": ([_VP, _I32, _VP, _VP], C.c_int),
    "svr_matrix_destroy": ([_VP], None),
    "svr_matrix_get_tuning": ([_VP, C.POINTER(svr_tuning_t)], C.c_int),
    "svr_matrix_set_tuning": ([_VP, C.POINTER(svr_tuning_t)], C.c_int),
    "svr_matrix_tune": ([_VP, _VP, C.POINTER(svr_tuning_t)], C.c_int),
    "svr_project": ([_VP, _I32, _VP, _I32, _VP, _VP], C.c_int),
    "svr_backproject": ([_VP, _I32, _VP, _I32, _VP, _VP], C.c_int),
    "svr_project_noalloc": ([_VP, _I32, _VP, _I32, _VP, _VP], C.c_int),
    "svr_recon_create": ([_VP, _VP, _VP, _VP, _I32, C.POINTER(svr_params), _VP, C.POINTER(_VP)], C.c_int),
    "svr_objective": ([_VP, C.POINTER(C.c_double), _VP], C.c_int),
    "svr_get_image": ([_VP, _VP, _VP], C.c_int),
    "svr_recon_info": ([_VP, C.POINTER(svr_recon_info_t)], C.c_int),
    "svr_recon_get_state": ([_VP, _VP, C.POINTER(C.c_size_t), _VP], C.c_int),
    "svr_recon_set_state": ([_VP, _VP, C.c_size_t, _VP], C.c_int),
    "svr_recon_destroy": ([_VP], None),
    "svr_recon_set_profiling": ([_VP, _I32], C.c_int),
    "svr_recon_kernel_times": ([_VP, C.POINTER(svr_kernel_times_t)], C.c_int),
    "svr_serve_create": ([C.POINTER(svr_serve_config), C.POINTER(_VP)], C.c_int),
    "svr_serve_submit": ([_VP, C.POINTER(svr_serve_request), C.POINTER(C.c_uint64)], C.c_int),
    "svr_serve_step": ([_VP, _I32], C.c_int),
    "svr_serve_poll": ([_VP, C.c_uint64, C.POINTER(svr_serve_result)], C.c_int),
    "svr_serve_cancel": ([_VP, C.c_uint64], C.c_int),
    "svr_serve_destroy": ([_VP], None),
    "svr_serve_stats": ([_VP, C.POINTER(svr_serve_stats_t)], C.c_int),
    "svr_serve_done": ([_VP, C.POINTER(C.c_uint64), _I32, C.POINTER(_I32)], C.c_int),
    "svr_serve_trim": ([_VP, _I32, _I64], C.c_int),
}
for _e in ("osem", "svrem", "svrg", "saga", "sga", "bsrem", "sem"):
    _SIGS[f"svr_{_e}_epoch"] = ([_VP, _VP, _I32, _VP], C.c_int)
_SIGS["svr_sagaem_epoch"] = ([_VP, _VP, _VP, _I32, _VP], C.c_int)

EXPORTED = tuple(_SIGS)


def lib():
    """Loads the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or python -m paper_2106_03172_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise SvrError(rc, lib().svr_last_error().decode())
    return rc


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype_name="float32"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def geometry(geom) -> svr_geometry:
    return svr_geometry(int(geom.nx), int(geom.ny), float(geom.pixel_mm), int(geom.n_views),
                        int(geom.n_bins), float(geom.bin_mm), float(getattr(geom, "arc_rad", np.pi)))


def params(algo="svrem", alpha=1.0, eta=1, beta=0.0, penalty="quadratic", delta=1.0,
           precond="full_frozen", flags=0, decay=0.001, ll_eps=0.0) -> svr_params:
    """svr_params; ``ll_eps > 0`` also sets FLAG_MODIFIED_LL (the modified likelihood).  ``precond``
    (SVRG, SAGA) defaults to the one frozen vector f0 / A^T 1 of Theorem 1."""
    if ll_eps > 0:
        flags |= FLAG_MODIFIED_LL
    return svr_params(ALGO[algo] if isinstance(algo, str) else int(algo), float(alpha), int(eta),
                      float(beta), PEN[penalty] if isinstance(penalty, str) else int(penalty),
                      float(delta), PRECOND[precond] if isinstance(precond, str) else int(precond),
                      int(flags), float(decay), float(ll_eps))


# ---------------------------------------------------------------------------
# C-named thin wrappers
# ---------------------------------------------------------------------------
def svr_build_system_matrix(geom, n_subsets: int, wtype: int = SVR_W_F32, mu=None, stream=None):
    h = C.c_void_p()
    g = geometry(geom)
    _check(lib().svr_build_system_matrix(C.byref(g), int(n_subsets), int(wtype), _dev(mu),
                                         _stream(stream), C.byref(h)))
    return h


def svr_project(A, subset: int, x, n_slices: int, y, stream=None):
    _check(lib().svr_project(A, int(subset), _dev(x), int(n_slices), _dev(y), _stream(stream)))


def svr_project_noalloc(A, subset: int, x, n_slices: int, y, stream=None):
    _check(lib().svr_project_noalloc(A, int(subset), _dev(x), int(n_slices), _dev(y), _stream(stream)))


def svr_backproject(A, subset: int, y, n_slices: int, x, stream=None):
    _check(lib().svr_backproject(A, int(subset), _dev(y), int(n_slices), _dev(x), _stream(stream)))


def svr_recon_create(A, g, w, f0, n_slices: int, prm: svr_params, stream=None):
    h = C.c_void_p()
    _check(lib().svr_recon_create(A, _dev(g), _dev(w), _dev(f0), int(n_slices), C.byref(prm),
                                  _stream(stream), C.byref(h)))
    return h


def _epoch(name, R, order, stream=None):
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    _check(getattr(lib(), f"svr_{name}_epoch")(R, o.ctypes.data_as(C.c_void_p), int(o.size), _stream(stream)))


def svr_osem_epoch(R, order, stream=None): _epoch("osem", R, order, stream)
def svr_svrem_epoch(R, order, stream=None): _epoch("svrem", R, order, stream)
def svr_svrg_epoch(R, order, stream=None): _epoch("svrg", R, order, stream)
def svr_saga_epoch(R, order, stream=None): _epoch("saga", R, order, stream)
def svr_sga_epoch(R, order, stream=None): _epoch("sga", R, order, stream)
def svr_bsrem_epoch(R, order, stream=None): _epoch("bsrem", R, order, stream)
def svr_sem_epoch(R, order, stream=None): _epoch("sem", R, order, stream)


def svr_sagaem_epoch(R, order, refresh=None, stream=None):
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    rf = None
    if refresh is not None:
        rf = np.ascontiguousarray(np.asarray(refresh, dtype=np.int32))
        if rf.size != o.size:
            raise ValueError("refresh must have one entry per order entry")
    _check(lib().svr_sagaem_epoch(R, o.ctypes.data_as(C.c_void_p),
                                  None if rf is None else rf.ctypes.data_as(C.c_void_p), int(o.size),
                                  _stream(stream)))


def svr_objective(R, stream=None) -> float:
    v = C.c_double()
    _check(lib().svr_objective(R, C.byref(v), _stream(stream)))
    return v.value


# ---------------------------------------------------------------------------
# handle wrappers
# ---------------------------------------------------------------------------
def _slices(t, per_slice: int, name: str) -> int:
    """Number of slices in t, which must hold a positive whole number of
    per_slice values (the library reads and writes S * per_slice values)."""
    n = int(t.numel() if hasattr(t, "numel") else np.size(t))
    if n == 0 or n % per_slice:
        raise ValueError(f"{name} holds {n} values, not a positive multiple of {per_slice}")
    return n // per_slice


class SystemMatrix:
    """A system matrix built on the device (``svr_build_system_matrix``)."""

    def __init__(self, geom, n_subsets: int, wtype: int = SVR_W_F32, mu=None, stream=None):
        import torch
        self.geom = geom
        self.n_subsets = int(n_subsets)
        if mu is not None and not isinstance(mu, torch.Tensor):
            mu = torch.as_tensor(np.asarray(mu, dtype=np.float32), device="cuda")
        self.h = svr_build_system_matrix(geom, n_subsets, wtype, mu, stream)
        self.M = geom.n_views * geom.n_bins
        self.N = geom.nx * geom.ny

    def info(self):
        inf = svr_matrix_info_t()
        per = np.zeros(self.n_subsets, dtype=np.int64)
        _check(lib().svr_matrix_info(self.h, C.byref(inf), per.ctypes.data_as(C.c_void_p)))
        return inf, per

    def export(self, which: int):
        inf, _ = self.info()
        nrows = self.M if which == 0 else self.n_subsets * self.N
        ptr = np.zeros(nrows + 1, dtype=np.int32)
        idx = np.zeros(inf.nnz, dtype=np.int32)
        val = np.zeros(inf.nnz, dtype=np.float32)
        _check(lib().svr_matrix_export(self.h, int(which), ptr.ctypes.data_as(C.c_void_p),
                                       idx.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p)))
        return ptr, idx, val

    def sensitivity(self, subset: int, stream=None):
        import torch
        out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(lib().svr_sensitivity(self.h, int(subset), _dev(out, "float64"), _stream(stream)))
        return out

    def tuning(self):
        """Effective run lengths of the whole-matrix passes: (row pairs per wavefront, rows per lane group)."""
        t = svr_tuning_t()
        _check(lib().svr_matrix_get_tuning(self.h, C.byref(t)))
        return int(t.fwd_pairs_per_wave), int(t.bp_rows_per_group)

    def set_tuning(self, fwd_pairs_per_wave: int = 0, bp_rows_per_group: int = 0, fwd_pair_rows=None,
                   fwd_natural_order=None, subset_fwd_batch=None, subset_bp_batch=None):
        """Sets the run lengths (0: size-based); fwd_pair_rows (None: unchanged) is the row count above
        which a forward pass runs a pair of rows per wavefront (0: from the device); fwd_natural_order
        (None: unchanged) 1 takes the rows of one-row-per-wavefront passes in order, 0 in XCD bin bands;
        subset_fwd_batch / subset_bp_batch (None: unchanged, 0: default) the per-subset batch widths."""
        cur = svr_tuning_t()
        _check(lib().svr_matrix_get_tuning(self.h, C.byref(cur)))
        pr = cur.fwd_pair_rows if fwd_pair_rows is None else int(fwd_pair_rows)
        no = cur.fwd_natural_order if fwd_natural_order is None else int(fwd_natural_order)
        fu = cur.subset_fwd_batch if subset_fwd_batch is None else int(subset_fwd_batch)
        bu = cur.subset_bp_batch if subset_bp_batch is None else int(subset_bp_batch)
        t = svr_tuning_t(int(fwd_pairs_per_wave), int(bp_rows_per_group), pr, 0.0, 0.0, no, fu, bu)
        _check(lib().svr_matrix_set_tuning(self.h, C.byref(t)))

    def batch_widths(self):
        """Batch widths of the per-subset passes in use: (forward loads per lane, update loads per lane)."""
        t = svr_tuning_t()
        _check(lib().svr_matrix_get_tuning(self.h, C.byref(t)))
        return int(t.subset_fwd_batch), int(t.subset_bp_batch)

    def pair_rows(self) -> int:
        """Effective row count above which a forward pass runs a pair of rows per wavefront."""
        t = svr_tuning_t()
        _check(lib().svr_matrix_get_tuning(self.h, C.byref(t)))
        return int(t.fwd_pair_rows)

    def tune(self, stream=None):
        """Autotunes the run lengths and the per-subset batch widths on the device; returns
        (fwd, bp, fwd_us, bp_us); batch_widths() then gives the chosen widths."""
        t = svr_tuning_t()
        _check(lib().svr_matrix_tune(self.h, _stream(stream), C.byref(t)))
        return int(t.fwd_pairs_per_wave), int(t.bp_rows_per_group), float(t.fwd_us), float(t.bp_us)

    def project(self, x, subset: int = -1, y=None, stream=None):
        """y = A_t x for every slice of x ([S][N]); y ([S][M], natural order) is
        allocated when not given, else must hold exactly S*M floats."""
        import torch
        S = _slices(x, self.N, "x")
        if y is None:
            y = torch.zeros(S, self.M, dtype=torch.float32, device=x.device)
        elif y.numel() != S * self.M:
            raise ValueError(f"y holds {y.numel()} values, the projection of {S} slice(s) needs {S * self.M}")
        svr_project(self.h, subset, x, S, y, stream)
        return y

    def backproject(self, y, subset: int = -1, x=None, stream=None):
        """x = A_t^T y for every slice of y ([S][M]); x ([S][N]) is allocated when
        not given, else must hold exactly S*N floats."""
        import torch
        S = _slices(y, self.M, "y")
        if x is None:
            x = torch.empty(S, self.N, dtype=torch.float32, device=y.device)
        elif x.numel() != S * self.N:
            raise ValueError(f"x holds {x.numel()} values, the back-projection of {S} slice(s) needs {S * self.N}")
        svr_backproject(self.h, subset, y, S, x, stream)
        return x

    def close(self):
        if getattr(self, "h", None):
            lib().svr_matrix_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Recon:
    """A reconstruction (``svr_recon_create``) bound to a SystemMatrix."""

    def __init__(self, A: SystemMatrix, g, w, f0, prm: svr_params, stream=None):
        import torch

        def dev(x):
            if isinstance(x, torch.Tensor):
                return x.to(device="cuda", dtype=torch.float32).contiguous()
            return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda")
        self.A = A
        S = _slices(g, A.M, "g")
        if _slices(w, A.M, "w") != S or _slices(f0, A.N, "f0") != S:
            raise ValueError(f"g, w and f0 must describe the same number of slices ({S})")
        self.g, self.w, f0 = dev(g), dev(w), dev(f0)
        self.S = S
        self.prm = prm
        self.h = svr_recon_create(A.h, self.g, self.w, f0, self.S, prm, stream)

    def epoch(self, name: str, order, stream=None):
        if name == "sagaem":
            svr_sagaem_epoch(self.h, order, None, stream)
        else:
            _epoch(name, self.h, order, stream)

    def osem_epoch(self, order, stream=None): _epoch("osem", self.h, order, stream)
    def svrem_epoch(self, order, stream=None): _epoch("svrem", self.h, order, stream)
    def svrg_epoch(self, order, stream=None): _epoch("svrg", self.h, order, stream)
    def saga_epoch(self, order, stream=None): _epoch("saga", self.h, order, stream)
    def sga_epoch(self, order, stream=None): _epoch("sga", self.h, order, stream)
    def bsrem_epoch(self, order, stream=None): _epoch("bsrem", self.h, order, stream)
    def sem_epoch(self, order, stream=None): _epoch("sem", self.h, order, stream)
    def sagaem_epoch(self, order, refresh=None, stream=None): svr_sagaem_epoch(self.h, order, refresh, stream)

    def objective(self, stream=None) -> float:
        return svr_objective(self.h, stream)

    def image(self, stream=None):
        import torch
        out = torch.empty(self.S, self.A.N, dtype=torch.float32, device="cuda")
        _check(lib().svr_get_image(self.h, _dev(out), _stream(stream)))
        return out

    def info(self) -> svr_recon_info_t:
        inf = svr_recon_info_t()
        _check(lib().svr_recon_info(self.h, C.byref(inf)))
        return inf

    def get_state(self, stream=None) -> bytes:
        n = C.c_size_t(0)
        _check(lib().svr_recon_get_state(self.h, None, C.byref(n), _stream(stream)))
        buf = C.create_string_buffer(n.value)
        _check(lib().svr_recon_get_state(self.h, buf, C.byref(n), _stream(stream)))
        return buf.raw[:n.value]

    def set_state(self, state: bytes, stream=None):
        buf = C.create_string_buffer(state, len(state))
        _check(lib().svr_recon_set_state(self.h, buf, len(state), _stream(stream)))

    def set_profiling(self, enable: bool):
        _check(lib().svr_recon_set_profiling(self.h, int(bool(enable))))

    def kernel_times(self):
        """{kind: (launches, total_ms)} since the last call (synchronises)."""
        kt = svr_kernel_times_t()
        _check(lib().svr_recon_kernel_times(self.h, C.byref(kt)))
        names = ("forward", "update", "anchor_forward", "anchor_table", "anchor_sum", "epoch")
        return {names[i]: (int(kt.launches[i]), float(kt.total_ms[i])) for i in range(6)}

    def close(self):
        if getattr(self, "h", None):
            lib().svr_recon_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching SVREM server (``svr_serve_*``)."""

    def __init__(self, mem_budget_bytes: int, max_slots: int = 8, n_streams: int = 4, batch: bool = True,
                 share_matrices: bool = True):
        cfg = svr_serve_config(int(mem_budget_bytes), int(max_slots), int(n_streams), 1 if batch else 0,
                               1 if share_matrices else 0)
        self.h = C.c_void_p()
        _check(lib().svr_serve_create(C.byref(cfg), C.byref(self.h)))
        self._keep = {}

    def submit(self, geom, n_subsets: int, g, w, prm: svr_params, epochs: int, order_seed: int,
               f0_value: float = 1.0, wtype: int = SVR_W_F32) -> int:
        g = np.ascontiguousarray(g, dtype=np.float32).ravel()
        w = np.ascontiguousarray(w, dtype=np.float32).ravel()
        M = int(geom.n_views) * int(geom.n_bins)
        if g.size != M or w.size != M:
            raise ValueError(f"g and w must hold n_views * n_bins = {M} values (got {g.size}, {w.size})")
        req = svr_serve_request(geometry(geom), int(n_subsets), int(wtype), prm, int(epochs),
                                int(order_seed), g.ctypes.data_as(C.POINTER(C.c_float)),
                                w.ctypes.data_as(C.POINTER(C.c_float)), float(f0_value))
        t = C.c_uint64()
        _check(lib().svr_serve_submit(self.h, C.byref(req), C.byref(t)))
        self._keep[t.value] = geom.nx * geom.ny
        return t.value

    def step(self, max_ticks: int = 0):
        _check(lib().svr_serve_step(self.h, int(max_ticks)))

    def poll(self, ticket: int):
        """None while pending, else a dict with the image and timings."""
        n = self._keep.get(ticket, 1)  # unknown tickets are reported by the library
        f = np.empty(n, dtype=np.float32)  # the library fills all n floats once the request is done
        res = svr_serve_result(f.ctypes.data_as(C.POINTER(C.c_float)), 0.0, 0.0, 0.0, 0)
        rc = lib().svr_serve_poll(self.h, C.c_uint64(ticket), C.byref(res))
        if rc == SVR_PENDING:
            return None
        _check(rc)
        self._keep.pop(ticket, None)
        return dict(f=f, phi=res.phi, queue_ms=res.queue_ms, run_ms=res.run_ms, status=res.status)

    def cancel(self, ticket: int):
        _check(lib().svr_serve_cancel(self.h, C.c_uint64(ticket)))

    def done(self, cap: int = 1024) -> list:
        """Tickets of finished requests not yet polled (svr_serve_done), ascending."""
        buf = (C.c_uint64 * cap)()
        n = C.c_int32()
        _check(lib().svr_serve_done(self.h, buf, int(cap), C.byref(n)))
        return list(buf[:n.value])

    def trim(self, drop_matrices: bool = True, keep_bytes: int = 0):
        """Gives back kept device memory (svr_serve_trim): idle matrices, then kept blocks beyond
        ``keep_bytes``."""
        _check(lib().svr_serve_trim(self.h, 1 if drop_matrices else 0, int(keep_bytes)))

    def stats(self) -> dict:
        """Queue depth, slots in use, device memory held and running totals (svr_serve_stats)."""
        st = svr_serve_stats_t()
        _check(lib().svr_serve_stats(self.h, C.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in svr_serve_stats_t._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().svr_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def splitmix64_orders(seed: int, n_subsets: int, epochs: int):
    """The server's subset sequence: SplitMix64 (Steele, Lea and Flood, 2014)
    from ``seed``, index = ((z >> 32) * Ns) >> 32, one epoch of Ns draws per tick."""
    M64 = (1 << 64) - 1
    s = int(seed) & M64
    out = []
    for _ in range(epochs):
        o = []
        for _ in range(n_subsets):
            s = (s + 0x9E3779B97F4A7C15) & M64
            z = s
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
            z ^= z >> 31
            o.append(((z >> 32) * n_subsets) >> 32)
        out.append(np.array(o, dtype=np.int32))
    return out
