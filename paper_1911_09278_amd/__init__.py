"""Python binding of the MI355X MACE library (libmace.so, C ABI in include/mace.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of the library.  torch is used, when a caller wants it, only to hold
device memory and streams (``solve_dev`` takes ``tensor.data_ptr()`` values).
The library must have been built (``paper_1911_09278_amd.build.build()``);
importing this package raises if it has not.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libmace.so")

MACE_OK = 0
MACE_E_ARG = -1
MACE_E_MATRIX = -2
MACE_E_PARTITION = -3
MACE_E_NOMEM = -4
MACE_E_HIP = -5
MACE_E_NONFINITE = -6
MACE_E_CANCELLED = -7
MACE_W_MAXITER = 1


class MaceError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mace error {code}: {msg}")
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("n_views", ctypes.c_int32), ("n_channels", ctypes.c_int32)]


class Prior(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("sigma_x", ctypes.c_double), ("p", ctypes.c_double),
                ("q", ctypes.c_double), ("T", ctypes.c_double), ("b_edge", ctypes.c_double),
                ("b_diag", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("sv_size", ctypes.c_int32),
                ("rows_per_agent", ctypes.c_int32), ("fp32_tail_iters", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("refresh_every", ctypes.c_int32),
                ("format", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("residual", ctypes.c_double),
                ("equits", ctypes.c_double), ("status", ctypes.c_int32),
                ("sweep_ms", ctypes.c_double), ("sweep_launches", ctypes.c_int32),
                ("iter_ms", ctypes.c_double), ("fp32_tail_iters", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("sv_size", ctypes.c_int32), ("rows_per_agent", ctypes.c_int32),
                ("ms_per_iter", ctypes.c_double), ("residual", ctypes.c_double),
                ("status", ctypes.c_int32), ("format", ctypes.c_int32)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("in_flight", ctypes.c_int32),
                ("max_in_flight", ctypes.c_int32), ("bytes_in_use", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1911_09278_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.mace_load_system.argtypes = [P(Geom), vp, vp, vp, i32, vp, P(Opts), P(vp)]
    L.mace_load_system.restype = ctypes.c_int
    L.mace_solve.argtypes = [vp, vp, vp, P(Prior), d, d, i32, i32, d, vp, vp, P(Info)]
    L.mace_solve.restype = ctypes.c_int
    L.mace_solve_resume.argtypes = [vp, vp, vp, P(Prior), d, d, i32, i32, d, vp, vp, vp, P(Info)]
    L.mace_solve_resume.restype = ctypes.c_int
    L.mace_solve_pnp.argtypes = [vp, vp, vp, d, d, i32, i32, d, i32, vp, P(Info)]
    L.mace_solve_pnp.restype = ctypes.c_int
    L.mace_solve_dev.argtypes = [vp, vp, vp, P(Prior), d, d, i32, i32, d, vp, vp, P(Info), vp]
    L.mace_solve_dev.restype = ctypes.c_int
    L.mace_solve_dev_noalloc.argtypes = [vp, vp, vp, P(Prior), d, d, i32, i32, d, vp, vp,
                                         P(Info), vp]
    L.mace_solve_dev_noalloc.restype = ctypes.c_int
    L.mace_noalloc_capacity.argtypes = []
    L.mace_noalloc_capacity.restype = i64
    L.mace_solve_batch.argtypes = [vp, i32, vp, vp, P(Prior), d, d, i32, i32, d, vp, vp]
    L.mace_solve_batch.restype = ctypes.c_int
    L.mace_solve_batch_dev.argtypes = [vp, i32, vp, vp, P(Prior), d, d, i32, i32, d, vp, vp, vp]
    L.mace_solve_batch_dev.restype = ctypes.c_int
    L.mace_prox.argtypes = [vp, i32, vp, vp, P(Prior), d, vp, vp, i32, vp]
    L.mace_prox.restype = ctypes.c_int
    L.mace_visit_order.argtypes = [vp, vp]
    L.mace_visit_order.restype = ctypes.c_int
    L.mace_get_state.argtypes = [vp, vp, vp]
    L.mace_get_state.restype = ctypes.c_int
    L.mace_get_slot_state.argtypes = [vp, i32, vp, vp]
    L.mace_get_slot_state.restype = ctypes.c_int
    L.mace_solve_volume.argtypes = [vp, i32, vp, vp, P(Prior), d, d, d, i32, i32, d, vp, P(Info)]
    L.mace_solve_volume.restype = ctypes.c_int
    L.mace_get_error_sinogram.argtypes = [vp, vp]
    L.mace_get_error_sinogram.restype = ctypes.c_int
    L.mace_set_relaxation.argtypes = [vp, d]
    L.mace_set_relaxation.restype = ctypes.c_int
    L.mace_set_slice_group.argtypes = [vp, i32]
    L.mace_set_slice_group.restype = ctypes.c_int
    L.mace_set_fp32_tail.argtypes = [vp, i32]
    L.mace_set_fp32_tail.restype = ctypes.c_int
    L.mace_set_timing.argtypes = [vp, i32]
    L.mace_set_timing.restype = ctypes.c_int
    L.mace_system_bytes.argtypes = [vp]
    L.mace_system_bytes.restype = i64
    L.mace_scan_bytes.argtypes = [vp]
    L.mace_scan_bytes.restype = i64
    L.mace_check_layout.argtypes = [P(Geom), vp, vp, vp, i32, vp, P(Opts), vp]
    L.mace_check_layout.restype = ctypes.c_int
    L.mace_server_create.argtypes = [vp, i32, i64, P(vp)]
    L.mace_server_create.restype = ctypes.c_int
    L.mace_server_submit.argtypes = [vp, i32, vp, vp, P(Prior), d, d, i32, d, i32, P(i64)]
    L.mace_server_submit.restype = ctypes.c_int
    L.mace_server_wait.argtypes = [vp, i64, vp, P(Info), P(d)]
    L.mace_server_wait.restype = ctypes.c_int
    L.mace_server_cancel.argtypes = [vp, i64]
    L.mace_server_cancel.restype = ctypes.c_int
    L.mace_server_stats.argtypes = [vp, P(ServerCounters)]
    L.mace_server_stats.restype = ctypes.c_int
    L.mace_server_destroy.argtypes = [vp]
    L.mace_server_destroy.restype = None
    L.mace_autotune.argtypes = [P(Geom), vp, vp, vp, i32, vp, P(Opts), i32, P(Opts),
                                P(d), vp, i32, P(i32)]
    L.mace_autotune.restype = ctypes.c_int
    L.mace_get_config.argtypes = [vp, P(Opts)]
    L.mace_get_config.restype = ctypes.c_int
    L.mace_free_system.argtypes = [vp]
    L.mace_free_system.restype = None
    L.mace_test_fail_alloc.argtypes = [i32]
    L.mace_test_fail_alloc.restype = ctypes.c_int
    L.mace_last_error.argtypes = []
    L.mace_last_error.restype = ctypes.c_char_p
    return L


_lib = _load()

# Entry points of the C ABI, by name.
EXPORTED = ("mace_load_system", "mace_solve", "mace_solve_pnp", "mace_solve_dev", "mace_solve_batch",
            "mace_solve_batch_dev", "mace_prox", "mace_visit_order", "mace_get_state",
            "mace_get_error_sinogram", "mace_system_bytes", "mace_scan_bytes",
            "mace_check_layout", "mace_set_timing", "mace_set_relaxation", "mace_server_create",
            "mace_server_submit", "mace_server_wait", "mace_server_stats", "mace_server_destroy",
            "mace_autotune", "mace_get_config",
            "mace_free_system", "mace_last_error", "mace_test_fail_alloc",
            "mace_solve_dev_noalloc", "mace_noalloc_capacity", "mace_set_fp32_tail",
            "mace_solve_resume", "mace_server_cancel", "mace_solve_volume",
            "mace_get_slot_state", "mace_set_slice_group")


def noalloc_capacity() -> int:
    """Bytes of the static per-GPU workspace of the allocation-free solve."""
    return int(_lib.mace_noalloc_capacity())


def last_error() -> str:
    return _lib.mace_last_error().decode()


def test_fail_alloc(after: int) -> None:
    """Testing hook: make the after-th next device allocation fail (-1: off)."""
    _lib.mace_test_fail_alloc(int(after))


def _check(rc, allow=(MACE_OK, MACE_W_MAXITER)):
    if rc not in allow:
        raise MaceError(rc, last_error())
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data


def make_prior(kind=0, sigma_x=0.02, p=2.0, q=2.0, T=1.0, b_edge=0.0, b_diag=0.0) -> Prior:
    return Prior(int(kind), float(sigma_x), float(p), float(q), float(T), float(b_edge),
                 float(b_diag))


def check_layout(nx, ny, n_views, n_channels, col_ptr, row, val, n_agents, view_to_agent=None,
                 precision=0, sv_size=0, rows_per_agent=0, fp32_tail_iters=0, format=0) -> int:
    """Host-only dry run of the device layout and schedules (no GPU needed).
    Returns the LDS bytes per workgroup; raises MaceError on any bad index."""
    cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
    rw = np.ascontiguousarray(row, dtype=np.int32)
    vl = np.ascontiguousarray(val, dtype=np.float32)
    va = None if view_to_agent is None else np.ascontiguousarray(view_to_agent, dtype=np.int32)
    g = Geom(int(nx), int(ny), int(n_views), int(n_channels))
    o = Opts(int(precision), int(sv_size), int(rows_per_agent), int(fp32_tail_iters), 0, 0,
             int(format))
    lds = ctypes.c_int64(0)
    _check(_lib.mace_check_layout(ctypes.byref(g), _ptr(cp), _ptr(rw), _ptr(vl), int(n_agents),
                                  _ptr(va), ctypes.byref(o), ctypes.byref(lds)))
    return int(lds.value)


def autotune(nx, ny, n_views, n_channels, col_ptr, row, val, n_agents, view_to_agent=None,
             precision=0, sv_size=0, rows_per_agent=0, iters=6) -> dict:
    """Measured choice of super-voxel side and rows per agent (C ABI
    mace_autotune).  Returns {"sv_size", "rows_per_agent", "ms_per_iter",
    "table": [candidate dicts]}."""
    cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
    rw = np.ascontiguousarray(row, dtype=np.int32)
    vl = np.ascontiguousarray(val, dtype=np.float32)
    va = None if view_to_agent is None else np.ascontiguousarray(view_to_agent, dtype=np.int32)
    g = Geom(int(nx), int(ny), int(n_views), int(n_channels))
    base = Opts(int(precision), int(sv_size), int(rows_per_agent), 0, 0, 0)
    best = Opts()
    ms = ctypes.c_double(0.0)
    res = (TuneResult * 16)()
    nres = ctypes.c_int32(0)
    _check(_lib.mace_autotune(ctypes.byref(g), _ptr(cp), _ptr(rw), _ptr(vl), int(n_agents),
                              _ptr(va), ctypes.byref(base), int(iters), ctypes.byref(best),
                              ctypes.byref(ms), res, 16, ctypes.byref(nres)))
    table = [{f: getattr(res[i], f) for f, _ in TuneResult._fields_}
             for i in range(min(nres.value, 16))]
    return {"sv_size": best.sv_size, "rows_per_agent": best.rows_per_agent,
            "format": best.format, "ms_per_iter": ms.value, "table": table}


class System:
    """A loaded scanner geometry: repacked system matrix and view partition."""

    def __init__(self, nx, ny, n_views, n_channels, col_ptr, row, val, n_agents,
                 view_to_agent=None, precision=0, sv_size=0, rows_per_agent=0,
                 fp32_tail_iters=0, hbm_budget_bytes=0, refresh_every=0, format=0):
        self._h = None
        # held by the object: at interpreter exit the module's globals may
        # already be cleared when __del__ runs
        self._free = _lib.mace_free_system
        cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
        rw = np.ascontiguousarray(row, dtype=np.int32)
        vl = np.ascontiguousarray(val, dtype=np.float32)
        va = None if view_to_agent is None else np.ascontiguousarray(view_to_agent, dtype=np.int32)
        self.geom = Geom(int(nx), int(ny), int(n_views), int(n_channels))
        self.nx, self.ny = int(nx), int(ny)
        self.n = self.nx * self.ny
        self.n_rows = int(n_views) * int(n_channels)
        self.N = int(n_agents)
        self.nnz = int(cp[-1])
        opts = Opts(int(precision), int(sv_size), int(rows_per_agent), int(fp32_tail_iters),
                    int(hbm_budget_bytes), int(refresh_every), int(format))
        h = ctypes.c_void_p()
        _check(_lib.mace_load_system(ctypes.byref(self.geom), _ptr(cp), _ptr(rw), _ptr(vl),
                                     self.N, _ptr(va), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            self._free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def matrix_bytes(self) -> int:
        return int(_lib.mace_system_bytes(self._h))

    @property
    def config(self) -> dict:
        """Configuration in use (super-voxel side, rows per agent, ...)."""
        o = Opts()
        _check(_lib.mace_get_config(self._h, ctypes.byref(o)))
        return {f: getattr(o, f) for f, _ in Opts._fields_}

    @property
    def scan_bytes(self) -> int:
        """Device bytes of one scan's state (a batch slot / a served scan)."""
        return int(_lib.mace_scan_bytes(self._h))

    def solve(self, y, lam, prior: Prior, rho, sigma, max_iters, tol=0.0, sweeps=1,
              w_init=None):
        """Host arrays in, (x, info) out."""
        yy = np.ascontiguousarray(y, dtype=np.float32)
        ll = np.ascontiguousarray(lam, dtype=np.float32)
        if yy.size != self.n_rows or ll.size != self.n_rows:
            raise ValueError("y / lambda have the wrong size")
        wi = None if w_init is None else np.ascontiguousarray(w_init, dtype=np.float32)
        if wi is not None and wi.size != self.N * self.n:
            raise ValueError("w_init has the wrong size")
        x = np.empty(self.n, dtype=np.float32)
        info = Info()
        rc = _lib.mace_solve(self._h, _ptr(yy), _ptr(ll), ctypes.byref(prior), float(rho),
                             float(sigma), int(sweeps), int(max_iters), float(tol), _ptr(wi),
                             _ptr(x), ctypes.byref(info))
        _check(rc)
        return x, info

    def solve_resume(self, y, lam, prior: Prior, rho, sigma, max_iters, w0, X0, tol=0.0,
                     sweeps=1):
        """Continue a solve from a checkpoint (w0, X0) of state(); returns
        (x, info)."""
        yy = np.ascontiguousarray(y, dtype=np.float32)
        ll = np.ascontiguousarray(lam, dtype=np.float32)
        ww = np.ascontiguousarray(w0, dtype=np.float32).reshape(-1)
        XX = np.ascontiguousarray(X0, dtype=np.float32).reshape(-1)
        if yy.size != self.n_rows or ll.size != self.n_rows:
            raise ValueError("y / lambda have the wrong size")
        if ww.size != self.N * self.n or XX.size != self.N * self.n:
            raise ValueError("w0 / X0 have the wrong size")
        x = np.empty(self.n, dtype=np.float32)
        info = Info()
        rc = _lib.mace_solve_resume(self._h, _ptr(yy), _ptr(ll), ctypes.byref(prior), float(rho),
                                    float(sigma), int(sweeps), int(max_iters), float(tol),
                                    _ptr(ww), _ptr(XX), _ptr(x), ctypes.byref(info))
        _check(rc)
        return x, info

    def solve_volume(self, y, lam, prior: Prior, b_axial, rho, sigma, max_iters, tol=0.0,
                     sweeps=1):
        """A volume of nz slices (C ABI mace_solve_volume): y, lam of shape
        (nz, n_rows); returns (x of shape (nz, n), info)."""
        yy = np.ascontiguousarray(y, dtype=np.float32)
        ll = np.ascontiguousarray(lam, dtype=np.float32)
        nz = yy.size // self.n_rows
        if yy.size != nz * self.n_rows or ll.size != yy.size or nz < 1:
            raise ValueError("y / lambda must hold nz whole sinograms")
        x = np.empty((nz, self.n), dtype=np.float32)
        info = Info()
        rc = _lib.mace_solve_volume(self._h, nz, _ptr(yy), _ptr(ll), ctypes.byref(prior),
                                    float(b_axial), float(rho), float(sigma), int(sweeps),
                                    int(max_iters), float(tol), _ptr(x), ctypes.byref(info))
        _check(rc)
        return x, info

    def slot_state(self, slot):
        """(w, X) of scan slot `slot` (slice `slot` of a volume)."""
        w = np.empty(self.N * self.n, dtype=np.float32)
        X = np.empty(self.N * self.n, dtype=np.float32)
        _check(_lib.mace_get_slot_state(self._h, int(slot), _ptr(w), _ptr(X)))
        return w.reshape(self.N, self.n), X.reshape(self.N, self.n)

    def solve_pnp(self, y, lam, rho, sigma, max_iters, h_passes=1, tol=0.0, sweeps=1):
        """MACE with the stand-in PnP denoiser (C ABI mace_solve_pnp): host
        arrays in, (x = H(mean w), info) out."""
        yy = np.ascontiguousarray(y, dtype=np.float32)
        ll = np.ascontiguousarray(lam, dtype=np.float32)
        if yy.size != self.n_rows or ll.size != self.n_rows:
            raise ValueError("y / lambda have the wrong size")
        x = np.empty(self.n, dtype=np.float32)
        info = Info()
        rc = _lib.mace_solve_pnp(self._h, _ptr(yy), _ptr(ll), float(rho), float(sigma),
                                 int(sweeps), int(max_iters), float(tol), int(h_passes), _ptr(x),
                                 ctypes.byref(info))
        _check(rc)
        return x, info

    def solve_dev(self, y_ptr, lam_ptr, prior: Prior, rho, sigma, max_iters, x_ptr, tol=0.0,
                  sweeps=1, w_init_ptr=None, stream_ptr=None):
        """Device pointers (e.g. torch tensor.data_ptr()) in; returns info."""
        info = Info()
        rc = _lib.mace_solve_dev(self._h, ctypes.c_void_p(y_ptr), ctypes.c_void_p(lam_ptr),
                                 ctypes.byref(prior), float(rho), float(sigma), int(sweeps),
                                 int(max_iters), float(tol),
                                 None if w_init_ptr is None else ctypes.c_void_p(w_init_ptr),
                                 ctypes.c_void_p(x_ptr), ctypes.byref(info),
                                 None if stream_ptr is None else ctypes.c_void_p(stream_ptr))
        _check(rc)
        return info

    def solve_dev_noalloc(self, y_ptr, lam_ptr, prior: Prior, rho, sigma, max_iters, x_ptr,
                          tol=0.0, sweeps=1, w_init_ptr=None, stream_ptr=None):
        """mace_solve_dev without device allocation (static per-GPU
        workspace); device pointers in, returns info."""
        info = Info()
        rc = _lib.mace_solve_dev_noalloc(self._h, ctypes.c_void_p(y_ptr), ctypes.c_void_p(lam_ptr),
                                         ctypes.byref(prior), float(rho), float(sigma),
                                         int(sweeps), int(max_iters), float(tol),
                                         None if w_init_ptr is None else ctypes.c_void_p(w_init_ptr),
                                         ctypes.c_void_p(x_ptr), ctypes.byref(info),
                                         None if stream_ptr is None else ctypes.c_void_p(stream_ptr))
        _check(rc)
        return info

    def solve_batch(self, ys, lams, prior: Prior, rho, sigma, max_iters, tol=0.0, sweeps=1):
        """Several scans of this geometry at once (host arrays); returns
        (list of x, list of info)."""
        n = len(ys)
        if n != len(lams) or n == 0:
            raise ValueError("need one lambda per y and at least one scan")
        yy = [np.ascontiguousarray(y, dtype=np.float32) for y in ys]
        ll = [np.ascontiguousarray(l, dtype=np.float32) for l in lams]
        if any(a.size != self.n_rows for a in yy + ll):
            raise ValueError("y / lambda have the wrong size")
        xs = [np.empty(self.n, dtype=np.float32) for _ in range(n)]
        arr = ctypes.c_void_p * n
        infos = (Info * n)()
        rc = _lib.mace_solve_batch(self._h, n, arr(*[a.ctypes.data for a in yy]),
                                   arr(*[a.ctypes.data for a in ll]), ctypes.byref(prior),
                                   float(rho), float(sigma), int(sweeps), int(max_iters),
                                   float(tol), arr(*[a.ctypes.data for a in xs]), infos)
        _check(rc)
        return xs, list(infos)

    def solve_batch_dev(self, y_ptrs, lam_ptrs, prior: Prior, rho, sigma, max_iters, x_ptrs,
                        tol=0.0, sweeps=1, stream_ptr=None):
        """Device pointers per scan; returns the list of info records."""
        n = len(y_ptrs)
        if n != len(lam_ptrs) or n != len(x_ptrs) or n == 0:
            raise ValueError("need matching, non-empty pointer lists")
        arr = ctypes.c_void_p * n
        infos = (Info * n)()
        rc = _lib.mace_solve_batch_dev(self._h, n, arr(*y_ptrs), arr(*lam_ptrs),
                                       ctypes.byref(prior), float(rho), float(sigma), int(sweeps),
                                       int(max_iters), float(tol), arr(*x_ptrs), infos,
                                       None if stream_ptr is None else ctypes.c_void_p(stream_ptr))
        _check(rc)
        return list(infos)

    def prox(self, agent, y, lam, prior: Prior, sigma, v, x_init, sweeps=1):
        yy = np.ascontiguousarray(y, dtype=np.float32)
        ll = np.ascontiguousarray(lam, dtype=np.float32)
        vv = np.ascontiguousarray(v, dtype=np.float32)
        xi = np.ascontiguousarray(x_init, dtype=np.float32)
        out = np.empty(self.n, dtype=np.float32)
        _check(_lib.mace_prox(self._h, int(agent), _ptr(yy), _ptr(ll), ctypes.byref(prior),
                              float(sigma), _ptr(vv), _ptr(xi), int(sweeps), _ptr(out)))
        return out

    def visit_order(self):
        o = np.empty(self.n, dtype=np.int64)
        _check(_lib.mace_visit_order(self._h, _ptr(o)))
        return o

    def set_relaxation(self, gamma):
        _check(_lib.mace_set_relaxation(self._h, float(gamma)))

    def set_slice_group(self, slices):
        """Consecutive slices per super-voxel group of later volume solves
        (see mace_set_slice_group)."""
        _check(_lib.mace_set_slice_group(self._h, int(slices)))

    def set_fp32_tail(self, iters):
        """FP32 tail of later solves (precision-1 systems; see mace_opts)."""
        _check(_lib.mace_set_fp32_tail(self._h, int(iters)))

    def set_timing(self, enable=True):
        _check(_lib.mace_set_timing(self._h, 1 if enable else 0))

    def error_sinogram(self):
        e = np.empty(self.n_rows, dtype=np.float32)
        _check(_lib.mace_get_error_sinogram(self._h, _ptr(e)))
        return e

    def state(self):
        w = np.empty(self.N * self.n, dtype=np.float32)
        X = np.empty(self.N * self.n, dtype=np.float32)
        _check(_lib.mace_get_state(self._h, _ptr(w), _ptr(X)))
        return w.reshape(self.N, self.n), X.reshape(self.N, self.n)


class Server:
    """Continuous-batching reconstruction service over loaded systems.

    The systems must stay open while the server exists and must not be used
    by other calls meanwhile.  submit() returns at once; wait() blocks for one
    scan (ctypes releases the GIL during the call)."""

    def __init__(self, systems, hbm_budget_bytes=0):
        self._h = None
        self._destroy = _lib.mace_server_destroy  # see System.__init__
        self.systems = list(systems)
        arr = (ctypes.c_void_p * len(self.systems))(*[s._h.value for s in self.systems])
        h = ctypes.c_void_p()
        _check(_lib.mace_server_create(arr, len(self.systems), int(hbm_budget_bytes),
                                       ctypes.byref(h)))
        self._h = h

    def submit(self, system_idx, y, lam, prior: Prior, rho, sigma, tol, max_iters, sweeps=1):
        s = self.systems[system_idx]
        yy = np.ascontiguousarray(y, dtype=np.float32)
        ll = np.ascontiguousarray(lam, dtype=np.float32)
        if yy.size != s.n_rows or ll.size != s.n_rows:
            raise ValueError("y / lambda have the wrong size")
        t = ctypes.c_int64(0)
        _check(_lib.mace_server_submit(self._h, int(system_idx), _ptr(yy), _ptr(ll),
                                       ctypes.byref(prior), float(rho), float(sigma), int(sweeps),
                                       float(tol), int(max_iters), ctypes.byref(t)))
        return int(t.value)

    def wait(self, ticket, n_pixels):
        """Returns (x, info, latency_s); raises MaceError if the scan failed."""
        x = np.empty(int(n_pixels), dtype=np.float32)
        info = Info()
        lat = ctypes.c_double(0.0)
        _check(_lib.mace_server_wait(self._h, int(ticket), _ptr(x), ctypes.byref(info),
                                     ctypes.byref(lat)))
        return x, info, float(lat.value)

    def cancel(self, ticket):
        """Cancel a submitted scan (see mace_server_cancel)."""
        _check(_lib.mace_server_cancel(self._h, int(ticket)))

    def stats(self) -> dict:
        c = ServerCounters()
        _check(_lib.mace_server_stats(self._h, ctypes.byref(c)))
        return {f: int(getattr(c, f)) for f, _ in ServerCounters._fields_}

    def close(self):
        if self._h:
            self._destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
