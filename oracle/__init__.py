"""FP64 CPU oracle for partial-update MACE (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this package.  It shares no code with the GPU library and
the library never calls it.

The C source (``mace_oracle.c``) implements, in double precision and in the
paper's order:
  * the MAP cost f (eq. (global_obj)) and the agent costs f_i (eq. (local_obj)),
    their gradients, and the proximal cost f_i(z) + ||z - v||^2 / (2 sigma^2)
    (eq. (prox_F));
  * one ICD partial update of an agent (Algorithm 2), with the closed-form
    surrogate step (mode 0) or the exact 1-D minimiser (mode 1);
  * partial-update MACE (Algorithm 1) with the Mann update (eq. (Mann));
  * the exact proximal map by repeated passes, and the centralised ICD baseline
    (Sec. IV-B);
  * the MAP image of the quadratic prior by preconditioned conjugate gradients
    on the normal equations of eq. (global_obj) (an algorithm independent of
    ICD and MACE, for fixed-point checks at sizes a dense solve cannot reach).
The Python side adds partial-update MACE with PnP priors (Algorithm 3, Sec.
III): the agents' data terms alone (prior kind PRIOR_NONE, beta = 0) at
sqrt(N) sigma, and the consensus G_H(v) = H(mean v) with a stand-in denoiser H
(``binomial_smooth``, a linear smoother that is firmly non-expansive).
Reading of the prior (the paper names the Q-GGMRF prior without its formula):
  rho(d) = |d|^p/(p sigma_x^p) / (1 + (|d|/(T sigma_x))^(p-q)); quadratic prior
  rho(d) = d^2/(2 sigma_x^2); 8-neighbour cliques, each unordered pair once;
  beta = 1 (sigma_x carries the scale).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mace_oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "libmace_oracle.so")

MODE_SURROGATE = 0
MODE_EXACT = 1
PRIOR_QUADRATIC = 0
PRIOR_QGGMRF = 1
PRIOR_NONE = 2  # beta = 0: the data term alone (MACE-PnP agents)


def binomial_smooth(x, nx, ny, passes):
    """Stand-in PnP denoiser H: `passes` applications of the 3x3 binomial
    filter (1/4, 1/2, 1/4) along rows, then along columns, with zero values
    outside the image.  Per axis the filter is the symmetric tridiagonal
    matrix tridiag(1/4, 1/2, 1/4), whose eigenvalues 1/2 + 1/2 cos(k pi/(m+1))
    lie in (0, 1); so H is symmetric with spectrum in (0, 1), i.e. firmly
    non-expansive, and it is the proximal map of the quadratic
    phi(x) = x^T (H^-1 - I) x / 2."""
    img = np.asarray(x, dtype=np.float64).reshape(ny, nx)
    for _ in range(int(passes)):
        pad = np.zeros((ny + 2, nx + 2))
        pad[1:-1, 1:-1] = img
        rows = 0.25 * pad[:, :-2] + 0.5 * pad[:, 1:-1] + 0.25 * pad[:, 2:]
        img = 0.25 * rows[:-2, :] + 0.5 * rows[1:-1, :] + 0.25 * rows[2:, :]
    return img.reshape(-1)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no fast-math, OpenMP over agents."""
    if not force and os.path.exists(_LIB):
        return _LIB
    os.makedirs(_LIB_DIR, exist_ok=True)
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                           "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _In(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("n_views", ctypes.c_int32), ("n_ch", ctypes.c_int32),
                ("col_ptr", ctypes.c_void_p), ("row", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("y", ctypes.c_void_p), ("lam", ctypes.c_void_p),
                ("n_agents", ctypes.c_int32), ("view_agent", ctypes.c_void_p),
                ("prior_kind", ctypes.c_int32),
                ("sigma_x", ctypes.c_double), ("p", ctypes.c_double), ("q", ctypes.c_double),
                ("T", ctypes.c_double), ("b_edge", ctypes.c_double),
                ("b_diag", ctypes.c_double), ("nz", ctypes.c_int32),
                ("b_axial", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, d, i32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
        L.orc_create.argtypes = [ctypes.POINTER(_In)]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_set_data.argtypes = [vp, vp, vp]
        L.orc_error_sinogram.argtypes = [vp, i32, vp, vp]
        L.orc_prior.argtypes = [vp, vp]
        L.orc_prior.restype = d
        L.orc_data.argtypes = [vp, i32, vp]
        L.orc_data.restype = d
        L.orc_cost.argtypes = [vp, i32, vp, vp, d]
        L.orc_cost.restype = d
        L.orc_gradient.argtypes = [vp, i32, vp, vp]
        L.orc_icd_pass.argtypes = [vp, i32, d, vp, vp, vp, vp, i32, d, vp]
        L.orc_icd_pass.restype = i32
        L.orc_mace_solve.argtypes = [vp, d, d, i32, i32, d, vp, vp, i32, d, vp, vp, vp]
        L.orc_mace_solve.restype = i32
        L.orc_prox.argtypes = [vp, i32, d, vp, vp, i32, d, i32]
        L.orc_prox.restype = i32
        L.orc_centralized_icd.argtypes = [vp, vp, i32, d, i32]
        L.orc_centralized_icd.restype = i32
        L.orc_map_cg.argtypes = [vp, vp, i32, d, vp]
        L.orc_map_cg.restype = i32
        L.orc_num_threads.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def num_threads() -> int:
    return int(_load().orc_num_threads())


class Oracle:
    """One problem: geometry, A (CSC), data y/Lambda, partition and prior.

    Volumes: nz slices of nx x ny pixels measured by the same 2-D matrix,
    y / lam of shape [nz * n_views * n_ch] (slice-major), images of shape
    [nz * nx * ny]; b_axial weights the cliques between a voxel and the ones
    above and below it.  nz = 1 (default) is the 2-D problem."""

    def __init__(self, nx, ny, n_views, n_ch, col_ptr, row, val, y, lam, view_agent,
                 prior_kind, sigma_x, p=2.0, q=2.0, T=1.0, b_edge=None, b_diag=None, nz=1,
                 b_axial=0.0):
        L = _load()
        if b_edge is None:
            b_edge = 1.0 / (4.0 + 2.0 * np.sqrt(2.0))
        if b_diag is None:
            b_diag = 1.0 / (4.0 * np.sqrt(2.0) + 4.0)
        self._keep = [np.ascontiguousarray(col_ptr, dtype=np.int64),
                      np.ascontiguousarray(row, dtype=np.int32),
                      np.ascontiguousarray(val, dtype=np.float32),
                      np.ascontiguousarray(y, dtype=np.float32),
                      np.ascontiguousarray(lam, dtype=np.float32),
                      np.ascontiguousarray(view_agent, dtype=np.int32)]
        cp, rw, vl, yy, ll, va = self._keep
        self.nx, self.ny, self.n_views, self.n_ch = int(nx), int(ny), int(n_views), int(n_ch)
        self.nz = int(nz)
        self.n = self.nx * self.ny * self.nz
        self.n_rows = self.n_views * self.n_ch * self.nz
        if yy.size != self.n_rows or ll.size != self.n_rows:
            raise ValueError("y / lam need nz * n_views * n_ch entries")
        self.N = int(va.max()) + 1
        inp = _In(self.nx, self.ny, self.n_views, self.n_ch, _p(cp), _p(rw), _p(vl), _p(yy),
                  _p(ll), self.N, _p(va), int(prior_kind), float(sigma_x), float(p), float(q),
                  float(T), float(b_edge), float(b_diag), self.nz, float(b_axial))
        # held by the object: at interpreter exit the module's globals may
        # already be cleared when __del__ runs
        self._destroy = L.orc_destroy
        self._h = L.orc_create(ctypes.byref(inp))
        if not self._h:
            raise ValueError("oracle: bad problem description")
        # the C state copies everything it needs
        self._keep = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    def set_data(self, y, lam):
        yy = np.ascontiguousarray(y, dtype=np.float32)
        ll = np.ascontiguousarray(lam, dtype=np.float32)
        _load().orc_set_data(self._h, _p(yy), _p(ll))

    # ---- objective pieces ----
    def error_sinogram(self, x, agent=-1, e=None):
        xd = np.ascontiguousarray(x, dtype=np.float64)
        if e is None:
            e = np.zeros(self.n_rows)
        _load().orc_error_sinogram(self._h, int(agent), _p(xd), _p(e))
        return e

    def prior(self, x):
        return float(_load().orc_prior(self._h, _p(np.ascontiguousarray(x, dtype=np.float64))))

    def cost(self, x, agent=-1, v=None, sigma=0.0):
        xd = np.ascontiguousarray(x, dtype=np.float64)
        vd = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        return float(_load().orc_cost(self._h, int(agent), _p(xd), _p(vd), float(sigma)))

    def gradient(self, x, agent=-1):
        xd = np.ascontiguousarray(x, dtype=np.float64)
        g = np.empty(self.n)
        _load().orc_gradient(self._h, int(agent), _p(xd), _p(g))
        return g

    # ---- Algorithm 2 ----
    def icd_pass(self, agent, sigma, v, z, e, order=None, mode=MODE_SURROGATE,
                 trace=False, relax=1.0):
        """One ICD pass, in place on z (float64 [n]) and e (float64 [n_rows]).
        relax scales each coordinate step (1 = Algorithm 2)."""
        assert z.dtype == np.float64 and z.flags.c_contiguous
        assert e.dtype == np.float64 and e.flags.c_contiguous
        vd = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        od = None if order is None else np.ascontiguousarray(order, dtype=np.int64)
        tr = np.empty(self.n) if trace else None
        _load().orc_icd_pass(self._h, int(agent), float(sigma), _p(vd), _p(z), _p(e), _p(od),
                             int(mode), float(relax), _p(tr))
        return tr

    # ---- Algorithm 1 ----
    def mace_solve(self, rho, sigma, max_iters, tol=0.0, sweeps=1, w_init=None, order=None,
                   mode=MODE_SURROGATE, relax=1.0):
        """Returns dict(x, w, X, resid, iters)."""
        w = (np.zeros(self.N * self.n) if w_init is None
             else np.ascontiguousarray(w_init, dtype=np.float64).reshape(-1).copy())
        X = np.empty(self.N * self.n)
        x = np.empty(self.n)
        res = np.zeros(max(1, int(max_iters)))
        od = None if order is None else np.ascontiguousarray(order, dtype=np.int64)
        k = _load().orc_mace_solve(self._h, float(rho), float(sigma), int(sweeps),
                                   int(max_iters), float(tol), _p(w), _p(od), int(mode),
                                   float(relax), _p(x), _p(X), _p(res))
        return dict(x=x, w=w.reshape(self.N, self.n), X=X.reshape(self.N, self.n),
                    resid=res[:k], iters=int(k))

    # ---- Algorithm 3 (partial-update MACE with PnP priors) ----
    def mace_pnp_solve(self, rho, sigma, max_iters, h_passes, sweeps=1, order=None,
                       relax=1.0):
        """Algorithm 3 with F of eq. (FG_PnP): each agent's partial update is
        `sweeps` ICD passes on its data term alone (the oracle must be built
        with prior_kind PRIOR_NONE) at sqrt(N) sigma, starting from its
        previous state; G_H(w) = H(mean_i w_i) for every agent, H =
        binomial_smooth(., h_passes); w^0 = 0, X^0 = G_H(w^0).  Returns
        dict(x = H(mean w), w, X, resid) with the residual of Algorithm 1's
        statistic, ||X^{k+1} - G_H(w^k)|| / ||w^k||."""
        N, n = self.N, self.n

        def H(v):
            return binomial_smooth(v, self.nx, self.ny, h_passes)

        w = np.zeros((N, n))
        X = np.tile(H(w.mean(axis=0)), (N, 1))
        e = [self.error_sinogram(X[i], agent=i) for i in range(N)]
        sp = float(sigma) * np.sqrt(N)
        resid = []
        for _ in range(int(max_iters)):
            g = H(w.mean(axis=0))            # one copy of G_H(w^k)
            v = 2.0 * g[None, :] - w         # v^k = (2 G_H - I) w^k
            for i in range(N):
                for _ in range(int(sweeps)):
                    self.icd_pass(i, sp, v[i], X[i], e[i], order=order, relax=relax)
            num = np.linalg.norm(X - g[None, :])
            den = np.linalg.norm(w)
            if den == 0.0:
                den = np.linalg.norm(X)
            resid.append(num / den if den > 0 else 0.0)
            w = rho * (2.0 * X - v) + (1.0 - rho) * w
        return dict(x=H(w.mean(axis=0)), w=w, X=X, resid=np.array(resid))

    def prox(self, agent, sigma, v, z0=None, max_passes=100000, rtol=1e-14,
             mode=MODE_EXACT):
        """Exact F_i(v) (eq. (prox_F)) by ICD passes to convergence."""
        vd = np.ascontiguousarray(v, dtype=np.float64)
        z = np.zeros(self.n) if z0 is None else np.array(z0, dtype=np.float64)
        it = _load().orc_prox(self._h, int(agent), float(sigma), _p(vd), _p(z),
                              int(max_passes), float(rtol), int(mode))
        return z, int(it)

    def map_cg(self, x0=None, max_iters=100000, rtol=1e-13):
        """MAP image for the quadratic prior: the normal equations
        (A^T Lambda A + L_b / sigma_x^2) x = A^T Lambda y of eq. (global_obj)
        solved by Jacobi-preconditioned conjugate gradients.  Returns
        (x, iterations, ||b - H x|| / ||b||)."""
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        rr = np.zeros(1)
        it = _load().orc_map_cg(self._h, _p(x), int(max_iters), float(rtol), _p(rr))
        if it < 0:
            raise ValueError("map_cg needs the quadratic prior")
        return x, int(it), float(rr[0])

    def centralized_icd(self, x0=None, max_passes=100000, rtol=1e-14, mode=MODE_EXACT):
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        it = _load().orc_centralized_icd(self._h, _p(x), int(max_passes), float(rtol),
                                         int(mode))
        return x, int(it)
