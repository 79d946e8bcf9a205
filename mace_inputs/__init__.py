"""Seeded synthetic CT inputs shared by the oracle, the tests and the benchmark.

This package generates *inputs* only -- the scanner's sparse system matrix,
ellipse phantoms and Poisson-noise measurements -- and holds none of the
reconstruction method's arithmetic.  It stands in for the paper's real CT
datasets (Table I: 2-D scans of 512x512 images with 720-1024 views), which are
not available; shapes follow those scans.

Conventions
  * 2-D parallel beam, square pixels of 1 mm, channel spacing 1 mm, views at
    theta_k = k*pi/n_views (k = 0..n_views-1).
  * Row index r = k * n_channels + d (view-major), column index = raster pixel
    index s = i * nx + j (row i from the top).
  * A is returned in compressed sparse column form: col_ptr int64[n+1],
    row int32[nnz] (ascending within a column), val float32[nnz] (mm).
  * Measurements follow the usual transmission model: counts ~ Poisson(I0 *
    exp(-(A x_true)_r)), clamped to >= 1; y_r = -ln(counts_r / I0) and the
    inverse-variance weight is lambda_r = counts_r (the diagonal of Lambda in
    the MAP cost, Sec. II-A).
  * Ellipse phantom: 10 ellipses, centres uniform in the disc of radius 0.7R,
    semi-axes U(0.05R, 0.35R), angle U(0, pi), attenuation
    U(0.01, 0.05) * (64 / n) mm^-1 (the 64/n factor keeps line integrals in
    the same range at every image size), R = n * pix / 2.  All draws -- the
    phantom's, then the Poisson counts -- come from one numpy PCG64 generator.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sysmat.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "libmace_inputs.so")


def build(force: bool = True) -> str:
    """Compile the C generator with gcc (OpenMP). Returns the library path."""
    if not force and os.path.exists(_LIB):
        return _LIB
    os.makedirs(_LIB_DIR, exist_ok=True)
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("n_views", ctypes.c_int32), ("n_ch", ctypes.c_int32),
                ("pix", ctypes.c_double), ("chan", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.mi_sysmat_colptr.argtypes = [P(_Geom), P(ctypes.c_int64)]
        lib.mi_sysmat_colptr.restype = ctypes.c_int64
        lib.mi_sysmat_fill.argtypes = [P(_Geom), P(ctypes.c_int64), P(ctypes.c_int32),
                                       P(ctypes.c_float)]
        lib.mi_sysmat_fill.restype = ctypes.c_int
        lib.mi_forward_project.argtypes = [P(_Geom), P(ctypes.c_double), P(ctypes.c_double)]
        lib.mi_forward_project.restype = ctypes.c_int
        lib.mi_image_chord.argtypes = [P(_Geom), ctypes.c_int32, ctypes.c_int32]
        lib.mi_image_chord.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    n_views: int
    n_channels: int
    pix: float = 1.0
    chan: float = 1.0

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def n_rows(self) -> int:
        return self.n_views * self.n_channels

    def _c(self) -> _Geom:
        return _Geom(self.nx, self.ny, self.n_views, self.n_channels, self.pix, self.chan)


def system_matrix(g: Geometry):
    """Exact line/pixel intersection lengths in CSC: (col_ptr, row, val)."""
    lib = _load()
    cg = g._c()
    col_ptr = np.empty(g.n + 1, dtype=np.int64)
    nnz = lib.mi_sysmat_colptr(ctypes.byref(cg), _ptr(col_ptr, ctypes.c_int64))
    if nnz < 0:
        raise ValueError(f"bad geometry {g}")
    row = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float32)
    lib.mi_sysmat_fill(ctypes.byref(cg), _ptr(col_ptr, ctypes.c_int64),
                       _ptr(row, ctypes.c_int32), _ptr(val, ctypes.c_float))
    return col_ptr, row, val


def forward_project(g: Geometry, x: np.ndarray) -> np.ndarray:
    """A @ x in float64 using the float32-rounded entries of A (data synthesis only)."""
    lib = _load()
    xd = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    if xd.size != g.n:
        raise ValueError("x has the wrong size")
    out = np.empty(g.n_rows, dtype=np.float64)
    lib.mi_forward_project(ctypes.byref(g._c()), _ptr(xd, ctypes.c_double),
                           _ptr(out, ctypes.c_double))
    return out


def image_chord(g: Geometry, k: int, d: int) -> float:
    """Exact length of ray (k, d) through the whole image rectangle."""
    return float(_load().mi_image_chord(ctypes.byref(g._c()), int(k), int(d)))


def phantom(g: Geometry, rng: np.random.Generator, n_ellipses: int = 10) -> np.ndarray:
    """Sum of random ellipses (float64 image, raster order, mm^-1)."""
    R = 0.5 * min(g.nx, g.ny) * g.pix
    scale = 64.0 / min(g.nx, g.ny)
    xs = (np.arange(g.nx) - 0.5 * (g.nx - 1)) * g.pix
    ys = (0.5 * (g.ny - 1) - np.arange(g.ny)) * g.pix
    X, Y = np.meshgrid(xs, ys)
    img = np.zeros((g.ny, g.nx), dtype=np.float64)
    for _ in range(n_ellipses):
        r = 0.7 * R * np.sqrt(rng.uniform())
        phi = rng.uniform(0.0, 2.0 * np.pi)
        cx, cy = r * np.cos(phi), r * np.sin(phi)
        a = rng.uniform(0.05 * R, 0.35 * R)
        b = rng.uniform(0.05 * R, 0.35 * R)
        ang = rng.uniform(0.0, np.pi)
        mu = rng.uniform(0.01, 0.05) * scale
        dx, dy = X - cx, Y - cy
        u = dx * np.cos(ang) + dy * np.sin(ang)
        v = -dx * np.sin(ang) + dy * np.cos(ang)
        img += mu * ((u / a) ** 2 + (v / b) ** 2 <= 1.0)
    return img.reshape(-1)


@dataclass
class Scan:
    y: np.ndarray        # float32 [n_rows]
    lam: np.ndarray      # float32 [n_rows]
    x_true: np.ndarray   # float64 [n]


def scan(g: Geometry, seed: int, I0: float = 1e4) -> Scan:
    """Phantom + Poisson transmission data from one PCG64(seed) stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x_true = phantom(g, rng)
    p = forward_project(g, x_true)
    counts = rng.poisson(I0 * np.exp(-p)).astype(np.float64)
    counts = np.maximum(counts, 1.0)
    y = (-np.log(counts / I0)).astype(np.float32)
    lam = counts.astype(np.float32)
    return Scan(y=y, lam=lam, x_true=x_true)


# Named workloads (image, views, channels, agents, prior, solver settings).
# Prior weights: 8-neighbour, edge 1/(4+2*sqrt 2), diagonal 1/(4*sqrt 2+4).
B_EDGE = 1.0 / (4.0 + 2.0 * np.sqrt(2.0))
B_DIAG = 1.0 / (4.0 * np.sqrt(2.0) + 4.0)


@dataclass(frozen=True)
class Workload:
    name: str
    geom: Geometry
    n_agents: int
    prior_kind: int          # 0 quadratic, 1 q-GGMRF
    sigma_x: float
    p: float
    q: float
    T: float
    sigma: float
    rho: float
    iters: int
    seed: int


WORKLOADS = {
    "plain64": Workload("plain64", Geometry(64, 64, 90, 96), 4, 0, 0.02, 2.0, 2.0, 1.0,
                        0.05, 0.8, 100, 1912),
    "scan512": Workload("scan512", Geometry(512, 512, 720, 736), 16, 1, 0.01, 2.0, 1.2, 1.0,
                        0.05, 0.8, 60, 1913),
    "slices512": Workload("slices512", Geometry(512, 512, 720, 736), 16, 1, 0.01, 2.0, 1.2,
                          1.0, 0.05, 0.8, 60, 1914000),
    "scan1024": Workload("scan1024", Geometry(1024, 1024, 1440, 1472), 32, 1, 0.01, 2.0, 1.2,
                         1.0, 0.05, 0.8, 60, 1915),
    "serve256": Workload("serve256", Geometry(256, 256, 360, 368), 8, 1, 0.01, 2.0, 1.2, 1.0,
                         0.05, 0.8, 60, 1916),
}


def interleaved_partition(n_views: int, n_agents: int) -> np.ndarray:
    """View k -> agent k mod N (interleaved view subsets, Sec. II-A)."""
    return (np.arange(n_views) % n_agents).astype(np.int32)
