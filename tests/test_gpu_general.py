"""GPU parity of the general record format (any CSC matrix) against the oracle.

The general records take what the compact ones cannot: several nonzeros of
a column in one view (channel spacing below the pixel width over sqrt 2,
e.g. Table I's 2560-channel scan of a 512-pixel image: 0.4 mm channels for
1 mm pixels), more than 128 views per agent (one agent holding all 720
views: the centralised single-node case of Sec. IV-B), and super-voxels of
16 and 32 pixels.

1. Sequential schedule: the trajectory equals the oracle's, run in the GPU's
   visiting order with the same coordinate rule, element by element
   (5e-5 of max|x|; the FP32 error budget of test_gpu_parity).
2. Concurrent schedule: the fixed point equals the MAP image (the oracle's
   conjugate-gradient solve, quadratic prior) to NRMSE 1e-4.
3. The general records on a matrix the compact ones also take give the same
   trajectory as the compact records.
"""
import numpy as np
import pytest

import mace_inputs as mi
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1911_09278_amd as lib
    return lib


def _setup(g, seed, N, kind, sx, q=2.0):
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, seed)
    va = mi.interleaved_partition(g.n_views, N)
    O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, s.y, s.lam, va, kind,
                      sx, 2.0, q, 1.0)
    return (cp, row, val), s, O


def _nrmse(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


SEQ_CASES = [
    # geometry, N, prior kind, sigma_x, q, sigma, sv_size, iterations
    (mi.Geometry(32, 32, 48, 113, pix=1.0, chan=0.4), 2, 1, 0.002, 1.2, 0.001, 4, 4),
    (mi.Geometry(30, 28, 40, 140, pix=1.0, chan=0.3), 2, 0, 0.002, 2.0, 0.001, 8, 3),
    (mi.Geometry(24, 24, 720, 40), 1, 1, 0.002, 1.2, 0.001, 4, 3),      # 720 views, one agent
    (mi.Geometry(40, 40, 180, 60), 2, 1, 0.002, 1.2, 0.001, 16, 3),     # 16-pixel SVs, ragged
    (mi.Geometry(48, 40, 96, 72), 4, 0, 0.002, 2.0, 0.001, 32, 3),      # 32-pixel SVs, ragged
    (mi.Geometry(24, 24, 4, 8), 4, 1, 0.003, 1.2, 0.003, 8, 4),         # empty columns
]


@pytest.mark.parametrize("case", SEQ_CASES,
                         ids=lambda c: f"{c[0].nx}x{c[0].ny}v{c[0].n_views}c{c[0].chan}_N{c[1]}_S{c[6]}")
def test_general_sequential_trajectory_matches_oracle(m, case):
    g, N, kind, sx, q, sigma, S, iters = case
    (cp, row, val), s, O = _setup(g, 201 + g.nx, N, kind, sx, q)
    print(f"case {g} N={N} S={S}", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=S,
                    rows_per_agent=1, format=2)
    assert sysm.config["format"] == 2 and sysm.config["sv_size"] == S
    prior = m.make_prior(kind, sx, 2.0, q, 1.0)
    x, info = sysm.solve(s.y, s.lam, prior, 0.8, sigma, iters)
    w, X = sysm.state()
    order = sysm.visit_order()
    ref = O.mace_solve(0.8, sigma, iters, order=order, mode=oracle.MODE_SURROGATE)
    scale = np.abs(ref["x"]).max()
    assert np.all(np.isfinite(x))
    assert np.abs(X - ref["X"]).max() <= 5e-5 * scale, np.abs(X - ref["X"]).max() / scale
    assert np.abs(x - ref["x"]).max() <= 5e-5 * scale
    assert abs(info.residual - ref["resid"][-1]) <= 1e-3 * ref["resid"][-1] + 1e-7
    # the kept error sinogram is y - A X_i
    e = sysm.error_sinogram()
    va = mi.interleaved_partition(g.n_views, N)
    for i in range(N):
        ei = O.error_sinogram(X[i].astype(np.float64), agent=i)
        r = np.where(va[np.arange(g.n_rows) // g.n_channels] == i)[0]
        assert np.abs(e[r] - ei[r]).max() <= 1e-4 * np.abs(s.y).max()


FIXED_CASES = [
    (mi.Geometry(32, 32, 48, 113, pix=1.0, chan=0.4), 2, 4),   # 0.4 mm channels
    (mi.Geometry(24, 24, 720, 40), 1, 4),                      # one agent, 720 views
    (mi.Geometry(128, 128, 96, 184), 4, 16),                   # 16-pixel super-voxels
]


@pytest.mark.parametrize("case", FIXED_CASES,
                         ids=lambda c: f"{c[0].nx}x{c[0].ny}v{c[0].n_views}c{c[0].chan}_N{c[1]}_S{c[2]}")
def test_general_concurrent_fixed_point_is_the_map(m, case):
    g, N, S = case
    sx, sigma = 0.001, 5e-4
    (cp, row, val), s, O = _setup(g, 61, N, 0, sx)
    xmap, _, rel = O.map_cg(rtol=1e-13)
    assert rel <= 1e-12
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=S, format=2)
    assert sysm.config["rows_per_agent"] > 1
    sysm.set_relaxation(0.5)
    x, info = sysm.solve(s.y, s.lam, m.make_prior(0, sx), 0.8, sigma, 20000, tol=1e-8)
    print(f"{g} N={N} S={S}: {info.iters} iterations, r {info.residual:.2e}, "
          f"nrmse {_nrmse(x, xmap):.2e}", flush=True)
    assert info.status == m.MACE_OK
    assert _nrmse(x, xmap) <= 1e-4


def test_general_records_match_compact_records(m):
    """Same matrix (1 mm channels, 45 views per agent), same sequential
    schedule: the two record formats give the same iterates up to FP32
    rounding of the summation order."""
    g = mi.Geometry(40, 40, 180, 60)
    N = 4
    (cp, row, val), s, O = _setup(g, 77, N, 1, 0.002, 1.2)
    prior = m.make_prior(1, 0.002, 2.0, 1.2, 1.0)
    xs = {}
    for fmt in (1, 2):
        sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=8,
                        rows_per_agent=1, format=fmt)
        xs[fmt], _ = sysm.solve(s.y, s.lam, prior, 0.8, 0.001, 5)
        sysm.close()
    scale = np.abs(xs[1]).max()
    assert np.abs(xs[1] - xs[2]).max() <= 5e-5 * scale


def _dense_columns(nx, ny, n_views, n_ch, seed):
    """A synthetic CSC matrix whose every column has a nonzero in every
    channel of every view (values in [0.05, 0.35)), with Poisson data from
    a random image: far more nonzeros per view than a ray geometry gives,
    on bands of only n_ch channels."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n, rows = nx * ny, n_views * n_ch
    cp = np.arange(n + 1, dtype=np.int64) * rows
    row = np.tile(np.arange(rows, dtype=np.int32), n)
    val = rng.uniform(0.05, 0.35, size=n * rows).astype(np.float32)
    x_true = rng.uniform(0.0, 0.04, size=n)
    A = np.zeros((rows, n))
    A[row, np.repeat(np.arange(n), rows)] = val.astype(np.float64)
    counts = np.maximum(rng.poisson(1e4 * np.exp(-(A @ x_true))), 1).astype(np.float64)
    y = (-np.log(counts / 1e4)).astype(np.float32)
    return (cp, row, val), y, counts.astype(np.float32)


DENSE_CASES = [
    # views, channels, agents: records per (agent, pixel), view slots
    (60, 6, 1),   # 360 entries (read in the pixel loop), 64 slots: staged e in 64 registers
    (45, 6, 1),   # 270 entries, 48 slots: 48 registers
    (60, 6, 2),   # 180 entries (16 per lane in registers), 32 slots: 32 registers
    (45, 4, 1),   # 180 entries, 48 slots: too many beside 16 record registers, e in LDS
]


@pytest.mark.parametrize("case", DENSE_CASES, ids=lambda c: f"v{c[0]}c{c[1]}_N{c[2]}")
def test_general_dense_columns_trajectory_matches_oracle(m, case):
    """Columns with many nonzeros per view and narrow bands: the staged-e
    register variants for long records, against the oracle's trajectory."""
    nv, nc, N = case
    nx = ny = 8
    (cp, row, val), y, lam = _dense_columns(nx, ny, nv, nc, 500 + nv + nc + N)
    va = mi.interleaved_partition(nv, N)
    O = oracle.Oracle(nx, ny, nv, nc, cp, row, val, y, lam, va, 1, 0.002, 2.0, 1.2, 1.0)
    print(f"dense columns {nx}x{ny}, {nv} views x {nc} channels, N={N}", flush=True)
    sysm = m.System(nx, ny, nv, nc, cp, row, val, N, sv_size=4, rows_per_agent=1, format=2)
    assert sysm.config["format"] == 2
    prior = m.make_prior(1, 0.002, 2.0, 1.2, 1.0)
    x, info = sysm.solve(y, lam, prior, 0.8, 0.002, 4)
    w, X = sysm.state()
    ref = O.mace_solve(0.8, 0.002, 4, order=sysm.visit_order(), mode=oracle.MODE_SURROGATE)
    scale = np.abs(ref["x"]).max()
    assert np.all(np.isfinite(x))
    assert np.abs(X - ref["X"]).max() <= 5e-5 * scale, np.abs(X - ref["X"]).max() / scale
    assert np.abs(x - ref["x"]).max() <= 5e-5 * scale
    assert abs(info.residual - ref["resid"][-1]) <= 1e-3 * ref["resid"][-1] + 1e-7
