"""GPU tests of the launch-configuration autotuner.

The tuner times candidate (super-voxel side, rows per agent) pairs on a
synthetic scan and keeps the fastest.  Checked here: the table covers the
super-voxel sides 4 and 8 (compact records) and 16 and 32 (general records),
the choice is the fastest finite candidate, a second call
is served from the cache, and a system loaded with sv_size = -1 runs the
chosen configuration and still reaches the MAP image of the quadratic prior
(dense Cholesky, NRMSE <= 1e-4 -- every candidate has the same fixed point).
"""
import time

import numpy as np
import pytest

import mace_inputs as mi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1911_09278_amd as lib
    return lib


def test_autotune_choice_cache_and_fixed_point(m):
    from tests import dense_ref as dr
    g = mi.Geometry(64, 64, 90, 96)
    N = 4
    cp, row, val = mi.system_matrix(g)
    print("autotune 64x64, 90 views, 4 agents", flush=True)
    t0 = time.perf_counter()
    res = m.autotune(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, iters=4)
    t1 = time.perf_counter()
    print(res, f"{t1 - t0:.2f} s", flush=True)
    table = res["table"]
    # sides 4 and 8 in the compact records, 16 and 32 in the general ones
    assert {(r["sv_size"], r["format"]) for r in table} == {(4, 1), (8, 1), (16, 2), (32, 2)}
    ok = [r for r in table if r["status"] == m.MACE_OK]
    assert ok and all(np.isfinite(r["residual"]) for r in ok)
    fastest = min(ok, key=lambda r: r["ms_per_iter"])
    assert (res["sv_size"], res["rows_per_agent"]) == (fastest["sv_size"], fastest["rows_per_agent"])
    # cached: same answer, no new measurements
    res2 = m.autotune(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, iters=4)
    t2 = time.perf_counter()
    assert (res2["sv_size"], res2["rows_per_agent"]) == (res["sv_size"], res["rows_per_agent"])
    assert res2["table"] == table
    assert t2 - t1 < 0.5 * (t1 - t0)
    # a system loaded with sv_size = -1 runs the tuned configuration
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=-1)
    cfg = sysm.config
    assert (cfg["sv_size"], cfg["rows_per_agent"], cfg["format"]) == \
        (res["sv_size"], res["rows_per_agent"], res["format"])
    s = mi.scan(g, 1912)
    sx, sigma = 0.001, 5e-4
    x, info = sysm.solve(s.y, s.lam, m.make_prior(0, sx), 0.8, sigma, 6000, tol=1e-6)
    print("iters", info.iters, "resid", info.residual, flush=True)
    assert info.status == m.MACE_OK
    A = dr.dense_A(g, cp, row, val)
    xmap = dr.map_quadratic(A, s.lam.astype(np.float64), s.y.astype(np.float64),
                            dr.laplacian(g.nx, g.ny), sx)
    err = float(np.linalg.norm(x - xmap) / np.linalg.norm(xmap))
    print("nrmse", err, flush=True)
    assert err <= 1e-4
