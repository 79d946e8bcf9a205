"""GPU parity of the batched solve (several scans of one geometry per launch).

1. Sequential schedule: with one super-voxel per (scan, agent) in flight, each
   scan of a batch follows exactly the iterates of its own single-scan solve,
   which the oracle run in the same visiting order reproduces.
2. Concurrent schedule with per-scan stopping: every scan of the batch reaches
   its own MAP (quadratic prior: dense Cholesky) while the scans stop at
   different iterations; an all-zero scan is done after one iteration.
3. The captured iteration graph and the eager launches (timing mode) give the
   same iterates.
4. FP16 matrix values with an FP32 tail: each scan of a batch follows its own
   single-scan solve through the precision switch.
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


def _nrmse(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_sequential_batch_follows_single_scans(m):
    g = mi.Geometry(32, 32, 64, 48)
    N, sx, sigma, iters = 4, 0.002, 0.002, 5
    cp, row, val = mi.system_matrix(g)
    va = mi.interleaved_partition(g.n_views, N)
    scans = [mi.scan(g, seed) for seed in (11, 12, 13)]
    print("sequential batch of 3, 32x32 N=4", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=4,
                    rows_per_agent=1)
    prior = m.make_prior(1, sx, 2.0, 1.2, 1.0)
    xs, infos = sysm.solve_batch([s.y for s in scans], [s.lam for s in scans], prior, 0.8,
                                 sigma, iters)
    order = sysm.visit_order()
    for s, x, info in zip(scans, xs, infos):
        alone, _ = sysm.solve(s.y, s.lam, prior, 0.8, sigma, iters)
        assert np.abs(x - alone).max() <= 1e-6 * np.abs(alone).max()
        O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, s.y, s.lam, va, 1,
                          sx, 2.0, 1.2, 1.0)
        ref = O.mace_solve(0.8, sigma, iters, order=order, mode=oracle.MODE_SURROGATE)
        assert np.abs(x - ref["x"]).max() <= 5e-5 * np.abs(ref["x"]).max()
        assert info.iters == iters and info.status == m.MACE_OK


def test_sequential_fp16_batch_with_fp32_tail_follows_single_scans(m):
    """FP16 matrix values with a two-iteration FP32 tail: every scan of a
    batch follows its own single-scan solve, through the precision switch
    (e-refresh with FP32 A, theta2 rebuilt)."""
    g = mi.Geometry(32, 32, 64, 48)
    N, sx, sigma, iters = 4, 0.002, 0.002, 5
    cp, row, val = mi.system_matrix(g)
    scans = [mi.scan(g, seed) for seed in (14, 15, 16)]
    print("sequential FP16 batch of 3 with FP32 tail, 32x32 N=4", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=4,
                    rows_per_agent=1, precision=1, fp32_tail_iters=2)
    prior = m.make_prior(1, sx, 2.0, 1.2, 1.0)
    xs, infos = sysm.solve_batch([s.y for s in scans], [s.lam for s in scans], prior, 0.8,
                                 sigma, iters)
    fp32 = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=4,
                    rows_per_agent=1)
    for s, x, info in zip(scans, xs, infos):
        alone, _ = sysm.solve(s.y, s.lam, prior, 0.8, sigma, iters)
        assert np.abs(x - alone).max() <= 1e-6 * np.abs(alone).max()
        assert info.iters == iters and info.status == m.MACE_OK
        # FP16 values for 3 iterations, then FP32: close to the FP32 path
        x32, _ = fp32.solve(s.y, s.lam, prior, 0.8, sigma, iters)
        err = np.abs(x - x32).max() / np.abs(x32).max()
        print("max rel. difference to FP32", err, flush=True)
        assert 0 < err <= 2e-3


def test_concurrent_batch_per_scan_stopping(m):
    from tests import dense_ref as dr
    g = mi.Geometry(32, 32, 64, 48)
    N, sx, sigma = 4, 0.001, 0.001
    cp, row, val = mi.system_matrix(g)
    A = dr.dense_A(g, cp, row, val)
    L = dr.laplacian(g.nx, g.ny)
    scans = [mi.scan(g, seed) for seed in (21, 22)]
    ys = [scans[0].y, np.zeros_like(scans[0].y), scans[1].y]
    lams = [scans[0].lam, scans[0].lam, scans[1].lam]
    print("concurrent batch of 3 with a zero scan, 32x32 N=4", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N)
    sysm.set_relaxation(0.5)
    xs, infos = sysm.solve_batch(ys, lams, m.make_prior(0, sx), 0.8, sigma, 4000, tol=1e-6)
    for i, info in enumerate(infos):
        print(i, "iters", info.iters, "resid", info.residual, flush=True)
        assert info.status == m.MACE_OK
        assert info.residual < 1e-6
    # the zero scan: x = 0 is the fixed point and r_0 = 0
    assert infos[1].iters == 1
    assert np.all(xs[1] == 0.0)
    assert infos[0].iters > 1 and infos[2].iters > 1
    for i in (0, 2):
        xmap = dr.map_quadratic(A, lams[i].astype(np.float64), ys[i].astype(np.float64), L, sx)
        assert _nrmse(xs[i], xmap) <= 1e-4, _nrmse(xs[i], xmap)


def test_graph_replay_equals_eager_launches(m):
    g = mi.Geometry(36, 36, 90, 56)
    N = 2
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, 5)
    print("graph vs eager, 36x36 N=2", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, rows_per_agent=1)
    prior = m.make_prior(1, 0.01, 2.0, 1.2, 1.0)
    # graph path (timing off); tol > 0 makes the host read the residual
    # between replays
    xg, ig = sysm.solve(s.y, s.lam, prior, 0.8, 2e-4, 7, tol=1e-12)
    wg, Xg = sysm.state()
    sysm.set_timing(True)
    xe, ie = sysm.solve(s.y, s.lam, prior, 0.8, 2e-4, 7, tol=1e-12)
    we, Xe = sysm.state()
    assert ie.sweep_launches == 7 * 4
    assert ig.iters == ie.iters == 7
    assert np.array_equal(xg, xe)
    assert np.array_equal(Xg, Xe)
    assert np.array_equal(wg, we)
    # and a second graph solve replays the cached graph to the same result
    sysm.set_timing(False)
    xg2, _ = sysm.solve(s.y, s.lam, prior, 0.8, 2e-4, 7, tol=1e-12)
    assert np.array_equal(xg, xg2)
