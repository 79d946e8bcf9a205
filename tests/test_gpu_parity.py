"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

1. Sequential schedule (one super-voxel of an agent at a time): the GPU visits
   pixels in exactly the order mace_visit_order reports, so its trajectory must
   match the oracle run in that order with the same (surrogate) coordinate rule,
   element by element, to FP32 accuracy.
2. Concurrent schedule (the launch configuration of the benchmark): the fixed
   point must match the oracle's / the dense MAP within the FP32 tolerance
   NRMSE <= 1e-4.
3. Properties that hold at any size: the kept error sinogram equals y - A X_i,
   x = mean_i w_i, everything finite.

Tolerances (FP32 path, unit roundoff u = 6e-8): a pass updates each pixel once
from sums of ~60-90 terms, so one pass carries relative error ~1e2 u; over k
passes of a contraction the error stays within ~k * 1e2 u ~ 1e-5 relative to
max|x| for k <= 10; the trajectory bar below is 5e-5 * max|x| (a 5x margin).
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


def _setup(geom, seed, N, kind, sx, q=2.0, T=1.0):
    cp, row, val = mi.system_matrix(geom)
    s = mi.scan(geom, seed)
    va = mi.interleaved_partition(geom.n_views, N)
    O = oracle.Oracle(geom.nx, geom.ny, geom.n_views, geom.n_channels, cp, row, val, s.y, s.lam,
                      va, kind, sx, 2.0, q, T)
    return (cp, row, val), s, va, O


def _nrmse(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


SEQ_CASES = [
    # geometry, N, prior kind, sigma_x, q, sigma, sv_size, iterations, relaxation
    (mi.Geometry(32, 32, 64, 48), 4, 0, 0.001, 2.0, 0.001, 4, 6, 1.0),    # 16 views/agent: 1 slot
    (mi.Geometry(42, 38, 180, 64), 4, 1, 0.002, 1.2, 0.002, 4, 4, 1.0),  # 45 views/agent, ragged
    (mi.Geometry(24, 24, 100, 40), 2, 1, 0.002, 1.2, 0.002, 8, 3, 1.0),  # 50 views: 4 slots, S = 8
    (mi.Geometry(20, 20, 30, 32), 1, 1, 0.003, 1.5, 0.003, 4, 3, 1.0),   # single agent
    (mi.Geometry(36, 36, 90, 56), 2, 1, 0.01, 1.2, 2e-4, 4, 5, 0.5),     # under-relaxed
    # more than 64 views per agent: the staged e lives in LDS, and large
    # bands take 8 or 4 rows per workgroup
    (mi.Geometry(24, 24, 150, 40), 2, 1, 0.002, 1.2, 0.002, 8, 3, 1.0),  # 75 views: 5 slots, 8 rows
    (mi.Geometry(26, 26, 200, 40), 2, 0, 0.002, 2.0, 0.002, 4, 3, 1.0),  # 100 views: 7 slots, 16 rows
    (mi.Geometry(20, 20, 128, 32), 1, 1, 0.003, 1.5, 0.003, 8, 3, 1.0),  # 128 views: 8 slots (most)
    # 4 views on 8 channels: 24 pixels no ray crosses (empty columns of A),
    # and with one view per agent most of each agent's columns are empty
    (mi.Geometry(24, 24, 4, 8), 4, 1, 0.003, 1.2, 0.003, 4, 4, 1.0),
    (mi.Geometry(24, 24, 4, 8), 2, 0, 0.003, 2.0, 0.003, 8, 4, 1.0),
    # an odd pixel count (399)
    (mi.Geometry(21, 19, 40, 32), 2, 1, 0.003, 1.2, 0.003, 4, 4, 1.0),
    # many agents of one or two views each (45 and 90 agents on 90 views)
    (mi.Geometry(32, 32, 90, 48), 45, 1, 0.002, 1.2, 0.002, 8, 3, 1.0),
    (mi.Geometry(32, 32, 90, 48), 90, 0, 0.002, 2.0, 0.002, 4, 3, 1.0),
]


@pytest.mark.parametrize("case", SEQ_CASES,
                         ids=lambda c: f"{c[0].nx}x{c[0].ny}v{c[0].n_views}_N{c[1]}_k{c[2]}_S{c[6]}_g{c[8]}")
def test_sequential_trajectory_matches_oracle(m, case):
    g, N, kind, sx, q, sigma, S, iters, relax = case
    (cp, row, val), s, va, O = _setup(g, 101 + g.nx, N, kind, sx, q)
    print(f"case {g} N={N} kind={kind} S={S}", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=S,
                    rows_per_agent=1)
    prior = m.make_prior(kind, sx, 2.0, q, 1.0)
    sysm.set_relaxation(relax)
    x, info = sysm.solve(s.y, s.lam, prior, 0.8, sigma, iters)
    w, X = sysm.state()
    order = sysm.visit_order()
    assert np.array_equal(np.sort(order), np.arange(g.n))
    ref = O.mace_solve(0.8, sigma, iters, order=order, mode=oracle.MODE_SURROGATE, relax=relax)
    scale = np.abs(ref["x"]).max()
    assert np.all(np.isfinite(x))
    assert np.abs(X - ref["X"]).max() <= 5e-5 * scale, np.abs(X - ref["X"]).max() / scale
    assert np.abs(w - ref["w"]).max() <= 5e-5 * np.abs(ref["w"]).max()
    assert np.abs(x - ref["x"]).max() <= 5e-5 * scale
    # residual trace: FP64 on both sides from FP32 / FP64 states
    assert info.iters == iters
    assert abs(info.residual - ref["resid"][-1]) <= 1e-3 * ref["resid"][-1] + 1e-7


def test_sequential_two_sweeps_and_warm_start_match_oracle(m):
    """Two ICD passes per partial update (Algorithm 1 with sweeps = 2) from a
    nonzero w^0: the trajectory still matches the oracle."""
    g = mi.Geometry(32, 32, 64, 48)
    N, sx, sigma = 4, 0.002, 0.002
    (cp, row, val), s, va, O = _setup(g, 77, N, 1, sx, 1.2)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, rows_per_agent=1)
    prior = m.make_prior(1, sx, 2.0, 1.2, 1.0)
    rng = np.random.default_rng(5)
    w0 = rng.uniform(0.0, 0.03, N * g.n).astype(np.float32)
    x, info = sysm.solve(s.y, s.lam, prior, 0.8, sigma, 3, sweeps=2, w_init=w0)
    order = sysm.visit_order()
    ref = O.mace_solve(0.8, sigma, 3, sweeps=2, w_init=w0.astype(np.float64), order=order,
                       mode=oracle.MODE_SURROGATE)
    scale = np.abs(ref["x"]).max()
    assert info.iters == 3 and info.equits == 6
    assert np.abs(x - ref["x"]).max() <= 5e-5 * scale, np.abs(x - ref["x"]).max() / scale


def test_prox_single_pass_matches_oracle(m):
    g = mi.Geometry(32, 32, 90, 48)
    N = 3
    (cp, row, val), s, va, O = _setup(g, 7, N, 1, 0.002, 1.2)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, rows_per_agent=1)
    prior = m.make_prior(1, 0.002, 2.0, 1.2, 1.0)
    rng = np.random.default_rng(3)
    v = rng.uniform(0.0, 0.05, g.n).astype(np.float32)
    x0 = rng.uniform(0.0, 0.05, g.n).astype(np.float32)
    for agent in range(N):
        out = sysm.prox(agent, s.y, s.lam, prior, 0.01, v, x0, sweeps=2)
        z = x0.astype(np.float64)
        e = O.error_sinogram(z, agent=agent)
        order = sysm.visit_order()
        for _ in range(2):
            O.icd_pass(agent, 0.01, v.astype(np.float64), z, e, order=order)
        assert np.abs(out - z).max() <= 5e-5 * np.abs(z).max()


def test_concurrent_fixed_point_is_the_map(m):
    """Quadratic prior: the MACE fixed point is the MAP (dense Cholesky)."""
    from tests import dense_ref as dr
    g = mi.Geometry(32, 32, 64, 48)
    N, sx, sigma = 4, 0.001, 0.001
    (cp, row, val), s, va, O = _setup(g, 7, N, 0, sx)
    A = dr.dense_A(g, cp, row, val)
    xmap = dr.map_quadratic(A, s.lam.astype(np.float64), s.y.astype(np.float64),
                            dr.laplacian(g.nx, g.ny), sx)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N)
    sysm.set_relaxation(0.5)
    x, info = sysm.solve(s.y, s.lam, m.make_prior(0, sx), 0.8, sigma, 4000, tol=1e-6)
    print("iters", info.iters, "resid", info.residual, flush=True)
    assert info.status == m.MACE_OK
    assert _nrmse(x, xmap) <= 1e-4, _nrmse(x, xmap)


def test_concurrent_many_views_fixed_point_is_the_map(m):
    """75 views per agent with 8x8 super-voxels: bands too large for 16 rows
    per workgroup, so the concurrent schedule runs smaller workgroups (4
    rows: three of them per CU keep 12 rows resident, against 8 in one
    8-row workgroup); its fixed point is still the MAP (dense Cholesky,
    quadratic prior)."""
    from tests import dense_ref as dr
    g = mi.Geometry(64, 64, 150, 96)
    N, sx, sigma = 2, 0.001, 3e-4
    (cp, row, val), s, va, O = _setup(g, 29, N, 0, sx)
    lds = m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=8)
    # a row of this band takes about 11 KB (75 views of ~10 channels at
    # 12 B), so a workgroup of 4 rows takes more than 40 KB, and 16 rows
    # (176 KB) would not fit in 160 KiB
    assert 40 * 1024 < lds <= 80 * 1024
    A = dr.dense_A(g, cp, row, val)
    xmap = dr.map_quadratic(A, s.lam.astype(np.float64), s.y.astype(np.float64),
                            dr.laplacian(g.nx, g.ny), sx)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=8)
    assert sysm.config["rows_per_agent"] > 1
    sysm.set_relaxation(0.5)
    x, info = sysm.solve(s.y, s.lam, m.make_prior(0, sx), 0.8, sigma, 6000, tol=1e-6)
    print("iters", info.iters, "resid", info.residual, flush=True)
    assert info.status == m.MACE_OK
    assert _nrmse(x, xmap) <= 1e-4, _nrmse(x, xmap)


def test_concurrent_qggmrf_fixed_point(m):
    g = mi.Geometry(40, 40, 96, 60)
    N, sx, sigma = 4, 0.0015, 0.001
    (cp, row, val), s, va, O = _setup(g, 17, N, 1, sx, 1.2)
    # undamped passes diverge here; under-relaxed ones reach the same fixed point
    ref = O.mace_solve(0.8, sigma, 20000, tol=1e-12, relax=0.5)
    assert ref["resid"][-1] < 1e-12
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, refresh_every=100)
    sysm.set_relaxation(0.5)
    x, info = sysm.solve(s.y, s.lam, m.make_prior(1, sx, 2.0, 1.2, 1.0), 0.8, sigma, 10000,
                         tol=1e-7)
    print("iters", info.iters, "resid", info.residual, flush=True)
    assert _nrmse(x, ref["x"]) <= 1e-4, _nrmse(x, ref["x"])


def test_fp16_matrix_fixed_point_and_fp32_tail(m):
    """FP16 matrix values with a per-(agent, pixel) scale: the fixed point is
    within 1e-3 of the oracle's; with the last iterations in FP32 (after an
    error-sinogram refresh) within 1e-4."""
    g = mi.Geometry(40, 40, 96, 60)
    N, sx, sigma = 4, 0.0015, 0.001
    (cp, row, val), s, va, O = _setup(g, 17, N, 1, sx, 1.2)
    ref = O.mace_solve(0.8, sigma, 20000, tol=1e-12, relax=0.5)
    prior = m.make_prior(1, sx, 2.0, 1.2, 1.0)
    h = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, precision=1)
    h.set_relaxation(0.5)
    x16, info = h.solve(s.y, s.lam, prior, 0.8, sigma, 1500)
    print("fp16 nrmse", _nrmse(x16, ref["x"]), "resid", info.residual, flush=True)
    assert _nrmse(x16, ref["x"]) <= 1e-3
    t = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, precision=1,
                 fp32_tail_iters=300)
    t.set_relaxation(0.5)
    xt, info = t.solve(s.y, s.lam, prior, 0.8, sigma, 1800)
    print("fp16 + fp32 tail nrmse", _nrmse(xt, ref["x"]), "resid", info.residual, flush=True)
    assert _nrmse(xt, ref["x"]) <= 1e-4
    assert t.matrix_bytes > h.matrix_bytes  # the tail keeps the FP32 values too


def test_error_sinogram_and_consensus_invariants(m):
    g = mi.Geometry(48, 48, 96, 72)
    N = 4
    (cp, row, val), s, va, O = _setup(g, 23, N, 1, 0.002, 1.2)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N)
    sysm.set_relaxation(0.5)
    x, info = sysm.solve(s.y, s.lam, m.make_prior(1, 0.002, 2.0, 1.2, 1.0), 0.8, 0.002, 7)
    w, X = sysm.state()
    e = sysm.error_sinogram()
    np.testing.assert_allclose(x, w.astype(np.float64).mean(axis=0), atol=1e-6 * np.abs(x).max())
    ref = np.zeros(g.n_rows)
    for i in range(N):
        ei = O.error_sinogram(X[i].astype(np.float64), agent=i)
        r = np.where(va[np.arange(g.n_rows) // g.n_channels] == i)[0]
        ref[r] = ei[r]
    # e accumulates ~ (pixels per ray) FP32 updates per sweep
    assert np.abs(e - ref).max() <= 1e-4 * np.abs(s.y).max()


def test_full_size_scan512(m):
    """512x512, 720 views, 736 channels, 16 agents (the benchmark workload).
    Sequential schedule: one iteration matches the oracle element by element.
    Benchmark schedule: invariants after 3 iterations."""
    w8 = mi.WORKLOADS["scan512"]
    g = w8.geom
    print("building 512x512 system matrix", flush=True)
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, w8.seed)
    va = mi.interleaved_partition(g.n_views, w8.n_agents)
    sigma, sx = 2e-4, w8.sigma_x
    prior = m.make_prior(1, sx, 2.0, w8.q, w8.T)
    print("oracle setup", flush=True)
    O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, s.y, s.lam, va, 1, sx,
                      2.0, w8.q, w8.T)
    seq = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w8.n_agents,
                   rows_per_agent=1)
    seq.set_relaxation(0.5)
    x1, _ = seq.solve(s.y, s.lam, prior, w8.rho, sigma, 1)
    order = seq.visit_order()
    seq.close()
    print("oracle iteration", flush=True)
    ref = O.mace_solve(w8.rho, sigma, 1, order=order, relax=0.5)
    assert np.abs(x1 - ref["x"]).max() <= 5e-5 * np.abs(ref["x"]).max()
    print("benchmark schedule", flush=True)
    con = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w8.n_agents)
    con.set_relaxation(0.5)
    x, info = con.solve(s.y, s.lam, prior, w8.rho, sigma, 3)
    w, X = con.state()
    assert np.all(np.isfinite(x)) and np.isfinite(info.residual)
    np.testing.assert_allclose(x, w.astype(np.float64).mean(axis=0), atol=1e-6 * np.abs(x).max())
    e = con.error_sinogram()
    rng = np.random.default_rng(0)
    for i in rng.choice(w8.n_agents, 3, replace=False):
        ei = O.error_sinogram(X[i].astype(np.float64), agent=int(i))
        r = np.where(va[np.arange(g.n_rows) // g.n_channels] == i)[0]
        assert np.abs(e[r] - ei[r]).max() <= 1e-4 * np.abs(s.y).max()


def test_full_size_scan1024_fp16(m):
    """1024x1024, 1440 views, 1472 channels, 32 agents (the FP16 workload).
    Sequential schedule, FP32 values: one iteration matches the oracle element
    by element.  Benchmark schedule, both run to the workload's stopping
    tolerance r < 1e-4: the FP16 path's result stays within 1e-3 of the FP32
    path's (before any FP32 refinement), and its error sinogram equals
    y - A X_i up to the FP16 rounding of A.  (Early iterates differ by more:
    the transient of the concurrent schedule amplifies the rounding of A, to
    2.2e-3 after 3 iterations; the benchmark's 60-iteration runs differ by
    about 3e-4.  The FP16 path's parity with the oracle's fixed point is in
    test_gpu_fixed_point.)"""
    w = mi.WORKLOADS["scan1024"]
    g = w.geom
    print("building 1024x1024 system matrix", flush=True)
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, w.seed)
    va = mi.interleaved_partition(g.n_views, w.n_agents)
    sigma = 5e-5
    prior = m.make_prior(1, w.sigma_x, 2.0, w.q, w.T)
    seq = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w.n_agents,
                   rows_per_agent=1)
    seq.set_relaxation(0.5)
    x1, _ = seq.solve(s.y, s.lam, prior, w.rho, sigma, 1)
    order = seq.visit_order()
    seq.close()
    print("oracle setup and iteration", flush=True)
    O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, s.y, s.lam, va, 1,
                      w.sigma_x, 2.0, w.q, w.T)
    ref = O.mace_solve(w.rho, sigma, 1, order=order, relax=0.5)
    assert np.abs(x1 - ref["x"]).max() <= 5e-5 * np.abs(ref["x"]).max()
    print("FP16 vs FP32, benchmark schedule", flush=True)
    xs = {}
    for prec in (0, 1):
        sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w.n_agents,
                        precision=prec)
        sysm.set_relaxation(0.5)
        xs[prec], info = sysm.solve(s.y, s.lam, prior, w.rho, sigma, 2000, tol=1e-4)
        print("precision", prec, "iterations", info.iters, "residual", info.residual, flush=True)
        assert info.status == m.MACE_OK and info.residual < 1e-4
        if prec == 1:
            _, X = sysm.state()
            e = sysm.error_sinogram()
            i = 5
            ei = O.error_sinogram(X[i].astype(np.float64), agent=i)
            r = np.where(va[np.arange(g.n_rows) // g.n_channels] == i)[0]
            assert np.abs(e[r] - ei[r]).max() <= 2e-3 * np.abs(s.y).max()
        sysm.close()
    err = _nrmse(xs[1], xs[0].astype(np.float64))
    print("fp16 vs fp32 nrmse", err, flush=True)
    assert err <= 1e-3


def test_diverging_iteration_is_reported_not_converged(m):
    """At 512x512 with 16 agents the iteration diverges for sigma = 3e-3 (the
    stable sigma there is about 2e-4) and its states become NaN.  The solve
    ends with MACE_E_NONFINITE with or without a stopping tolerance, never as
    converged, and the system stays usable."""
    w8 = mi.WORKLOADS["scan512"]
    g = w8.geom
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, w8.seed)
    print("diverging sigma 3e-3 at 512x512 N=16", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w8.n_agents)
    sysm.set_relaxation(0.5)
    prior = m.make_prior(w8.prior_kind, w8.sigma_x, w8.p, w8.q, w8.T)
    for tol in (0.0, 1e-4):
        with pytest.raises(m.MaceError) as e:
            sysm.solve(s.y, s.lam, prior, w8.rho, 3e-3, 120, tol=tol)
        assert e.value.code == m.MACE_E_NONFINITE, (tol, e.value)
    x, info = sysm.solve(s.y, s.lam, prior, w8.rho, 1e-4, 5)
    assert np.all(np.isfinite(x)) and np.isfinite(info.residual) and info.residual > 0


def test_zero_iterations_return_the_initial_consensus(m):
    """max_iters = 0 runs no Mann iteration: x = mean_i w_init (0 without a
    warm start), no iteration counted, and a tolerance cannot have been met
    (MACE_W_MAXITER), for one scan and for a volume."""
    g = mi.Geometry(32, 32, 64, 48)
    N = 4
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, 7)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N)
    prior = m.make_prior(0, 0.002)
    w0 = np.random.default_rng(3).uniform(0.0, 0.03, N * g.n).astype(np.float32)
    x, info = sysm.solve(s.y, s.lam, prior, 0.8, 1e-3, 0, w_init=w0)
    mean = w0.reshape(N, g.n).astype(np.float64).mean(axis=0)
    assert info.iters == 0 and info.status == m.MACE_OK
    assert np.abs(x - mean).max() <= 1e-6 * np.abs(mean).max()
    x, info = sysm.solve(s.y, s.lam, prior, 0.8, 1e-3, 0)
    assert info.iters == 0 and np.all(x == 0.0)
    x, info = sysm.solve(s.y, s.lam, prior, 0.8, 1e-3, 0, tol=1e-3)
    assert info.iters == 0 and info.status == m.MACE_W_MAXITER
    xv, iv = sysm.solve_volume(np.stack([s.y, s.y]), np.stack([s.lam, s.lam]), prior, 0.5, 0.8,
                               1e-3, 0, tol=1e-3)
    assert iv.iters == 0 and iv.status == m.MACE_W_MAXITER and np.all(xv == 0.0)


TINY_CASES = [
    # nx, ny, views, channels, agents: every super-voxel ragged, one-pixel-wide images
    (1, 1, 4, 4, 2), (1, 5, 6, 8, 2), (5, 1, 6, 8, 3), (3, 2, 5, 6, 1), (2, 2, 2, 4, 2),
]


@pytest.mark.parametrize("fmt", [1, 2])
@pytest.mark.parametrize("case", TINY_CASES, ids=lambda c: f"{c[0]}x{c[1]}v{c[2]}c{c[3]}_N{c[4]}")
def test_tiny_images_match_oracle(m, case, fmt):
    """Images of one to six pixels (a single ragged super-voxel, neighbours
    mostly outside the image): the sequential trajectory equals the
    oracle's, in both record formats."""
    nx, ny, nv, nc, N = case
    g = mi.Geometry(nx, ny, nv, nc)
    (cp, row, val), s, va, O = _setup(g, 400 + nx + 7 * ny, N, 1, 0.002, 1.2)
    print(f"tiny {g} N={N} format {fmt}", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, rows_per_agent=1,
                    format=fmt)
    prior = m.make_prior(1, 0.002, 2.0, 1.2, 1.0)
    x, info = sysm.solve(s.y, s.lam, prior, 0.8, 0.002, 4)
    w, X = sysm.state()
    ref = O.mace_solve(0.8, 0.002, 4, order=sysm.visit_order(), mode=oracle.MODE_SURROGATE)
    scale = np.abs(ref["x"]).max()
    assert np.all(np.isfinite(x))
    assert np.abs(X - ref["X"]).max() <= 5e-5 * scale, np.abs(X - ref["X"]).max() / scale
    assert np.abs(x - ref["x"]).max() <= 5e-5 * scale
    assert info.iters == 4
    assert abs(info.residual - ref["resid"][-1]) <= 1e-3 * ref["resid"][-1] + 1e-7
