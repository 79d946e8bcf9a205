"""Host logic of bench.py's convergence study (no GPU): the sampled
iteration counts and the equits read off an NRMSE curve (Sec. IV-B)."""
import math

import numpy as np

import bench


def test_study_grid_is_increasing_and_capped():
    ks = bench.study_grid(400)
    assert ks[:20] == list(range(1, 21))
    assert all(b > a for a, b in zip(ks, ks[1:]))
    assert ks[-1] == 400
    assert bench.study_grid(30)[-1] == 30 and bench.study_grid(7) == list(range(1, 8))


def test_equits_exact_on_a_geometric_curve():
    # NRMSE = 0.5^k: log-linear interpolation is exact, 1e-2 is crossed at
    # k = log(100) / log(2) even when only every 5th iteration is sampled
    ks = [1, 5, 10, 15]
    es = [0.5 ** k for k in ks]
    e = bench.equits_to_reach(ks, es, 1e-2)
    assert math.isclose(e, math.log(100) / math.log(2), rel_tol=1e-12)


def test_equits_first_crossing_and_failures():
    assert bench.equits_to_reach([1, 2, 3], [5e-3, 1e-3, 1e-4], 1e-2) == 1
    assert bench.equits_to_reach([1, 2, 3], [0.5, 0.2, 0.1], 1e-2) is None
    assert bench.equits_to_reach([1, 2], [0.5, float("inf")], 1e-2) is None
    # one Mann iteration with two ICD passes per agent costs two equits
    assert bench.equits_to_reach([1, 2], [0.1, 0.001], 1e-2, equits_per_iter=2.0) == 3.0
    # a curve that rises before it crosses takes the crossing sample itself
    assert bench.equits_to_reach([1, 2, 3], [0.1, 0.2, 0.005], 1e-2) > 2
    assert np.isfinite(bench.equits_to_reach([1, 2, 3], [0.01, 0.02, 0.005], 1e-2))


def test_study_reference_is_the_map():
    """The stored x* of the convergence study (written by
    tests/golden/make_study_reference.py with the oracle) matches its
    checksum and is the minimiser of f: the oracle's gradient of f at the
    stored (float32-rounded) image is below 1e-7 of its value at 0."""
    import mace_inputs as mi
    import oracle
    x, meta = bench.load_study_reference()
    p = meta["problem"]
    g = mi.Geometry(p["nx"], p["ny"], p["n_views"], p["n_channels"])
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, p["seed"])
    pr = p["prior"]
    O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, s.y, s.lam,
                      mi.interleaved_partition(g.n_views, 1), pr["kind"], pr["sigma_x"], pr["p"],
                      pr["q"], pr["T"])
    g0 = np.abs(O.gradient(np.zeros(g.n))).max()
    assert np.abs(O.gradient(x)).max() < 1e-7 * g0
    assert meta["grad_ratio"] < 1e-10
    c = meta["centralized_equits"]
    assert all(c[t] is not None for t in c)
    assert c["0.01"] < c["0.003"] < c["0.001"]
