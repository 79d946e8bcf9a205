"""Pins of the FP64 oracle against facts fixed by the paper and the mathematics.

P1  one raster ICD pass == the closed form of eq. (ICDUpdate1)
P2  MACE fixed point == dense Cholesky MAP (quadratic prior; MAP equivalence of
    the MACE equations, Sec. II-B); q-GGMRF: == centralised exact ICD and the
    gradient of f vanishes (checked by finite differences of f)
P3  invariants at the fixed point: X_i = mean(w) (proof of Theorem 1), one more
    pass is a no-op (Lemma B.1), exact prox of v_i returns x*, u_i sums to 0
P4  the agent cost never increases during a pass (both coordinate rules)
P5  partial-update MACE == the exact augmented linear map of Theorem 2; its
    limit is the map's fixed point
P6  special cases: N = 1, q-GGMRF limits (p = q, T -> inf, large |d|)
P7  MACE-PnP (Algorithm 3): the stand-in denoiser's spectrum equals the closed
    form of the binomial filter (symmetric, in (0, 1): firmly non-expansive),
    and the PnP fixed point is the minimiser of f(x) + phi(x)/sigma^2 with
    H = prox of phi (dense solve), every agent's state equal to H(mean w)
    (Theorem 3, Appendix C)
plus the divergence of Algorithm 1 at sigma = 0.05 on the 64x64 workload.
"""
import numpy as np
import pytest

import mace_inputs as mi
import oracle
from tests import dense_ref as dr


def _problem(geom, seed, N, kind=0, sx=0.001, p=2.0, q=2.0, T=1.0):
    cp, row, val = mi.system_matrix(geom)
    s = mi.scan(geom, seed)
    va = mi.interleaved_partition(geom.n_views, N)
    O = oracle.Oracle(geom.nx, geom.ny, geom.n_views, geom.n_channels, cp, row, val, s.y, s.lam,
                      va, kind, sx, p, q, T)
    A = dr.dense_A(geom, cp, row, val)
    return O, A, s.lam.astype(np.float64), s.y.astype(np.float64), va


# ---------------- P1 ----------------
@pytest.mark.parametrize("N,agent", [(1, 0), (3, 1)])
def test_P1_icd_pass_equals_gauss_seidel_closed_form(N, agent):
    g = mi.Geometry(8, 8, 12, 12)
    sx, sigma = 0.01, 0.02
    O, A, lam, y, va = _problem(g, 21, N, 0, sx)
    Lb = dr.laplacian(g.nx, g.ny)
    Hs, bs = dr.agent_system(g, A, lam, y, Lb, sx, va, N)
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 0.05, g.n)
    v = rng.uniform(0, 0.05, g.n)
    z = x.copy()
    e = O.error_sinogram(x, agent=agent)
    O.icd_pass(agent, sigma, v, z, e)
    ref = dr.icd_pass_closed_form(Hs[agent], bs[agent], x, v, sigma)
    np.testing.assert_allclose(z, ref, rtol=1e-11, atol=1e-14)
    # the kept error sinogram equals y - A z on the agent's rows
    r = dr.agent_rows(g, va, agent)
    np.testing.assert_allclose(e[r], y[r] - A[r] @ z, atol=1e-10)


@pytest.mark.parametrize("omega", [0.5, 0.8])
def test_P1_relaxed_pass_equals_sor_closed_form(omega):
    # relax scales every coordinate step: a quadratic pass is then textbook SOR
    g = mi.Geometry(8, 8, 12, 12)
    sx, sigma = 0.01, 0.02
    O, A, lam, y, va = _problem(g, 24, 2, 0, sx)
    Hs, bs = dr.agent_system(g, A, lam, y, dr.laplacian(8, 8), sx, va, 2)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 0.05, g.n)
    v = rng.uniform(0, 0.05, g.n)
    z = x.copy()
    e = O.error_sinogram(x, agent=1)
    O.icd_pass(1, sigma, v, z, e, relax=omega)
    ref = dr.sor_pass_closed_form(Hs[1], bs[1], x, v, sigma, omega)
    np.testing.assert_allclose(z, ref, rtol=1e-11, atol=1e-14)


def test_relaxation_keeps_the_fixed_point(quad32):
    # under-relaxed passes reach the same MAP fixed point (the stationarity
    # argument of Lemma B.1 does not depend on the step length)
    d = quad32
    r = d["O"].mace_solve(d["rho"], d["sigma"], 8000, tol=1e-13, relax=0.6)
    assert r["resid"][-1] < 1e-13
    assert np.linalg.norm(r["x"] - d["xmap"]) / np.linalg.norm(d["xmap"]) < 1e-9


def test_P1_visiting_order_is_respected():
    g = mi.Geometry(8, 8, 12, 12)
    O, A, lam, y, va = _problem(g, 22, 2, 0, 0.01)
    Lb = dr.laplacian(g.nx, g.ny)
    Hs, bs = dr.agent_system(g, A, lam, y, Lb, 0.01, va, 2)
    perm = np.random.default_rng(1).permutation(g.n)
    x = np.full(g.n, 0.01)
    v = np.full(g.n, 0.02)
    z = x.copy()
    e = O.error_sinogram(x, agent=0)
    O.icd_pass(0, 0.05, v, z, e, order=perm)
    # Gauss-Seidel in the permuted order == closed form on the permuted system
    Hp = Hs[0][np.ix_(perm, perm)]
    ref = dr.icd_pass_closed_form(Hp, bs[0][perm], x[perm], v[perm], 0.05)
    np.testing.assert_allclose(z[perm], ref, rtol=1e-11, atol=1e-14)


# ---------------- P2 / P3 ----------------
@pytest.fixture(scope="module")
def quad32():
    g = mi.Geometry(32, 32, 64, 48)
    N, sx, sigma, rho = 4, 0.001, 0.001, 0.8
    O, A, lam, y, va = _problem(g, 7, N, 0, sx)
    Lb = dr.laplacian(g.nx, g.ny)
    xmap = dr.map_quadratic(A, lam, y, Lb, sx)
    res = O.mace_solve(rho, sigma, 5000, tol=1e-13)
    return dict(g=g, N=N, sx=sx, sigma=sigma, rho=rho, O=O, A=A, lam=lam, y=y, va=va,
                Lb=Lb, xmap=xmap, res=res)


def test_P2_mace_fixed_point_is_the_map(quad32):
    r, xmap = quad32["res"], quad32["xmap"]
    assert r["resid"][-1] < 1e-13
    nrmse = np.linalg.norm(r["x"] - xmap) / np.linalg.norm(xmap)
    assert nrmse < 1e-9, nrmse


def test_P3_fixed_point_invariants(quad32):
    d = quad32
    O, r, N, sigma = d["O"], d["res"], d["N"], d["sigma"]
    x = r["x"]
    w = r["w"]
    # X* = G w*: every agent state equals the consensus
    assert np.abs(r["X"] - x[None, :]).max() < 1e-11 * np.abs(x).max()
    wbar = w.mean(axis=0)
    np.testing.assert_allclose(wbar, x, rtol=0, atol=1e-15)
    grads = []
    for i in range(N):
        v = 2.0 * wbar - w[i]
        # Lemma B.1: one more partial update leaves the fixed point unchanged
        z = x.copy()
        e = O.error_sinogram(x, agent=i)
        O.icd_pass(i, sigma, v, z, e)
        assert np.abs(z - x).max() < 1e-10 * np.abs(x).max()
        # F_i(v_i*) = x*: the exact proximal map returns the consensus
        zp, _ = O.prox(i, sigma, v, z0=x, rtol=1e-15, max_passes=200)
        assert np.abs(zp - x).max() < 1e-10 * np.abs(x).max()
        # sigma^2 grad f_i(x*) = v_i* - x*
        gi = O.gradient(x, agent=i)
        np.testing.assert_allclose(sigma ** 2 * gi, v - x, atol=1e-9 * np.abs(x).max())
        grads.append(gi)
    # the agents' forces balance: sum_i grad f_i(x*) = grad f(x*) = 0
    gsum = np.sum(grads, axis=0)
    scale = np.abs(grads).max()
    assert np.abs(gsum).max() < 1e-8 * scale


def test_P2_conjugate_gradient_map_is_the_dense_map(quad32):
    """The oracle's CG solve of the normal equations returns the dense
    Cholesky MAP; its reported residual is the true one."""
    d = quad32
    x, it, rel = d["O"].map_cg(rtol=1e-14)
    assert it > 0 and rel <= 1e-13
    H = d["A"].T @ (d["lam"][:, None] * d["A"]) + d["Lb"] / d["sx"] ** 2
    b = d["A"].T @ (d["lam"] * d["y"])
    assert abs(np.linalg.norm(b - H @ x) / np.linalg.norm(b) - rel) <= 1e-13
    nrmse = np.linalg.norm(x - d["xmap"]) / np.linalg.norm(d["xmap"])
    assert nrmse < 1e-11, nrmse


def test_P2_conjugate_gradient_map_larger_than_a_dense_solve():
    """At 48x48 with 72 views (no dense solve here): the CG MAP zeroes the gradient of f (the
    oracle's gradient routine, checked against finite differences of f in
    the q-GGMRF test) and equals the centralised exact ICD, an unrelated
    algorithm, and the MACE fixed point of 3 agents."""
    g = mi.Geometry(48, 48, 72, 72)
    sx = 0.002
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, 31)
    va = mi.interleaved_partition(g.n_views, 3)
    O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, s.y, s.lam, va, 0, sx)
    x, it, rel = O.map_cg(rtol=1e-13)
    assert rel <= 1e-13
    g0 = np.abs(O.gradient(np.zeros(g.n))).max()
    assert np.abs(O.gradient(x)).max() < 1e-10 * g0
    xc, _ = O.centralized_icd(rtol=1e-15, max_passes=20000)
    assert np.linalg.norm(xc - x) / np.linalg.norm(x) < 1e-10
    res = O.mace_solve(0.8, 5e-4, 20000, tol=1e-13)
    assert res["resid"][-1] < 1e-13
    assert np.linalg.norm(res["x"] - x) / np.linalg.norm(x) < 1e-10


def test_P2_conjugate_gradient_refuses_a_non_quadratic_prior():
    g = mi.Geometry(8, 8, 12, 12)
    O, A, lam, y, va = _problem(g, 3, 1, 1, 0.01, 2.0, 1.2, 1.0)
    with pytest.raises(ValueError):
        O.map_cg()


@pytest.mark.parametrize("kind,relax", [(0, 1.0), (1, 0.5)])
def test_stopping_statistic_is_the_mann_step_over_two_rho(kind, relax):
    """Algorithm 1: w^{k+1} - w^k = rho (2 X^{k+1} - v^k) - rho w^k
    = 2 rho (X^{k+1} - G w^k), since v^k = 2 G w^k - w^k.  So the residual the
    oracle reports, r_k = ||X^{k+1} - G w^k|| / ||w^k||, must equal
    ||w^{k+1} - w^k|| / (2 rho ||w^k||) computed from the iterates w the oracle
    returns after k and k + 1 iterations (k >= 1, where w^k != 0)."""
    g = mi.Geometry(16, 16, 24, 24)
    N, rho, sigma = 3, 0.7, 0.002
    O, A, lam, y, va = _problem(g, 41, N, kind, 0.002, 2.0, 1.2, 1.0)
    K = 6
    full = O.mace_solve(rho, sigma, K, relax=relax)
    ws = [O.mace_solve(rho, sigma, k, relax=relax)["w"] for k in range(1, K + 1)]
    for k in range(1, K):
        step = np.linalg.norm(ws[k] - ws[k - 1]) / (2 * rho * np.linalg.norm(ws[k - 1]))
        assert abs(full["resid"][k] - step) <= 1e-12 * step, (k, full["resid"][k], step)
    # k = 0: w^0 = 0, and the statistic's denominator is ||X^1||
    X1 = O.mace_solve(rho, sigma, 1, relax=relax)["X"]
    num = np.linalg.norm(ws[0]) / (2 * rho)
    assert abs(full["resid"][0] - num / np.linalg.norm(X1)) <= 1e-12 * full["resid"][0]


def test_P2_qggmrf_fixed_point_matches_centralised_icd():
    g = mi.Geometry(24, 24, 48, 36)
    N, sx, sigma = 2, 0.001, 0.001
    O, A, lam, y, va = _problem(g, 9, N, 1, sx, 2.0, 1.2, 1.0)
    res = O.mace_solve(0.8, sigma, 6000, tol=1e-13, mode=oracle.MODE_SURROGATE)
    assert res["resid"][-1] < 1e-13
    xc, it = O.centralized_icd(rtol=1e-15, max_passes=20000, mode=oracle.MODE_EXACT)
    nrmse = np.linalg.norm(res["x"] - xc) / np.linalg.norm(xc)
    assert nrmse < 1e-8, nrmse
    # grad f(x*) = 0: central finite differences of the oracle's cost f
    rng = np.random.default_rng(3)
    x = res["x"]
    for s in rng.choice(g.n, 6, replace=False):
        h = 1e-7
        xp, xm = x.copy(), x.copy()
        xp[s] += h
        xm[s] -= h
        fd = (O.cost(xp) - O.cost(xm)) / (2 * h)
        gs = O.gradient(x)[s]
        # the gradient routine agrees with the cost ...
        assert abs(fd - gs) < 1e-4 * (abs(O.cost(x)) / np.abs(x).max() + 1)
        # ... and vanishes at the fixed point relative to its scale at x = 0
    g0 = np.abs(O.gradient(np.zeros(g.n))).max()
    assert np.abs(O.gradient(x)).max() < 1e-8 * g0
    # strict convexity: random perturbations never lower f
    f0 = O.cost(x)
    for _ in range(5):
        assert O.cost(x + 1e-4 * rng.standard_normal(g.n)) > f0


# ---------------- P4 ----------------
@pytest.mark.parametrize("mode", [oracle.MODE_SURROGATE, oracle.MODE_EXACT])
def test_P4_agent_cost_monotone_within_a_pass(mode):
    g = mi.Geometry(10, 10, 16, 16)
    O, A, lam, y, va = _problem(g, 31, 2, 1, 0.002, 2.0, 1.1, 1.0)
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 0.1, g.n)
    v = rng.uniform(0, 0.1, g.n)
    z = x.copy()
    e = O.error_sinogram(x, agent=1)
    phi0 = O.cost(x, agent=1, v=v, sigma=0.01)
    tr = O.icd_pass(1, 0.01, v, z, e, mode=mode, trace=True)
    seq = np.concatenate([[phi0], tr])
    assert np.all(np.diff(seq) <= 1e-12 * abs(phi0)), np.diff(seq).max()
    assert seq[-1] < seq[0]


def test_P4_exact_rule_solves_the_coordinate_problem():
    # after an exact-rule update of pixel s, the partial derivative of the
    # agent cost along s vanishes (finite differences of the cost)
    g = mi.Geometry(8, 8, 12, 12)
    O, A, lam, y, va = _problem(g, 32, 2, 1, 0.003, 2.0, 1.2, 1.0)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 0.1, g.n)
    v = rng.uniform(0, 0.1, g.n)
    z = x.copy()
    e = O.error_sinogram(x, agent=0)
    order = np.array([27], dtype=np.int64)
    order = np.concatenate([order, np.full(g.n - 1, 27)])  # visit pixel 27 repeatedly
    O.icd_pass(0, 0.02, v, z, e, order=order, mode=oracle.MODE_EXACT)
    h = 1e-7
    zp, zm = z.copy(), z.copy()
    zp[27] += h
    zm[27] -= h
    d = (O.cost(zp, 0, v, 0.02) - O.cost(zm, 0, v, 0.02)) / (2 * h)
    curv = (O.cost(zp, 0, v, 0.02) - 2 * O.cost(z, 0, v, 0.02) + O.cost(zm, 0, v, 0.02)) / h ** 2
    assert abs(d) < 1e-5 * curv * max(abs(z[27]), 1e-3)


# ---------------- P5 ----------------
def test_P5_theorem2_linear_map():
    g = mi.Geometry(8, 8, 16, 12)
    N, sx, rho = 2, 0.003, 0.8
    O, A, lam, y, va = _problem(g, 5, N, 0, sx)
    Lb = dr.laplacian(g.nx, g.ny)
    Hs, bs = dr.agent_system(g, A, lam, y, Lb, sx, va, N)
    sigma = 0.002
    M, c = dr.pu_mace_linear_map(Hs, bs, sigma, rho)
    # iterate the exact map from w = 0, X = G(0) = 0 and compare trajectories
    z = np.zeros(2 * N * g.n)
    for k in range(25):
        z = M @ z + c
    r = O.mace_solve(rho, sigma, 25)
    np.testing.assert_allclose(r["w"].reshape(-1), z[:N * g.n], rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(r["X"].reshape(-1), z[N * g.n:], rtol=1e-9, atol=1e-13)
    # small sigma: spectral radius < 1, the oracle reaches the map's fixed point
    srad = np.abs(np.linalg.eigvals(M)).max()
    assert srad < 1.0
    zfix = np.linalg.solve(np.eye(M.shape[0]) - M, c)
    r = O.mace_solve(rho, sigma, 20000, tol=1e-14)
    np.testing.assert_allclose(r["w"].reshape(-1), zfix[:N * g.n], rtol=1e-8,
                               atol=1e-10 * np.abs(zfix).max())


def test_configured_sigma_diverges_on_64x64():
    """At sigma = 0.05 (sigma^2 theta2 >> 1) Algorithm 1 does not converge on the
    64x64 4-agent workload: the exact linear map of Theorem 2 for the same
    problem class has spectral radius > 1, and the oracle's iterates grow."""
    w = mi.WORKLOADS["plain64"]
    g = w.geom
    O, A, lam, y, va = _problem(g, w.seed, w.n_agents, 0, w.sigma_x)
    r = O.mace_solve(w.rho, w.sigma, 1200)
    assert not np.all(np.isfinite(r["x"])) or np.abs(r["x"]).max() > 1e3
    # a stable setting (small sigma) stays bounded on the same data
    r2 = O.mace_solve(w.rho, 2.5e-4, 300)
    assert np.abs(r2["x"]).max() < 1.0
    # the small analogue: 12x12, 4 agents, same prior and sigma
    gs = mi.Geometry(12, 12, 24, 18)
    O2, A2, lam2, y2, va2 = _problem(gs, 5, 4, 0, w.sigma_x)
    Hs, bs = dr.agent_system(gs, A2, lam2, y2, dr.laplacian(12, 12), w.sigma_x, va2, 4)
    M, _ = dr.pu_mace_linear_map(Hs, bs, w.sigma, w.rho)
    assert np.abs(np.linalg.eigvals(M)).max() > 1.0


def test_P5_partial_updates_lose_stability_in_a_band_of_sigma():
    """Theorem 2 covers small sigma only.  The exact linear map of partial-
    update MACE (12x12, 24 views, 4 agents, rho = 0.8) has spectral radius
    below 1 at small sigma; with a weak prior (sigma_x = 0.02) it exceeds 1
    in a middle band of sigma (sigma^2 theta2 from about 1 to about 400),
    and with a prior ten times stronger (sigma_x = 0.002) it stays below 1
    at every sigma, smallest near sigma^2 theta2 = 1."""
    gs = mi.Geometry(12, 12, 24, 18)

    def radius(sx, sigma):
        O2, A2, lam2, y2, va2 = _problem(gs, 5, 4, 0, sx)
        Hs, bs = dr.agent_system(gs, A2, lam2, y2, dr.laplacian(12, 12), sx, va2, 4)
        M, _ = dr.pu_mace_linear_map(Hs, bs, sigma, 0.8)
        return float(np.abs(np.linalg.eigvals(M)).max())

    assert radius(0.02, 1e-3) < 1.0
    assert radius(0.02, 3e-3) > 1.0
    assert radius(0.02, 1e-2) > 1.15
    assert radius(0.02, 1e-1) > 1.0
    strong = [radius(0.002, sg) for sg in (1e-3, 3e-3, 1e-2, 3e-2, 1e-1)]
    assert max(strong) < 1.0
    assert min(strong) == strong[1] and strong[1] < 0.8


# ---------------- P6 ----------------
def test_P6_single_agent_reaches_centralised_map():
    g = mi.Geometry(16, 16, 32, 24)
    sx = 0.002
    O, A, lam, y, va = _problem(g, 13, 1, 0, sx)
    xmap = dr.map_quadratic(A, lam, y, dr.laplacian(16, 16), sx)
    r = O.mace_solve(0.8, 0.01, 20000, tol=1e-13)
    assert np.linalg.norm(r["x"] - xmap) / np.linalg.norm(xmap) < 1e-9
    xc, _ = O.centralized_icd(rtol=1e-15, max_passes=50000)
    assert np.linalg.norm(xc - xmap) / np.linalg.norm(xmap) < 1e-9


def test_P2_empty_columns_fixed_point_is_the_map():
    """4 views on 8 channels leave 24 pixels that no ray crosses (empty
    columns of A), and with one view per agent most of each agent's columns
    are empty: there the update is set by the prior and the prox term alone,
    and the fixed point is still the dense MAP (Theorem 1)."""
    g = mi.Geometry(24, 24, 4, 8)
    sx = 0.003
    O, A, lam, y, va = _problem(g, 125, 4, 0, sx)
    assert int((np.abs(A).sum(axis=0) == 0).sum()) == 24
    xmap = dr.map_quadratic(A, lam, y, dr.laplacian(g.nx, g.ny), sx)
    r = O.mace_solve(0.8, 0.003, 20000, tol=1e-13)
    assert r["resid"][-1] < 1e-13
    assert np.linalg.norm(r["x"] - xmap) / np.linalg.norm(xmap) < 1e-9


def test_P6_reflection_is_an_involution():
    rng = np.random.default_rng(6)
    N, n = 5, 7
    w = rng.standard_normal((N, n))
    refl = lambda u: 2 * u.mean(axis=0)[None, :] - u
    np.testing.assert_allclose(refl(refl(w)), w, atol=1e-14)


def test_P6_qggmrf_special_cases():
    g = mi.Geometry(8, 8, 12, 12)
    rng = np.random.default_rng(8)
    x = rng.uniform(0, 0.05, g.n)
    sx = 0.01
    Oq, *_ = _problem(g, 1, 1, 0, sx)
    # T -> infinity: q-GGMRF equals the quadratic prior
    Ot, *_ = _problem(g, 1, 1, 1, sx, 2.0, 1.2, 1e20)
    assert abs(Ot.prior(x) - Oq.prior(x)) < 1e-10 * Oq.prior(x)
    # p = q: rho(d) = |d|^p / (2 p sigma_x^p), half the quadratic for p = 2
    Op, *_ = _problem(g, 1, 1, 1, sx, 2.0, 2.0, 1.0)
    assert abs(Op.prior(x) - 0.5 * Oq.prior(x)) < 1e-12 * Oq.prior(x)
    # one clique, large difference: rho ~ |d|^q T^(p-q) / (p sigma_x^q)
    g2 = mi.Geometry(2, 1, 2, 4)
    O2, *_ = _problem(g2, 1, 1, 1, sx, 2.0, 1.2, 1.0)
    d = 1e4 * sx
    val = O2.prior(np.array([d, 0.0]))
    asym = mi.B_EDGE * d ** 1.2 / (2.0 * sx ** 1.2)
    assert abs(val / asym - 1.0) < 1e-2
    # small difference: quadratic with curvature 1/sigma_x^2
    d = 1e-6 * sx
    val = O2.prior(np.array([d, 0.0]))
    assert abs(val / (mi.B_EDGE * d * d / (2 * sx * sx)) - 1.0) < 1e-3


def test_P8_oracle_is_deterministic():
    g = mi.Geometry(16, 16, 24, 24)
    O, *_ = _problem(g, 2, 3, 1, 0.003, 2.0, 1.2, 1.0)
    a = O.mace_solve(0.8, 0.003, 20)
    b = O.mace_solve(0.8, 0.003, 20)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["resid"], b["resid"])


# ---------------- P7: MACE-PnP ----------------
def _dense_smoother(nx, ny, passes):
    n = nx * ny
    return np.stack([oracle.binomial_smooth(np.eye(n)[j], nx, ny, passes) for j in range(n)],
                    axis=1)


@pytest.mark.parametrize("passes", [1, 2])
def test_P7_denoiser_spectrum_is_the_binomial_closed_form(passes):
    nx, ny = 5, 4
    Hm = _dense_smoother(nx, ny, passes)
    assert np.array_equal(Hm, Hm.T)
    # per axis tridiag(1/4, 1/2, 1/4): eigenvalues 1/2 + 1/2 cos(k pi / (m + 1))
    lx = 0.5 + 0.5 * np.cos(np.arange(1, nx + 1) * np.pi / (nx + 1))
    ly = 0.5 + 0.5 * np.cos(np.arange(1, ny + 1) * np.pi / (ny + 1))
    ref = np.sort(np.outer(ly, lx).reshape(-1) ** passes)
    got = np.sort(np.linalg.eigvalsh(Hm))
    assert np.allclose(got, ref, rtol=0, atol=1e-14)
    assert got.min() > 0.0 and got.max() < 1.0


@pytest.mark.parametrize("passes", [1, 2])
def test_P7_pnp_fixed_point_is_the_pnp_map(passes):
    """H = prox of phi(x) = x^T (H^-1 - I) x / 2, so the PnP equilibrium
    F(x - a; sigma) = x, H(x + a) = x is the minimiser of
    f(x) + phi(x) / sigma^2 (f without prior); MACE-PnP with F_i at
    sqrt(N) sigma reaches it, with X_i = H(mean w) for every agent."""
    g = mi.Geometry(10, 10, 24, 16)
    N, sigma = 3, 0.001
    O, A, lam, y, va = _problem(g, 41, N, kind=oracle.PRIOR_NONE, sx=1.0)
    res = O.mace_pnp_solve(0.8, sigma, 3000, passes)
    M = np.linalg.inv(_dense_smoother(g.nx, g.ny, passes)) - np.eye(g.n)
    xref = np.linalg.solve(A.T @ (lam[:, None] * A) + M / sigma ** 2, A.T @ (lam * y))
    assert res["resid"][-1] < 1e-12
    assert np.linalg.norm(res["x"] - xref) <= 1e-10 * np.linalg.norm(xref)
    assert np.abs(res["X"] - res["x"][None, :]).max() <= 1e-10 * np.abs(res["x"]).max()


# ---------------- volumes (slice stacks with axial cliques) ----------------
def _volume(g, nz, seed, N, kind, sx, b_axial, q=2.0):
    cp, row, val = mi.system_matrix(g)
    scans = [mi.scan(g, seed + z) for z in range(nz)]
    y = np.concatenate([s.y for s in scans])
    lam = np.concatenate([s.lam for s in scans])
    va = mi.interleaved_partition(g.n_views, N)
    O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, y, lam, va, kind, sx,
                      2.0, q, 1.0, nz=nz, b_axial=b_axial)
    A = dr.dense_A(g, cp, row, val)
    return O, A, lam.astype(np.float64), y.astype(np.float64), (cp, row, val), scans, va


def test_P2_volume_fixed_point_is_the_dense_map():
    """A stack of 3 slices with axial cliques: the MACE fixed point equals the
    minimiser of the volume's quadratic MAP cost, solved densely, and the
    oracle's CG solve of the same normal equations."""
    g = mi.Geometry(8, 8, 12, 12)
    nz, N, sx, ba = 3, 2, 0.004, 0.3
    O, A, lam, y, _, _, _ = _volume(g, nz, 51, N, 0, sx, ba)
    H, b = dr.volume_system(A, lam, y, nz)
    H += dr.laplacian3(g.nx, g.ny, nz, ba) / sx ** 2
    xmap = np.linalg.solve(H, b)
    res = O.mace_solve(0.8, 0.005, 20000, tol=1e-13)
    assert res["resid"][-1] < 1e-13
    assert np.linalg.norm(res["x"] - xmap) / np.linalg.norm(xmap) < 1e-9
    xcg, _, rel = O.map_cg(rtol=1e-14)
    assert np.linalg.norm(xcg - xmap) / np.linalg.norm(xmap) < 1e-10


def test_P1_volume_icd_pass_equals_gauss_seidel_closed_form():
    """One raster ICD pass over the voxels of a volume (slice-major) equals the
    Gauss-Seidel closed form of eq. (ICDUpdate1) with the volume's agent
    Hessian (data of the agent's views in every slice, prior / N including
    the axial cliques)."""
    g = mi.Geometry(6, 6, 10, 10)
    nz, N, agent, sx, ba, sigma = 3, 2, 1, 0.01, 0.4, 0.02
    O, A, lam, y, _, _, va = _volume(g, nz, 61, N, 0, sx, ba)
    r = dr.agent_rows(g, va, agent)
    Ai = np.zeros_like(A)
    Ai[r] = A[r]
    H, b = dr.volume_system(Ai, lam, y, nz)
    H += dr.laplacian3(g.nx, g.ny, nz, ba) / (N * sx ** 2)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 0.05, nz * g.n)
    v = rng.uniform(0, 0.05, nz * g.n)
    z = x.copy()
    e = O.error_sinogram(x, agent=agent)
    O.icd_pass(agent, sigma, v, z, e)
    ref = dr.icd_pass_closed_form(H, b, x, v, sigma)
    np.testing.assert_allclose(z, ref, rtol=1e-11, atol=1e-14)


def test_P6_volume_without_axial_cliques_is_independent_slices():
    """b_axial = 0: the volume's MACE iterates are each slice's 2-D iterates."""
    g = mi.Geometry(10, 10, 16, 16)
    nz, N, sx = 3, 2, 0.003
    O, A, lam, y, (cp, row, val), scans, va = _volume(g, nz, 71, N, 1, sx, 0.0, q=1.2)
    res = O.mace_solve(0.8, 0.003, 12, relax=0.5)
    for zz, s in enumerate(scans):
        O2 = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, s.y, s.lam, va, 1,
                           sx, 2.0, 1.2, 1.0)
        r2 = O2.mace_solve(0.8, 0.003, 12, relax=0.5)
        np.testing.assert_allclose(res["x"][zz * g.n:(zz + 1) * g.n], r2["x"], rtol=0,
                                   atol=1e-13 * np.abs(r2["x"]).max())


def test_P2_volume_qggmrf_gradient_and_fixed_point():
    """q-GGMRF volume: the oracle's gradient matches central differences of
    its cost (axial cliques included) and vanishes at the MACE fixed point,
    which equals the centralised ICD's."""
    g = mi.Geometry(8, 8, 12, 12)
    nz, N, sx, ba = 3, 2, 0.003, 0.5
    O, A, lam, y, _, _, _ = _volume(g, nz, 81, N, 1, sx, ba, q=1.2)
    res = O.mace_solve(0.8, 0.003, 20000, tol=1e-13, relax=0.5)
    assert res["resid"][-1] < 1e-13
    x = res["x"]
    xc, _ = O.centralized_icd(rtol=1e-15, max_passes=20000, mode=oracle.MODE_EXACT)
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) < 1e-8
    g0 = np.abs(O.gradient(np.zeros(nz * g.n))).max()
    assert np.abs(O.gradient(x)).max() < 1e-8 * g0
    rng = np.random.default_rng(5)
    xr = x + 1e-3 * rng.standard_normal(x.size)
    gr = O.gradient(xr)
    for s in rng.choice(nz * g.n, 6, replace=False):
        h = 1e-7
        xp, xm = xr.copy(), xr.copy()
        xp[s] += h
        xm[s] -= h
        fd = (O.cost(xp) - O.cost(xm)) / (2 * h)
        assert abs(fd - gr[s]) < 1e-4 * (abs(gr[s]) + 1.0)
