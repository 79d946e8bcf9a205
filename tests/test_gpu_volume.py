"""GPU parity of volume reconstruction (slice stacks with axial cliques)
against the oracle's 3-D problem.

A volume is nz slices measured by one 2-D matrix; the prior adds the axial
cliques (z, s)-(z + 1, s) with weight b_axial to every slice's 8 in-plane
cliques, and partial-update MACE runs over the stacked voxels.  The GPU
sweeps each colour phase twice, the even slices and then the odd ones, with
either record format (compact: the axial neighbours are read a pixel step
ahead with the records; general: staged with the super-voxel).

1. Sequential schedule (one row per agent): the trajectory equals the
   oracle's, run in the GPU's visiting order (colour c, then the even
   slices, then the odd slices; super-voxels and raster order inside), with
   the same coordinate rule -- every slice's X_i and x, element by element
   (5e-5 of max|x|, the FP32 budget of the 2-D parity tests), and the stacked
   residual.
2. Concurrent schedule: the fixed point equals the volume's MAP image (the
   oracle's conjugate-gradient solve of the 3-D normal equations, pinned to
   the dense 3-D MAP in the oracle tests) to NRMSE 1e-4.
3. b_axial = 0: every slice of the volume equals the same slice solved alone
   (the sequential schedule, same visiting order inside a slice).
4. Argument errors.
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


def _volume(g, nz, seed, N, kind, sx, ba, q=2.0):
    cp, row, val = mi.system_matrix(g)
    scans = [mi.scan(g, seed + z) for z in range(nz)]
    y = np.stack([s.y for s in scans])
    lam = np.stack([s.lam for s in scans])
    va = mi.interleaved_partition(g.n_views, N)
    O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, y.reshape(-1),
                      lam.reshape(-1), va, kind, sx, 2.0, q, 1.0, nz=nz, b_axial=ba)
    return (cp, row, val), y, lam, O


def _volume_order(sysm, g, nz, S):
    """The GPU's sequential visiting order over the voxels v = z n + s."""
    o2 = sysm.visit_order()
    col = ((o2 % g.nx) // S & 1) + 2 * ((o2 // g.nx) // S & 1)
    out = []
    for c in range(4):
        part = o2[col == c]
        for par in (0, 1):
            for z in range(par, nz, 2):
                out.append(z * g.n + part)
    return np.concatenate(out)


SEQ_CASES = [
    # geometry, nz, N, prior kind, sigma_x, q, b_axial, sigma, S, iterations, record format
    (mi.Geometry(24, 24, 24, 36), 3, 2, 1, 0.002, 1.2, 0.5, 0.001, 8, 4, 2),
    (mi.Geometry(20, 18, 30, 30), 4, 3, 0, 0.003, 2.0, 0.25, 0.002, 4, 3, 2),
    (mi.Geometry(16, 16, 16, 24), 2, 2, 1, 0.002, 1.2, 1.0, 0.001, 4, 3, 2),
    (mi.Geometry(24, 24, 24, 36), 3, 2, 1, 0.002, 1.2, 0.5, 0.001, 8, 4, 1),
    (mi.Geometry(20, 18, 30, 30), 5, 3, 0, 0.003, 2.0, 0.25, 0.002, 4, 3, 1),   # ragged SVs
    (mi.Geometry(16, 16, 16, 24), 2, 2, 1, 0.002, 1.2, 1.0, 0.001, 8, 3, 1),
]


@pytest.mark.parametrize("case", SEQ_CASES,
                         ids=lambda c: f"{c[0].nx}x{c[0].ny}z{c[1]}_N{c[2]}_k{c[3]}_ba{c[6]}_S{c[8]}_f{c[10]}")
def test_volume_sequential_trajectory_matches_oracle(m, case):
    g, nz, N, kind, sx, q, ba, sigma, S, iters, fmt = case
    (cp, row, val), y, lam, O = _volume(g, nz, 301 + g.nx, N, kind, sx, ba, q)
    print(f"case {g} nz={nz} N={N} b_axial={ba} S={S} format={fmt}", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=S,
                    rows_per_agent=1, format=fmt)
    assert sysm.config["format"] == fmt
    prior = m.make_prior(kind, sx, 2.0, q, 1.0)
    x, info = sysm.solve_volume(y, lam, prior, ba, 0.8, sigma, iters)
    order = _volume_order(sysm, g, nz, S)
    assert np.array_equal(np.sort(order), np.arange(nz * g.n))
    ref = O.mace_solve(0.8, sigma, iters, order=order, mode=oracle.MODE_SURROGATE)
    scale = np.abs(ref["x"]).max()
    assert np.all(np.isfinite(x))
    assert np.abs(x.reshape(-1) - ref["x"]).max() <= 5e-5 * scale
    for z in range(nz):
        _, Xz = sysm.slot_state(z)
        err = np.abs(Xz - ref["X"][:, z * g.n:(z + 1) * g.n]).max()
        assert err <= 5e-5 * scale, (z, err / scale)
    assert info.iters == iters
    assert abs(info.residual - ref["resid"][-1]) <= 1e-3 * ref["resid"][-1] + 1e-7


@pytest.fixture(scope="module")
def volume_map():
    g = mi.Geometry(64, 64, 48, 96)
    nz, N, sx, ba = 4, 4, 0.001, 0.5
    (cp, row, val), y, lam, O = _volume(g, nz, 17, N, 0, sx, ba)
    xmap, _, rel = O.map_cg(rtol=1e-13)
    assert rel <= 1e-12
    return g, nz, N, sx, ba, (cp, row, val), y, lam, xmap


@pytest.mark.parametrize("fmt", [2, 1])
def test_volume_concurrent_fixed_point_is_the_map(m, volume_map, fmt):
    g, nz, N, sx, ba, (cp, row, val), y, lam, xmap = volume_map
    sigma = 5e-4
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, format=fmt)
    assert sysm.config["format"] == fmt
    assert sysm.config["rows_per_agent"] > 1
    sysm.set_relaxation(0.5)
    # r < 1e-7: the concurrent schedule's FP32 iterates level off near
    # r = 1e-8, and 1e-7 already leaves NRMSE ~2e-5 to the MAP
    x, info = sysm.solve_volume(y, lam, m.make_prior(0, sx), ba, 0.8, sigma, 20000, tol=1e-7)
    e = float(np.linalg.norm(x.reshape(-1).astype(np.float64) - xmap) / np.linalg.norm(xmap))
    print(f"volume {g} nz={nz} format {fmt}: {info.iters} iterations, r {info.residual:.2e}, "
          f"nrmse {e:.2e}",
          flush=True)
    assert info.status == m.MACE_OK
    assert e <= 1e-4


@pytest.mark.parametrize("fmt", [2, 1])
def test_volume_without_axial_cliques_is_independent_slices(m, fmt):
    g = mi.Geometry(24, 24, 24, 36)
    nz, N, sx, sigma = 3, 2, 0.002, 0.001
    (cp, row, val), y, lam, _ = _volume(g, nz, 41, N, 1, sx, 0.0, 1.2)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=8,
                    rows_per_agent=1, format=fmt)
    prior = m.make_prior(1, sx, 2.0, 1.2, 1.0)
    xv, _ = sysm.solve_volume(y, lam, prior, 0.0, 0.8, sigma, 5)
    for z in range(nz):
        xs, _ = sysm.solve(y[z], lam[z], prior, 0.8, sigma, 5)
        assert np.abs(xv[z] - xs).max() <= 1e-6 * np.abs(xs).max()


def test_volume_argument_errors(m):
    g = mi.Geometry(24, 24, 24, 36)
    (cp, row, val), y, lam, _ = _volume(g, 2, 5, 2, 0, 0.002, 0.5)
    prior = m.make_prior(0, 0.002)
    fp16 = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 2, precision=1)
    with pytest.raises(m.MaceError) as ei:
        fp16.solve_volume(y, lam, prior, 0.5, 0.8, 0.001, 2)
    assert ei.value.code == m.MACE_E_ARG and "FP32 matrix values" in str(ei.value)
    general = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 2, format=2)
    with pytest.raises(m.MaceError) as ei:
        general.solve_volume(y, lam, prior, -1.0, 0.8, 0.001, 2)
    assert ei.value.code == m.MACE_E_ARG
    with pytest.raises(ValueError):
        general.solve_volume(y[:, :-1], lam[:, :-1], prior, 0.5, 0.8, 0.001, 2)


@pytest.mark.parametrize("fmt", [2, 1])
def test_volume_of_one_slice_is_the_2d_solve(m, fmt):
    """nz = 1: no axial neighbour exists, so the volume is the slice's own
    2-D problem, whatever b_axial says."""
    g = mi.Geometry(24, 24, 24, 36)
    (cp, row, val), y, lam, _ = _volume(g, 1, 63, 2, 1, 0.002, 0.5, 1.2)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 2, sv_size=8,
                    rows_per_agent=1, format=fmt)
    prior = m.make_prior(1, 0.002, 2.0, 1.2, 1.0)
    xv, iv = sysm.solve_volume(y, lam, prior, 0.5, 0.8, 0.001, 5)
    xs, i2 = sysm.solve(y[0], lam[0], prior, 0.8, 0.001, 5)
    assert np.abs(xv[0] - xs).max() <= 1e-6 * np.abs(xs).max()
    assert abs(iv.residual - i2.residual) <= 1e-5 * i2.residual


def test_volume_of_128_slices_matches_oracle(m):
    """The largest volume (128 slices, every scan slot), sequential schedule:
    the trajectory equals the oracle's 3-D one in the GPU's visiting order."""
    g = mi.Geometry(16, 16, 8, 24)
    nz, N, S, iters = 128, 2, 8, 2
    (cp, row, val), y, lam, O = _volume(g, nz, 900, N, 0, 0.003, 0.5)
    print(f"volume of {nz} slices {g}", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=S,
                    rows_per_agent=1, format=1)
    prior = m.make_prior(0, 0.003)
    x, info = sysm.solve_volume(y, lam, prior, 0.5, 0.8, 0.002, iters)
    order = _volume_order(sysm, g, nz, S)
    ref = O.mace_solve(0.8, 0.002, iters, order=order, mode=oracle.MODE_SURROGATE)
    scale = np.abs(ref["x"]).max()
    assert np.abs(x.reshape(-1) - ref["x"]).max() <= 5e-5 * scale
    assert abs(info.residual - ref["resid"][-1]) <= 1e-3 * ref["resid"][-1] + 1e-7


def test_volume_slice_count_out_of_range(m):
    """nz outside [1, 128] is an argument error at the C ABI, raised before
    any input is read."""
    import ctypes
    g = mi.Geometry(16, 16, 8, 24)
    cp, row, val = mi.system_matrix(g)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 2)
    prior = m.make_prior(0, 0.003)
    y = np.zeros(g.n_rows, dtype=np.float32)
    x = np.zeros(g.n, dtype=np.float32)
    info = m.Info()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    for nz in (0, -1, 129):
        rc = m._lib.mace_solve_volume(sysm._h, nz, p(y), p(y), ctypes.byref(prior), 0.5, 0.8,
                                      0.002, 1, 2, 0.0, p(x), ctypes.byref(info))
        assert rc == m.MACE_E_ARG, (nz, rc)
        assert "nz must be in [1, 128]" in m.last_error()


def _group_order(sysm, g, nz, S, Z):
    """The GPU's sequential visiting order with slice groups of Z: colour c,
    then the even groups, then the odd ones; inside a group each
    super-voxel (in the 2-D visiting order) through the group's slices in
    turn, raster order inside."""
    o2 = sysm.visit_order()
    col = ((o2 % g.nx) // S & 1) + 2 * ((o2 // g.nx) // S & 1)
    gx = (g.nx + S - 1) // S
    svid = (o2 // g.nx // S) * gx + (o2 % g.nx) // S
    ngroups = (nz + Z - 1) // Z
    out = []
    for c in range(4):
        part, sv = o2[col == c], svid[col == c]
        runs = np.split(part, np.flatnonzero(np.diff(sv)) + 1)
        for par in (0, 1):
            for gi in range(par, ngroups, 2):
                for run in runs:
                    for z in range(gi * Z, min(nz, (gi + 1) * Z)):
                        out.append(z * g.n + run)
    return np.concatenate(out)


GROUP_CASES = [
    # geometry, nz, N, prior kind, sigma_x, q, b_axial, sigma, S, iterations, format, slices per group
    (mi.Geometry(24, 24, 24, 36), 4, 2, 1, 0.002, 1.2, 0.5, 0.001, 8, 3, 1, 2),
    (mi.Geometry(20, 18, 30, 30), 7, 3, 0, 0.003, 2.0, 0.25, 0.002, 4, 3, 1, 3),   # ragged last group
    (mi.Geometry(24, 24, 24, 36), 4, 2, 1, 0.002, 1.2, 0.5, 0.001, 8, 3, 2, 2),
    (mi.Geometry(20, 18, 30, 30), 5, 3, 0, 0.003, 2.0, 1.0, 0.002, 4, 3, 2, 8),   # one group
]


@pytest.mark.parametrize("case", GROUP_CASES,
                         ids=lambda c: f"{c[0].nx}x{c[0].ny}z{c[1]}_N{c[2]}_S{c[8]}_f{c[10]}_G{c[11]}")
def test_slice_groups_sequential_trajectory_matches_oracle(m, case):
    g, nz, N, kind, sx, q, ba, sigma, S, iters, fmt, Z = case
    (cp, row, val), y, lam, O = _volume(g, nz, 501 + g.nx, N, kind, sx, ba, q)
    print(f"slice groups of {Z}: {g} nz={nz} N={N} S={S} format={fmt}", flush=True)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=S,
                    rows_per_agent=1, format=fmt)
    sysm.set_slice_group(Z)
    prior = m.make_prior(kind, sx, 2.0, q, 1.0)
    x, info = sysm.solve_volume(y, lam, prior, ba, 0.8, sigma, iters)
    order = _group_order(sysm, g, nz, S, Z)
    assert np.array_equal(np.sort(order), np.arange(nz * g.n))
    ref = O.mace_solve(0.8, sigma, iters, order=order, mode=oracle.MODE_SURROGATE)
    scale = np.abs(ref["x"]).max()
    assert np.all(np.isfinite(x))
    assert np.abs(x.reshape(-1) - ref["x"]).max() <= 5e-5 * scale
    for z in range(nz):
        _, Xz = sysm.slot_state(z)
        err = np.abs(Xz - ref["X"][:, z * g.n:(z + 1) * g.n]).max()
        assert err <= 5e-5 * scale, (z, err / scale)
    assert abs(info.residual - ref["resid"][-1]) <= 1e-3 * ref["resid"][-1] + 1e-7


@pytest.mark.parametrize("fmt", [1, 2])
def test_slice_groups_concurrent_fixed_point_is_the_map(m, volume_map, fmt):
    g, nz, N, sx, ba, (cp, row, val), y, lam, xmap = volume_map
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, format=fmt)
    sysm.set_relaxation(0.5)
    sysm.set_slice_group(2)
    x, info = sysm.solve_volume(y, lam, m.make_prior(0, sx), ba, 0.8, 5e-4, 20000, tol=1e-7)
    e = float(np.linalg.norm(x.reshape(-1).astype(np.float64) - xmap) / np.linalg.norm(xmap))
    print(f"slice groups of 2, format {fmt}: {info.iters} iterations, r {info.residual:.2e}, "
          f"nrmse {e:.2e}", flush=True)
    assert info.status == m.MACE_OK
    assert e <= 1e-4


def test_slice_group_argument_errors(m):
    g = mi.Geometry(16, 16, 8, 24)
    cp, row, val = mi.system_matrix(g)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 2)
    for bad in (0, -2, 129):
        with pytest.raises(m.MaceError) as ei:
            sysm.set_slice_group(bad)
        assert ei.value.code == m.MACE_E_ARG
