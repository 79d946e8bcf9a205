"""GPU test of the allocation-free solve (mace_solve_dev_noalloc).

It must return what mace_solve_dev returns for the same system and inputs.
With the sequential schedule (one super-voxel of an agent at a time) both
entry points are deterministic and run the same kernels with the same
arguments, so the images, residuals and iteration counts must be identical.
Two calls in a row, the second on a smaller system, check that the static
workspace carries nothing from one call to the next (compact and general
record formats); a concurrent-schedule
case checks the fixed point to the FP32 tolerance; a system whose scan state
exceeds the workspace is refused before any launch.
"""
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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _both(m, sysm, s, prior, sigma, iters, tol=0.0, w0=None):
    import torch
    y, lam = _dev(s.y), _dev(s.lam)
    wd = None if w0 is None else _dev(w0)
    xa = torch.full((sysm.n,), float("nan"), device="cuda")
    xb = torch.full((sysm.n,), float("nan"), device="cuda")
    ia = sysm.solve_dev(y.data_ptr(), lam.data_ptr(), prior, 0.8, sigma, iters, xa.data_ptr(),
                        tol=tol, w_init_ptr=None if wd is None else wd.data_ptr())
    ib = sysm.solve_dev_noalloc(y.data_ptr(), lam.data_ptr(), prior, 0.8, sigma, iters,
                                xb.data_ptr(), tol=tol,
                                w_init_ptr=None if wd is None else wd.data_ptr())
    torch.cuda.synchronize()
    return xa.cpu().numpy(), ia, xb.cpu().numpy(), ib


def test_noalloc_equals_solve_dev_twice_second_smaller(m):
    prior = m.make_prior(1, 0.002, 2.0, 1.2, 1.0)
    cases = [(mi.Geometry(48, 48, 96, 72), 4, 31), (mi.Geometry(24, 24, 40, 32), 2, 32)]
    for g, N, seed in cases:
        print("case", g, "N", N, flush=True)
        cp, row, val = mi.system_matrix(g)
        s = mi.scan(g, seed)
        sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, rows_per_agent=1)
        xa, ia, xb, ib = _both(m, sysm, s, prior, 0.002, 9)
        assert np.all(np.isfinite(xb))
        assert np.array_equal(xa, xb), np.abs(xa - xb).max()
        assert ia.iters == ib.iters == 9 and ia.residual == ib.residual
        sysm.close()


def test_noalloc_general_records_equal_solve_dev(m):
    """The general record format (0.4 mm channels: several nonzeros of a
    column per view) through both entry points, sequential schedule: the
    same image, residual and iteration count, on two calls in a row, the
    second smaller."""
    prior = m.make_prior(1, 0.002, 2.0, 1.2, 1.0)
    cases = [(mi.Geometry(32, 32, 48, 113, pix=1.0, chan=0.4), 2, 41),
             (mi.Geometry(24, 24, 30, 64, pix=1.0, chan=0.4), 2, 42)]
    for g, N, seed in cases:
        print("general records", g, "N", N, flush=True)
        cp, row, val = mi.system_matrix(g)
        s = mi.scan(g, seed)
        sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, rows_per_agent=1,
                        format=2)
        assert sysm.config["format"] == 2
        xa, ia, xb, ib = _both(m, sysm, s, prior, 0.002, 6)
        assert np.all(np.isfinite(xb))
        assert np.array_equal(xa, xb), np.abs(xa - xb).max()
        assert ia.iters == ib.iters == 6 and ia.residual == ib.residual
        sysm.close()


def test_noalloc_warm_start_and_tolerance(m):
    g = mi.Geometry(32, 32, 64, 48)
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, 33)
    N = 4
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, rows_per_agent=1)
    sysm.set_relaxation(0.5)
    prior = m.make_prior(0, 0.002)
    rng = np.random.default_rng(1)
    w0 = rng.uniform(0.0, 0.03, N * g.n).astype(np.float32)
    xa, ia, xb, ib = _both(m, sysm, s, prior, 0.001, 2000, tol=1e-5, w0=w0)
    assert ia.status == ib.status == m.MACE_OK
    assert ia.iters == ib.iters and ia.residual == ib.residual < 1e-5
    assert np.array_equal(xa, xb)


def test_noalloc_zero_iterations(m):
    """max_iters = 0: both entry points return mean_i w_init with no
    iteration counted, and MACE_W_MAXITER when a tolerance is set."""
    g = mi.Geometry(24, 24, 40, 32)
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, 36)
    N = 2
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N)
    prior = m.make_prior(0, 0.002)
    w0 = np.random.default_rng(2).uniform(0.0, 0.03, N * g.n).astype(np.float32)
    xa, ia, xb, ib = _both(m, sysm, s, prior, 1e-3, 0, w0=w0)
    assert np.array_equal(xa, xb)
    assert ia.iters == ib.iters == 0 and ia.status == ib.status == m.MACE_OK
    xa, ia, xb, ib = _both(m, sysm, s, prior, 1e-3, 0, tol=1e-3)
    assert ia.status == ib.status == m.MACE_W_MAXITER and np.all(xb == 0.0)
    sysm.close()


def test_noalloc_concurrent_schedule_same_fixed_point(m):
    """Concurrent super-voxels (float atomics: not bit-reproducible); both
    entry points reach the same fixed point within the FP32 tolerance."""
    g = mi.Geometry(64, 64, 90, 96)
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, 34)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 4)
    assert sysm.config["rows_per_agent"] > 1
    sysm.set_relaxation(0.5)
    prior = m.make_prior(0, 0.001)
    xa, ia, xb, ib = _both(m, sysm, s, prior, 5e-4, 20000, tol=1e-8)
    assert ia.status == ib.status == m.MACE_OK
    assert np.linalg.norm(xb - xa) / np.linalg.norm(xa) <= 1e-5


def test_noalloc_refuses_a_scan_larger_than_the_workspace(m):
    import torch
    g = mi.Geometry(192, 192, 96, 272)
    N = 48  # 48 agents x 36864 pixels x 3 images x 4 B = 21 MB > 16 MiB
    cp, row, val = mi.system_matrix(g)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N)
    assert sysm.scan_bytes > m.noalloc_capacity()
    s = mi.scan(g, 35)
    y, lam = _dev(s.y), _dev(s.lam)
    x = torch.zeros(g.n, device="cuda")
    with pytest.raises(m.MaceError) as e:
        sysm.solve_dev_noalloc(y.data_ptr(), lam.data_ptr(), m.make_prior(0, 0.002), 0.8, 1e-3, 3,
                               x.data_ptr())
    assert e.value.code == m.MACE_E_NOMEM
    torch.cuda.synchronize()
    assert float(x.abs().max()) == 0.0  # nothing was launched into x
