"""A solve that fails on device memory leaves its system usable.

The library's allocation-failure hook makes the k-th device allocation of a
solve fail, for every allocation the first solve on a fresh system makes
(its input copies, the scan slot's buffers, the slot table).  That solve
must report MACE_E_NOMEM; the next solve on the same system must allocate
what is missing and return exactly the result of an undisturbed system (the
sequential schedule is deterministic), never running a kernel on a buffer
that was not allocated.
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


def test_failed_allocation_then_retry(m):
    g = mi.Geometry(32, 32, 64, 48)
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, 51)
    prior = m.make_prior(1, 0.002, 2.0, 1.2, 1.0)

    def load():
        return m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 4, rows_per_agent=1)

    ref = load()
    x_ref, i_ref = ref.solve(s.y, s.lam, prior, 0.8, 0.002, 6)
    ref.close()
    failed = 0
    for k in range(24):
        sysm = load()
        print("allocation", k, flush=True)
        m.test_fail_alloc(k)
        try:
            x1, _ = sysm.solve(s.y, s.lam, prior, 0.8, 0.002, 6)
            hit = False
        except m.MaceError as e:
            assert e.code == m.MACE_E_NOMEM, e
            hit = True
        finally:
            m.test_fail_alloc(-1)
        if hit:
            failed += 1
        else:
            assert np.array_equal(x1, x_ref)
        x2, info = sysm.solve(s.y, s.lam, prior, 0.8, 0.002, 6)
        assert np.array_equal(x2, x_ref), k
        assert info.residual == i_ref.residual
        sysm.close()
    # the first solve on a system makes more than a dozen allocations
    assert failed >= 12, failed
