"""GPU test of the library under concurrent host threads.

Two threads solve on two systems at once (each solve captures its iteration
graph on its own stream) while a third thread loads and frees another system
(device allocations).  With the sequential schedule every solve is
deterministic, so each result must equal the same solve run alone.
"""
import threading

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


def test_threads_solve_and_load_concurrently(m):
    ga, gb, gc = mi.Geometry(32, 32, 64, 48), mi.Geometry(48, 48, 96, 72), mi.Geometry(40, 40, 96, 60)
    mats = {g: mi.system_matrix(g) for g in (ga, gb, gc)}
    prior = m.make_prior(1, 0.002, 2.0, 1.2, 1.0)
    iters = 12

    def load(g, N=4):
        cp, row, val = mats[g]
        return m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=4,
                        rows_per_agent=1)

    sa, sb = load(ga), load(gb)
    scans = {ga: [mi.scan(ga, 71 + i) for i in range(3)], gb: [mi.scan(gb, 81 + i) for i in range(3)]}
    alone = {g: [sys_.solve(s.y, s.lam, prior, 0.8, 0.002, iters)[0] for s in scans[g]]
             for g, sys_ in ((ga, sa), (gb, sb))}
    print("alone runs done", flush=True)

    out = {ga: [], gb: []}
    errors = []

    def solver(g, sys_):
        try:
            for s in scans[g]:
                out[g].append(sys_.solve(s.y, s.lam, prior, 0.8, 0.002, iters)[0])
        except Exception as e:  # surfaced below
            errors.append(e)

    def loader():
        try:
            for _ in range(3):
                sc = load(gc)
                sc.close()
        except Exception as e:
            errors.append(e)

    th = [threading.Thread(target=solver, args=(ga, sa)), threading.Thread(target=solver, args=(gb, sb)),
          threading.Thread(target=loader)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for g in (ga, gb):
        assert len(out[g]) == len(scans[g])
        for x, xa in zip(out[g], alone[g]):
            assert np.array_equal(x, xa)
    print("threaded runs equal the single-threaded ones", flush=True)
