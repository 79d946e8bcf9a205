"""Host-side checks of the C ABI that run without a GPU: the library loads,
exports every function include/mace.h declares, and rejects malformed input
before touching the device."""
import os
import re
import sys

import numpy as np
import pytest

import mace_inputs as mi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mace.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mace_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1911_09278_amd as m
    names = _declared()
    assert "mace_load_system" in names and "mace_solve" in names and "mace_prox" in names
    for nm in names:
        assert hasattr(m._lib, nm), nm
    assert set(names) <= set(m.EXPORTED)


def test_library_has_no_oracle_dependency():
    # the product library links no oracle code
    import paper_1911_09278_amd as m
    out = open(m.LIB_PATH, "rb").read()
    assert b"orc_" not in out and b"mace_oracle" not in out


def _small():
    g = mi.Geometry(16, 16, 24, 24)
    return g, mi.system_matrix(g)


def test_rejects_malformed_csc():
    import paper_1911_09278_amd as m
    g, (cp, row, val) = _small()
    bad = row.copy()
    bad[5] = bad[4]
    with pytest.raises(m.MaceError) as e:
        m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, bad, val, 4)
    assert e.value.code == m.MACE_E_MATRIX
    bad = row.copy()
    bad[0] = g.n_rows
    with pytest.raises(m.MaceError) as e:
        m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, bad, val, 4)
    assert e.value.code == m.MACE_E_MATRIX
    v2 = val.copy()
    v2[3] = np.nan
    with pytest.raises(m.MaceError) as e:
        m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, v2, 4)
    assert e.value.code == m.MACE_E_MATRIX
    cp2 = cp.copy()
    cp2[0] = 1
    with pytest.raises(m.MaceError) as e:
        m.System(g.nx, g.ny, g.n_views, g.n_channels, cp2, row, val, 4)
    assert e.value.code == m.MACE_E_MATRIX


def test_rejects_bad_partition_and_args():
    import paper_1911_09278_amd as m
    g, (cp, row, val) = _small()
    va = np.zeros(g.n_views, dtype=np.int32)  # agents 1..3 own nothing
    with pytest.raises(m.MaceError) as e:
        m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 4, view_to_agent=va)
    assert e.value.code == m.MACE_E_PARTITION
    va = np.full(g.n_views, 7, dtype=np.int32)
    with pytest.raises(m.MaceError) as e:
        m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 4, view_to_agent=va)
    assert e.value.code == m.MACE_E_PARTITION
    with pytest.raises(m.MaceError) as e:
        m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 0)
    assert e.value.code == m.MACE_E_ARG
    with pytest.raises(m.MaceError) as e:
        m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 4, precision=3)
    assert e.value.code == m.MACE_E_ARG
    with pytest.raises(m.MaceError) as e:
        m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 2, format=3)
    assert e.value.code == m.MACE_E_ARG
    with pytest.raises(m.MaceError) as e:
        m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 2, sv_size=12)
    assert e.value.code == m.MACE_E_ARG


def test_record_format_choice():
    """The compact records cover 1 mm channels with at most 128 views per
    agent and 4 / 8 pixel super-voxels; anything else takes the general
    records (check_layout builds and checks either without a device)."""
    import paper_1911_09278_amd as m
    # one agent with more than 128 views: general records only
    g2 = mi.Geometry(8, 8, 130, 12)
    cp3, row3, val3 = mi.system_matrix(g2)
    assert m.check_layout(g2.nx, g2.ny, g2.n_views, g2.n_channels, cp3, row3, val3, 1) > 0
    with pytest.raises(m.MaceError) as e:
        m.check_layout(g2.nx, g2.ny, g2.n_views, g2.n_channels, cp3, row3, val3, 1, format=1)
    assert e.value.code == m.MACE_E_ARG
    with pytest.raises(m.MaceError) as e:  # FP16 values need the compact records
        m.check_layout(g2.nx, g2.ny, g2.n_views, g2.n_channels, cp3, row3, val3, 1, precision=1)
    assert e.value.code == m.MACE_E_ARG
    # channel spacing 0.4 mm: a 1 mm pixel covers up to 4 channels per view
    g = mi.Geometry(8, 8, 6, 40, pix=1.0, chan=0.4)
    cp, row, val = mi.system_matrix(g)
    assert m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 2) > 0
    with pytest.raises(m.MaceError) as e:
        m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 2, format=1)
    assert e.value.code == m.MACE_E_MATRIX
    # super-voxels of 16 and 32 pixels
    g3 = mi.Geometry(40, 40, 48, 60)
    cp4, row4, val4 = mi.system_matrix(g3)
    for S in (16, 32):
        assert m.check_layout(g3.nx, g3.ny, g3.n_views, g3.n_channels, cp4, row4, val4, 2,
                              sv_size=S) > 0


GENERAL_CASES = [
    # geometry, agents, super-voxel side
    (mi.Geometry(24, 24, 30, 64, pix=1.0, chan=0.4), 2, 4),   # 0.4 mm channels
    (mi.Geometry(20, 22, 24, 90, pix=1.0, chan=0.3), 3, 8),   # up to 6 channels per view
    (mi.Geometry(16, 16, 720, 24), 1, 4),                     # 720 views, one agent
    (mi.Geometry(36, 36, 48, 56), 4, 16), (mi.Geometry(40, 33, 48, 60), 2, 32),
    (mi.Geometry(24, 24, 4, 8), 4, 8),                        # empty columns
]


@pytest.mark.parametrize("case", GENERAL_CASES,
                         ids=lambda c: f"{c[0].nx}x{c[0].ny}v{c[0].n_views}c{c[0].chan}_N{c[1]}_S{c[2]}")
def test_general_layout_indices_in_bounds(case):
    import paper_1911_09278_amd as m
    g, N, S = case
    cp, row, val = mi.system_matrix(g)
    lds = m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=S,
                         format=2)
    assert 0 < lds <= 160 * 1024


def test_general_band_too_large_for_lds():
    """One agent with all 720 views of a 32x32 image: 8x8 super-voxels fit
    one row of 16 lanes per workgroup (89 KB); 16x16 ones need more than a
    CU's 160 KiB for one row and are refused with the size and the fix."""
    import paper_1911_09278_amd as m
    g = mi.Geometry(32, 32, 720, 48)
    cp, row, val = mi.system_matrix(g)
    lds = m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 1, sv_size=8,
                         format=2)
    assert 80 * 1024 < lds <= 160 * 1024
    with pytest.raises(m.MaceError) as e:
        m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 1, sv_size=16, format=2)
    assert e.value.code == m.MACE_E_ARG
    assert "more than 160 KiB of LDS per row" in str(e.value) and "smaller sv_size" in str(e.value)


LAYOUT_CASES = [
    (mi.Geometry(32, 32, 64, 48), 4, 4), (mi.Geometry(42, 38, 180, 64), 4, 4),
    (mi.Geometry(24, 24, 100, 40), 2, 8), (mi.Geometry(20, 20, 30, 32), 1, 4),
    (mi.Geometry(32, 32, 90, 48), 3, 4), (mi.Geometry(40, 40, 96, 60), 4, 4),
    (mi.Geometry(48, 48, 96, 72), 4, 4), (mi.Geometry(64, 64, 90, 96), 4, 4),
    (mi.Geometry(33, 17, 45, 40), 3, 8), (mi.Geometry(16, 16, 24, 24), 8, 4),
    # 75 to 128 views per agent: bands too large for 16 rows per workgroup
    (mi.Geometry(24, 24, 150, 40), 2, 8), (mi.Geometry(26, 26, 200, 40), 2, 4),
    (mi.Geometry(20, 20, 128, 32), 1, 8),
    # 4 views on 8 channels: empty columns, one view per agent
    (mi.Geometry(24, 24, 4, 8), 4, 4), (mi.Geometry(24, 24, 4, 8), 2, 8),
    (mi.Geometry(21, 19, 40, 32), 2, 4),
]


@pytest.mark.parametrize("case", LAYOUT_CASES,
                         ids=lambda c: f"{c[0].nx}x{c[0].ny}v{c[0].n_views}_N{c[1]}_S{c[2]}")
def test_device_layout_indices_in_bounds(case):
    import paper_1911_09278_amd as m
    g, N, S = case
    cp, row, val = mi.system_matrix(g)
    for prec in (0, 1):
        lds = m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, N, sv_size=S,
                             precision=prec, fp32_tail_iters=2)
        assert 0 < lds <= 160 * 1024


@pytest.mark.slow
def test_device_layout_scan512():
    import paper_1911_09278_amd as m
    w = mi.WORKLOADS["scan512"]
    g = w.geom
    cp, row, val = mi.system_matrix(g)
    lds = m.check_layout(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w.n_agents)
    assert lds <= 160 * 1024


def test_server_rejects_bad_arguments_without_a_device():
    import ctypes
    import paper_1911_09278_amd as m
    L = m._lib
    h = ctypes.c_void_p()
    assert L.mace_server_create(None, 0, 0, ctypes.byref(h)) == m.MACE_E_ARG
    assert not h.value
    arr = (ctypes.c_void_p * 1)(None)
    assert L.mace_server_create(arr, 1, 0, ctypes.byref(h)) == m.MACE_E_ARG
    t = ctypes.c_int64(0)
    pr = m.make_prior(0, 0.01)
    assert L.mace_server_submit(None, 0, None, None, ctypes.byref(pr), 0.8, 0.01, 1, 0.0, 10,
                                ctypes.byref(t)) == m.MACE_E_ARG
    assert L.mace_server_wait(None, 1, None, None, None) == m.MACE_E_ARG
    assert L.mace_server_stats(None, None) == m.MACE_E_ARG
    L.mace_server_destroy(None)
    assert L.mace_scan_bytes(None) == 0


def test_batch_and_autotune_reject_bad_arguments_without_a_device():
    import ctypes
    import paper_1911_09278_amd as m
    L = m._lib
    pr = m.make_prior(0, 0.01)
    info = (m.Info * 2)()
    assert L.mace_solve_batch(None, 2, None, None, ctypes.byref(pr), 0.8, 0.01, 1, 10, 0.0,
                              None, info) == m.MACE_E_ARG
    assert L.mace_solve_batch_dev(None, 2, None, None, ctypes.byref(pr), 0.8, 0.01, 1, 10, 0.0,
                                  None, info, None) == m.MACE_E_ARG
    assert L.mace_solve_pnp(None, None, None, 0.8, 0.01, 1, 10, 0.0, 1, None, None) == m.MACE_E_ARG
    best = m.Opts()
    g = m.Geom(8, 8, 4, 8)
    assert L.mace_autotune(None, None, None, None, 2, None, None, 4, ctypes.byref(best), None,
                           None, 0, None) == m.MACE_E_ARG
    cp = np.zeros(65, dtype=np.int64)
    row = np.zeros(1, dtype=np.int32)
    val = np.zeros(1, dtype=np.float32)
    assert L.mace_autotune(ctypes.byref(g), cp.ctypes.data, row.ctypes.data, val.ctypes.data, 0,
                           None, None, 4, ctypes.byref(best), None, None, 0,
                           None) == m.MACE_E_ARG
    assert L.mace_autotune(ctypes.byref(g), cp.ctypes.data, row.ctypes.data, val.ctypes.data, 2,
                           None, None, 0, ctypes.byref(best), None, None, 0,
                           None) == m.MACE_E_ARG
    assert L.mace_get_config(None, ctypes.byref(best)) == m.MACE_E_ARG
    assert "NULL" in m.last_error()


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU and says so for --gpus N > 1 (exit 2)."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_binding_refuses_to_import_without_the_library(tmp_path):
    """No fallback: the package raises at import when libmace.so is not built."""
    import shutil
    import subprocess
    pkg = tmp_path / "paper_1911_09278_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1911_09278_amd", "__init__.py"), pkg / "__init__.py")
    r = subprocess.run([sys.executable, "-c", "import paper_1911_09278_amd"], cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libmace.so is missing" in r.stderr
