#!/usr/bin/env python3
"""Benchmark: partial-update MACE on the 512x512 / 720-view / 736-channel /
16-agent scan (q-GGMRF prior), one GPU.

A step is one whole scan reconstruction: load the scan's state (error
sinogram, weights, theta2, w = 0, X = 0), then 60 Mann iterations of 4
super-voxel colour phases each plus the consensus epilogue, then the output
image.  The system matrix is loaded once per geometry before timing (it is
precomputed for a fixed scanner); y and Lambda are resident in HBM when the
timed region starts.  value = agent-voxel updates per second over the timed
steps (one update = one coordinate step of one agent, Algorithm 2).

Prints ONE JSON line.  --gpus N > 1 is not supported (one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_per_iter(nnz, N, n, K_rows_total):
    """Bytes one Mann iteration must move at minimum (FP32 path):
    the system matrix once (FP32 value + int32 row index per nonzero), the
    agent state per agent-voxel update (X read+write, w read+write, w-bar read:
    20 B) and each agent's error sinogram and weights once per sweep (e read +
    write, Lambda read: 12 B per row)."""
    return nnz * 8 + N * n * 20 + K_rows_total * 12


def kernel_source_hash(csrc):
    """Short hash of the sweep kernel's sources (template header + units)."""
    import hashlib
    hh = hashlib.sha256()
    for f in ("mace_internal.h", "mace_sweep.h", "mace_sweep_s8f32.hip"):
        hh.update(open(os.path.join(csrc, f), "rb").read())
    return hh.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    or None when the kernel source has changed since the counters were taken."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1911_09278_amd", "csrc")
    summ = os.path.join(ROOT, "profiles", "sv_kernel_scan512_hbm_counters.md")
    try:
        h = kernel_source_hash(csrc)
        txt = open(summ).read()
    except OSError:
        return None
    m_h = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", txt)
    m_t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_h or not m_t or m_h.group(1) != h:
        return None
    return float(m_t.group(1))


def cpu_baseline(g, cp, row, val, scan, va, w8, sigma, budget_s=20.0):
    """The FP64 oracle (as it stands) on a bounded sample: whole Mann iterations
    of the same scan, timed on this host."""
    import oracle
    O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, scan.y, scan.lam, va,
                      w8.prior_kind, w8.sigma_x, w8.p, w8.q, w8.T)
    t0 = time.perf_counter()
    O.mace_solve(w8.rho, sigma, 1)
    t1 = time.perf_counter() - t0
    iters = max(1, min(200, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    O.mace_solve(w8.rho, sigma, iters)
    dt = time.perf_counter() - t0
    upd = iters * w8.n_agents * g.n
    return {"value": upd / dt, "unit": "voxel-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{iters} Mann iteration(s) of the same 512x512 16-agent scan "
                      f"({upd} agent-voxel updates, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--sigma", type=float, default=1e-4)
    ap.add_argument("--rows-per-agent", type=int, default=0)
    ap.add_argument("--sv-size", type=int, default=0)
    ap.add_argument("--relax", type=float, default=0.5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        n = 1 << 28  # 2^28 floats = 1 GiB
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                          "launches": 3}))
        return
    import mace_inputs as mi
    from __graft_entry__ import _ensure_built
    _ensure_built()
    import paper_1911_09278_amd as m

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w8 = mi.WORKLOADS["scan512"]
    g = w8.geom
    log("generating system matrix and scan")
    cp, row, val = mi.system_matrix(g)
    scan = mi.scan(g, w8.seed)
    va = mi.interleaved_partition(g.n_views, w8.n_agents)
    nnz = int(cp[-1])
    log(f"nnz={nnz}; loading system")
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w8.n_agents,
                    rows_per_agent=args.rows_per_agent, sv_size=args.sv_size)
    sysm.set_relaxation(args.relax)
    prior = m.make_prior(w8.prior_kind, w8.sigma_x, w8.p, w8.q, w8.T)
    dev = torch.device("cuda:0")
    y = torch.from_numpy(scan.y).to(dev)
    lam = torch.from_numpy(scan.lam).to(dev)
    x = torch.empty(g.n, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream

    def step():
        return sysm.solve_dev(y.data_ptr(), lam.data_ptr(), prior, w8.rho, args.sigma,
                              args.iters, x.data_ptr(), stream_ptr=sp)

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    log("timed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        info = step()  # returns after its stream has finished
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert np.isfinite(info.residual), "non-finite residual"
    updates = args.steps * args.iters * w8.n_agents * g.n
    value = updates / dt
    K_rows = g.n_views * g.n_channels
    bytes_iter = algorithmic_bytes_per_iter(nnz, w8.n_agents, g.n, K_rows)

    # dominant kernel: the super-voxel sweep, timed with HIP events on the
    # solve's stream over one more scan
    sysm.set_timing(True)
    tinfo = step()
    sysm.set_timing(False)
    launches = tinfo.sweep_launches
    avg_launch_s = tinfo.sweep_ms / 1e3 / launches
    bytes_launch = bytes_iter / 4.0  # one launch = one of 4 colour phases
    achieved = bytes_launch / avg_launch_s / 1e9
    out = {
        "metric": "agent-voxel updates/s (HBM GB/s, p50/p99 scan latency alongside)",
        "value": value,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "scan512: 512x512 image, 720 views, 736 channels, 16 agents, "
                               "q-GGMRF p=2 q=1.2 T=1 sigma_x=0.01, rho=0.8",
                   "mann_iters": args.iters, "sigma": args.sigma, "relaxation": args.relax,
                   "nnz": nnz, "sv_size": args.sv_size or 8,
                   "rows_per_agent": args.rows_per_agent or "auto"},
        "hbm_gbps_algorithmic": bytes_iter * args.steps * args.iters / dt / 1e9,
        "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
        "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
        "final_residual": info.residual,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "sv_kernel sweep", "avg_launch_us": avg_launch_s * 1e6,
                     "bytes_per_launch": bytes_launch},
    }
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(g, cp, row, val, scan, va, w8, args.sigma)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
