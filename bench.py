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


def cpu_baseline(g, cp, row, val, scan, va, w8, sigma, budget_s=50.0):
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


def host_info():
    """CPU model, RAM and hardware threads of this host (for the CPU baseline)."""
    model, ram = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = int(line.split()[1]) * 1024
                break
    except OSError:
        pass
    return {"cpu_model": model, "ram_bytes": ram, "host_threads": os.cpu_count()}


def copy_bandwidth_gbs(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (read + write) timed with events: the
    HBM bandwidth a plain streaming kernel reaches on this GPU."""
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def bench_oracle(mi):
    """The FP64 oracle timed per Mann iteration on the 64^2 (4 agents), 512^2
    (16 agents) and 1024^2 (32 agents) workloads: the median over repeats of
    (time of 1 + K iterations - time of 1 iteration) / K, so that the set-up
    of a solve (theta2, e = y) drops out, with K sized for about 2 s (at most
    200).  The 64 batched 512^2 slices are the
    512^2 iteration times 64 (the oracle solves each slice alone), labelled
    as extrapolated.  Host only; no GPU is used."""
    import statistics
    import oracle
    res = {}
    for cfg, name, sigma, reps in (("config1", "plain64", 1e-3, 5), ("config2", "scan512", 1e-4, 5),
                                   ("config4", "scan1024", 5e-5, 3)):
        w = mi.WORKLOADS[name]
        g = w.geom
        log(f"oracle: {name}")
        cp, row, val = mi.system_matrix(g)
        sc = mi.scan(g, w.seed)
        va = mi.interleaved_partition(g.n_views, w.n_agents)
        O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, sc.y, sc.lam, va,
                          w.prior_kind, w.sigma_x, w.p, w.q, w.T)
        nnz = int(cp[-1])
        del cp, row, val
        t0 = time.perf_counter()
        O.mace_solve(w.rho, sigma, 2)
        t2 = time.perf_counter() - t0
        K = max(2, min(200, int(2.0 / max(t2 / 2.0, 1e-4))))
        per = []
        for _ in range(reps):
            t0 = time.perf_counter()
            O.mace_solve(w.rho, sigma, 1)
            t1 = time.perf_counter()
            O.mace_solve(w.rho, sigma, 1 + K)
            tk = time.perf_counter()
            per.append(((tk - t1) - (t1 - t0)) / K)
        del O
        med = statistics.median(per)
        res[cfg] = {"workload": f"{name}: {g.nx}x{g.ny}, {g.n_views} views, {g.n_channels} "
                                f"channels, {w.n_agents} agents, nnz {nnz}",
                    "sigma": sigma, "repeats": reps, "iterations_per_sample": K,
                    "ms_per_mann_iter": med * 1e3,
                    "voxel_updates_per_s": w.n_agents * g.n / med}
    res["config3_extrapolated"] = {
        "workload": "64 slices of 512x512 (each solved alone by the oracle)",
        "ms_per_mann_iter": 64 * res["config2"]["ms_per_mann_iter"],
        "note": "extrapolated: 64 x the 512x512 iteration"}
    return {"oracle": res, "cores": oracle.num_threads(), **host_info()}


def leg_slices(sysm, w8, m, mi, torch, sigma, iters, n_slices=64):
    """Batched slices (64 independent 512x512 slices, each its own phantom,
    sharing the loaded scan512 system): all slices advance together through
    mace_solve_batch_dev, against the same slices solved one at a time with
    mace_solve_dev, both for `iters` Mann iterations."""
    g = w8.geom
    dev = torch.device("cuda:0")
    log(f"slices: {n_slices} scans")
    ys, ls, xs = [], [], []
    for i in range(n_slices):
        sc = mi.scan(g, mi.WORKLOADS["slices512"].seed + i)
        ys.append(torch.from_numpy(sc.y).to(dev))
        ls.append(torch.from_numpy(sc.lam).to(dev))
        xs.append(torch.empty(g.n, dtype=torch.float32, device=dev))
    prior = m.make_prior(w8.prior_kind, w8.sigma_x, w8.p, w8.q, w8.T)
    sp = torch.cuda.current_stream(dev).cuda_stream
    yp, lp, xp = ([t.data_ptr() for t in v] for v in (ys, ls, xs))
    log("slices: batched")
    sysm.solve_batch_dev(yp, lp, prior, w8.rho, sigma, iters, xp, stream_ptr=sp)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info_b = sysm.solve_batch_dev(yp, lp, prior, w8.rho, sigma, iters, xp, stream_ptr=sp)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    xb = torch.stack(xs).cpu().numpy()
    log("slices: one at a time")
    t0 = time.perf_counter()
    info_s = [sysm.solve_dev(yp[i], lp[i], prior, w8.rho, sigma, iters, xp[i], stream_ptr=sp)
              for i in range(n_slices)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    x1 = torch.stack(xs).cpu().numpy()
    nnz = sysm.nnz
    rows = g.n_views * g.n_channels
    hbm_floor_ms = (nnz * 8 + n_slices * (w8.n_agents * g.n * 20 + rows * 12)) / 8e12 * 1e3
    return {"workload": f"slices512: {n_slices} slices 512x512, 720 views, 736 channels, "
                        "16 agents, one shared matrix", "mann_iters": iters, "sigma": sigma,
            "slices_per_s_batched": n_slices / tb, "slices_per_s_one_at_a_time": n_slices / ts,
            "speedup": ts / tb, "ms_per_mann_iter_batched": tb / iters * 1e3,
            "hbm_floor_ms_per_mann_iter": hbm_floor_ms,
            "mean_residual_batched": float(np.mean([i.residual for i in info_b])),
            "mean_residual_one_at_a_time": float(np.mean([i.residual for i in info_s])),
            "nrmse_batched_vs_one_at_a_time":
                float(np.sqrt(((xb - x1) ** 2).sum() / (x1 ** 2).sum()))}


def leg_fp16(m, mi, torch, iters=60):
    """1024x1024, 1440 views, 1472 channels, 32 agents (q-GGMRF): FP16 matrix
    values with a per agent-pixel scale, FP16 throughout and with the last 5
    Mann iterations on the FP32 values, against all-FP32; `iters` Mann
    iterations each.  The FP16 sweep launch is priced against the roofline
    of FP16 values + 16-bit rows (4 B per nonzero) plus the state bytes."""
    w = mi.WORKLOADS["scan1024"]
    g = w.geom
    sigma = 5e-5
    log("fp16: 1024x1024 matrix")
    cp, row, val = mi.system_matrix(g)
    sc = mi.scan(g, w.seed)
    nnz = int(cp[-1])
    prior = m.make_prior(w.prior_kind, w.sigma_x, w.p, w.q, w.T)
    dev = torch.device("cuda:0")
    y = torch.from_numpy(sc.y).to(dev)
    lam = torch.from_numpy(sc.lam).to(dev)
    x = torch.empty(g.n, dtype=torch.float32, device=dev)
    sp = torch.cuda.current_stream(dev).cuda_stream
    out = {"workload": "scan1024: 1024x1024, 1440 views, 1472 channels, 32 agents, "
                       "q-GGMRF p=2 q=1.2 T=1 sigma_x=0.01, rho=0.8",
           "mann_iters": iters, "sigma": sigma, "nnz": nnz}
    xs = {}
    for prec in (0, 1):
        log(f"fp16: loading precision {prec}")
        t = time.perf_counter()
        sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w.n_agents,
                        precision=prec, fp32_tail_iters=5 if prec else 0)
        log(f"fp16: loaded in {time.perf_counter() - t:.1f} s")
        sysm.set_relaxation(0.5)
        runs = (("fp32", 0),) if prec == 0 else (("fp16", 0), ("fp16_tail5", 5))
        for name, tail in runs:
            if prec:
                sysm.set_fp32_tail(tail)
            sysm.solve_dev(y.data_ptr(), lam.data_ptr(), prior, w.rho, sigma, iters,
                           x.data_ptr(), stream_ptr=sp)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = sysm.solve_dev(y.data_ptr(), lam.data_ptr(), prior, w.rho, sigma, iters,
                                  x.data_ptr(), stream_ptr=sp)
            dt = time.perf_counter() - t0
            xs[name] = x.cpu().numpy().astype(np.float64)
            sysm.set_timing(True)
            ti = sysm.solve_dev(y.data_ptr(), lam.data_ptr(), prior, w.rho, sigma, iters,
                                x.data_ptr(), stream_ptr=sp)
            sysm.set_timing(False)
            out[name] = {"voxel_updates_per_s": iters * w.n_agents * g.n / dt,
                         "ms_per_scan": dt * 1e3, "residual": info.residual,
                         "sweep_launch_us": ti.sweep_ms * 1e3 / ti.sweep_launches,
                         "matrix_bytes": sysm.matrix_bytes}
        sysm.close()
    del cp, row, val
    state = w.n_agents * g.n * 20 + g.n_views * g.n_channels * 12
    for name, per_nnz in (("fp32", 8), ("fp16", 4)):
        launch_bytes = (nnz * per_nnz + state) / 4.0
        ach = launch_bytes / (out[name]["sweep_launch_us"] * 1e-6) / 1e9
        out[name]["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                 "bytes_per_launch": launch_bytes,
                                 "bytes_per_nnz": per_nnz}
    ref = xs["fp32"]
    for name in ("fp16", "fp16_tail5"):
        out[name]["nrmse_vs_fp32"] = float(np.linalg.norm(xs[name] - ref) / np.linalg.norm(ref))
    return out


def leg_time_to_tol(sysm, w8, m, mi, torch, y, lam, sigma, tol=1e-4, max_iters=3000):
    """Finished reconstructions rather than iterations: the headline scan
    solved to r_k < tol (iterations, ms), and the 256x256 study problem,
    whose converged x* the oracle wrote, solved to r_k < 1e-4 and 1e-5 with
    NRMSE(x, x*) (8 agents, sigma = 2e-4, rho = 0.8, relaxation 0.5)."""
    dev = torch.device("cuda:0")
    sp = torch.cuda.current_stream(dev).cuda_stream
    prior = m.make_prior(w8.prior_kind, w8.sigma_x, w8.p, w8.q, w8.T)
    x = torch.empty(w8.geom.n, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sysm.solve_dev(y.data_ptr(), lam.data_ptr(), prior, w8.rho, sigma, max_iters,
                          x.data_ptr(), tol=tol, stream_ptr=sp)
    torch.cuda.synchronize()
    out = {"scan512": {"tol": tol, "sigma": sigma, "iters": info.iters,
                       "ms": (time.perf_counter() - t0) * 1e3, "residual": info.residual,
                       "converged": info.status == m.MACE_OK}}
    x_star, meta = load_study_reference()
    p = meta["problem"]
    g = mi.Geometry(p["nx"], p["ny"], p["n_views"], p["n_channels"])
    cp, row, val = mi.system_matrix(g)
    sc = mi.scan(g, p["seed"])
    pr = p["prior"]
    prior = m.make_prior(pr["kind"], pr["sigma_x"], pr["p"], pr["q"], pr["T"])
    s256 = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 8)
    s256.set_relaxation(0.5)
    yd = torch.from_numpy(sc.y).to(dev)
    ld = torch.from_numpy(sc.lam).to(dev)
    xd = torch.empty(g.n, dtype=torch.float32, device=dev)
    out["study256"] = {"sigma": 2e-4, "rho": 0.8, "n_agents": 8}
    for t in (1e-4, 1e-5):
        s256.solve_dev(yd.data_ptr(), ld.data_ptr(), prior, 0.8, 2e-4, 5, xd.data_ptr(),
                       stream_ptr=sp)  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s256.solve_dev(yd.data_ptr(), ld.data_ptr(), prior, 0.8, 2e-4, 20000,
                              xd.data_ptr(), tol=t, stream_ptr=sp)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        xh = xd.cpu().numpy().astype(np.float64)
        out["study256"][f"tol{t:.0e}"] = {
            "iters": info.iters, "ms": ms, "residual": info.residual,
            "nrmse_vs_xstar": float(np.linalg.norm(xh - x_star) / np.linalg.norm(x_star))}
    s256.close()
    return out


def leg_volume(m, mi, torch, iters=60, nz=16, b_axial=0.5):
    """A volume of 16 slices of 256x256 (360 views, 368 channels, 8 agents,
    q-GGMRF) with the 3-D prior's axial cliques (b_axial = 0.5 against the
    in-plane weights' sum of 1), `iters` Mann iterations through
    mace_solve_volume (host arrays in and out), with the compact and with
    the general records, also with super-voxels in groups of 8 slices,
    against the same 16 slices solved as an independent batch
    (mace_solve_batch) with the same records."""
    w = mi.WORKLOADS["serve256"]
    g = w.geom
    sigma = 2e-4
    cp, row, val = mi.system_matrix(g)
    scans = [mi.scan(g, w.seed + 100 + z) for z in range(nz)]
    y = np.stack([sc.y for sc in scans])
    lam = np.stack([sc.lam for sc in scans])
    prior = m.make_prior(w.prior_kind, w.sigma_x, w.p, w.q, w.T)
    nnz = int(cp[-1])
    rows = g.n_views * g.n_channels
    # the matrix once per colour phase and slice parity (shared by that
    # parity's slices), each slice's state and sinogram once per iteration
    hbm_floor_ms = (2 * nnz * 8 + nz * (w.n_agents * g.n * 20 + rows * 12)) / 8e12 * 1e3
    out = {"workload": f"volume256: {nz} slices of 256x256, 360 views, 368 channels, 8 agents, "
                       f"q-GGMRF, b_axial={b_axial}", "mann_iters": iters, "sigma": sigma,
           "hbm_floor_ms_per_mann_iter": hbm_floor_ms}
    for fmt, name in ((1, "compact"), (2, "general")):
        sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w.n_agents, format=fmt)
        sysm.set_relaxation(0.5)
        sysm.solve_volume(y, lam, prior, b_axial, w.rho, sigma, 2)  # warm-up
        t0 = time.perf_counter()
        _, info = sysm.solve_volume(y, lam, prior, b_axial, w.rho, sigma, iters)
        tv = time.perf_counter() - t0
        sysm.solve_batch(list(y), list(lam), prior, w.rho, sigma, 2)
        t0 = time.perf_counter()
        infos = sysm.solve_batch(list(y), list(lam), prior, w.rho, sigma, iters)[1]
        tb = time.perf_counter() - t0
        # super-voxels in groups of 8 slices (SV-ICD's slice groups)
        sysm.set_slice_group(8)
        sysm.solve_volume(y, lam, prior, b_axial, w.rho, sigma, 2)
        t0 = time.perf_counter()
        _, info8 = sysm.solve_volume(y, lam, prior, b_axial, w.rho, sigma, iters)
        tg = time.perf_counter() - t0
        out[name] = {"volume_ms_per_mann_iter": tv / iters * 1e3, "volume_residual": info.residual,
                     "volume_voxel_updates_per_s": iters * w.n_agents * g.n * nz / tv,
                     "groups8_ms_per_mann_iter": tg / iters * 1e3,
                     "groups8_residual": info8.residual,
                     "batch_ms_per_mann_iter": tb / iters * 1e3,
                     "batch_mean_residual": float(np.mean([i.residual for i in infos]))}
        sysm.close()
    return out


def leg_serve(m, mi, torch, n_arrivals=300, tol=1e-4, max_iters=3000):
    """Served 256x256 scans (360 views, 368 channels, 8 agents, q-GGMRF, a
    pool of up to 300 phantoms taken in turn) stopping at r < tol: the
    one-scan-at-a-time FP32 path (mace_solve_dev, one scan after the other),
    the server's capacity (64 scans submitted at once), then Poisson arrivals
    at 70% of that capacity; latency from submit to result, the first
    min(100, 10%) arrivals dropped as warm-up."""
    w = mi.WORKLOADS["serve256"]
    g = w.geom
    sigma = 2e-4
    cp, row, val = mi.system_matrix(g)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w.n_agents)
    del cp, row, val
    prior = m.make_prior(w.prior_kind, w.sigma_x, w.p, w.q, w.T)
    n_pool = min(n_arrivals, 300)
    log(f"serve: {n_pool + 64} scans")
    scans = [mi.scan(g, 1916000 + i) for i in range(n_pool + 64)]
    dev = torch.device("cuda:0")
    sp = torch.cuda.current_stream(dev).cuda_stream
    n_seq = 32
    ys = [torch.from_numpy(scans[i].y).to(dev) for i in range(n_seq)]
    ls = [torch.from_numpy(scans[i].lam).to(dev) for i in range(n_seq)]
    x = torch.empty(g.n, dtype=torch.float32, device=dev)
    log("serve: one scan at a time")
    sysm.solve_dev(ys[0].data_ptr(), ls[0].data_ptr(), prior, w.rho, sigma, max_iters,
                   x.data_ptr(), tol=tol, stream_ptr=sp)
    t0 = time.perf_counter()
    it_seq = []
    for i in range(n_seq):
        info = sysm.solve_dev(ys[i].data_ptr(), ls[i].data_ptr(), prior, w.rho, sigma, max_iters,
                              x.data_ptr(), tol=tol, stream_ptr=sp)
        it_seq.append(info.iters)
    seq_rate = n_seq / (time.perf_counter() - t0)
    srv = m.Server([sysm])
    log("serve: capacity (64 at once)")
    t0 = time.perf_counter()
    tk = [srv.submit(0, scans[n_pool + i].y, scans[n_pool + i].lam, prior, w.rho, sigma,
                     tol, max_iters) for i in range(64)]
    for t in tk:
        srv.wait(t, g.n)
    capacity = 64 / (time.perf_counter() - t0)
    rate = 0.7 * capacity
    log(f"serve: {n_arrivals} Poisson arrivals at {rate:.1f}/s")
    rng = np.random.default_rng(1916)
    gaps = rng.exponential(1.0 / rate, n_arrivals)
    tickets = []
    t0 = time.perf_counter()
    t_next = t0
    for i in range(n_arrivals):
        t_next += gaps[i]
        d = t_next - time.perf_counter()
        if d > 0:
            time.sleep(d)
        sc = scans[i % n_pool]
        tickets.append(srv.submit(0, sc.y, sc.lam, prior, w.rho, sigma, tol, max_iters))
    lat, its, ok = [], [], 0
    for t in tickets:
        _, info, l = srv.wait(t, g.n)
        lat.append(l)
        its.append(info.iters)
        ok += info.status == m.MACE_OK
    span = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    sysm.close()
    dropped = min(100, n_arrivals // 10)
    kept = lat[dropped:]
    return {"workload": "serve256: 256x256, 360 views, 368 channels, 8 agents, q-GGMRF "
                        f"p=2 q=1.2 T=1 sigma_x=0.01, rho=0.8, {n_pool} phantoms in turn",
            "sigma": sigma, "tol": tol, "arrivals": n_arrivals, "dropped_warmup": dropped,
            "offered_rate": rate,
            "served_rate": n_arrivals / span, "converged": ok,
            "latency_p50_ms": float(np.percentile(kept, 50) * 1e3),
            "latency_p99_ms": float(np.percentile(kept, 99) * 1e3),
            "mean_iters_served": float(np.mean(its)),
            "capacity_scans_per_s": capacity,
            "one_at_a_time_fp32_scans_per_s": seq_rate,
            "mean_iters_one_at_a_time": float(np.mean(it_seq)),
            "max_in_flight": st["max_in_flight"]}


def _common(metric, value, unit, steps, warmup, ms, dtype, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def bench_slices(args, m, mi, torch):
    """64 independent 512x512 slices (own phantoms) sharing one system matrix:
    all slices advance together through mace_solve_batch_dev (one round of
    launches per Mann iteration for every slice) versus the same slices solved
    one at a time with mace_solve_dev.  A step = all slices, 60 iterations."""
    w8 = mi.WORKLOADS["slices512"]
    g = w8.geom
    ns = args.slices
    log(f"slices: {ns} slices of 512x512; matrix")
    cp, row, val = mi.system_matrix(g)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w8.n_agents)
    del cp, row, val
    prior = m.make_prior(w8.prior_kind, w8.sigma_x, w8.p, w8.q, w8.T)
    dev = torch.device("cuda:0")
    ys, ls, xs = [], [], []
    for i in range(ns):
        sc = mi.scan(g, w8.seed + i)
        ys.append(torch.from_numpy(sc.y).to(dev))
        ls.append(torch.from_numpy(sc.lam).to(dev))
        xs.append(torch.empty(g.n, dtype=torch.float32, device=dev))
    sp = torch.cuda.current_stream(dev).cuda_stream
    yp = [t.data_ptr() for t in ys]
    lp = [t.data_ptr() for t in ls]
    xp = [t.data_ptr() for t in xs]

    def batched():
        return sysm.solve_batch_dev(yp, lp, prior, w8.rho, args.sigma, args.iters, xp, stream_ptr=sp)

    def one_by_one():
        return [sysm.solve_dev(yp[i], lp[i], prior, w8.rho, args.sigma, args.iters, xp[i],
                               stream_ptr=sp) for i in range(ns)]

    log("slices: warm-up")
    for _ in range(args.warmup):
        batched()
    one_by_one()
    torch.cuda.synchronize()
    x1 = torch.stack(xs).cpu().numpy()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info_b = batched()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    xb = torch.stack(xs).cpu().numpy()
    t0 = time.perf_counter()
    info_s = one_by_one()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    diff = float(np.sqrt(((xb - x1) ** 2).sum() / (x1 ** 2).sum()))
    upd = ns * args.iters * w8.n_agents * g.n
    out = _common("slices/s (64 x 512x512 slices sharing A, 60 Mann iterations each)",
                  ns / tb, "slices/s", args.steps, args.warmup, tb * 1e3, "f32",
                  {"workload": f"slices512: {ns} slices 512x512, 720 views, 736 channels, "
                               "16 agents, q-GGMRF p=2 q=1.2 T=1 sigma_x=0.01, rho=0.8",
                   "mann_iters": args.iters, "sigma": args.sigma, "batched": True})
    out.update({"voxel_updates_per_s": upd / tb,
                "one_at_a_time_slices_per_s": ns / ts,
                "speedup_vs_one_at_a_time": ts / tb,
                "mean_residual_batched": float(np.mean([i.residual for i in info_b])),
                "mean_residual_one_at_a_time": float(np.mean([i.residual for i in info_s])),
                "nrmse_batched_vs_one_at_a_time": diff})
    return out


SERVE_SIZES = (("serve256", 2e-4), ("scan512", 1e-4), ("scan1024", 5e-5))


def bench_serve(args, m, mi, torch):
    """Reconstruction service: Poisson arrivals (rate --rate) of scans drawn
    uniformly from 256^2/360 views/8 agents, 512^2/720/16 and 1024^2/1440/32,
    each with its own phantom, q-GGMRF prior, stopping at r_k < 1e-4.  The
    server admits them as memory allows and batches all scans in flight; the
    latency of a scan runs from its arrival to its result."""
    import threading
    rng = np.random.default_rng(2024)
    systems, pars = [], []
    for name, sigma in SERVE_SIZES:
        w = mi.WORKLOADS[name]
        g = w.geom
        log(f"serve: loading {name}")
        cp, row, val = mi.system_matrix(g)
        systems.append(m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w.n_agents))
        del cp, row, val
        pars.append((w, sigma))
    kinds = rng.integers(0, len(systems), args.scans)
    gaps = rng.exponential(1.0 / args.rate, args.scans)
    log("serve: generating scans")
    scans = [mi.scan(pars[k][0].geom, 5000 + i) for i, k in enumerate(kinds)]
    srv = m.Server(systems, hbm_budget_bytes=64 << 30)
    tickets = [None] * args.scans
    t_sub = [0.0] * args.scans

    def producer():
        t_next = time.perf_counter()
        for i, k in enumerate(kinds):
            t_next += gaps[i]
            dt = t_next - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            w, sigma = pars[k]
            prior = m.make_prior(w.prior_kind, w.sigma_x, w.p, w.q, w.T)
            t_sub[i] = time.perf_counter()
            tickets[i] = srv.submit(int(k), scans[i].y, scans[i].lam, prior, w.rho, sigma, 1e-4, 3000)

    log("serve: arrivals")
    t0 = time.perf_counter()
    th = threading.Thread(target=producer)
    th.start()
    th.join()
    lat, iters, ok = [], [], 0
    for i, k in enumerate(kinds):
        x, info, l = srv.wait(tickets[i], systems[k].n)
        lat.append(l)
        iters.append(info.iters)
        ok += info.status == m.MACE_OK
    t_end = time.perf_counter()
    st = srv.stats()
    srv.close()
    span = t_end - t0
    by = {}
    for name_i, (name, _) in enumerate(SERVE_SIZES):
        li = [lat[i] for i in range(args.scans) if kinds[i] == name_i]
        it = [iters[i] for i in range(args.scans) if kinds[i] == name_i]
        if li:
            by[name] = {"scans": len(li), "p50_ms": float(np.percentile(li, 50) * 1e3),
                        "p99_ms": float(np.percentile(li, 99) * 1e3),
                        "mean_iters": float(np.mean(it))}
    out = _common("scans/s served (Poisson arrivals, mixed sizes, stop at r < 1e-4)",
                  args.scans / span, "scans/s", args.scans, 0, span / args.scans * 1e3, "f32",
                  {"workload": f"serve: {args.scans} Poisson arrivals at {args.rate}/s, uniform "
                               "over 256^2/360 views/8 agents, 512^2/720/16, 1024^2/1440/32; "
                               "q-GGMRF p=2 q=1.2 T=1 sigma_x=0.01, rho=0.8, tol 1e-4",
                   "sigma": {n: sg for n, sg in SERVE_SIZES}})
    out.update({"latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
                "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
                "offered_rate": args.rate, "converged": ok, "by_size": by,
                "max_in_flight": st["max_in_flight"], "peak_state_bytes": st["peak_bytes"]})
    return out


def bench_fp16(args, m, mi, torch):
    """1024x1024, 1440 views, 1472 channels, 32 agents, q-GGMRF: system
    matrix values in FP16 (per agent-pixel FP32 scale) with the last 5 Mann
    iterations on FP32 values, against the all-FP32 path, same scan and
    schedule.  A step = one scan, 60 Mann iterations."""
    w = mi.WORKLOADS["scan1024"]
    g = w.geom
    sigma = 5e-5
    log("fp16: matrix")
    cp, row, val = mi.system_matrix(g)
    sc = mi.scan(g, w.seed)
    prior = m.make_prior(w.prior_kind, w.sigma_x, w.p, w.q, w.T)
    dev = torch.device("cuda:0")
    y = torch.from_numpy(sc.y).to(dev)
    lam = torch.from_numpy(sc.lam).to(dev)
    x = torch.empty(g.n, dtype=torch.float32, device=dev)
    sp = torch.cuda.current_stream(dev).cuda_stream
    res = {}
    for prec, tail in ((0, 0), (1, 5), (1, 0)):
        log(f"fp16: loading precision {prec}, FP32 tail {tail}")
        sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w.n_agents,
                        precision=prec, fp32_tail_iters=tail)
        sysm.set_relaxation(0.5)
        for _ in range(args.warmup):
            sysm.solve_dev(y.data_ptr(), lam.data_ptr(), prior, w.rho, sigma, args.iters,
                           x.data_ptr(), stream_ptr=sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            info = sysm.solve_dev(y.data_ptr(), lam.data_ptr(), prior, w.rho, sigma, args.iters,
                                  x.data_ptr(), stream_ptr=sp)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[(prec, tail)] = (dt, x.cpu().numpy().copy(), info.residual, sysm.matrix_bytes)
        sysm.close()
    res[0], res[1], r16 = res[(0, 0)], res[(1, 5)], res[(1, 0)]
    x32, x16 = res[0][1], res[1][1]
    nrmse = float(np.linalg.norm(x16.astype(np.float64) - x32) / np.linalg.norm(x32))
    nrmse_pure = float(np.linalg.norm(r16[1].astype(np.float64) - x32) / np.linalg.norm(x32))
    upd = args.iters * w.n_agents * g.n
    out = _common("voxel-updates/s, 1024x1024 FP16 matrix values (+5 FP32 iterations)",
                  upd / res[1][0], "voxel-updates/s", args.steps, args.warmup, res[1][0] * 1e3,
                  "f16->f32",
                  {"workload": "scan1024: 1024x1024, 1440 views, 1472 channels, 32 agents, "
                               "q-GGMRF p=2 q=1.2 T=1 sigma_x=0.01, rho=0.8",
                   "mann_iters": args.iters, "sigma": sigma, "fp32_tail_iters": 5})
    out.update({"fp32_voxel_updates_per_s": upd / res[0][0],
                "fp16_only_voxel_updates_per_s": upd / r16[0],
                "matrix_bytes_fp16_only": r16[3], "nrmse_fp16_only_vs_fp32": nrmse_pure,
                "matrix_bytes_fp16": res[1][3], "matrix_bytes_fp32": res[0][3],
                "nrmse_fp16_vs_fp32": nrmse,
                "residual_fp16": res[1][2], "residual_fp32": res[0][2]})
    return out


def bench_pnp(args, m, mi, torch):
    """MACE-PnP (Algorithm 3) on the scan512 workload: the agents' data terms
    alone at sqrt(N) sigma and the consensus H(mean w), H = one pass of the
    3x3 binomial smoother.  Host arrays in and out (mace_solve_pnp): the time
    includes 4.2 MB of y / Lambda uploads per scan.  A step = one scan, 60
    Mann iterations."""
    w = mi.WORKLOADS["scan512"]
    g = w.geom
    sigma, passes = 5e-5, 1
    log("pnp: matrix")
    cp, row, val = mi.system_matrix(g)
    sc = mi.scan(g, w.seed)
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w.n_agents)
    sysm.set_relaxation(0.5)
    for _ in range(args.warmup):
        sysm.solve_pnp(sc.y, sc.lam, w.rho, sigma, args.iters, h_passes=passes)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, info = sysm.solve_pnp(sc.y, sc.lam, w.rho, sigma, args.iters, h_passes=passes)
    dt = (time.perf_counter() - t0) / args.steps
    upd = args.iters * w.n_agents * g.n
    out = _common("agent-voxel updates/s, MACE-PnP (binomial stand-in denoiser), 512x512",
                  upd / dt, "voxel-updates/s", args.steps, args.warmup, dt * 1e3, "f32",
                  {"workload": "scan512: 512x512 image, 720 views, 736 channels, 16 agents, "
                               "no prior in the agents, H = 1 pass of the 3x3 binomial smoother, "
                               "rho=0.8",
                   "mann_iters": args.iters, "sigma": sigma, "h_passes": passes})
    out.update({"final_residual": info.residual, "x_finite": bool(np.all(np.isfinite(x)))})
    return out


def study_grid(k_max):
    """Mann-iteration counts at which the convergence study samples NRMSE:
    every iteration up to 20, then every 2nd to 60, every 5th to 200 and every
    10th beyond."""
    ks = list(range(1, 21)) + list(range(22, 61, 2)) + list(range(65, 201, 5)) + \
        list(range(210, k_max + 1, 10))
    return [k for k in ks if k <= k_max]


def equits_to_reach(ks, nrmse, thr, equits_per_iter=1.0):
    """Equits (Sec. IV-B: voxel updates / (voxels x view subsets)) until
    NRMSE(x_k, x*) first falls below thr, interpolating log NRMSE linearly
    between the sampled iteration counts; None if it never does.  One Mann
    iteration with one ICD pass per agent updates every voxel once per view
    subset, so it costs one equit."""
    prev_k, prev_e = 0, None
    for k, e in zip(ks, nrmse):
        if not np.isfinite(e):
            return None
        if e < thr:
            if prev_e is None or prev_e <= e:
                return k * equits_per_iter
            f = (np.log(prev_e) - np.log(thr)) / (np.log(prev_e) - np.log(e))
            return (prev_k + f * (k - prev_k)) * equits_per_iter
        prev_k, prev_e = k, e
    return None


STUDY_DIR = os.path.join(ROOT, "tests", "golden")


def load_study_reference():
    """The converged image x* of the study problem and the centralised
    baseline's equits, as written by tests/golden/make_study_reference.py
    (FP64 oracle, centralised ICD to a pass change of 1e-12)."""
    import hashlib
    meta = json.load(open(os.path.join(STUDY_DIR, "study256_reference.json")))
    raw = open(os.path.join(STUDY_DIR, "study256_xstar.f32"), "rb").read()
    if hashlib.sha256(raw).hexdigest() != meta["xstar_sha256"]:
        raise RuntimeError("study256_xstar.f32 does not match its reference record")
    return np.frombuffer(raw, dtype="<f4").astype(np.float64), meta


SIGMA_GRID = (1e-4, 1.41e-4, 2e-4, 2.83e-4, 4e-4, 5.66e-4, 8e-4, 1.13e-3)


def bench_study(args, m, mi, torch):
    """Synthetic re-run of the paper's convergence studies (Sec. IV-B):
    equits for MACE to reach NRMSE thresholds against the fully converged
    image x* (Table II: against rho at N = 8; Fig. 4: against the number of
    view subsets N at rho = 0.8), the speedup N x equits(centralised) /
    equits(N) of Sec. IV-B, and the system-matrix bytes each agent holds
    (Table III).  Problem: 256x256, 360 views, 368 channels, q-GGMRF p = 2,
    q = 1.2, T = 1, sigma_x = 1e-3; x* and the centralised ICD's equits come
    from the oracle (tests/golden/make_study_reference.py).  One Mann
    iteration with one ICD pass per agent is one equit.  The NRMSE curve of
    a run is sampled by stopping it, reading x = mean w, and resuming from
    the checkpoint (w, X).  For every N the prox parameter sigma and rho are
    searched over SIGMA_GRID x {0.5, 0.8} and the fewest equits per threshold
    are reported with the (sigma, rho) that gave them; the agents run the
    concurrent super-voxel schedule.  At N = 8 the agents also run one
    sequential ICD pass (the paper's Algorithm 2 as written) for comparison."""
    x_star, meta = load_study_reference()
    p = meta["problem"]
    g = mi.Geometry(p["nx"], p["ny"], p["n_views"], p["n_channels"])
    pr = p["prior"]
    prior = m.make_prior(pr["kind"], pr["sigma_x"], pr["p"], pr["q"], pr["T"])
    thresholds = tuple(float(t) for t in meta["centralized_equits"])
    central = {t: meta["centralized_equits"][t] for t in meta["centralized_equits"]}
    k_max = args.iters if args.iters != 60 else 3000
    log("study: matrix")
    cp, row, val = mi.system_matrix(g)
    sc = mi.scan(g, p["seed"])
    ref = float(np.linalg.norm(x_star))
    t_start = time.perf_counter()

    def curve(sysm, rho, sigma, k_last=None):
        """NRMSE(x_k, x*) at k = 1, 2, ... (every iteration to 20, then
        every 2nd, 5th and 10th), through checkpoint / resume."""
        ks, es = [], []
        k_done, w, X = 0, None, None
        for k in study_grid(k_last or k_max):
            try:
                if w is None:
                    x, _ = sysm.solve(sc.y, sc.lam, prior, rho, sigma, k)
                else:
                    x, _ = sysm.solve_resume(sc.y, sc.lam, prior, rho, sigma, k - k_done, w, X)
                w, X = sysm.state()
                e = float(np.linalg.norm(x.astype(np.float64) - x_star)) / ref
            except m.MaceError as err:
                if err.code != m.MACE_E_NONFINITE:
                    raise
                e = float("inf")
            k_done = k
            ks.append(k)
            es.append(e if np.isfinite(e) else float("inf"))
            if not np.isfinite(e) or e > 10.0 or e < 0.3 * min(thresholds):
                break
        return {"sigma": sigma, "k": ks, "nrmse": es,
                "equits": {str(t): equits_to_reach(ks, es, t) for t in thresholds}}

    def speedup(eq, n_agents):
        return {t: None if eq[t] is None or central[t] is None
                else n_agents * central[t] / eq[t] for t in eq}

    def best_of(curves):
        """Fewest equits per threshold over the searched (sigma, rho)."""
        best = {}
        for t in (str(x) for x in thresholds):
            cands = [(c["equits"][t], c["sigma"], c["rho"]) for c in curves
                     if c["equits"][t] is not None]
            best[t] = None if not cands else dict(zip(("equits", "sigma", "rho"), min(cands)))
        return best

    # sigma is the user's choice (Sec. II-B); for small sigma the iteration
    # is gradient descent on f with step 2 rho sigma^2 / N in the consensus
    # direction, and partial updates lose stability in a band of larger
    # sigma (Theorem 2 covers small sigma only), so each N gets a search
    out_n, out_rho = {}, {}
    for n_agents in (2, 4, 8, 12, 24):
        t = time.perf_counter()
        sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, n_agents)
        sysm.set_relaxation(args.relax)
        cfg = sysm.config
        log(f"study: N={n_agents} loaded in {time.perf_counter() - t:.1f} s "
            f"(format {cfg['format']}, S {cfg['sv_size']}, rows {cfg['rows_per_agent']})")
        curves = []
        for sigma in SIGMA_GRID:
            for rho in (0.5, 0.8):
                c = curve(sysm, rho, sigma)
                c["rho"] = rho
                curves.append(c)
                log(f"study: N={n_agents} sigma={sigma:.1e} rho={rho}: {c['equits']}")
        best = best_of(curves)
        entry = {"matrix_bytes": sysm.matrix_bytes,
                 "matrix_bytes_per_agent": sysm.matrix_bytes / n_agents,
                 "csc_bytes_per_agent": int(cp[-1]) * 8 / n_agents,
                 "record_format": cfg["format"], "best": best,
                 "speedup": {t: None if b is None or central[t] is None
                             else n_agents * central[t] / b["equits"] for t, b in best.items()},
                 "curves": curves}
        if n_agents == 8:
            # Table II: against rho, at the largest sigma of the grid at which
            # both rho = 0.5 and rho = 0.8 reach the loosest threshold
            loose = str(thresholds[0])
            ok = [sg for sg in SIGMA_GRID
                  if all(c["equits"][loose] is not None for c in curves
                         if c["sigma"] == sg and c["rho"] in (0.5, 0.8))]
            s8 = max(ok) if ok else SIGMA_GRID[0]
            for rho in (0.5, 0.6, 0.7, 0.8, 0.9):
                c = next((c for c in curves if c["sigma"] == s8 and c["rho"] == rho), None)
                if c is None:
                    c = curve(sysm, rho, s8)
                    c["rho"] = rho
                c = dict(c, speedup=speedup(c["equits"], 8))
                out_rho[str(rho)] = c
                log(f"study: N=8 sigma={s8:.1e} rho={rho}: {c['equits']}")
        log(f"study: N={n_agents} best {best} speedup {entry['speedup']}")
        out_n[str(n_agents)] = entry
        sysm.close()
    # the agent update as the paper writes it: one ICD pass over the
    # super-voxels one after another (one 16-lane row per agent), exact
    # coordinate minimiser and under-relaxed, at N = 8, rho = 0.8
    seq = {}
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, 8, rows_per_agent=1)
    for relax in (1.0, 0.5):
        sysm.set_relaxation(relax)
        for sigma in (1e-4, 2e-4, 4e-4):
            c = curve(sysm, 0.8, sigma, k_last=min(k_max, 300))
            c["speedup"] = speedup(c["equits"], 8)
            seq[f"relax{relax}_sigma{sigma:.0e}"] = c
            log(f"study: N=8 sequential relax={relax} sigma={sigma:.0e}: {c['equits']}")
    sysm.close()
    return {"metric": "MACE convergence study: equits to NRMSE thresholds against x*, 256x256",
            "unit": "equits", "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "study256: 256x256 image, 360 views, 368 channels, "
                                   "q-GGMRF p=2 q=1.2 T=1 sigma_x=1e-3, interleaved view "
                                   "subsets", "thresholds": list(thresholds), "k_max": k_max,
                       "relaxation": args.relax},
            "x_star": {"centralized_icd_passes": meta["passes"],
                       "grad_ratio": meta["grad_ratio"]},
            "sigma_grid": list(SIGMA_GRID),
            "centralized_equits": central, "vs_N": out_n, "vs_rho_N8": out_rho,
            "sequential_N8_rho0.8": seq,
            "elapsed_s": time.perf_counter() - t_start}


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
    ap.add_argument("--format", type=int, default=0, choices=(0, 1, 2),
                    help="record format of the headline scan: 0 automatic (compact here), "
                         "1 compact, 2 general")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline scan (no slices / FP16 / serving legs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--mode", default="scan",
                    choices=("scan", "slices", "serve", "fp16", "pnp", "study", "volume", "oracle"),
                    help="scan: the headline one-scan benchmark (default); slices: 64 "
                         "512x512 slices sharing one matrix, batched vs one at a time; "
                         "serve: Poisson arrivals of mixed-size scans through the server; "
                         "fp16: 1024x1024 FP16 matrix values vs FP32; "
                         "pnp: MACE-PnP with the binomial stand-in denoiser; "
                         "study: equits to convergence vs rho and vs the number of agents; "
                         "volume: 16 coupled 256x256 slices vs the same slices as a batch; "
                         "oracle: the FP64 oracle's time per Mann iteration on this host")
    ap.add_argument("--scans", type=int, default=30, help="serve: number of arrivals")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: arrivals per second")
    ap.add_argument("--slices", type=int, default=64, help="slices: batch size")
    ap.add_argument("--serve-arrivals", type=int, default=300,
                    help="Poisson arrivals of the default run's served 256x256 leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the library runs every agent on one GPU; sharding agents over GPUs is "
              "designed but not implemented)", file=sys.stderr)
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
    if args.mode == "oracle":
        print(json.dumps(bench_oracle(mi)), flush=True)
        return
    from __graft_entry__ import _ensure_built
    _ensure_built()
    import paper_1911_09278_amd as m

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.mode != "scan":
        out = {"slices": bench_slices, "serve": bench_serve, "fp16": bench_fp16,
               "pnp": bench_pnp, "study": bench_study,
               "volume": lambda a, *r: leg_volume(*r, a.iters)}[args.mode](args, m, mi, torch)
        print(json.dumps(out), flush=True)
        return
    w8 = mi.WORKLOADS["scan512"]
    g = w8.geom
    log("generating system matrix and scan")
    cp, row, val = mi.system_matrix(g)
    scan = mi.scan(g, w8.seed)
    va = mi.interleaved_partition(g.n_views, w8.n_agents)
    nnz = int(cp[-1])
    log(f"nnz={nnz}; loading system")
    sysm = m.System(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, w8.n_agents,
                    rows_per_agent=args.rows_per_agent, sv_size=args.sv_size,
                    format=args.format)
    general = sysm.config["format"] == 2
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
                   "records": "general" if general else "compact",
                   "rows_per_agent": args.rows_per_agent or "auto"},
        "hbm_gbps_algorithmic": bytes_iter * args.steps * args.iters / dt / 1e9,
        "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
        "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
        "final_residual": info.residual,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     # the counter summary covers the compact-record sweep
                     "traffic": None if general else measured_traffic(),
                     "kernel": "sv_kernel_gen sweep" if general else "sv_kernel sweep",
                     "avg_launch_us": avg_launch_s * 1e6,
                     "bytes_per_launch": bytes_launch},
    }
    # the same bandwidth against what a plain 1 GiB device copy reaches
    copy_gbs = copy_bandwidth_gbs(torch)
    out["roofline"]["copy_gbs"] = copy_gbs
    out["roofline"]["frac_of_copy"] = achieved / copy_gbs
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(g, cp, row, val, scan, va, w8, args.sigma)
        out["cpu_baseline"].update(host_info())
    if not args.no_extra:
        del cp, row, val
        extra = {"time_to_tol": leg_time_to_tol(sysm, w8, m, mi, torch, y, lam, args.sigma)}
        extra["slices"] = leg_slices(sysm, w8, m, mi, torch, args.sigma, args.iters)
        sysm.close()
        extra["fp16_1024"] = leg_fp16(m, mi, torch, args.iters)
        extra["serve256"] = leg_serve(m, mi, torch, n_arrivals=args.serve_arrivals)
        extra["volume256"] = leg_volume(m, mi, torch, args.iters)
        out["extra"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
