"""Writes the converged reference image of the convergence study and the
centralised baseline's equits (Sec. IV-B), calling only the FP64 oracle and
the seeded input generator.

Problem: 256x256 pixels, 360 views, 368 channels, ellipse phantom seed 1916
(the serve256 workload's geometry), q-GGMRF prior p = 2, q = 1.2, T = 1,
sigma_x = 1e-3.  x* is the minimiser of f (eq. (global_obj)), reached by the
oracle's centralised ICD (the paper's single-node baseline: one node, all
views, no prox term; surrogate coordinate rule, whose fixed points are the
exact rule's) run until a pass changes no pixel by more than 1e-12 of
max|x|.  The centralised baseline's convergence is its NRMSE(x_k, x*) after
k passes; one pass is one equit (Sec. IV-B).

Outputs (next to this script):
  study256_xstar.f32          x* as little-endian float32, raster order
  study256_reference.json     problem, passes, final change, |grad f(x*)|
                              relative to |grad f(0)|, the centralised NRMSE
                              curve and its equits to each threshold.
Run: python tests/golden/make_study_reference.py  (about 2 minutes)
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mace_inputs as mi  # noqa: E402
import oracle  # noqa: E402

PROBLEM = {"nx": 256, "ny": 256, "n_views": 360, "n_channels": 368, "seed": 1916,
           "prior": {"kind": 1, "sigma_x": 1e-3, "p": 2.0, "q": 1.2, "T": 1.0}}
THRESHOLDS = (1e-2, 3e-3, 1e-3)


def equits_to_reach(es, thr):
    """First pass count k with NRMSE(x_k) < thr (curve sampled every pass),
    log-linear between the two passes around the crossing."""
    prev = None
    for k, e in enumerate(es, start=1):
        if e < thr:
            if prev is None or prev <= e:
                return float(k)
            f = (np.log(prev) - np.log(thr)) / (np.log(prev) - np.log(e))
            return k - 1 + f
        prev = e
    return None


def main():
    p = PROBLEM
    g = mi.Geometry(p["nx"], p["ny"], p["n_views"], p["n_channels"])
    cp, row, val = mi.system_matrix(g)
    s = mi.scan(g, p["seed"])
    va = mi.interleaved_partition(g.n_views, 1)
    pr = p["prior"]
    O = oracle.Oracle(g.nx, g.ny, g.n_views, g.n_channels, cp, row, val, s.y, s.lam, va,
                      pr["kind"], pr["sigma_x"], pr["p"], pr["q"], pr["T"])
    print("centralised ICD to convergence", flush=True)
    xs, passes = O.centralized_icd(rtol=1e-12, max_passes=20000, mode=oracle.MODE_SURROGATE)
    g0 = float(np.abs(O.gradient(np.zeros(g.n))).max())
    gr = float(np.abs(O.gradient(xs)).max()) / g0
    print(f"  {passes} passes, |grad f(x*)| / |grad f(0)| = {gr:.2e}", flush=True)
    # the centralised baseline's NRMSE curve, one pass at a time
    x = np.zeros(g.n)
    ref = float(np.linalg.norm(xs))
    curve = []
    while len(curve) < passes:
        x, _ = O.centralized_icd(x0=x, rtol=0.0, max_passes=1, mode=oracle.MODE_SURROGATE)
        curve.append(float(np.linalg.norm(x - xs) / ref))
        if curve[-1] < 0.1 * THRESHOLDS[-1]:
            break
    out = dict(problem=p, passes=passes, grad_ratio=gr,
               centralized_nrmse=curve,
               centralized_equits={str(t): equits_to_reach(curve, t) for t in THRESHOLDS})
    x32 = xs.astype("<f4")
    x32.tofile(os.path.join(HERE, "study256_xstar.f32"))
    out["xstar_sha256"] = hashlib.sha256(x32.tobytes()).hexdigest()
    with open(os.path.join(HERE, "study256_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("  centralised equits:", out["centralized_equits"], flush=True)


if __name__ == "__main__":
    main()
