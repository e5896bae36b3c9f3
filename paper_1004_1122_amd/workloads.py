"""Throughput of the two HBM-sized workloads beside the contrast sweep that
bench.py times: the 243^3 cell and the 512-problem batch.

* ``c3``: 243^3, 200 RSA spheres (seed 3, radii U[0.03, 0.08]), contrast 1e3,
  l0 = (1 + rho) / 2, E = e1, e2, e3, CG to 1e-6 in FP64 and in the mixed form
  (autotuned schedules; one untimed solve per case first).
* ``c4``: 512 two-phase problems (seeds 400000 + i: grid uniform over
  {81, 243, 729}, GRF threshold, contrast log-uniform in [1e1, 1e4]), E = (1, 0),
  CG to 1e-6, all in one lshom_solve_batched call per form (autotuned
  schedules; one untimed run first).

Prints one JSON line per measurement: GVoxel-CG-iters/s = sum |N| iterations /
wall time, iterations and the worst FP64 true residual.

  python -m paper_1004_1122_amd.workloads c3|c4 [--reps 1]
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import microstructure as ms


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def c3(reps):
    import torch
    from . import lshom
    t = time.perf_counter()
    m = ms.spheres_243(seed=3)
    log(f"generated 243^3 cell in {time.perf_counter() - t:.1f} s, vf {m.info['vf']:.4f}")
    s = lshom.Solver(torch.from_numpy(m.phase).cuda(), [1.0, 1e3])
    for prec in (lshom.PRECISION_FP64, lshom.PRECISION_MIXED):
        sched = s.autotune(precision=prec, reps=5)
        for E in ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)):
            s.solve(E, tol=1e-6, precision=prec, want_field=False)
            best = None
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, leff, info = s.solve(E, tol=1e-6, precision=prec, want_field=False)
                dt = time.perf_counter() - t
                best = dt if best is None else min(best, dt)
            print(json.dumps({"workload": "243^3 spheres seed 3 rho 1e3", "precision": prec, "E": E,
                              "iterations": info["iterations"], "refreshes": info["refreshes"],
                              "ms": best * 1e3, "GVoxel-CG-iters/s": m.phase.size * info["iterations"] / best / 1e9,
                              "rel_res_true": info["rel_res_true"], "leff": leff.tolist(),
                              "schedule": sched}), flush=True)


def c4(reps):
    import torch
    from . import lshom
    t = time.perf_counter()
    probs = []
    for i in range(512):
        m = ms.batched_problem(i)
        probs.append(dict(phase=m.phase, cond=m.cond, E=(1.0, 0.0), tol=1e-6))
    vox = [p["phase"].size for p in probs]
    log(f"generated 512 problems ({sum(vox) / 1e6:.1f} M voxels) in {time.perf_counter() - t:.1f} s")
    bs = lshom.BatchSolver()
    need = bs.prepare(probs, precision=lshom.PRECISION_MIXED)
    log(f"workspace {need / 1e9:.2f} GB")
    for prec in (lshom.PRECISION_FP64, lshom.PRECISION_MIXED):
        sched = bs.autotune(precision=prec, reps=3)
        bs.run(precision=prec)
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, _, infos = bs.run(precision=prec)
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        its = [i["iterations"] for i in infos]
        vi = sum(v * k for v, k in zip(vox, its))
        print(json.dumps({"workload": "512 problems seeds 400000+i", "precision": prec, "ms": best * 1e3,
                          "GVoxel-CG-iters/s": vi / best / 1e9,
                          "iterations": {"min": min(its), "median": float(np.median(its)), "max": max(its)},
                          "worst_rel_res_true": max(i["rel_res_true"] for i in infos),
                          "status": sorted(set(i["status"] for i in infos)), "schedules": sched}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c3", "c4"])
    ap.add_argument("--reps", type=int, default=1)
    args = ap.parse_args()
    (c3 if args.which == "c3" else c4)(args.reps)


if __name__ == "__main__":
    main()
