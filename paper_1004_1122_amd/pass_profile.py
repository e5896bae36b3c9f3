"""Launches of the pass kernels with known work, for hardware-counter runs.

Builds the 729x729 circle cell (40 RSA circles, seed 2, contrast 1e4; or
with --workload spheres243 the 243^3 sphere cell, seed 3, contrast 1e3; or
with --workload random729cube a 729^3 cell with 30% of the nodes in the
second phase, seed 5, contrast 1e2),
applies the autotuned schedule of each precision (or, with --schedules, the
schedules another run saved, e.g. bench.py --save-schedules), and launches
every pass kernel of one CG iteration `--reps` times back to back (all blocks
active, as in the middle of a solve).  Prints one JSON line with each pass's
average launch time and algorithmic bytes.

The timed launches of form k (1: FP64, 2: mixed) are bracketed by the k-th
pair of dispatches of a small elementwise |x| kernel, so that counter records
can be cut to exactly those launches (profiling.py traffic --window k).  With
--copy-mib, finishes with an elementwise kernel that reads and writes that
many MiB once (the counter calibration).

  python -m paper_1004_1122_amd.pass_profile [--reps 20] [--copy-mib 256] [--schedules F ...]
      [--workload circles729|spheres243|random729cube] [--save-schedules F]
"""

from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--rho", type=float, default=None,
                    help="contrast (default 1e4 at 729^2, 1e3 at 243^3, 1e2 at 729^3)")
    ap.add_argument("--workload", choices=["circles729", "spheres243", "random729cube"], default="circles729")
    ap.add_argument("--schedules", nargs="*", default=None,
                    help="schedule files (lshom_save_schedules format) to load instead of autotuning")
    ap.add_argument("--save-schedules", default=None, help="write the schedules used to this file")
    args = ap.parse_args()
    import torch
    from . import lshom
    from . import microstructure as ms

    if args.workload == "circles729":
        rho = 1e4 if args.rho is None else args.rho
        m = ms.circles_729(seed=2)
        E = (1.0, 0.0)
        name = "729x729 circles seed 2, rho %g" % rho
    elif args.workload == "spheres243":
        rho = 1e3 if args.rho is None else args.rho
        m = ms.spheres_243(seed=3)
        E = (1.0, 0.0, 0.0)
        name = "243^3 spheres seed 3, rho %g" % rho
    else:
        import numpy as np
        rho = 1e2 if args.rho is None else args.rho
        m = ms.Microstructure(phase=(np.random.default_rng(5).random((729, 729, 729)) < 0.3).astype(np.uint8),
                              cond=np.array([1.0, rho]), info={})
        E = (1.0, 0.0, 0.0)
        name = "729^3 random 30%% seed 5, rho %g" % rho
    s = lshom.Solver(torch.from_numpy(m.phase).cuda(), [1.0, rho])
    out = {"workload": name, "reps": args.reps, "forms": {}}
    marker = torch.ones(64, device="cuda")
    if args.schedules:
        for path in args.schedules:
            s.load_schedules(path)
    for form, prec in (("fp64", lshom.PRECISION_FP64), ("mixed", lshom.PRECISION_MIXED)):
        s.solve(E, tol=1e-6, precision=prec, want_field=False)
        sched = s.get_schedule(prec) if args.schedules else s.autotune(precision=prec, reps=10)
        torch.cuda.synchronize()
        torch.abs(marker)
        passes = s.time_passes(prec, reps=args.reps)
        torch.abs(marker)
        torch.cuda.synchronize()
        out["forms"][form] = {"schedule": sched,
                              "passes": {k: {"ms": v[0], "algorithmic_bytes": v[1]} for k, v in passes.items()}}
    if args.save_schedules:
        s.save_schedules(args.save_schedules)
    if args.copy_mib > 0:
        nbytes = args.copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        out["copy_bytes"] = nbytes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
