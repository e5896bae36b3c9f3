"""Benchmark of the FFT-accelerated CG homogenisation solve on one MI355X.

Timed workload (one step): the 243^3 sphere cell, the HBM-sized 3-D case.
200 random non-overlapping spheres (RSA, radii U[0.03, 0.08], seed 3) of
contrast rho = 1e3 in a matrix of conductivity 1, l0 = (1 + rho) / 2; one step
solves the three load cases E = e1, e2, e3 to relative residual 1e-6 by plain
FP64 CG and writes each field e (3 x 243^3 FP64) and <lambda e>.  Inputs
(phase image, workspace, autotuned schedules) are resident in HBM before the
timed region.

Metric: GVoxel-CG-iters/s = sum over solves of |N| * (CG iterations) / wall
time / 1e9 (`value`: plain FP64 on the 243^3 cell), plus the time to a 1e-6
residual of every solve.  Reported beside it, each measured in its own loop
after the timed steps:
  * the same cell by FP32-apply / FP64-refinement CG (mixed form);
  * the 512 uneven-size 2-D problems (seeds 400000 + i, grids uniform over
    {81, 243, 729}, GRF phases, contrast log-uniform in [1e1, 1e4]) in one
    batched call per form;
  * the 729^2 contrast sweep (40 RSA circles, seed 2, rho 1e1..1e4, E = e1, e2;
    cache-resident: its working set fits the 256 MB Infinity Cache);
  * the learned warm start on held-out GRF problems (64 at 243^2, 16 at 729^2),
    time including network inference, against the cold start.

Printed: one JSON line with the metric, the roofline of the dominant pass
kernel of the timed workload (algorithmic bytes / HIP-event durations of its
launches inside real solves, against 8 TB/s HBM) and the CPU oracle timed on a
bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import glob
import json
import os
import platform
import re
import statistics
import sys
import tempfile
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GVoxel-CG-iters/s + time-to-1e-6 residual: plain FP64 CG vs warm-start/mixed"
HBM_PEAK_GBS = 8000.0
TOL = 1e-6
C3_RHO = 1e3
C3_LOADS = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))
C2_CONTRASTS = (1e1, 1e2, 1e3, 1e4)
C2_LOADS = ((1.0, 0.0), (0.0, 1.0))
FORMS = (("fp64", 0), ("mixed", 1))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def measured_traffic(pass_name, form, grid_tag):
    """HBM bytes per algorithmic byte of one pass kernel from the committed
    counter summary of this grid, if it was taken on the current kernel
    sources (else None)."""
    from paper_1004_1122_amd.profiling import kernel_source_hash
    src = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"traffic_*_{grid_tag}.md"))):
        with open(path) as f:
            for line in f:
                m = re.match(r"^traffic-json:\s*(\{.*\})\s*$", line)
                if not m:
                    continue
                rec = json.loads(m.group(1))
                if rec.get("pass") == pass_name and rec.get("form") == form and rec.get("source_hash") == src:
                    return rec
    return None


def _c4_item(i):
    from paper_1004_1122_amd import microstructure as ms
    m = ms.batched_problem(i)
    return m.phase, m.cond


def _c5_item(args):
    from paper_1004_1122_amd import microstructure as ms
    i, n = args
    m = ms.warmstart_eval_problem(i, n)
    return m.phase, m.info["log10_rho"], m.cond, m.info["rho"]


def cpu_baseline(phase, n_iter):
    """The oracle (NumPy/SciPy FP64, untuned) on a bounded sample of the timed
    workload: CG on the 243^3 cell for load case e1, stopped after n_iter
    iterations (its initial residual and the n_iter operator applies timed)."""
    workers = min(16, os.cpu_count() or 1)
    os.environ.setdefault("LSHOM_ORACLE_WORKERS", str(workers))
    from oracle import lshom_oracle as o
    from paper_1004_1122_amd import microstructure as ms
    lam = ms.lam_field(phase, [1.0, C3_RHO])
    l0 = 0.5 * (1.0 + C3_RHO)
    t0 = time.perf_counter()
    res = o.cg(lam, l0, [1.0, 0.0, 0.0], n_iter=n_iter)
    dt = time.perf_counter() - t0
    return {"value": phase.size * res["iterations"] / dt / 1e9, "unit": "GVoxel-CG-iters/s",
            "cores": o._WORKERS, "kind": "oracle",
            "sample": f"243^3 spheres seed 3, rho 1e3, E=e1, FP64 CG stopped after {res['iterations']} iterations "
                      f"(initial residual + {res['iterations']} applies) in {dt:.1f} s",
            "host": {"os.cpu_count": os.cpu_count(), "cpu_model": cpu_model(), "scipy_fft_workers": o._WORKERS}}


def cpu_baseline_c2(phase, runs=3):
    """The oracle on the whole 729^2 contrast sweep (8 solves to 1e-6, about
    half a minute on 16 host cores): the median of `runs` sweeps."""
    from oracle import lshom_oracle as o
    from paper_1004_1122_amd import microstructure as ms
    times, its = [], 0
    for _ in range(runs):
        t0 = time.perf_counter()
        its = 0
        for rho in C2_CONTRASTS:
            lam = ms.lam_field(phase, [1.0, rho])
            for E in C2_LOADS:
                its += o.cg(lam, 0.5 * (1.0 + rho), list(E), tol=TOL)["iterations"]
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    return {"value": phase.size * its / med / 1e9, "unit": "GVoxel-CG-iters/s", "cores": o._WORKERS,
            "kind": "oracle", "sample": f"729^2 circles seed 2, rho 1e1..1e4 x E=e1,e2: 8 FP64 CG solves to 1e-6, "
                                        f"{its} iterations, median of {runs} sweeps {med:.1f} s"}


def c3_leg(lshom, torch, phase_dev, n_vox, steps, warmup, sched_prefix=None):
    """The timed steps (FP64) and the same loop for the mixed form."""
    s = lshom.Solver(phase_dev, [1.0, C3_RHO])
    sched = {}
    for form, prec in FORMS:
        t = time.perf_counter()
        sched[form] = s.autotune(precision=prec, reps=3)
        log(f"C3 autotune {form}: {time.perf_counter() - t:.1f} s")
    if sched_prefix:
        s.save_schedules(sched_prefix + ".243cube")
    e = torch.empty((3,) + tuple(phase_dev.shape), dtype=torch.float64, device=phase_dev.device)
    out = {}
    for form, prec in FORMS:
        def one_step(record):
            for E in C3_LOADS:
                t = time.perf_counter()
                _, leff, info = s.solve(E, tol=TOL, precision=prec, out=e)
                dt = time.perf_counter() - t
                if record is not None:
                    record.append((E, dt, info, leff))
        for _ in range(warmup):
            one_step(None)
        torch.cuda.synchronize()
        rec = []
        t0 = time.perf_counter()
        for k in range(steps):
            one_step(rec)
            if form == "fp64":
                log(f"step {k + 1}/{steps} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        iters = sum(r[2]["iterations"] for r in rec)
        per_load = {}
        for E, dt, info, leff in rec:
            key = "E=e%d" % (1 + int(np.argmax(E)))
            p = per_load.setdefault(key, {"ms": [], "iterations": info["iterations"],
                                          "refreshes": info["refreshes"], "rel_res_true": info["rel_res_true"],
                                          "leff": [float(v) for v in leff]})
            p["ms"].append(1e3 * dt)
        for p in per_load.values():
            p["ms"] = statistics.median(p["ms"])
        out[form] = {"GVoxel-CG-iters/s": n_vox * iters / elapsed / 1e9, "elapsed_s": elapsed,
                     "ms_per_step": 1e3 * elapsed / steps, "iterations_per_step": iters // steps,
                     "time_to_1e-6": per_load, "schedule": sched[form]}
        log(f"C3 {form}: {out[form]['GVoxel-CG-iters/s']:.2f} GVoxel-CG-iters/s")
    # one more FP64 step with HIP events around every pass launch of the CG loops
    s.set_pass_timing(True)
    for E in C3_LOADS:
        s.solve(E, tol=TOL, precision=0, out=e)
    timing = s.pass_timing()
    s.set_pass_timing(False)
    s.set_pass_timing(True)
    for E in C3_LOADS:
        s.solve(E, tol=TOL, precision=1, out=e)
    timing_mixed = s.pass_timing()
    s.set_pass_timing(False)
    s.close()
    return out, timing, timing_mixed


def roofline_of(timing, form, grid_tag):
    name, (ms_tot, by_tot, n) = max(timing.items(), key=lambda kv: kv[1][0])
    achieved = by_tot / (ms_tot * 1e-3) / 1e9
    rec = measured_traffic(name, form, grid_tag)
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": rec["traffic_ratio"] * by_tot / n if rec else None,
           "kernel": f"{name} ({form})", "avg_launch_ms": ms_tot / n, "algorithmic_bytes_per_launch": by_tot / n,
           "launches": n}
    if rec:
        out["traffic_source"] = rec.get("summary")
    return out


def pass_table(timing):
    return {name: {"ms_total": v[0], "launches": v[2], "avg_ms": v[0] / v[2], "GB/s": v[1] / (v[0] * 1e-3) / 1e9,
                   "frac_of_8TBs": v[1] / (v[0] * 1e-3) / 1e9 / HBM_PEAK_GBS}
            for name, v in timing.items()}


def c4_leg(lshom, torch, items, reps=2):
    """All 512 problems in one lshom_solve_batched call per form."""
    probs = [dict(phase=ph, cond=cond, E=(1.0, 0.0), tol=TOL) for ph, cond in items]
    vox = [p["phase"].size for p in probs]
    bs = lshom.BatchSolver()
    need = bs.prepare(probs, precision=1)
    out = {"problems": len(probs), "voxels_total": int(sum(vox)), "workspace_GB": need / 1e9}
    for form, prec in FORMS:
        t = time.perf_counter()
        bs.autotune(precision=prec, reps=2)
        log(f"C4 autotune {form}: {time.perf_counter() - t:.1f} s")
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
        out[form] = {"GVoxel-CG-iters/s": vi / best / 1e9, "ms": 1e3 * best,
                     "iterations": {"min": min(its), "median": float(np.median(its)), "max": max(its)},
                     "worst_rel_res_true": max(i["rel_res_true"] for i in infos),
                     "status": sorted(set(i["status"] for i in infos))}
        log(f"C4 {form}: {out[form]['GVoxel-CG-iters/s']:.2f} GVoxel-CG-iters/s")
    bs.close()
    return out


def c2_leg(lshom, torch, phase_np, reps=3):
    """The 729^2 contrast sweep, each form's 8 solves in one batch."""
    phase_dev = torch.from_numpy(phase_np).cuda()
    probs = [dict(phase=phase_dev, cond=[1.0, rho], E=E, tol=TOL) for rho in C2_CONTRASTS for E in C2_LOADS]
    n_vox = phase_np.size
    out = {"note": "working set about 45 MB: resident in the 256 MB Infinity Cache"}
    for form, prec in FORMS:
        bs = lshom.BatchSolver()
        bs.prepare(probs, precision=prec)
        bs.autotune(precision=prec, reps=5)
        bs.run(precision=prec)
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, _, infos = bs.run(precision=prec)
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        its = [i["iterations"] for i in infos]
        out[form] = {"GVoxel-CG-iters/s": n_vox * sum(its) / best / 1e9, "ms_per_sweep": 1e3 * best,
                     "iterations_per_solve": its}
        bs.close()
        log(f"C2 {form}: {out[form]['GVoxel-CG-iters/s']:.2f} GVoxel-CG-iters/s")
    return out


def warm_start_leg(items243, items729):
    """Time to 1e-6 from e = E and from the learned initial guess (network
    inference included) on held-out problems, plain FP64."""
    from paper_1004_1122_amd import cnn, warmstart
    if not os.path.exists(cnn.DEFAULT_WEIGHTS):
        return None
    net = cnn.WarmStartNet.load(cnn.DEFAULT_WEIGHTS)
    out = {"weights": os.path.relpath(cnn.DEFAULT_WEIGHTS, ROOT)}
    for n, items, scale in ((243, items243, 1), (729, items729, 3)):
        ev = [(ph, lr, cond) for ph, lr, cond, _ in items]
        rows = warmstart.evaluate(net, ev, scale=scale, reps=3)
        out[f"{n}x{n}"] = dict(warmstart.summarize(rows), network_grid=n // scale)
        log(f"warm start {n}^2 (single solves): {out[f'{n}x{n}']}")
        out[f"{n}x{n}_batched"] = warmstart.evaluate_batched(net, ev, scale=scale)
        log(f"warm start {n}^2 (one batch): {out[f'{n}x{n}_batched']}")
    net.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="c4,c2,c5",
                    help="comma list of the legs reported beside the timed workload (c4, c2, c5, or none)")
    ap.add_argument("--cpu-iters", type=int, default=10, help="oracle CG iterations of the CPU sample")
    ap.add_argument("--save-schedules", default=None,
                    help="write the autotuned schedules of the timed workload to this file prefix")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy a device buffer of this size (the counter calibration kernel)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the solver runs each "
              "problem on one GPU and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x and x != "none"]

    from paper_1004_1122_amd import microstructure as ms
    t = time.perf_counter()
    c3 = ms.spheres_243(seed=3, rho=C3_RHO)
    items4 = items5a = items5b = None
    c2 = None
    # inputs of the other legs are generated on the host before the GPU is
    # touched (worker processes fork here)
    workers = min(16, os.cpu_count() or 1)
    with ProcessPoolExecutor(workers) as ex:
        if "c4" in legs:
            items4 = list(ex.map(_c4_item, range(512), chunksize=8))
        if "c5" in legs:
            items5a = list(ex.map(_c5_item, [(i, 243) for i in range(64)], chunksize=4))
            items5b = list(ex.map(_c5_item, [(i, 729) for i in range(16)], chunksize=1))
    if "c2" in legs:
        c2 = ms.circles_729(seed=2)
    log(f"inputs generated in {time.perf_counter() - t:.1f} s (243^3 vf {c3.info['vf']:.4f})")

    import torch
    from paper_1004_1122_amd import lshom
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    phase_dev = torch.from_numpy(c3.phase).cuda()
    n_vox = c3.phase.size

    forms, timing, timing_mixed = c3_leg(lshom, torch, phase_dev, n_vox, args.steps, args.warmup,
                                         args.save_schedules)
    fp = forms["fp64"]
    roof = roofline_of(timing, "fp64", "243cube")
    roof["by_form"] = {"mixed": {k: v for k, v in roofline_of(timing_mixed, "mixed", "243cube").items()
                                 if k in ("kernel", "achieved", "frac", "avg_launch_ms", "traffic")}}
    t_fp = fp["time_to_1e-6"]
    t_mx = forms["mixed"]["time_to_1e-6"]
    out = {
        "metric": METRIC,
        "value": fp["GVoxel-CG-iters/s"],
        "unit": "GVoxel-CG-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "3-D 243^3 cell, 200 RSA spheres r~U[0.03,0.08] seed 3, rho 1e3, l0 (1+rho)/2, "
                        "E=e1,e2,e3, plain FP64 CG to relative residual 1e-6, field and <lambda e> written",
            "solves_per_step": 3,
            "voxels": n_vox,
            "vf": c3.info["vf"],
            "schedule": fp["schedule"],
        },
        "forms": {
            "fp64": {k: v for k, v in fp.items() if k != "schedule"},
            "mixed": {k: v for k, v in forms["mixed"].items() if k != "schedule"},
        },
        "time_to_1e-6": {k: {"fp64_ms": t_fp[k]["ms"], "mixed_ms": t_mx[k]["ms"],
                             "mixed_speedup": t_fp[k]["ms"] / t_mx[k]["ms"]} for k in t_fp},
        "roofline": roof,
        "pass_timing": {"fp64": pass_table(timing), "mixed": pass_table(timing_mixed)},
    }
    if "c4" in legs:
        log("C4: 512 problems")
        out["batched_512"] = c4_leg(lshom, torch, items4)
    if "c2" in legs:
        log("C2: 729^2 contrast sweep")
        out["sweep_729"] = c2_leg(lshom, torch, c2.phase)
    if "c5" in legs:
        log("C5: learned warm start")
        ws = warm_start_leg(items5a, items5b)
        if ws is not None:
            out["warm_start"] = ws
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(c3.phase, args.cpu_iters)
        if "c2" in legs:
            log("timing the CPU oracle on the 729^2 sweep")
            out["cpu_baseline"]["sweep_729"] = cpu_baseline_c2(c2.phase)
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
