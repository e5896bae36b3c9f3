"""Training and evaluation of the learned initial guess (include/lshom_cnn.h).

Data: two-phase Gaussian-random-field images of the 512-problem generator
with the grid forced to 81^2 (even i) or 243^2 (odd i), seeds 500000 + i;
targets are FP64 CG solutions (tol 1e-8, E = e1) computed by the batched GPU
solver.  Held out: 243^2 (seeds 600000 + i) and 729^2 (seeds 610000 + i).

Evaluation: each held-out problem is solved to 1e-6 twice, from e = E and
from the projected prediction E + P(x_pred) (the library falls back to E
when the prediction does not lower the residual), recording iterations and
the wall time of network inference + solve.

  python -m paper_1004_1122_amd.warmstart --train 20000 --epochs 8 --out weights.npz --eval
  python -m paper_1004_1122_amd.warmstart --weights W.npz --time-inference 64
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import microstructure as ms


def _train_item(i):
    m = ms.warmstart_train_problem(i)
    return m.phase, m.info["log10_rho"], m.cond


def _eval_item(args):
    i, n = args
    m = ms.warmstart_eval_problem(i, n)
    return m.phase, m.info["log10_rho"], m.cond


def generate(fn, items, workers=None):
    workers = workers or min(16, os.cpu_count() or 1)
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(fn, items, chunksize=16))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def solve_targets(items, chunk=1024, tol=1e-8):
    """FP64 solutions for E = e1 of [(phase, log10_rho, cond)] (one grid size)."""
    import torch
    from . import lshom
    bs = lshom.BatchSolver()
    out = []
    for k in range(0, len(items), chunk):
        part = items[k:k + chunk]
        probs = [dict(phase=ph, cond=cond, E=(1.0, 0.0), tol=tol, want_field=True) for ph, _, cond in part]
        bs.prepare(probs, precision=0)
        fields, _, infos = bs.run(precision=0)
        bad = [i for i, inf in enumerate(infos) if inf["status"] != 0]
        if bad:
            raise RuntimeError(f"{len(bad)} training solves failed")
        out.append(torch.stack(fields))
        log(f"  solved {k + len(part)}/{len(items)} targets at {part[0][0].shape[0]}^2")
    bs.close()
    return torch.cat(out)


def train(net, sets, epochs=8, lr=1e-3, seed=0, log_every=500):
    """sets: list of (phase uint8 [M,N,N] cuda, log10_rho [M] cuda, targets [M,2,N,N] cuda, batch)."""
    import torch
    rng = np.random.default_rng(seed)
    steps_per_epoch = sum(math.ceil(len(s[0]) / s[3]) for s in sets)
    total = epochs * steps_per_epoch
    step = 0
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = []
        for si, (ph, lr_, tg, B) in enumerate(sets):
            perm = rng.permutation(len(ph))
            order += [(si, perm[k:k + B]) for k in range(0, len(ph) - B + 1, B)]
        rng.shuffle(order)
        run = 0.0
        for si, idx in order:
            ph, lr_, tg, B = sets[si]
            ix = torch.as_tensor(idx, device=ph.device)
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / total))  # cosine decay
            loss = net.train_step(ph[ix], lr_[ix], tg[ix], lr=cur)
            run += loss
            step += 1
            if step % log_every == 0:
                log(f"  step {step}/{total} epoch {ep} loss {run / log_every:.4f} lr {cur:.2e} "
                    f"({time.perf_counter() - t0:.0f} s)")
                hist.append((step, run / log_every))
                run = 0.0
    return hist


def evaluate(net, items, tol=1e-6, precision=0, reps=1, scale=1):
    """Cold vs warm single solves of [(phase, log10_rho, cond)]; the network
    runs at 1/scale of the grid (see lshom_cnn_forward)."""
    import torch
    from . import lshom
    rows = []
    for ph, lrho, cond in items:
        phd = torch.from_numpy(ph).cuda()
        s = lshom.Solver(phd, cond)
        s.solve((1.0, 0.0), tol=tol, precision=precision, want_field=False)  # warm-up (graphs)
        rec = {}
        for form in ("cold", "warm"):
            best = None
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                x0 = net.forward(phd[None], lrho, scale=scale)[0] if form == "warm" else None
                _, _, info = s.solve((1.0, 0.0), tol=tol, precision=precision, x0=x0, want_field=False)
                dt = time.perf_counter() - t
                best = dt if best is None else min(best, dt)
            rec[form] = {"iterations": info["iterations"], "ms": best * 1e3, "used": info["warm_start_used"],
                         "rel_res_true": info["rel_res_true"]}
        rec["log10_rho"] = lrho
        rows.append(rec)
        s.close()
    return rows


def evaluate_batched(net, items, tol=1e-6, precision=0, reps=3, scale=1):
    """Cold vs warm solves of [(phase, log10_rho, cond)] (one grid size) as one
    batch each: lshom_solve_batched from e = E, against one network
    inference over every image followed by lshom_solve_batched from the
    predictions (inference included in the warm time).  Best of reps."""
    import torch
    from . import lshom
    phd = torch.from_numpy(np.stack([ph for ph, _, _ in items])).cuda()
    lr = torch.tensor([lrho for _, lrho, _ in items], dtype=torch.float32, device="cuda")
    probs = [dict(phase=phd[i], cond=cond, E=(1.0, 0.0), tol=tol) for i, (_, _, cond) in enumerate(items)]
    n = phd.shape[1]
    pred = torch.empty((len(items), 2, n, n), dtype=torch.float64, device="cuda")
    cold = lshom.BatchSolver()
    cold.prepare(probs, precision=precision)
    warm = lshom.BatchSolver()
    warm.prepare([dict(p, x0=pred[i]) for i, p in enumerate(probs)], precision=precision)
    pred.copy_(net.forward(phd, lr, scale=scale))
    cold.run(precision=precision)  # graphs and schedules
    warm.run(precision=precision)
    best = {"cold": None, "warm": None, "inference": None}
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, ic = cold.run(precision=precision)
        dt = time.perf_counter() - t
        best["cold"] = dt if best["cold"] is None else min(best["cold"], dt)
        torch.cuda.synchronize()
        t = time.perf_counter()
        pred.copy_(net.forward(phd, lr, scale=scale))
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t
        _, _, iw = warm.run(precision=precision)
        dt = time.perf_counter() - t
        if best["warm"] is None or dt < best["warm"]:
            best["warm"], best["inference"] = dt, t_inf
    cold.close()
    warm.close()
    itc = np.array([i["iterations"] for i in ic], float)
    itw = np.array([i["iterations"] for i in iw], float)
    return {"n": len(items), "network_grid": n // scale, "iters_cold_mean": float(itc.mean()),
            "iters_warm_mean": float(itw.mean()), "iters_cold_max": int(itc.max()), "iters_warm_max": int(itw.max()),
            "saved_frac_mean": float(((itc - itw) / itc).mean()),
            "ms_cold": 1e3 * best["cold"], "ms_warm": 1e3 * best["warm"], "ms_inference": 1e3 * best["inference"],
            "time_ratio_warm_over_cold": best["warm"] / best["cold"],
            "warm_used": int(sum(i["warm_start_used"] for i in iw)),
            "worst_rel_res_true": max(i["rel_res_true"] for i in list(ic) + list(iw))}


def summarize(rows):
    cold = np.array([r["cold"]["iterations"] for r in rows], float)
    warm = np.array([r["warm"]["iterations"] for r in rows], float)
    saved = cold - warm
    tc = np.array([r["cold"]["ms"] for r in rows])
    tw = np.array([r["warm"]["ms"] for r in rows])
    return {"n": len(rows), "iters_cold_mean": float(cold.mean()), "iters_warm_mean": float(warm.mean()),
            "saved_mean": float(saved.mean()), "saved_median": float(np.median(saved)),
            "saved_min": float(saved.min()), "saved_frac_mean": float((saved / cold).mean()),
            "time_ratio_warm_over_cold": float(tw.sum() / tc.sum()),
            "ms_cold_total": float(tc.sum()), "ms_warm_total": float(tw.sum()),
            "warm_used": int(sum(r["warm"]["used"] for r in rows))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=None, help="skip training and load these weights")
    ap.add_argument("--eval", action="store_true")
    ap.add_argument("--eval243", type=int, default=64)
    ap.add_argument("--eval729", type=int, default=16)
    ap.add_argument("--json", default=None)
    ap.add_argument("--time-inference", type=int, default=0, metavar="B",
                    help="with --weights: time the network on B random 243^2 images (four runs) and exit")
    args = ap.parse_args()
    if args.time_inference and args.weights:
        import torch
        from . import cnn
        net = cnn.WarmStartNet.load(args.weights)
        B = args.time_inference
        ph = torch.randint(0, 2, (B, 243, 243), dtype=torch.uint8, device="cuda")
        lr = torch.full((B,), 2.0, device="cuda")
        for _ in range(4):
            torch.cuda.synchronize()
            t = time.perf_counter()
            net.forward(ph, lr)
            torch.cuda.synchronize()
            log(f"inference of {B} images of 243^2: {1e3 * (time.perf_counter() - t):.2f} ms")
        return
    # every image is generated in worker processes before the GPU is touched
    t = time.perf_counter()
    items = [] if args.weights else generate(_train_item, range(args.train))
    eval_items = {}
    if args.eval:
        for n, cnt in ((243, args.eval243), (729, args.eval729)):
            if cnt > 0:
                eval_items[n] = generate(_eval_item, [(i, n) for i in range(cnt)])
    log(f"generated {len(items)} training and {sum(len(v) for v in eval_items.values())} evaluation images "
        f"in {time.perf_counter() - t:.0f} s")
    import torch
    from . import cnn

    report = {}
    if args.weights:
        net = cnn.WarmStartNet.load(args.weights)
    else:
        sets = []
        for n, B in ((81, 16), (243, 8)):
            sub = [it for it in items if it[0].shape[0] == n]
            if not sub:
                continue
            t = time.perf_counter()
            tg = solve_targets(sub)
            log(f"solved {len(sub)} targets at {n}^2 in {time.perf_counter() - t:.0f} s")
            ph = torch.from_numpy(np.stack([it[0] for it in sub])).cuda()
            lr_ = torch.tensor([it[1] for it in sub], dtype=torch.float32, device="cuda")
            sets.append((ph, lr_, tg, B))
        del items
        net = cnn.WarmStartNet(args.base, seed=0)
        t = time.perf_counter()
        hist = train(net, sets, epochs=args.epochs, lr=args.lr)
        report["train"] = {"samples": args.train, "epochs": args.epochs, "seconds": time.perf_counter() - t,
                           "loss_history": hist}
        log(f"trained in {time.perf_counter() - t:.0f} s")
        if args.out:
            net.save(args.out)
            log(f"saved {args.out}")
        del sets
    if args.eval:
        for n, ev in eval_items.items():
            for scale in ((1,) if n <= 243 else (1, 3)):
                rows = evaluate(net, ev, scale=scale)
                key = f"eval{n}" + ("" if scale == 1 else f"_scale{scale}")
                report[key] = summarize(rows)
                log(f"eval {n}^2 (network at {n // scale}^2): {json.dumps(report[key])}")
    if args.json:
        with open(args.json, "w") as f:
            json.dump(report, f)
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
