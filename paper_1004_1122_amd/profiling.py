"""Summaries of rocprofv3 output for the pass kernels (text for the profile
records kept with the sources).

  python -m paper_1004_1122_amd.profiling stats --dir D --title T --command C --out F.md
      kernel statistics table from D/*kernel_stats.csv (and launch shapes
      from D/*kernel_trace.csv)

  python -m paper_1004_1122_amd.profiling traffic --fetch D1 --write D2 --kernel REGEX
      --pass NAME --form FORM --copy REGEX --copy-bytes N --command-fetch C1
      --command-write C2 --alg-bytes B --out F.md
      HBM bytes per launch of the kernels matching REGEX from two counter runs
      (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by what the
      same counter reads for a copy kernel of N bytes read and N written, and
      their ratio to the algorithmic bytes B of one such launch.  --window K
      keeps only dispatches between the (2K-1)-th and 2K-th dispatch of the
      marker kernel (--marker REGEX, default the |x| kernel of torch.abs).
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("passes.hip", "wave3d.hip", "wave_fft.hpp", "fft_engine.hpp", "reduce.hpp", "kernels.hpp",
                  "radix_consts.hpp")


def code_only(text):
    """C++ source without its comments and blank lines, each line stripped of
    surrounding white space (string and character literals kept as they are),
    so that an edit of the comments does not change the hash of the code."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            while i < n and text[i] != "\n":
                i += 1
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    lines = (line.strip() for line in "".join(out).split("\n"))
    return "\n".join(line for line in lines if line)


def kernel_source_hash():
    """Hash of the code of the kernel sources (comments and layout excluded):
    a traffic summary taken on other code does not describe these kernels."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()[:16]


def _rows(pattern):
    out = []
    for path in sorted(glob.glob(pattern, recursive=True)):
        with open(path, newline="") as f:
            out.extend(csv.DictReader(f))
    return out


def _col(row, *names):
    for n in names:
        for k in row:
            if k.lower() == n.lower():
                return row[k]
    raise KeyError(names)


def stats(args):
    rows = _rows(os.path.join(args.dir, "**", "*kernel_stats.csv"))
    trace = _rows(os.path.join(args.dir, "**", "*kernel_trace.csv"))
    shapes = {}
    for t in trace:
        name = _col(t, "Kernel_Name")
        try:
            dur = int(_col(t, "End_Timestamp")) - int(_col(t, "Start_Timestamp"))
        except KeyError:
            dur = None
        grid = tuple(int(_col(t, f"Grid_Size_{a}")) for a in "XYZ") if "Grid_Size_X" in t else None
        wg = tuple(int(_col(t, f"Workgroup_Size_{a}")) for a in "XYZ") if "Workgroup_Size_X" in t else None
        rec = shapes.setdefault(name, {"dur": [], "shapes": set()})
        if dur is not None:
            rec["dur"].append(dur)
        if grid and wg:
            rec["shapes"].add((tuple(g // w for g, w in zip(grid, wg)), wg[0]))
    lines = [f"# {args.title}", "", "Command (on the GPU host, repository root in $R):", "", "```", args.command, "```", ""]
    if args.note:
        lines += [args.note, ""]
    lines += ["| Kernel | Calls | Total ns | Average ns | Median ns | Min ns | Max ns | % | Blocks x threads |",
              "|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        name = _col(r, "Name", "Kernel_Name")
        med = ""
        sh = ""
        if name in shapes:
            if shapes[name]["dur"]:
                med = str(int(statistics.median(shapes[name]["dur"])))
            sh = "; ".join(f"{'x'.join(map(str, b))} x {w}" for b, w in sorted(shapes[name]["shapes"])[:3])
        lines.append(f"| `{name}` | {_col(r, 'Calls')} | {_col(r, 'TotalDurationNs')} | "
                     f"{float(_col(r, 'AverageNs')):.0f} | {med} | {_col(r, 'MinNs')} | {_col(r, 'MaxNs')} | "
                     f"{float(_col(r, 'Percentage')):.2f} | {sh} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_sums(pattern, counter):
    per = {}
    for r in _rows(pattern):
        if _col(r, "Counter_Name") != counter:
            continue
        key = (_col(r, "Kernel_Name"), int(_col(r, "Dispatch_Id")))
        per[key] = per.get(key, 0.0) + float(_col(r, "Counter_Value"))
    return per


def _window(per, marker_rx, k):
    """Entries between the (2k-1)-th and 2k-th dispatch of the marker kernel."""
    ids = sorted(d for (name, d) in per if marker_rx.search(name))
    if len(ids) < 2 * k:
        raise SystemExit(f"only {len(ids)} marker dispatches, window {k} needs {2 * k}")
    lo, hi = ids[2 * k - 2], ids[2 * k - 1]
    return {key: v for key, v in per.items() if lo < key[1] < hi}


def traffic(args):
    fetch = _counter_sums(os.path.join(args.fetch, "**", "*counter_collection.csv"), "FETCH_SIZE")
    write = _counter_sums(os.path.join(args.write, "**", "*counter_collection.csv"), "WRITE_SIZE")
    kre, cre = re.compile(args.kernel), re.compile(args.copy)

    def pick(per, rx):
        vals = [v for (name, _), v in per.items() if rx.search(name)]
        return vals

    cf, cw = pick(fetch, cre), pick(write, cre)
    if args.window:
        mre = re.compile(args.marker)
        fetch, write = _window(fetch, mre, args.window), _window(write, mre, args.window)
    kf, kw = pick(fetch, kre), pick(write, kre)
    if not (cf and cw and kf and kw):
        raise SystemExit(f"missing dispatches: copy {len(cf)}/{len(cw)}, kernel {len(kf)}/{len(kw)}")
    copy_kib = args.copy_bytes / 1024.0
    fetch_scale = copy_kib / max(cf)
    write_scale = copy_kib / max(cw)
    fetch_b = statistics.mean(kf) * fetch_scale * 1024.0
    write_b = statistics.mean(kw) * write_scale * 1024.0
    rec = {
        "pass": args.pass_name, "form": args.form, "kernel_regex": args.kernel,
        "launches": len(kf), "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
        "bytes_per_launch": fetch_b + write_b, "algorithmic_bytes_per_launch": args.alg_bytes,
        "traffic_ratio": (fetch_b + write_b) / args.alg_bytes,
        "fetch_scale": fetch_scale, "write_scale": write_scale,
        "copy_bytes": args.copy_bytes, "source_hash": kernel_source_hash(), "summary": os.path.basename(args.out),
    }
    lines = [
        f"# HBM traffic of `{args.kernel}` ({args.pass_name}, {args.form})", "",
        "Counter runs (on the GPU host, repository root in $R):", "", "```", args.command_fetch, args.command_write, "```", "",
        f"Calibration: the copy kernel matching `{args.copy}` reads and writes {args.copy_bytes} bytes; "
        f"FETCH_SIZE read {max(cf):.0f} KiB (scale {fetch_scale:.4f}), WRITE_SIZE {max(cw):.0f} KiB "
        f"(scale {write_scale:.4f}).", "",
        f"Kernel: {len(kf)} dispatches; mean FETCH_SIZE {statistics.mean(kf):.1f} KiB, "
        f"WRITE_SIZE {statistics.mean(kw):.1f} KiB per dispatch; scaled: {fetch_b / 1e6:.3f} MB read + "
        f"{write_b / 1e6:.3f} MB written = {(fetch_b + write_b) / 1e6:.3f} MB per launch, against "
        f"{args.alg_bytes / 1e6:.3f} MB algorithmic (ratio {(fetch_b + write_b) / args.alg_bytes:.3f}).", "",
        "traffic-json: " + json.dumps(rec), "",
    ]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def issue(args):
    """SQ counters of the pass kernels per dispatch, inside each form's marker
    window (window 1: FP64, 2: mixed), with the time their VALU instructions
    take to issue against the pass time that pass_profile measured.  A wave64
    VALU instruction occupies its SIMD for 4 cycles (FP32 as FP64, the packed
    forms unused), so SQ_INSTS_VALU x 4 / (SIMDs x clock) is the time the
    VALU needs if every SIMD issues back to back."""
    counters = [c for c in args.counters.split(",") if c]
    pattern = os.path.join(args.dir, "**", "*counter_collection.csv")
    per = {c: _counter_sums(pattern, c) for c in counters}
    with open(args.passes) as f:
        pj = json.load(f)
    kernels = [kv.split("=", 1) for kv in args.kernel]
    mre = re.compile(args.marker)
    lines = [f"# {args.title}", "", "Commands (on the GPU host, repository root in $R):", "", "```"] + args.command + ["```", ""]
    if args.note:
        lines += [args.note, ""]
    lines += ["| Form | Pass | µs per launch | Waves | VALU instr. per wave | LDS instr. per wave | "
              "VALU issue µs | VALU issue / pass time | LDS bank-conflict / LDS-active cycles |",
              "|---|---|---|---|---|---|---|---|---|"]
    recs = []
    for win, (form, tname) in enumerate((("fp64", "double"), ("mixed", "float")), start=1):
        wc = {c: _window(per[c], mre, win) for c in counters}
        for pname, rx in kernels:
            kre = re.compile(rx.format(t=tname))
            vals = {c: [v for (name, _), v in wc[c].items() if kre.search(name)] for c in counters}
            if not all(vals.values()):
                continue
            m = {c: statistics.mean(v) for c, v in vals.items()}
            us = pj["forms"][form]["passes"][pname]["ms"] * 1e3
            waves = m.get("SQ_WAVES", 0.0)
            valu_us = m.get("SQ_INSTS_VALU", 0.0) * 4.0 / (args.simds * args.clock_ghz * 1e3)
            lds_act = m.get("SQ_ACTIVE_INST_LDS", 0.0)
            conf = m.get("SQ_LDS_BANK_CONFLICT", 0.0) / lds_act if lds_act else float("nan")
            rec = {"form": form, "pass": pname, "us": us, "dispatches": len(vals[counters[0]])}
            rec.update(m)
            recs.append(rec)
            lines.append(f"| {form} | {pname} | {us:.1f} | {waves:.0f} | "
                         f"{m.get('SQ_INSTS_VALU', 0.0) / max(waves, 1.0):.0f} | "
                         f"{m.get('SQ_INSTS_LDS', 0.0) / max(waves, 1.0):.0f} | {valu_us:.1f} | "
                         f"{valu_us / us:.2f} | {conf:.3f} |")
    lines += ["", f"Model: {args.simds} SIMDs at {args.clock_ghz} GHz, 4 cycles per wave64 VALU instruction.", "",
              "issue-json: " + json.dumps({"source_hash": kernel_source_hash(), "passes": recs}), ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--note", default="")
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--pass", dest="pass_name", required=True)
    t.add_argument("--form", required=True)
    t.add_argument("--copy", default=r"neg")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--alg-bytes", type=float, required=True)
    t.add_argument("--window", type=int, default=0)
    t.add_argument("--marker", default=r"AbsFunctor")
    t.add_argument("--out", required=True)
    i = sub.add_parser("issue")
    i.add_argument("--dir", required=True)
    i.add_argument("--passes", required=True, help="pass_profile JSON of the same workload")
    i.add_argument("--kernel", action="append", required=True,
                   help="pass=regex ({t} stands for the element type), repeated")
    i.add_argument("--counters", default="SQ_WAVES,SQ_INSTS_VALU,SQ_INSTS_LDS,SQ_ACTIVE_INST_LDS,"
                                         "SQ_LDS_BANK_CONFLICT,SQ_BUSY_CYCLES,SQ_WAVE_CYCLES,SQ_ACTIVE_INST_VALU")
    i.add_argument("--simds", type=int, default=1024)
    i.add_argument("--clock-ghz", type=float, default=2.4)
    i.add_argument("--marker", default=r"AbsFunctor")
    i.add_argument("--title", required=True)
    i.add_argument("--command", action="append", required=True)
    i.add_argument("--note", default="")
    i.add_argument("--out", required=True)
    a = ap.parse_args()
    {"stats": stats, "traffic": traffic, "issue": issue}[a.cmd](a)


if __name__ == "__main__":
    main()
