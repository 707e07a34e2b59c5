"""Summaries of rocprofv3 output for the bench workloads (CPU only).

    python -m paper_2411_10751_amd.profile_summary kernels DIR OUT.md  --cmd "..."
    python -m paper_2411_10751_amd.profile_summary traffic FETCH_DIR WRITE_DIR OUT.txt --kernel NAME
           --cells N --bytes-per-cell B --cmd "..." --cmd "..."
    python -m paper_2411_10751_amd.profile_summary counters OUT.md DIR [DIR ...] --kernel NAME
           --cells N [--kernel NAME --cells N ...] --cmd "..." [--cmd "..."]

`kernels` condenses the kernel statistics of a `--kernel-trace --stats`
run (CSV output) into a table.  `traffic` reads two `--pmc` runs, one with
FETCH_SIZE and one with WRITE_SIZE (KiB per dispatch), takes the mean of the
named kernel's dispatches, and scales each counter by what it reads for the
reference streaming dispatch of known size that bench.py issues with
--copy-calibration (an elementwise negation of 2^28 float32 values: 1 GiB read,
1 GiB written).  The result is HBM bytes per launch, stamped with a hash of the
kernel sources so that bench.py ignores it once the kernels have changed.
`counters` reads any number of `--pmc` runs (each a set of SQ counters) and
tabulates, for each named kernel, each counter's mean per dispatch, per cell
updated and per wavefront (when SQ_WAVES is among them).
"""
import argparse
import csv
import glob
import hashlib
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CALIB_BYTES = 1 << 30


def source_sha256():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_10751_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def short_name(name):
    """Kernel name without the library namespace, argument list and spaces."""
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]
    # drop the parameter list: the last top-level parenthesised group
    depth = 0
    for k, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            n = n[:k]
            break
    n = n.replace("holb::", "").replace(" ", "")
    return n


def _csv(dirname, suffix):
    files = sorted(glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit("no *%s under %s" % (suffix, dirname))
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _overlap(trace):
    """From the dispatch trace: per kernel, the time it ran with no other
    kernel on the device, and the device's busy time (the union of all
    dispatch intervals), in ns."""
    ev = []
    for r in trace:
        k = short_name(r["Kernel_Name"])
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        ev.append((t0, 1, k))
        ev.append((t1, -1, k))
    ev.sort(key=lambda e: (e[0], e[1]))
    alone, busy, active, last = {}, 0, {}, None
    for t, d, k in ev:
        if last is not None and active:
            busy += t - last
            if sum(active.values()) == 1:
                (only,) = [a for a, n in active.items() if n]
                alone[only] = alone.get(only, 0) + (t - last)
        active[k] = active.get(k, 0) + d
        if active[k] == 0:
            del active[k]
        last = t
    return alone, busy


def kernels(args):
    rows = _csv(args.dir, "kernel_stats.csv")
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    try:
        alone, busy = _overlap(_csv(args.dir, "kernel_trace.csv"))
    except SystemExit:
        alone, busy = {}, 0
    out = ["# Kernel time, %s" % args.title, "", "Command (from the repository root):", "",
           "    " + args.cmd, "",
           "| kernel | calls | average us | min us | max us | share of summed durations | "
           "alone, us per call |",
           "|---|---|---|---|---|---|---|"]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows[: args.top]:
        k = short_name(r["Name"])
        out.append("| `%s` | %s | %.2f | %.2f | %.2f | %.1f%% | %s |" % (
            k, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, 100.0 * float(r["TotalDurationNs"]) / total,
            "%.2f" % (alone.get(k, 0) / 1e3 / int(r["Calls"])) if busy else ""))
    if busy:
        out += ["", "Summed kernel durations %.3f ms; device busy (union of the dispatch intervals) %.3f ms. "
                "\"Alone\" is the time a dispatch ran with no other kernel on the device: kernels launched on "
                "the library's second stream overlap others, and a duration then includes the time it shared "
                "the device." % (total / 1e6, busy / 1e6)]
    open(args.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def _counter_means(dirname, counter):
    """{short kernel name: mean counter value per dispatch} of one pmc run."""
    rows = _csv(dirname, "counter_collection.csv")
    acc = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        k = short_name(r["Kernel_Name"])
        s, n = acc.get(k, (0.0, 0))
        acc[k] = (s + float(r["Counter_Value"]), n + 1)
    return {k: s / n for k, (s, n) in acc.items()}


def _calibration(means):
    cands = [k for k in means if re.search(r"neg", k)]
    if not cands:
        raise SystemExit("no calibration dispatch (elementwise negation) in the counter output")
    return max(means[k] for k in cands)


def traffic(args):
    fetch = _counter_means(args.fetch_dir, "FETCH_SIZE")
    write = _counter_means(args.write_dir, "WRITE_SIZE")
    key = args.kernel.replace(" ", "")
    fk = [k for k in fetch if k == key]
    wk = [k for k in write if k == key]
    if not fk or not wk:
        raise SystemExit("kernel %s not in the counter output (have: %s)" % (key, sorted(fetch)))
    f_kib, w_kib = fetch[fk[0]], write[wk[0]]
    cf_kib, cw_kib = _calibration(fetch), _calibration(write)
    f_scale = CALIB_BYTES / (cf_kib * 1024.0)
    w_scale = CALIB_BYTES / (cw_kib * 1024.0)
    hbm = f_kib * 1024.0 * f_scale + w_kib * 1024.0 * w_scale
    alg = args.cells * args.bytes_per_cell
    lines = [
        "# HBM traffic per launch of the dominant kernel, %s" % args.title,
        "# Commands (from the repository root), one rocprofv3 pass per counter:",
    ] + ["#   " + c for c in args.cmd] + [
        "# Counters are KiB per dispatch; each is scaled by its reading for the",
        "# calibration dispatch (elementwise negation of 2^28 float32: 1 GiB read, 1 GiB written).",
        "kernel: %s" % key,
        "source_sha256: %s" % source_sha256(),
        "fetch_kib_per_dispatch: %.1f" % f_kib,
        "write_kib_per_dispatch: %.1f" % w_kib,
        "calibration_fetch_kib: %.1f" % cf_kib,
        "calibration_write_kib: %.1f" % cw_kib,
        "fetch_scale: %.5f" % f_scale,
        "write_scale: %.5f" % w_scale,
        "hbm_bytes_per_launch: %.0f" % hbm,
        "algorithmic_bytes_per_launch: %d" % alg,
        "traffic_over_algorithmic: %.4f" % (hbm / alg),
    ]
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters(args):
    """One table per kernel named by --kernel (repeatable)."""
    rows = []
    for d in args.dirs:
        rows.append(_csv(d, "counter_collection.csv"))
    out = ["# Instruction counters, %s" % args.title, "",
           "Commands (from the repository root), one rocprofv3 pass each:", ""]
    out += ["    " + c for c in args.cmd]
    for kname, cells in zip(args.kernel, args.cells):
        key = kname.replace(" ", "")
        vals = {}
        for run in rows:
            acc = {}
            for r in run:
                if short_name(r["Kernel_Name"]) != key:
                    continue
                s, n = acc.get(r["Counter_Name"], (0.0, 0))
                acc[r["Counter_Name"]] = (s + float(r["Counter_Value"]), n + 1)
            for c, (s, n) in acc.items():
                vals[c] = s / n
        if not vals:
            raise SystemExit("kernel %s not in the counter output" % key)
        waves = vals.get("SQ_WAVES")
        out += ["", "## `%s`" % key, "",
                "Means over the kernel's dispatches; %d cells per dispatch%s." % (
                    cells, "" if waves is None else ", %.0f wavefronts" % waves), "",
                "| counter | per dispatch | per cell | per wavefront |", "|---|---|---|---|"]
        for c in sorted(vals):
            v = vals[c]
            out.append("| %s | %.4g | %.4g | %s |" % (c, v, v / cells, "" if not waves else "%.4g" % (v / waves)))
    if args.note:
        out += [""] + args.note
    open(args.out, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("dir")
    k.add_argument("out")
    k.add_argument("--cmd", required=True)
    k.add_argument("--title", default="")
    k.add_argument("--top", type=int, default=12)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("out")
    t.add_argument("--kernel", required=True)
    t.add_argument("--cells", type=int, required=True)
    t.add_argument("--bytes-per-cell", type=int, required=True)
    t.add_argument("--cmd", action="append", required=True)
    t.add_argument("--title", default="")
    n = sub.add_parser("counters")
    n.add_argument("out")
    n.add_argument("dirs", nargs="+")
    n.add_argument("--kernel", action="append", required=True)
    n.add_argument("--cells", type=int, action="append", required=True)
    n.add_argument("--cmd", action="append", required=True)
    n.add_argument("--title", default="")
    n.add_argument("--note", action="append", default=[])
    args = ap.parse_args()
    {"kernels": kernels, "traffic": traffic, "counters": counters}[args.what](args)


if __name__ == "__main__":
    main()
