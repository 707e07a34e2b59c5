"""Throughput of the fused high-order LBM step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--storage f32|f16|bf16]

Default workload: the D3Q39 Rayleigh-Benard box, 256^3 cells, body force +
thermal-dissipation source, TMS walls normal to z, FP32 population storage.
One step is one pass of the whole per-step update over every cell (wall
closure, streaming, shifted moments, sources, equilibrium, collision, store);
the timed region also ends with one FP64 conservation reduction.  Inputs are
synthetic (seeded fields of the workload recipe) and resident in HBM before
timing starts.

Prints one JSON line with the throughput (MLUPS = cell updates / s / 1e6),
the roofline of the step against MI355X HBM bandwidth, and the FP64 CPU oracle
timed on a bounded sample of the same workload as a baseline.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + % of HBM peak for fused collide-stream-source, FP32/FP16-store vs FP64"
HBM_PEAK_GBS = 8000.0
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
STORE_BYTES = {0: 4, 1: 2, 2: 2}
DTYPE_NAME = {0: "f32", 1: "f32 (f16-deviation storage)", 2: "f32 (bf16-deviation storage)"}


def workload(name):
    from paper_2411_10751_amd import inputs
    if name == "rb3d":
        return inputs.rayleigh_benard_3d(n=256, steps=200)
    if name == "thermal2d":
        return inputs.thermal_2d(n=1024, steps=200)
    if name == "ptensor2d":
        return inputs.ptensor_2d(n=2048, steps=200)
    if name == "body2d":
        return inputs.body_force_2d(n=2048, steps=200)
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(name, storage):
    """FP64 oracle on a bounded sample of the workload (about 10-30 s of CPU)."""
    import numpy as np
    from oracle import orc
    from paper_2411_10751_amd import inputs
    if name == "rb3d":
        w = inputs.rayleigh_benard_3d(n=64, steps=300)
        sample = "D3Q39 Rayleigh-Benard 64^3 with walls, body+thermal, 300 steps"
    elif name == "thermal2d":
        w = inputs.thermal_2d(n=256, steps=1500)
        sample = "D2Q37 thermal 256^2, 1500 steps"
    elif name == "ptensor2d":
        w = inputs.ptensor_2d(n=256, steps=1000, ndrops=6, rmin=10, rmax=20, gap=8)
        sample = "D2Q37 pressure tensor 256^2 droplets, 1000 steps"
    else:
        w = inputs.body_force_2d(n=256, steps=1500)
        sample = "D2Q37 body force 256^2, 1500 steps"
    c = w["config"]
    s = orc.Sim(c["lattice"], c["nx"], c["ny"], c.get("nz", 1), tau_hat=c["tau_hat"], sources=c["sources"],
                isothermal=c.get("isothermal", 0), g=c["g"], prandtl=c["prandtl"], eos_a=c["eos_a"],
                eos_b=c["eos_b"], eos_T=c["eos_T"], sc_G=c["sc_G"], ptensor_k=c["ptensor_k"],
                walls=c["walls"], theta_wall=c["theta_wall"], u_wall=c["u_wall"], eos=c.get("eos", 0))
    s.init(w["rho"].astype(np.float64), w["u"].astype(np.float64), w["theta"].astype(np.float64))
    s.step(1)
    t0 = time.perf_counter()
    s.step(w["steps"])
    dt = time.perf_counter() - t0
    cells = c["nx"] * c["ny"] * c.get("nz", 1)
    cores = orc.num_threads()
    # the same oracle on one thread, over a twentieth of the steps
    n1 = max(w["steps"] // 20, 1)
    orc.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        s.step(n1)
        dt1 = time.perf_counter() - t1
    finally:
        orc.set_num_threads(cores)
    return {"value": round(cells * w["steps"] / dt / 1e6, 4), "unit": "MLUPS", "cores": cores,
            "kind": "oracle", "sample": sample + " (FP64, %.1f s)" % dt,
            "single_thread": {"value": round(cells * n1 / dt1 / 1e6, 4), "unit": "MLUPS", "cores": 1,
                              "sample": "the same state, %d more steps on one thread (%.1f s)" % (n1, dt1)}}


def frames_of_kernel(kernel):
    """Frame mode of a single-run step kernel from its name (its last template
    argument: 0 per cell, 1 per plane, 2 per cell with momentum)."""
    try:
        return {0: "cell", 1: "plane", 2: "cellu"}[int(kernel.rstrip(">").rsplit(",", 1)[1])]
    except (ValueError, IndexError, KeyError):
        return "unknown"


def traffic_from_profile(kernel, name, storage, variant):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the kernel source as it is now, on this kernel and in this
    block order (the traffic depends on it)."""
    import re
    from paper_2411_10751_amd.profile_summary import source_sha256
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (name, {0: "f32", 1: "f16", 2: "bf16"}[storage]))
    if not os.path.exists(path):
        return None
    lines = open(path).read().splitlines()
    m = re.search(r"variant (\d+)", lines[0] if lines else "")
    if m is None or int(m.group(1)) != variant:
        return None
    vals = {}
    for line in lines:
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_sha256() or vals.get("kernel") != kernel:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(torch):
    """The reference dispatch that scales the profiler's byte counters: an
    elementwise negation of 2^28 float32 (1 GiB in, 1 GiB out), three times."""
    a = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b


def bench_batched(args):
    """512 independent D2Q37 body-force + thermal runs (sizes 32^2..256^2,
    uneven parameters) advanced together by the batched form, FP32."""
    import torch
    from paper_2411_10751_amd import holb, inputs
    runs = inputs.batched_runs(nruns=512, steps=200)
    if args.grad_lag:
        for r in runs:
            r["config"] = dict(r["config"], grad_lag=1)
    cells = sum(r["config"]["nx"] * r["config"]["ny"] for r in runs)
    torch.cuda.set_device(0)
    b = holb.Batch([r["config"] for r in runs])
    b.init([r["rho"] for r in runs], [r["u"] for r in runs], [r["theta"] for r in runs])
    if args.variant is not None and args.variant >= 0:
        b.set_variant(args.variant)
        variant = args.variant
    else:
        variant = b.tune()
    b.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    b.timing_start(args.steps)  # eager steps, HIP events around each collision launch
    e0.record(stream)
    b.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / args.steps
    kern_ms, launches, kcells, kernel = b.timing_stop()
    kern_ms /= max(launches, 1)
    # the same steps replayed from the captured graph, for comparison
    torch.cuda.synchronize()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    b.step(args.steps)
    g1.record(stream)
    torch.cuda.synchronize()
    graph_ms = g0.elapsed_time(g1) / args.steps
    # the plain alternative: the same runs advanced one at a time, each as its
    # own simulation (same frames as the batch)
    sims = []
    for r in runs:
        sm = holb.Sim(dict(r["config"], frames=2))
        sm.init(r["rho"], r["u"], r["theta"])
        sims.append(sm)
    for sm in sims:
        sm.step(1)
    torch.cuda.synchronize()
    single_steps = 10
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for sm in sims:
        sm.step(single_steps)
    s1.record(stream)
    torch.cuda.synchronize()
    single_ms = s0.elapsed_time(s1) / single_steps
    for sm in sims:
        sm.close()
    if args.copy_calibration:
        copy_calibration(torch)
    bpc = 2 * 37 * 4
    achieved = bpc * kcells / (kern_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(kernel, "batched", 0, variant)
    line = {
        "metric": METRIC,
        "value": round(cells / (step_ms * 1e-3) / 1e6, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 5),
        "wall_s_timed": round(wall, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded fields of the workload recipe)",
        "config": {"workload": "d2q37_batched_512_runs", "runs": len(runs), "cells": cells,
                   "grad_lag": int(bool(args.grad_lag)),
                   "variant": variant, "graph_replay_ms_per_step": round(graph_ms, 5),
                   "one_run_at_a_time_ms_per_step": round(single_ms, 5),
                   "one_run_at_a_time_mlups": round(cells / (single_ms * 1e-3) / 1e6, 2)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
                     "kernel_ms": round(kern_ms, 5), "cells_per_launch": kcells, "alg_bytes_per_cell": bpc,
                     "step_frac": round(bpc * cells / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    if not args.no_cpu_baseline:
        from oracle import orc
        import numpy as np
        sample = runs[:16]
        t0 = time.perf_counter()
        ncell = 0
        for r in sample:
            c = r["config"]
            sim = orc.Sim(c["lattice"], c["nx"], c["ny"], 1, tau_hat=c["tau_hat"], sources=c["sources"],
                          g=c["g"], prandtl=c["prandtl"])
            sim.init(r["rho"].astype(np.float64), r["u"].astype(np.float64), r["theta"].astype(np.float64))
            sim.step(250)
            ncell += c["nx"] * c["ny"] * 250
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(ncell / dt / 1e6, 4), "unit": "MLUPS", "cores": orc.num_threads(),
                                "kind": "oracle", "sample": "first 16 runs of the batch, 250 steps each (FP64, %.1f s)"
                                % dt}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="rb3d", choices=["rb3d", "thermal2d", "ptensor2d", "body2d", "batched"])
    ap.add_argument("--storage", default="f32", choices=list(STORAGE))
    ap.add_argument("--variant", type=int, default=None,
                    help="kernel block order (for the batched workload: its launch shape); -1: autotune; "
                         "default: 0 for the single-run workloads (the order their rocprofv3 summaries were "
                         "taken in; the orders differ by at most 3%% there), autotuned for the batched one")
    ap.add_argument("--frames", default="auto", choices=["auto", "cell", "plane", "cellu"],
                    help="reference frames of the stored populations")
    ap.add_argument("--grad-lag", action="store_true",
                    help="thermal source: gradient of the previous step's theta (one pass per step) instead of "
                         "the same step's (the default, two passes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true", help="time every kernel variant (to stderr) before the run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, stream 1 GiB in and 1 GiB out three times (elementwise "
                         "negation of 2^28 float32: the reference dispatch that scales profiler byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (each run fits one "
              "MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2411_10751_amd import holb

    storage = STORAGE[args.storage]
    if args.workload == "batched":
        return bench_batched(args)
    w = workload(args.workload)
    frames = {"auto": 0, "cell": 1, "plane": 2, "cellu": 3}[args.frames]
    cfg = dict(w["config"], storage=storage, frames=frames)
    if args.grad_lag:
        cfg["grad_lag"] = 1
    Q = 37 if cfg["lattice"] == 0 else 39
    cells = cfg["nx"] * cfg["ny"] * cfg.get("nz", 1)
    torch.cuda.set_device(0)
    sim = holb.Sim(cfg)
    sim.init(w["rho"], w["u"], w["theta"])
    if args.sweep:
        # a warm-up first (the device clocks ramp up), then the fastest of two
        # round-robin passes of 20 steps per variant
        sim.step(20)
        best = {}
        for _ in range(2):
            for v in range(sim.num_variants()):
                try:
                    sim.set_variant(v)
                except Exception:
                    continue
                sim.step(2)
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                sim.step(20)
                b.record()
                torch.cuda.synchronize()
                best[v] = min(best.get(v, 1e30), a.elapsed_time(b) / 20)
        for v in sorted(best):
            print("variant %d: %.4f ms/step" % (v, best[v]), file=sys.stderr, flush=True)
        sim.init(w["rho"], w["u"], w["theta"])
    if args.variant is None:
        args.variant = 0
    if args.variant >= 0:
        sim.set_variant(args.variant)
        variant = args.variant
    else:
        variant = sim.tune()
    sim.step(args.warmup)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.timing_start(args.steps)  # HIP events around the dominant kernel of each step
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    totals = sim.reduce()  # FP64 conservation totals (synchronises)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / args.steps
    kern_ms, launches, kcells, kernel = sim.timing_stop()
    kern_ms /= max(launches, 1)

    if args.copy_calibration:
        copy_calibration(torch)

    mlups = cells / (step_ms * 1e-3) / 1e6
    bpc = 2 * Q * STORE_BYTES[storage]  # read + write every population once
    achieved = bpc * kcells / (kern_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(kernel, args.workload, storage, variant)
    line = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 5),
        "wall_s_timed": round(wall, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_NAME[storage],
        "data": "synthetic (seeded fields of the workload recipe)",
        "config": {
            "workload": w["name"],
            "lattice": "D2Q37" if cfg["lattice"] == 0 else "D3Q39",
            "grid": [cfg["nx"], cfg["ny"], cfg.get("nz", 1)],
            "sources": cfg["sources"],
            "walls": cfg["walls"],
            "storage": args.storage,
            "grad_lag": int(bool(args.grad_lag)),
            "variant": variant,
            # frames as the library resolved them: the last template argument
            # of the dominant kernel
            "frames": frames_of_kernel(kernel),
            "mass": totals[0],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": kernel,
            "kernel_ms": round(kern_ms, 5),
            "cells_per_launch": kcells,
            "alg_bytes_per_cell": bpc,
            "whole_step_gbs": round(bpc * cells / (step_ms * 1e-3) / 1e9, 1),
            # the whole step (every launch) at the same algorithmic bytes
            "step_frac": round(bpc * cells / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, storage)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
