"""Benchmark: zone-updates/s of the fp64 MHD step on one MI355X.

A step is one full two-stage step of the hot path (ghost fill, both
finite-volume stages, CFL dt, time update, sample) over the equidistant full domain
r in [0.1, 2] AU x theta in [30, 150] deg x phi in [0, 360) deg with
512 x 60 x 180 cells (2,400 blocks of 16 x 12 x 12), seeded wind and cone
CME, starting from the relaxation initial state.  One zone-update is one leaf
cell advanced by one full step.

Prints one JSON line.  The roofline entry is for the dominant kernel (the
fused stage kernel): algorithmic bytes per launch (128 B/cell for stage 1:
read U^n, write U*; 192 B/cell for stage 2: read U*, U^n, write U^{n+1};
160 B/cell on average) over its mean launch duration from HIP events on the
library's stream, in a pass after the timed region (the timed region replays
the captured step graph without events).  cpu_baseline times the oracle on
the host on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-updates/s (fp64 MHD, 1 GPU); AMR+learned flags vs equidistant to arrival"
PEAK_HBM_GBS = 8000.0
# schedules measured by the autotuner on MI355X (gfx950, 256 CUs); a device or
# work-list size without an entry is timed and appended
TUNE_CACHE = os.path.join(ROOT, "paper_2211_12867_amd", "tune_cache.txt")
BYTES_PER_CELL_LAUNCH = 160.0


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("csrc/stage.hip", "csrc/common.h", "csrc/physics.h", "csrc/kernels.h", "csrc/device.h", "build.py"):
        with open(os.path.join(ROOT, "paper_2211_12867_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(schedule=None):
    """HBM bytes per stage launch (FETCH_SIZE + WRITE_SIZE, each scaled by a
    plain 1 GiB copy) from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source and build flags with this schedule
    (waves, grid, xcd_order, ksplit); else None."""
    path = os.path.join(ROOT, "profiles", "stage_traffic_equidistant_full.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("kernel_source_hash", "bytes_per_launch_hbm", "schedule"):
                k, v = line.split(":", 1)
                vals[k] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash() or "bytes_per_launch_hbm" not in vals:
        return None
    if schedule is not None and vals.get("schedule") != ",".join(str(x) for x in schedule):
        return None
    return float(vals["bytes_per_launch_hbm"])


def measured_valu():
    """VALU issue fraction and executed fp64 rate of the stage kernel from the
    committed rocprofv3 counter summary (same kernel source only); else None."""
    import re
    path = os.path.join(ROOT, "profiles", "stage_valu_equidistant_full.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_hash: (\w+)", text)
    q = re.search(r": ([0-9.]+)% of one wave64 VALU instruction.*executed fp64 rate ([0-9.]+) TFLOP/s", text)
    if not m or m.group(1) != kernel_source_hash() or not q:
        return None
    return {"issue_frac": float(q.group(1)) / 100.0, "fp64_tflops_executed": float(q.group(2)), "fp64_peak": 78.6,
            "source": "profiles/stage_valu_equidistant_full.md"}


def _cpu_model():
    """CPU model name from lscpu with its family / model / stepping numbers
    (a virtual machine may report only a generic name); fallback /proc/cpuinfo."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True,
                             timeout=20).stdout
        f = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f.setdefault(k.strip(), v.strip())
        if "Model name" in f:
            extra = ", ".join("%s %s" % (k.lower(), f[k]) for k in ("CPU family", "Model", "Stepping") if k in f)
            return f["Model name"] + (" (%s)" % extra if extra else "")
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            return next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown"


def _oracle_sample(nr, seconds_target, max_steps):
    """Steps of the oracle on the inner nr radial cells of the equidistant grid
    (same spacing); returns (zone-updates/s, steps, seconds, cells)."""
    from oracle import solver
    from synthetic import as_dict, workload
    w = workload("equidistant_full")
    g = as_dict(w.grid)
    dr = (g["x1"][0] - g["x0"][0]) / g["n"][0]
    g["n"] = (nr, g["n"][1], g["n"][2])
    g["x1"] = (g["x0"][0] + nr * dr, g["x1"][1], g["x1"][2])
    s = solver.PatchSolver(g, as_dict(w.wind), as_dict(w.cmes[0]))
    cells = nr * g["n"][1] * g["n"][2]
    steps = 0
    t0 = time.perf_counter()
    while True:
        s.step()
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds_target or steps >= max_steps:
            break
    return cells * steps / el, steps, el, cells


def cpu_baseline(seconds_target=15.0):
    """The oracle (plain fp64 C core with OpenMP) on a bounded sample of the
    workload: the same grid spacing over the inner 64 radial cells, on every
    core the process may run on (affinity mask, capped by OMP_NUM_THREADS when
    set), and on one thread (inner 16 radial cells, a child process)."""
    import subprocess
    affinity = len(os.sched_getaffinity(0))
    threads = affinity
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    # the oracle's OpenMP runtime starts on first use: fix its team here
    os.environ["OMP_NUM_THREADS"] = str(threads)
    os.environ.setdefault("OMP_PROC_BIND", "close")
    rate, steps, el, cells = _oracle_sample(64, seconds_target, 50)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import sys, json; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench._oracle_sample(16, 10.0, 8)))" % ROOT)
    single = None
    try:
        res = subprocess.run([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                             text=True, env=env, timeout=120)
        r1, s1, e1, c1 = json.loads(res.stdout.strip().splitlines()[-1])
        single = {"value": r1, "cores": 1, "sample": "%d steps of the 16 x 60 x 180 inner-radius part (%.1f s)"
                                                       % (s1, e1)}
    except (OSError, subprocess.SubprocessError, ValueError, IndexError):
        single = None
    return {"value": rate, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
            "cpu": _cpu_model(), "affinity_cpus": affinity,
            "sample": "%d steps of the 64 x 60 x 180 inner-radius part of the same grid (%.1f s, %d threads)"
                      % (steps, el, threads),
            "single_thread": single}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default stage schedule (profiling runs: no tuning launches in the trace)")
    ap.add_argument("--schedule", default=None,
                    help="force the stage schedule waves,grid,xcd_order,ksplit (e.g. 2,0,1,1) instead of tuning")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="schedule cache of the autotuner ('' = time the candidates)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (known bytes) to scale HBM counters")
    ap.add_argument("--no-forecast", action="store_true",
                    help="skip the forecast comparison (equidistant vs learned AMR to the 1 AU arrival, ~40 s)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the single-run hot path has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    import paper_2211_12867_amd as ic
    from synthetic import as_dict, workload

    w = workload("equidistant_full")
    g = as_dict(w.grid)
    print("bench: creating %s %s blocks %s" % (w.name, g["n"], g["block"]), file=sys.stderr, flush=True)
    sim = ic.Sim(g, as_dict(w.wind), [as_dict(w.cmes[0])])
    cells = g["n"][0] * g["n"][1] * g["n"][2]
    for _ in range(args.warmup):
        sim.step()
    if args.schedule:
        sim.set_tuning(*[int(x) for x in args.schedule.split(",")])
    elif not args.no_autotune:
        sim.autotune(args.tune_cache or None, reps=3)
    tune = dict(zip(("waves_per_simd", "grid", "xcd_order", "ksplit"), sim.tuning()))
    print("bench: schedule %s" % tune, file=sys.stderr, flush=True)
    n0 = sim.step()["steps"]                    # captures the step graph for the tuned schedule
    # timed region: exactly K steps of the captured step graph in one advance
    # call (the library reads the time back every 20 steps, not after each
    # step), no per-launch events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sim.advance(1e12, max_steps=args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert info["steps"] - n0 == args.steps, (info["steps"], n0, args.steps)
    # kernel time of the dominant kernel: HIP events around every stage launch on
    # the library's stream, over a separate pass of the same steps
    sim.set_kernel_timing(True)
    for q in range(max(2, min(args.steps, 10))):
        sim.step()
    launches, mean_ms = sim.stage_timing()
    sim.set_kernel_timing(False)
    t_s, dt_s = sim.time()
    sim.close()
    print("bench: %d steps in %.3f s, stage kernel %d launches, mean %.3f ms, t = %.0f s, dt = %.1f s"
          % (args.steps, el, launches, mean_ms, t_s, dt_s), file=sys.stderr, flush=True)

    if args.copy_calibration:
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("bench: copy calibration, 3 copies of %d bytes" % (n * 8), file=sys.stderr, flush=True)
        del src, dst

    bytes_launch = BYTES_PER_CELL_LAUNCH * cells
    achieved = bytes_launch / (mean_ms * 1e-3) / 1e9
    traffic = measured_traffic(tuple(tune[k] for k in ("waves_per_simd", "grid", "xcd_order", "ksplit")))
    out = {
        "metric": METRIC,
        "value": cells * args.steps / el,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "equidistant_full: 512x60x180 cells, r 0.1-2 AU, theta 30-150 deg, "
                               "phi 0-360 deg, 2400 blocks of 16x12x12, seeded wind + cone CME",
                   "cells": cells, "block": list(g["block"]), "parallelism": "single GPU",
                   "schedule": {k: tune[k] for k in ("waves_per_simd", "grid", "xcd_order", "ksplit")}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "k_stage<16, 12, 12, 8, %d, 0>" % tune["waves_per_simd"], "mean_launch_ms": mean_ms,
                     "bytes_per_launch": bytes_launch, "valu": measured_valu()},
    }
    if not args.no_forecast:
        # the forecast target: the learned-flag AMR runs against the equidistant
        # run to the shock arrival at 1 AU (wall times on this GPU, each run's
        # relaxation included, and of the CME phase alone); after the timed
        # region, outside it
        from paper_2211_12867_amd import forecast
        print("bench: forecast comparison (equidistant vs learned AMR, 4 and 5 levels)", file=sys.stderr, flush=True)
        res = forecast.arrival_comparison(levels=(4, 5), log=lambda m: print("bench: " + m, file=sys.stderr,
                                                                           flush=True))
        out["forecast"] = {"workload": "equidistant_full vs learned_flags (stretched 60x24x48, 12^3 blocks), "
                                       "wind seed 0, cone CME 1500 km/s, relax 14 d then 3 d",
                           "target": "arrival within 1 h of the equidistant run at >= 10x lower wall time",
                           "runs": res}
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
