"""Forecast runs on the library: wind relaxation, the CME phase with the
sample-point record and the shock arrival there, look-ahead training pairs for
the learned refinement flags, their training, and the comparison of
refinement sources.

Everything here drives the C ABI through the binding; every step of the
method runs in the library's kernels.  Times at this interface are seconds
unless a name says hours or days.

    python -m paper_2211_12867_amd.forecast train  --out flags.npz ...
    python -m paper_2211_12867_amd.forecast compare --net flags.npz ...
    python -m paper_2211_12867_amd.forecast fig1 --out fig1.npz
    python -m paper_2211_12867_amd.forecast tracer --out tracer.npz
"""
import argparse
import atexit
import json
import os
import sys
import tempfile
import time

import numpy as np

from . import IC_SOURCE_LEARNED_JUDGED, IC_SOURCE_PLAIN, Sim, mlp_infer, mlp_init, mlp_train, shock_diagnostics, units

DAY = 86400.0
HOUR = 3600.0
SAMPLE = (1.0, 90.0, 0.0)          # r [AU], colatitude, longitude [deg] in the co-rotating frame
TUNE_CACHE = None                  # schedule cache file of ic_autotune (None: a file of this process)
_tune_file = None


def _tune_cache():
    """Cache file for ic_autotune: each block shape and work-list size is timed
    once per process (or per TUNE_CACHE file) and looked up afterwards."""
    global _tune_file
    if TUNE_CACHE:
        return TUNE_CACHE
    if _tune_file is None:
        fd, _tune_file = tempfile.mkstemp(prefix="icarus_tune_", suffix=".txt")
        os.close(fd)
        atexit.register(lambda path=_tune_file: os.path.exists(path) and os.remove(path))
    return _tune_file


def _log(log, msg):
    if log:
        log(msg)


def relax(grid, wind, cme, t_end_s, chunk_s=DAY, log=print):
    """Advance the relaxation initial state on the base grid (no regrids) to
    t_end_s.  Returns dict(blocks, U, t_s, steps, wall_s)."""
    g = dict(grid, max_level=1)
    sim = Sim(g, wind, [cme], dict(regrid_every=0))
    t0 = time.perf_counter()
    sim.autotune(_tune_cache(), reps=3)
    steps = 0
    while sim.time()[0] < t_end_s * (1.0 - 1e-12):
        info = sim.advance(min(chunk_s, t_end_s - sim.time()[0]))
        steps = info["steps"]
        _log(log, "relax: t = %.2f d, %d steps, %.1f s" % (info["t_s"] / DAY, steps, time.perf_counter() - t0))
    bl, U = sim.state()
    out = dict(blocks=bl, U=U, t_s=sim.time()[0], steps=steps, wall_s=time.perf_counter() - t0)
    sim.close()
    return out


MIN_JUMP_KMS = 100.0   # a rise of v_r smaller than this within the window is no shock arrival


def _series_diagnostics(ts, t_cme_s, window_h=96.0):
    """(t [h], v_r [km/s]) of the record and its shock diagnostics
    (ic_shock_diagnostics: arrival and width [h], peak speed [km/s], average
    gradient [km/s per h]; NaN without a rise of at least MIN_JUMP_KMS)."""
    t_h = ts[:, 0] / HOUR
    v = ts[:, 2] * units()["speed_m_s"] / 1e3
    d = shock_diagnostics(ts[:, 0], v, t_cme_s, window_h * HOUR, MIN_JUMP_KMS)
    out = dict(arrival_h=d["arrival_s"] / HOUR, width_h=d["width_s"] / HOUR, peak_kms=d["v_max"],
               gradient_kms_h=d["gradient"] * HOUR, v_pre_kms=d["v_pre"])
    return t_h, v, out


def _series_arrival(ts, t_cme_s, window_h=96.0):
    """(t [h], v_r [km/s], arrival [h], width [h]) of the record."""
    t_h, v, d = _series_diagnostics(ts, t_cme_s, window_h)
    return t_h, v, d["arrival_h"], d["width_h"]


def cme_run(grid, wind, cme, amr, start, t_end_s, network=None, chunk_s=DAY / 4, log=print, max_blocks=0,
            tracer=False):
    """From a relaxed state (relax's dict; None starts a plain equidistant run
    from the initial state and runs it through the relaxation too) advance to
    t_end_s with regrids at amr's cadence, recording the sample point every
    step.  network = (params, mean, std) for the learned sources; tracer
    carries the CME density tracer (a relaxed wind holds no CME material:
    rho s = 0).  Returns dict(arrival_h, width_h, wall_s, cme_wall_s, steps,
    leaf_block_steps, max_leaves, leaves_end, max_level, regrid_stats, t_h,
    v_kms); cme_wall_s is the wall time from the CME start on (the whole run
    when it starts from a relaxed state at the CME start)."""
    sim = Sim(grid, wind, [cme], amr, max_blocks=max_blocks, tracer=tracer)
    if start is not None:
        U = start["U"]
        if tracer and U.shape[1] == 8:
            U = np.concatenate([U, np.zeros_like(U[:, :1])], axis=1)
        sim.set_state(start["blocks"], U, start["t_s"])
    if network is not None:
        sim.mlp_set(*network)
    sim.set_sample_point(*SAMPLE)
    cells = grid["block"][0] * grid["block"][1] * grid["block"][2]
    zu0 = 0.0
    max_leaves = len(sim.blocks())
    max_level = 1
    ts = []
    t0 = time.perf_counter()
    t_cme_wall = t0 if sim.time()[0] >= cme["t_start_s"] * (1.0 - 1e-12) else None
    info = None
    while sim.time()[0] < t_end_s * (1.0 - 1e-12):
        if t_cme_wall is None and sim.time()[0] >= cme["t_start_s"] * (1.0 - 1e-12):
            t_cme_wall = time.perf_counter()
        sim.autotune(_tune_cache(), reps=3)      # the work list changes with the forest
        info = sim.advance(min(chunk_s, t_end_s - sim.time()[0]))
        ts.append(sim.timeseries())
        sim.timeseries_clear()
        max_leaves = max(max_leaves, info["leaves"])
        max_level = max([max_level] + [l + 1 for l, c in enumerate(info["leaves_per_level"]) if c > 0])
        _log(log, "cme: t = %.2f d, %d steps, %d leaves %s, %.1f s"
             % (info["t_s"] / DAY, info["steps"], info["leaves"], info["leaves_per_level"][:6],
                time.perf_counter() - t0))
    t1 = time.perf_counter()
    wall = t1 - t0
    cme_wall = t1 - t_cme_wall if t_cme_wall is not None else 0.0
    ts = np.concatenate(ts) if ts else np.zeros((0, 9))
    t_h, v, diag = _series_diagnostics(ts, cme["t_start_s"])
    a, w = diag["arrival_h"], diag["width_h"]
    out = dict(arrival_h=a, width_h=w, peak_kms=diag["peak_kms"], gradient_kms_h=diag["gradient_kms_h"],
               wall_s=wall, cme_wall_s=cme_wall, steps=info["steps"] if info else 0,
               leaf_block_steps=((info["zone_updates"] if info else 0.0) - zu0) / cells, max_leaves=max_leaves,
               leaves_end=info["leaves"] if info else max_leaves, max_level=max_level,
               regrid_stats=sim.regrid_stats(), t_h=t_h, v_kms=v)
    sim.close()
    return out


def stretching_comparison(relax_days=14.0, cme_days=3.0, log=print):
    """The low-resolution pair of paper Sect. 2.2 (Fig. 1): the same seeded
    wind and cone CME (the full-domain workload's) on the equidistant grid of
    300 radial cells (1.362 R_sun at 1 AU) and on the radially stretched grid
    of 60 cells (10.7 R_sun at 1 AU), 24 x 96 angular cells, no refinement;
    each relaxes from the initial state and runs cme_days after the CME
    start.  Returns {name: cme_run's dict plus dr_1au_rsun}."""
    from synthetic import as_dict, workload
    w = workload("equidistant_full")
    wind = as_dict(w.wind)
    cme = dict(as_dict(w.cmes[0]), t_start_s=relax_days * DAY)
    base = dict(geometry="spherical", x0=(0.1, 30.0, 0.0), x1=(2.0, 150.0, 360.0), block=(12, 12, 12),
                periodic=(False, False, True), max_level=1, gamma=1.5, cfl=0.4)
    rsun = units()["length_m"] / 6.957e8
    out = {}
    for name, n, stretched in (("low_equidistant", (300, 24, 96), False), ("low_stretched", (60, 24, 96), True)):
        g = dict(base, n=n, stretched_r=stretched)
        _log(log, "== %s %s" % (name, n))
        r = cme_run(g, wind, cme, dict(regrid_every=0), None, (relax_days + cme_days) * DAY, log=log, chunk_s=DAY)
        if stretched:
            q = (2.0 / 0.1) ** (1.0 / n[0])
            r["dr_1au_rsun"] = (q ** 0.5 - q ** -0.5) * rsun
        else:
            r["dr_1au_rsun"] = 1.9 / n[0] * rsun
        out[name] = r
    return out


def tracer_comparison(relax_days=14.0, cme_days=3.0, max_level=3, log=print):
    """CME-tracing refinement (paper Sect. 3.1) against unrefined grids and the
    shock criterion (Sect. 3.2), on the stretched AMR workload's wind and CME:
    its base grid and the grid twice as fine everywhere (each relaxed on
    itself), and from the base grid's relaxed wind the tracer criterion
    (refine where CME material is, s > tracer_refine) up to levels 2 and
    max_level and the shock criterion up to max_level.  The paper finds the
    tracer run of three levels arriving with the uniformly twice-finer grid
    (the CME material at level 3 in level-2 surroundings): resolving the
    material itself does not move the shock.  Returns {name: cme_run's
    dict}."""
    from synthetic import as_dict, workload
    w = workload("stretched_amr")
    grid = dict(as_dict(w.grid), max_level=1)
    wind = as_dict(w.wind)
    cme = dict(as_dict(w.cmes[0]), t_start_s=relax_days * DAY)
    amr = as_dict(w.amr)
    t_end = (relax_days + cme_days) * DAY
    out = {}
    fine = dict(grid, n=tuple(2 * x for x in grid["n"]))
    for name, g in (("base", grid), ("uniform_x2", fine)):
        _log(log, "== %s %s" % (name, g["n"]))
        st = relax(g, wind, cme, relax_days * DAY, log=log)
        out[name] = cme_run(g, wind, cme, dict(amr, regrid_every=0), st, t_end, log=log)
        if name == "base":
            start = st
    runs = [("tracer_L2", 2, "tracer"), ("tracer_L%d" % max_level, max_level, "tracer"),
            ("shock_L%d" % max_level, max_level, "shock")]
    for name, lv, crit in runs:
        _log(log, "== %s" % name)
        out[name] = cme_run(dict(grid, max_level=lv), wind, cme, dict(amr, criterion=crit), start, t_end,
                            log=log, tracer=crit != "shock")
    return out


def arrival_comparison(levels=(4, 5), relax_days=14.0, cme_days=3.0, log=print):
    """The forecast comparison the learned flags are for (paper Sect. 3.2,
    Tab. 5): the equidistant full-domain run (512 x 60 x 180, its own
    relaxation) against stretched AMR runs with the learned flags (judged, no
    buffer, the stored network and threshold) up to each of `levels`, the same
    seeded wind and cone CME, to the shock arrival at the sample point.  AMR
    wall times include their shared base-grid relaxation.  Returns {name:
    dict(arrival_h, width_h, wall_s, cme_wall_s, steps, leaf_block_steps)},
    the AMR runs with speedup (equidistant wall / own wall, relaxations
    included), speedup_cme (the same for the CME phase alone) and
    arrival_diff_h."""
    net, meta = load_network(os.path.join(os.path.dirname(os.path.abspath(__file__)), "flags_net.npz"))
    grid, wind, cme, amr, _ = _workload_parts("learned_flags")
    t_end = (relax_days + cme_days) * DAY
    cme = dict(cme, t_start_s=relax_days * DAY)
    st = relax(grid, wind, cme, relax_days * DAY, log=log)
    keys = ("arrival_h", "width_h", "wall_s", "cme_wall_s", "steps", "leaf_block_steps")
    out = {}
    for lv in levels:
        a = dict(amr, source=IC_SOURCE_LEARNED_JUDGED, buffer_blocks=0, learned_threshold=meta.get("threshold", 0.5))
        _log(log, "== learned_L%d" % lv)
        r = cme_run(dict(grid, max_level=lv), wind, cme, a, st, t_end, network=net, log=log)
        r["wall_s"] += st["wall_s"]
        out["learned_L%d" % lv] = {k: r[k] for k in keys}
    g1, w1, c1, _, _ = _workload_parts("equidistant_full")
    _log(log, "== equidistant")
    r = cme_run(g1, w1, dict(c1, t_start_s=relax_days * DAY), dict(regrid_every=0), None, t_end, log=log, chunk_s=DAY)
    eq = {k: r[k] for k in keys}
    for v in out.values():
        v["speedup"] = eq["wall_s"] / v["wall_s"]
        v["speedup_cme"] = eq["cme_wall_s"] / v["cme_wall_s"]
        v["arrival_diff_h"] = v["arrival_h"] - eq["arrival_h"]
    out["equidistant"] = eq
    return out


def collect_pairs(grid, wind, cme, amr, start, t_end_s, every, log=print, max_blocks=0, keep_every=1):
    """Training pairs of a plain run (buffer and cadence as in amr): at each
    regrid time the features of every leaf that touches the refinement
    windows (the others never refine, whatever the network says), labelled
    1 if the leaf meets the refinement condition (ic_eval_hot) at that time or
    after any of the next `every` steps, else 0; pairs are kept from every
    keep_every-th regrid cycle.  Returns (raw float32 [n, 512], y uint8 [n])."""
    sim = Sim(grid, wind, [cme], dict(amr, source=IC_SOURCE_PLAIN), max_blocks=max_blocks)
    sim.set_state(start["blocks"], start["U"], start["t_s"])
    X, Y = [], []
    t0 = time.perf_counter()
    cycle = 0
    while sim.time()[0] < t_end_s:
        keep = cycle % keep_every == 0
        if keep:
            win = sim.eval_window().astype(bool)
            x = sim.features()[win]
            lab = sim.eval_hot().astype(bool)
        for _ in range(every):
            sim.step()
            if keep:
                lab |= sim.eval_hot().astype(bool)
        if keep:
            X.append(x)
            Y.append(lab[win].astype(np.uint8))
        info = sim.regrid()
        cycle += 1
        if cycle % 20 == 0:
            n = sum(len(y) for y in Y)
            pos = sum(int(y.sum()) for y in Y)
            _log(log, "collect: t = %.2f d, %d pairs (%.3f positive), %d leaves, %.1f s"
                 % (sim.time()[0] / DAY, n, pos / max(n, 1), info["leaves"], time.perf_counter() - t0))
    sim.close()
    return np.concatenate(X), np.concatenate(Y)


def train(raw, y, epochs=10, batch=4096, lr=1e-3, seed=0):
    """Weighted BCE (pos_weight = N_neg / N_pos) with Adam on the GPU from a
    He-uniform start.  Returns (params, mean, std, loss per epoch)."""
    return mlp_train(raw, y, mlp_init(seed), epochs=epochs, batch=batch, lr=lr, seed=seed, pos_weight=0.0)


def evaluate(raw, y, network):
    """REFINE recall and precision, accuracy and positive rate of the
    network's p >= 1/2 decision on labelled rows."""
    p = mlp_infer(raw, *network) >= 0.5
    y = np.asarray(y).astype(bool)
    tp = int(np.sum(p & y))
    return dict(rows=int(len(y)), positive=float(y.mean()), recall=tp / max(int(y.sum()), 1),
                precision=tp / max(int(p.sum()), 1), accuracy=float(np.mean(p == y)))


def save_network(path, params, mean, std, meta):
    np.savez(path, params=np.asarray(params, np.float32), mean=np.asarray(mean, np.float32),
             std=np.asarray(std, np.float32), meta=np.array(json.dumps(meta)))


def load_network(path):
    d = np.load(path, allow_pickle=False)
    return (d["params"], d["mean"], d["std"]), json.loads(str(d["meta"]))


def ensemble_run(grid, wind, cmes, amr, start, t_end_s, chunk_s=DAY / 4, log=print):
    """All members in one sim from one relaxed state: every leaf of every member
    in the same launches, per-member dt and regrids.  Returns dict(arrival_h
    and width_h per member, wall_s, steps per member, zone_updates, max_leaves)."""
    sim = Sim(grid, wind, cmes, amr)
    for m in range(len(cmes)):
        sim.set_state(start["blocks"], start["U"], start["t_s"], member=m)
    sim.set_sample_point(*SAMPLE)
    series = [[] for _ in cmes]
    t0 = time.perf_counter()
    info = None
    max_leaves = 0
    while min(sim.time(m)[0] for m in range(len(cmes))) < t_end_s * (1.0 - 1e-12):
        sim.autotune(_tune_cache(), reps=3)
        info = sim.advance(min(chunk_s, t_end_s - sim.time(0)[0]))
        for m in range(len(cmes)):
            series[m].append(sim.timeseries(m))
        sim.timeseries_clear()
        nl = sum(len(sim.blocks(m)) for m in range(len(cmes)))
        max_leaves = max(max_leaves, nl)
        _log(log, "ensemble: t = %.2f d, %d leaves over %d members, %.1f s"
             % (sim.time(0)[0] / DAY, nl, len(cmes), time.perf_counter() - t0))
    wall = time.perf_counter() - t0
    arr, wid, steps = [], [], []
    for m, c in enumerate(cmes):
        ts = np.concatenate(series[m])
        _, _, a, w = _series_arrival(ts, c["t_start_s"])
        arr.append(a)
        wid.append(w)
        steps.append(len(ts))
    out = dict(arrival_h=arr, width_h=wid, wall_s=wall, steps=steps,
               zone_updates=info["zone_updates"] if info else 0.0, max_leaves=max_leaves)
    sim.close()
    return out


# --- command line ---------------------------------------------------------------

def _workload_parts(name, wind_seed=None, cme=None, max_level=None):
    from synthetic import Wind, as_dict, workload
    w = workload(name)
    grid = as_dict(w.grid)
    if max_level is not None:
        grid["max_level"] = max_level
    wind = as_dict(w.wind if wind_seed is None else Wind(seed=wind_seed))
    c = as_dict(w.cmes[0]) if cme is None else cme
    return grid, wind, c, as_dict(w.amr), w


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2211_12867_amd.forecast")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train", help="collect look-ahead pairs from seeded plain runs and train the network")
    t.add_argument("--out", required=True)
    t.add_argument("--runs", type=int, default=16)
    t.add_argument("--max-level", type=int, default=5)
    t.add_argument("--relax-days", type=float, default=14.0)
    t.add_argument("--cme-days", type=float, default=1.5)
    t.add_argument("--every", type=int, default=10)
    t.add_argument("--epochs", type=int, default=10)
    t.add_argument("--keep-every", type=int, default=4)
    t.add_argument("--time-budget", type=float, default=900.0,
                   help="seconds after which no further run is started (training uses what was collected)")
    c = sub.add_parser("compare", help="equidistant vs plain AMR (buffer) vs learned AMR (no buffer) to arrival")
    c.add_argument("--net", required=True)
    c.add_argument("--max-level", type=int, default=5)
    c.add_argument("--relax-days", type=float, default=14.0)
    c.add_argument("--cme-days", type=float, default=3.0)
    c.add_argument("--skip-equidistant", action="store_true")
    c.add_argument("--out")
    c.add_argument("--only", help="comma-separated subset of the AMR runs")
    f = sub.add_parser("fig1", help="low resolution, equidistant vs radially stretched: series at Earth")
    f.add_argument("--relax-days", type=float, default=14.0)
    f.add_argument("--cme-days", type=float, default=3.0)
    f.add_argument("--out")
    r = sub.add_parser("tracer", help="unrefined grids vs CME-tracer refinement vs shock refinement at Earth")
    r.add_argument("--relax-days", type=float, default=14.0)
    r.add_argument("--cme-days", type=float, default=3.0)
    r.add_argument("--max-level", type=int, default=3)
    r.add_argument("--out")
    e = sub.add_parser("ensemble", help="the 32-member cone-CME ensemble on the stretched 3-level grid")
    e.add_argument("--members", type=int, default=32)
    e.add_argument("--relax-days", type=float, default=14.0)
    e.add_argument("--cme-days", type=float, default=3.0)
    e.add_argument("--out")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if args.cmd == "train":
        from synthetic import as_dict, cme_ensemble
        Xs, Ys = [], []
        t_start = time.perf_counter()
        done = 0
        for r in range(args.runs):
            if time.perf_counter() - t_start > args.time_budget:
                log("time budget reached after %d runs" % r)
                break
            cme = as_dict(cme_ensemble(1, 2000 + r, t_start_s=args.relax_days * DAY)[0])
            grid, wind, cme, amr, _ = _workload_parts("learned_flags", wind_seed=1 + r, cme=cme,
                                                      max_level=args.max_level)
            log("run %d: wind seed %d, cme %s" % (r, 1 + r, {k: round(v, 1) for k, v in cme.items()
                                                                if isinstance(v, float)}))
            st = relax(grid, wind, cme, args.relax_days * DAY, log=log)
            amr = dict(amr, buffer_blocks=1, regrid_every=args.every)
            X, y = collect_pairs(grid, wind, cme, amr, st, (args.relax_days + args.cme_days) * DAY, args.every,
                                 log=log, keep_every=args.keep_every)
            Xs.append(X)
            Ys.append(y)
            done += 1
            log("run %d: %d pairs, %.3f positive, %.0f s" % (r, len(y), y.mean(), time.perf_counter() - t_start))
        X = np.concatenate(Xs)
        y = np.concatenate(Ys)
        del Xs, Ys
        npairs, ppos = len(y), y.mean()
        params, mean, std, loss = train(X, y, epochs=args.epochs)
        del X, y
        # held out: wind seed 0 with the evaluation CME
        grid, wind, cme, amr, _ = _workload_parts("learned_flags", max_level=args.max_level)
        cme = dict(cme, t_start_s=args.relax_days * DAY)
        st = relax(grid, wind, cme, args.relax_days * DAY, log=log)
        Xh, yh = collect_pairs(grid, wind, cme, dict(amr, buffer_blocks=1, regrid_every=args.every), st,
                               (args.relax_days + args.cme_days) * DAY, args.every, log=log,
                               keep_every=args.keep_every)
        held = evaluate(Xh, yh, (params, mean, std))
        log("held-out: %s" % json.dumps(held))
        meta = dict(pairs=int(npairs), positive=float(ppos), runs=done, held_out=held, wind_seeds=[1, done],
                    cme_seeds=[2000, 1999 + done], max_level=args.max_level, every=args.every,
                    cme_days=args.cme_days, epochs=args.epochs, loss=[float(v) for v in loss])
        save_network(args.out, params, mean, std, meta)
        log("trained: %s" % json.dumps(meta))
        return 0

    if args.cmd == "fig1":
        res = stretching_comparison(args.relax_days, args.cme_days, log=log)
        keys = ("arrival_h", "width_h", "peak_kms", "gradient_kms_h", "wall_s", "steps", "dr_1au_rsun")
        summary = {k: {q: v[q] for q in keys} for k, v in res.items()}
        log(json.dumps(summary))
        if args.out:
            np.savez(args.out, **{"%s_%s" % (k, q): res[k][q] for k in res for q in ("t_h", "v_kms")},
                     summary=np.array(json.dumps(summary)))
        return 0

    if args.cmd == "tracer":
        res = tracer_comparison(args.relax_days, args.cme_days, args.max_level, log=log)
        keys = ("arrival_h", "width_h", "peak_kms", "gradient_kms_h", "wall_s", "steps", "leaf_block_steps",
                "max_leaves", "leaves_end", "max_level")
        summary = {k: {q: v[q] for q in keys} for k, v in res.items()}
        log(json.dumps(summary))
        if args.out:
            np.savez(args.out, **{"%s_%s" % (k, q): res[k][q] for k in res for q in ("t_h", "v_kms")},
                     summary=np.array(json.dumps(summary)))
        return 0

    if args.cmd == "ensemble":
        from synthetic import as_dict, workload
        w = workload("ensemble")
        grid, wind, amr = as_dict(w.grid), as_dict(w.wind), as_dict(w.amr)
        cmes = [dict(as_dict(c), t_start_s=args.relax_days * DAY) for c in w.cmes[:args.members]]
        st = relax(grid, wind, cmes[0], args.relax_days * DAY, log=log)
        r = ensemble_run(grid, wind, cmes, dict(amr, buffer_blocks=1), st, (args.relax_days + args.cme_days) * DAY,
                         log=log)
        cells = grid["block"][0] * grid["block"][1] * grid["block"][2]
        summary = dict(members=len(cmes), wall_s=r["wall_s"], relax_wall_s=st["wall_s"],
                       zone_updates=r["zone_updates"], zone_updates_per_s=r["zone_updates"] / r["wall_s"],
                       max_leaves=r["max_leaves"], leaf_cells_peak=r["max_leaves"] * cells,
                       arrival_h=[round(x, 3) for x in r["arrival_h"]], width_h=[round(x, 3) for x in r["width_h"]],
                       steps=r["steps"],
                       cmes=[{k: round(c[k], 1) for k in ("v_kms", "half_width_deg", "colat_deg", "lon_deg", "n_cm3")}
                             for c in cmes])
        log(json.dumps(summary))
        if args.out:
            with open(args.out, "w") as fh:
                json.dump(summary, fh, indent=1)
        return 0

    net, meta = load_network(args.net)
    grid, wind, cme, amr, w = _workload_parts("learned_flags", max_level=args.max_level)
    t_end = (args.relax_days + args.cme_days) * DAY
    cme = dict(cme, t_start_s=args.relax_days * DAY)
    res = {}
    st = relax(grid, wind, cme, args.relax_days * DAY, log=log)
    lv = args.max_level
    runs = {"plain_buffer_L%d" % (lv - 1): (lv - 1, dict(amr, source=IC_SOURCE_PLAIN, buffer_blocks=1), None),
            "plain_buffer_L%d" % lv: (lv, dict(amr, source=IC_SOURCE_PLAIN, buffer_blocks=1), None),
            "learned_L%d" % lv: (lv, dict(amr, source=IC_SOURCE_LEARNED_JUDGED, buffer_blocks=0,
                                          learned_threshold=meta.get("threshold", 0.5)), net),
            "plain_no_buffer_L%d" % lv: (lv, dict(amr, source=IC_SOURCE_PLAIN, buffer_blocks=0), None)}
    for name, (level, a, n) in runs.items():
        if args.only and name not in args.only.split(","):
            continue
        log("== %s" % name)
        r = cme_run(dict(grid, max_level=level), wind, cme, a, st, t_end, network=n, log=log)
        r["relax_wall_s"] = st["wall_s"]
        res[name] = r
    if not args.skip_equidistant:
        g1, w1, c1, _, _ = _workload_parts("equidistant_full")
        c1 = dict(c1, t_start_s=args.relax_days * DAY)
        log("== equidistant")
        res["equidistant"] = cme_run(g1, w1, c1, dict(regrid_every=0), None, t_end, log=log, chunk_s=DAY)
    summary = {k: {q: v[q] for q in ("arrival_h", "width_h", "wall_s", "cme_wall_s", "steps", "leaf_block_steps",
                                     "max_leaves", "regrid_stats")} for k, v in res.items()}
    log(json.dumps(summary))
    if args.out:
        np.savez(args.out, **{"%s_%s" % (k, q): res[k][q] for k in res for q in ("t_h", "v_kms")},
                 summary=np.array(json.dumps(summary)))
    return 0


if __name__ == "__main__":
    sys.exit(main())
