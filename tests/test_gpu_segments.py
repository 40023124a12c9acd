"""GPU parity segments through the C ABI against the oracle (paper Sect. 2.1,
3; the parity contract: <= 1e-12 per step, <= 1e-9 over a segment, flags and
forests bit-exact):

- 12^3 blocks (the block shape of the stretched-grid AMR runs) on a stretched
  wedge with three levels, plain flags and regrids, the stage kernel split
  four ways along phi: every step from identical inputs, flags, forests and
  the data movement of every regrid;
- the full 512 x 60 x 180 equidistant grid in the benchmark's launch
  configuration: 10 CFL steps from the initial state, each from identical
  inputs and as one segment, and 10 steps after the CME start (inner
  boundary with the cone CME open) from a state the GPU evolved and handed
  to the oracle;
- the density floor acting (the zero-velocity branch) with equal floor
  counts; a step whose second stage makes a non-physical state fails at once;
- advancing in pieces regrids after the same steps as one advance;
- the shock diagnostics of a recorded series against the oracle's.
"""
import os
import math
import shutil
import tempfile

import numpy as np
import pytest

from gpu_helpers import rel_err
from oracle import analysis, boundary, solver, units
from synthetic import Cme, Wind, as_dict, workload

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ic():
    import paper_2211_12867_amd as ic
    return ic


def _wedge12():
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=(48, 24, 24),
                block=(12, 12, 12), stretched_r=True, max_level=3, periodic=(False, False, False),
                gamma=1.5, cfl=0.4)
    wind = as_dict(Wind(seed=3))
    cme = as_dict(Cme(t_start_s=0.0, duration_s=6 * 3600.0, v_kms=1400.0, half_width_deg=35.0,
                      colat_deg=90.0, lon_deg=20.0, n_cm3=1500.0, T_K=0.8e6))
    amr = dict(eps_lohner=0.01, tol_refine=0.1, tol_coarsen=0.0125, w_rho=0.5, w_v=0.5,
               lon_earth_deg=0.0, clt_earth_deg=90.0, dlon_earth_deg=60.0, dclt_earth_deg=30.0,
               dlon_cme_deg=90.0, use_windows=True, regrid_every=4, buffer_blocks=1)
    return grid, wind, cme, amr


def test_amr_12cubed_three_levels_each_step_ksplit4():
    ic = _ic()
    grid, wind, cme, amr = _wedge12()
    ora = solver.Solver(grid, wind, cme, amr)
    gpu = ic.Sim(grid, wind, [cme], amr)
    gpu.set_tuning(waves_per_simd=2, grid=0, xcd_order=0, ksplit=4)
    gpu.set_state(*ora.state(), 0.0)
    worst = 0.0
    levels = set()
    for cycle in range(4):
        for _ in range(4):
            gpu.set_state(*ora.state(), ora.t * units.T0)     # identical inputs
            info = gpu.step()
            dt = ora.step()
            assert abs(info["dt_s"] / units.T0 - dt) <= 1e-13 * dt
            e = rel_err(gpu.state()[1], ora.state()[1])
            worst = max(worst, e)
            assert e <= 1e-12, (cycle, e)
        assert gpu.tuning()[3] == 4
        gpu.set_state(*ora.state(), ora.t * units.T0)
        ties = []
        f = ora.flags(ties)
        assert not ties, ties[:3]
        assert [int(x) for x in gpu.eval_flags()] == [f[b] for b in ora.blocks()]
        ora.regrid(f)
        gpu.regrid()
        assert gpu.blocks() == ora.blocks()
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-13, (cycle, e)
        levels |= {b[0] for b in ora.blocks()}
    assert levels == {1, 2, 3}, levels
    # coarse-fine faces were present (slabs, reflux)
    assert len(ora.blocks()) > 16
    gpu.close()


# --- the full equidistant grid ------------------------------------------------------

def _full(cme_start_s=None):
    w = workload("equidistant_full")
    g, wind, cme = as_dict(w.grid), as_dict(w.wind), as_dict(w.cmes[0])
    if cme_start_s is not None:
        cme = dict(cme, t_start_s=cme_start_s)
    return g, wind, cme


def _bench_schedule(gpu):
    cache = os.path.join(ROOT, "paper_2211_12867_amd", "tune_cache.txt")
    with tempfile.TemporaryDirectory() as d:
        tmp = os.path.join(d, "tune.txt")
        if os.path.exists(cache):
            shutil.copy(cache, tmp)
        gpu.autotune(tmp, reps=2)


def _patch_from_blocks(ora, bl, U, block):
    P = np.empty_like(ora.U)
    for b, u in zip(bl, U):
        assert b[0] == 1
        P[:, b[3] * block[2]:(b[3] + 1) * block[2], b[2] * block[1]:(b[2] + 1) * block[1],
          b[1] * block[0]:(b[1] + 1) * block[0]] = u
    return P


def _segment(ic, g, wind, cme, ora, gpu, steps=10):
    """steps CFL steps: per step from identical inputs (<= 1e-12), and the
    GPU's own segment against the oracle's (<= 1e-9)."""
    bl0, U0 = ora.to_blocks(g["block"])
    t0 = ora.t
    states, times = [], []
    for _ in range(steps):
        ora.step()
        states.append(ora.to_blocks(g["block"])[1].copy())
        times.append(ora.t)
    # the GPU's own segment from the same start
    gpu.set_state(bl0, U0, t0 * units.T0)
    for n in range(steps):
        gpu.step()
    e_seg = rel_err(gpu.state()[1], states[-1])
    t_gpu, _ = gpu.time()
    assert abs(t_gpu / units.T0 - times[-1]) <= 1e-12 * times[-1]
    # each step from identical inputs
    worst = 0.0
    prev, tprev = U0, t0
    for n in range(steps):
        gpu.set_state(bl0, prev, tprev * units.T0)
        info = gpu.step()
        assert abs(info["t_s"] / units.T0 - times[n]) <= 1e-13 * times[n]
        e = rel_err(gpu.state()[1], states[n])
        worst = max(worst, e)
        assert e <= 1e-12, (n, e)
        prev, tprev = states[n], times[n]
    assert e_seg <= 1e-9, e_seg
    return worst, e_seg


def test_equidistant_full_cfl_segment_from_the_initial_state():
    ic = _ic()
    g, wind, cme = _full()
    gpu = ic.Sim(g, wind, [cme])
    _bench_schedule(gpu)
    ora = solver.PatchSolver(g, wind, cme)
    bl, U = gpu.state()
    bo, Uo = ora.to_blocks(g["block"])
    assert bl == bo and rel_err(U, Uo) <= 1e-14      # the same initial condition up to rounding
    _segment(ic, g, wind, cme, ora, gpu)
    gpu.close()


def test_equidistant_full_segment_after_the_cme_start():
    """The GPU relaxes to one hour after the CME start (the cone open at the
    inner boundary); its state goes to the oracle; then 10 steps on both."""
    ic = _ic()
    t_cme = 6 * 3600.0
    g, wind, cme = _full(t_cme)
    gpu = ic.Sim(g, wind, [cme])
    _bench_schedule(gpu)
    gpu.advance(t_cme + 3600.0)
    t_s, _ = gpu.time()
    assert abs(t_s - (t_cme + 3600.0)) <= 1e-6
    bl, U = gpu.state()
    ora = solver.PatchSolver(g, wind, cme)
    ora.U = _patch_from_blocks(ora, bl, U, g["block"])
    ora.t = t_s / units.T0
    # the cone is open: inner-boundary cells inside the CME mask
    th = np.array([ora.geo.centre(1, j) for j in range(ora.n[1])])[:, None]
    ph = np.array([ora.geo.centre(2, k) for k in range(ora.n[2])])[None, :]
    mask = boundary.cme_mask(cme, th + 0 * ph, ph + 0 * th, ora.r_in, ora.t)
    assert mask.sum() > 50
    _segment(ic, g, wind, cme, ora, gpu)
    gpu.close()


# --- floors and non-physical results ------------------------------------------------

def _box_state(s, v_amp, p0, width):
    for leaf in s.forest.leaves:
        x = s.centres(leaf, 0)[None, None, :]
        y = s.centres(leaf, 1)[None, :, None]
        z = s.centres(leaf, 2)[:, None, None]
        W = np.zeros((8,) + np.broadcast(x, y, z).shape)
        W[0] = 1.0 + 0.1 * np.sin(2 * math.pi * y / 0.5) * np.cos(2 * math.pi * z / 0.5)
        W[1] = v_amp * np.tanh((x - 0.5) / width) * (1 + 0 * y * z)
        W[2] = 0.1 * np.sin(2 * math.pi * x) + 0 * y * z
        W[4] = p0 + 0 * x * y * z
        W[5] = 0.05
        W[7] = 0.05 * np.cos(2 * math.pi * x) + 0 * y * z
        s.U[leaf] = boundary.prims_to_cons(W, 1.5)


def _box():
    return dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 0.5, 0.5), n=(32, 8, 8), block=(8, 8, 8),
                periodic=(True, True, True), max_level=1, gamma=1.5, cfl=0.4)


def test_density_floor_branch_matches_the_oracle():
    """A rarefaction between two receding streams drains the middle of a
    periodic box below the density floor: floored cells take the floor at
    zero velocity.  The floor acts in the last steps; states match the
    oracle every step and the floor counts agree."""
    ic = _ic()
    g = _box()
    ora = solver.Solver(g, initial="zero", rho_floor=0.45, p_floor=1e-5)
    _box_state(ora, 1.5, 0.5, 0.08)
    gpu = ic.Sim(g, rho_floor=0.45, p_floor=1e-5)
    gpu.set_state(*ora.state(), 0.0)
    for n in range(20):
        gpu.step()
        ora.step()
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-12 * (n + 1), (n, e)
    rho, p = gpu.floor_counts()
    assert ora.floor_counts[0] > 0, "the density floor never acted"
    assert (rho, p) == tuple(ora.floor_counts), ((rho, p), ora.floor_counts)
    gpu.close()


def test_nonphysical_second_stage_fails_the_step():
    """Floors off, a cold strong rarefaction and a fixed dt for which the
    first stage stays physical but the step's result has p < 0 (both checked
    on the oracle): the step itself returns IC_E_UNPHYSICAL."""
    ic = _ic()
    g = _box()
    ora = solver.Solver(g, initial="zero", rho_floor=0.0, p_floor=0.0)
    _box_state(ora, 2.0, 0.02, 0.03)
    for leaf in ora.forest.leaves:          # no transverse velocity, no B_z wave
        W = boundary.cons_to_prims(ora.U[leaf], 1.5)
        W[2] = 0.0
        W[7] = 0.0
        ora.U[leaf] = boundary.prims_to_cons(W, 1.5)
    bl, U0 = ora.state()
    dt = 0.8 * ora.cfl_dt()
    L1, _ = ora.operator(ora.U, 0.0)
    Us = {b: ora.U[b] + 0.5 * dt * L1[b] for b in ora.U}
    p_star = min(boundary.cons_to_prims(u.reshape(8, -1), 1.5)[4].min() for u in Us.values())
    L2, _ = ora.operator(Us, 0.5 * dt)
    U1 = {b: ora.U[b] + dt * L2[b] for b in ora.U}
    p_one = min(boundary.cons_to_prims(u.reshape(8, -1), 1.5)[4].min() for u in U1.values())
    assert p_star > 1e-4 and p_one < -1e-5, (p_star, p_one)
    gpu = ic.Sim(g, rho_floor=0.0, p_floor=0.0)
    gpu.set_state(bl, U0, 0.0)
    with pytest.raises(ic.ICError) as ex:
        gpu.step(dt * units.T0)
    assert ex.value.status == ic.IC_E_UNPHYSICAL
    gpu.close()


# --- regrid cadence across calls ------------------------------------------------------

def test_advance_in_pieces_regrids_like_one_advance():
    ic = _ic()
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=(32, 16, 16),
                block=(8, 8, 8), stretched_r=True, max_level=3, periodic=(False, False, False),
                gamma=1.5, cfl=0.4)
    _, wind, cme, amr = _wedge12()
    runs = []
    for split in ((30,), (13, 17), (4, 3, 23)):
        s = ic.Sim(grid, wind, [cme], amr)
        for k in split:
            s.advance(1e9, max_steps=k)
        runs.append((s.blocks(), s.state()[1], s.time(), s.regrid_stats()))
        s.close()
    for r in runs[1:]:
        assert r[0] == runs[0][0]
        assert np.array_equal(r[1], runs[0][1])
        assert r[2] == runs[0][2]
    assert max(b[0] for b in runs[0][0]) >= 2


# --- shock diagnostics of a recorded series ---------------------------------------------

def test_shock_diagnostics_of_a_recorded_series():
    ic = _ic()
    w = workload("tiny_wedge")
    g, wind, cme, amr = as_dict(w.grid), as_dict(w.wind), as_dict(w.cmes[0]), as_dict(w.amr)
    ora = solver.Solver(g, wind, cme, amr)
    gpu = ic.Sim(g, wind, [cme], amr)
    gpu.set_state(*ora.state(), 0.0)
    point = (0.3, 90.0, 45.0)
    gpu.set_sample_point(*point)
    gpu.timeseries_clear()
    ser = []
    for _ in range(120):
        ora.step()
        ser.append([ora.t * units.T0] + list(ora.sample(*point)))
    ser = np.array(ser)
    gpu.advance(1e9, max_steps=120)
    ts = gpu.timeseries()
    assert ts.shape == ser.shape
    assert np.allclose(ts[:, 0], ser[:, 0], rtol=1e-12)
    assert np.allclose(ts[:, 1:], ser[:, 1:], rtol=1e-9, atol=1e-12 * np.abs(ser[:, 1:]).max())
    v_kms = lambda a: a[:, 2] * units.V0 / 1e3
    ref = analysis.diagnostics(ser[:, 0] / 3600.0, v_kms(ser), 0.0, 96.0, 100.0)
    got = ic.shock_diagnostics(ts[:, 0], v_kms(ts), 0.0, 96 * 3600.0, 100.0)
    assert not math.isnan(ref["arrival"]) and ref["width"] > 0.0
    assert abs(got["arrival_s"] / 3600.0 - ref["arrival"]) <= 1e-6
    assert abs(got["width_s"] / 3600.0 - ref["width"]) <= 1e-6
    assert abs(got["v_max"] - ref["v_max"]) <= 1e-6 * ref["v_max"]
    assert abs(got["gradient"] * 3600.0 - ref["gradient"]) <= 1e-5 * abs(ref["gradient"])
    gpu.close()
