"""The CME density tracer and the tracer / combined refinement criteria
through the C ABI against the oracle (paper Sect. 3.1: a density tracer
injected with the CME, the grid refined where it is present; Sect. 3.3: the
tracer condition combined with the shock criterion inside the windows).

- Passivity: on a refined periodic box (ghost restriction and prolongation,
  reflux) the eight MHD variables of a tracer run are bit-identical with
  those of a run without it.
- With s = 1 everywhere rho s stays equal to rho bit for bit on the GPU too
  (the same flux form, maximum speed, reflux and ghost operators).
- Parity of all nine variables with the oracle on the refined box and on the
  cone-CME wedge (both time schemes, each limiter), where the inner boundary
  brings s = 1 inside the cone and s = 0 in the wind.
- Criterion parity: block flags bit-exact with the oracle's on identical
  states, then the regridded forest and the moved state, over several cycles
  of a refined wedge with the tracer and the combined criteria.
Bars as for the MHD variables: <= 1e-12 per step, <= 1e-10 over 20 steps."""
import math

import numpy as np
import pytest

from gpu_helpers import rel_err, tiny_wedge
from oracle import boundary, forest as fo, solver, units
from synthetic import Cme, Wind, as_dict, smooth_modes

pytestmark = pytest.mark.gpu

GAMMA = 1.5


def _ic():
    import paper_2211_12867_amd as ic
    return ic


def _box():
    return dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 1.0, 0.5), n=(16, 16, 8), block=(8, 8, 8),
                periodic=(True, True, True), max_level=2, gamma=GAMMA, cfl=0.4)


def _smooth_state(s, seed, unit_fraction=False):
    for leaf in s.forest.leaves:
        x = [s.centres(leaf, d) for d in range(3)]
        Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        W = np.zeros((9,) + X.shape)
        base = [1.0, 0.3, -0.2, 0.1, 1.0, 0.3, 0.2, -0.1, 0.5]
        for v in range(9):
            ks, amps, ph = smooth_modes(seed + v, 3, 0.15 if v in (0, 4) else 0.25)
            f = np.zeros_like(X)
            for kk, a, p in zip(ks, amps, ph):
                f += a * np.sin(2 * math.pi * (kk[0] * X + kk[1] * Y + kk[2] * Z / 0.5) + p)
            W[v] = base[v] + f
        if unit_fraction:
            W[8] = 1.0
        s.U[leaf] = boundary.prims_to_cons(W, GAMMA)


def _refined_box(seed, unit_fraction=False):
    ora = solver.Solver(_box(), initial="zero", tracer=True, amr=dict(buffer_blocks=0))
    _smooth_state(ora, seed, unit_fraction)
    ora.regrid({b: (fo.REFINE if b in {(1, 0, 0, 0), (1, 1, 1, 0)} else fo.KEEP) for b in ora.forest.leaves},
               buffer_blocks=0)
    assert max(b[0] for b in ora.blocks()) == 2
    return ora


def test_tracer_is_passive_on_a_refined_box():
    ic = _ic()
    ora = _refined_box(700)
    bl, U = ora.state()
    g9 = ic.Sim(_box(), amr=dict(buffer_blocks=0), tracer=True)
    g8 = ic.Sim(_box(), amr=dict(buffer_blocks=0))
    g9.set_state(bl, U, 0.0)
    g8.set_state(bl, U[:, :8].copy(), 0.0)
    for n in range(10):
        i9, i8 = g9.step(), g8.step()
        assert i9["dt_s"] == i8["dt_s"]
        ora.step()
        U9 = g9.state()[1]
        assert np.array_equal(U9[:, :8], g8.state()[1]), n
        e = rel_err(U9, ora.state()[1])
        assert e <= 1e-12 * (n + 1), (n, e)
    s = U9[:, 8] / U9[:, 0]
    assert s.min() > -0.5 and s.max() > 0.5       # the tracer moved, not flattened


def test_unit_fraction_tracer_is_the_density_on_the_gpu():
    ic = _ic()
    ora = _refined_box(710, unit_fraction=True)
    gpu = ic.Sim(_box(), amr=dict(buffer_blocks=0), tracer=True)
    gpu.set_state(*ora.state(), 0.0)
    for n in range(10):
        gpu.step()
        U = gpu.state()[1]
        assert np.array_equal(U[:, 8], U[:, 0]), n
    assert gpu.floor_counts() == (0, 0)


@pytest.mark.parametrize("sch,cd,lim", [("two_stage", 0.0, "mc"), ("hancock", 0.0, "mc"), ("two_stage", 0.3, "mc"),
                                        ("two_stage", 0.0, "minmod"), ("hancock", 0.0, "vanleer")])
def test_cme_wedge_tracer_parity(sch, cd, lim):
    """Both time schemes, the parabolic cleaning and the other limiters beside
    the tracer."""
    ic = _ic()
    g, wind, cme, amr = tiny_wedge()
    ora = solver.Solver(g, wind, cme, amr, tracer=True, scheme=sch, divb_cd=cd, limiter=lim)
    gpu = ic.Sim(g, wind, [cme], amr, tracer=True, scheme=sch, divb_cd=cd, limiter=lim)
    bl, U = gpu.state()
    assert U.shape[1] == 9 and np.all(U[:, 8] == 0.0)     # no CME material initially
    gpu.set_state(*ora.state(), 0.0)
    for n in range(20):
        info = gpu.step()
        dt = ora.step()
        assert abs(info["dt_s"] / units.T0 - dt) <= 1e-12 * dt
        if n == 0:
            assert rel_err(gpu.state()[1], ora.state()[1]) <= 1e-12
    U = gpu.state()[1]
    e = rel_err(U, ora.state()[1])
    assert e <= 1e-10, e
    s = U[:, 8] / U[:, 0]
    # CME material entered the domain; the limited scheme undershoots s = 0 by
    # a few 1e-8 at the edge of the material (the oracle likewise: parity above)
    assert s.max() > 0.5 and s.min() >= -1e-6


def _wedge(crit):
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=(32, 16, 16),
                block=(8, 8, 8), stretched_r=True, max_level=3, periodic=(False, False, False), gamma=1.5, cfl=0.4)
    wind = as_dict(Wind(seed=3))
    cme = as_dict(Cme(t_start_s=0.0, duration_s=6 * 3600.0, v_kms=1400.0, half_width_deg=35.0,
                      colat_deg=90.0, lon_deg=20.0, n_cm3=1500.0, T_K=0.8e6))
    amr = dict(eps_lohner=0.01, tol_refine=0.1, tol_coarsen=0.0125, w_rho=0.5, w_v=0.5,
               lon_earth_deg=0.0, clt_earth_deg=90.0, dlon_earth_deg=60.0, dclt_earth_deg=30.0,
               dlon_cme_deg=90.0, use_windows=True, regrid_every=5, buffer_blocks=1,
               criterion=crit, tracer_refine=0.01, tracer_coarsen=0.00125)
    return grid, wind, cme, amr


@pytest.mark.parametrize("crit", ["tracer", "combined"])
def test_tracer_criteria_flags_forest_and_state(crit):
    """Three cycles of steps, flags on identical states (bit-exact: the
    tracer condition compares the correctly rounded (rho s) / rho on both
    sides) and regrids."""
    ic = _ic()
    grid, wind, cme, amr = _wedge(crit)
    ora = solver.Solver(grid, wind, cme, amr, tracer=True)
    gpu = ic.Sim(grid, wind, [cme], amr, tracer=True)
    gpu.set_state(*ora.state(), 0.0)
    refined = 0
    for cycle in range(3):
        for _ in range(5):
            ora.step()
            gpu.step()
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-10, (cycle, e)
        gpu.set_state(*ora.state(), ora.t * units.T0)
        ties = []
        f = ora.flags(ties)
        assert not ties, "near-tie in the indicator: %r" % ties[:3]
        assert [int(x) for x in gpu.eval_flags()] == [f[b] for b in ora.blocks()]
        refined += sum(v == fo.REFINE for v in f.values())
        ora.regrid(f)
        gpu.regrid()
        assert gpu.blocks() == ora.blocks()
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-13, (cycle, e)
    assert refined > 0 and max(b[0] for b in ora.blocks()) >= 2


def test_resolving_the_cme_material_leaves_the_arrival():
    """Sect. 3.1: resolving the CME plasma does not move the shock arrival.
    On the stretched workload (shortened relaxation), tracer refinement to
    three levels also resolves the shock -- a 12^3 block holding CME material
    spans the sheath -- and arrives with shock refinement to three levels,
    which resolves the shock alone, at several times the leaf-block-steps.
    The tracer runs reach their top level; the three-level one coarsens
    behind the CME faster than it refines ahead of it by the end (its leaf
    count falls from its peak)."""
    from paper_2211_12867_amd import forecast
    res = forecast.tracer_comparison(relax_days=2.0, cme_days=2.5, max_level=3, log=None)
    for name, r in res.items():
        assert not math.isnan(r["arrival_h"]) and r["width_h"] > 0.0, (name, r["arrival_h"])
    tr, sh = res["tracer_L3"], res["shock_L3"]
    assert abs(tr["arrival_h"] - sh["arrival_h"]) < 0.25, (tr["arrival_h"], sh["arrival_h"])
    assert tr["leaf_block_steps"] > 3.0 * sh["leaf_block_steps"]
    assert res["tracer_L2"]["max_level"] == 2 and tr["max_level"] == 3
    assert tr["leaves_end"] < tr["max_leaves"], (tr["leaves_end"], tr["max_leaves"])
    # the unrefined base grid smears the shock the most
    assert res["base"]["width_h"] > 2.0 * max(tr["width_h"], res["uniform_x2"]["width_h"])
