"""Scheme variants through the C ABI against the oracle (paper Sect. 2.1: the
code offers scheme and limiter combinations beyond the TVDLF + Woodward
runs): minmod and van Leer limiters in the stage kernel, and the Hancock
one-step form (k_hancock predictor, then the stage kernel as corrector), on
the cone-CME wedge, a refined periodic box (reflux in the corrector) and a
stretched three-level wedge with regrids.  Bars: <= 1e-12 per step, <= 1e-10
over 20 steps, forests bit-exact."""
import numpy as np
import pytest

from gpu_helpers import rel_err, tiny_wedge
from oracle import forest as fo, solver, units
from synthetic import Cme, Wind, as_dict

pytestmark = pytest.mark.gpu

VARIANTS = [(lim, sch) for lim in ("mc", "minmod", "vanleer") for sch in ("two_stage", "hancock")]


def _ic():
    import paper_2211_12867_amd as ic
    return ic


@pytest.mark.parametrize("lim,sch", VARIANTS)
def test_wedge_each_variant(lim, sch):
    ic = _ic()
    g, wind, cme, amr = tiny_wedge()
    ora = solver.Solver(g, wind, cme, amr, limiter=lim, scheme=sch)
    gpu = ic.Sim(g, wind, [cme], amr, limiter=lim, scheme=sch)
    gpu.set_state(*ora.state(), 0.0)
    for n in range(20):
        info = gpu.step()
        dt = ora.step()
        assert abs(info["dt_s"] / units.T0 - dt) <= 1e-12 * dt
        e = rel_err(gpu.state()[1], ora.state()[1])
        if n == 0:
            assert e <= 1e-12, e
    assert e <= 1e-10, e
    gpu.close()


@pytest.mark.parametrize("lim", ["mc", "vanleer"])
def test_hancock_refined_periodic_box(lim):
    import math
    ic = _ic()
    g = dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 1.0, 0.5), n=(16, 16, 8), block=(8, 8, 8),
             periodic=(True, True, True), max_level=2, gamma=1.5, cfl=0.4)
    ora = solver.Solver(g, initial="zero", limiter=lim, scheme="hancock")
    from synthetic import smooth_modes
    from oracle import boundary
    for leaf in ora.forest.leaves:
        x = [ora.centres(leaf, d) for d in range(3)]
        Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
        W = np.zeros((8,) + X.shape)
        base = [1.0, 0.1, -0.1, 0.05, 1.0, 0.3, 0.2, -0.1]
        for v in range(8):
            ks, amps, ph = smooth_modes(300 + v, 3, 0.2)
            f = np.zeros_like(X)
            for kk, a, p in zip(ks, amps, ph):
                f += a * np.sin(2 * math.pi * (kk[0] * X + kk[1] * Y + kk[2] * Z / 0.5) + p)
            W[v] = base[v] + f
        ora.U[leaf] = boundary.prims_to_cons(W, 1.5)
    ora.regrid({b: (fo.REFINE if b in {(1, 0, 0, 0), (1, 1, 1, 0)} else fo.KEEP) for b in ora.forest.leaves},
               buffer_blocks=0)
    gpu = ic.Sim(g, amr=dict(buffer_blocks=0), limiter=lim, scheme="hancock")
    gpu.set_state(*ora.state(), 0.0)
    assert gpu.blocks() == ora.blocks()
    tot0 = ora.total()
    for n in range(5):
        ora.step(1e-3)
        gpu.step(1e-3 * units.T0)
        e = rel_err(gpu.state()[1], ora.state()[1])
        assert e <= 1e-12 * (n + 1), (n, e)
    # the corrector's reflux keeps the total
    assert np.all(np.abs(ora.total() - tot0) <= 1e-12 * np.abs(tot0).max())
    gpu.close()


def test_hancock_stretched_amr_wedge_with_regrids():
    ic = _ic()
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=(32, 16, 16),
                block=(8, 8, 8), stretched_r=True, max_level=3, periodic=(False, False, False),
                gamma=1.5, cfl=0.4)
    wind = as_dict(Wind(seed=3))
    cme = as_dict(Cme(t_start_s=0.0, duration_s=6 * 3600.0, v_kms=1400.0, half_width_deg=35.0,
                      colat_deg=90.0, lon_deg=20.0, n_cm3=1500.0, T_K=0.8e6))
    amr = dict(eps_lohner=0.01, tol_refine=0.1, tol_coarsen=0.0125, w_rho=0.5, w_v=0.5,
               lon_earth_deg=0.0, clt_earth_deg=90.0, dlon_earth_deg=60.0, dclt_earth_deg=30.0,
               dlon_cme_deg=90.0, use_windows=True, regrid_every=5, buffer_blocks=1)
    ora = solver.Solver(grid, wind, cme, amr, limiter="minmod", scheme="hancock")
    gpu = ic.Sim(grid, wind, [cme], amr, limiter="minmod", scheme="hancock")
    gpu.set_state(*ora.state(), 0.0)
    for cycle in range(3):
        for _ in range(5):
            gpu.set_state(*ora.state(), ora.t * units.T0)
            gpu.step()
            ora.step()
            e = rel_err(gpu.state()[1], ora.state()[1])
            assert e <= 1e-12, (cycle, e)
        ties = []
        f = ora.flags(ties)
        assert not ties
        assert [int(x) for x in gpu.eval_flags()] == [f[b] for b in ora.blocks()]
        ora.regrid(f)
        gpu.regrid()
        assert gpu.blocks() == ora.blocks()
    assert max(b[0] for b in ora.blocks()) >= 2
    gpu.close()


def test_unknown_scheme_rejected(monkeypatch):
    """The library refuses limiter and scheme codes it does not have."""
    ic = _ic()
    g, wind, cme, amr = tiny_wedge()
    monkeypatch.setitem(ic.LIMITERS, "bogus", 7)
    monkeypatch.setitem(ic.SCHEMES, "bogus", 9)
    for kw in (dict(limiter="bogus"), dict(scheme="bogus")):
        with pytest.raises(ic.ICError) as ex:
            ic.Sim(g, wind, [cme], amr, **kw)
        assert ex.value.status == ic.IC_E_INVALID
