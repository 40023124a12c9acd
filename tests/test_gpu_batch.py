"""Batched members and the graph-replayed advance loop, through the C ABI.

- Every member of a batched ensemble (one launch per kernel over all members'
  leaves, per-member dt, per-member regrid) equals the run of that member
  alone, bit for bit.
- A batch of members against one oracle run per member: forests and states.
- ic_advance with regrids every few steps (the captured step graph replayed
  across forest changes) matches the oracle doing the same, including the
  time series recorded at the sample point after every step.
- K calls of ic_step and one ic_advance of K steps agree bit for bit, and an
  advance that ends at its end time leaves no end time for later steps.
"""
import numpy as np
import pytest

from gpu_helpers import rel_err
from oracle import solver, units
from synthetic import Cme, Wind, as_dict, cme_ensemble

pytestmark = pytest.mark.gpu


def _grid(max_level=2):
    return dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=(32, 16, 16),
                block=(8, 8, 8), stretched_r=True, max_level=max_level, periodic=(False, False, False),
                gamma=1.5, cfl=0.4)


def _amr(every=3):
    return dict(eps_lohner=0.01, tol_refine=0.1, tol_coarsen=0.0125, w_rho=0.5, w_v=0.5,
                lon_earth_deg=20.0, clt_earth_deg=90.0, dlon_earth_deg=60.0, dclt_earth_deg=30.0,
                dlon_cme_deg=90.0, use_windows=True, regrid_every=every, buffer_blocks=1)


def test_ensemble_members_equal_standalone_runs():
    import paper_2211_12867_amd as ic
    wind = as_dict(Wind(seed=5))
    cmes = [as_dict(c) for c in cme_ensemble(4, 1000, t_start_s=0.0)]
    for c in cmes:
        c["lon_deg"] = (c["lon_deg"] + 30.0) % 360.0      # aim into the wedge
        c["duration_s"] = 6 * 3600.0
    g, amr = _grid(), _amr(3)
    batch = ic.Sim(g, wind, cmes, amr)
    batch.advance(1e9, max_steps=9)
    for m, c in enumerate(cmes):
        one = ic.Sim(g, wind, [c], amr)
        one.advance(1e9, max_steps=9)
        assert batch.blocks(m) == one.blocks(0)
        bl, U = batch.state(m)
        _, U1 = one.state(0)
        assert np.array_equal(U, U1), m
        assert batch.time(m) == one.time(0)
        one.close()
    assert len({len(batch.blocks(m)) for m in range(4)}) >= 1
    batch.close()


def test_advance_with_regrids_matches_oracle():
    import paper_2211_12867_amd as ic
    wind = as_dict(Wind(seed=3))
    cme = as_dict(Cme(t_start_s=0.0, duration_s=6 * 3600.0, v_kms=1400.0, half_width_deg=35.0,
                      colat_deg=90.0, lon_deg=20.0, n_cm3=1500.0, T_K=0.8e6))
    g, amr = _grid(3), _amr(4)
    ora = solver.Solver(g, wind, cme, amr)
    gpu = ic.Sim(g, wind, [cme], amr)
    gpu.set_state(*ora.state(), 0.0)
    point = (0.45, 92.0, 21.0)
    gpu.set_sample_point(*point)
    gpu.timeseries_clear()
    series = []
    for cycle in range(3):
        for _ in range(4):
            ora.step()
            series.append([ora.t * units.T0] + list(ora.sample(*point)))
        ties = []
        f = ora.flags(ties)
        assert not ties
        ora.regrid(f)
    gpu.advance(1e9, max_steps=12)
    assert gpu.blocks() == ora.blocks()
    e = rel_err(gpu.state()[1], ora.state()[1])
    assert e <= 1e-10, e
    ts = gpu.timeseries()
    assert ts.shape == (12, 9)
    ref = np.array(series)
    assert np.allclose(ts[:, 0], ref[:, 0], rtol=1e-12)
    assert np.allclose(ts[:, 1:], ref[:, 1:], rtol=1e-9, atol=1e-12 * np.abs(ref[:, 1:]).max())
    gpu.close()


def _batch_cmes(n):
    cmes = [as_dict(c) for c in cme_ensemble(n, 1000, t_start_s=0.0)]
    for c in cmes:
        c["lon_deg"] = (c["lon_deg"] + 30.0) % 360.0      # aim into the wedge
        c["duration_s"] = 6 * 3600.0
    return cmes


def test_batch_members_match_the_oracle():
    """A batch of three members (different cone CMEs, uneven forests, each
    its own dt and regrids, one launch per kernel over all their leaves)
    against one oracle run per member: forests equal and states within the
    multi-step bar after three regrid cycles."""
    import paper_2211_12867_amd as ic
    wind = as_dict(Wind(seed=5))
    cmes = _batch_cmes(3)
    g, amr = _grid(3), _amr(4)
    oras = [solver.Solver(g, wind, c, amr) for c in cmes]
    for cycle in range(3):
        for ora in oras:
            for _ in range(4):
                ora.step()
            ties = []
            f = ora.flags(ties)
            assert not ties, ties[:3]
            ora.regrid(f)
    gpu = ic.Sim(g, wind, cmes, amr)
    gpu.advance(1e9, max_steps=12)
    sizes = set()
    for m, ora in enumerate(oras):
        assert gpu.blocks(m) == ora.blocks(), m
        sizes.add(len(ora.blocks()))
        e = rel_err(gpu.state(m)[1], ora.state()[1])
        assert e <= 1e-10, (m, e)
        t, _ = gpu.time(m)
        assert abs(t / units.T0 - ora.t) <= 1e-12 * ora.t, m
    assert len(sizes) > 1 and max(max(b[0] for b in o.blocks()) for o in oras) >= 2   # uneven, refined
    gpu.close()


def test_step_and_advance_agree_and_end_times_do_not_leak():
    """K single steps and one advance of K steps give the same state, time and
    step count; an advance that stops at its end time leaves no end time
    behind (the next single step takes a full CFL step)."""
    import paper_2211_12867_amd as ic
    wind = as_dict(Wind(seed=7))
    cme = as_dict(Cme(t_start_s=0.0, duration_s=6 * 3600.0, v_kms=1200.0, half_width_deg=30.0,
                      colat_deg=90.0, lon_deg=20.0, n_cm3=1200.0, T_K=0.8e6))
    g = _grid(1)
    a = ic.Sim(g, wind, [cme])
    b = ic.Sim(g, wind, [cme])
    infos = [a.step() for _ in range(6)]
    ib = b.advance(1e12, max_steps=6)
    assert [i["steps"] for i in infos] == list(range(1, 7))
    assert ib["steps"] == 6 and ib["t_s"] == infos[-1]["t_s"]
    assert a.time() == b.time()
    assert np.array_equal(a.state()[1], b.state()[1])
    # an advance to a time inside the next step clips that step to the end time
    t0 = b.time()[0]
    dt_full = infos[-1]["dt_s"]
    ic2 = b.advance(0.25 * dt_full)
    assert ic2["t_s"] == pytest.approx(t0 + 0.25 * dt_full, rel=1e-12)
    # the next single step is a full CFL step again, not held at the old end time
    i3 = b.step()
    assert i3["t_s"] > ic2["t_s"] + 0.5 * dt_full
    a.close()
    b.close()
