"""The stage-kernel schedule and its autotuner, through the C ABI.

- every schedule (waves per SIMD 1 or 2, one work-group per leaf or a
  persistent grid, plain or XCD-contiguous work order) gives the same state
  bit for bit on the equidistant 512 x 60 x 180 domain (2,400 blocks);
- ic_autotune leaves the state and time untouched, picks a schedule no
  slower than the default on its own measurement, and returns the same
  choice from its cache on the second call;
- invalid schedules are rejected.
"""
import numpy as np
import pytest

from synthetic import as_dict, workload

pytestmark = pytest.mark.gpu


def _ic():
    import paper_2211_12867_amd as ic
    return ic


def _sim(ic):
    w = workload("equidistant_full")
    return ic.Sim(as_dict(w.grid), as_dict(w.wind), [as_dict(w.cmes[0])])


def test_schedules_are_bit_identical():
    ic = _ic()
    ref = None
    for waves in (2, 1):
        for grid in (0, 1024):
            for xcd in (0, 1):
                sim = _sim(ic)
                sim.set_tuning(waves, grid, xcd)
                for _ in range(2):
                    sim.step()
                U = sim.state()[1]
                t = sim.time()
                sim.close()
                if ref is None:
                    ref = (U, t)
                else:
                    assert t == ref[1], (waves, grid, xcd)
                    assert np.array_equal(U, ref[0]), (waves, grid, xcd)


def test_autotune_keeps_state_and_caches(tmp_path):
    ic = _ic()
    sim = _sim(ic)
    sim.step()
    U0, t0 = sim.state()[1], sim.time()[0]
    cache = str(tmp_path / "tune.txt")
    r1 = sim.autotune(cache, reps=2)
    assert r1["from_cache"] == 0 and r1["candidates"] >= 4
    assert r1["stage_ms"] <= r1["default_ms"]
    assert np.array_equal(sim.state()[1], U0) and sim.time()[0] == t0
    r2 = sim.autotune(cache, reps=2)
    assert r2["from_cache"] == 1
    assert (r2["waves_per_simd"], r2["grid"], r2["xcd_order"]) == (r1["waves_per_simd"], r1["grid"], r1["xcd_order"])
    sim.step()
    sim.close()


def test_invalid_schedule_rejected():
    ic = _ic()
    sim = _sim(ic)
    with pytest.raises(ic.ICError) as e:
        sim.set_tuning(3, 0, 0)
    assert e.value.status == ic.IC_E_INVALID
    sim.close()
