"""Checkpoint and restart, and run-to-run determinism, through the C ABI.

The paper starts every CME run from a saved relaxed wind (Sect. 2.1, 3.1).
A checkpoint is the member's blocks, conserved state and clock (code-unit
time and the steps since the last regrid); a fresh sim restored from it
continues bit for bit like the run that was never interrupted, through
regrids at the original cadence.  Two sims of the same configuration give
bit-identical blocks and states (no order-dependent reductions on the
path), and an advance over captured multi-step graphs gives what single
steps with the same regrids give."""
import numpy as np
import pytest

from synthetic import Cme, Wind, as_dict

pytestmark = pytest.mark.gpu

BIG = 1e12     # an advance span no run reaches: the step count ends each call


def _ic():
    import paper_2211_12867_amd as ic
    return ic


def _wedge(tracer=False):
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=(48, 12, 24),
                block=(12, 12, 12), stretched_r=True, max_level=3, periodic=(False, False, False), gamma=1.5,
                cfl=0.4)
    wind = as_dict(Wind(seed=5))
    cme = as_dict(Cme(t_start_s=0.0, duration_s=6 * 3600.0, v_kms=1400.0, half_width_deg=35.0,
                      colat_deg=90.0, lon_deg=30.0, n_cm3=1500.0, T_K=0.8e6))
    amr = dict(dlon_earth_deg=60.0, dclt_earth_deg=30.0, regrid_every=5, buffer_blocks=1)
    if tracer:
        amr = dict(amr, criterion="combined")
    return grid, wind, cme, amr


@pytest.mark.parametrize("tracer", [False, True])
def test_checkpoint_restart_is_bit_exact(tracer):
    ic = _ic()
    grid, wind, cme, amr = _wedge(tracer)
    a = ic.Sim(grid, wind, [cme], amr, tracer=tracer)
    a.advance(BIG, 13)                        # regrids after steps 5 and 10
    ck = a.checkpoint()
    assert ck["since_regrid"] == 3 and ck["U"].shape[1] == (9 if tracer else 8)
    a.advance(BIG, 17)                        # regrids after steps 15, 20, 25, 30
    b = ic.Sim(grid, wind, [cme], amr, tracer=tracer)
    b.restore(ck)
    assert b.clock() == (ck["t_code"], 3)
    b.advance(BIG, 17)
    assert a.blocks() == b.blocks()
    assert max(blk[0] for blk in a.blocks()) >= 2
    assert np.array_equal(a.state()[1], b.state()[1])
    assert a.clock() == b.clock()


def test_two_runs_are_bit_identical():
    ic = _ic()
    grid, wind, cme, amr = _wedge()
    out = []
    for _ in range(2):
        s = ic.Sim(grid, wind, [cme], amr)
        s.advance(BIG, 22)
        out.append((s.blocks(), s.state()[1], s.clock(), s.timeseries()))
        s.close()
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]
    assert np.array_equal(out[0][3], out[1][3])


def test_advance_equals_single_steps_and_regrids():
    """ic_advance replays captured graphs of five steps (and of one step for
    the rest of a batch); 13 steps with regrids after steps 5 and 10 equal 13
    single ic_step calls with ic_regrid after the 5th and 10th, bit for bit."""
    ic = _ic()
    grid, wind, cme, amr = _wedge()
    a = ic.Sim(grid, wind, [cme], amr)
    a.advance(BIG, 13)
    b = ic.Sim(grid, wind, [cme], amr)
    for n in range(1, 14):
        b.step()
        if n in (5, 10):
            b.regrid()
    assert a.blocks() == b.blocks()
    assert max(blk[0] for blk in a.blocks()) >= 2
    assert np.array_equal(a.state()[1], b.state()[1])
    assert a.clock() == b.clock() and a.clock()[1] == 3
    assert np.array_equal(a.timeseries(), b.timeseries())


def test_clock_rejects_bad_values():
    ic = _ic()
    grid, wind, cme, amr = _wedge()
    s = ic.Sim(grid, wind, [cme], amr)
    for t, n in ((float("nan"), 0), (0.0, -1)):
        with pytest.raises(ic.ICError) as ex:
            s.set_clock(t, n)
        assert ex.value.status == ic.IC_E_INVALID
