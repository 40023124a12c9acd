"""Shock diagnostics at a point (paper Sect. 3.1: arrival time and shock width,
measured from the arrival to the peak speed once the speed has jumped, read as
the top of the jump; Sect. 3.2: peak speed and average gradient of the shock).

The oracle's diagnostics are pinned by closed-form series; the library's
ic_shock_diagnostics (a host computation, so these run without a GPU) must
give the oracle's values on the same series, including the cases the
definition excludes: a crossing on a segment that starts before the CME
start, a rise below the minimum jump, no sample in the window.
"""
import math

import numpy as np
import pytest

from oracle import analysis


def _tri(t):
    # 400 until 40, rises to 800 at 46, falls to 500 at 60 and 450 at 100
    return np.interp(t, [0, 40, 46, 60, 100], [400, 400, 800, 500, 450])


def test_oracle_triangle_closed_forms():
    """Linear rise 400 -> 800 over [40, 46]: half-rise level 600 at t = 43,
    peak at 46, width 3, average gradient (800 - 600) / 3."""
    t = np.arange(0.0, 100.0, 0.5)
    d = analysis.diagnostics(t, _tri(t), 5.0, 96.0)
    assert abs(d["arrival"] + 5.0 - 43.0) < 1e-12 and abs(d["width"] - 3.0) < 1e-12
    assert d["v_pre"] == 400.0 and d["v_max"] == 800.0 and d["t_max"] == 46.0 and d["t_top"] == 46.0
    assert abs(d["gradient"] - 200.0 / 3.0) < 1e-12


def test_oracle_width_ends_at_the_top_of_the_jump():
    """A jump to 700 topping out at 46, a dip, then a second, higher hump to 800
    at 60: the level is 400 + (800 - 400)/2 = 600, crossed on the jump at
    t = 40 + 6 * 200/300 = 44; the width runs to the top of the jump (46), not
    to the later maximum, and the average gradient is (700 - 600)/2."""
    t = np.arange(0.0, 100.0, 0.5)
    v = np.interp(t, [0, 40, 46, 52, 60, 100], [400, 400, 700, 650, 800, 450])
    d = analysis.diagnostics(t, v, 5.0, 96.0)
    assert abs(d["arrival"] + 5.0 - 44.0) < 1e-12 and abs(d["width"] - 2.0) < 1e-12
    assert d["t_top"] == 46.0 and d["v_top"] == 700.0 and d["t_max"] == 60.0 and d["v_max"] == 800.0
    assert abs(d["gradient"] - 50.0) < 1e-12


def test_oracle_tanh_ramp_gradient():
    """A tanh ramp of height H and scale s between samples: arrival at its
    midpoint, peak at the last sample of the window, average gradient =
    (v_max - level) / width."""
    t = np.arange(0.0, 120.0, 0.1)
    ta = 50.05
    v = 400.0 + 300.0 * 0.5 * (1.0 + np.tanh((t - ta) / 2.0))
    d = analysis.diagnostics(t, v, 10.0, 96.0)
    assert abs(d["arrival"] + 10.0 - ta) < 1e-9
    level = d["v_pre"] + 0.5 * (d["v_max"] - d["v_pre"])
    assert abs(d["gradient"] - (d["v_top"] - level) / d["width"]) < 1e-12
    assert abs(d["t_top"] - (d["arrival"] + 10.0 + d["width"])) < 1e-9
    # the ramp tops out where it stops rising (to rounding, at its maximum)
    assert abs(d["v_top"] - d["v_max"]) <= 1e-12 * d["v_max"] and d["t_top"] <= d["t_max"]


def test_oracle_exclusions():
    t = np.arange(0.0, 100.0, 0.5)
    # a rise below the minimum jump is no arrival
    d = analysis.diagnostics(t, _tri(t), 5.0, 96.0, min_jump=500.0)
    assert math.isnan(d["arrival"]) and d["v_max"] == 800.0
    # coarse samples, the CME starts inside the rising segment [10, 20]: the
    # half-rise crossing lies on that segment, which starts before the launch,
    # so there is no arrival; a launch at the segment start counts
    tc, vc = np.array([0.0, 10.0, 20.0, 30.0]), np.array([400.0, 400.0, 800.0, 800.0])
    assert math.isnan(analysis.diagnostics(tc, vc, 12.0, 96.0)["arrival"])
    d = analysis.diagnostics(tc, vc, 10.0, 96.0)
    assert abs(d["arrival"] - 5.0) < 1e-12 and d["width"] == 5.0
    # no sample inside the window
    d = analysis.diagnostics(t, _tri(t), 200.0, 10.0)
    assert math.isnan(d["arrival"]) and d["v_max"] == d["v_pre"]


def _series():
    out = []
    t = np.arange(0.0, 100.0, 0.5)
    out.append(("triangle", t, _tri(t), 5.0, 96.0, 0.0))
    out.append(("triangle gated", t, _tri(t), 5.0, 96.0, 500.0))
    tc, vc = np.array([0.0, 10.0, 20.0, 30.0]), np.array([400.0, 400.0, 800.0, 800.0])
    out.append(("crossing segment starts before launch", tc, vc, 12.0, 96.0, 0.0))
    out.append(("launch at a segment start", tc, vc, 10.0, 96.0, 0.0))
    out.append(("launch on a sample inside the rise", t, np.interp(t, [0, 42, 44, 100], [400, 400, 800, 800]),
                42.5, 96.0, 0.0))
    out.append(("empty window", t, _tri(t), 200.0, 10.0, 0.0))
    out.append(("double hump", t, np.interp(t, [0, 40, 46, 52, 60, 100], [400, 400, 700, 650, 800, 450]),
                5.0, 96.0, 0.0))
    tt = np.arange(0.0, 120.0, 0.1)
    out.append(("tanh", tt, 400.0 + 150.0 * (1.0 + np.tanh((tt - 50.05) / 2.0)), 10.0, 96.0, 100.0))
    rng = np.random.default_rng(11)
    for q in range(6):
        tr = np.cumsum(rng.uniform(0.05, 0.3, 600))
        vr = 400.0 + np.cumsum(rng.normal(0.0, 8.0, 600)) + 300.0 * (tr > tr[300])
        out.append(("random %d" % q, tr, vr, float(tr[150] + 0.01 * q), 40.0, 50.0 * (q % 3)))
    return out


@pytest.mark.parametrize("case", _series(), ids=lambda c: c[0])
def test_library_matches_the_oracle(case):
    import paper_2211_12867_amd as ic
    _, t_h, v, t0, win, jump = case
    ref = analysis.diagnostics(t_h, v, t0, win, jump)
    got = ic.shock_diagnostics(np.asarray(t_h) * 3600.0, v, t0 * 3600.0, win * 3600.0, jump)
    pairs = [("arrival", "arrival_s", 3600.0), ("width", "width_s", 3600.0), ("v_pre", "v_pre", 1.0),
             ("v_max", "v_max", 1.0), ("gradient", "gradient", 1.0 / 3600.0), ("t_max", "t_max_s", 3600.0),
             ("t_top", "t_top_s", 3600.0), ("v_top", "v_top", 1.0)]
    for a, b, scale in pairs:
        x, y = ref[a] * scale, got[b]
        if math.isnan(x):
            assert math.isnan(y), (a, x, y)
        else:
            assert abs(x - y) <= 1e-9 * max(1.0, abs(x)), (a, x, y)
    # the hour-based convenience call gives the same arrival and width
    a, w = ic.arrival(t_h, v, t0, win, jump)
    for x, y in ((ref["arrival"], a), (ref["width"], w)):
        assert (math.isnan(x) and math.isnan(y)) or abs(x - y) <= 1e-9 * max(1.0, abs(x))


def test_library_rejects_bad_input():
    import paper_2211_12867_amd as ic
    with pytest.raises(ic.ICError) as ex:
        ic.shock_diagnostics(np.array([0.0, 2.0, 1.0]), np.array([1.0, 2.0, 3.0]), 0.0)
    assert ex.value.status == ic.IC_E_INVALID
