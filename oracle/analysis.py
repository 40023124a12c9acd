"""Shock diagnostics at a sample point (test infrastructure only).

The paper reports the shock arrival time and the shock width, measured from
the arrival to the peak speed reached once the speed has jumped (Sect. 3.1),
and in Sect. 3.2 the peak speed and the average gradient of the
shock, without defining arrival.  Readings: v_pre = v_r at the CME start
(linear between samples), v_max = the maximum of v_r within the window after
it (4 days; the peak speed), arrival = the first time v_r crosses
v_pre + (v_max - v_pre)/2 on a segment that starts at or after the CME
start, linearly interpolated between samples; the top of the jump = the first
sample from the end of that segment on after which v_r no longer rises (or
the last sample in the window); width = t(top) - arrival; average gradient = the mean
slope of v_r from the arrival (where v_r is at the half-rise level) to the
top, (v_top - level) / width; a rise v_max - v_pre below min_jump counts as
no arrival.  Times in any unit (the caller's), speeds in any unit.
"""
import numpy as np


def arrival(t_h, v, t_cme_h, window_h=96.0, min_jump=0.0):
    """(arrival time after the CME start, width, v_pre, v_max).
    Returns (nan, nan, v_pre, v_max) if the threshold is never crossed."""
    d = diagnostics(t_h, v, t_cme_h, window_h, min_jump)
    return d["arrival"], d["width"], d["v_pre"], d["v_max"]


def diagnostics(t, v, t_cme, window, min_jump=0.0):
    """dict(arrival, width, v_pre, v_max, gradient, t_top, v_top, t_max);
    arrival, width, gradient, t_top and v_top are nan without an arrival."""
    t = np.asarray(t, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    nan = float("nan")
    out = dict(arrival=nan, width=nan, v_pre=nan, v_max=nan, gradient=nan, t_top=nan, v_top=nan, t_max=nan)
    if len(t) == 0:
        return out
    v_pre = float(np.interp(t_cme, t, v))
    out["v_pre"] = v_pre
    sel = (t >= t_cme) & (t <= t_cme + window)
    if not np.any(sel):
        out["v_max"] = v_pre
        return out
    idx = np.nonzero(sel)[0]
    imax = idx[int(np.argmax(v[idx]))]
    v_max = float(v[imax])
    out["v_max"], out["t_max"] = v_max, float(t[imax])
    if v_max - v_pre < min_jump:
        return out
    thr = v_pre + 0.5 * (v_max - v_pre)
    tol = 1e-12 * max(1.0, abs(t_cme))
    last = idx[-1]
    for a in idx:
        if a == 0:
            continue
        if v[a - 1] < thr <= v[a] and t[a - 1] >= t_cme - tol:
            ta = t[a - 1] + (thr - v[a - 1]) * (t[a] - t[a - 1]) / (v[a] - v[a - 1])
            q = a
            while q < last and v[q + 1] > v[q]:
                q += 1
            out["arrival"] = float(ta - t_cme)
            out["t_top"], out["v_top"] = float(t[q]), float(v[q])
            out["width"] = float(t[q] - ta)
            if out["width"] > 0.0:
                out["gradient"] = (float(v[q]) - thr) / out["width"]
            return out
    return out
