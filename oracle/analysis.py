"""Shock diagnostics at a sample point (test infrastructure only).

The paper reports the shock arrival time and the shock width, the time from
arrival to the maximum speed after the jump (Sect. 3.1), and in Sect. 3.2 the
peak speed and the average gradient of the shock, without defining arrival.
Readings: v_pre = v_r at the CME start (linear between samples), v_max = the
maximum of v_r within the window after it (4 days), arrival = the first time
v_r crosses v_pre + (v_max - v_pre)/2 on a segment that starts at or after
the CME start, linearly interpolated between samples; width = t(v_max) -
arrival; average gradient = the mean slope of v_r from the arrival (where
v_r is at the half-rise level) to the peak, (v_max - level) / width; a rise
v_max - v_pre below min_jump counts as no arrival.  Times in any unit (the
caller's), speeds in any unit.
"""
import numpy as np


def arrival(t_h, v, t_cme_h, window_h=96.0, min_jump=0.0):
    """(arrival time after the CME start, width, v_pre, v_max).
    Returns (nan, nan, v_pre, v_max) if the threshold is never crossed."""
    d = diagnostics(t_h, v, t_cme_h, window_h, min_jump)
    return d["arrival"], d["width"], d["v_pre"], d["v_max"]


def diagnostics(t, v, t_cme, window, min_jump=0.0):
    """dict(arrival, width, v_pre, v_max, gradient, t_max); arrival, width and
    gradient are nan without an arrival."""
    t = np.asarray(t, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    nan = float("nan")
    out = dict(arrival=nan, width=nan, v_pre=nan, v_max=nan, gradient=nan, t_max=nan)
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
    for a in idx:
        if a == 0:
            continue
        if v[a - 1] < thr <= v[a] and t[a - 1] >= t_cme - tol:
            ta = t[a - 1] + (thr - v[a - 1]) * (t[a] - t[a - 1]) / (v[a] - v[a - 1])
            out["arrival"] = float(ta - t_cme)
            out["width"] = float(t[imax] - ta)
            if out["width"] > 0.0:
                out["gradient"] = (v_max - thr) / out["width"]
            return out
    return out
