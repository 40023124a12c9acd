"""Shock diagnostics at a sample point (test infrastructure only).

The paper reports the shock arrival time and the shock width, the time from
arrival to the maximum speed after the jump (Sect. 3.1), without defining
arrival.  Reading: v_pre = v_r at the CME start, v_max = the maximum of v_r
within 4 days after it, arrival = the first time v_r crosses
v_pre + (v_max - v_pre)/2, linearly interpolated between samples.
"""
import numpy as np


def arrival(t_h, v, t_cme_h, window_h=96.0):
    """(arrival time after the CME start [h], width [h], v_pre, v_max).
    Returns (nan, nan, v_pre, v_max) if the threshold is never crossed."""
    t_h = np.asarray(t_h, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    v_pre = float(np.interp(t_cme_h, t_h, v))
    sel = (t_h >= t_cme_h) & (t_h <= t_cme_h + window_h)
    if not np.any(sel):
        return float("nan"), float("nan"), v_pre, v_pre
    idx = np.nonzero(sel)[0]
    imax = idx[int(np.argmax(v[idx]))]
    v_max = float(v[imax])
    thr = v_pre + 0.5 * (v_max - v_pre)
    for a in idx:
        if a == 0:
            continue
        if v[a - 1] < thr <= v[a] and t_h[a - 1] >= t_cme_h - 1e-12:
            ta = t_h[a - 1] + (thr - v[a - 1]) * (t_h[a] - t_h[a - 1]) / (v[a] - v[a - 1])
            return ta - t_cme_h, float(t_h[imax] - ta), v_pre, v_max
    return float("nan"), float("nan"), v_pre, v_max
