"""Pins of the refinement-indicator quantities and of the arrival-time analysis.

- The Loehner-type estimator vanishes on linear data and equals 1/(1+eps) on
  a unit step in one direction (closed forms).
- div V of the linear field (ax, by, cz) is a + b + c, and of v = r r_hat on an
  equidistant spherical grid it is 3 (the face means are then exact).
- The Earth/CME windows of Sect. 3.2 select the cells they should.
- Arrival time: a tanh ramp crosses its midpoint at its centre; a triangular
  pulse gives arrival and width in closed form.
"""
import math

import numpy as np

from oracle import _clib, analysis, solver


def _cart_patch(n, h=1.0):
    f = [np.arange(-2, n[d] + 3, dtype=np.float64) * h for d in range(3)]
    return _clib.PatchGeom(f[0], f[1], f[2], True, 1.5, 0.0, 0.0)


def _ghosted_from_prims(W, gamma=1.5):
    from oracle.boundary import prims_to_cons
    return prims_to_cons(W, gamma)


def test_loehner_zero_on_linear_data_and_step_value():
    n = (6, 5, 4)
    pg = _cart_patch(n)
    K, J, I = np.meshgrid(np.arange(-2, n[2] + 2), np.arange(-2, n[1] + 2), np.arange(-2, n[0] + 2),
                          indexing="ij")
    W = np.zeros((8,) + K.shape)
    W[0] = 10.0 + I + 2 * J + 3 * K           # exact integers
    W[1] = 100.0 + 0.0 * I                      # |v| constant
    W[4] = 1.0
    er, ev, dv, ds = _clib.indicator(pg, _ghosted_from_prims(W), 0.01)
    assert np.all(er == 0.0) and np.all(ev == 0.0)
    # a unit step along j between j = 1 and j = 2 (u- = 0, u = 0, u+ = 1)
    W[0] = np.where(J >= 2, 2.0, 1.0)
    er, _, _, _ = _clib.indicator(pg, _ghosted_from_prims(W), 0.01)
    # cell j = 1: u- = u = 1, u+ = 2 -> num = 1, den = (1 + 5 eps)^2 along j plus
    # (4 eps)^2 from each of the two flat directions
    eps = 0.01
    assert abs(er[0, 1, 0] - 1.0 / math.sqrt((1 + 5 * eps) ** 2 + 2 * (4 * eps) ** 2)) < 1e-15
    # a 0/0/1 step: u- = u = 0, u+ = 1 -> 1/(1+eps)
    W[0] = np.where(J >= 2, 1.0, 1e-300)
    er, _, _, _ = _clib.indicator(pg, _ghosted_from_prims(W), 0.01)
    assert abs(er[0, 1, 0] - 1.0 / 1.01) < 1e-12


def test_divv_linear_field_cartesian():
    n = (5, 4, 3)
    pg = _cart_patch(n, 0.25)
    K, J, I = np.meshgrid(np.arange(-2, n[2] + 2), np.arange(-2, n[1] + 2), np.arange(-2, n[0] + 2),
                          indexing="ij")
    x, y, z = (I + 0.5) * 0.25, (J + 0.5) * 0.25, (K + 0.5) * 0.25
    W = np.zeros((8,) + K.shape)
    W[0], W[4] = 1.0, 1.0
    W[1], W[2], W[3] = 2.0 * x, -3.0 * y, 0.5 * z
    _, _, dv, _ = _clib.indicator(pg, _ghosted_from_prims(W), 0.01)
    assert np.allclose(dv, -0.5, atol=1e-13)


def test_divv_radial_field_spherical():
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 60.0), n=(10, 6, 6),
                block=(10, 6, 6), gamma=1.5, bc=[("outflow", "outflow")] * 3)
    s = solver.PatchSolver(grid, omega=0.0, gm=0.0, initial="zero")
    f = s.geo.f
    rc = 0.5 * (f[0][:-1] + f[0][1:])
    W = np.zeros((8, 10, 10, 14))
    W[0], W[4] = 1.0, 1.0
    W[1] = rc[None, None, :]
    _, _, dv, _ = _clib.indicator(s.pg, _ghosted_from_prims(W), 0.01)
    assert np.allclose(dv, 3.0, rtol=1e-12)


def test_windows():
    grid = dict(geometry="spherical", x0=(0.1, 30.0, 0.0), x1=(2.0, 150.0, 360.0), n=(12, 24, 48),
                block=(12, 24, 48), periodic=(False, False, True), gamma=1.5)
    s = solver.Solver(grid, initial="zero")
    leaf = (1, 0, 0, 0)
    w = s.window(leaf, dict(lon_deg=0.0))
    th = np.degrees(s.centres(leaf, 1))
    ph = np.degrees(s.centres(leaf, 2))
    for k in range(48):
        for j in range(24):
            lon = ph[k] if ph[k] <= 180 else ph[k] - 360
            expect = abs(lon) <= 30 and abs(th[j] - 90) <= 10
            assert w[k, j, 0] == expect
    w2 = s.window(leaf, dict(lon_deg=200.0))      # CME window excludes the Earth side
    assert not w2.any()


def test_arrival_tanh_ramp():
    t = np.arange(0.0, 120.0, 0.1)
    ta = 50.05                        # midway between two samples
    v = 400.0 + 300.0 * 0.5 * (1.0 + np.tanh((t - ta) / 2.0))
    a, _, vpre, vmax = analysis.arrival(t, v, 10.0)
    assert abs((a + 10.0) - ta) < 1e-9


def test_arrival_triangle_width():
    t = np.arange(0.0, 100.0, 0.5)
    v = np.interp(t, [0, 40, 46, 60, 100], [400, 400, 800, 500, 450])
    a, width, vpre, vmax = analysis.arrival(t, v, 5.0)
    assert abs(a + 5.0 - 43.0) < 1e-12 and abs(width - 3.0) < 1e-12
    assert vpre == 400.0 and vmax == 800.0


def test_hot_is_the_uncapped_refine_condition():
    """hot() marks the leaves the plain criterion refines when the level cap
    does not bind, and is independent of the cap."""
    from synthetic import as_dict, workload
    w = workload("tiny_wedge")
    amr = dict(as_dict(w.amr), lon_earth_deg=45.0, dlon_earth_deg=60.0, dclt_earth_deg=30.0)
    g1 = dict(as_dict(w.grid), max_level=1)
    g2 = dict(as_dict(w.grid), max_level=2)
    s1 = solver.Solver(g1, as_dict(w.wind), as_dict(w.cmes[0]), amr)
    for _ in range(12):
        s1.step()
    s2 = solver.Solver(g2, as_dict(w.wind), as_dict(w.cmes[0]), amr)
    s2.set_state(*s1.state(), s1.t)
    h1, h2 = s1.hot(), s2.hot()
    assert h1 == h2
    f1, f2 = s1.flags(), s2.flags()
    assert all(f == 0 for f in f1.values())                     # level 1 = max level: never REFINE
    assert {b: int(f == 1) for b, f in f2.items()} == h2
    assert 0 < sum(h2.values()) < len(h2)
