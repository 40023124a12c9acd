"""Whole-scheme pins of the oracle against what the mathematics fixes.

- Sod shock tube with B = 0 against the exact Riemann solution (gamma 1.4 and
  1.5) along x, y and z: L1 error and convergence, and the three axis runs
  identical after relabelling.
- Linear Alfven wave (B0 parallel to k, periodic) in 1-D and oblique 2-D:
  second-order convergence over one period.
- Free stream A: a uniform state at rest on stretched and equidistant
  spherical wedges stays uniform (hoop terms balance the flux differences).
- Free stream B: a spherically symmetric radial wind keeps v_theta = v_phi = 0
  and identical (theta, phi) columns.
- Conservation: sum(V U) on a periodic box.
- div B: in 1-D the normal field is constant exactly; the Parker field of a
  uniform wind has discrete div B of second order.
"""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from exact_riemann import sample  # noqa: E402

from oracle import _clib, boundary, solver, units  # noqa: E402
from synthetic import smooth_modes, uniform_wind, as_dict  # noqa: E402


def _cart_grid(n, x1=(1.0, 1.0, 1.0), periodic=(False, False, False), gamma=1.4, cfl=0.4):
    return dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=x1, n=n, block=n, periodic=periodic,
                gamma=gamma, cfl=cfl)


def _sod(N, axis, gamma, t_end=0.2, dt=None):
    n = [1, 1, 1]
    n[axis] = N
    x1 = [1.0, 1.0, 1.0]
    s = solver.PatchSolver(_cart_grid(tuple(n), tuple(x1), gamma=gamma), initial="zero")
    xc = (np.arange(N) + 0.5) / N
    W = np.zeros((8, N))
    W[0] = np.where(xc < 0.5, 1.0, 0.125)
    W[4] = np.where(xc < 0.5, 1.0, 0.1)
    U = boundary.prims_to_cons(W, gamma)
    shape = [1, 1, 1]
    shape[2 - axis] = N
    s.U = U.reshape((8,) + tuple(shape)).copy()
    t = 0.0
    while t < t_end - 1e-14:
        h = dt if dt is not None else min(s.cfl_dt(), t_end - t)
        h = min(h, t_end - t)
        s.step(h)
        t += h
    return s, xc


@pytest.mark.parametrize("gamma", [1.4, 1.5])
def test_sod_against_exact_riemann(gamma):
    errs = []
    for N in (100, 200, 400):
        s, xc = _sod(N, 0, gamma)
        Wn = boundary.cons_to_prims(s.U.reshape(8, -1), gamma)
        ex = sample(xc, 0.2, 0.5, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma)
        errs.append(np.mean(np.abs(Wn[0] - ex[0])))
    assert errs[2] <= 1e-2, errs
    order = math.log(errs[0] / errs[2], 4.0)
    assert order >= 0.6, (errs, order)


def test_sod_axes_identical():
    ref, _ = _sod(64, 0, 1.4, t_end=0.05, dt=1e-3)
    u0 = ref.U.reshape(8, -1)
    for axis in (1, 2):
        s, _ = _sod(64, axis, 1.4, t_end=0.05, dt=1e-3)
        u = s.U.reshape(8, -1)
        assert np.array_equal(u[0], u0[0]) and np.array_equal(u[4], u0[4])
        assert np.array_equal(u[1 + axis], u0[1])
        for c in range(3):
            if c != axis:
                assert np.all(u[1 + c] == 0.0)


def _alfven(N, oblique):
    """Right-going Alfven wave, B0 = 1 along k, rho = 1, p = 1; one period."""
    gamma = 5.0 / 3.0
    A = 1e-6
    if oblique:
        n = (N, N, 1)
        grid = _cart_grid(n, (1.0, 1.0, 1.0 / N), periodic=(True, True, True), gamma=gamma)
        k = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
        wavelength = 1.0 / math.sqrt(2.0)
        perp = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0)
    else:
        n = (N, 1, 1)
        grid = _cart_grid(n, (1.0, 1.0 / N, 1.0 / N), periodic=(True, True, True), gamma=gamma)
        k = np.array([1.0, 0.0, 0.0])
        wavelength = 1.0
        perp = np.array([0.0, 1.0, 0.0])
    s = solver.PatchSolver(grid, initial="zero")
    x = (np.arange(n[0]) + 0.5) / n[0]
    y = (np.arange(n[1]) + 0.5) / n[1] if oblique else np.zeros(1)
    X = x[None, None, :] + 0.0 * y[None, :, None]
    Y = y[None, :, None] + 0.0 * x[None, None, :]
    phase = 2 * math.pi * (k[0] * X + k[1] * Y) / wavelength
    dv = A * np.sin(phase)
    W = np.zeros((8,) + X.shape)
    W[0] = 1.0
    W[4] = 1.0
    for c in range(3):
        W[1 + c] = dv * perp[c]
        W[5 + c] = k[c] - dv * perp[c]       # dB = -sqrt(rho) dv
    s.U = boundary.prims_to_cons(W, gamma)
    U0 = s.U.copy()
    T = wavelength / 1.0
    t = 0.0
    while t < T - 1e-14:
        h = min(s.cfl_dt(), T - t)
        s.step(h)
        t += h
    Wt = boundary.cons_to_prims(s.U, gamma)
    vperp = sum(Wt[1 + c] * perp[c] for c in range(3))
    v0 = sum(boundary.cons_to_prims(U0, gamma)[1 + c] * perp[c] for c in range(3))
    return np.mean(np.abs(vperp - v0)) / A


def test_alfven_wave_second_order_1d():
    e1, e2 = _alfven(64, False), _alfven(128, False)
    order = math.log(e1 / e2, 2.0)
    assert order >= 1.8, (e1, e2, order)


def test_alfven_wave_oblique_converges_to_second_order():
    # the limiter clips the extrema, so the observed order approaches 2 from
    # below as the grid is refined: 1.65 (24->48), 1.80 (48->96)
    e = [_alfven(n, True) for n in (24, 48, 96)]
    o1, o2 = math.log(e[0] / e[1], 2.0), math.log(e[1] / e[2], 2.0)
    assert o2 >= 1.75 and o2 > o1, (e, o1, o2)


def _wedge(stretched, n=(24, 8, 8), x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 40.0)):
    return dict(geometry="spherical", x0=x0, x1=x1, n=n, block=n, stretched_r=stretched,
                bc=[("outflow", "outflow")] * 3, gamma=1.5, cfl=0.4)


@pytest.mark.parametrize("stretched", [False, True])
def test_free_stream_uniform_state_at_rest(stretched):
    s = solver.PatchSolver(_wedge(stretched), omega=0.0, gm=0.0, initial="zero")
    W = np.zeros((8,) + s.U.shape[1:])
    W[0] = 2.0
    W[4] = 0.7
    s.U = boundary.prims_to_cons(W, 1.5)
    U0 = s.U.copy()
    for _ in range(100):
        s.step()
    dev = np.abs(s.U - U0).max(axis=(1, 2, 3))
    scale = np.array([2.0, 1, 1, 1, 0.7 / 0.5, 1, 1, 1])
    assert np.all(dev <= 1e-13 * scale), dev


def test_free_stream_radial_wind_keeps_symmetry():
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 40.0), n=(32, 8, 8),
                block=(32, 8, 8), stretched_r=True, gamma=1.5, cfl=0.4,
                bc=[("inner", "outflow"), ("outflow", "outflow"), ("outflow", "outflow")])
    wind = as_dict(uniform_wind(450.0, 300.0, 1e6, 0.0))
    s = solver.PatchSolver(grid, wind, None, omega=0.0, gm=units.GM_CODE)
    for _ in range(100):
        s.step()
    U = s.U
    mr = np.abs(U[1]).max()
    assert np.abs(U[2]).max() <= 1e-14 * mr and np.abs(U[3]).max() <= 1e-14 * mr
    for v in (0, 1, 4):
        col = U[v][0:1, 0:1, :]
        rel = np.abs(U[v] - col).max() / np.abs(U[v]).max()
        assert rel <= 1e-15, (v, rel)


def test_conservation_periodic_box():
    n = (16, 12, 8)
    grid = _cart_grid(n, (1.0, 0.75, 0.5), periodic=(True, True, True), gamma=1.5)
    s = solver.PatchSolver(grid, initial="zero")
    X = (np.arange(n[0]) + 0.5) / n[0]
    Y = 0.75 * (np.arange(n[1]) + 0.5) / n[1]
    Z = 0.5 * (np.arange(n[2]) + 0.5) / n[2]
    Z3, Y3, X3 = np.meshgrid(Z, Y, X, indexing="ij")
    W = np.zeros((8,) + X3.shape)
    base = [1.0, 0.0, 0.0, 0.0, 1.0, 0.3, 0.2, -0.1]
    for v in range(8):
        ks, amps, ph = smooth_modes(100 + v, 3, 0.2 if v in (0, 4) else 0.3)
        f = np.zeros_like(X3)
        for kk, a, p in zip(ks, amps, ph):
            f += a * np.sin(2 * math.pi * (kk[0] * X3 + kk[1] * Y3 / 0.75 + kk[2] * Z3 / 0.5) + p)
        W[v] = base[v] + f
    s.U = boundary.prims_to_cons(W, 1.5)
    tot0 = s.total()
    V = (1.0 / 16) * (0.75 / 12) * (0.5 / 8)
    scale = np.abs(s.U).reshape(8, -1).sum(axis=1) * V
    for _ in range(100):
        s.step()
    assert np.all(np.abs(s.total() - tot0) <= 1e-13 * scale), (s.total() - tot0) / scale


def test_normal_field_constant_in_1d():
    gamma = 2.0
    N = 64
    grid = _cart_grid((N, 1, 1), periodic=(False, False, False), gamma=gamma)
    s = solver.PatchSolver(grid, initial="zero")
    xc = (np.arange(N) + 0.5) / N
    W = np.zeros((8, 1, 1, N))
    W[0] = np.where(xc < 0.5, 1.0, 0.125)
    W[4] = np.where(xc < 0.5, 1.0, 0.1)
    W[5] = 0.75
    W[6] = np.where(xc < 0.5, 1.0, -1.0)
    s.U = boundary.prims_to_cons(W, gamma)
    for _ in range(40):
        s.step()
    assert np.all(s.U[5] == 0.75)


def _div_b_parker(n):
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 60.0), n=n, block=n,
                gamma=1.5)
    wind = as_dict(uniform_wind(450.0, 300.0, 1e6, 300.0))
    s = solver.PatchSolver(grid, wind, None)
    G = s.ghosted(s.U, 0.0)
    # discrete div B with the indicator's face-mean form, on the velocity slots
    Gb = G.copy()
    Gb[1:4] = G[5:8] * G[0:1]      # so that v == B in the primitive recovery
    Gb[4] = G[4] + 1.0             # keep the recovered pressure positive
    _, _, dv, ds = _clib.indicator(s.pg, Gb, 0.01)
    # a fixed physical region away from the boundary ghosts: r >= 0.5 AU
    rc = np.array([s.geo.centre(0, i) for i in range(n[0])])
    sel = (slice(1, -1), slice(1, -1), (rc >= 0.5) & (np.arange(n[0]) < n[0] - 1))
    return np.abs(dv[sel]).max(), np.abs(ds[sel]).max()


def test_parker_field_div_b_second_order():
    e1, s1 = _div_b_parker((16, 8, 8))
    e2, s2 = _div_b_parker((32, 16, 16))
    e3, s3 = _div_b_parker((64, 32, 32))
    assert e1 / s1 < 1e-2
    assert math.log(e2 / e3, 2) >= 1.8, (e1, e2, e3)
