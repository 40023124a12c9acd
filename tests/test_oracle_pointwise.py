"""Pins of the oracle's pointwise physics against textbook MHD facts.

Pins: the flux Jacobian's eigenvalues are the seven MHD characteristic
speeds (plus the zero of the B_n row); the fast speed reduces to the sound
speed (B = 0) and the Alfven speed (p = 0); the MHD flux reduces to the Euler
flux for B = 0; directions are interchangeable by relabelling; the Rusanov
flux of equal states is the physical flux; the MC limiter's truth table;
the frame sources cancel the hoop terms for a parcel at rest in the inertial
frame.
"""
import math

import numpy as np
import pytest

from oracle import _clib

G = 1.5


def _jacobian(w, d, g):
    u0 = _clib.cons(w, g)
    J = np.zeros((8, 8))
    for a in range(8):
        h = 1e-6 * max(1.0, abs(u0[a]))
        up, um = u0.copy(), u0.copy()
        up[a] += h
        um[a] -= h
        fp = _clib.flux(_clib.prim(up, g), d, g)
        fm = _clib.flux(_clib.prim(um, g), d, g)
        J[:, a] = (fp - fm) / (2 * h)
    return J


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_flux_jacobian_eigenvalues_are_mhd_wave_speeds(d, seed):
    rng = np.random.default_rng(seed)
    w = np.array([rng.uniform(0.5, 2), *rng.uniform(-1, 1, 3), rng.uniform(0.3, 2), *rng.uniform(-1.5, 1.5, 3)])
    rho, p = w[0], w[4]
    b2 = float(np.sum(w[5:] ** 2))
    bn = w[5 + d]
    a2 = G * p / rho
    s = a2 + b2 / rho
    disc = math.sqrt(s * s - 4 * a2 * bn * bn / rho)
    cf = math.sqrt(0.5 * (s + disc))
    cs = math.sqrt(max(0.0, 0.5 * (s - disc)))
    ca = abs(bn) / math.sqrt(rho)
    vn = w[1 + d]
    expect = sorted([vn - cf, vn - ca, vn - cs, vn, vn + cs, vn + ca, vn + cf, 0.0])
    ev = np.sort(np.linalg.eigvals(_jacobian(w, d, G)).real)
    assert np.allclose(ev, expect, atol=2e-5)
    assert abs(_clib.fast_speed(w, d, G) - cf) < 1e-13 * cf


def test_fast_speed_limits():
    w = np.array([1.3, 0.1, -0.2, 0.3, 0.7, 0, 0, 0])
    for d in range(3):
        assert abs(_clib.fast_speed(w, d, G) - math.sqrt(G * 0.7 / 1.3)) < 1e-15
    w = np.array([1.3, 0.1, -0.2, 0.3, 0.0, 0.4, -0.5, 0.2])
    for d in range(3):
        assert abs(_clib.fast_speed(w, d, G) - math.sqrt(0.45 / 1.3)) < 1e-15


def test_b0_flux_is_euler_flux():
    rho, v, p = 1.7, np.array([0.3, -0.4, 0.9]), 0.8
    w = np.array([rho, *v, p, 0, 0, 0])
    E = p / (G - 1) + 0.5 * rho * v.dot(v)
    for d in range(3):
        f = _clib.flux(w, d, G)
        ref = np.zeros(8)
        ref[0] = rho * v[d]
        ref[1:4] = rho * v[d] * v
        ref[1 + d] += p
        ref[4] = (E + p) * v[d]
        assert np.allclose(f, ref, rtol=1e-15, atol=1e-15)


def test_directions_are_relabellings():
    rng = np.random.default_rng(7)
    w = np.array([1.2, *rng.uniform(-1, 1, 3), 0.9, *rng.uniform(-1, 1, 3)])
    f0 = _clib.flux(w, 0, G)
    for d, perm in ((1, [1, 2, 0]), (2, [2, 0, 1])):
        # move component 0 of v and B to slot d
        wp = w.copy()
        vp = np.zeros(3); bp = np.zeros(3)
        for c in range(3):
            vp[(c + d) % 3] = w[1 + c]
            bp[(c + d) % 3] = w[5 + c]
        wp[1:4], wp[5:8] = vp, bp
        fd = _clib.flux(wp, d, G)
        for c in range(3):
            assert fd[1 + (c + d) % 3] == f0[1 + c]
            assert fd[5 + (c + d) % 3] == f0[5 + c]
        assert fd[0] == f0[0] and fd[4] == f0[4]
    del perm


def test_rusanov_of_equal_states_is_physical_flux():
    w = np.array([1.1, 0.2, 0.3, -0.1, 0.6, 0.5, 0.2, -0.3])
    for d in range(3):
        assert np.array_equal(_clib.rusanov(w, w, d, G), _clib.flux(w, d, G))


def test_prim_cons_round_trip():
    rng = np.random.default_rng(3)
    for _ in range(20):
        w = np.array([rng.uniform(0.1, 3), *rng.uniform(-2, 2, 3), rng.uniform(0.01, 3), *rng.uniform(-2, 2, 3)])
        assert np.allclose(_clib.prim(_clib.cons(w, G), G), w, rtol=1e-12, atol=1e-13)


def test_mc_limiter_truth_table():
    # linear data on a non-uniform grid is reproduced exactly
    x = [0.0, 0.3, 1.1]
    s = _clib.mc_slope(2 * x[0] + 1, 2 * x[1] + 1, 2 * x[2] + 1, *x)
    assert abs(s - 2.0) < 1e-15
    # extremum -> 0
    assert _clib.mc_slope(1.0, 2.0, 1.0, 0.0, 1.0, 2.0) == 0.0
    assert _clib.mc_slope(1.0, 1.0, 2.0, 0.0, 1.0, 2.0) == 0.0
    # min(2|dm|, |dc|, 2|dp|) with the sign of dc
    assert _clib.mc_slope(0.0, 1.0, 4.0, 0.0, 1.0, 2.0) == 2.0      # dm=1, dp=3, dc=2
    assert _clib.mc_slope(0.0, 1.0, 11.0, 0.0, 1.0, 2.0) == 2.0     # dm=1, dp=10: 2|dm|
    assert _clib.mc_slope(0.0, 3.0, 4.0, 0.0, 1.0, 2.0) == 2.0      # dm=3, dp=1: 2|dp| = |dc|
    assert _clib.mc_slope(0.0, 10.0, 11.0, 0.0, 1.0, 2.0) == 2.0    # 2|dp|
    assert _clib.mc_slope(4.0, 1.0, 0.0, 0.0, 1.0, 2.0) == -2.0


def test_frame_sources_cancel_hoop_terms_for_inertial_rest():
    """A parcel at rest in the inertial frame moves with v = -Omega x r in the
    co-rotating frame; with p = 0, B = 0 the total force is zero."""
    om = 0.43
    for r, th in ((0.3, 1.1), (1.0, 1.57), (1.7, 2.2)):
        w = np.array([2.0, 0.0, 0.0, -om * r * math.sin(th), 0.0, 0, 0, 0])
        S = _clib.sources(w, 1.0 / r, math.cos(th) / math.sin(th), r, math.sin(th), math.cos(th), om, 0.0)
        scale = 2.0 * om * om * r
        assert np.all(np.abs(S) <= 1e-14 * scale), S


def test_gravity_source():
    w = np.array([2.0, 0.5, 0.0, 0.0, 1.0, 0, 0, 0])
    S = _clib.sources(w, 0.0, 0.0, 0.5, 1.0, 0.0, 0.0, 1e-3)
    g = -1e-3 / 0.25
    assert S[1] == 2.0 * g and S[4] == 2.0 * 0.5 * g


def test_small_value_floors():
    from oracle.solver import apply_floors
    g = 1.5
    U = np.array([[2e-7, 1.0], [4e-7, 0.5], [0.0, 0.1], [0.0, 0.0], [1e-3, 1.0], [0.1, 0.2],
                  [0.0, 0.0], [0.0, 0.0]])
    U0 = U.copy()
    n = apply_floors(U, g, 1e-6, 1e-9)
    # cell 0: density raised at zero velocity, then pressure floored exactly
    assert U[0, 0] == 1e-6 and U[1, 0] == 0.0 and U[2, 0] == 0.0 and U[3, 0] == 0.0
    W = np.array(_clib.prim(U[:, 0], g))
    assert abs(W[4] - 1e-9) <= 1e-9 * 1e-6 * (U[4, 0] / 1e-9)
    # cell 1 is physical and untouched
    assert np.array_equal(U[:, 1], U0[:, 1]) and n == 2
