"""Pins of the oracle's spherical source terms with B != 0, its CFL widths, its
initial state and its point sampling (paper Sect. 2.1: ideal MHD in spherical
co-rotating coordinates, finite volumes, two ghost layers).

Steady states.  Each field below is an exact stationary solution of ideal MHD
with the frame rotation and gravity switched off.  Written in spherical
components, every such field has gradients that the flux differences and the
geometric (hoop) source terms must cancel, so the discrete operator L(U) of a
smooth steady state is a truncation error: it must fall as h^2 under grid
refinement, for every conserved component.  A dropped hoop term, a wrong sign
or a swapped index leaves an O(1) residual that does not converge.  Ghost
cells take the exact field at their centres (no boundary condition enters).

  U   uniform flow across a uniform field, v and B constant in cartesian
      terms (all six spherical components vary with theta and phi):
      S_m_r (rho v_t^2 + rho v_p^2, B_t^2 + B_p^2, 2 p_tot), S_m_theta
      (rho v_r v_t, B_r B_t, cot-terms rho v_p^2, B_p^2, p_tot), S_m_phi
      (rho v_p v_r, B_p B_r, rho v_p v_t, B_p B_t), S_B_theta (v_r B_t,
      v_t B_r), S_B_phi (v_p B_r, B_p v_r, v_p B_t, B_p v_t).
  Z   the field B0 z at rest with uniform p: the magnetic part of S_m_r and
      S_m_theta (B_t^2, B_r B_t) with no flow.
  T   the current-free field B0 z + C/(r sin theta) phi at rest, uniform p:
      |B| varies, magnetic pressure gradients balance the tension terms
      B_p^2 (S_m_r, S_m_theta) and B_p B_r, B_p B_t (S_m_phi).
  R   rigid rotation v_phi = W r sin(theta) about the field B0 z with
      p = p0 + rho W^2 (r sin theta)^2 / 2: the centrifugal hoop terms
      rho v_p^2 against the pressure gradient, and the induction terms
      v_p B_r, v_p B_t of S_B_phi.
"""
import math

import numpy as np
import pytest

from oracle import _clib, boundary, geometry, solver, units
from synthetic import Wind, as_dict

GAMMA = 1.5
TH0, TH1, PH0, PH1 = 50.0, 70.0, 30.0, 50.0
R0, R1 = 0.3, 0.6

V_U = np.array([-0.25, -0.82, 0.32]) * 0.6
B_U = np.array([0.75, 0.13, 0.93]) * 0.5


def _sph(vec, th, ph):
    """Spherical components (r, theta, phi) of a constant cartesian vector."""
    vx, vy, vz = vec
    r = vx * np.sin(th) * np.cos(ph) + vy * np.sin(th) * np.sin(ph) + vz * np.cos(th)
    t = vx * np.cos(th) * np.cos(ph) + vy * np.cos(th) * np.sin(ph) - vz * np.sin(th)
    p = -vx * np.sin(ph) + vy * np.cos(ph)
    return r, t, p


def _field(case, r, th, ph):
    W = np.zeros((8,) + np.broadcast(r, th, ph).shape)
    one = np.ones_like(W[0])
    if case == "U":
        W[0] = 1.3 * one
        W[4] = 0.8 * one
        W[1], W[2], W[3] = [c * one for c in _sph(V_U, th, ph)]
        W[5], W[6], W[7] = [c * one for c in _sph(B_U, th, ph)]
    elif case == "Z":
        W[0] = one
        W[4] = 0.6 * one
        W[5], W[6], W[7] = [c * one for c in _sph((0.0, 0.0, 0.7), th, ph)]
    elif case == "T":
        W[0] = one
        W[4] = 0.9 * one
        W[5], W[6], _ = [c * one for c in _sph((0.0, 0.0, 0.5), th, ph)]
        W[7] = 0.08 / (r * np.sin(th)) * one
    elif case == "R":
        Wr = 1.7
        s = r * np.sin(th)
        W[0] = 1.2 * one
        W[3] = Wr * s * one
        W[4] = (0.5 + 0.5 * 1.2 * Wr * Wr * s * s) * one
        W[5], W[6], W[7] = [c * one for c in _sph((0.0, 0.0, 0.6), th, ph)]
    return W


def _grid(n, stretched):
    return dict(geometry="spherical", x0=(R0, TH0, PH0), x1=(R1, TH1, PH1), n=(n, n, n),
                block=(n, n, n), stretched_r=stretched, gamma=GAMMA)


def _residual(case, n, stretched):
    """max over interior cells of |L_v(U)| per conserved variable, U = the
    exact field at the cell centres (ghosts included)."""
    g = geometry.LevelGeometry(_grid(n, stretched), 1)
    pg = _clib.PatchGeom(g.f[0], g.f[1], g.f[2], False, GAMMA, 0.0, 0.0)
    rc, tc, pc = [geometry.centres(g.f[d]) for d in range(3)]
    W = _field(case, rc[None, None, :], tc[None, :, None], pc[:, None, None])
    G = boundary.prims_to_cons(W, GAMMA)
    L, _, bad = _clib.rhs(pg, G)
    assert bad == 0
    return np.abs(L).reshape(8, -1).max(axis=1)


def test_uniform_fields_have_no_interior_extrema():
    """The limiter clips slopes at extrema (first order there): the cases are
    set up so that no primitive has an extremum along a coordinate line of the
    ghosted domain."""
    th = np.radians(np.linspace(TH0 - 8.0, TH1 + 8.0, 801))
    ph = np.radians(np.linspace(PH0 - 8.0, PH1 + 8.0, 801))
    for case in ("U", "Z", "T", "R"):
        W = _field(case, 0.45, th[:, None], ph[None, :])
        for v in range(8):
            for ax in (0, 1):
                d = np.diff(W[v], axis=ax)
                assert np.all(d > 0) or np.all(d < 0) or np.all(np.abs(d) < 1e-15), (case, v, ax)


@pytest.mark.parametrize("stretched", [False, True])
@pytest.mark.parametrize("case", ["U", "Z", "T", "R"])
def test_steady_states_converge_at_second_order(case, stretched):
    e = [_residual(case, n, stretched) for n in (8, 16, 32)]
    for v in range(8):
        if max(x[v] for x in e) <= 1e-12:
            continue                       # the component balances to round-off
        o1 = math.log(e[0][v] / e[1][v], 2.0)
        o2 = math.log(e[1][v] / e[2][v], 2.0)
        assert o2 >= 1.8 and o1 >= 1.6, (case, v, [x[v] for x in e], o1, o2)


def test_a_flipped_hoop_term_would_not_converge():
    """The residual of the uniform state is a truncation error only because the
    hoop terms cancel the flux differences: take the hoop terms out (via the
    pointwise sources at the cell centres) and an O(1) residual appears."""
    n = 16
    g = geometry.LevelGeometry(_grid(n, False), 1)
    rc, tc = geometry.centres(g.f[0])[2:-2], geometry.centres(g.f[1])[2:-2]
    i, j = n // 2, n // 2
    W = _field("U", rc[i], tc[j], math.radians(40.0))
    rm, rp = g.f[0][i + 2], g.f[0][i + 3]
    tm, tp = g.f[1][j + 2], g.f[1][j + 3]
    rt = 1.5 * (rp * rp - rm * rm) / (rp ** 3 - rm ** 3)
    ct = (math.sin(tp) - math.sin(tm)) / (math.cos(tm) - math.cos(tp))
    S = _clib.sources(W[:, 0, 0, 0] if W.ndim == 4 else W, rt, ct, rc[i], math.sin(tc[j]),
                      math.cos(tc[j]), 0.0, 0.0)
    # the hoop terms are O(1) for this state, against an O(h^2) residual
    assert np.abs(S[[1, 2, 3, 6, 7]]).min() > 0.05
    assert _residual("U", n, False)[[1, 2, 3, 6, 7]].max() < 1e-2


# --- CFL rate: the spherical cell widths ------------------------------------------

def _rate_case(v, stretched, p=1e-2, rho=2.0):
    n = (6, 5, 4)
    grid = dict(geometry="spherical", x0=(0.2, 50.0, 10.0), x1=(0.8, 110.0, 70.0), n=n, block=n,
                stretched_r=stretched, gamma=GAMMA)
    g = geometry.LevelGeometry(grid, 1)
    pg = _clib.PatchGeom(g.f[0], g.f[1], g.f[2], False, GAMMA, 0.0, 0.0)
    W = np.zeros((8, n[2] + 4, n[1] + 4, n[0] + 4))
    W[0] = rho
    W[4] = p
    W[1:4] = np.asarray(v, dtype=np.float64)[:, None, None, None]
    G = boundary.prims_to_cons(W, GAMMA)
    return g, _clib.max_rate(pg, G)


@pytest.mark.parametrize("stretched", [False, True])
def test_cfl_rate_uses_the_spherical_widths(stretched):
    """Uniform state with B = 0: rate = max over cells of
    (|v_r| + c)/dr + (|v_t| + c)/(r_c dtheta) + (|v_p| + c)/(r_c sin(theta_c) dphi),
    c = sqrt(gamma p / rho); the widths written out here by hand."""
    for v in ((3.0, 0.0, 0.0), (0.0, -2.5, 0.0), (0.0, 0.0, 1.75), (0.4, -0.3, 0.9)):
        g, got = _rate_case(v, stretched)
        c = math.sqrt(GAMMA * 1e-2 / 2.0)
        best = 0.0
        for i in range(6):
            r_lo, r_hi = g.f[0][i + 2], g.f[0][i + 3]
            r_c = 0.5 * (r_lo + r_hi)
            for j in range(5):
                t_lo, t_hi = g.f[1][j + 2], g.f[1][j + 3]
                t_c = 0.5 * (t_lo + t_hi)
                for k in range(4):
                    dphi = g.f[2][k + 3] - g.f[2][k + 2]
                    rate = ((abs(v[0]) + c) / (r_hi - r_lo) + (abs(v[1]) + c) / (r_c * (t_hi - t_lo))
                            + (abs(v[2]) + c) / (r_c * math.sin(t_c) * dphi))
                    best = max(best, rate)
        assert abs(got - best) <= 1e-13 * best, (v, got, best)


# --- initial state and sampling --------------------------------------------------

def test_initial_state_laws_along_rays():
    """Relaxation start: at r = r_in it is the inner-boundary wind, and along
    each ray rho r^2, p r^(2 gamma), B_r r^2 and v_r stay constant, v_phi =
    -Omega r sin(theta) and B is parallel to v (B_phi / B_r = v_phi / v_r)."""
    wind = as_dict(Wind(seed=5))
    r_in = 0.1
    om = units.OMEGA_CODE
    th = np.radians(np.linspace(31.0, 149.0, 7))[None, :, None]
    ph = np.radians(np.linspace(0.0, 350.0, 9))[:, None, None]
    r = np.array([0.1, 0.37, 1.0, 1.9])[None, None, :]
    W = boundary.initial_prims(wind, r + 0 * th + 0 * ph, th + 0 * r + 0 * ph, ph + 0 * r + 0 * th,
                               r_in, om, GAMMA)
    Wb = boundary.boundary_prims(wind, None, th[:, :, 0] + 0 * ph[:, :, 0], ph[:, :, 0] + 0 * th[:, :, 0],
                                 r_in, om, 0.0)
    assert np.allclose(W[:, :, :, 0], Wb, rtol=1e-14, atol=0.0)
    x = r / r_in
    for a, b in ((W[0] * x ** 2, Wb[0]), (W[4] * x ** (2 * GAMMA), Wb[4]), (W[5] * x ** 2, Wb[5]),
                 (W[1], Wb[1])):
        assert np.allclose(a, b[:, :, None], rtol=1e-13, atol=0.0)
    assert np.allclose(W[3], -om * r * np.sin(th), rtol=1e-14, atol=0.0)
    assert np.allclose(W[7] * W[1], W[5] * W[3], rtol=1e-13, atol=0.0)
    assert np.all(W[2] == 0.0) and np.all(W[6] == 0.0)


def _linear_prims(r, th, ph):
    W = np.zeros((8,) + np.broadcast(r, th, ph).shape)
    one = np.ones_like(W[0])
    W[0] = 2.0 + 0.5 * r + 0.3 * th - 0.2 * ph
    W[1] = 0.7 - 0.1 * r + 0.05 * th + 0.02 * ph
    W[2] = -0.1 + 0.2 * r * one
    W[3] = 0.03 * th - 0.01 * ph + 0 * r
    W[4] = 1.0 + 0.1 * r + 0.2 * th + 0.1 * ph
    W[5] = 0.3 - 0.2 * r * one
    W[6] = 0.1 * th * one
    W[7] = -0.2 + 0.05 * ph * one
    return W


@pytest.mark.parametrize("stretched", [False, True])
def test_sample_reproduces_a_linear_field(stretched):
    """Trilinear interpolation between cell centres reproduces primitives
    that are linear in (r, theta, phi) exactly (single level, the state built
    from the field at the cell centres)."""
    grid = dict(geometry="spherical", x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=(16, 8, 8),
                block=(8, 8, 8), stretched_r=stretched, max_level=1, gamma=GAMMA)
    s = solver.Solver(grid, initial="zero")
    for leaf in s.forest.leaves:
        r = s.centres(leaf, 0)[None, None, :]
        th = s.centres(leaf, 1)[None, :, None]
        ph = s.centres(leaf, 2)[:, None, None]
        s.U[leaf] = boundary.prims_to_cons(_linear_prims(r, th, ph), GAMMA)
    for p in ((0.5, 90.0, 45.0), (0.137, 71.3, 12.9), (1.02, 113.0, 80.0), (0.73, 88.9, 44.9)):
        got = s.sample(*p)
        want = _linear_prims(p[0], math.radians(p[1]), math.radians(p[2]))[:, ...].reshape(8)
        assert np.allclose(got, want, rtol=1e-13, atol=1e-14), (p, got, want)


def test_sample_across_a_level_change_cartesian():
    """Two levels on a cartesian box with a field linear in x, y, z (rho and
    E; m = 0, B constant): points in the coarse leaf whose interpolation
    stencil reaches into refined cells read the volume-weighted mean of the
    children, which equals the linear field at the coarse centre, so the
    interpolation stays exact; points deep in the fine leaves are exact as
    well."""
    grid = dict(geometry="cartesian", x0=(0.0, 0.0, 0.0), x1=(1.0, 1.0, 1.0), n=(8, 8, 8), block=(4, 4, 4),
                periodic=(False, False, False), max_level=2, gamma=GAMMA)
    s = solver.Solver(grid, initial="zero")
    s.regrid({b: (1 if b == (1, 1, 0, 0) else 0) for b in s.forest.leaves}, buffer_blocks=0)
    assert (2, 2, 0, 0) in s.forest.leaves and (1, 0, 0, 0) in s.forest.leaves

    def U_of(x, y, z):
        U = np.zeros((8,) + np.broadcast(x, y, z).shape)
        U[0] = 1.0 + 0.4 * x - 0.3 * y + 0.2 * z
        U[4] = 3.0 + 0.5 * x + 0.25 * y - 0.1 * z
        U[5] = 0.2
        U[7] = -0.1
        return U

    for leaf in s.forest.leaves:
        x = s.centres(leaf, 0)[None, None, :]
        y = s.centres(leaf, 1)[None, :, None]
        z = s.centres(leaf, 2)[:, None, None]
        s.U[leaf] = U_of(x, y, z)
    # (0.45, 0.3, 0.2): coarse leaf (1, 0, 0, 0), stencil reaches x = 0.5625 (refined)
    # (0.7, 0.2, 0.3): fine leaf (2, 2, 0, 0)... (2, 2, 1, 1), stencil inside fine cells
    for p in ((0.45, 0.3, 0.2), (0.7, 0.2, 0.3), (0.9, 0.4, 0.1)):
        got = s.sample(*p)
        want = boundary.cons_to_prims(U_of(*p).reshape(8, 1), GAMMA)[:, 0]
        assert np.allclose(got, want, rtol=1e-13, atol=1e-15), (p, got, want)


# --- floors -------------------------------------------------------------------------

def test_floors_invariants():
    """After the floors every cell has rho >= rho_floor and p >= p_floor (up to
    rounding); cells above both are untouched; a density-floored cell is at
    rest with rho = rho_floor; the energy never decreases; the floors are
    idempotent; the count is the density-floored cells plus the cells whose
    pressure, after the density floor, was below p_floor."""
    rng = np.random.default_rng(7)
    N = 4000
    U = np.zeros((8, N))
    U[0] = 10.0 ** rng.uniform(-8, 1, N)
    U[1:4] = rng.normal(0, 1, (3, N)) * U[0]
    U[5:8] = rng.normal(0, 0.3, (3, N))
    kin = 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]
    mag = 0.5 * (U[5] ** 2 + U[6] ** 2 + U[7] ** 2)
    U[4] = kin + mag + 10.0 ** rng.uniform(-12, 0, N)
    rf, pf = 1e-4, 1e-6
    V = U.copy()
    n = solver.apply_floors(V, GAMMA, rf, pf)
    W = boundary.cons_to_prims(V, GAMMA)
    assert np.all(V[0] >= rf) and np.all(W[4] >= pf - 1e-14 * V[4])      # p up to the rounding of E
    low = U[0] < rf
    Wu = boundary.cons_to_prims(U, GAMMA)
    keep = ~low & (Wu[4] >= pf)
    assert np.array_equal(V[:, keep], U[:, keep])
    assert np.all(V[1:4, low] == 0.0) and np.all(V[0, low] == rf)
    assert np.all(V[4] >= U[4])
    mid = U.copy()
    mid[0, low] = rf
    mid[1:4, low] = 0.0
    lowp = boundary.cons_to_prims(mid, GAMMA)[4] < pf
    assert n == int(low.sum()) + int(lowp.sum())
    assert low.sum() > 100 and lowp.sum() > 100
    V2 = V.copy()
    assert solver.apply_floors(V2, GAMMA, rf, pf) <= int(lowp.sum())
    assert np.allclose(V2, V, rtol=1e-15, atol=0.0)
