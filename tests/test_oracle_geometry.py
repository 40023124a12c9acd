"""Pins of the oracle's mesh geometry and cone-CME geometry.

Printed values (tests/golden/paper_values.json): Eq. (5)'s worked value,
the equidistant and stretched radial cell sizes of Sect. 2.2 and Table 3.
Closed forms: the wedge volume, the metric identities of the finite-volume
factors, coarse-fine face coincidence.  Cone CME: Eqs. (1)-(3) give
theta(0) = 0 and max theta = omega/2, and Eq. (4) is the great-circle
distance (checked against the haversine form).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import boundary, geometry, units

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_eq5_worked_value():
    g = GOLD["eq5_optimal_cells_low"]
    n = geometry.stretched_cell_count(g["r_in_au"], g["r_out_au"], math.radians(g["dphi_deg"]))
    assert round(n) == g["value"]


def test_equidistant_radial_sizes():
    g = GOLD["equidistant_low_dr_rsun"]
    f = geometry.radial_faces(0.1, 2.0, g["n_r"], False)
    assert round((f[3] - f[2]) * units.AU_IN_RSUN, 3) == g["value"]
    g = GOLD["equidistant_middle_high_dr_rsun"]
    for n, ref in zip(g["n_r"], g["value"]):
        f = geometry.radial_faces(0.1, 2.0, n, False)
        assert round((f[3] - f[2]) * units.AU_IN_RSUN, 2) == ref


def test_stretched_radial_size_at_1au_per_level():
    g = GOLD["stretched_dr_at_1au_rsun"]
    for n, ref in zip(g["n_r"], g["value"]):
        f = geometry.radial_faces(0.1, 2.0, n, True)
        q = f[10] / f[9]  # face ratio from the oracle's own faces
        width = 1.0 * (math.sqrt(q) - 1.0 / math.sqrt(q)) * units.AU_IN_RSUN
        # the printed values are 10.7 halved per level, to 3-4 digits
        assert abs(width - ref) <= 0.005 * ref, (n, width, ref)
    # face-based widths r(q - 1) do not reproduce the printed numbers
    f = geometry.radial_faces(0.1, 2.0, 60, True)
    assert abs((f[10] / f[9] - 1.0) * units.AU_IN_RSUN - 10.7) > 0.2


def test_stretching_keeps_cells_cubical():
    """Eq. (5)'s ratio q = (2 + dth)/(2 - dth) is exactly dr = r_c dth for
    r_c the arithmetic centre of [r, q r]."""
    dth = math.radians(3.75)
    q = (2 + dth) / (2 - dth)
    r = 0.37
    rc = 0.5 * (r + q * r)
    assert abs((q * r - r) - rc * dth) < 1e-15


@pytest.mark.parametrize("stretched", [False, True])
def test_volumes_sum_to_wedge(stretched):
    grid = dict(geometry="spherical", x0=(0.1, 30.0, 0.0), x1=(2.0, 150.0, 360.0), n=(24, 12, 16),
                stretched_r=stretched)
    g = geometry.LevelGeometry(grid, 1)
    tot = sum(g.volume(i, j, k) for i in range(24) for j in range(12) for k in range(16))
    ref = (2.0 ** 3 - 0.1 ** 3) / 3.0 * (math.cos(math.radians(30)) - math.cos(math.radians(150))) * 2 * math.pi
    assert abs(tot - ref) < 1e-13 * ref


def test_metric_identities():
    """(A_r+ - A_r-)/V = 2 rtinv and (A_t+ - A_t-)/V = rtinv ctil."""
    grid = dict(geometry="spherical", x0=(0.1, 30.0, 0.0), x1=(2.0, 150.0, 360.0), n=(20, 10, 8),
                stretched_r=True)
    g = geometry.LevelGeometry(grid, 1)
    for (i, j, k) in [(0, 0, 0), (7, 4, 3), (19, 9, 7)]:
        V = g.volume(i, j, k)
        rm, rp = g.f[0][i + 2], g.f[0][i + 3]
        tm, tp = g.f[1][j + 2], g.f[1][j + 3]
        rtinv = 1.5 * (rp * rp - rm * rm) / (rp ** 3 - rm ** 3)
        ctil = (math.sin(tp) - math.sin(tm)) / (math.cos(tm) - math.cos(tp))
        dAr = g.area(0, i, j, k, True) - g.area(0, i, j, k, False)
        dAt = g.area(1, i, j, k, True) - g.area(1, i, j, k, False)
        assert abs(dAr / V - 2 * rtinv) < 1e-12 * rtinv
        assert abs(dAt / V - rtinv * ctil) < 1e-11 * rtinv


@pytest.mark.parametrize("stretched", [False, True])
def test_children_faces_coincide_with_parent_faces(stretched):
    grid = dict(geometry="spherical", x0=(0.1, 30.0, 0.0), x1=(2.0, 150.0, 360.0), n=(60, 24, 48),
                stretched_r=stretched)
    for l in (1, 2, 3):
        a, b = geometry.LevelGeometry(grid, l), geometry.LevelGeometry(grid, l + 1)
        for d in range(3):
            n = a.n[d]
            assert np.array_equal(a.f[d][2:n + 3], b.f[d][2:2 * n + 3:2])


# --- cone CME ----------------------------------------------------------------

CME = dict(t_start_s=0.0, duration_s=1e9, v_kms=1500.0, half_width_deg=45.0, colat_deg=90.0,
           lon_deg=0.0, n_cm3=1200.0, T_K=0.8e6)


def test_cme_opening_angle_closed_forms():
    R = 0.1
    r_half, v, t_act = boundary.cme_geometry(CME, R)
    assert abs(r_half - R * math.sin(math.radians(45.0))) < 1e-16
    assert boundary.cme_opening_angle(CME, R, 0.0) == 0.0
    # the maximum opening angle is omega/2, reached when R_c = sqrt(R^2 - r_1/2^2)
    tau_max = (math.sqrt(R * R - r_half * r_half) - (R - r_half)) / v
    th = boundary.cme_opening_angle(CME, R, tau_max)
    assert abs(th - math.radians(45.0)) < 1e-7
    taus = np.linspace(0, t_act, 401)
    ths = [boundary.cme_opening_angle(CME, R, t) for t in taus]
    assert max(ths) <= math.radians(45.0) + 1e-12
    # closes again when the sphere has passed: R_c = R + r_1/2
    assert abs(t_act - 2 * r_half / v) < 1e-15
    assert boundary.cme_opening_angle(CME, R, t_act) < 1e-6
    # for the equidistant-run CME: 2 r_1/2 / v = 3.92 h
    assert abs(units.time_seconds(t_act) / 3600 - 3.92) < 0.01


def test_cme_distance_is_great_circle():
    rng = np.random.default_rng(5)
    th = rng.uniform(0.3, 2.8, 200)
    ph = rng.uniform(0, 2 * math.pi, 200)
    cme = dict(CME, colat_deg=70.0, lon_deg=33.0)
    d = boundary.cme_distance(cme, th, ph)
    la1, la2 = math.pi / 2 - th, math.pi / 2 - math.radians(70.0)
    dl = ph - math.radians(33.0)
    hav = np.sin((la2 - la1) / 2) ** 2 + np.cos(la1) * math.cos(la2) * np.sin(dl / 2) ** 2
    ref = 2 * np.arcsin(np.sqrt(hav))
    assert np.allclose(d, ref, atol=1e-7)


def test_cme_mask_area_grows_then_shrinks():
    th, ph = np.meshgrid(np.radians(np.linspace(30, 150, 121)), np.radians(np.linspace(-90, 90, 181)))
    R = 0.1
    _, _, t_act = boundary.cme_geometry(CME, R)
    areas = [int(boundary.cme_mask(CME, th, ph, R, t).sum()) for t in np.linspace(0, t_act, 41)]
    k = int(np.argmax(areas))
    assert 0 < k < 40
    assert all(a <= b for a, b in zip(areas[:k], areas[1:k + 1]))
    assert all(a >= b for a, b in zip(areas[k:-1], areas[k + 1:]))
    assert boundary.cme_mask(CME, th, ph, R, t_act * 1.01).sum() == 0


def test_cme_mask_cosine_form_agrees_away_from_the_edge_and_edge_ties_are_flagged():
    """Eqs. (2)-(4) compare two angles, d <= theta(t); comparing their cosines
    instead, cos d >= cos theta(t), is the same test in exact arithmetic
    (arccos decreases).  On 200,000 random boundary points over the active
    span the two forms decide alike wherever |d - theta| exceeds the near-tie
    margin; a point placed on the cone edge lands inside the margin and is
    recorded, so a parity test can refuse such a case."""
    rng = np.random.default_rng(9)
    R = 0.1
    cme = dict(CME, colat_deg=80.0, lon_deg=20.0)
    _, _, t_act = boundary.cme_geometry(cme, R)
    tc, pc = math.radians(80.0), math.radians(20.0)
    for t in np.linspace(0.05, 0.95, 7) * t_act:
        th = rng.uniform(0.2, 2.9, 200000 // 7)
        ph = rng.uniform(-math.pi, math.pi, th.size)
        del boundary.MASK_NEAR_TIES[:]
        m = boundary.cme_mask(cme, th, ph, R, t)
        theta = boundary.cme_opening_angle(cme, R, t)
        cosd = np.clip(np.sin(th) * math.sin(tc) * np.cos(ph - pc) + np.cos(th) * math.cos(tc), -1.0, 1.0)
        m_cos = cosd >= math.cos(theta)
        far = np.abs(boundary.cme_distance(cme, th, ph) - theta) >= boundary.MASK_TIE_RAD
        assert np.array_equal(m[far], m_cos[far])
        assert 0 < m.sum() < m.size
    # a point on the edge: same colatitude as the centre, longitude offset by theta(t)
    t = 0.5 * t_act
    theta = boundary.cme_opening_angle(cme, R, t)
    del boundary.MASK_NEAR_TIES[:]
    boundary.cme_mask(cme, np.array([math.pi / 2]), np.array([theta]), R, t)
    assert not boundary.MASK_NEAR_TIES                     # (centre at colatitude 80: not on the edge)
    c90 = dict(cme, colat_deg=90.0, lon_deg=0.0)
    theta = boundary.cme_opening_angle(c90, R, t)
    boundary.cme_mask(c90, np.array([math.pi / 2]), np.array([theta]), R, t)
    assert boundary.MASK_NEAR_TIES and boundary.MASK_NEAR_TIES[-1][1] == 1
    del boundary.MASK_NEAR_TIES[:]


def test_wind_harmonics_orthonormal():
    n = 200
    th = (np.arange(n) + 0.5) * math.pi / n
    ph = (np.arange(2 * n) + 0.5) * math.pi / n
    T, P = np.meshgrid(th, ph, indexing="ij")
    Y = boundary.real_harmonics(T, P)
    w = np.sin(T) * (math.pi / n) ** 2
    M = np.einsum("aij,bij,ij->ab", Y, Y, w)
    assert np.allclose(M, np.eye(15), atol=1e-4)


def test_wind_speed_range_and_density_law():
    from synthetic import Wind, as_dict
    wind = as_dict(Wind(seed=0))
    th, ph = np.meshgrid(np.radians(np.arange(181.0)), np.radians(np.arange(360.0)), indexing="ij")
    v = boundary.wind_speed_kms(wind, th, ph)
    assert abs(v.min() - 350) < 1e-9 and abs(v.max() - 700) < 1e-9
    W = boundary.wind_prims(wind, np.array([1.2]), np.array([0.4]), 0.1, units.OMEGA_CODE)
    vk = W[1, 0] * 1000.0
    assert abs(W[0, 0] - 300 * (vk / 450) ** -2) < 1e-9
    # |B| at the boundary is 300 nT and B is parallel to v in the co-rotating frame
    assert abs(math.hypot(W[5, 0], W[7, 0]) * units.B0_T * 1e9 - 300.0) < 1e-9
    assert abs(W[7, 0] / W[5, 0] - W[3, 0] / W[1, 0]) < 1e-15
