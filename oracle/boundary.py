"""Inner-boundary driving of the oracle: seeded wind + cone CME (test infrastructure only).

Paper Sect. 2.1: the wind is super-sonic at the inner boundary (0.1 AU);
plasma variables are prescribed there and held constant in the co-rotating
frame (no differential rotation).  A cone CME enters by changing the inner
boundary values inside the region where the CME sphere crosses the boundary
shell, Eqs. (1)-(4):
    r_1/2   = R sin(omega_CME / 2)                              (1)
    theta(t)= arccos((R_c^2 + R^2 - r_1/2^2) / (2 R_c R))       (2)
    R_c(t)  = t v_CME + R - r_1/2                               (3)
    d       = arccos(sin th_p sin th_CME cos(ph_p - ph_CME)
                      + cos th_p cos th_CME)                    (4)
and a boundary point p is inside the CME when d <= theta(t).

Readings (the paper leaves these open): both ghost layers take the boundary
state of their own (theta, phi) evaluated at r_in; the wind is radial in the
inertial frame, so v_phi = -Omega r_in sin(theta) in the co-rotating frame;
B is a unipolar Parker field parallel to v in that frame; p = 2 n k_B T;
inside the CME: n_CME, T_CME, v_r = v_CME, the same v_phi, the ambient B.
The mask is active for 0 <= t - t_CME <= min(T_inj, 2 r_1/2 / v_CME), the
time in which Eqs. (1)-(3) keep the sphere crossing the shell.
"""
import math

import numpy as np

from . import units

NV = 8


def real_harmonics(theta, phi):
    """Orthonormal real spherical harmonics l = 1..3, no Condon-Shortley phase,
    (l, m) order with m = -l..l; m > 0 -> cos(m phi), m < 0 -> sin(|m| phi)."""
    theta, phi = np.broadcast_arrays(np.asarray(theta, dtype=np.float64),
                                     np.asarray(phi, dtype=np.float64))
    x, s = np.cos(theta), np.sin(theta)
    legendre = {
        (1, 0): x, (1, 1): s,
        (2, 0): (3.0 * x * x - 1.0) / 2.0, (2, 1): 3.0 * x * s, (2, 2): 3.0 * s * s,
        (3, 0): (5.0 * x ** 3 - 3.0 * x) / 2.0, (3, 1): 1.5 * (5.0 * x * x - 1.0) * s,
        (3, 2): 15.0 * x * s * s, (3, 3): 15.0 * s ** 3,
    }
    rows = []
    for l in (1, 2, 3):
        for m in range(-l, l + 1):
            a = abs(m)
            N = math.sqrt((2 * l + 1) / (4.0 * math.pi) * math.factorial(l - a) / math.factorial(l + a))
            if m == 0:
                rows.append(N * legendre[(l, 0)])
            elif m > 0:
                rows.append(math.sqrt(2.0) * N * legendre[(l, a)] * np.cos(a * phi))
            else:
                rows.append(math.sqrt(2.0) * N * legendre[(l, a)] * np.sin(a * phi))
    return np.array(rows)


def wind_speed_kms(wind, theta, phi):
    f = np.tensordot(np.asarray(wind["alm"], dtype=np.float64), real_harmonics(theta, phi), axes=1)
    vmin, vmax = wind["v_min_kms"], wind["v_max_kms"]
    if wind["f_max"] <= wind["f_min"]:
        return np.full(np.shape(f), vmin)
    v = vmin + (vmax - vmin) * (f - wind["f_min"]) / (wind["f_max"] - wind["f_min"])
    return np.clip(v, vmin, vmax)


def wind_prims(wind, theta, phi, r_in, omega):
    """Primitive state W of the wind at boundary points (theta, phi), code units.
    Returns an array [8, ...]."""
    theta, phi = np.broadcast_arrays(np.asarray(theta, dtype=np.float64),
                                     np.asarray(phi, dtype=np.float64))
    vk = wind_speed_kms(wind, theta, phi)
    n = wind["n_ref_cm3"] * (vk / wind["v_ref_kms"]) ** -2
    vr = units.speed_code(vk)
    vp = -omega * r_in * np.sin(theta)
    Bmag = units.field_code(wind["B_nT"])
    br = Bmag / np.sqrt(1.0 + (vp / vr) ** 2)
    bp = br * vp / vr
    W = np.zeros((NV,) + np.shape(theta))
    W[0] = units.density_code(n)
    W[1] = vr
    W[3] = vp
    W[4] = units.pressure_code(n, wind["T_K"])
    W[5] = br
    W[7] = bp
    return W


def cme_geometry(cme, r_in):
    """(r_1/2 [code], v [code], active duration [code]) of a cone CME."""
    half = math.radians(cme["half_width_deg"])
    R = r_in
    r_half = R * math.sin(half)                          # Eq. (1), omega/2 = half-width
    v = units.speed_code(cme["v_kms"])
    t_geo = 2.0 * r_half / v                             # sphere fully through the shell
    return r_half, v, min(units.time_code(cme["duration_s"]), t_geo)


def cme_opening_angle(cme, r_in, tau):
    """theta(t) of Eq. (2) at time tau after the CME start (code units)."""
    r_half, v, _ = cme_geometry(cme, r_in)
    R = r_in
    Rc = tau * v + R - r_half                            # Eq. (3)
    arg = (Rc * Rc + R * R - r_half * r_half) / (2.0 * Rc * R)
    return math.acos(min(1.0, max(-1.0, arg)))


def cme_distance(cme, theta, phi):
    """Angular distance d of Eq. (4) from boundary points to the CME centre."""
    tc, pc = math.radians(cme["colat_deg"]), math.radians(cme["lon_deg"])
    arg = np.sin(theta) * math.sin(tc) * np.cos(phi - pc) + np.cos(theta) * math.cos(tc)
    return np.arccos(np.clip(arg, -1.0, 1.0))


# Boundary points whose angular distance lies within MASK_TIE_RAD of the
# opening angle: there the decision d <= theta(t) rests on the last bits of
# two arccos evaluations (an implementation comparing the cosines, or
# computing them in another order, may decide the other way), so parity tests
# check that none occurred.  Entries (t, count) are appended by cme_mask.
MASK_TIE_RAD = 1e-10
MASK_NEAR_TIES = []


def cme_mask(cme, theta, phi, r_in, t):
    """Boolean mask of boundary points inside the CME at code time t."""
    tau = t - units.time_code(cme["t_start_s"])
    _, _, t_act = cme_geometry(cme, r_in)
    shape = np.shape(theta)
    if not (0.0 <= tau <= t_act):
        return np.zeros(shape, dtype=bool)
    d = cme_distance(cme, theta, phi)
    th = cme_opening_angle(cme, r_in, tau)
    near = int(np.count_nonzero(np.abs(d - th) < MASK_TIE_RAD))
    if near:
        MASK_NEAR_TIES.append((t, near))
    return d <= th


def boundary_prims(wind, cme, theta, phi, r_in, omega, t):
    """Inner-boundary primitive state at (theta, phi) and code time t."""
    theta, phi = np.broadcast_arrays(np.asarray(theta, dtype=np.float64),
                                     np.asarray(phi, dtype=np.float64))
    W = wind_prims(wind, theta, phi, r_in, omega)
    if cme is None:
        return W
    m = cme_mask(cme, theta, phi, r_in, t)
    if np.any(m):
        rho_c = units.density_code(cme["n_cm3"])
        p_c = units.pressure_code(cme["n_cm3"], cme["T_K"])
        W[0] = np.where(m, rho_c, W[0])
        W[1] = np.where(m, units.speed_code(cme["v_kms"]), W[1])
        W[4] = np.where(m, p_c, W[4])
    return W


def initial_prims(wind, r, theta, phi, r_in, omega, gamma):
    """Starting state for the relaxation (arrays broadcast over r, theta, phi):
    rho ~ (r_in/r)^2, v_r constant along rays, p ~ (r_in/r)^(2 gamma),
    B_r ~ (r_in/r)^2, v_phi = -Omega r sin(theta), B_phi = B_r v_phi / v_r."""
    r, theta, phi = np.broadcast_arrays(np.asarray(r, dtype=np.float64),
                                        np.asarray(theta, dtype=np.float64),
                                        np.asarray(phi, dtype=np.float64))
    Wb = wind_prims(wind, theta, phi, r_in, omega)
    x = r_in / r
    W = np.zeros((NV,) + r.shape)
    W[0] = Wb[0] * x * x
    W[1] = Wb[1] + 0.0 * x
    W[3] = -omega * r * np.sin(theta)
    W[4] = Wb[4] * x ** (2.0 * gamma)
    W[5] = Wb[5] * x * x
    with np.errstate(divide="ignore", invalid="ignore"):
        W[7] = np.where(W[5] != 0.0, W[5] * W[3] / W[1], 0.0)
    return W


def prims_to_cons(W, gamma):
    rho = W[0]
    U = np.empty_like(W)
    U[0] = rho
    U[1:4] = rho * W[1:4]
    v2 = W[1] ** 2 + W[2] ** 2 + W[3] ** 2
    b2 = W[5] ** 2 + W[6] ** 2 + W[7] ** 2
    U[4] = W[4] / (gamma - 1.0) + 0.5 * rho * v2 + 0.5 * b2
    U[5:8] = W[5:8]
    if len(W) > 8:
        U[8] = rho * W[8]              # density tracer rho s
    return U


def cons_to_prims(U, gamma):
    rho = U[0]
    W = np.empty_like(U)
    W[0] = rho
    W[1:4] = U[1:4] / rho
    v2 = W[1] ** 2 + W[2] ** 2 + W[3] ** 2
    b2 = U[5] ** 2 + U[6] ** 2 + U[7] ** 2
    W[4] = (gamma - 1.0) * (U[4] - 0.5 * rho * v2 - 0.5 * b2)
    W[5:8] = U[5:8]
    if len(U) > 8:
        W[8] = U[8] / rho              # CME mass fraction s
    return W
