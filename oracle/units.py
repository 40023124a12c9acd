"""Physical constants and code units of the oracle (test infrastructure only).

Code units: length L0 = 1 AU, speed v0 = 1000 km/s, time t0 = L0/v0,
density rho0 = m_p * 1 cm^-3, pressure p0 = rho0 v0^2, magnetic field
B0 = sqrt(mu0 rho0 v0^2) (so mu0 = 1 in the equations).
The paper works in the Sun's co-rotating frame (Sect. 2.1); the sidereal
rotation period 25.38 d is taken, with the rotation axis at colatitude 0.
"""
import math

AU_M = 1.495978707e11
RSUN_M = 6.957e8
V0 = 1.0e6                       # m/s
T0 = AU_M / V0                   # s
MP = 1.67262192e-27              # kg
KB = 1.380649e-23                # J/K
MU0 = 4.0e-7 * math.pi
RHO0 = MP * 1.0e6                # kg/m^3 (1 proton per cm^3)
P0 = RHO0 * V0 * V0              # Pa
B0_T = math.sqrt(MU0 * P0)       # T
GM_SI = 1.32712440018e20         # m^3/s^2
OMEGA_SI = 2.0 * math.pi / (25.38 * 86400.0)

GM_CODE = GM_SI / (AU_M * V0 * V0)
OMEGA_CODE = OMEGA_SI * T0
AU_IN_RSUN = AU_M / RSUN_M


def density_code(n_cm3):
    """rho = n m_p (no helium)."""
    return n_cm3 * 1.0e6 * MP / RHO0


def pressure_code(n_cm3, T_K):
    """p = 2 n k_B T (electrons and protons at the same temperature)."""
    return 2.0 * n_cm3 * 1.0e6 * KB * T_K / P0


def speed_code(v_kms):
    return v_kms * 1.0e3 / V0


def field_code(B_nT):
    return B_nT * 1.0e-9 / B0_T


def time_code(t_s):
    return t_s / T0


def time_seconds(t_code):
    return t_code * T0
