"""Seeded synthetic inputs for the Icarus hot path.

This module only draws random numbers and states workload shapes.  It holds
none of the solver's arithmetic (no fluxes, limiters, geometry or boundary
physics), so both the CPU oracle and the HIP library's tests can take their
inputs from here without sharing any method code.

The paper's solar wind comes from the WSA coronal model for a real event
(Sect. 2.1); that data is not available, so a seeded, smooth wind-speed map
stands in for it:

    f(theta, phi) = sum_{l=1..3} sum_{m=-l..l} a_lm Y_lm(theta, phi)
    v_r = v_min + (v_max - v_min) (f - f_min) / (f_max - f_min)

with a_lm ~ N(0, 1) drawn by ``numpy.random.default_rng(seed)`` in (l, m)
order, Y_lm the orthonormal real spherical harmonics without the
Condon-Shortley phase, and (f_min, f_max) taken over a 1-degree full-sphere
grid of 181 x 360 points.  The map itself is part of the *input*; each
consumer evaluates it from (a_lm, f_min, f_max) with its own code.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List, Optional

import numpy as np

N_ALM = 15  # l = 1..3, m = -l..l


def wind_coefficients(seed: int) -> np.ndarray:
    """The 15 harmonic coefficients a_lm of the seeded wind, (l, m) order."""
    return np.random.default_rng(seed).standard_normal(N_ALM)


def _real_harmonics(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Y_lm for l=1..3 (orthonormal, no Condon-Shortley phase), shape (15, ...).

    Generator-side evaluation used only to fix the normalisation range.
    """
    x = np.cos(theta)
    s = np.sin(theta)
    # associated Legendre P_l^m(x) for m >= 0 without the (-1)^m phase
    P = {
        (1, 0): x, (1, 1): s,
        (2, 0): 0.5 * (3 * x * x - 1), (2, 1): 3 * x * s, (2, 2): 3 * s * s,
        (3, 0): 0.5 * (5 * x ** 3 - 3 * x), (3, 1): 1.5 * (5 * x * x - 1) * s,
        (3, 2): 15 * x * s * s, (3, 3): 15 * s ** 3,
    }
    out = []
    for l in (1, 2, 3):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                out.append(norm * P[(l, 0)])
            elif m > 0:
                out.append(math.sqrt(2) * norm * P[(l, am)] * np.cos(am * phi))
            else:
                out.append(math.sqrt(2) * norm * P[(l, am)] * np.sin(am * phi))
    return np.array(out)


def wind_range(alm: np.ndarray) -> tuple:
    """(f_min, f_max) of the harmonic sum over the 1-degree 181 x 360 grid."""
    th = np.radians(np.arange(181.0))
    ph = np.radians(np.arange(360.0))
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    f = np.tensordot(np.asarray(alm, dtype=np.float64), _real_harmonics(T, Ph), axes=1)
    return float(f.min()), float(f.max())


@dataclass
class Wind:
    """Inner-boundary wind at 0.1 AU (stand-in for the coronal model output)."""
    seed: int = 0
    alm: Optional[List[float]] = None
    f_min: float = 0.0
    f_max: float = 0.0
    v_min_kms: float = 350.0
    v_max_kms: float = 700.0
    n_ref_cm3: float = 300.0      # n = n_ref (v_r / v_ref)^-2
    v_ref_kms: float = 450.0
    T_K: float = 1.0e6
    B_nT: float = 300.0

    def __post_init__(self):
        if self.alm is None:
            a = wind_coefficients(self.seed)
            self.alm = [float(v) for v in a]
            self.f_min, self.f_max = wind_range(a)


def uniform_wind(v_kms: float, n_cm3: float, T_K: float, B_nT: float = 0.0) -> Wind:
    """A wind with the same state at every boundary point (tests)."""
    return Wind(seed=-1, alm=[0.0] * N_ALM, f_min=0.0, f_max=0.0,
                v_min_kms=v_kms, v_max_kms=v_kms, n_ref_cm3=n_cm3, v_ref_kms=v_kms,
                T_K=T_K, B_nT=B_nT)


@dataclass
class Cme:
    """Cone-CME parameters (Eqs. 1-4 geometry; ABI units)."""
    t_start_s: float = 0.0
    duration_s: float = 6 * 3600.0
    v_kms: float = 1200.0
    half_width_deg: float = 30.0
    colat_deg: float = 90.0
    lon_deg: float = 45.0
    n_cm3: float = 1200.0
    T_K: float = 0.8e6


def cme_ensemble(n: int = 32, seed0: int = 1000, t_start_s: float = 0.0) -> List[Cme]:
    """Ensemble members: speed U(800,2000) km/s, half-width U(30,70) deg,
    latitude and longitude offsets U(-20,20) deg, density U(600,2400) cm^-3,
    drawn in that order from default_rng(seed0 + m).  T = 0.8 MK, 8 h cap,
    centre (90 deg - lat, 0 deg + lon)."""
    out = []
    for m in range(n):
        g = np.random.default_rng(seed0 + m)
        v = g.uniform(800.0, 2000.0)
        hw = g.uniform(30.0, 70.0)
        lat = g.uniform(-20.0, 20.0)
        lon = g.uniform(-20.0, 20.0)
        dens = g.uniform(600.0, 2400.0)
        out.append(Cme(t_start_s=t_start_s, duration_s=8 * 3600.0, v_kms=float(v),
                       half_width_deg=float(hw), colat_deg=90.0 - float(lat),
                       lon_deg=float(lon) % 360.0, n_cm3=float(dens), T_K=0.8e6))
    return out


def smooth_modes(seed: int, n_modes: int = 3, amp: float = 1.0):
    """Random Fourier modes (k vector in integers, amplitude, phase) for a
    smooth periodic perturbation; the consumer evaluates them on its grid."""
    g = np.random.default_rng(seed)
    ks = g.integers(-2, 3, size=(n_modes, 3))
    ks[np.all(ks == 0, axis=1)] = (1, 0, 0)
    amps = amp * g.uniform(0.2, 1.0, size=n_modes)
    phases = g.uniform(0.0, 2 * math.pi, size=n_modes)
    return ks, amps, phases


def random_normal(seed: int, shape) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape)


def random_uniform(seed: int, shape, lo=0.0, hi=1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


# ---------------------------------------------------------------------------
# Workloads (shapes and parameters of the paper's runs, stated as data)
# ---------------------------------------------------------------------------

@dataclass
class Grid:
    geometry: str = "spherical"        # or "cartesian"
    x0: tuple = (0.1, 60.0, 0.0)       # r [AU], colatitude [deg], longitude [deg]
    x1: tuple = (1.1, 120.0, 90.0)
    n: tuple = (48, 12, 24)            # base-level cells (r, theta, phi)
    block: tuple = (12, 12, 12)        # cells per block
    stretched_r: bool = False
    max_level: int = 1
    periodic: tuple = (False, False, False)
    gamma: float = 1.5
    cfl: float = 0.4


@dataclass
class Amr:
    eps_lohner: float = 0.01
    tol_refine: float = 0.1
    tol_coarsen: float = 0.0125        # tol_refine / 8
    w_rho: float = 0.5
    w_v: float = 0.5
    lon_earth_deg: float = 0.0
    clt_earth_deg: float = 90.0
    dlon_earth_deg: float = 30.0
    dclt_earth_deg: float = 10.0
    dlon_cme_deg: float = 90.0
    use_windows: bool = True
    regrid_every: int = 10
    buffer_blocks: int = 1


@dataclass
class Workload:
    name: str
    grid: Grid
    wind: Wind
    cmes: List[Cme]
    amr: Amr = field(default_factory=Amr)
    steps: int = 50
    relax_s: float = 0.0
    cme_phase_s: float = 0.0
    sample_point: tuple = (1.0, 90.0, 0.0)
    omega_on: bool = True
    gravity_on: bool = True


DAY = 86400.0


def workload(name: str) -> Workload:
    """The paper-shaped workloads; see the module docstring for the wind."""
    if name == "tiny_wedge":
        return Workload(
            name, Grid(x0=(0.1, 60.0, 0.0), x1=(1.1, 120.0, 90.0), n=(48, 12, 24),
                       block=(12, 12, 12)),
            Wind(seed=0),
            [Cme(t_start_s=0.0, duration_s=6 * 3600.0, v_kms=1200.0, half_width_deg=30.0,
                 colat_deg=90.0, lon_deg=45.0, n_cm3=1200.0, T_K=0.8e6)],
            steps=50)
    if name == "equidistant_full":
        return Workload(
            name, Grid(x0=(0.1, 30.0, 0.0), x1=(2.0, 150.0, 360.0), n=(512, 60, 180),
                       block=(16, 12, 12), periodic=(False, False, True)),
            Wind(seed=0),
            [Cme(t_start_s=14 * DAY, duration_s=8 * 3600.0, v_kms=1500.0, half_width_deg=45.0,
                 colat_deg=90.0, lon_deg=0.0, n_cm3=1200.0, T_K=0.8e6)],
            steps=50, relax_s=14 * DAY, cme_phase_s=3 * DAY)
    if name == "stretched_amr":
        return Workload(
            name, Grid(x0=(0.1, 30.0, 0.0), x1=(2.0, 150.0, 360.0), n=(60, 24, 48),
                       block=(12, 12, 12), stretched_r=True, max_level=4,
                       periodic=(False, False, True)),
            Wind(seed=0),
            [Cme(t_start_s=14 * DAY, duration_s=8 * 3600.0, v_kms=1500.0, half_width_deg=45.0,
                 colat_deg=90.0, lon_deg=0.0, n_cm3=1200.0, T_K=0.8e6)],
            steps=50, relax_s=14 * DAY, cme_phase_s=3 * DAY)
    if name == "ensemble":
        w = workload("stretched_amr")
        w.name = name
        w.grid.max_level = 3
        w.cmes = cme_ensemble(32, 1000, t_start_s=14 * DAY)
        return w
    if name == "learned_flags":
        w = workload("stretched_amr")
        w.name = name
        w.grid.max_level = 5
        w.amr.buffer_blocks = 0
        return w
    raise KeyError(name)


WORKLOADS = ("tiny_wedge", "equidistant_full", "stretched_amr", "ensemble", "learned_flags")


def as_dict(obj) -> dict:
    return asdict(obj)
