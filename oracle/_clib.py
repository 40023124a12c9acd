"""ctypes binding of the oracle's C core (test infrastructure only)."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

NV = 8


def build(force=True):
    """Compile the oracle with gcc: -O2, no FMA contraction, OpenMP."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c99", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


class Patch(ctypes.Structure):
    _fields_ = [("ni", ctypes.c_int), ("nj", ctypes.c_int), ("nk", ctypes.c_int),
                ("cartesian", ctypes.c_int),
                ("f0", ctypes.POINTER(ctypes.c_double)),
                ("f1", ctypes.POINTER(ctypes.c_double)),
                ("f2", ctypes.POINTER(ctypes.c_double)),
                ("gamma", ctypes.c_double), ("omega", ctypes.c_double), ("gm", ctypes.c_double),
                ("limiter", ctypes.c_int), ("nv", ctypes.c_int)]

LIMITERS = {"mc": 0, "minmod": 1, "vanleer": 2}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Patch)
        L.ora_prim.argtypes = [dp, dp, ctypes.c_double]
        L.ora_cons.argtypes = [dp, dp, ctypes.c_double]
        L.ora_fast_speed.argtypes = [dp, ctypes.c_int, ctypes.c_double]
        L.ora_fast_speed.restype = ctypes.c_double
        L.ora_flux.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp]
        L.ora_rusanov.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, dp]
        L.ora_mc_slope.argtypes = [ctypes.c_double] * 6
        L.ora_mc_slope.restype = ctypes.c_double
        L.ora_slope.argtypes = [ctypes.c_int] + [ctypes.c_double] * 6
        L.ora_slope.restype = ctypes.c_double
        L.ora_rhs_hancock.argtypes = [pp, dp, dp]
        L.ora_divb.argtypes = [pp, dp, dp]
        L.ora_divb.restype = None
        L.ora_rhs_hancock.restype = ctypes.c_int
        L.ora_sources.argtypes = [dp] + [ctypes.c_double] * 7 + [dp]
        L.ora_rhs.argtypes = [pp, dp, dp, dp, dp, dp]
        L.ora_rhs.restype = ctypes.c_int
        L.ora_max_rate.argtypes = [pp, dp]
        L.ora_max_rate.restype = ctypes.c_double
        L.ora_indicator.argtypes = [pp, dp, ctypes.c_double, dp, dp, dp, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def prim(u, gamma):
    u = _vec(u); w = np.empty(NV)
    lib().ora_prim(_p(u), _p(w), gamma)
    return w


def cons(w, gamma):
    w = _vec(w); u = np.empty(NV)
    lib().ora_cons(_p(w), _p(u), gamma)
    return u


def fast_speed(w, d, gamma):
    w = _vec(w)
    return lib().ora_fast_speed(_p(w), d, gamma)


def flux(w, d, gamma):
    w = _vec(w); f = np.empty(NV)
    lib().ora_flux(_p(w), d, gamma, _p(f))
    return f


def rusanov(wl, wr, d, gamma):
    wl = _vec(wl); wr = _vec(wr); f = np.empty(NV)
    lib().ora_rusanov(_p(wl), _p(wr), d, gamma, _p(f))
    return f


def sources(w, rtinv, ctil, rc, sc, cc, omega, gm):
    w = _vec(w); S = np.empty(NV)
    lib().ora_sources(_p(w), rtinv, ctil, rc, sc, cc, omega, gm, _p(S))
    return S


def mc_slope(wm, w0, wp, xm, x0, xp):
    return lib().ora_mc_slope(wm, w0, wp, xm, x0, xp)


def slope(limiter, wm, w0, wp, xm, x0, xp):
    return lib().ora_slope(LIMITERS[limiter], wm, w0, wp, xm, x0, xp)


class PatchGeom:
    """Keeps the face arrays alive for a Patch struct."""

    def __init__(self, f0, f1, f2, cartesian, gamma, omega, gm, limiter="mc", nv=NV):
        self.f = [_vec(f0), _vec(f1), _vec(f2)]
        self.n = tuple(len(a) - 5 for a in self.f)
        self.nv = nv
        self.s = Patch(self.n[0], self.n[1], self.n[2], 1 if cartesian else 0,
                       _p(self.f[0]), _p(self.f[1]), _p(self.f[2]), gamma, omega, gm, LIMITERS[limiter], nv)


def rhs(pg, G, want_fluxes=True):
    """L(U) of a ghosted patch G [nv, nk+4, nj+4, ni+4].  Returns (L, (F0, F1, F2), n_bad)."""
    ni, nj, nk = pg.n
    nv = pg.nv
    G = np.ascontiguousarray(G, dtype=np.float64)
    assert G.shape == (nv, nk + 4, nj + 4, ni + 4)
    L = np.empty((nv, nk, nj, ni))
    F0 = np.empty((nv, nk, nj, ni + 1))
    F1 = np.empty((nv, nk, nj + 1, ni))
    F2 = np.empty((nv, nk + 1, nj, ni))
    bad = lib().ora_rhs(ctypes.byref(pg.s), _p(G), _p(L), _p(F0), _p(F1), _p(F2))
    return L, (F0, F1, F2), bad


def rhs_hancock(pg, G):
    """Hancock predictor operator of a ghosted patch.  Returns (L, n_bad)."""
    ni, nj, nk = pg.n
    G = np.ascontiguousarray(G, dtype=np.float64)
    assert G.shape == (pg.nv, nk + 4, nj + 4, ni + 4)
    L = np.empty((pg.nv, nk, nj, ni))
    bad = lib().ora_rhs_hancock(ctypes.byref(pg.s), _p(G), _p(L))
    return L, bad


def divb(pg, G):
    """Discrete div B of the interior cells of a ghosted patch, [nk, nj, ni]."""
    ni, nj, nk = pg.n
    G = np.ascontiguousarray(G, dtype=np.float64)
    D = np.empty((nk, nj, ni))
    lib().ora_divb(ctypes.byref(pg.s), _p(G), _p(D))
    return D


def max_rate(pg, G):
    G = np.ascontiguousarray(G, dtype=np.float64)
    return lib().ora_max_rate(ctypes.byref(pg.s), _p(G))


def indicator(pg, G, eps):
    ni, nj, nk = pg.n
    G = np.ascontiguousarray(G, dtype=np.float64)
    out = [np.empty((nk, nj, ni)) for _ in range(4)]
    lib().ora_indicator(ctypes.byref(pg.s), _p(G), eps, *[_p(o) for o in out])
    return out
