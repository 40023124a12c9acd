"""Python binding of libicarus, the MI355X library for the Icarus hot path.

Argument marshalling only: every step of the method runs in the library's
HIP kernels (paper Sect. 2.1-2.2 and 3: finite-volume ideal MHD in the
co-rotating frame on a radially stretched spherical grid with block AMR,
cone-CME inner boundary, refinement indicator).  The names follow the C ABI
in include/icarus.h (ic_create, ic_step, ...); ``Sim`` wraps one sim object.
PyTorch is used only to hand the library the current HIP stream.

torch is imported before the library is loaded so that the process holds a
single HIP runtime (torch's).  The library must have been built (``python paper_2211_12867_amd/build.py`` or
``__graft_entry__.build()``); importing fails loudly otherwise.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libicarus.so")

IC_OK, IC_E_INVALID, IC_E_NOMEM, IC_E_DEVICE, IC_E_UNPHYSICAL, IC_E_OUTSIDE, IC_E_CAPACITY, IC_E_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7
IC_GEOM_SPHERICAL, IC_GEOM_CARTESIAN = 0, 1
IC_BC_OUTFLOW, IC_BC_PERIODIC, IC_BC_INNER = 0, 1, 2
IC_FLAG_COARSEN, IC_FLAG_KEEP, IC_FLAG_REFINE = -1, 0, 1
IC_SOURCE_PLAIN, IC_SOURCE_LEARNED, IC_SOURCE_LEARNED_JUDGED = 0, 1, 2
MLP_IN, MLP_HID, MLP_NPARAM = 512, 128, 82305

OMEGA_SUN = 2.0 * math.pi / (25.38 * 86400.0)     # sidereal, rad/s
RHO_FLOOR = 1.0e-6                                  # code units
P_FLOOR = 1.0e-9
GM_SUN = 1.32712440018e20                           # m^3/s^2

_BC_NAMES = {"outflow": IC_BC_OUTFLOW, "periodic": IC_BC_PERIODIC, "inner": IC_BC_INNER}


class ICError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


class GridCfg(ctypes.Structure):
    _fields_ = [("geometry", ctypes.c_int), ("x0", ctypes.c_double * 3), ("x1", ctypes.c_double * 3),
                ("n", ctypes.c_int * 3), ("block", ctypes.c_int * 3), ("stretched_r", ctypes.c_int),
                ("max_level", ctypes.c_int), ("bc", (ctypes.c_int * 2) * 3), ("max_blocks", ctypes.c_int)]


class PhysCfg(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("omega", ctypes.c_double),
                ("gm", ctypes.c_double), ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
                ("limiter", ctypes.c_int), ("scheme", ctypes.c_int), ("divb_cd", ctypes.c_double),
                ("tracer", ctypes.c_int)]


LIMITERS = {"mc": 0, "minmod": 1, "vanleer": 2}
SCHEMES = {"two_stage": 0, "hancock": 1}
CRITERIA = {"shock": 0, "tracer": 1, "combined": 2}


class WindCfg(ctypes.Structure):
    _fields_ = [("alm", ctypes.c_double * 15), ("f_min", ctypes.c_double), ("f_max", ctypes.c_double),
                ("v_min_kms", ctypes.c_double), ("v_max_kms", ctypes.c_double),
                ("n_ref_cm3", ctypes.c_double), ("v_ref_kms", ctypes.c_double), ("T_K", ctypes.c_double),
                ("B_nT", ctypes.c_double)]


class CmeCfg(ctypes.Structure):
    _fields_ = [("t_start_s", ctypes.c_double), ("duration_s", ctypes.c_double), ("v_kms", ctypes.c_double),
                ("half_width_deg", ctypes.c_double), ("colat_deg", ctypes.c_double),
                ("lon_deg", ctypes.c_double), ("n_cm3", ctypes.c_double), ("T_K", ctypes.c_double),
                ("enabled", ctypes.c_int)]


class AmrCfg(ctypes.Structure):
    _fields_ = [("eps_lohner", ctypes.c_double), ("tol_refine", ctypes.c_double),
                ("tol_coarsen", ctypes.c_double), ("w_rho", ctypes.c_double), ("w_v", ctypes.c_double),
                ("lon_earth_deg", ctypes.c_double), ("clt_earth_deg", ctypes.c_double),
                ("dlon_earth_deg", ctypes.c_double), ("dclt_earth_deg", ctypes.c_double),
                ("dlon_cme_deg", ctypes.c_double), ("use_windows", ctypes.c_int),
                ("regrid_every", ctypes.c_int), ("buffer_blocks", ctypes.c_int), ("source", ctypes.c_int),
                ("judge_every", ctypes.c_int), ("judge_recall", ctypes.c_double),
                ("learned_threshold", ctypes.c_double), ("criterion", ctypes.c_int),
                ("tracer_refine", ctypes.c_double), ("tracer_coarsen", ctypes.c_double)]


class MlpHparams(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint), ("pos_weight", ctypes.c_float)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("waves_per_simd", ctypes.c_int), ("grid", ctypes.c_int), ("xcd_order", ctypes.c_int),
                ("stage_ms", ctypes.c_double), ("default_ms", ctypes.c_double), ("from_cache", ctypes.c_int),
                ("candidates", ctypes.c_int), ("ksplit", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_long), ("t_s", ctypes.c_double), ("dt_s", ctypes.c_double),
                ("zone_updates", ctypes.c_double), ("leaves", ctypes.c_int),
                ("leaves_per_level", ctypes.c_int * 8)]

    def as_dict(self):
        return dict(steps=self.steps, t_s=self.t_s, dt_s=self.dt_s, zone_updates=self.zone_updates,
                    leaves=self.leaves, leaves_per_level=list(self.leaves_per_level))


EXPORTS = ("ic_create", "ic_destroy", "ic_step", "ic_advance", "ic_regrid", "ic_eval_flags", "ic_eval_hot",
           "ic_eval_window", "ic_sample", "ic_set_sample_point", "ic_timeseries", "ic_timeseries_clear", "ic_get_blocks",
           "ic_get_state", "ic_set_state", "ic_get_time", "ic_units", "ic_block_supported", "ic_set_kernel_timing",
           "ic_stage_timing", "ic_pool_capacity", "ic_features", "ic_mlp_set", "ic_eval_learned",
           "ic_regrid_stats", "ic_mlp_train", "ic_mlp_grad", "ic_mlp_infer", "ic_autotune", "ic_set_tuning",
           "ic_get_tuning", "ic_floor_counts", "ic_shock_diagnostics", "ic_mlp_infer_noalloc", "ic_get_clock",
           "ic_set_clock", "ic_set_device_allocator", "ic_last_error")


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64 with the
    # same soname; loading torch first makes libicarus bind to that copy
    # instead of pulling in a second runtime from /opt/rocm.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libicarus.so is not built: run __graft_entry__.build() or "
                          "python paper_2211_12867_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.ic_create.argtypes = [P(GridCfg), P(PhysCfg), P(WindCfg), P(CmeCfg), ctypes.c_int, P(AmrCfg), vp, P(vp)]
    L.ic_destroy.argtypes = [vp]
    L.ic_destroy.restype = None
    L.ic_step.argtypes = [vp, ctypes.c_double, P(Info)]
    L.ic_advance.argtypes = [vp, ctypes.c_double, ctypes.c_long, P(Info)]
    L.ic_regrid.argtypes = [vp, P(ctypes.c_int8), P(Info)]
    L.ic_eval_flags.argtypes = [vp, ctypes.c_int, P(ctypes.c_int8), ctypes.c_int]
    L.ic_eval_hot.argtypes = [vp, ctypes.c_int, P(ctypes.c_int8), ctypes.c_int]
    L.ic_eval_window.argtypes = [vp, ctypes.c_int, P(ctypes.c_int8), ctypes.c_int]
    L.ic_sample.argtypes = [vp, ctypes.c_int] + [ctypes.c_double] * 3 + [P(ctypes.c_double)]
    L.ic_set_sample_point.argtypes = [vp] + [ctypes.c_double] * 3
    L.ic_timeseries.argtypes = [vp, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_int)]
    L.ic_timeseries_clear.argtypes = [vp]
    L.ic_get_blocks.argtypes = [vp, ctypes.c_int, P(ctypes.c_int32), P(ctypes.c_int)]
    L.ic_get_state.argtypes = [vp, ctypes.c_int, P(ctypes.c_double), ctypes.c_size_t]
    L.ic_set_state.argtypes = [vp, ctypes.c_int, P(ctypes.c_int32), ctypes.c_int, P(ctypes.c_double),
                               ctypes.c_double]
    L.ic_get_time.argtypes = [vp, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double)]
    L.ic_floor_counts.argtypes = [vp, ctypes.c_int, P(ctypes.c_long), P(ctypes.c_long)]
    L.ic_get_clock.argtypes = [vp, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_long)]
    L.ic_set_device_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
    L.ic_set_clock.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_long]
    dp = P(ctypes.c_double)
    L.ic_shock_diagnostics.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    L.ic_units.argtypes = [P(ctypes.c_double)]
    L.ic_units.restype = None
    L.ic_block_supported.argtypes = [ctypes.c_int] * 3
    L.ic_block_supported.restype = ctypes.c_int
    L.ic_set_kernel_timing.argtypes = [vp, ctypes.c_int]
    L.ic_stage_timing.argtypes = [vp, P(ctypes.c_long), P(ctypes.c_double)]
    fp, u8p, i8p = P(ctypes.c_float), P(ctypes.c_uint8), P(ctypes.c_int8)
    L.ic_features.argtypes = [vp, ctypes.c_int, fp, ctypes.c_int]
    L.ic_mlp_set.argtypes = [vp, fp, fp, fp]
    L.ic_eval_learned.argtypes = [vp, ctypes.c_int, fp, i8p, ctypes.c_int]
    L.ic_regrid_stats.argtypes = [vp, P(ctypes.c_long), P(ctypes.c_long), P(ctypes.c_long), P(ctypes.c_double)]
    L.ic_mlp_train.argtypes = [fp, u8p, ctypes.c_long, P(MlpHparams), fp, fp, fp, fp]
    L.ic_mlp_grad.argtypes = [fp, u8p, ctypes.c_int, ctypes.c_float, fp, fp, fp]
    L.ic_mlp_infer.argtypes = [fp, ctypes.c_long, fp, fp, fp, fp]
    L.ic_mlp_infer_noalloc.argtypes = [vp, ctypes.c_long, vp, vp, vp, vp, vp]
    L.ic_autotune.argtypes = [vp, ctypes.c_char_p, ctypes.c_int, P(TuneInfo)]
    L.ic_set_tuning.argtypes = [vp, P(TuneInfo)]
    L.ic_get_tuning.argtypes = [vp, P(TuneInfo)]
    L.ic_pool_capacity.argtypes = [vp]
    L.ic_pool_capacity.restype = ctypes.c_int
    L.ic_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("ic_destroy", "ic_units", "ic_block_supported", "ic_pool_capacity", "ic_last_error"):
            getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(status):
    if status != IC_OK:
        raise ICError(status, lib.ic_last_error().decode())


def units():
    out = (ctypes.c_double * 6)()
    lib.ic_units(out)
    keys = ("length_m", "speed_m_s", "time_s", "density_kg_m3", "pressure_pa", "field_t")
    return dict(zip(keys, list(out)))


def block_supported(b):
    return bool(lib.ic_block_supported(int(b[0]), int(b[1]), int(b[2])))


def _get(obj, key, default=None):
    if obj is None:
        return default
    if isinstance(obj, dict):
        return obj.get(key, default)
    return getattr(obj, key, default)


def grid_cfg(grid, max_blocks=0):
    g = GridCfg()
    geom = _get(grid, "geometry", "spherical")
    g.geometry = IC_GEOM_CARTESIAN if geom == "cartesian" else IC_GEOM_SPHERICAL
    for d in range(3):
        g.x0[d] = float(_get(grid, "x0")[d])
        g.x1[d] = float(_get(grid, "x1")[d])
        g.n[d] = int(_get(grid, "n")[d])
        g.block[d] = int(_get(grid, "block")[d])
    g.stretched_r = int(bool(_get(grid, "stretched_r", False)))
    g.max_level = int(_get(grid, "max_level", 1))
    bc = _get(grid, "bc")
    per = _get(grid, "periodic", (False, False, False))
    for d in range(3):
        for side in range(2):
            if bc is not None:
                kind = _BC_NAMES[bc[d][side]]
            elif per[d]:
                kind = IC_BC_PERIODIC
            elif g.geometry == IC_GEOM_SPHERICAL and d == 0 and side == 0:
                kind = IC_BC_INNER
            else:
                kind = IC_BC_OUTFLOW
            g.bc[d][side] = kind
    g.max_blocks = int(max_blocks)
    return g


def wind_cfg(wind):
    w = WindCfg()
    alm = _get(wind, "alm")
    for q in range(15):
        w.alm[q] = float(alm[q])
    for key in ("f_min", "f_max", "v_min_kms", "v_max_kms", "n_ref_cm3", "v_ref_kms", "T_K", "B_nT"):
        setattr(w, key, float(_get(wind, key)))
    return w


def cme_cfg(cme):
    c = CmeCfg()
    if cme is None:
        c.enabled = 0
        return c
    for key in ("t_start_s", "duration_s", "v_kms", "half_width_deg", "colat_deg", "lon_deg", "n_cm3", "T_K"):
        setattr(c, key, float(_get(cme, key)))
    c.enabled = 1
    return c


def amr_cfg(amr):
    a = AmrCfg()
    defaults = dict(eps_lohner=0.01, tol_refine=0.1, tol_coarsen=0.0125, w_rho=0.5, w_v=0.5,
                    lon_earth_deg=0.0, clt_earth_deg=90.0, dlon_earth_deg=30.0, dclt_earth_deg=10.0,
                    dlon_cme_deg=90.0, use_windows=True, regrid_every=10, buffer_blocks=1, source=0,
                    judge_every=10, judge_recall=0.9, learned_threshold=0.5,
                    tracer_refine=0.01, tracer_coarsen=0.00125)
    for key, dv in defaults.items():
        v = _get(amr, key, dv)
        setattr(a, key, int(v) if isinstance(dv, (bool, int)) and not isinstance(dv, float) else float(v))
    crit = _get(amr, "criterion", "shock")
    a.criterion = CRITERIA[crit] if isinstance(crit, str) else int(crit)
    return a


_alloc_keepalive = []      # installed callbacks stay alive: buffers go back through the one they came from
_live_sims = None


def use_torch_allocator(enable=True):
    """Route the library's device buffers through PyTorch's caching allocator
    (torch.cuda.caching_allocator_alloc / caching_allocator_delete on the
    current device and stream) -- the library's ic_set_device_allocator;
    enable=False restores hipMalloc.  Buffers keep the allocator they came
    from.  Sims still open when the interpreter exits are closed first."""
    import atexit
    import weakref
    global _live_sims
    if not enable:
        _check(lib.ic_set_device_allocator(_ALLOC_FN(), _FREE_FN(), None))
        return
    import torch

    def _alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:
            return None

    def _free(ptr, user):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass

    cbs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _alloc_keepalive.append(cbs)
    if _live_sims is None:
        _live_sims = weakref.WeakSet()
        atexit.register(lambda: [s.close() for s in list(_live_sims)])
    _check(lib.ic_set_device_allocator(cbs[0], cbs[1], None))


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return ctypes.c_void_p(0)


class Sim:
    """One library sim: n_members runs of the same grid and wind, one CME each."""

    def __init__(self, grid, wind=None, cmes=None, amr=None, omega=None, gm=None, max_blocks=0, stream=None,
                 rho_floor=RHO_FLOOR, p_floor=P_FLOOR, limiter="mc", scheme="two_stage", divb_cd=0.0,
                 tracer=False):
        self.grid = grid
        self.nv = 9 if tracer else 8
        g = grid_cfg(grid, max_blocks)
        cart = g.geometry == IC_GEOM_CARTESIAN
        p = PhysCfg(float(_get(grid, "gamma", 1.5)), float(_get(grid, "cfl", 0.4)),
                    0.0 if cart else (OMEGA_SUN if omega is None else float(omega)),
                    0.0 if cart else (GM_SUN if gm is None else float(gm)),
                    float(rho_floor), float(p_floor), LIMITERS[limiter], SCHEMES[scheme], float(divb_cd),
                    1 if tracer else 0)
        w = wind_cfg(wind) if wind is not None else None
        if cmes is None or len(cmes) == 0:
            self.n_members = 1
            carr = None
        else:
            self.n_members = len(cmes)
            carr = (CmeCfg * len(cmes))(*[cme_cfg(c) for c in cmes])
        a = amr_cfg(amr)
        self.block = tuple(int(x) for x in _get(grid, "block"))
        self.ncell = self.block[0] * self.block[1] * self.block[2]
        h = ctypes.c_void_p()
        st = stream if stream is not None else _current_stream()
        _check(lib.ic_create(ctypes.byref(g), ctypes.byref(p), ctypes.byref(w) if w is not None else None,
                             carr, self.n_members, ctypes.byref(a), st, ctypes.byref(h)))
        self.h = h
        if _live_sims is not None:
            _live_sims.add(self)

    def close(self):
        if getattr(self, "h", None):
            lib.ic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- stepping -------------------------------------------------------------
    def step(self, dt_s=0.0):
        info = Info()
        _check(lib.ic_step(self.h, float(dt_s), ctypes.byref(info)))
        return info.as_dict()

    def advance(self, dt_s, max_steps=10 ** 9):
        info = Info()
        _check(lib.ic_advance(self.h, float(dt_s), int(max_steps), ctypes.byref(info)))
        return info.as_dict()

    def regrid(self, flags=None):
        """flags: None (plain criterion) or a list per member of per-leaf flags
        in blocks() order."""
        info = Info()
        buf = None
        if flags is not None:
            cap = self._max_blocks()
            arr = np.zeros((self.n_members, cap), dtype=np.int8)
            for m, f in enumerate(flags):
                arr[m, :len(f)] = f
            buf = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
            self._keep = arr
        _check(lib.ic_regrid(self.h, buf, ctypes.byref(info)))
        return info.as_dict()

    def _max_blocks(self):
        return int(lib.ic_pool_capacity(self.h))

    def n_leaves(self, member=0):
        n = ctypes.c_int(0)
        st = lib.ic_get_blocks(self.h, member, None, ctypes.byref(n))
        if st not in (IC_OK, IC_E_INVALID):
            _check(st)
        return n.value

    def eval_flags(self, member=0):
        n = self.n_leaves(member)
        out = np.zeros(n, dtype=np.int8)
        _check(lib.ic_eval_flags(self.h, member, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n))
        return out

    def eval_hot(self, member=0):
        n = self.n_leaves(member)
        out = np.zeros(n, dtype=np.int8)
        _check(lib.ic_eval_hot(self.h, member, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n))
        return out

    def eval_window(self, member=0):
        n = self.n_leaves(member)
        out = np.zeros(n, dtype=np.int8)
        _check(lib.ic_eval_window(self.h, member, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n))
        return out

    # --- sampling ---------------------------------------------------------------
    def sample(self, r_au, colat_deg, lon_deg, member=0):
        out = (ctypes.c_double * 8)()
        _check(lib.ic_sample(self.h, member, float(r_au), float(colat_deg), float(lon_deg), out))
        return np.array(list(out))

    def set_sample_point(self, r_au, colat_deg, lon_deg):
        _check(lib.ic_set_sample_point(self.h, float(r_au), float(colat_deg), float(lon_deg)))

    def timeseries(self, member=0, cap=1 << 16):
        out = np.zeros((cap, 9))
        n = ctypes.c_int(cap)
        _check(lib.ic_timeseries(self.h, member, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 ctypes.byref(n)))
        return out[:n.value]

    def timeseries_clear(self):
        _check(lib.ic_timeseries_clear(self.h))

    # --- state exchange ---------------------------------------------------------
    def blocks(self, member=0):
        n = ctypes.c_int(0)
        st = lib.ic_get_blocks(self.h, member, None, ctypes.byref(n))
        if st not in (IC_OK, IC_E_INVALID):
            _check(st)
        arr = np.zeros((max(n.value, 1), 4), dtype=np.int32)
        n2 = ctypes.c_int(n.value)
        _check(lib.ic_get_blocks(self.h, member, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 ctypes.byref(n2)))
        return [tuple(int(x) for x in row) for row in arr[:n2.value]]

    def state(self, member=0):
        bl = self.blocks(member)
        U = np.zeros((len(bl), self.nv, self.block[2], self.block[1], self.block[0]))
        _check(lib.ic_get_state(self.h, member, U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), U.size))
        return bl, U

    def set_state(self, blocks, U, t_s=0.0, member=0):
        b = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 4))
        U = np.ascontiguousarray(np.asarray(U, dtype=np.float64))
        assert U.shape == (len(b), self.nv, self.block[2], self.block[1], self.block[0])
        _check(lib.ic_set_state(self.h, member, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(b),
                                U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(t_s)))

    def time(self, member=0):
        t, dt = ctypes.c_double(), ctypes.c_double()
        _check(lib.ic_get_time(self.h, member, ctypes.byref(t), ctypes.byref(dt)))
        return t.value, dt.value

    def clock(self, member=0):
        """(time in code units, steps since the last regrid): the exact restart clock."""
        t, n = ctypes.c_double(), ctypes.c_long()
        _check(lib.ic_get_clock(self.h, member, ctypes.byref(t), ctypes.byref(n)))
        return t.value, n.value

    def set_clock(self, t_code, since_regrid, member=0):
        _check(lib.ic_set_clock(self.h, member, float(t_code), int(since_regrid)))

    def checkpoint(self, member=0):
        """Everything a bit-exact restart of the member needs: blocks, state, clock."""
        bl, U = self.state(member)
        t_code, since = self.clock(member)
        return dict(blocks=bl, U=U, t_code=t_code, since_regrid=since)

    def restore(self, ck, member=0):
        self.set_state(ck["blocks"], ck["U"], ck["t_code"] * units()["time_s"], member)
        self.set_clock(ck["t_code"], ck["since_regrid"], member)

    def floor_counts(self, member=0):
        """(density-floored, pressure-floored) cell updates since creation."""
        a, b = ctypes.c_long(), ctypes.c_long()
        _check(lib.ic_floor_counts(self.h, member, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # --- measurement ------------------------------------------------------------
    def set_kernel_timing(self, enable):
        _check(lib.ic_set_kernel_timing(self.h, int(bool(enable))))

    def stage_timing(self):
        n, ms = ctypes.c_long(), ctypes.c_double()
        _check(lib.ic_stage_timing(self.h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    # --- schedule ------------------------------------------------------------------
    def autotune(self, cache_path=None, reps=5):
        """Pick the stage-kernel schedule (cached by device and block shape)."""
        t = TuneInfo()
        _check(lib.ic_autotune(self.h, cache_path.encode() if cache_path else None, int(reps), ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, waves_per_simd=2, grid=0, xcd_order=0, ksplit=1):
        """Force a schedule; it holds across regrids until the next autotune."""
        t = TuneInfo(waves_per_simd, grid, xcd_order, 0.0, 0.0, 0, 0, ksplit)
        _check(lib.ic_set_tuning(self.h, ctypes.byref(t)))

    def tuning(self):
        """The schedule in force: (waves_per_simd, grid, xcd_order, ksplit)."""
        t = TuneInfo()
        _check(lib.ic_get_tuning(self.h, ctypes.byref(t)))
        return (t.waves_per_simd, t.grid, t.xcd_order, t.ksplit)

    # --- learned flags ------------------------------------------------------------
    def features(self, member=0):
        n = self.n_leaves(member)
        out = np.zeros((n, MLP_IN), dtype=np.float32)
        _check(lib.ic_features(self.h, member, _fptr(out), n))
        return out

    def mlp_set(self, params, mean, std):
        self._mlp = [np.ascontiguousarray(params, dtype=np.float32), np.ascontiguousarray(mean, dtype=np.float32),
                     np.ascontiguousarray(std, dtype=np.float32)]
        _check(lib.ic_mlp_set(self.h, *[_fptr(a) for a in self._mlp]))

    def eval_learned(self, member=0):
        n = self.n_leaves(member)
        prob = np.zeros(n, dtype=np.float32)
        flags = np.zeros(n, dtype=np.int8)
        _check(lib.ic_eval_learned(self.h, member, _fptr(prob), flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), n))
        return prob, flags

    def regrid_stats(self):
        v = [ctypes.c_long(), ctypes.c_long(), ctypes.c_long(), ctypes.c_double()]
        _check(lib.ic_regrid_stats(self.h, *[ctypes.byref(x) for x in v]))
        return dict(learned=v[0].value, judged=v[1].value, fallbacks=v[2].value, last_recall=v[3].value)


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def mlp_train(raw, y, params, epochs=10, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0,
              pos_weight=0.0):
    """Train the learned-flag network on the GPU; returns (params, mean, std, loss per epoch)."""
    raw = np.ascontiguousarray(raw, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    params = np.array(params, dtype=np.float32, copy=True)
    mean = np.zeros(MLP_IN, dtype=np.float32)
    std = np.zeros(MLP_IN, dtype=np.float32)
    loss = np.zeros(max(epochs, 1), dtype=np.float32)
    hp = MlpHparams(epochs, batch, lr, beta1, beta2, eps, seed, pos_weight)
    _check(lib.ic_mlp_train(_fptr(raw), y.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), len(y), ctypes.byref(hp),
                            _fptr(params), _fptr(mean), _fptr(std), _fptr(loss)))
    return params, mean, std, loss[:epochs]


def mlp_grad(xnorm, y, params, pos_weight=1.0):
    """Gradient of the mean weighted BCE on the GPU for already normalised inputs."""
    xnorm = np.ascontiguousarray(xnorm, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    params = np.ascontiguousarray(params, dtype=np.float32)
    grad = np.zeros(MLP_NPARAM, dtype=np.float32)
    loss = ctypes.c_float()
    _check(lib.ic_mlp_grad(_fptr(xnorm), y.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), len(y),
                           float(pos_weight), _fptr(params), _fptr(grad), ctypes.byref(loss)))
    return grad, loss.value


def mlp_infer(raw, params, mean, std):
    """Network probabilities of rows of raw inputs on the GPU."""
    raw = np.ascontiguousarray(raw, dtype=np.float32)
    prob = np.zeros(len(raw), dtype=np.float32)
    ps = [np.ascontiguousarray(a, dtype=np.float32) for a in (params, mean, std)]
    _check(lib.ic_mlp_infer(_fptr(raw), len(raw), *[_fptr(a) for a in ps], _fptr(prob)))
    return prob


MLP_NOALLOC_ROWS = 4096


def mlp_infer_noalloc(raw_dev, n, params_dev, mean_dev, std_dev, prob_dev, stream=None):
    """ic_mlp_infer_noalloc on device arrays given by address (e.g. a torch
    tensor's data_ptr()); enqueued on stream (default: torch's current
    stream), no synchronisation and no allocation."""
    st = stream if stream is not None else _current_stream()
    _check(lib.ic_mlp_infer_noalloc(ctypes.c_void_p(raw_dev), int(n), ctypes.c_void_p(params_dev),
                                    ctypes.c_void_p(mean_dev), ctypes.c_void_p(std_dev), ctypes.c_void_p(prob_dev), st))


def mlp_init(seed=0):
    """He-uniform initial parameters (fp32) in the library's parameter layout."""
    g = np.random.default_rng(seed)
    p = np.zeros(MLP_NPARAM, dtype=np.float32)
    o = 0
    for fan_in, fan_out in ((MLP_IN, MLP_HID), (MLP_HID, MLP_HID), (MLP_HID, 1)):
        lim = math.sqrt(6.0 / fan_in)
        p[o:o + fan_in * fan_out] = g.uniform(-lim, lim, fan_in * fan_out)
        o += fan_in * fan_out + fan_out
    return p


def shock_diagnostics(t_s, v, t_cme_s, window_s=96 * 3600.0, min_jump=0.0):
    """ic_shock_diagnostics: dict(arrival_s, width_s, v_pre, v_max, gradient,
    t_top_s, v_top, t_max_s) of a radial-speed series (times in s, speeds in
    any unit)."""
    t = np.ascontiguousarray(t_s, dtype=np.float64)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    if t.shape != vv.shape or t.ndim != 1:
        raise ValueError("t_s and v must be 1-D arrays of one length")
    out = (ctypes.c_double * 8)()
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.ic_shock_diagnostics(t.ctypes.data_as(dp), vv.ctypes.data_as(dp), len(t), float(t_cme_s),
                                    float(window_s), float(min_jump), out))
    keys = ("arrival_s", "width_s", "v_pre", "v_max", "gradient", "t_top_s", "v_top", "t_max_s")
    return dict(zip(keys, list(out)))


def arrival(t_h, v, t_cme_h, window_h=96.0, min_jump=0.0):
    """Shock arrival after the CME start [h] and width [h] of a v_r series with
    times in hours (ic_shock_diagnostics); (nan, nan) without an arrival."""
    d = shock_diagnostics(np.asarray(t_h, dtype=np.float64) * 3600.0, v, t_cme_h * 3600.0, window_h * 3600.0,
                          min_jump)
    return d["arrival_s"] / 3600.0, d["width_s"] / 3600.0
