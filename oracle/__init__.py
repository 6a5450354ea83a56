"""ctypes front end of the FP64 CPU oracle (``btrirt_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check and
by the benchmark's CPU-baseline leg.  The product library never imports it.

The oracle evolves the enthalpy populations ``g`` and the Boussinesq flow
populations ``f`` of a D2Q9 lattice with the block triple-relaxation-time update
(Sec. 2, Eq. (2)), the enthalpy equilibrium of Eq. (3) and the rate relations of
Eqs. (4)-(5), in a cavity with a heated bottom strip (Sec. 3.2).
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

Q = 9
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)

PARAM_DIMENSIONLESS = 0
PARAM_LATTICE = 1
SOLID_SCALE, SOLID_DARCY, SOLID_PBB = 0, 1, 2


class Case(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("periodic_x", ctypes.c_int), ("periodic_y", ctypes.c_int),
        ("param_mode", ctypes.c_int),
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("Ste", ctypes.c_double), ("Ma", ctypes.c_double),
        ("nu", ctypes.c_double), ("alpha", ctypes.c_double), ("gbeta", ctypes.c_double), ("latent", ctypes.c_double),
        ("Cp", ctypes.c_double), ("Th", ctypes.c_double), ("Tm", ctypes.c_double), ("rho0", ctypes.c_double),
        ("heater_center", ctypes.c_double), ("heater_width", ctypes.c_double),
        ("k0_g", ctypes.c_double), ("k2_g", ctypes.c_double),
        ("k0_f", ctypes.c_double), ("k1_f", ctypes.c_double),
        ("solid_model", ctypes.c_int), ("darcy_c", ctypes.c_double), ("darcy_eps", ctypes.c_double),
    ]


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("periodic_x", ctypes.c_int), ("periodic_y", ctypes.c_int),
        ("nu", ctypes.c_double), ("alpha", ctypes.c_double), ("gbeta", ctypes.c_double), ("latent", ctypes.c_double),
        ("Cp", ctypes.c_double), ("Th", ctypes.c_double), ("Tm", ctypes.c_double), ("rho0", ctypes.c_double),
        ("k0_g", ctypes.c_double), ("k1_g", ctypes.c_double), ("k2_g", ctypes.c_double),
        ("k0_f", ctypes.c_double), ("k1_f", ctypes.c_double), ("k2_f", ctypes.c_double),
        ("heater_lo", ctypes.c_int), ("heater_hi", ctypes.c_int), ("n_heater", ctypes.c_int),
        ("solid_model", ctypes.c_int), ("darcy_c", ctypes.c_double), ("darcy_eps", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_long),
        ("melt_fraction", ctypes.c_double), ("nusselt", ctypes.c_double), ("heater_q", ctypes.c_double),
        ("total_H", ctypes.c_double), ("heat_in_cum", ctypes.c_double), ("budget_residual", ctypes.c_double),
        ("mass", ctypes.c_double), ("max_u", ctypes.c_double), ("fourier", ctypes.c_double),
        ("finite", ctypes.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_dp = ctypes.POINTER(ctypes.c_double)


def load_library(path):
    """A configured handle on an oracle shared library at `path`."""
    L = ctypes.CDLL(path)
    L.or_derive.argtypes = [ctypes.POINTER(Case), ctypes.POINTER(Params)]
    L.or_create.argtypes = [ctypes.POINTER(Case)]
    L.or_create.restype = ctypes.c_void_p
    L.or_destroy.argtypes = [ctypes.c_void_p]
    L.or_get_params.argtypes = [ctypes.c_void_p]
    L.or_get_params.restype = ctypes.POINTER(Params)
    L.or_init_solid.argtypes = [ctypes.c_void_p]
    L.or_init_liquid.argtypes = [ctypes.c_void_p, ctypes.c_double]
    L.or_init_gaussian.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.or_set_populations.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.or_get_populations.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.or_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
    L.or_fields.argtypes = [ctypes.c_void_p] + [_dp] * 6
    L.or_get_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(Stats)]
    L.or_enthalpy_map.argtypes = [ctypes.c_double] * 4 + [_dp, _dp]
    L.or_geq.argtypes = [ctypes.c_double] * 5 + [_dp]
    L.or_feq.argtypes = [ctypes.c_double] * 4 + [_dp]
    L.or_collide_cell.argtypes = [ctypes.POINTER(Params), _dp, _dp, _dp, _dp, _dp]
    L.or_num_threads.restype = ctypes.c_int
    L.or_set_threads.argtypes = [ctypes.c_int]
    return L


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libbtrirt_oracle.so")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _LIB = load_library(path)
    return _LIB


def use_library(path):
    """Loads the oracle from another build of the same source (e.g. one
    compiled for the host's instruction set) for the rest of the process."""
    global _LIB
    _LIB = load_library(path)
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(_dp)


def make_case(nx, ny, *, periodic_x=False, periodic_y=False, param_mode=PARAM_DIMENSIONLESS,
              Ra=1e4, Pr=1.0, Ste=1.0, Ma=0.1, nu=0.0, alpha=0.0, gbeta=0.0, latent=0.0,
              Cp=1.0, Th=1.0, Tm=0.0, rho0=1.0, heater_center=0.5, heater_width=0.25,
              k0_g=math.nan, k2_g=math.nan, k0_f=math.nan, k1_f=math.nan,
              solid_model=SOLID_SCALE, darcy_c=math.nan, darcy_eps=math.nan):
    return Case(nx, ny, int(periodic_x), int(periodic_y), param_mode, Ra, Pr, Ste, Ma,
                nu, alpha, gbeta, latent, Cp, Th, Tm, rho0, heater_center, heater_width,
                k0_g, k2_g, k0_f, k1_f, int(solid_model), darcy_c, darcy_eps)


def case_from_dict(d):
    """Build a Case from a plain dict of the same field names (missing -> defaults)."""
    d = dict(d)
    nx, ny = d.pop("nx"), d.pop("ny")
    return make_case(nx, ny, **{k: v for k, v in d.items() if k in {f for f, _ in Case._fields_}})


def derive(case):
    p = Params()
    rc = lib().or_derive(ctypes.byref(case), ctypes.byref(p))
    if rc != 0:
        raise ValueError("invalid case")
    return p


class Oracle:
    """One cavity on the CPU oracle.  Populations are numpy arrays [9, ny, nx]."""

    def __init__(self, case):
        if isinstance(case, dict):
            case = case_from_dict(case)
        self.case = case
        self._h = lib().or_create(ctypes.byref(case))
        if not self._h:
            raise ValueError("invalid case")
        self.params = lib().or_get_params(self._h).contents
        self.nx, self.ny = case.nx, case.ny

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _LIB is not None:
            try:
                _LIB.or_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    def init_solid(self):
        lib().or_init_solid(self._h)
        return self

    def init_liquid(self, T0):
        lib().or_init_liquid(self._h, T0)
        return self

    def init_gaussian(self, T0, amp, sigma):
        lib().or_init_gaussian(self._h, T0, amp, sigma)
        return self

    def set_populations(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(Q, self.ny, self.nx)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(Q, self.ny, self.nx)
        lib().or_set_populations(self._h, _ptr(f), _ptr(g))
        return self

    def populations(self):
        f = np.empty((Q, self.ny, self.nx))
        g = np.empty((Q, self.ny, self.nx))
        lib().or_get_populations(self._h, _ptr(f), _ptr(g))
        return f, g

    def step(self, n=1):
        lib().or_step(self._h, int(n))
        return self

    def fields(self):
        out = {k: np.empty((self.ny, self.nx)) for k in ("T", "fl", "H", "ux", "uy", "rho")}
        lib().or_fields(self._h, *(_ptr(out[k]) for k in ("T", "fl", "H", "ux", "uy", "rho")))
        return out

    def stats(self):
        s = Stats()
        lib().or_get_stats(self._h, ctypes.byref(s))
        return s.as_dict()


def enthalpy_map(H, Cp, Tm, latent):
    T = ctypes.c_double()
    fl = ctypes.c_double()
    lib().or_enthalpy_map(H, Cp, Tm, latent, ctypes.byref(T), ctypes.byref(fl))
    return T.value, fl.value


def geq(H, T, ux, uy, Cp):
    out = np.empty(Q)
    lib().or_geq(H, T, ux, uy, Cp, _ptr(out))
    return out


def feq(rho, ux, uy, rho0):
    out = np.empty(Q)
    lib().or_feq(rho, ux, uy, rho0, _ptr(out))
    return out


def collide_cell(params, f, g):
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    fo, go, m = np.empty(Q), np.empty(Q), np.empty(6)
    lib().or_collide_cell(ctypes.byref(params), _ptr(f), _ptr(g), _ptr(fo), _ptr(go), _ptr(m))
    return fo, go, dict(zip(("T", "fl", "H", "ux", "uy", "rho"), m))


def num_threads():
    return lib().or_num_threads()


def set_threads(n):
    """Threads of the row loops; 1-D columns run fastest on one."""
    lib().or_set_threads(int(n))
