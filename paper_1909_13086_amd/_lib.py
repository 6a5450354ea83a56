"""ctypes binding of ``liblbm.so`` (include/lbm.h): argument marshalling only.

Every call of the hot path runs in the HIP library; this module converts
Python values to the C structs, checks return codes and raises ``LbmError``
with the library's message.  There is no fallback: if the library is missing
the import fails.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE, LBM_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
LBM_FP64, LBM_FP32_SHIFTED = 0, 1
LBM_PATTERN_AA, LBM_PATTERN_AB = 0, 1
LBM_SOLID_SCALE, LBM_SOLID_DARCY, LBM_SOLID_PBB = 0, 1, 2
LBM_PARAM_DIMENSIONLESS, LBM_PARAM_LATTICE = 0, 1
LBM_INIT_SOLID_AT_TM, LBM_INIT_LIQUID_T0, LBM_INIT_GAUSSIAN = 0, 1, 2
LBM_FIELD_T, LBM_FIELD_FL, LBM_FIELD_H, LBM_FIELD_UX, LBM_FIELD_UY, LBM_FIELD_RHO = 1, 2, 4, 8, 16, 32
FIELD_NAMES = ("T", "fl", "H", "ux", "uy", "rho")
LBM_ALL = -1
LBM_LAUNCH_XCD_BANDS, LBM_LAUNCH_NONTEMPORAL, LBM_LAUNCH_ALTERNATE, LBM_LAUNCH_ZIGZAG = 1, 2, 4, 8
LBM_LAUNCH_STAGED = 16
LBM_LAUNCH_DEFAULT = LBM_LAUNCH_XCD_BANDS | LBM_LAUNCH_ALTERNATE | LBM_LAUNCH_ZIGZAG | LBM_LAUNCH_STAGED

# Names exported by include/lbm.h and include/lbm_serve.h.
EXPORTS = (
    "lbm_strerror", "lbm_last_error", "lbm_derive", "lbm_footprint", "lbm_version",
    "lbm_create", "lbm_destroy", "lbm_set_case", "lbm_release", "lbm_step", "lbm_reduce",
    "lbm_fields", "lbm_set_report", "lbm_series", "lbm_state_load", "lbm_state_save",
    "lbm_set_launch", "lbm_get_launch", "lbm_set_graph_chunk", "lbm_autotune", "lbm_sync",
    "lbm_stream", "lbm_slot_info", "lbm_slot_fusion", "lbm_step_many", "lbm_set_group_bytes",
    "lbm_checkpoint_bytes", "lbm_checkpoint_save", "lbm_checkpoint_load", "lbm_checkpoint_info",
    "lbm_set_fusion", "lbm_get_fusion",
    "lbm_server_create", "lbm_server_destroy", "lbm_server_submit", "lbm_server_run",
    "lbm_server_request", "lbm_server_summary", "lbm_server_on_finish", "lbm_fields_noalloc",
    "lbm_stream_probe",
)


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class lbm_case(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("pattern", ctypes.c_int32), ("param_mode", ctypes.c_int32),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32), ("init", ctypes.c_int32),
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("Ste", ctypes.c_double), ("Ma", ctypes.c_double),
        ("nu", ctypes.c_double), ("alpha", ctypes.c_double), ("gbeta", ctypes.c_double), ("latent", ctypes.c_double),
        ("Cp", ctypes.c_double), ("Th", ctypes.c_double), ("Tm", ctypes.c_double), ("rho0", ctypes.c_double),
        ("heater_center", ctypes.c_double), ("heater_width", ctypes.c_double),
        ("k0_g", ctypes.c_double), ("k2_g", ctypes.c_double), ("k0_f", ctypes.c_double), ("k1_f", ctypes.c_double),
        ("T0", ctypes.c_double), ("gauss_amp", ctypes.c_double), ("gauss_sigma", ctypes.c_double),
        ("solid_model", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("darcy_c", ctypes.c_double), ("darcy_eps", ctypes.c_double),
    ]


class lbm_lattice(ctypes.Structure):
    _fields_ = [
        ("nu", ctypes.c_double), ("alpha", ctypes.c_double), ("gbeta", ctypes.c_double), ("latent", ctypes.c_double),
        ("k0_g", ctypes.c_double), ("k1_g", ctypes.c_double), ("k2_g", ctypes.c_double),
        ("k0_f", ctypes.c_double), ("k1_f", ctypes.c_double), ("k2_f", ctypes.c_double),
        ("heater_lo", ctypes.c_int32), ("heater_hi", ctypes.c_int32), ("n_heater", ctypes.c_int32),
        ("pitch", ctypes.c_int32),
        ("darcy_c", ctypes.c_double), ("darcy_eps", ctypes.c_double),
    ]


class lbm_stats(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("melt_fraction", ctypes.c_double), ("nusselt", ctypes.c_double), ("heater_q", ctypes.c_double),
        ("total_H", ctypes.c_double), ("heat_in_cum", ctypes.c_double), ("budget_residual", ctypes.c_double),
        ("mass", ctypes.c_double), ("max_u", ctypes.c_double), ("fourier", ctypes.c_double),
        ("finite", ctypes.c_int32), ("parity", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_CASE_DEFAULTS = dict(
    precision=LBM_FP64, pattern=LBM_PATTERN_AA, param_mode=LBM_PARAM_DIMENSIONLESS,
    periodic_x=0, periodic_y=0, init=LBM_INIT_SOLID_AT_TM,
    Ra=1e4, Pr=1.0, Ste=1.0, Ma=0.1, nu=0.0, alpha=0.0, gbeta=0.0, latent=0.0,
    Cp=1.0, Th=1.0, Tm=0.0, rho0=1.0, heater_center=0.5, heater_width=0.25,
    k0_g=math.nan, k2_g=math.nan, k0_f=math.nan, k1_f=math.nan,
    T0=0.0, gauss_amp=0.0, gauss_sigma=1.0,
    solid_model=0, reserved=0, darcy_c=math.nan, darcy_eps=math.nan,
)
CASE_FIELDS = tuple(name for name, _ in lbm_case._fields_)


def make_case(d=None, **kw):
    """lbm_case from a dict of problem parameters (unknown keys are ignored)."""
    vals = dict(_CASE_DEFAULTS)
    if d:
        vals.update({k: v for k, v in d.items() if k in CASE_FIELDS})
    vals.update({k: v for k, v in kw.items() if k in CASE_FIELDS})
    c = lbm_case()
    for name in CASE_FIELDS:
        setattr(c, name, vals[name])
    return c


_L = None
_dp = ctypes.POINTER(ctypes.c_double)
_BUILD_HINT = "`python -c 'import __graft_entry__ as g; g.build()'`"


def _newest_source():
    """Newest modification time among the library's sources and headers."""
    srcs = [os.path.join(_HERE, "csrc", f) for f in os.listdir(os.path.join(_HERE, "csrc"))]
    inc = os.path.join(os.path.dirname(_HERE), "include")
    srcs += [os.path.join(inc, f) for f in os.listdir(inc)]
    srcs.append(os.path.join(_HERE, "build.py"))
    return max(os.path.getmtime(f) for f in srcs if os.path.isfile(f))


def lib():
    """The loaded library.  Raises if it has not been built, or if a source
    is newer than the built library (a stale binary would run other code than
    the sources show)."""
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with {_BUILD_HINT}")
        if os.path.getmtime(LIB_PATH) < _newest_source():
            raise ImportError(f"{LIB_PATH} is older than its sources: rebuild it with {_BUILD_HINT}")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        sig = {
            "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "lbm_last_error": (ctypes.c_char_p, []),
            "lbm_version": (ctypes.c_char_p, []),
            "lbm_derive": (ctypes.c_int, [ctypes.POINTER(lbm_case), ctypes.POINTER(lbm_lattice)]),
            "lbm_footprint": (ctypes.c_size_t, [ctypes.POINTER(lbm_case)]),
            "lbm_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_size_t, ctypes.c_int]),
            "lbm_destroy": (None, [vp]),
            "lbm_set_case": (ctypes.c_int, [vp, ctypes.POINTER(lbm_case), vp, ctypes.c_size_t,
                                             ctypes.POINTER(ctypes.c_int)]),
            "lbm_release": (ctypes.c_int, [vp, ctypes.c_int]),
            "lbm_step": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int64]),
            "lbm_step_many": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int64)]),
            "lbm_set_group_bytes": (ctypes.c_int, [vp, ctypes.c_size_t]),
            "lbm_reduce": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(lbm_stats)]),
            "lbm_fields": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_uint32, _dp, ctypes.c_size_t]),
            "lbm_fields_noalloc": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_uint32, _dp, ctypes.c_size_t]),
            "lbm_stream_probe": (ctypes.c_int, [vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_double)]),
            "lbm_set_report": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int32]),
            "lbm_series": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(lbm_stats), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]),
            "lbm_state_load": (ctypes.c_int, [vp, ctypes.c_int, _dp, _dp, ctypes.c_size_t]),
            "lbm_state_save": (ctypes.c_int, [vp, ctypes.c_int, _dp, _dp, ctypes.c_size_t]),
            "lbm_set_launch": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int]),
            "lbm_get_launch": (ctypes.c_int, [vp, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 4),
            "lbm_set_graph_chunk": (ctypes.c_int, [vp, ctypes.c_int]),
            "lbm_set_fusion": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "lbm_get_fusion": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int)]),
            "lbm_autotune": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_char_p]),
            "lbm_sync": (ctypes.c_int, [vp]),
            "lbm_checkpoint_bytes": (ctypes.c_size_t, [vp, ctypes.c_int]),
            "lbm_checkpoint_save": (ctypes.c_int, [vp, ctypes.c_int, vp, ctypes.c_size_t]),
            "lbm_checkpoint_load": (ctypes.c_int, [vp, ctypes.c_int, vp, ctypes.c_size_t]),
            "lbm_checkpoint_info": (ctypes.c_int, [vp, ctypes.c_size_t, ctypes.POINTER(lbm_case),
                                                   ctypes.POINTER(ctypes.c_int64)]),
            "lbm_stream": (ctypes.c_int, [vp, ctypes.POINTER(vp)]),
            "lbm_slot_info": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_size_t)]),
            "lbm_slot_fusion": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                               ctypes.POINTER(ctypes.c_int)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _L = L
    return _L


def _check(rc):
    if rc != LBM_OK:
        msg = lib().lbm_last_error().decode() or lib().lbm_strerror(rc).decode()
        raise LbmError(rc, msg)
    return rc


def _ptr(a):
    return a.ctypes.data_as(_dp)


# ---- host-only calls --------------------------------------------------------

def lbm_strerror(code):
    return lib().lbm_strerror(code).decode()


def lbm_version():
    return lib().lbm_version().decode()


def lbm_derive(case):
    out = lbm_lattice()
    _check(lib().lbm_derive(ctypes.byref(case), ctypes.byref(out)))
    return out


def lbm_footprint(case):
    return int(lib().lbm_footprint(ctypes.byref(case)))


# ---- context and slots --------------------------------------------------------

def lbm_create(device=0, stream=None, hbm_budget=0, max_slots=1):
    """stream: a hipStream_t handle as int (e.g. torch.cuda.current_stream().cuda_stream) or None."""
    h = ctypes.c_void_p()
    _check(lib().lbm_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream) if stream else None,
                            int(hbm_budget), int(max_slots)))
    return h


def lbm_destroy(ctx):
    lib().lbm_destroy(ctx)


def lbm_set_case(ctx, case, dev_buf=None, buf_bytes=0):
    """dev_buf: device pointer (int) of a lent buffer, e.g. tensor.data_ptr(), or None."""
    slot = ctypes.c_int(-1)
    _check(lib().lbm_set_case(ctx, ctypes.byref(case), ctypes.c_void_p(dev_buf) if dev_buf else None,
                              int(buf_bytes), ctypes.byref(slot)))
    return slot.value


def lbm_release(ctx, slot):
    _check(lib().lbm_release(ctx, int(slot)))


def lbm_step(ctx, slot, nsteps):
    _check(lib().lbm_step(ctx, int(slot), int(nsteps)))


def lbm_step_many(ctx, slots, nsteps):
    n = len(slots)
    a = (ctypes.c_int32 * max(n, 1))(*[int(v) for v in slots])
    b = (ctypes.c_int64 * max(n, 1))(*[int(v) for v in nsteps])
    _check(lib().lbm_step_many(ctx, n, a, b))


def lbm_set_group_bytes(ctx, nbytes):
    _check(lib().lbm_set_group_bytes(ctx, int(nbytes)))


def lbm_reduce(ctx, slot, allow_unstable=False):
    s = lbm_stats()
    rc = lib().lbm_reduce(ctx, int(slot), ctypes.byref(s))
    if rc == LBM_EUNSTABLE and allow_unstable:
        return s.as_dict()
    _check(rc)
    return s.as_dict()


def lbm_fields(ctx, slot, nx, ny, mask=63):
    names = [n for b, n in enumerate(FIELD_NAMES) if mask & (1 << b)]
    buf = np.empty((len(names), ny, nx), dtype=np.float64)
    _check(lib().lbm_fields(ctx, int(slot), int(mask), _ptr(buf), buf.size))
    return {n: buf[k] for k, n in enumerate(names)}


def lbm_fields_noalloc(ctx, slot, nx, ny, mask=63):
    """lbm_fields through the library's fixed device staging array (no
    device allocation)."""
    names = [n for b, n in enumerate(FIELD_NAMES) if mask & (1 << b)]
    buf = np.empty((len(names), ny, nx), dtype=np.float64)
    _check(lib().lbm_fields_noalloc(ctx, int(slot), int(mask), _ptr(buf), buf.size))
    return {n: buf[k] for k, n in enumerate(names)}


def lbm_stream_probe(ctx, nbytes, pattern, launches=40):
    """Microseconds per launch of the layout's streaming probe (lbm.h)."""
    us = ctypes.c_double()
    _check(lib().lbm_stream_probe(ctx, int(nbytes), int(pattern), int(launches), ctypes.byref(us)))
    return us.value


def lbm_set_report(ctx, slot, every, capacity):
    _check(lib().lbm_set_report(ctx, int(slot), int(every), int(capacity)))


def lbm_series(ctx, slot, max_entries=1 << 16):
    arr = (lbm_stats * max(1, max_entries))()
    cnt = ctypes.c_int32(0)
    _check(lib().lbm_series(ctx, int(slot), arr, int(max_entries), ctypes.byref(cnt)))
    return [arr[k].as_dict() for k in range(cnt.value)]


def lbm_state_load(ctx, slot, f, g):
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    if f.size != g.size:
        raise ValueError("f and g differ in size")
    _check(lib().lbm_state_load(ctx, int(slot), _ptr(f), _ptr(g), f.size))


def lbm_state_save(ctx, slot, nx, ny):
    f = np.empty((9, ny, nx))
    g = np.empty((9, ny, nx))
    _check(lib().lbm_state_save(ctx, int(slot), _ptr(f), _ptr(g), f.size))
    return f, g


def lbm_checkpoint_save(ctx, slot):
    """Checkpoint of a slot as bytes."""
    n = int(lib().lbm_checkpoint_bytes(ctx, int(slot)))
    if n == 0:
        raise LbmError(LBM_ESTATE, f"slot {slot} is not in use")
    buf = ctypes.create_string_buffer(n)
    _check(lib().lbm_checkpoint_save(ctx, int(slot), ctypes.cast(buf, ctypes.c_void_p), n))
    return buf.raw


def lbm_checkpoint_load(ctx, slot, blob):
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    _check(lib().lbm_checkpoint_load(ctx, int(slot), ctypes.cast(buf, ctypes.c_void_p), len(blob)))


def lbm_checkpoint_info(blob):
    """(case, step) of a checkpoint, validated on the host (no GPU needed)."""
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    cs, step = lbm_case(), ctypes.c_int64()
    _check(lib().lbm_checkpoint_info(ctypes.cast(buf, ctypes.c_void_p), len(blob), ctypes.byref(cs),
                                     ctypes.byref(step)))
    return cs, step.value


# ---- execution control --------------------------------------------------------

def lbm_set_launch(ctx, precision, bx, by, cpl, flags=LBM_LAUNCH_DEFAULT):
    _check(lib().lbm_set_launch(ctx, int(precision), int(bx), int(by), int(cpl), int(flags)))


def lbm_get_launch(ctx, precision):
    v = [ctypes.c_int() for _ in range(4)]
    _check(lib().lbm_get_launch(ctx, int(precision), *(ctypes.byref(x) for x in v)))
    return tuple(x.value for x in v)


def lbm_get_fusion(ctx, precision):
    n, seg = ctypes.c_int(), ctypes.c_int()
    _check(lib().lbm_get_fusion(ctx, int(precision), ctypes.byref(n), ctypes.byref(seg)))
    return n.value, seg.value


def lbm_set_fusion(ctx, precision, steps_per_launch, segment_rows=None):
    # None keeps the segment rows stored for that number of steps per launch
    _check(lib().lbm_set_fusion(ctx, int(precision), int(steps_per_launch),
                                0 if segment_rows is None else int(segment_rows)))


def lbm_set_graph_chunk(ctx, chunk):
    _check(lib().lbm_set_graph_chunk(ctx, int(chunk)))


def lbm_autotune(ctx, precision, nx, ny, cache_path=None):
    _check(lib().lbm_autotune(ctx, int(precision), int(nx), int(ny),
                              cache_path.encode() if cache_path else None))
    return lbm_get_launch(ctx, precision)


def lbm_sync(ctx):
    _check(lib().lbm_sync(ctx))


def lbm_stream(ctx):
    s = ctypes.c_void_p()
    _check(lib().lbm_stream(ctx, ctypes.byref(s)))
    return s.value


def lbm_slot_fusion(ctx, slot):
    n, seg = ctypes.c_int(), ctypes.c_int()
    _check(lib().lbm_slot_fusion(ctx, int(slot), ctypes.byref(n), ctypes.byref(seg)))
    return n.value, seg.value


def lbm_slot_info(ctx, slot):
    step, parity, nbytes = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_size_t()
    _check(lib().lbm_slot_info(ctx, int(slot), ctypes.byref(step), ctypes.byref(parity), ctypes.byref(nbytes)))
    return step.value, parity.value, nbytes.value
