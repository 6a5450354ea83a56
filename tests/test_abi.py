"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and its host-only calls (validation, parameter derivation,
footprint) behave as documented.  No kernel runs here."""
import math
import os
import re

import pytest

import oracle
import paper_1909_13086_amd as P
from btrirt_workloads import batch_sweep, cavity, large_cavity, small_cavity

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(lbm_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    names = declared_functions()
    assert "lbm_step" in names and "lbm_set_case" in names
    for n in sorted(names):
        assert hasattr(lib, n), f"{n} declared but not exported"
    assert set(P.EXPORTS) <= names


def test_version_and_errors():
    assert "gfx950" in P.lbm_version()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert P.lbm_strerror(code)
    assert P.lbm_strerror(-99) == "unknown error"


@pytest.mark.parametrize("case", [small_cavity("literal"), small_cavity("eq6"), small_cavity("distinct"),
                                  large_cavity(), *batch_sweep()[:6],
                                  cavity(17, 9, heater_center=0.1, heater_width=0.5, Pr=6.2, Ste=0.125, Ra=1e8)])
def test_derivation_matches_oracle(case):
    """The library and the oracle derive the lattice parameters independently."""
    got = P.lbm_derive(P.make_case(case))
    want = oracle.derive(oracle.case_from_dict(case))
    for k in ("nu", "alpha", "gbeta", "latent", "k0_g", "k1_g", "k2_g", "k0_f", "k1_f", "k2_f"):
        assert getattr(got, k) == pytest.approx(getattr(want, k), rel=1e-15, abs=0), k
    if want.n_heater > 0:
        assert (got.heater_lo, got.heater_hi) == (want.heater_lo, want.heater_hi)
    assert got.n_heater == want.n_heater
    assert got.pitch % 64 == 0 and got.pitch >= case["nx"]


@pytest.mark.parametrize("extra", [dict(solid_model=1), dict(solid_model=1, darcy_c=5.0, darcy_eps=0.3),
                                   dict(solid_model=2)])
def test_solid_model_constants_match_oracle(extra):
    case = cavity(40, 20, **extra)
    got = P.lbm_derive(P.make_case(case))
    want = oracle.derive(oracle.case_from_dict(case))
    assert (got.darcy_c, got.darcy_eps) == (want.darcy_c, want.darcy_eps)


def test_literal_small_cavity_rates():
    lat = P.lbm_derive(P.make_case(small_cavity("literal")))
    assert lat.k0_g == 1.0 and lat.k2_g == 1.0
    assert lat.k1_g == pytest.approx(1.637060, abs=1e-6)
    assert (lat.heater_lo, lat.heater_hi, lat.n_heater) == (48, 79, 32)


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-3), dict(precision=2), dict(pattern=5), dict(init=7), dict(param_mode=3),
    dict(Ra=0.0), dict(Th=0.0), dict(k0_g=2.0), dict(k2_g=0.0), dict(k1_f=-1.0), dict(Cp=0.0),
    dict(heater_center=math.inf), dict(init=2, gauss_sigma=0.0),
    dict(param_mode=1, nu=0.1, alpha=0.0, latent=1.0), dict(param_mode=1, nu=0.1, alpha=0.1, latent=-1.0),
    dict(solid_model=3), dict(solid_model=-1), dict(solid_model=1, darcy_c=-1.0),
    dict(solid_model=1, darcy_eps=0.0), dict(solid_model=1, darcy_c=math.inf),
])
def test_invalid_cases_rejected(bad):
    c = P.make_case(cavity(32, 16), **bad)
    with pytest.raises(P.LbmError) as ei:
        P.lbm_derive(c)
    assert ei.value.code == P.LBM_EINVAL
    assert P.lbm_footprint(c) == 0


def test_footprint_layout():
    for prec, elem in ((P.LBM_FP64, 8), (P.LBM_FP32_SHIFTED, 4)):
        for pat, lattices in ((P.LBM_PATTERN_AA, 1), (P.LBM_PATTERN_AB, 2)):
            c = P.make_case(large_cavity(), precision=prec, pattern=pat)
            pops = 18 * 2048 * 1024 * elem
            # populations, per-column strip flux, one 256-byte block of diagnostics
            assert P.lbm_footprint(c) == lattices * pops + 2048 * 8 + 256
    # ragged width: rows padded to a 64-cell pitch
    c = P.make_case(cavity(100, 10))
    assert P.lbm_footprint(c) == (18 * 128 * 10 * 8 + 255) // 256 * 256 + 1024 + 256


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    with pytest.raises(P.LbmError) as ei:
        P.lbm_create(0, None, 0, 1)
    assert ei.value.code == P.LBM_EDEVICE


def test_context_calls_reject_a_null_context():
    """Calls on a context return LBM_EINVAL for a NULL context (no GPU needed)."""
    import ctypes
    lib = P.lib()
    n, seg = ctypes.c_int(), ctypes.c_int()
    assert lib.lbm_slot_fusion(None, 0, ctypes.byref(n), ctypes.byref(seg)) == P.LBM_EINVAL
    assert lib.lbm_get_fusion(None, 0, ctypes.byref(n), ctypes.byref(seg)) == P.LBM_EINVAL
    assert lib.lbm_set_fusion(None, 0, 3, 4) == P.LBM_EINVAL
    assert lib.lbm_set_group_bytes(None, 1 << 30) == P.LBM_EINVAL
    us = ctypes.c_double()
    assert lib.lbm_stream_probe(None, 1 << 20, P.LBM_PATTERN_AB, 4, ctypes.byref(us)) == P.LBM_EINVAL


class _CkptHeader(__import__("ctypes").Structure):
    """Host layout of a checkpoint header (magic, version, header bytes,
    precision, pattern, parity, step, region bytes, case)."""
    import ctypes as _c
    _fields_ = [("magic", _c.c_char * 8), ("version", _c.c_uint32), ("header_bytes", _c.c_uint32),
                ("precision", _c.c_int32), ("pattern", _c.c_int32), ("parity", _c.c_int32), ("pad", _c.c_int32),
                ("step", _c.c_int64), ("region_bytes", _c.c_uint64), ("cs", P.lbm_case)]


def _blob(case, **over):
    import ctypes
    c = P.make_case(case)
    h = _CkptHeader()
    h.magic = b"BTRIRTCK"
    h.version = 1
    h.header_bytes = ctypes.sizeof(_CkptHeader)
    h.precision, h.pattern, h.parity, h.step = c.precision, c.pattern, 1, 437
    h.region_bytes = P.lbm_footprint(c)
    h.cs = c
    for k, v in over.items():
        if k.startswith("cs_"):
            setattr(h.cs, k[3:], v)
        else:
            setattr(h, k, v)
    return bytes(h) + bytes(h.region_bytes)


def test_checkpoint_info_accepts_a_consistent_checkpoint():
    case = dict(small_cavity("distinct"), pattern=P.LBM_PATTERN_AB)
    cs, step = P.lbm_checkpoint_info(_blob(case))
    assert step == 437 and (cs.nx, cs.ny, cs.pattern, cs.k0_g) == (128, 64, P.LBM_PATTERN_AB, 0.8)


@pytest.mark.parametrize("over", [
    dict(magic=b"NOTACKPT"), dict(version=2), dict(parity=2), dict(step=-1),
    # header and embedded case disagree: an in-place FP64 header over a two-lattice case
    dict(pattern=P.LBM_PATTERN_AA), dict(precision=P.LBM_FP32_SHIFTED),
    # embedded case invalid, or of another size than the region
    dict(cs_k0_g=2.5), dict(cs_nx=0), dict(cs_ny=65), dict(region_bytes=1 << 20),
])
def test_checkpoint_info_rejects_an_inconsistent_checkpoint(over):
    case = dict(small_cavity("distinct"), pattern=P.LBM_PATTERN_AB)
    with pytest.raises(P.LbmError) as ei:
        P.lbm_checkpoint_info(_blob(case, **over))
    assert ei.value.code == P.LBM_EINVAL


def test_checkpoint_info_rejects_a_truncated_checkpoint():
    blob = _blob(small_cavity("eq6"))
    for n in (0, 50, len(blob) - 1):
        with pytest.raises(P.LbmError):
            P.lbm_checkpoint_info(blob[:n])


def test_stale_library_is_refused(tmp_path, monkeypatch):
    """A built library older than a source is not loaded."""
    import shutil
    from paper_1909_13086_amd import _lib
    old = tmp_path / "liblbm.so"
    shutil.copy(_lib.LIB_PATH, old)
    os.utime(old, (1, 1))
    monkeypatch.setattr(_lib, "LIB_PATH", str(old))
    monkeypatch.setattr(_lib, "_L", None)
    with pytest.raises(ImportError, match="older than its sources"):
        _lib.lib()
