"""The allocation-free variant of lbm_fields, called through the C ABI: its
fields equal lbm_fields' bit for bit on two calls in a row (the second on a
smaller cavity with fewer fields), and a request above its fixed staging size
is refused with LBM_EINVAL."""
import ctypes

import numpy as np
import pytest

from btrirt_workloads import cavity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1909_13086_amd as P
    return P


def _noalloc(P, ctx, slot, nx, ny, mask):
    """Direct C-ABI call of lbm_fields_noalloc into a numpy buffer."""
    planes = bin(mask & 63).count("1")
    buf = np.full((planes, ny, nx), np.nan)
    rc = P.lib().lbm_fields_noalloc(ctx.h, slot, mask, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    buf.size)
    return rc, buf


def test_fields_noalloc_equals_fields(P):
    print("case lbm_fields_noalloc vs lbm_fields, 256x128 FP64 then 96x40 FP32", flush=True)
    with P.Context(device=0, max_slots=2) as ctx:
        a = ctx.add(cavity(256, 128, Ra=1e6, heater_center=0.4))
        b = ctx.add(dict(cavity(96, 40, Ra=1e5), precision=P.LBM_FP32_SHIFTED, pattern=P.LBM_PATTERN_AB))
        ctx.step(a, 700)
        ctx.step(b, 333)
        for slot, (nx, ny), mask in ((a, (256, 128), 63), (b, (96, 40), P.LBM_FIELD_FL | P.LBM_FIELD_UY)):
            rc, got = _noalloc(P, ctx, slot, nx, ny, mask)
            assert rc == P.LBM_OK
            want = ctx.fields(slot, mask)
            names = [n for k, n in enumerate(P.FIELD_NAMES) if mask & (1 << k)]
            for k, n in enumerate(names):
                assert np.array_equal(got[k], want[n]), n
            assert np.isfinite(got).all()


def test_fields_noalloc_refuses_more_than_its_staging(P):
    with P.Context(device=0, max_slots=1) as ctx:
        s = ctx.add(cavity(2048, 1024))
        rc, _ = _noalloc(P, ctx, s, 2048, 1024, P.LBM_FIELD_H)  # 16 MiB: fits exactly
        assert rc == P.LBM_OK
        rc, _ = _noalloc(P, ctx, s, 2048, 1024, P.LBM_FIELD_H | P.LBM_FIELD_T)
        assert rc == P.LBM_EINVAL
        assert "16777216" in P.lib().lbm_last_error().decode()
