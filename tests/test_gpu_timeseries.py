"""Melt-fraction and Nusselt time series of the large cavity's physics on a
256x128 downscale (Ra 1e8, Pr 1, Ste 1, heater W/4 centred), 20000 steps from
all solid, recorded every 100 steps on the device and compared with the FP64
oracle at the same steps, in place and on the benchmark's kernel (two
lattices, three steps per launch, 4-row segments; a report every 100 steps
makes each 100-step stretch 32 three-step launches and two two-step ones);
the FP32-shifted path is compared with it too."""
import numpy as np
import pytest

import oracle
from btrirt_workloads import large_cavity

pytestmark = pytest.mark.gpu

STEPS, EVERY = 20000, 100


@pytest.fixture(scope="module")
def P():
    import paper_1909_13086_amd as P
    return P


@pytest.fixture(scope="module")
def oracle_series():
    o = oracle.Oracle(oracle.case_from_dict(large_cavity(256, 128))).init_solid()
    out = []
    for _ in range(STEPS // EVERY):
        o.step(EVERY)
        out.append(o.stats())
    return out


def gpu_series(P, precision, pattern=0):
    case = dict(large_cavity(256, 128), precision=precision, pattern=pattern)
    with P.Context(device=0, max_slots=1) as ctx:
        if pattern == 1:
            ctx.set_fusion(precision, 3, 4)
        s = ctx.add(case)
        if pattern == 1:
            assert ctx.slot_fusion(s) == (3, 4)
        ctx.set_report(s, EVERY, STEPS // EVERY)
        ctx.step(s, STEPS)
        return ctx.series(s)


@pytest.mark.parametrize("pattern", [0, 1], ids=["in_place", "three_step"])
def test_fp64_series_matches_oracle(P, oracle_series, pattern):
    print(f"case 256x128 Ra 1e8 FP64 pattern {pattern}, 20000 steps, series every 100", flush=True)
    ser = gpu_series(P, P.LBM_FP64, pattern)
    assert [e["step"] for e in ser] == [EVERY * (k + 1) for k in range(STEPS // EVERY)]
    dphi = max(abs(a["melt_fraction"] - b["melt_fraction"]) for a, b in zip(ser, oracle_series))
    dnu = max(abs(a["nusselt"] - b["nusselt"]) / abs(b["nusselt"]) for a, b in zip(ser, oracle_series))
    dres = max(abs(a["budget_residual"]) / a["total_H"] for a in ser)
    print(f"  max|dphi|={dphi:.2e} max|dNu|/Nu={dnu:.2e} max|R|/H={dres:.2e} "
          f"phi(20000)={ser[-1]['melt_fraction']:.6f} Nu(20000)={ser[-1]['nusselt']:.4f}", flush=True)
    assert dphi <= 1e-10
    assert dnu <= 1e-8
    assert dres <= 1e-12
    assert all(e["finite"] == 1 for e in ser)


@pytest.mark.parametrize("pattern", [0, 1], ids=["in_place", "three_step"])
def test_fp32_series_tracks_fp64(P, oracle_series, pattern):
    print(f"case 256x128 Ra 1e8 FP32 shifted pattern {pattern}, 20000 steps, series every 100", flush=True)
    ser = gpu_series(P, P.LBM_FP32_SHIFTED, pattern)
    dphi = np.array([abs(a["melt_fraction"] - b["melt_fraction"]) for a, b in zip(ser, oracle_series)])
    dnu = np.array([abs(a["nusselt"] - b["nusselt"]) / abs(b["nusselt"]) for a, b in zip(ser, oracle_series)])
    print(f"  max|dphi|={dphi.max():.2e} max|dNu|/Nu={dnu.max():.2e}", flush=True)
    assert dphi.max() <= 1e-4
    assert dnu.max() <= 5e-3
