"""FP32 shifted-population path: populations stored as f_i - w_i rho0 and
g_i - w_i Cp Tm in FP32, diagnostics reduced in FP64.  Error against the FP64
oracle is reported per result (liquid-fraction field, melt fraction, Nusselt
number); the bar is 1e-4 in melt fraction and 0.5 % in Nusselt number.  The
liquid-fraction field is bounded by FL_LINF: in the mushy cells fl = (H - Cp
Tm)/L with L = 1 here, so its error is the enthalpy error of the few cells at
the front, where FP32 rounding of order 1e-7 per step gathers over 20000 steps
(about 3e-4 observed); the bound leaves a factor of three."""
import numpy as np
import pytest

import oracle
from btrirt_workloads import small_cavity
from tests.test_gpu_parity import _random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1909_13086_amd as P
    return P


FL_LINF = 1e-3


@pytest.mark.parametrize("pattern,fuse", [(0, 1), (1, 3), (1, 4)], ids=["in_place", "three_step", "four_step"])
@pytest.mark.parametrize("variant", ["literal", "eq6"])
def test_fp32_shifted_small_cavity_to_20k_steps(P, variant, pattern, fuse):
    case = dict(small_cavity(variant), precision=P.LBM_FP32_SHIFTED, pattern=pattern)
    print(f"case small_cavity[{variant}] FP32 shifted pattern {pattern} fuse {fuse} to 20000 steps", flush=True)
    o = oracle.Oracle(oracle.case_from_dict(case)).init_solid()
    rows = []
    with P.Context(device=0, max_slots=2) as ctx:
        if pattern == 1:
            ctx.set_fusion(P.LBM_FP32_SHIFTED, fuse, 6)
        s = ctx.add(case)
        done = 0
        for t in (5000, 10000, 20000):
            ctx.step(s, t - done)
            o.step(t - done)
            done = t
            st, ost = ctx.reduce(s), o.stats()
            fl_err = float(np.max(np.abs(ctx.fields(s, 2)["fl"] - o.fields()["fl"])))
            dphi = abs(st["melt_fraction"] - ost["melt_fraction"])
            dnu = abs(st["nusselt"] - ost["nusselt"]) / abs(ost["nusselt"])
            rows.append((t, fl_err, dphi, dnu))
            print(f"  t={t}: Linf(fl)={fl_err:.2e} |dphi|={dphi:.2e} |dNu|/Nu={dnu:.2e} "
                  f"phi={ost['melt_fraction']:.5f} Nu={ost['nusselt']:.4f} "
                  f"budget={st['budget_residual']:.2e}", flush=True)
            assert dphi <= 1e-4
            assert dnu <= 5e-3
            assert fl_err <= FL_LINF
            assert st["finite"] == 1


def test_fp32_shifted_short_run_tracks_oracle(P):
    from btrirt_workloads import cavity
    nx, ny = 96, 40
    case = dict(cavity(nx, ny, param_mode=1, nu=0.04, alpha=0.06, gbeta=3e-3, latent=0.8, Tm=0.1,
                       Th=0.9, heater_center=0.3, heater_width=0.4), precision=P.LBM_FP32_SHIFTED)
    f0, g0 = _random_state(77, nx, ny)
    with P.Context(device=0, max_slots=1) as ctx:
        s = ctx.add(case)
        ctx.state_load(s, f0, g0)
        ctx.step(s, 25)
        fg, gg = ctx.state_save(s)
    o = oracle.Oracle(oracle.case_from_dict(case)).set_populations(f0, g0).step(25)
    fo, go = o.populations()
    # FP32 storage: a few units in the last place of values of order 1
    assert np.max(np.abs(fg - fo)) <= 2e-6
    assert np.max(np.abs(gg - go)) <= 2e-6


@pytest.mark.parametrize("fuse", [3, 4])
def test_fp32_fused_full_size_tracks_oracle(P, fuse):
    """The FP32-shifted variant at the benchmark's size (2048x1024, two
    lattices, three or four steps per launch, 6-row segments) from a random
    state, 12 steps, against the FP64 oracle."""
    from btrirt_workloads import large_cavity
    case = dict(large_cavity(), precision=P.LBM_FP32_SHIFTED, pattern=P.LBM_PATTERN_AB)
    f0, g0 = _random_state(29, 2048, 1024)
    print(f"case 2048x1024 FP32 {fuse} steps per launch, 12 steps vs oracle", flush=True)
    with P.Context(device=0, max_slots=1) as ctx:
        ctx.set_fusion(1, fuse, 6)
        s = ctx.add(case)
        ctx.state_load(s, f0, g0)
        ctx.step(s, 12)
        fg, gg = ctx.state_save(s)
        st = ctx.reduce(s)
    o = oracle.Oracle(oracle.case_from_dict(case)).set_populations(f0, g0).step(12)
    fo, go = o.populations()
    assert np.max(np.abs(fg - fo)) <= 2e-6
    assert np.max(np.abs(gg - go)) <= 2e-6
    ost = o.stats()
    assert abs(st["melt_fraction"] - ost["melt_fraction"]) <= 1e-6
    assert st["total_H"] == pytest.approx(ost["total_H"], rel=1e-6)
