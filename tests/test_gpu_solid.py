"""The solid-phase readings (velocity scaling, Carman-Kozeny drag, partial
bounce-back) on the GPU against the FP64 oracle, in every launch path."""
import numpy as np
import pytest

from btrirt_workloads import cavity, small_cavity
from tests.test_gpu_parity import _random_state, max_field_err, oracle_run

pytestmark = pytest.mark.gpu

MODELS = [1, 2]  # LBM_SOLID_DARCY, LBM_SOLID_PBB (0 is covered by every other test)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1909_13086_amd as P
    return P


def _geom_case(nx, ny, px, py, model, **kw):
    return cavity(nx, ny, periodic_x=px, periodic_y=py, heater_center=0.4, heater_width=0.5,
                  param_mode=1, nu=0.04, alpha=0.06, gbeta=3e-3, latent=0.8, Tm=0.1, Th=0.9,
                  k0_g=0.9, k2_g=1.2, k0_f=1.1, k1_f=0.85, solid_model=model, **kw)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("geom", [(65, 7, 0, 0), (130, 33, 1, 0), (64, 64, 1, 1)])
def test_random_states_match_oracle(P, model, geom):
    nx, ny, px, py = geom
    case = _geom_case(nx, ny, px, py, model, darcy_c=50.0, darcy_eps=1e-2)
    print(f"case solid model {model} random {nx}x{ny} periodic=({px},{py})", flush=True)
    f0, g0 = _random_state(3000 + nx + ny + model, nx, ny)
    with P.Context(device=0, max_slots=1) as ctx:
        s = ctx.add(case)
        ctx.state_load(s, f0, g0)
        ctx.step(s, 9)
        fg, gg = ctx.state_save(s)
        got = ctx.fields(s)
    o = oracle_run(case, 9, f0, g0)
    fo, go = o.populations()
    assert np.max(np.abs(fg - fo)) <= 1e-13
    assert np.max(np.abs(gg - go)) <= 1e-13
    assert max(max_field_err(got, o.fields()).values()) <= 1e-13


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("precision", [0, 1])
def test_melting_cavity_matches_oracle(P, model, precision):
    case = dict(small_cavity("distinct"), Ra=1e5, solid_model=model, precision=precision)
    print(f"case solid model {model} small cavity Ra 1e5 precision {precision} 1500 steps", flush=True)
    with P.Context(device=0, max_slots=1) as ctx:
        s = ctx.add(case)
        ctx.step(s, 1500)
        got, st = ctx.fields(s), ctx.reduce(s)
    o = oracle_run(case, 1500)
    want, ost = o.fields(), o.stats()
    err = max_field_err(got, want)
    if precision == 0:
        assert max(err.values()) <= 1e-10, err
        assert st["melt_fraction"] == pytest.approx(ost["melt_fraction"], abs=1e-12)
        assert st["nusselt"] == pytest.approx(ost["nusselt"], rel=1e-10)
    else:  # FP32-shifted storage: the bar of that variant
        assert abs(st["melt_fraction"] - ost["melt_fraction"]) <= 1e-4
        assert abs(st["nusselt"] - ost["nusselt"]) <= 5e-3 * abs(ost["nusselt"])
    # FP32 storage rounds each cell's enthalpy every step (about 6e-8 of the
    # stored value); over 1500 steps the budget drifts by 1e-5 of the total
    assert abs(st["budget_residual"]) <= (1e-12 if precision == 0 else 1e-4) * st["total_H"]
    assert st["max_u"] == pytest.approx(ost["max_u"], rel=1e-6 if precision == 0 else 2e-2)


@pytest.mark.parametrize("model", MODELS)
def test_fused_and_batched_paths_equal_single_steps(P, model):
    """Two-lattice launches of two and three steps (rows staged and direct)
    and batched launches of mixed solid models give the single-step results
    bit for bit."""
    cases = [dict(_geom_case(130, 40, 0, 0, model), pattern=P.LBM_PATTERN_AB),
             dict(_geom_case(96, 33, 1, 0, 0), pattern=P.LBM_PATTERN_AB),
             dict(_geom_case(77, 21, 0, 0, model), precision=P.LBM_FP32_SHIFTED),
             dict(_geom_case(70, 30, 0, 1, 3 - model), pattern=P.LBM_PATTERN_AB, precision=P.LBM_FP32_SHIFTED)]
    states = [_random_state(90 + k, c["nx"], c["ny"]) for k, c in enumerate(cases)]
    print(f"case solid model {model} two-step / batched bitwise", flush=True)
    want = []
    for c, (f0, g0) in zip(cases, states):
        with P.Context(device=0, max_slots=1) as ctx:
            for prec in (0, 1):
                ctx.set_fusion(prec, 1)
            s = ctx.add(c)
            ctx.state_load(s, f0, g0)
            ctx.step(s, 11)
            want.append(ctx.state_save(s))
    for flags in (P.LBM_LAUNCH_DEFAULT, 13):
        with P.Context(device=0, max_slots=8) as ctx:
            for prec in (0, 1):
                ctx.set_launch(prec, 256, 1, 1, flags)
            ctx.set_graph_chunk(4)
            slots = []
            for c, (f0, g0) in zip(cases, states):
                s = ctx.add(c)
                ctx.state_load(s, f0, g0)
                slots.append(s)
            ctx.step(slots[0], 11)            # single-cavity fused path (default depth)
            ctx.step_many(slots[1:], [11, 11, 11])  # batched paths
            got = [ctx.state_save(s) for s in slots]
        for k in range(len(cases)):
            assert np.array_equal(got[k][0], want[k][0]) and np.array_equal(got[k][1], want[k][1]), (flags, k)
    # both fused depths on the single-cavity path, FP64 and FP32
    for fuse in (2, 3):
        with P.Context(device=0, max_slots=2) as ctx:
            for prec in (0, 1):
                ctx.set_fusion(prec, fuse)
            for k in (0, 3):
                s = ctx.add(cases[k])
                ctx.state_load(s, *states[k])
                ctx.step(s, 11)
                f, g = ctx.state_save(s)
                assert np.array_equal(f, want[k][0]) and np.array_equal(g, want[k][1]), (fuse, k)

