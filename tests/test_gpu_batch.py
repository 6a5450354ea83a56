"""Batched launch: many cavities of uneven size and precision advance in one
launch per step (optionally replayed from a captured graph); each cavity's
result must equal its own solo run bitwise, and the oracle's: FP64 cavities
per population at 1e-13, FP32-shifted ones at 2e-6 (a few units in the last
place of FP32 values of order one)."""
import numpy as np
import pytest

from btrirt_workloads import batch_sweep, cavity
from tests.test_gpu_parity import _random_state, oracle_run

FP64_POP_TOL, FP32_POP_TOL = 1e-13, 2e-6


def assert_matches_oracle(case, f0, g0, steps, pops):
    """Populations after `steps` steps from (f0, g0) against the oracle."""
    o = oracle_run(case, steps, f0, g0)
    fo, go = o.populations()
    tol = FP64_POP_TOL if case.get("precision", 0) == 0 else FP32_POP_TOL
    df, dg = float(np.max(np.abs(pops[0] - fo))), float(np.max(np.abs(pops[1] - go)))
    assert df <= tol and dg <= tol, (case["nx"], case["ny"], case.get("precision", 0), df, dg)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1909_13086_amd as P
    return P


def _cases(P):
    return [
        dict(cavity(256, 128, Ra=1e6, heater_center=0.3), precision=P.LBM_FP32_SHIFTED),
        dict(cavity(130, 33, periodic_x=1, Ra=3e5, heater_center=0.7), precision=P.LBM_FP64),
        dict(cavity(64, 64, Ra=1e7), precision=P.LBM_FP64, pattern=P.LBM_PATTERN_AB),
        dict(cavity(77, 21, Ra=2e6, heater_center=0.5), precision=P.LBM_FP32_SHIFTED,
             pattern=P.LBM_PATTERN_AB),
        dict(cavity(320, 160, Ra=1e8, heater_center=0.2), precision=P.LBM_FP32_SHIFTED),
    ]


def _solo(P, case, f0, g0, steps):
    with P.Context(device=0, max_slots=1) as ctx:
        s = ctx.add(case)
        ctx.state_load(s, f0, g0)
        ctx.step(s, steps)
        return ctx.state_save(s)


@pytest.mark.parametrize("chunk", [0, 10])
@pytest.mark.parametrize("steps", [1, 33])
def test_batch_equals_solo_bitwise(P, chunk, steps):
    print(f"case batch of 5, graph chunk {chunk}, steps {steps}", flush=True)
    cases = _cases(P)
    states = [_random_state(40 + k, c["nx"], c["ny"]) for k, c in enumerate(cases)]
    with P.Context(device=0, max_slots=8) as ctx:
        ctx.set_graph_chunk(chunk)
        slots = []
        for c, (f0, g0) in zip(cases, states):
            s = ctx.add(c)
            ctx.state_load(s, f0, g0)
            slots.append(s)
        # one slot starts one step ahead, so parities differ inside the batch
        ctx.step(slots[1], 1)
        ctx.step(P.LBM_ALL, steps)
        got = [ctx.state_save(s) for s in slots]
        infos = [ctx.info(s) for s in slots]
    for k, (c, (f0, g0)) in enumerate(zip(cases, states)):
        n = steps + (1 if k == 1 else 0)
        assert infos[k][0] == n
        want = _solo(P, c, f0, g0, n)
        assert np.array_equal(got[k][0], want[0]) and np.array_equal(got[k][1], want[1]), k
        assert_matches_oracle(c, f0, g0, n, got[k])


def test_batch_membership_changes_keep_results(P):
    """Slots join and leave between batched chunks; the captured graph is reused."""
    cases = _cases(P)
    states = [_random_state(60 + k, c["nx"], c["ny"]) for k, c in enumerate(cases)]
    with P.Context(device=0, max_slots=8) as ctx:
        ctx.set_graph_chunk(10)
        sl = {}
        for k in (0, 1, 2):
            sl[k] = ctx.add(cases[k])
            ctx.state_load(sl[k], *states[k])
        ctx.step(P.LBM_ALL, 20)
        ctx.release(sl.pop(1))
        for k in (3, 4):
            sl[k] = ctx.add(cases[k])
            ctx.state_load(sl[k], *states[k])
        ctx.step(P.LBM_ALL, 20)
        got = {k: ctx.state_save(s) for k, s in sl.items()}
        steps = {k: ctx.info(s)[0] for k, s in sl.items()}
    assert steps == {0: 40, 2: 40, 3: 20, 4: 20}
    for k, st in got.items():
        want = _solo(P, cases[k], *states[k], steps[k])
        assert np.array_equal(st[0], want[0]) and np.array_equal(st[1], want[1]), k


def test_batch_sweep_generator_shapes():
    cav = batch_sweep()
    assert len(cav) == 64
    assert all(256 <= c["nx"] <= 1024 and c["nx"] % 64 == 0 and c["ny"] == c["nx"] // 2 for c in cav)


def _ab_cases(P):
    return [
        dict(cavity(200, 50, Ra=1e6, heater_center=0.4), precision=P.LBM_FP64, pattern=P.LBM_PATTERN_AB),
        dict(cavity(130, 40, periodic_x=1, Ra=3e6, heater_center=0.6), precision=P.LBM_FP32_SHIFTED,
             pattern=P.LBM_PATTERN_AB),
        dict(cavity(96, 33, periodic_x=1, periodic_y=1, Ra=1e5), precision=P.LBM_FP64,
             pattern=P.LBM_PATTERN_AB),
        dict(cavity(150, 64, Ra=1e7, heater_center=0.5), precision=P.LBM_FP64),
    ]


@pytest.mark.parametrize("fuse,flags,seg,chunk", [(None, None, None, 4), (2, 13, 5, 4), (2, 21, 3, 4),
                                                  (2, 29, 1, 4), (3, None, None, 5), (3, 29, 2, 4),
                                                  (3, 21, 1, 5)])
def test_fused_batch_uneven_steps_equal_solo(P, fuse, flags, seg, chunk):
    """Two-lattice cavities advance two or three steps per batched launch (the
    one or two steps left of a chunk in its last launch), next to an in-place
    cavity, with per-slot step counts, graph chunks and every launch mode."""
    print(f"case fused batch fuse={fuse} flags={flags} seg={seg} chunk={chunk}", flush=True)
    cases = _ab_cases(P)
    states = [_random_state(70 + k, c["nx"], c["ny"]) for k, c in enumerate(cases)]
    counts = [7, 12, 1, 9]
    with P.Context(device=0, max_slots=8) as ctx:
        for prec in (0, 1):
            if flags is not None:
                ctx.set_launch(prec, 256, 1, 1, flags)
            if fuse is not None:
                ctx.set_fusion(prec, fuse, seg)
        ctx.set_graph_chunk(chunk)
        slots = []
        for c, (f0, g0) in zip(cases, states):
            s = ctx.add(c)
            ctx.state_load(s, f0, g0)
            slots.append(s)
        ctx.step_many(slots, counts)
        ctx.step(P.LBM_ALL, 10)
        got = [(ctx.state_save(s), ctx.reduce(s)) for s in slots]
    for k, c in enumerate(cases):
        n = counts[k] + 10
        with P.Context(device=0, max_slots=1) as ctx:
            s = ctx.add(c)
            ctx.state_load(s, *states[k])
            ctx.step(s, n)
            want = (ctx.state_save(s), ctx.reduce(s))
        assert got[k][1]["step"] == n
        assert np.array_equal(got[k][0][0], want[0][0]) and np.array_equal(got[k][0][1], want[0][1]), k
        for key in ("melt_fraction", "total_H", "heat_in_cum", "heater_q", "budget_residual"):
            assert got[k][1][key] == want[1][key], (k, key)
        assert_matches_oracle(c, *states[k], n, got[k][0])


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_autotune_choice_is_valid_cached_and_exact(P, tmp_path, prec):
    import json
    path = str(tmp_path / "tune.json")
    case = dict(cavity(200, 90, Ra=1e6, heater_center=0.4), pattern=P.LBM_PATTERN_AB, precision=prec)
    f0, g0 = _random_state(81, 200, 90)
    print(f"case autotune 200x90 precision {prec}", flush=True)
    with P.Context(device=0, max_slots=2) as ctx:
        ctx.autotune(prec, 200, 90, path)
        bx, by, cpl, flags = ctx.get_launch(prec)
        fuse, seg = ctx.get_fusion(prec)
        assert bx % 64 == 0 and bx * by <= 256 and cpl in (1, 2, 4) and 1 <= seg <= 12
        assert fuse in ((2, 3) if prec == 0 else (2, 3, 4))
        assert flags & P.LBM_LAUNCH_ZIGZAG
        s = ctx.add(case)
        ctx.state_load(s, f0, g0)
        ctx.step(s, 9)
        tuned = ctx.state_save(s)
    entry = list(json.load(open(path)).values())
    assert len(entry) == 1 and len(entry[0]) == (9 if prec == 0 else 11) and entry[0][:4] == [bx, by, cpl, flags]
    e = entry[0]
    per = {2: e[6] / 2, 3: e[8] / 3}
    if prec == 1:
        per[4] = e[10] / 4
    want = 3 if per[3] < per[2] else 2
    if prec == 1 and per[4] < per[want]:
        want = 4
    assert fuse == want and seg == {2: e[5], 3: e[7], 4: e[9] if prec == 1 else None}[fuse]
    with P.Context(device=0, max_slots=2) as ctx:
        ctx.autotune(prec, 200, 90, path)  # reuses the cached entry
        assert ctx.get_launch(prec) == (bx, by, cpl, flags) and ctx.get_fusion(prec) == (fuse, seg)
        ctx.set_fusion(prec, 1)
        s = ctx.add(case)
        ctx.state_load(s, f0, g0)
        ctx.step(s, 9)
        single = ctx.state_save(s)
    assert np.array_equal(tuned[0], single[0]) and np.array_equal(tuned[1], single[1])


@pytest.mark.parametrize("pattern", ["aa", "ab"])
def test_full_batch_sweep_equals_solo_runs(P, pattern):
    """The 64-cavity workload in the launch configuration the benchmark times
    (FP32 shifted, 100-step graphs, cache groups of at most 192 MiB): every
    cavity's diagnostics equal its solo run's bit for bit after a graph chunk
    and an odd remainder."""
    pat = P.LBM_PATTERN_AA if pattern == "aa" else P.LBM_PATTERN_AB
    cases = [dict(c, precision=P.LBM_FP32_SHIFTED, pattern=pat) for c in batch_sweep()]
    steps = 107
    print(f"case 64-cavity sweep ({pattern}) batched vs solo, {steps} steps", flush=True)
    with P.Context(device=0, max_slots=len(cases)) as ctx:
        ctx.set_graph_chunk(100)
        slots = [ctx.add(c) for c in cases]
        ctx.step(P.LBM_ALL, steps)
        got = [ctx.reduce(s) for s in slots]
    keys = ("melt_fraction", "total_H", "heat_in_cum", "heater_q", "mass", "max_u")
    with P.Context(device=0, max_slots=1) as ctx:
        for k, c in enumerate(cases):
            s = ctx.add(c)
            ctx.step(s, steps)
            want = ctx.reduce(s)
            ctx.release(s)
            assert got[k]["step"] == steps
            for key in keys:
                assert got[k][key] == want[key], (k, key)
