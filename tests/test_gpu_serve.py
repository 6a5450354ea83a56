"""Serving on the GPU: requests that arrive while others run are admitted as
memory frees up, share batched launches, and each result equals the same
solve run alone (bitwise, since the batched and single-cavity launches
perform the same arithmetic) and the FP64 oracle's: FP64 requests at the FP64
bar, FP32-shifted ones within 1e-4 in melt fraction and 0.5 % in Nusselt
number.  A request that goes non-finite fails alone."""
import numpy as np
import pytest

import oracle
from btrirt_workloads import cavity

_ORACLE = {}


def oracle_result(case, steps):
    """Fields and stats of the oracle after `steps` steps from all solid (the
    oracle ignores precision and storage pattern, so runs are shared)."""
    key = (tuple(sorted((k, v) for k, v in case.items() if k not in ("precision", "pattern"))), steps)
    if key not in _ORACLE:
        o = oracle.Oracle(oracle.case_from_dict(case)).init_solid().step(steps)
        _ORACLE[key] = (o.fields(), o.stats())
    return _ORACLE[key]

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1909_13086_amd as P
    return P


def solo_stats(P, case, steps, fields=False):
    with P.Context(device=0, max_slots=1) as ctx:
        s = ctx.add(case)
        ctx.step(s, steps)
        st = ctx.reduce(s, allow_unstable=True)
        return (st, ctx.fields(s)) if fields else st


def _trace(P, patterns):
    sizes = [(64, 32), (128, 64), (256, 128), (96, 48), (200, 100)]
    out = []
    for k in range(12):
        nx, ny = sizes[k % len(sizes)]
        prec = P.LBM_FP32_SHIFTED if k % 2 else P.LBM_FP64
        case = dict(cavity(nx, ny, Ra=10 ** (5 + (k % 3)), heater_center=0.2 + 0.05 * k), precision=prec,
                    pattern=patterns[k % len(patterns)], solid_model=(k // 4) % 3)
        out.append((case, 1500 + 97 * k, 0.0005 * k))
    return out


@pytest.mark.parametrize("patterns", ["aa", "ab", "mixed"])
def test_served_results_equal_solo_runs(P, patterns):
    """In place, on two lattices (two-step batched launches, odd remainders
    included) and both mixed, with all three solid readings in the mix."""
    from paper_1909_13086_amd import serve
    pat = {"aa": [P.LBM_PATTERN_AA], "ab": [P.LBM_PATTERN_AB],
           "mixed": [P.LBM_PATTERN_AA, P.LBM_PATTERN_AB, P.LBM_PATTERN_AB]}[patterns]
    trace = _trace(P, pat)
    fp = [P.lbm_footprint(P.make_case(c)) for c, _, _ in trace]
    budget = 4 * max(fp) + (8 << 20)  # admission binds: a few resident at a time
    print(f"case serving 12 requests ({patterns}), budget {budget} bytes", flush=True)
    with P.Context(device=0, max_slots=16, lend_memory=False) as ctx:
        ctx.set_graph_chunk(50)
        srv = serve.Server(ctx.h, budget, chunk=50)
        for c, steps, t in trace:
            srv.submit(c, steps, t)
        srv.run(1.0)
        recs, summ = srv.requests(), srv.summary()
        srv.close()
    assert summ["completed"] == len(trace) and summ["failed"] == 0
    assert summ["peak_bytes"] <= budget
    assert summ["max_resident"] >= 2
    for r, (c, steps, _) in zip(recs, trace):
        assert r["status"] == serve.LBM_REQ_DONE
        want, fields = solo_stats(P, c, steps, fields=True)
        got = r["stats"]
        assert got["step"] == steps
        for k in ("melt_fraction", "total_H", "heat_in_cum", "nusselt", "mass", "max_u", "budget_residual"):
            assert got[k] == want[k], (r["id"], k)
        # the request in the mix against the oracle
        ofields, ost = oracle_result(c, steps)
        if c["precision"] == P.LBM_FP64:
            err = {n: float(np.max(np.abs(fields[n] - ofields[n]))) for n in ("H", "ux", "uy", "T", "fl")}
            assert max(err.values()) <= 1e-10, (r["id"], err)
            assert got["melt_fraction"] == pytest.approx(ost["melt_fraction"], abs=1e-12), r["id"]
            assert got["nusselt"] == pytest.approx(ost["nusselt"], rel=1e-10), r["id"]
            assert got["total_H"] == pytest.approx(ost["total_H"], rel=1e-12), r["id"]
            assert got["heat_in_cum"] == pytest.approx(ost["heat_in_cum"], rel=1e-12), r["id"]
        else:
            assert abs(got["melt_fraction"] - ost["melt_fraction"]) <= 1e-4, r["id"]
            assert abs(got["nusselt"] - ost["nusselt"]) <= 5e-3 * abs(ost["nusselt"]), r["id"]


def test_unstable_request_fails_alone(P):
    from paper_1909_13086_amd import serve
    good = [dict(cavity(128, 64, Ra=1e5), precision=P.LBM_FP64),
            dict(cavity(96, 48, Ra=1e6), precision=P.LBM_FP32_SHIFTED)]
    # a lattice Mach number far above 1 drives the flow unstable within a few hundred steps
    bad = dict(cavity(64, 64, Ra=1e6, Ma=4.0), init=P.LBM_INIT_GAUSSIAN, T0=0.5, gauss_amp=1.0,
               gauss_sigma=10.0, precision=P.LBM_FP64)
    with P.Context(device=0, max_slots=8, lend_memory=False) as ctx:
        srv = serve.Server(ctx.h, 256 << 20, chunk=40)
        ids = [srv.submit(good[0], 400, 0.0), srv.submit(bad, 400, 0.0), srv.submit(good[1], 300, 0.0)]
        srv.run(1.0)
        recs = [srv.request(i) for i in ids]
        srv.close()
    assert [r["status"] for r in recs] == [serve.LBM_REQ_DONE, serve.LBM_REQ_FAILED, serve.LBM_REQ_DONE]
    assert recs[1]["stats"]["finite"] == 0
    for r, c, steps in ((recs[0], good[0], 400), (recs[2], good[1], 300)):
        want = solo_stats(P, c, steps)
        assert r["stats"]["melt_fraction"] == want["melt_fraction"]
        assert r["stats"]["total_H"] == want["total_H"]


@pytest.mark.parametrize("group_bytes", [2 << 20, 1 << 20])
def test_step_many_uneven_counts_equal_solo(P, group_bytes):
    """Batched steps with uneven counts over several cache groups (2 MiB), and
    with the two in-place cavities larger than a group (1 MiB), which then
    step on the single-cavity path beside the batched one."""
    import numpy as np
    print(f"case step_many uneven counts, groups of {group_bytes} B", flush=True)
    cases = [dict(cavity(128, 64, Ra=1e5), precision=P.LBM_FP64),
             dict(cavity(192, 96, Ra=1e6, heater_center=0.3), precision=P.LBM_FP32_SHIFTED),
             dict(cavity(64, 32, Ra=1e7), precision=P.LBM_FP64, pattern=P.LBM_PATTERN_AB)]
    counts = [131, 57, 200]
    with P.Context(device=0, max_slots=4) as ctx:
        ctx.set_graph_chunk(25)
        ctx.set_group_bytes(group_bytes)
        slots = [ctx.add(c) for c in cases]
        ctx.step_many(slots, counts)
        got = [ctx.state_save(s) for s in slots]
    for c, n, g in zip(cases, counts, got):
        with P.Context(device=0, max_slots=1) as ctx:
            s = ctx.add(c)
            ctx.step(s, n)
            want = ctx.state_save(s)
        assert np.array_equal(g[0], want[0]) and np.array_equal(g[1], want[1])
