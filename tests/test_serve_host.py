"""Scheduling of the request loop, on the host-only stand-in executor (no
GPU): admission by footprint within the budget, first fit in arrival order,
rejection of requests larger than the budget, continuous batching (new work
joins while other work is resident) and the latency summary."""
import numpy as np
import pytest

import paper_1909_13086_amd as P
from paper_1909_13086_amd import serve
from btrirt_workloads import cavity, serving_trace

MIB2 = 2 << 20


def footprint(case):
    return P.lbm_footprint(P.make_case(case))


def aligned(n):
    return (n + MIB2 - 1) // MIB2 * MIB2


def run(reqs, budget, chunk=100, mlups=2e4, scale=1.0):
    srv = serve.Server(None, budget, chunk, fake_mlups=mlups)
    for case, steps, t in reqs:
        srv.submit(case, steps, t)
    srv.run(scale)
    out = srv.requests(), srv.summary()
    srv.close()
    return out


def resident_bytes_over_time(recs):
    events = []
    for r in recs:
        if r["status"] == serve.LBM_REQ_DONE:
            events.append((r["t_admit"], aligned(r["bytes"])))
            events.append((r["t_done"], -aligned(r["bytes"])))
    events.sort(key=lambda e: (e[0], e[1]))
    cur, peak = 0, 0
    for _, d in events:
        cur += d
        peak = max(peak, cur)
    return peak


def test_all_requests_complete_with_exact_steps():
    reqs = [(cavity(256, 128, Ra=1e6), 300 + 50 * k, 0.002 * k) for k in range(8)]
    recs, s = run(reqs, 1 << 30, mlups=1e3)  # ~10 ms per request, arrivals every 2 ms
    assert s["completed"] == 8 and s["failed"] == 0 and s["rejected"] == 0
    for r, (_, steps, _) in zip(recs, reqs):
        assert r["status"] == serve.LBM_REQ_DONE
        assert r["stats"]["step"] == steps
        assert r["t_arrival"] <= r["t_admit"] <= r["t_done"]
    assert s["max_resident"] > 1  # later arrivals joined while others ran


def test_budget_is_never_exceeded_and_admission_waits():
    c = cavity(512, 256)
    fp = aligned(footprint(c))
    budget = 2 * fp + fp // 2  # room for two
    reqs = [(c, 400, 0.0), (c, 400, 0.0), (c, 400, 0.0), (c, 200, 0.0)]
    recs, s = run(reqs, budget, mlups=5e4)
    assert s["peak_bytes"] <= budget
    assert resident_bytes_over_time(recs) <= budget
    assert s["max_resident"] == 2
    first_done = min(recs[0]["t_done"], recs[1]["t_done"])
    assert recs[2]["t_admit"] >= first_done - 1e-9
    assert all(r["status"] == serve.LBM_REQ_DONE for r in recs)


def test_first_fit_lets_a_small_request_pass_a_large_one():
    big, small = cavity(1024, 512), cavity(128, 64)
    fb, fs = aligned(footprint(big)), aligned(footprint(small))
    budget = fb + fs  # one big plus one small
    reqs = [(big, 600, 0.0), (big, 100, 0.001), (small, 100, 0.002)]
    recs, s = run(reqs, budget, mlups=1e5)
    # the second big request waits for the first; the small one is admitted meanwhile
    assert recs[2]["t_admit"] < recs[1]["t_admit"]
    assert recs[1]["t_admit"] >= recs[0]["t_done"] - 1e-9


def test_oversized_request_is_rejected_alone():
    c = cavity(256, 128)
    reqs = [(c, 100, 0.0), (cavity(2048, 1024), 100, 0.0), (c, 100, 0.0)]
    recs, s = run(reqs, 4 * aligned(footprint(c)))
    assert [r["status"] for r in recs] == [serve.LBM_REQ_DONE, serve.LBM_REQ_REJECTED, serve.LBM_REQ_DONE]
    assert s["rejected"] == 1 and s["completed"] == 2


def test_latency_summary_matches_records():
    trace = serving_trace(seed=3, n=20, rate=400.0, steps_lo=100, steps_hi=400,
                          sizes=((128, 64), (256, 128)))
    reqs = [(dict(r["case"], precision=r["precision"]), r["steps"], r["arrival"]) for r in trace]
    recs, s = run(reqs, 64 << 20, mlups=1e4)
    lat = np.array([r["t_done"] - r["t_arrival"] for r in recs])
    assert s["completed"] == 20
    assert s["p50_s"] == pytest.approx(np.percentile(lat, 50), rel=1e-9)
    assert s["p99_s"] == pytest.approx(np.percentile(lat, 99), rel=1e-9)
    assert s["mean_s"] == pytest.approx(lat.mean(), rel=1e-9)
    lu = sum(r["cells"] * r["steps"] for r in recs)
    assert s["mlups"] == pytest.approx(lu / s["makespan_s"] / 1e6, rel=1e-9)
    assert 0.0 < s["busy_frac"] <= 1.0
    # arrivals are replayed on time: nobody is admitted before arriving
    for r, tr in zip(recs, trace):
        assert r["t_arrival"] == pytest.approx(tr["arrival"], abs=1e-12)
        assert r["t_admit"] >= r["t_arrival"]


def test_time_scale_compresses_arrivals():
    reqs = [(cavity(64, 32), 50, 0.2 * k) for k in range(4)]
    recs, _ = run(reqs, 64 << 20, scale=10.0)
    assert recs[-1]["t_arrival"] == pytest.approx(0.06, abs=1e-12)


def test_invalid_submissions():
    srv = serve.Server(None, 64 << 20, 100, fake_mlups=1e4)
    with pytest.raises(P.LbmError):
        srv.submit(cavity(0, 4), 10, 0.0)
    with pytest.raises(P.LbmError):
        srv.submit(cavity(8, 4), 0, 0.0)
    with pytest.raises(P.LbmError):
        serve.Server(None, 1 << 10, 100, fake_mlups=1e4)
    srv.close()


def test_finish_callback_reports_every_request_once_in_completion_order():
    c = cavity(256, 128)
    reqs = [(c, 300, 0.0), (cavity(2048, 1024), 100, 0.0), (c, 100, 0.01), (cavity(128, 64), 50, 0.02)]
    srv = serve.Server(None, 4 * aligned(footprint(c)), 100, fake_mlups=2e4)
    for case, steps, t in reqs:
        srv.submit(case, steps, t)
    seen = []
    srv.on_finish(seen.append)
    srv.run(1.0)
    recs = srv.requests()
    with pytest.raises(P.LbmError):  # the loop has run: no new callback
        srv.on_finish(None)
    srv.close()
    assert sorted(r["id"] for r in seen) == [0, 1, 2, 3]
    assert [r["t_done"] for r in seen] == sorted(r["t_done"] for r in seen)
    for r in seen:
        assert r == recs[r["id"]]
    assert [r["status"] for r in seen if r["id"] == 1] == [serve.LBM_REQ_REJECTED]
