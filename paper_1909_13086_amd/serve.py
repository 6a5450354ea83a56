"""Binding of the request loop (include/lbm_serve.h): argument marshalling only.

``Server`` queues melting solves with their arrival times and runs the
library's continuous-batching loop; ``bench_serving`` replays a seeded
Poisson trace of the paper's cavity problem for the benchmark.
"""
import ctypes

from . import _lib as L

LBM_REQ_QUEUED, LBM_REQ_RESIDENT, LBM_REQ_DONE, LBM_REQ_FAILED, LBM_REQ_REJECTED = 0, 1, 2, 3, 4


class lbm_request(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int32), ("status", ctypes.c_int32), ("precision", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("steps", ctypes.c_int64), ("cells", ctypes.c_int64),
        ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
        ("bytes", ctypes.c_size_t), ("stats", L.lbm_stats),
    ]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n not in ("stats", "pad")}
        d["stats"] = self.stats.as_dict()
        return d


class lbm_serve_summary(ctypes.Structure):
    _fields_ = [
        ("completed", ctypes.c_int32), ("failed", ctypes.c_int32), ("rejected", ctypes.c_int32),
        ("max_resident", ctypes.c_int32), ("chunks", ctypes.c_int64),
        ("makespan_s", ctypes.c_double), ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
        ("mean_s", ctypes.c_double), ("max_s", ctypes.c_double), ("mlups", ctypes.c_double),
        ("busy_frac", ctypes.c_double), ("peak_bytes", ctypes.c_size_t),
    ]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


REQUEST_FN = ctypes.CFUNCTYPE(None, ctypes.POINTER(lbm_request), ctypes.c_void_p)

_sig_done = False


def _lib():
    global _sig_done
    lib = L.lib()
    if not _sig_done:
        vp = ctypes.c_void_p
        lib.lbm_server_create.restype = ctypes.c_int
        lib.lbm_server_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_double]
        lib.lbm_server_destroy.restype = None
        lib.lbm_server_destroy.argtypes = [vp]
        lib.lbm_server_submit.restype = ctypes.c_int
        lib.lbm_server_submit.argtypes = [vp, ctypes.POINTER(L.lbm_case), ctypes.c_int64, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_int32)]
        lib.lbm_server_run.restype = ctypes.c_int
        lib.lbm_server_run.argtypes = [vp, ctypes.c_double]
        lib.lbm_server_request.restype = ctypes.c_int
        lib.lbm_server_request.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(lbm_request)]
        lib.lbm_server_summary.restype = ctypes.c_int
        lib.lbm_server_summary.argtypes = [vp, ctypes.POINTER(lbm_serve_summary)]
        lib.lbm_server_on_finish.restype = ctypes.c_int
        lib.lbm_server_on_finish.argtypes = [vp, REQUEST_FN, vp]
        _sig_done = True
    return lib


class Server:
    """ctx: an lbm context handle (Context.h) or None for the host-only
    stand-in executor running at fake_mlups."""

    def __init__(self, ctx, hbm_budget, chunk=100, fake_mlups=0.0):
        self.h = ctypes.c_void_p()
        L._check(_lib().lbm_server_create(ctypes.byref(self.h), ctx, int(hbm_budget), int(chunk),
                                          float(fake_mlups)))
        self.n = 0

    def submit(self, case, steps, arrival_s):
        c = case if isinstance(case, L.lbm_case) else L.make_case(case)
        rid = ctypes.c_int32()
        L._check(_lib().lbm_server_submit(self.h, ctypes.byref(c), int(steps), float(arrival_s),
                                          ctypes.byref(rid)))
        self.n += 1
        return rid.value

    def on_finish(self, fn):
        """fn(request dict) is called as each request leaves the loop."""
        self._cb = REQUEST_FN(lambda r, _user: fn(r.contents.as_dict())) if fn else REQUEST_FN()
        L._check(_lib().lbm_server_on_finish(self.h, self._cb, None))

    def run(self, time_scale=1.0):
        L._check(_lib().lbm_server_run(self.h, float(time_scale)))

    def request(self, rid):
        r = lbm_request()
        L._check(_lib().lbm_server_request(self.h, int(rid), ctypes.byref(r)))
        return r.as_dict()

    def requests(self):
        return [self.request(i) for i in range(self.n)]

    def summary(self):
        s = lbm_serve_summary()
        L._check(_lib().lbm_server_summary(self.h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self.h:
            _lib().lbm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bench_serving(P, n=48, rate=20.0, steps_lo=1000, steps_hi=5000, budget=16 << 30, chunk=100, seed=5,
                  progress_every=0, pattern=None):
    """Replays a seeded Poisson trace (sizes 256x128 ... 2048x1024, Ra
    log-uniform in [1e6, 1e8], random heater position, FP64 or FP32-shifted
    at random) through the loop and returns its summary.  pattern (None:
    in place) sets every request's streaming pattern.  With
    progress_every > 0 a line goes to stderr each time that many requests
    have finished."""
    import sys
    from btrirt_workloads import serving_trace
    trace = serving_trace(seed=seed, n=n, rate=rate, steps_lo=steps_lo, steps_hi=steps_hi)
    ctx = P.Context(device=0, max_slots=n, lend_memory=False)
    ctx.set_graph_chunk(chunk)
    srv = Server(ctx.h, budget, chunk)
    pattern = P.LBM_PATTERN_AA if pattern is None else pattern
    for r in trace:
        srv.submit(dict(r["case"], precision=r["precision"], pattern=pattern), r["steps"], r["arrival"])
    if progress_every > 0:
        done = [0]

        def report(req):
            done[0] += 1
            if done[0] % progress_every == 0 or done[0] == n:
                print(f"[serve] {done[0]}/{n} requests finished, t = {req['t_done']:.1f} s", file=sys.stderr,
                      flush=True)
        srv.on_finish(report)
    srv.run(1.0)
    s = srv.summary()
    srv.close()
    ctx.close()
    out = dict(requests=n, arrival_rate_per_s=rate, steps_range=[steps_lo, steps_hi], budget_bytes=budget,
               pattern="in place" if pattern == P.LBM_PATTERN_AA else
               "two lattices, fused launches (three steps; two for FP64 cavities below 2^18 cells, "
               "four for FP32 cavities from 2^21 cells)",
               p50_s=round(s["p50_s"], 4), p99_s=round(s["p99_s"], 4), mean_s=round(s["mean_s"], 4),
               mlups=round(s["mlups"], 1), makespan_s=round(s["makespan_s"], 3),
               busy_frac=round(s["busy_frac"], 4), max_resident=s["max_resident"],
               peak_bytes=s["peak_bytes"], completed=s["completed"], failed=s["failed"], chunks=s["chunks"])
    return out
