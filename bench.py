"""Throughput of the B-TriRT melting step on one MI355X.

Workload (the single-GPU configuration the metric is quoted on): one
2048x1024 D2Q9 cavity, FP64, Ra = 1e8, Pr = 1, Ste = 1, heater centred with
width W/4, starting all solid at Tm; flow and enthalpy populations advanced by
the fused collide-and-stream kernel on two lattices, three time steps per
launch (--path ab2: two steps per launch; --path aa: the in-place kernel, one
step per launch), diagnostics (melt fraction, Nusselt number, enthalpy
budget) reduced on the device every 100 steps.  A "step" is one time step of
that whole path.  Inputs are synthetic and resident in HBM before timing
starts.

Printed: one JSON line with MLUPS (10^6 lattice updates per second, one update
= one cell's f and g advanced one step), the roofline of the step kernel
(bytes a launch must move: the 18 populations of every cell read once from one
lattice and written once to the other, whatever the steps per launch), the
oracle timed on the host cores, the small-cavity solve latency, the FP32
error against FP64, and the in-place, FP32-shifted, 4096x2048, batched and
served variants.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# 18 populations read + written per cell and launch, FP64 / FP32: one lattice
# update for a one-step launch, and still the bytes a fused launch must move
BYTES_PER_LU = {0: 288, 1: 144}
REPORT_EVERY = 100
# per path: kernel name, sources (a change to any invalidates stored counter
# traffic), counter summary, steps per launch
CSRC = os.path.join(ROOT, "paper_1909_13086_amd", "csrc")
PATHS = {
    "ab": dict(kernel="k_step3<double,double,3>", src=("lbm_internal.h", "lbm_device.h", "lbm_step2.hip"),
               traffic=os.path.join(ROOT, "profiles", "traffic_k_step3_fp64_2048x1024.md"), per_launch=3,
               pattern="two lattices, three steps per launch, level-2 window in LDS"),
    "ab2": dict(kernel="k_step2<double,double,true,3>", src=("lbm_internal.h", "lbm_device.h", "lbm_step2.hip"),
                traffic=os.path.join(ROOT, "profiles", "traffic_k_step2_fp64_2048x1024.md"), per_launch=2,
                pattern="two lattices, two steps per launch, rows staged through LDS"),
    "aa": dict(kernel="k_step<double,double,1,false,0,SM> (SM = 0, 1: even and odd A-A steps)",
               src=("lbm_internal.h", "lbm_device.h", "lbm_step.hip"),
               traffic=os.path.join(ROOT, "profiles", "traffic_k_step_fp64_2048x1024.md"), per_launch=1,
               pattern="in-place A-A, one step per launch"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash(path):
    """sha256 of the path's kernel sources and of the build script (its
    compiler flags shape the kernel too)."""
    h = hashlib.sha256()
    for f in PATHS[path]["src"]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "paper_1909_13086_amd", "build.py"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path):
    """HBM bytes per launch of the path's step kernel from the committed
    rocprofv3 counter summary, or None when absent or taken on a different
    kernel source."""
    fn = PATHS[path]["traffic"]
    if not os.path.exists(fn):
        return None
    vals = {}
    for ln in open(fn):
        if ":" in ln:
            k, v = ln.split(":", 1)
            vals[k.strip().strip("-* `")] = v.strip().strip("` ")
    if vals.get("kernel_source_sha256") != kernel_hash(path):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_steps(P, ctx, slot, steps, events=True):
    """Runs `steps` steps; returns elapsed ms measured with events on the
    context's stream (the stream the kernels are launched on)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ctx.sync()
    e0.record(ctx.stream)
    ctx.step(slot, steps)
    e1.record(ctx.stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def run_cavity(P, path, steps, warmup, report_every=REPORT_EVERY, graph_chunk=0, tile=""):
    """The 2048x1024 FP64 cavity on a path ("ab", "ab2" or "aa"): `warmup`
    steps, then `steps` timed steps with diagnostics every `report_every`,
    then a kernel-only timing of whole launches."""
    from btrirt_workloads import large_cavity
    import torch

    per = PATHS[path]["per_launch"]
    case = dict(large_cavity(), pattern=P.LBM_PATTERN_AA if path == "aa" else P.LBM_PATTERN_AB)
    cells = case["nx"] * case["ny"]
    ctx = P.Context(device=0, max_slots=2)
    if path != "aa":
        ctx.set_fusion(0, per)
    if graph_chunk:
        ctx.set_graph_chunk(graph_chunk)
    if tile:
        bx, by, cpl, flags = (int(v) for v in tile.split(","))
        ctx.set_launch(0, bx, by, cpl, flags)
    slot = ctx.add(case)
    seg = ctx.get_fusion(0)[1]
    if report_every:
        ctx.set_report(slot, report_every, (steps + warmup) // report_every + 2)
    ctx.step(slot, warmup)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = time_steps(P, ctx, slot, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.reduce(slot)
    series = ctx.series(slot) if report_every else []
    # live time of the step kernel alone (whole launches, no diagnostics)
    slot2 = ctx.add(case)
    k2 = per * max(100, min(1000, steps // per))
    ctx.step(slot2, 20)
    kms = time_steps(P, ctx, slot2, k2)
    ctx.close()
    pattern = PATHS[path]["pattern"] + (f", {seg}-row segments" if path != "aa" else "")
    # diagnostics recorded inside the timed steps (warmup + 1 .. warmup + steps)
    in_window = sum(1 for e in series if warmup < e["step"] <= warmup + steps)
    return dict(case=case, cells=cells, ms=ms, wall=wall, stats=st, series=series, pattern=pattern,
                launch_ms=kms / k2 * per, launches=k2 // per, steps_per_launch=per, reports_in_window=in_window)


def roofline(path, m):
    """HBM roofline of the path's step kernel.  A launch, one step or a fused
    two or three, must read every cell's 18 populations once and write them
    once (the per-column strip flux adds 16 B per column): that is the
    algorithmic byte count per launch, so `frac` is at most 1.  The per-step
    rate (288 B per lattice update over the time per step) is reported apart
    as `effective_gbs`; for a fused launch it exceeds the bytes moved."""
    alg = BYTES_PER_LU[0] * m["cells"] + 16 * m["case"]["nx"]
    sec = m["launch_ms"] * 1e-3
    achieved = alg / sec / 1e9
    traffic = measured_traffic(path)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_over_algorithmic": round(traffic / alg, 4) if traffic else None,
            "kernel": PATHS[path]["kernel"], "kernel_avg_us": round(m["launch_ms"] * 1e3, 2),
            "steps_per_launch": m["steps_per_launch"], "algorithmic_bytes_per_launch": alg,
            "effective_gbs": round(BYTES_PER_LU[0] * m["cells"] * m["steps_per_launch"] / sec / 1e9, 1)}


def stream_ceiling(P, lattice_bytes, launches=40):
    """The layout's streaming ceiling at this lattice size, measured live with
    the library's probe (lbm_stream_probe: every 64-cell chunk read once and
    written once per launch, no arithmetic, in the step kernels' order): the
    two-lattice pattern (read one lattice, write the other) and in place.
    Each moves 2 x lattice_bytes per launch."""
    ctx = P.Context(device=0, max_slots=1)
    try:
        ab = ctx.stream_probe(lattice_bytes, P.LBM_PATTERN_AB, launches)
        aa = ctx.stream_probe(lattice_bytes, P.LBM_PATTERN_AA, launches)
    finally:
        ctx.close()
    moved = 2 * lattice_bytes
    res = {"lattice_bytes": lattice_bytes, "two_lattice_us": round(ab, 2), "in_place_us": round(aa, 2),
           "two_lattice_gbs": round(moved / (ab * 1e-6) / 1e9, 1), "in_place_gbs": round(moved / (aa * 1e-6) / 1e9, 1)}
    log(f"stream ceiling: {res}")
    return res


def in_place_variant(P, steps):
    """The same workload on the in-place A-A pattern (half the memory)."""
    m = run_cavity(P, "aa", steps, 100)
    mlups = m["cells"] * steps / (m["ms"] * 1e-3) / 1e6
    log(f"in-place A-A: {mlups:.0f} MLUPS, {m['launch_ms'] * 1e3:.2f} us/launch")
    return dict(mlups=round(mlups, 1), ms_per_step=round(m["ms"] / steps, 5), roofline=roofline("aa", m),
                melt_fraction=m["stats"]["melt_fraction"])


def fp32_variant(P, steps, path="ab"):
    from btrirt_workloads import large_cavity
    case = dict(large_cavity(), precision=P.LBM_FP32_SHIFTED,
                pattern=P.LBM_PATTERN_AA if path == "aa" else P.LBM_PATTERN_AB)
    ctx = P.Context(device=0, max_slots=1)
    if path == "ab2":
        ctx.set_fusion(P.LBM_FP32_SHIFTED, 2)
    slot = ctx.add(case)  # "ab": the default fusion for the cavity's size
    ctx.step(slot, 100)
    ms = time_steps(P, ctx, slot, steps)
    st = ctx.reduce(slot)
    fuse, seg = ctx.slot_fusion(slot)
    ctx.close()
    cells = case["nx"] * case["ny"]
    mlups = cells * steps / (ms * 1e-3) / 1e6
    pattern = (f"two lattices, {fuse} steps per launch, rows staged through LDS, {seg}-row segments"
               if path != "aa" else PATHS[path]["pattern"])
    log(f"fp32s ({pattern}): {mlups:.0f} MLUPS")
    per = fuse if path != "aa" else 1
    # bytes a launch must move (144 B per cell) over the time of one launch
    gbs = BYTES_PER_LU[1] * cells / (ms / steps * per * 1e-3) / 1e9
    return dict(mlups=round(mlups, 1), ms_per_step=round(ms / steps, 5), pattern=pattern, steps_per_launch=per,
                achieved_gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                effective_gbs=round(BYTES_PER_LU[1] * cells * steps / (ms * 1e-3) / 1e9, 1),
                melt_fraction=st["melt_fraction"])


def hbm_bound_variant(P, steps=240):
    """The same cavity physics on a 4096x2048 lattice, whose working set (1.2 GB
    FP64 and 604 MB FP32 in place, twice that on two lattices) is far above the
    256 MB Infinity Cache: the HBM-bound regime, in place and with the default
    fusion (three steps per launch in FP64, four in FP32)."""
    from btrirt_workloads import large_cavity
    out = {}
    for pattern, pname in ((P.LBM_PATTERN_AA, "in_place"), (P.LBM_PATTERN_AB, "fused")):
        for prec, name in ((0, "fp64"), (1, "fp32s")):
            case = dict(large_cavity(4096, 2048), precision=prec, pattern=pattern)
            ctx = P.Context(device=0, max_slots=1)
            slot = ctx.add(case)
            ctx.step(slot, 12)
            fuse = ctx.slot_fusion(slot)[0]
            ms = time_steps(P, ctx, slot, steps)
            ctx.close()
            cells = 4096 * 2048
            us = ms * 1e3 / steps
            # bytes a launch must move over the time of one launch (fuse steps)
            gbs = BYTES_PER_LU[prec] * cells / (us * fuse * 1e-6) / 1e9
            out[f"{pname}_{name}"] = dict(us_per_step=round(us, 2), mlups=round(cells / us, 1),
                                          steps_per_launch=fuse, achieved_gbs=round(gbs, 1),
                                          frac=round(gbs / HBM_PEAK_GBS, 4),
                                          effective_gbs=round(BYTES_PER_LU[prec] * cells / (us * 1e-6) / 1e9, 1))
    log(f"hbm-bound 4096x2048: {out}")
    return out


def fused_sizes_variant(P, steps=480):
    """The same cavity on the two-lattice pattern with two and three steps per
    launch (temporal blocking: each launch reads one lattice once and writes
    the other once) at 2048x1024 and 4096x2048, FP64."""
    from btrirt_workloads import large_cavity
    out = {}
    for fuse in (2, 3):
        for nx, ny in ((2048, 1024), (4096, 2048)):
            case = dict(large_cavity(nx, ny), pattern=P.LBM_PATTERN_AB)
            ctx = P.Context(device=0, max_slots=1)
            ctx.set_fusion(0, fuse)
            slot = ctx.add(case)
            ctx.step(slot, 12)
            ms = time_steps(P, ctx, slot, steps)
            ctx.close()
            us = ms * 1e3 / steps
            cells = nx * ny
            gbs = BYTES_PER_LU[0] * cells / (us * fuse * 1e-6) / 1e9
            out[f"{nx}x{ny}_{fuse}step"] = dict(us_per_step=round(us, 2), mlups=round(cells / us, 1),
                                                us_per_launch=round(fuse * us, 2),
                                                achieved_gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                                                effective_gbs=round(BYTES_PER_LU[0] * cells / (us * 1e-6) / 1e9, 1))
    log(f"fused two-lattice FP64: {out}")
    return out


def batched_variant(P, steps, chunk=100, pattern=None):
    """64 cavities of uneven size (seeded sweep), FP32 shifted: batched
    launches replayed from captured 100-step graphs (in place: one launch per
    step; two lattices: one launch per three steps, the FP32 default), against
    the same cavities solved one after another with the single-cavity path."""
    import torch
    from btrirt_workloads import batch_sweep
    pattern = P.LBM_PATTERN_AA if pattern is None else pattern
    cases = [dict(c, precision=P.LBM_FP32_SHIFTED, pattern=pattern) for c in batch_sweep()]
    cells = sum(c["nx"] * c["ny"] for c in cases)
    ctx = P.Context(device=0, max_slots=len(cases))
    ctx.set_graph_chunk(chunk)
    slots = [ctx.add(c) for c in cases]
    ctx.step(P.LBM_ALL, chunk)  # warm-up (captures the graph)
    ctx.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    ctx.step(P.LBM_ALL, steps)
    e1.record(ctx.stream)
    e1.synchronize()
    ms_b = e0.elapsed_time(e1)
    # the same work as sequential plain solves
    ctx.sync()
    e0.record(ctx.stream)
    for s in slots:
        ctx.step(s, steps)
    e1.record(ctx.stream)
    e1.synchronize()
    ms_s = e0.elapsed_time(e1)
    ctx.close()
    lu = cells * steps
    res = dict(cavities=len(cases), cells=cells, steps=steps,
               pattern="in place" if pattern == P.LBM_PATTERN_AA else "two lattices, three steps per launch",
               batched_mlups=round(lu / (ms_b * 1e-3) / 1e6, 1),
               sequential_mlups=round(lu / (ms_s * 1e-3) / 1e6, 1))
    res["speedup"] = round(res["batched_mlups"] / res["sequential_mlups"], 3)
    log(f"batched: {res}")
    return res


def small_cavity_solves(P, repeats=20, steps=2000):
    """The 128x64 FP64 cavity (Ra 1e4, literal rates k0 = k2 = 1) solved as a
    request: set up from all solid, 2000 steps, reduced.  Time to result of
    `repeats` solves after one warm-up solve (p50 / p99), with plain launches
    and with 100-step captured graphs (captured anew for each solve), and the
    device time per step.  The default launches apply (two lattices; an FP64
    cavity this small takes two steps per launch)."""
    import numpy as np
    from btrirt_workloads import small_cavity
    case = dict(small_cavity("literal"), pattern=P.LBM_PATTERN_AB)
    out = {}
    for chunk, name in ((0, "plain_launches"), (100, "graphs_100")):
        ctx = P.Context(device=0, max_slots=2)
        ctx.set_graph_chunk(chunk)
        times, phi = [], None
        for k in range(repeats + 1):
            t0 = time.perf_counter()
            s = ctx.add(case)
            ctx.step(s, steps)
            st = ctx.reduce(s)
            el = time.perf_counter() - t0
            fuse = ctx.slot_fusion(s)
            ctx.release(s)
            phi = st["melt_fraction"]
            if k > 0:
                times.append(el)
        s = ctx.add(case)
        ctx.step(s, 100)
        ms = time_steps(P, ctx, s, steps)
        ctx.close()
        out[name] = dict(p50_ms=round(float(np.percentile(times, 50)) * 1e3, 3),
                         p99_ms=round(float(np.percentile(times, 99)) * 1e3, 3),
                         us_per_step=round(ms * 1e3 / steps, 3), steps_per_launch=fuse[0], segment_rows=fuse[1])
    out.update(workload="128x64 FP64, Ra 1e4, k0 = k2 = 1, 2000 steps from all solid", repeats=repeats,
               melt_fraction=phi)
    log(f"small-cavity solves: {out}")
    return out


def fp32_error(P, times=(5000, 10000, 20000)):
    """The FP32-shifted variant of the small cavity (literal rates) against
    the same cavity in FP64, both on the GPU (the FP64 path equals the oracle
    to 1e-10 in the tests), at 5k, 10k and 20k steps: Linf of the liquid
    fraction field, |d melt fraction| and |d Nu|/Nu; in place and on two
    lattices with three steps per launch."""
    from btrirt_workloads import small_cavity
    out = {}
    for pattern, name in ((P.LBM_PATTERN_AA, "in_place"), (P.LBM_PATTERN_AB, "three_step")):
        ctx = P.Context(device=0, max_slots=2)
        if pattern == P.LBM_PATTERN_AB:
            ctx.set_fusion(0, 3, 4)
            ctx.set_fusion(1, 3, 6)
        s64 = ctx.add(dict(small_cavity("literal"), pattern=pattern))
        s32 = ctx.add(dict(small_cavity("literal"), pattern=pattern, precision=P.LBM_FP32_SHIFTED))
        rows, done = [], 0
        for t in times:
            ctx.step(s64, t - done)
            ctx.step(s32, t - done)
            done = t
            a, b = ctx.reduce(s64), ctx.reduce(s32)
            fa, fb = ctx.fields(s64, P.LBM_FIELD_FL)["fl"], ctx.fields(s32, P.LBM_FIELD_FL)["fl"]
            rows.append(dict(step=t, linf_fl=float(abs(fa - fb).max()),
                             dphi=abs(a["melt_fraction"] - b["melt_fraction"]),
                             dnu_rel=abs(a["nusselt"] - b["nusselt"]) / abs(a["nusselt"])))
        ctx.close()
        out[name] = rows
    log(f"fp32 vs fp64: {out}")
    return out


def serving_study(P, pattern):
    """The full serving workload (256 seeded Poisson requests at 20/s, sizes
    256x128 ... 2048x1024, 1000-50000 steps, FP64 / FP32-shifted 50/50, 16 GB
    budget), whose offered load is far above the device's, then the first 64
    requests of the same trace at an arrival rate that offers 70 % of the
    throughput the full run sustained."""
    from paper_1909_13086_amd import serve
    from btrirt_workloads import serving_trace
    full = serve.bench_serving(P, n=256, steps_hi=50000, progress_every=16, pattern=pattern)
    log(f"serving, full trace: {full}")
    n70 = 64
    tr = serving_trace(seed=5, n=n70, steps_hi=50000)
    mean_lu = sum(r["case"]["nx"] * r["case"]["ny"] * r["steps"] for r in tr) / n70
    rate = 0.7 * full["mlups"] * 1e6 / mean_lu
    at70 = serve.bench_serving(P, n=n70, rate=rate, steps_hi=50000, progress_every=8, pattern=pattern)
    at70["offered_mlups"] = round(rate * mean_lu / 1e6, 1)
    log(f"serving at 70 % of capacity: {at70}")
    return dict(full=full, at_70_percent=at70)


def cpu_baseline(target_s, single_steps=100):
    """The FP64 oracle on the host cores, on the same 2048x1024 cavity, for
    as many whole steps as fit in about target_s seconds, then on one thread
    for `single_steps` steps.  The oracle's source is compiled here, on the
    host that times it, at -O3 -march=native (as its plain C with the same
    floating-point contract), so the figure is that of this machine's cores."""
    import tempfile
    import oracle
    from oracle import build as obuild
    from btrirt_workloads import large_cavity
    tmp = tempfile.mkdtemp(prefix="oracle_native_")
    oracle.use_library(obuild.build_native(tmp))
    case = large_cavity()
    o = oracle.Oracle(oracle.case_from_dict(case)).init_solid()
    o.step(1)
    t0 = time.perf_counter()
    steps = 0
    while True:
        o.step(2)
        steps += 2
        el = time.perf_counter() - t0
        if el >= target_s:
            break
    cells = case["nx"] * case["ny"]
    mlups = cells * steps / el / 1e6
    threads = oracle.num_threads()
    log(f"cpu oracle: {steps} steps in {el:.1f} s = {mlups:.2f} MLUPS on {threads} threads")
    # the same on one thread
    oracle.set_threads(1)
    t0, steps1 = time.perf_counter(), 0
    for _ in range(single_steps // 10):
        o.step(10)
        steps1 += 10
    el1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    mlups1 = cells * steps1 / el1 / 1e6
    log(f"cpu oracle, one thread: {steps1} steps in {el1:.1f} s = {mlups1:.2f} MLUPS")
    return dict(value=round(mlups, 3), unit="MLUPS", cores=threads, kind="oracle",
                sample=f"2048x1024 FP64 cavity, {steps} steps after one warm-up step "
                       f"({el:.1f} s, OpenMP over rows; oracle built -O3 -march=native on this host)",
                single_thread_value=round(mlups1, 3), single_thread_steps=steps1,
                single_thread_seconds=round(el1, 1))


def heater_study(P, fo_end, precision, every_fo=0.005):
    """Heater-position study of Sec. 3.2 (the liquid-fraction curves of Fig. 3b):
    square 512x512 cavity, Ra = 1e8, Pr = 6.2, Ste = 0.125, heater width
    D = 0.5 L at centres C = 0.25, 0.375, 0.5 L, all three advanced together in
    fused batched launches on two lattices; melt fraction and Nusselt number
    every `every_fo` in Fourier number up to `fo_end`."""
    from btrirt_workloads import cavity
    cs = [0.25, 0.375, 0.5]
    cases = [dict(cavity(512, 512, Ra=1e8, Pr=6.2, Ste=0.125, heater_center=c, heater_width=0.5),
                  precision=precision, pattern=P.LBM_PATTERN_AB) for c in cs]
    lat = P.lbm_derive(P.make_case(cases[0]))
    steps_per = max(2, 2 * int(round(every_fo * 512 * 512 / lat.alpha / 2)))
    n_rep = int(round(fo_end / every_fo))
    ctx = P.Context(device=0, max_slots=3)
    ctx.set_graph_chunk(100)
    slots = [ctx.add(c) for c in cases]
    rows = []
    t0 = time.perf_counter()
    for k in range(n_rep):
        ctx.step_many(slots, [steps_per] * 3)
        st = [ctx.reduce(s, allow_unstable=True) for s in slots]
        rows.append(dict(fo=round(st[0]["fourier"], 5), step=st[0]["step"],
                         melt_fraction=[x["melt_fraction"] for x in st], nusselt=[x["nusselt"] for x in st],
                         finite=[x["finite"] for x in st]))
        log(f"study Fo={st[0]['fourier']:.4f} step={st[0]['step']} phi={[round(x['melt_fraction'], 5) for x in st]} "
            f"Nu={[round(x['nusselt'], 2) for x in st]} finite={[x['finite'] for x in st]} "
            f"({time.perf_counter() - t0:.0f} s)")
        if not all(x["finite"] for x in st):
            break
    ctx.close()
    return dict(study="heater position", centres=cs, alpha=lat.alpha, steps_per_report=steps_per,
                precision="fp64" if precision == 0 else "fp32s", series=rows)


def solid_study(P, fo_end, precision, every_fo=0.01, n=256):
    """Sensitivity of the melting to the readings the paper leaves open: the
    solid-phase treatment of the flow (velocity scaled by the liquid fraction,
    Carman-Kozeny drag, partial bounce-back) and the free rate k0 of the
    enthalpy populations (0.6, 1.0, 1.4 with the scaled velocity).  Square
    n x n cavity, Ra = 1e7, Pr = 6.2, Ste = 0.125, heater centred with width
    0.5 L; all cases advance together in fused batched launches."""
    from btrirt_workloads import cavity
    base = dict(cavity(n, n, Ra=1e7, Pr=6.2, Ste=0.125, heater_center=0.5, heater_width=0.5),
                precision=precision, pattern=P.LBM_PATTERN_AB)
    labels = ["scale k0=1", "darcy k0=1", "pbb k0=1", "scale k0=0.6", "scale k0=1.4"]
    cases = [dict(base, solid_model=0), dict(base, solid_model=1), dict(base, solid_model=2),
             dict(base, solid_model=0, k0_g=0.6), dict(base, solid_model=0, k0_g=1.4)]
    lat = P.lbm_derive(P.make_case(cases[0]))
    steps_per = max(2, 2 * int(round(every_fo * n * n / lat.alpha / 2)))
    ctx = P.Context(device=0, max_slots=len(cases))
    ctx.set_graph_chunk(100)
    slots = [ctx.add(c) for c in cases]
    rows = []
    t0 = time.perf_counter()
    for k in range(int(round(fo_end / every_fo))):
        ctx.step_many(slots, [steps_per] * len(slots))
        st = [ctx.reduce(s, allow_unstable=True) for s in slots]
        rows.append(dict(fo=round(st[0]["fourier"], 5), step=st[0]["step"],
                         melt_fraction=[x["melt_fraction"] for x in st], nusselt=[x["nusselt"] for x in st],
                         finite=[x["finite"] for x in st]))
        log(f"solid study Fo={st[0]['fourier']:.3f} phi={[round(x['melt_fraction'], 5) for x in st]} "
            f"Nu={[round(x['nusselt'], 2) for x in st]} ({time.perf_counter() - t0:.0f} s)")
        if not all(x["finite"] for x in st):
            break
    ctx.close()
    return dict(study="solid-phase readings and k0", cases=labels, alpha=lat.alpha, steps_per_report=steps_per,
                precision="fp64" if precision == 0 else "fp32s", series=rows)


def calib_copy(nbytes):
    """Plain device copy of a known size, for scaling HBM counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {nbytes} bytes x3")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--path", choices=["ab", "ab2", "aa"], default="ab",
                    help="ab: two lattices, three steps per launch (default); ab2: two lattices, two steps "
                         "per launch; aa: in place, one step per launch")
    ap.add_argument("--graph-chunk", type=int, default=0)
    ap.add_argument("--tile", default="", help="bx,by,cpl,flags for the FP64 step kernel")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extras", action="store_true", help="only the main workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving runs (about two minutes)")
    ap.add_argument("--calib-copy", type=int, default=0, help="run only a copy of this many bytes")
    ap.add_argument("--only", choices=["fp32", "batched", "batched_two_step", "serving", "serving_two_step",
                                       "serving_study", "sizes", "small_solve"],
                    default="",
                    help="run one variant alone (for profiling) and print its result")
    ap.add_argument("--study", choices=["heater", "solid"], default="",
                    help="run a study instead of the benchmark: heater position (Sec. 3.2) or solid-phase readings and k0")
    ap.add_argument("--fo", type=float, default=0.1, help="study: final Fourier number")
    ap.add_argument("--precision", choices=["fp64", "fp32s"], default="fp64", help="study precision")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}), flush=True)
        sys.exit(2)
    if args.calib_copy:
        calib_copy(args.calib_copy)
        return
    import paper_1909_13086_amd as P

    if args.study:
        prec = 0 if args.precision == "fp64" else 1
        res = heater_study(P, args.fo, prec) if args.study == "heater" else solid_study(P, args.fo, prec)
        print(json.dumps(res), flush=True)
        return

    if args.only:
        if args.only == "fp32":
            res = fp32_variant(P, max(500, args.steps // 4), args.path)
        elif args.only == "batched":
            res = batched_variant(P, args.steps)
        elif args.only == "batched_two_step":
            res = batched_variant(P, args.steps, pattern=P.LBM_PATTERN_AB)
        elif args.only == "sizes":
            res = fused_sizes_variant(P, args.steps)
        elif args.only == "small_solve":
            res = small_cavity_solves(P)
        elif args.only == "serving_study":
            res = serving_study(P, P.LBM_PATTERN_AA if args.path == "aa" else P.LBM_PATTERN_AB)
        elif args.only == "serving_two_step":
            from paper_1909_13086_amd import serve
            res = serve.bench_serving(P, pattern=P.LBM_PATTERN_AB)
        else:
            from paper_1909_13086_amd import serve
            res = serve.bench_serving(P)
        print(json.dumps({"only": args.only, **res}), flush=True)
        return

    path = args.path
    log(f"main: 2048x1024 FP64, {PATHS[path]['pattern']}, warmup {args.warmup}, steps {args.steps}")
    m = run_cavity(P, path, args.steps, args.warmup, graph_chunk=args.graph_chunk, tile=args.tile)
    log(f"main: {m['ms']:.1f} ms event, {m['wall'] * 1e3:.1f} ms wall, melt fraction "
        f"{m['stats']['melt_fraction']:.6f}, Nu {m['stats']['nusselt']:.3f}, finite {m['stats']['finite']}, "
        f"{len(m['series'])} reports, {m['launch_ms'] * 1e3:.2f} us/launch")
    mlups = m["cells"] * args.steps / (m["ms"] * 1e-3) / 1e6
    out = {
        "metric": "MLUPS (flow+enthalpy) & % HBM roofline; batched vs plain; p50/p99 solve latency",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single cavity 2048x1024 D2Q9, FP64, Ra=1e8 Pr=1 Ste=1, heater W/4 centred, "
                               "from all-solid at Tm; diagnostics every 100 steps",
                   "nx": 2048, "ny": 1024, "precision": "fp64", "pattern": m["pattern"],
                   "reports_in_timed_window": m["reports_in_window"]},
        "roofline": roofline(path, m),
        "melt_fraction": m["stats"]["melt_fraction"],
        "nusselt": m["stats"]["nusselt"],
        "budget_residual": m["stats"]["budget_residual"],
    }
    # the fused launch against what a pure stream of its pattern achieves on this device
    lattice_bytes = 18 * 8 * m["case"]["nx"] * m["case"]["ny"]
    ceil = stream_ceiling(P, lattice_bytes)
    pattern_us = ceil["in_place_us"] if path == "aa" else ceil["two_lattice_us"]
    out["roofline"]["stream_ceiling"] = ceil
    out["roofline"]["frac_of_stream_ceiling"] = round(pattern_us / (m["launch_ms"] * 1e3), 4)
    if not args.no_extras:
        if path != "aa":
            out["in_place_aa"] = in_place_variant(P, max(1000, args.steps // 4))
        out["fp32_shifted"] = fp32_variant(P, max(500, args.steps // 4), path)
        out["hbm_bound_4096x2048"] = hbm_bound_variant(P)
        out["small_cavity_solve"] = small_cavity_solves(P)
        out["fp32_vs_fp64"] = fp32_error(P)
        out["batched"] = batched_variant(P, 2000)
        out["batched_two_step"] = batched_variant(P, 2000, pattern=P.LBM_PATTERN_AB)
        if not args.no_serving:
            out["serving"] = serving_study(P, P.LBM_PATTERN_AB)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
