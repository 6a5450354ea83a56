"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

FP64 bar (from the problem statement of this path): max|dH|, max|du| <= 1e-10
after 2000 steps.  Storage patterns and tile shapes must agree bitwise, since
they only change where the same arithmetic reads and writes.
"""
import numpy as np
import pytest

import oracle
from btrirt_workloads import cavity, large_cavity, random_planes, small_cavity

pytestmark = pytest.mark.gpu

TOL = 1e-10
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1909_13086_amd as P
    return P


@pytest.fixture()
def ctx(P):
    c = P.Context(device=0, max_slots=16)
    yield c
    c.close()


def oracle_run(case, steps, f0=None, g0=None):
    o = oracle.Oracle(oracle.case_from_dict(case))
    if f0 is not None:
        o.set_populations(f0, g0)
    else:
        o.init_solid()
    o.step(steps)
    return o


def max_field_err(got, want, names=("H", "T", "fl", "ux", "uy", "rho")):
    return {n: float(np.max(np.abs(got[n] - want[n]))) for n in names}


_ORACLE_2000 = {}


def oracle_2000(variant):
    """The oracle's state of a small-cavity variant after 2000 steps (computed once)."""
    if variant not in _ORACLE_2000:
        o = oracle_run(small_cavity(variant), 2000)
        _ORACLE_2000[variant] = (o.fields(), o.stats())
    return _ORACLE_2000[variant]


# Launch paths of a single cavity: (pattern, steps per launch, segment rows).
# "ab3" is the benchmark's kernel (two lattices, three steps per launch,
# 4-row segments); "ab2" the two-step kernel; "ab1" single two-lattice steps.
PATHS = {"aa": (0, 1, 0), "ab1": (1, 1, 0), "ab2": (1, 2, 2), "ab3": (1, 3, 4)}


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("variant", ["literal", "eq6", "distinct"])
def test_small_cavity_2000_steps(P, variant, path):
    """Eq. (2) end to end: 2000 steps from all solid on every launch path,
    against the oracle at the FP64 bar."""
    pattern, fuse, seg = PATHS[path]
    case = dict(small_cavity(variant), pattern=pattern)
    print(f"case small_cavity[{variant}] 128x64 FP64 2000 steps, path {path}", flush=True)
    with P.Context(device=0, max_slots=1) as ctx:
        if pattern == 1:
            ctx.set_fusion(0, fuse, seg or None)
        s = ctx.add(case)
        if pattern == 1:
            assert ctx.slot_fusion(s)[0] == fuse
        ctx.step(s, 2000)
        got, st = ctx.fields(s), ctx.reduce(s)
    want, ost = oracle_2000(variant)
    _check_small_cavity(got, st, want, ost)


@pytest.mark.parametrize("fuse", [1, 2, 3])
def test_small_cavity_2000_steps_batched(P, fuse):
    """The three rate variants advance together in batched launches (two
    lattices, `fuse` steps per launch, 100-step graphs) beside an in-place copy
    of each; all six against the oracle at the FP64 bar."""
    variants = ["literal", "eq6", "distinct"]
    print(f"case small_cavity x3 batched, {fuse} steps per launch, 2000 steps", flush=True)
    with P.Context(device=0, max_slots=6) as ctx:
        ctx.set_fusion(0, fuse, 4 if fuse == 3 else None)
        ctx.set_graph_chunk(100)
        slots = [ctx.add(dict(small_cavity(v), pattern=pat)) for pat in (1, 0) for v in variants]
        ctx.step_many(slots, [2000] * len(slots))
        res = [(ctx.fields(s), ctx.reduce(s)) for s in slots]
    for k, (got, st) in enumerate(res):
        want, ost = oracle_2000(variants[k % 3])
        _check_small_cavity(got, st, want, ost)


def _check_small_cavity(got, st, want, ost):
    err = max_field_err(got, want)
    assert err["H"] <= TOL and err["ux"] <= TOL and err["uy"] <= TOL, err
    assert max(err.values()) <= TOL, err
    assert st["step"] == 2000 and st["finite"] == 1
    assert st["melt_fraction"] == pytest.approx(ost["melt_fraction"], abs=1e-12)
    assert st["nusselt"] == pytest.approx(ost["nusselt"], rel=1e-10)
    assert st["heater_q"] == pytest.approx(ost["heater_q"], rel=1e-10)
    assert st["total_H"] == pytest.approx(ost["total_H"], rel=1e-12)
    assert st["heat_in_cum"] == pytest.approx(ost["heat_in_cum"], rel=1e-12)
    # the oracle stores f unshifted and its mass drifts by ~1e-13 relative over
    # 2000 steps of round-off; the shifted storage keeps it to ~1e-16
    assert st["mass"] == pytest.approx(ost["mass"], rel=1e-12)
    assert st["max_u"] == pytest.approx(ost["max_u"], rel=1e-8)
    assert abs(st["budget_residual"]) <= 1e-12 * st["total_H"]
    assert st["fourier"] == pytest.approx(ost["fourier"], rel=1e-14)


def _random_state(seed, nx, ny):
    r = random_planes(seed, 18, ny, nx)
    f = W[:, None, None] * (1.0 + 0.1 * (r[:9] - 0.5))
    g = W[:, None, None] * (2.5 * r[9:] - 0.5)  # enthalpy spans solid, mushy and liquid cells
    return f, g


GEOMS = [
    # nx, ny, periodic_x, periodic_y, heater centre, width
    (1, 40, 1, 0, 0.5, 1.0),
    (3, 5, 0, 0, 0.5, 1.0),
    (65, 7, 0, 0, 0.1, 0.5),
    (130, 33, 1, 0, 0.9, 0.4),
    (64, 64, 1, 1, 0.5, 0.25),
    (200, 3, 0, 1, 0.5, 0.25),
    (77, 1, 0, 0, 0.5, 0.3),
]


@pytest.mark.parametrize("geom", GEOMS, ids=[f"{g[0]}x{g[1]}p{g[2]}{g[3]}" for g in GEOMS])
@pytest.mark.parametrize("steps", [1, 8, 13])
def test_random_states_and_boundaries(ctx, P, geom, steps):
    nx, ny, px, py, hc, hw = geom
    case = cavity(nx, ny, periodic_x=px, periodic_y=py, heater_center=hc, heater_width=hw,
                  param_mode=1, nu=0.04, alpha=0.06, gbeta=3e-3, latent=0.8, Tm=0.1, Th=0.9,
                  k0_g=0.9, k2_g=1.2, k0_f=1.1, k1_f=0.85)
    print(f"case random {nx}x{ny} periodic=({px},{py}) heater=({hc},{hw}) steps={steps}", flush=True)
    f0, g0 = _random_state(1000 + nx + ny, nx, ny)
    s = ctx.add(case)
    ctx.state_load(s, f0, g0)
    ctx.step(s, steps)
    fg, gg = ctx.state_save(s)
    o = oracle_run(case, steps, f0, g0)
    fo, go = o.populations()
    assert np.max(np.abs(fg - fo)) <= 1e-13
    assert np.max(np.abs(gg - go)) <= 1e-13
    err = max_field_err(ctx.fields(s), o.fields())
    assert max(err.values()) <= 1e-13, err
    st, ost = ctx.reduce(s), o.stats()
    for k in ("melt_fraction", "total_H", "mass", "heater_q", "heat_in_cum"):
        assert st[k] == pytest.approx(ost[k], rel=1e-12, abs=1e-13), k


def test_state_load_save_round_trip(ctx):
    nx, ny = 70, 9
    f0, g0 = _random_state(5, nx, ny)
    s = ctx.add(cavity(nx, ny))
    ctx.state_load(s, f0, g0)
    f1, g1 = ctx.state_save(s)
    assert np.max(np.abs(f1 - f0)) <= 2e-16 and np.max(np.abs(g1 - g0)) <= 4e-16


def _run_state(ctx, P, case, steps, f0, g0, launch=None):
    if launch is not None:
        ctx.set_launch(case.get("precision", 0), *launch)
    s = ctx.add(case)
    ctx.state_load(s, f0, g0)
    ctx.step(s, steps)
    out = ctx.state_save(s)
    ctx.release(s)
    return out


@pytest.mark.parametrize("steps", [37, 38])
def test_patterns_and_tiles_agree_bitwise(ctx, P, steps):
    base = small_cavity("distinct")
    f0, g0 = _random_state(9, 128, 64)
    ref = _run_state(ctx, P, dict(base, pattern=P.LBM_PATTERN_AB), steps, f0, g0)
    # (bx, by, cpl, flags): flags bit 0 = XCD bands, bit 1 = non-temporal access,
    # bit 2 = tiles walked backwards on every other step, bit 3 = zigzag
    # segment walk of the two-step kernel (no effect on the in-place pattern)
    for launch in [(256, 1, 1, 1), (64, 4, 2, 0), (128, 2, 4, 1), (64, 1, 1, 0), (256, 1, 1, 3), (128, 2, 2, 2),
                   (64, 1, 1, 5), (128, 2, 2, 4), (64, 4, 1, 7), (64, 4, 1, 15)]:
        got = _run_state(ctx, P, dict(base), steps, f0, g0, launch)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), launch
    for flags in (0, 5, 8, 13, 16, 29):
        got = _run_state(ctx, P, dict(base, pattern=P.LBM_PATTERN_AB), steps, f0, g0, (256, 1, 1, flags))
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), flags
    ctx.set_launch(0, 256, 1, 1, P.LBM_LAUNCH_DEFAULT)


def test_graph_chunks_equal_plain_launches(ctx, P):
    case = small_cavity("eq6")
    f0, g0 = _random_state(3, 128, 64)
    ref = _run_state(ctx, P, case, 47, f0, g0)
    ctx.set_graph_chunk(10)
    got = _run_state(ctx, P, case, 47, f0, g0)
    ctx.set_graph_chunk(0)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_recorded_series_matches_direct_reductions(ctx):
    case = small_cavity("eq6")
    s = ctx.add(case)
    ctx.set_report(s, 100, 16)
    ctx.step(s, 450)
    series = ctx.series(s)
    assert [e["step"] for e in series] == [100, 200, 300, 400]
    s2 = ctx.add(case)
    for e in series:
        ctx.step(s2, e["step"] - ctx.info(s2)[0])
        d = ctx.reduce(s2)
        for k in ("melt_fraction", "total_H", "heat_in_cum", "nusselt", "budget_residual"):
            assert e[k] == d[k], k


def test_large_cavity_full_size_20_steps(ctx):
    case = large_cavity()
    print("case 2048x1024 FP64 20 steps vs oracle", flush=True)
    f0, g0 = _random_state(21, 2048, 1024)
    s = ctx.add(case)
    ctx.state_load(s, f0, g0)
    ctx.step(s, 20)
    got = ctx.fields(s)
    o = oracle_run(case, 20, f0, g0)
    err = max_field_err(got, o.fields())
    assert max(err.values()) <= 1e-12, err
    st, ost = ctx.reduce(s), o.stats()
    assert st["total_H"] == pytest.approx(ost["total_H"], rel=1e-13)
    assert st["melt_fraction"] == pytest.approx(ost["melt_fraction"], abs=1e-13)


def test_non_finite_state_is_reported(ctx, P):
    nx, ny = 16, 8
    f0, g0 = _random_state(2, nx, ny)
    g0[0, 3, 5] = np.nan
    s = ctx.add(cavity(nx, ny))
    ctx.state_load(s, f0, g0)
    with pytest.raises(P.LbmError) as ei:
        ctx.reduce(s)
    assert ei.value.code == P.LBM_EUNSTABLE
    assert ctx.reduce(s, allow_unstable=True)["finite"] == 0


def test_budget_admission(P):
    case = P.make_case(cavity(256, 128))
    need = P.lbm_footprint(case)
    with P.Context(device=0, hbm_budget=2 * need + need // 2, max_slots=4, lend_memory=False) as c:
        a = c.add(case)
        c.add(case)
        with pytest.raises(P.LbmError) as ei:
            c.add(case)
        assert ei.value.code == P.LBM_ENOMEM
        c.release(a)
        c.add(case)


@pytest.mark.parametrize("pattern,prec", [(0, 0), (1, 0), (0, 1)])
def test_checkpoint_resume_is_bitwise(P, pattern, prec):
    case = dict(small_cavity("distinct"), pattern=pattern, precision=prec)
    print(f"case checkpoint pattern={pattern} precision={prec}", flush=True)
    with P.Context(device=0, max_slots=2) as ctx:
        a = ctx.add(case)
        ctx.step(a, 437)  # odd: the in-place pattern is in its swapped parity
        blob = ctx.checkpoint(a)
        ctx.step(a, 563)
        want, want_st = ctx.state_save(a), ctx.reduce(a)
    with P.Context(device=0, max_slots=2) as ctx:
        b = ctx.add(dict(case, Ra=3e4))  # restored slot takes the checkpoint's case
        ctx.restore(b, blob)
        assert ctx.info(b)[0] == 437
        ctx.step(b, 563)
        got, got_st = ctx.state_save(b), ctx.reduce(b)
        wrong = ctx.add(dict(case, nx=64))
        with pytest.raises(P.LbmError):
            ctx.restore(wrong, blob)
        with pytest.raises(P.LbmError):
            ctx.restore(b, blob[:100])
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    for k in ("step", "melt_fraction", "total_H", "heat_in_cum", "budget_residual", "nusselt"):
        assert got_st[k] == want_st[k], k
    # the resumed run against an uninterrupted oracle run of 1000 steps
    o = oracle_run(case, 1000)
    ost = o.stats()
    if prec == 0:
        with P.Context(device=0, max_slots=1) as ctx:
            s = ctx.add(case)
            ctx.state_load(s, *got)
            fields = ctx.fields(s)
        err = max_field_err(fields, o.fields())
        assert max(err.values()) <= TOL, err
        assert got_st["melt_fraction"] == pytest.approx(ost["melt_fraction"], abs=1e-12)
        assert got_st["nusselt"] == pytest.approx(ost["nusselt"], rel=1e-10)
    else:
        assert abs(got_st["melt_fraction"] - ost["melt_fraction"]) <= 1e-4
        assert abs(got_st["nusselt"] - ost["nusselt"]) <= 5e-3 * abs(ost["nusselt"])


FUSED_GEOMS = GEOMS + [(130, 70, 0, 0, 0.4, 0.3), (200, 37, 1, 1, 0.5, 0.25), (63, 17, 1, 0, 0.6, 0.5)]


# free rates of both populations: all distinct, and k0 = 1 for f and g, for
# which the fused kernels drop the (1 - k0) p term of Eq. (2) while the
# single-step kernel keeps it
FUSED_RATES = {"general": dict(k0_g=0.9, k2_g=1.2, k0_f=1.1, k1_f=0.85),
               "unit_k0": dict(k0_g=1.0, k2_g=1.2, k0_f=1.0, k1_f=0.85)}


@pytest.mark.parametrize("rates", sorted(FUSED_RATES))
@pytest.mark.parametrize("geom", FUSED_GEOMS, ids=[f"{g[0]}x{g[1]}p{g[2]}{g[3]}" for g in FUSED_GEOMS])
@pytest.mark.parametrize("prec,seg,steps", [(0, 8, 2), (0, 16, 7), (1, 32, 6), (0, 32, 13), (1, 8, 5),
                                             (0, 6, 4), (1, 5, 3), (0, 1, 2), (0, 3, 5), (1, 64, 4)])
def test_fused_kernels_equal_single_steps(P, geom, prec, seg, steps, rates):
    nx, ny, px, py, hc, hw = geom
    case = dict(cavity(nx, ny, periodic_x=px, periodic_y=py, heater_center=hc, heater_width=hw,
                       param_mode=1, nu=0.04, alpha=0.06, gbeta=3e-3, latent=0.8, Tm=0.1, Th=0.9,
                       **FUSED_RATES[rates]),
                precision=prec, pattern=P.LBM_PATTERN_AB)
    print(f"case two-step {nx}x{ny} periodic=({px},{py}) prec={prec} seg={seg} steps={steps} rates={rates}",
          flush=True)
    f0, g0 = _random_state(2000 + nx + ny, nx, ny)
    out = []
    # single steps, two-step launches with the zigzag segment walk (default)
    # and with every segment walked upwards, rows loaded directly or staged
    modes = [(1, P.LBM_LAUNCH_DEFAULT), (2, P.LBM_LAUNCH_DEFAULT), (2, 5), (2, 5 | P.LBM_LAUNCH_STAGED),
             (2, 13 | P.LBM_LAUNCH_STAGED), (3, P.LBM_LAUNCH_DEFAULT), (3, 5 | P.LBM_LAUNCH_STAGED)]
    if prec == 1:  # four steps per launch (FP32), zigzag and upward walks
        modes += [(4, P.LBM_LAUNCH_DEFAULT), (4, 5 | P.LBM_LAUNCH_STAGED)]
    for fuse, flags in modes:
        with P.Context(device=0, max_slots=1) as ctx:
            ctx.set_fusion(prec, fuse, seg)
            ctx.set_launch(prec, 256, 1, 1, flags)
            s = ctx.add(case)
            ctx.state_load(s, f0, g0)
            ctx.step(s, steps)
            out.append((ctx.state_save(s), ctx.reduce(s)))
    a, sa = out[0]
    for b, sb in out[1:]:
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        for k in ("melt_fraction", "total_H", "heat_in_cum", "heater_q", "budget_residual"):
            assert sa[k] == sb[k], k


@pytest.mark.parametrize("chunk", [7, 10])
def test_fused_kernels_in_graphs_and_with_reports(P, chunk):
    case = dict(small_cavity("distinct"), pattern=P.LBM_PATTERN_AB)
    f0, g0 = _random_state(31, 128, 64)
    res = []
    for fuse in (1, 2, 3):
        with P.Context(device=0, max_slots=1) as ctx:
            ctx.set_fusion(0, fuse, 16)
            ctx.set_graph_chunk(chunk)
            s = ctx.add(case)
            ctx.state_load(s, f0, g0)
            ctx.set_report(s, 5, 64)
            ctx.step(s, 53)
            res.append((ctx.state_save(s), ctx.series(s)))
    (a, sa) = res[0]
    for b, sb in res[1:]:
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert [e["step"] for e in sa] == [e["step"] for e in sb] == list(range(5, 53, 5))
        assert all(x["total_H"] == y["total_H"] for x, y in zip(sa, sb))


def test_fused_kernels_full_size_match_oracle(P):
    """The benchmark's FP64 workload in its launch configuration (three steps
    per launch, 4-row segments) and with two steps per launch, 6 steps from a
    random state, against the oracle."""
    case = dict(large_cavity(), pattern=P.LBM_PATTERN_AB)
    print("case 2048x1024 FP64 fused kernels, 6 steps vs oracle", flush=True)
    f0, g0 = _random_state(23, 2048, 1024)
    got = []
    for fuse in (3, 2):
        with P.Context(device=0, max_slots=1) as ctx:  # default launch configuration
            if fuse == 3:
                assert ctx.get_fusion(0) == (3, 4)
                assert ctx.get_launch(0)[3] == P.LBM_LAUNCH_DEFAULT
            else:
                ctx.set_fusion(0, 2)
                assert ctx.get_fusion(0) == (2, 2)
            s = ctx.add(case)
            ctx.state_load(s, f0, g0)
            ctx.step(s, 6)
            got.append(ctx.fields(s))
    o = oracle_run(case, 6, f0, g0)
    for fields in got:
        err = max_field_err(fields, o.fields())
        assert max(err.values()) <= 1e-12, err


def test_default_fusion_follows_cavity_size(P):
    """The default fusion adapts to the cavity (FP64 below 2^18 cells: two
    steps per launch; FP32 from 2^21 cells: four; segment rows minimising
    resident passes x rows collided x max(rho, waves per SIMD) when some
    length fits the launch in one pass, else 4 rows for FP64 three steps
    and 6 for FP32); an explicit
    setting is used as given.  The expected rows follow from the resident
    wavefronts of these kernels on MI355X (FP64 two and three steps and FP32
    four steps: 8 per CU; FP32 three steps: 12).  The adapted launches equal
    single steps bit for bit."""
    print("case default fusion per cavity size", flush=True)
    cases = [((2048, 1024, 0), (3, 4)), ((1536, 768, 0), (3, 4)), ((1024, 512, 0), (3, 6)),
             ((768, 384, 0), (3, 3)), ((512, 256, 0), (2, 2)), ((128, 64, 0), (2, 1)),
             ((2048, 1024, 1), (4, 6)), ((1536, 768, 1), (3, 8)), ((1024, 512, 1), (3, 6)),
             ((768, 384, 1), (3, 3)), ((512, 256, 1), (3, 2)), ((128, 64, 1), (3, 1))]
    with P.Context(device=0, max_slots=len(cases) + 1) as ctx:
        for (nx, ny, prec), want in cases:
            s = ctx.add(dict(cavity(nx, ny), precision=prec, pattern=P.LBM_PATTERN_AB))
            assert ctx.slot_fusion(s) == want, (nx, ny, prec)
            ctx.release(s)
        s = ctx.add(dict(cavity(128, 64), pattern=P.LBM_PATTERN_AA))
        assert ctx.slot_fusion(s)[0] == 1
        ctx.release(s)
        ctx.set_fusion(0, 3, 6)
        s = ctx.add(dict(cavity(256, 128), pattern=P.LBM_PATTERN_AB))
        assert ctx.slot_fusion(s) == (3, 6) and ctx.get_fusion(0) == (3, 6)
        # four steps per launch are FP32 only
        with pytest.raises(P.LbmError) as ei:
            ctx.set_fusion(0, 4)
        assert ei.value.code == P.LBM_EINVAL
        ctx.set_fusion(1, 4, 5)
        assert ctx.get_fusion(1) == (4, 5)
    # adapted three-step launches of a small FP32 cavity (1-row segments)
    case = dict(cavity(128, 64, heater_center=0.4), precision=P.LBM_FP32_SHIFTED, pattern=P.LBM_PATTERN_AB)
    f0, g0 = _random_state(57, 128, 64)
    out = []
    for fuse in (None, 1):
        with P.Context(device=0, max_slots=1) as ctx:
            if fuse:
                ctx.set_fusion(1, fuse)
            s = ctx.add(case)
            ctx.state_load(s, f0, g0)
            ctx.step(s, 14)
            out.append(ctx.state_save(s))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("nx,ny,prec,want", [(768, 384, 0, (3, 3)), (1024, 512, 0, (3, 6)),
                                             (512, 256, 0, (2, 2)), (768, 384, 1, (3, 3)),
                                             (1536, 768, 1, (3, 8)), (2048, 1024, 1, (4, 6))],
                         ids=["fp64_768", "fp64_1024", "fp64_512", "fp32_768", "fp32_1536", "fp32_2048"])
def test_adapted_fusion_equals_single_steps(P, nx, ny, prec, want):
    """The launches the size rule chooses at real sizes (three steps in 3-,
    6- and 8-row segments, two steps, four steps) advance a random state
    exactly as single two-lattice steps do, with a remainder launch."""
    print(f"case adapted fusion {nx}x{ny} precision {prec}", flush=True)
    case = dict(cavity(nx, ny, Ra=1e6, heater_center=0.35), precision=prec, pattern=P.LBM_PATTERN_AB)
    f0, g0 = _random_state(90 + nx, nx, ny)
    out = []
    for fuse in (None, 1):
        with P.Context(device=0, max_slots=1) as ctx:
            if fuse:
                ctx.set_fusion(prec, fuse)
            s = ctx.add(case)
            if fuse is None:
                assert ctx.slot_fusion(s) == want
            ctx.state_load(s, f0, g0)
            ctx.step(s, 14)
            out.append((ctx.state_save(s), ctx.reduce(s)))
    (a, sa), (b, sb) = out
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for k in ("melt_fraction", "total_H", "heat_in_cum", "budget_residual"):
        assert sa[k] == sb[k], k
