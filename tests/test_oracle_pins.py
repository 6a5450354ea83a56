"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's
update: they test moment identities, closed forms (the Neumann solution of
Eqs. (6)-(7), Gaussian diffusion, Poiseuille flow), special cases coded
independently (BGK with Guo forcing), exact invariants and discrete budgets.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import erf

import oracle
from btrirt_workloads import cavity, random_planes, small_cavity
from tests import d2q9_ref as R

CS2 = R.CS2


def lattice_case(nx, ny, **kw):
    base = dict(param_mode=oracle.PARAM_LATTICE, nu=0.1, alpha=0.1, gbeta=0.0, latent=1.0)
    base.update(kw)
    return cavity(nx, ny, **base)


# ---------------------------------------------------------------------------
# P1: moments of the enthalpy equilibrium, Eq. (3)
# ---------------------------------------------------------------------------
def test_geq_moments_match_energy_equation():
    rng = np.random.default_rng(1)
    for _ in range(50):
        H, T, ux, uy, Cp = rng.uniform(-1, 2), rng.uniform(-1, 2), *rng.uniform(-0.1, 0.1, 2), rng.uniform(0.5, 3)
        geq = oracle.geq(H, T, ux, uy, Cp)
        m0, m1x, m1y, m2xx, m2xy, m2yy = R.moments(geq)
        assert m0 == pytest.approx(H, abs=1e-14)
        assert m1x == pytest.approx(Cp * T * ux, abs=1e-15)
        assert m1y == pytest.approx(Cp * T * uy, abs=1e-15)
        assert m2xx == pytest.approx(Cp * T * CS2, abs=1e-14)
        assert m2yy == pytest.approx(Cp * T * CS2, abs=1e-14)
        assert m2xy == pytest.approx(0.0, abs=1e-15)
        # the rest population carries the latent part H - Cp*T
        assert geq[0] - R.W[0] * Cp * T == pytest.approx(H - Cp * T, abs=1e-14)


def test_feq_moments_incompressible():
    rng = np.random.default_rng(2)
    for _ in range(50):
        rho, ux, uy, rho0 = rng.uniform(0.9, 1.1), *rng.uniform(-0.1, 0.1, 2), rng.uniform(0.5, 2)
        feq = oracle.feq(rho, ux, uy, rho0)
        m0, m1x, m1y, m2xx, m2xy, m2yy = R.moments(feq)
        assert m0 == pytest.approx(rho, abs=1e-14)
        assert (m1x, m1y) == pytest.approx((rho0 * ux, rho0 * uy), abs=1e-15)
        assert m2xx == pytest.approx(rho * CS2 + rho0 * ux * ux, abs=1e-14)
        assert m2yy == pytest.approx(rho * CS2 + rho0 * uy * uy, abs=1e-14)
        assert m2xy == pytest.approx(rho0 * ux * uy, abs=1e-15)


# ---------------------------------------------------------------------------
# P2: Eq. (2) relaxes each Hermite moment at its own rate
# ---------------------------------------------------------------------------
def _random_params(rng, **over):
    c = lattice_case(4, 4, nu=rng.uniform(0.01, 0.3), alpha=rng.uniform(0.01, 0.3),
                     gbeta=rng.uniform(-1e-2, 1e-2), latent=rng.uniform(0.2, 2.0),
                     Cp=rng.uniform(0.5, 2.0), Tm=rng.uniform(-0.5, 0.5),
                     k0_g=rng.uniform(0.3, 1.7), k2_g=rng.uniform(0.3, 1.7),
                     k0_f=rng.uniform(0.3, 1.7), k1_f=rng.uniform(0.3, 1.7))
    c.update(over)
    return oracle.derive(oracle.case_from_dict(c))


@pytest.mark.parametrize("seed", range(8))
def test_collision_relaxes_each_moment_at_its_rate(seed):
    rng = np.random.default_rng(100 + seed)
    p = _random_params(rng)
    f = R.W * (1.0 + 0.2 * rng.uniform(-1, 1, 9))
    # enthalpy spread over solid, mushy and liquid cells
    g = R.W * p.Cp * p.Tm + R.W * rng.uniform(-0.5, 2.5) * p.latent + 0.05 * rng.uniform(-1, 1, 9)
    fo, go, m = oracle.collide_cell(p, f, g)
    H, T, fl, ux, uy = m["H"], m["T"], m["fl"], m["ux"], m["uy"]
    assert H == pytest.approx(g.sum(), abs=1e-14)
    # --- enthalpy: M0 kept, M1 relaxes with k1, M2 with k2, higher with k0
    geq = oracle.geq(H, T, ux, uy, p.Cp)
    mi, mo, me = R.moments(g), R.moments(go), R.moments(geq)
    assert mo[0] == pytest.approx(mi[0], abs=1e-13)
    for a in (1, 2):
        assert mo[a] == pytest.approx(mi[a] - p.k1_g * (mi[a] - me[a]), abs=1e-13)
    for a in (3, 4, 5):
        assert mo[a] == pytest.approx(mi[a] - p.k2_g * (mi[a] - me[a]), abs=1e-13)
    hi, ho, he = R.hermite_high(g), R.hermite_high(go), R.hermite_high(geq)
    for a in range(3):
        assert ho[a] == pytest.approx(hi[a] - p.k0_g * (hi[a] - he[a]), abs=1e-13)
    # --- flow: same structure plus a force that changes momentum by exactly F
    Fy = p.rho0 * p.gbeta * (T - p.Tm)
    assert uy == pytest.approx(fl * (R.moments(f)[2] + 0.5 * Fy) / p.rho0, abs=1e-15)
    feq = oracle.feq(m["rho"], ux, uy, p.rho0)
    mi, mo, me = R.moments(f), R.moments(fo), R.moments(feq)
    assert mo[0] == pytest.approx(mi[0], abs=1e-13)
    assert mo[1] == pytest.approx(mi[1] - p.k1_f * (mi[1] - me[1]), abs=1e-13)
    assert mo[2] == pytest.approx(mi[2] - p.k1_f * (mi[2] - me[2]) + (1 - p.k1_f / 2) * Fy, abs=1e-13)
    src = {3: 0.0, 4: (1 - p.k2_f / 2) * ux * Fy, 5: (1 - p.k2_f / 2) * 2 * uy * Fy}
    for a in (3, 4, 5):
        assert mo[a] == pytest.approx(mi[a] - p.k2_f * (mi[a] - me[a]) + src[a], abs=1e-13)
    hi, ho, he = R.hermite_high(f), R.hermite_high(fo), R.hermite_high(feq)
    for a in range(3):
        assert ho[a] == pytest.approx(hi[a] - p.k0_f * (hi[a] - he[a]), abs=1e-13)


def test_liquid_cell_momentum_gains_exactly_the_force():
    rng = np.random.default_rng(7)
    p = _random_params(rng, Tm=0.0)
    f = R.W * (1.0 + 0.1 * rng.uniform(-1, 1, 9))
    g = R.W * (p.latent + 0.7 * p.Cp) + 0.01 * rng.uniform(-1, 1, 9)  # liquid: H > Cp*Tm + L
    fo, go, m = oracle.collide_cell(p, f, g)
    assert m["fl"] == 1.0
    Fy = p.rho0 * p.gbeta * m["T"]
    assert R.moments(fo)[2] - R.moments(f)[2] == pytest.approx(Fy, abs=1e-15)
    assert R.moments(fo)[1] - R.moments(f)[1] == pytest.approx(0.0, abs=1e-15)


# ---------------------------------------------------------------------------
# P3: k0 = k1 = k2 reduces Eq. (2) to the textbook BGK model
# ---------------------------------------------------------------------------
def test_srt_limit_equals_independent_bgk():
    nx, ny = 24, 12
    nu, alpha = 0.05, 0.08
    kf = 1.0 / (nu / CS2 + 0.5)
    kg = 1.0 / (alpha / CS2 + 0.5)
    c = lattice_case(nx, ny, nu=nu, alpha=alpha, gbeta=2e-3, latent=0.5, Th=1.0, Tm=0.0,
                     heater_center=0.4, heater_width=0.5, k0_g=kg, k2_g=kg, k0_f=kf, k1_f=kf)
    o = oracle.Oracle(c)
    p = o.params
    ref = R.SRTLattice(nx, ny, omega_f=kf, omega_g=kg, Cp=1.0, Th=1.0, Tm=0.0, rho0=1.0, latent=0.5,
                       gbeta=2e-3, heater_cells=range(p.heater_lo, p.heater_hi + 1))
    # start from an uneven state so every term is exercised
    rnd = random_planes(11, 18, ny, nx)
    f0 = R.W[:, None, None] * (1.0 + 0.05 * (rnd[:9] - 0.5))
    g0 = R.W[:, None, None] * (1.2 * rnd[9:] + 0.2)
    o.set_populations(f0, g0)
    f, g = f0.copy(), g0.copy()
    for _ in range(40):
        o.step(1)
        f, g = ref.step(f, g)
    fo, go = o.populations()
    assert np.max(np.abs(fo - f)) < 1e-13
    assert np.max(np.abs(go - g)) < 1e-13


# ---------------------------------------------------------------------------
# P4: the enthalpy map of Sec. 2 (H = Cp*T + fl*L, isothermal melting at Tm)
# ---------------------------------------------------------------------------
def test_enthalpy_map_round_trip_and_continuity():
    Cp, Tm, L = 1.7, 0.3, 0.9
    Hs, Hl = Cp * Tm, Cp * Tm + L
    for H in np.linspace(Hs - 2, Hl + 2, 2001):
        T, fl = oracle.enthalpy_map(H, Cp, Tm, L)
        assert 0.0 <= fl <= 1.0
        assert Cp * T + fl * L == pytest.approx(H, abs=1e-13)
        if Hs < H < Hl:
            assert T == Tm
    eps = 1e-12
    for Hb in (Hs, Hl):
        a = oracle.enthalpy_map(Hb - eps, Cp, Tm, L)
        b = oracle.enthalpy_map(Hb + eps, Cp, Tm, L)
        assert abs(a[0] - b[0]) < 1e-11 and abs(a[1] - b[1]) < 1e-11
    Ts = [oracle.enthalpy_map(H, Cp, Tm, L)[0] for H in np.linspace(Hs - 1, Hl + 1, 101)]
    assert np.all(np.diff(Ts) >= 0)


# ---------------------------------------------------------------------------
# P5: parameter relations, Eqs. (4)-(5), and the reading of Sec. 3.2
# ---------------------------------------------------------------------------
def test_rate_relations_and_dimensionless_groups():
    for ra in (1e4, 1e6, 1e8):
        c = cavity(256, 128, Ra=ra, Pr=6.2, Ste=0.125)
        p = oracle.derive(oracle.case_from_dict(c))
        # Eq. (4) gives back alpha; Eq. (5) is the TRT product 1/4
        assert CS2 * (1 / p.k1_g - 0.5) == pytest.approx(p.alpha, rel=1e-14)
        assert p.k1_g + p.k2_g == pytest.approx(2.0, abs=1e-15)
        lam = (1 / p.k1_g - 0.5) * (1 / p.k2_g - 0.5)
        assert lam == pytest.approx(0.25, rel=1e-12)
        assert CS2 * (1 / p.k2_f - 0.5) == pytest.approx(p.nu, rel=1e-14)
        dT, ell = 1.0, 128
        assert p.gbeta * dT * ell**3 / (p.nu * p.alpha) == pytest.approx(ra, rel=1e-12)
        assert p.nu / p.alpha == pytest.approx(6.2, rel=1e-14)
        assert math.sqrt(p.gbeta * dT * ell) == pytest.approx(0.1 * math.sqrt(CS2), rel=1e-14)
        assert p.Cp * dT / p.latent == pytest.approx(0.125, rel=1e-14)


def test_heater_cells_of_the_small_cavity():
    p = oracle.derive(oracle.case_from_dict(small_cavity("eq6")))
    assert (p.heater_lo, p.heater_hi, p.n_heater) == (48, 79, 32)
    # a strip reaching past the walls is clipped; zero width means no strip
    p = oracle.derive(oracle.case_from_dict(cavity(10, 4, heater_center=0.0, heater_width=0.5)))
    assert (p.heater_lo, p.heater_hi) == (0, 2)
    p = oracle.derive(oracle.case_from_dict(cavity(10, 4, heater_width=0.0)))
    assert p.n_heater == 0


def test_invalid_cases_are_rejected():
    bad = [cavity(0, 4), cavity(4, 4, Ra=-1.0), cavity(4, 4, Th=0.0),
           lattice_case(4, 4, nu=0.0), lattice_case(4, 4, k0_g=2.0), lattice_case(4, 4, k2_g=0.0),
           lattice_case(4, 4, k1_f=2.5)]
    for c in bad:
        with pytest.raises(ValueError):
            oracle.derive(oracle.case_from_dict(c))


# ---------------------------------------------------------------------------
# P6: one-phase conduction melting, Sec. 3.1, Eqs. (6)-(7)
# ---------------------------------------------------------------------------
def stefan_constant(ste):
    """Root of Ste / (exp(k^2) erf(k)) = k sqrt(pi), Eq. (7)."""
    return brentq(lambda k: ste / (math.exp(k * k) * math.erf(k)) - k * math.sqrt(math.pi), 1e-9, 5.0)


def test_stefan_constants():
    # checks the root finder itself against values computed by bisection in
    # extended precision for Ste = 0.01, 0.125, 1
    assert stefan_constant(0.01) == pytest.approx(0.0705932766, abs=1e-9)
    assert stefan_constant(0.125) == pytest.approx(0.2450269931, abs=1e-9)
    assert stefan_constant(1.0) == pytest.approx(0.6200626333, abs=1e-9)


def stefan_oracle(ny, ste, k1, nx=1, k0=None, k2=None):
    """1-D melting column: the heated bottom wall plays the role of the hot wall
    of Sec. 3.1, x is periodic, flow is switched off (g*beta = 0)."""
    alpha = CS2 * (1.0 / k1 - 0.5)
    kw = dict(periodic_x=1, nu=0.1, alpha=alpha, gbeta=0.0, latent=1.0 / ste, Th=1.0, Tm=0.0,
              heater_center=0.5, heater_width=1.0)
    if k0 is not None:
        kw["k0_g"] = k0
    if k2 is not None:
        kw["k2_g"] = k2
    return oracle.Oracle(lattice_case(nx, ny, **kw)).init_solid(), alpha


def test_stefan_interface_temperature_and_nusselt():
    ste, ny = 1.0, 64
    o, alpha = stefan_oracle(ny, ste, k1=1.0)
    kappa = stefan_constant(ste)
    steps = 6000
    o.step(steps)
    fl = o.fields()["fl"][:, 0]
    T = o.fields()["T"][:, 0]
    Xi = 2 * kappa * math.sqrt(alpha * steps)
    assert fl.sum() == pytest.approx(Xi, rel=0.02)
    y = np.arange(ny) + 0.5
    liquid = y < Xi - 1.0
    Tan = 1.0 - erf(y / (2 * math.sqrt(alpha * steps))) / math.erf(kappa)
    assert np.max(np.abs(T[liquid] - Tan[liquid])) < 0.02
    assert np.all(T[y > Xi + 1.0] == 0.0)
    nu_an = ny / (math.sqrt(math.pi * alpha * steps) * math.erf(kappa))
    assert o.stats()["nusselt"] == pytest.approx(nu_an, rel=0.03)
    # the Fourier number the oracle reports places the front where Eq. (7)
    # puts it in units of the column height: X_i / ny = 2 kappa sqrt(Fo)
    fo = o.stats()["fourier"]
    assert fl.sum() / ny == pytest.approx(2 * kappa * math.sqrt(fo), rel=0.02)


def test_stefan_interface_converges_with_time():
    # relative error of the front position shrinks as the front crosses more cells
    ste, ny = 1.0, 96
    o, alpha = stefan_oracle(ny, ste, k1=1.0)
    kappa = stefan_constant(ste)
    errs = []
    t = 0
    for target in (1500, 6000, 13500):
        o.step(target - t)
        t = target
        Xi = 2 * kappa * math.sqrt(alpha * t)
        errs.append(abs(o.fields()["fl"].sum() - Xi) / Xi)
    assert errs[2] < errs[0]
    assert errs[2] < 0.01


# ---------------------------------------------------------------------------
# P7: Eq. (5) keeps the solid at Tm and the interface one cell wide
# ---------------------------------------------------------------------------
def _front_steps(k1, cells=10.0, ste=0.01):
    """Steps for the Neumann front of Eq. (7) to cross `cells` lattice cells."""
    alpha = CS2 * (1.0 / k1 - 0.5)
    return int((cells / (2 * stefan_constant(ste))) ** 2 / alpha)


def _interface_cells(fl):
    return int(((fl > 1e-13) & (fl < 1 - 1e-13)).sum())


@pytest.mark.parametrize("k1", [0.5, 1.5])
def test_eq5_keeps_solid_at_melting_temperature(k1):
    ste, ny = 0.01, 100
    steps = _front_steps(k1)
    o, _ = stefan_oracle(ny, ste, k1=k1)
    o.step(steps)
    fld = o.fields()
    H, fl = fld["H"][:, 0], fld["fl"][:, 0]
    assert fl.sum() > 8
    solid = fl < 1e-13
    assert solid.sum() > 50
    assert np.max(np.abs(H[solid])) <= 1e-12  # Cp*Tm = 0
    assert _interface_cells(fl) <= 1
    # in this 1-D column the k0 term only touches moments the column does not
    # carry: another k0 gives the same enthalpy field up to round-off gathered
    # over ~1e5 steps (relative to the latent heat L = 100 that sets the scale
    # of H); a leak of the k0 term into the carried moments would show at O(1)
    for k0 in (0.3, 1.7):
        o2, _ = stefan_oracle(ny, ste, k1=k1, k0=k0)
        o2.step(steps)
        assert np.max(np.abs(o2.fields()["H"][:, 0] - H)) < 1e-10 * np.max(np.abs(H))


@pytest.mark.parametrize("k1", [0.5, 1.5])
def test_srt_with_k1_not_one_diffuses_into_the_solid(k1):
    ste, ny = 0.01, 100
    o, _ = stefan_oracle(ny, ste, k1=k1, k0=k1, k2=k1)
    o.step(_front_steps(k1))
    fld = o.fields()
    H, fl = fld["H"][:, 0], fld["fl"][:, 0]
    # the solid ahead of the front is activated: H moves off Cp*Tm.  For
    # k1 < 1 it is warmed, so the partly liquid zone spreads over several
    # cells; for k1 > 1 it is cooled below Tm instead, and the deviation shows
    # in the temperature of the solid rather than in the width of the front.
    ahead = np.arange(ny) > np.argmax(fl < 0.5) + 1
    assert np.max(np.abs(H[ahead])) > 1e-3
    if k1 < 1.0:
        assert _interface_cells(fl) >= 2
        assert np.all(H[ahead][:3] > 0)
    else:
        assert np.all(H[ahead][:3] < 0)


def test_srt_with_k1_one_satisfies_eq5_case():
    # k1 = 1 with SRT is also k1 + k2 = 2: the solid stays at Tm
    o, _ = stefan_oracle(100, 0.01, k1=1.0, k0=1.0, k2=1.0)
    o.step(2000)
    fld = o.fields()
    solid = fld["fl"][:, 0] < 1e-9
    assert np.max(np.abs(fld["H"][solid, 0])) <= 1e-12


# ---------------------------------------------------------------------------
# P8: diffusion of a Gaussian (flow off, all liquid)
# ---------------------------------------------------------------------------
def _variance_along(field, axis):
    prof = field.sum(axis=1 - axis)
    x = np.arange(prof.size) + 0.5
    m = prof.sum()
    mu = (x * prof).sum() / m
    return ((x - mu) ** 2 * prof).sum() / m


def test_gaussian_variance_grows_at_twice_alpha_1d():
    ny, k1, T0 = 512, 1.3, 0.5
    alpha = CS2 * (1 / k1 - 0.5)
    c = lattice_case(1, ny, periodic_x=1, periodic_y=1, alpha=alpha, nu=0.1, gbeta=0.0, latent=1.0)
    o = oracle.Oracle(c).init_gaussian(T0, 0.1, 8.0)
    o.step(200)
    v1 = _variance_along(o.fields()["T"] - T0, 0)
    o.step(1000)
    v2 = _variance_along(o.fields()["T"] - T0, 0)
    assert (v2 - v1) / 1000 == pytest.approx(2 * alpha, rel=1e-4)


def test_gaussian_peak_and_isotropy_2d():
    n, T0, amp, s0 = 128, 0.5, 0.1, 6.0
    alpha = 0.12
    c = lattice_case(n, n, periodic_x=1, periodic_y=1, alpha=alpha, nu=0.1, gbeta=0.0, latent=1.0)
    o = oracle.Oracle(c).init_gaussian(T0, amp, s0)
    o.step(100)
    d1 = o.fields()["T"] - T0
    o.step(300)
    d2 = o.fields()["T"] - T0
    for ax in (0, 1):
        slope = (_variance_along(d2, ax) - _variance_along(d1, ax)) / 300
        assert slope == pytest.approx(2 * alpha, rel=1e-3)
    # peak of a 2-D Gaussian decays as s0^2 / (s0^2 + 2 alpha t)
    t = 400
    peak_an = amp * s0**2 / (s0**2 + 2 * alpha * t)
    # cell centres straddle the peak: compare with the analytic value there
    r2 = 0.0  # the centre lies on a lattice vertex; the 4 nearest cells sit at r^2 = 0.5
    r2 = 0.5
    s2 = s0**2 + 2 * alpha * t
    assert d2.max() == pytest.approx(peak_an * math.exp(-r2 / (2 * s2)), rel=1e-3)
    # conserved total
    assert abs(d2.sum() - d1.sum()) <= 1e-13 * n * n * T0


# ---------------------------------------------------------------------------
# P9 / P10: conservation and the discrete heater budget
# ---------------------------------------------------------------------------
def test_periodic_box_conserves_enthalpy_and_mass():
    n = 32
    c = lattice_case(n, n, periodic_x=1, periodic_y=1, nu=0.05, alpha=0.07, gbeta=1e-6, latent=0.3,
                     k0_g=0.9, k2_g=1.3, k0_f=1.1, k1_f=0.8)
    o = oracle.Oracle(c)
    rnd = random_planes(3, 18, n, n)
    f = R.W[:, None, None] * (1 + 0.02 * (rnd[:9] - 0.5))
    g = R.W[:, None, None] * (0.5 + rnd[9:])
    o.set_populations(f, g)
    s0 = o.stats()
    o.step(2000)
    s1 = o.stats()
    assert s1["finite"] == 1
    assert abs(s1["total_H"] - s0["total_H"]) <= 1e-13 * abs(s0["total_H"])
    assert abs(s1["mass"] - s0["mass"]) <= 1e-12 * s0["mass"]
    assert s1["heat_in_cum"] == 0.0


def test_walled_cavity_budget_closes():
    o = oracle.Oracle(oracle.case_from_dict(small_cavity("distinct"))).init_solid()
    for _ in range(4):
        o.step(500)
        s = o.stats()
        assert s["finite"] == 1
        assert abs(s["budget_residual"]) <= 1e-12 * max(1.0, abs(s["total_H"]))
        assert s["heat_in_cum"] > 0
        assert s["mass"] == pytest.approx(64 * 128, rel=1e-12)


# ---------------------------------------------------------------------------
# P11: Poiseuille flow between no-slip walls
# ---------------------------------------------------------------------------
def _poiseuille(nx, k0_f, steps=None):
    nu, gb, T0 = 0.1, 1e-5, 1.0
    c = lattice_case(nx, 1, periodic_y=1, nu=nu, alpha=0.1, gbeta=gb, latent=0.5, k0_f=k0_f,
                     heater_width=0.0)
    o = oracle.Oracle(c).init_liquid(T0)
    o.step(steps or int(12 * nx * nx / nu))
    uy = o.fields()["uy"][0]
    x = np.arange(nx) + 0.5
    F = gb * T0
    return uy, F * x * (nx - x) / (2 * nu)


def test_poiseuille_magic_rate_is_exact():
    # with (1/k2 - 1/2)(1/k0 - 1/2) = 3/16 the half-way wall sits exactly midway
    nu = 0.1
    k0 = 1.0 / (0.5 + 3.0 / 16.0 / (3 * nu))
    uy, an = _poiseuille(16, k0)
    assert np.max(np.abs(uy - an)) / an.max() < 1e-10


def test_poiseuille_second_order_convergence():
    errs = []
    for nx in (8, 16, 32):
        uy, an = _poiseuille(nx, 1.0)
        errs.append(np.max(np.abs(uy - an)) / an.max())
    order = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert min(order) > 1.9
    assert errs[2] < 2e-3


# ---------------------------------------------------------------------------
# P12: symmetry and quiescence
# ---------------------------------------------------------------------------
def test_centred_heater_is_mirror_symmetric():
    o = oracle.Oracle(oracle.case_from_dict(small_cavity("eq6"))).init_solid()
    o.step(2000)
    T = o.fields()["T"]
    assert np.max(np.abs(T - T[:, ::-1])) <= 1e-12
    ux = o.fields()["ux"]
    assert np.max(np.abs(ux + ux[:, ::-1])) <= 1e-12


def test_no_heating_leaves_state_unchanged():
    c = cavity(40, 20, Th=0.0, Tm=0.0, param_mode=oracle.PARAM_LATTICE, nu=0.05, alpha=0.05,
               gbeta=1e-3, latent=1.0)
    o = oracle.Oracle(c).init_solid()
    f0, g0 = o.populations()
    o.step(300)
    f1, g1 = o.populations()
    assert np.array_equal(g0, g1)
    assert np.max(np.abs(f1 - f0)) < 1e-15
    assert np.all(o.fields()["ux"] == 0.0) and np.all(o.fields()["uy"] == 0.0)


def test_solid_cells_never_move():
    o = oracle.Oracle(oracle.case_from_dict(small_cavity("eq6"))).init_solid()
    for _ in range(4):
        o.step(250)
        fld = o.fields()
        solid = fld["fl"] == 0.0
        assert solid.sum() > 0
        assert np.all(fld["ux"][solid] == 0.0) and np.all(fld["uy"][solid] == 0.0)


# ---------------------------------------------------------------------------
# max |u| of the reported diagnostics: a closed form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("u", [(0.03, -0.04), (-0.05, 0.0), (0.0, 0.05), (0.028, 0.096)])
def test_max_velocity_of_a_moving_cell(u):
    """One liquid cell at T = Tm (so no buoyancy) holds the second-order
    equilibrium of velocity u, every other cell is at rest: the first moment
    of that equilibrium is rho0 u exactly, so the reported max |u| is the
    Euclidean norm of u (0.05 or 0.1 here), whichever component carries it."""
    nx, ny, rho0, Tm, latent = 6, 5, 1.0, 0.1, 1.0
    case = lattice_case(nx, ny, periodic_x=1, periodic_y=1, Tm=Tm, Th=1.0, latent=latent, rho0=rho0)
    o = oracle.Oracle(case)
    cx, cy, w = oracle.CX, oracle.CY, oracle.W
    H = Tm + latent  # fully liquid at Tm: fl = 1, T = Tm
    f = np.broadcast_to((w * rho0)[:, None, None], (9, ny, nx)).copy()
    g = np.broadcast_to((w * H)[:, None, None], (9, ny, nx)).copy()
    g[0] = H - Tm + w[0] * Tm  # the latent part sits in the rest population, Eq. (3)
    g[1:] = (w[1:] * Tm)[:, None, None]
    cu = cx * u[0] + cy * u[1]
    uu = u[0] ** 2 + u[1] ** 2
    f[:, 2, 3] = w * (rho0 + rho0 * (3 * cu + 4.5 * cu ** 2 - 1.5 * uu))
    g[:, 2, 3] = w * Tm * (1 + 3 * cu)
    g[0, 2, 3] = H - Tm + w[0] * Tm
    o.set_populations(f, g)
    st = o.stats()
    assert st["max_u"] == pytest.approx(math.hypot(*u), rel=1e-12)
    fld = o.fields()
    assert fld["ux"][2, 3] == pytest.approx(u[0], abs=1e-15)
    assert fld["uy"][2, 3] == pytest.approx(u[1], abs=1e-15)
