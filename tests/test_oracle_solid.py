"""Pins of the oracle's three readings of how the solid holds the flow still
(the paper names none): velocity scaled by the liquid fraction, an
enthalpy-porosity (Carman-Kozeny) drag, and partial bounce-back.

They check what each reading fixes exactly: the drag's velocity is the mean of
the momenta before and after the collision while the momentum changes by the
buoyancy plus the drag; partial bounce-back is the affine mix of a free-fluid
collision and a full bounce-back; every reading conserves mass, leaves a
liquid cell as a free fluid, keeps the enthalpy budget closed and keeps the
centred-heater cavity mirror symmetric.
"""
import math

import numpy as np
import pytest

import oracle
from btrirt_workloads import cavity, small_cavity
from tests import d2q9_ref as R

OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]


def _params(rng, model, C=None, eps=None, **over):
    c = cavity(4, 4, param_mode=oracle.PARAM_LATTICE, nu=rng.uniform(0.01, 0.3),
               alpha=rng.uniform(0.01, 0.3), gbeta=rng.uniform(1e-3, 1e-2), latent=rng.uniform(0.2, 2.0),
               Cp=rng.uniform(0.5, 2.0), Tm=rng.uniform(-0.5, 0.5), k0_g=rng.uniform(0.3, 1.7),
               k2_g=rng.uniform(0.3, 1.7), k0_f=rng.uniform(0.3, 1.7), k1_f=rng.uniform(0.3, 1.7),
               solid_model=model, darcy_c=math.nan if C is None else C, darcy_eps=math.nan if eps is None else eps)
    c.update(over)
    return oracle.derive(oracle.case_from_dict(c))


def _cell(rng, p, fl_target):
    """Random flow populations and enthalpy populations with a given liquid
    fraction (0: solid below the melting point; 0 < fl < 1: mushy; 1: liquid
    above the melting point)."""
    f = R.W * (1.0 + 0.2 * rng.uniform(-1, 1, 9))
    H = p.Cp * p.Tm + fl_target * p.latent
    if fl_target >= 1.0:
        H += 0.3 * p.Cp
    elif fl_target <= 0.0:
        H -= 0.1 * p.Cp
    g = R.W * H + 0.02 * rng.uniform(-1, 1, 9)
    g[0] += H - g.sum()
    return f, g


def test_derived_defaults_and_validation():
    p = oracle.derive(oracle.case_from_dict(cavity(8, 8, solid_model=oracle.SOLID_DARCY)))
    assert (p.solid_model, p.darcy_c, p.darcy_eps) == (oracle.SOLID_DARCY, 1e3, 1e-3)
    for bad in (dict(solid_model=3), dict(solid_model=-1), dict(solid_model=1, darcy_c=-1.0),
                dict(solid_model=1, darcy_eps=0.0)):
        with pytest.raises(ValueError):
            oracle.derive(oracle.case_from_dict(cavity(8, 8, **bad)))


@pytest.mark.parametrize("model", [oracle.SOLID_DARCY, oracle.SOLID_PBB])
def test_liquid_cell_is_a_free_fluid_under_every_reading(model):
    rng = np.random.default_rng(11)
    for _ in range(20):
        p = _params(rng, model)
        f, g = _cell(rng, p, 1.0)
        ref = _params(np.random.default_rng(0), oracle.SOLID_SCALE)
        for name in ("nu", "alpha", "gbeta", "latent", "Cp", "Tm", "Th", "rho0", "k0_g", "k1_g", "k2_g",
                     "k0_f", "k1_f", "k2_f"):
            setattr(ref, name, getattr(p, name))
        fo, go, m = oracle.collide_cell(p, f, g)
        fr, gr, mr = oracle.collide_cell(ref, f, g)
        assert m["fl"] == 1.0
        assert np.array_equal(fo, fr) and np.array_equal(go, gr)


@pytest.mark.parametrize("seed", range(6))
def test_darcy_velocity_is_the_mean_momentum_and_momentum_gains_the_total_force(seed):
    rng = np.random.default_rng(200 + seed)
    C = 10.0 ** rng.uniform(0, 4)
    p = _params(rng, oracle.SOLID_DARCY, C=C, eps=10.0 ** rng.uniform(-4, -1))
    for fl in (0.0, 0.2, 0.5, 0.9, 0.999):
        f, g = _cell(rng, p, fl)
        fo, go, m = oracle.collide_cell(p, f, g)
        assert m["fl"] == pytest.approx(fl, abs=1e-12)
        j0 = np.array(R.moments(f)[1:3])
        j1 = np.array(R.moments(fo)[1:3])
        u = np.array([m["ux"], m["uy"]])
        # the Guo-type forcing makes the velocity the mean of the momenta
        assert np.allclose(p.rho0 * u, 0.5 * (j0 + j1), rtol=0, atol=1e-14)
        # and the momentum change the total force: buoyancy plus drag
        A = p.darcy_c * (1 - m["fl"]) ** 2 / (m["fl"] ** 3 + p.darcy_eps)
        Fb = np.array([0.0, p.rho0 * p.gbeta * (m["T"] - p.Tm)])
        assert np.allclose(j1 - j0, Fb - A * p.rho0 * u, rtol=0, atol=1e-13)
        assert R.moments(fo)[0] == pytest.approx(R.moments(f)[0], abs=1e-14)


def test_darcy_drag_holds_the_solid_and_grows_with_the_constant():
    rng = np.random.default_rng(5)
    p0 = _params(rng, oracle.SOLID_DARCY, C=0.0)
    f, g = _cell(rng, p0, 0.4)
    speeds = []
    for C in (0.0, 1.0, 1e2, 1e4, 1e6):
        p = _params(np.random.default_rng(5), oracle.SOLID_DARCY, C=C)
        speeds.append(math.hypot(*[oracle.collide_cell(p, f, g)[2][k] for k in ("ux", "uy")]))
    assert all(a > b for a, b in zip(speeds, speeds[1:]))
    assert speeds[-1] < 1e-5 * speeds[0]


@pytest.mark.parametrize("seed", range(6))
def test_partial_bounce_back_mixes_free_fluid_and_full_bounce_back(seed):
    rng = np.random.default_rng(300 + seed)
    p = _params(rng, oracle.SOLID_PBB)
    free = _params(np.random.default_rng(300 + seed), oracle.SOLID_DARCY, C=0.0)  # no drag: a free fluid
    for fl in (0.0, 0.3, 0.75):
        f, g = _cell(rng, p, fl)
        fo, go, m = oracle.collide_cell(p, f, g)
        ff, gf, mf = oracle.collide_cell(free, f, g)
        ns = 1.0 - m["fl"]
        assert np.allclose(fo, (1 - ns) * ff + ns * f[OPP], rtol=0, atol=1e-15)
        assert np.array_equal(go, gf)  # the enthalpy sees the free-fluid velocity
        assert fo.sum() == pytest.approx(f.sum(), abs=1e-14)
        if fl == 0.0:
            assert np.array_equal(fo, f[OPP])  # full bounce-back in the solid


@pytest.mark.parametrize("model", [oracle.SOLID_SCALE, oracle.SOLID_DARCY, oracle.SOLID_PBB])
def test_cavity_budget_symmetry_and_still_solid_under_every_reading(model):
    c = dict(small_cavity("eq6"), solid_model=model, Ra=1e5)
    o = oracle.Oracle(oracle.case_from_dict(c)).init_solid()
    o.step(1200)
    s = o.stats()
    assert s["finite"] == 1
    assert abs(s["budget_residual"]) <= 1e-12 * max(1.0, abs(s["total_H"]))
    assert s["mass"] == pytest.approx(128 * 64, rel=1e-12)
    fld = o.fields()
    assert np.max(np.abs(fld["T"] - fld["T"][:, ::-1])) <= 1e-12
    assert np.max(np.abs(fld["ux"] + fld["ux"][:, ::-1])) <= 1e-12
    solid = fld["fl"] == 0.0
    assert solid.sum() > 0.5 * solid.size
    speed = np.hypot(fld["ux"], fld["uy"])
    assert s["melt_fraction"] > 0.0 and speed.max() > 1e-5
    # solid cells whose eight neighbours are solid too (cells touching the
    # melt receive the populations it streams in)
    padded = np.pad(solid, 1, constant_values=True)  # the walls hold nothing that moves
    deep = np.ones_like(solid)
    for dy in (0, 1, 2):
        for dx in (0, 1, 2):
            deep &= padded[dy:dy + solid.shape[0], dx:dx + solid.shape[1]]
    assert deep.sum() > 0.4 * solid.size
    # the drag leaves about 2/A = 2 eps/C of a cell's momentum as velocity;
    # under bounce-back a solid cell only swaps its own populations, so it
    # keeps what it held when the front passed nearby (a trapped oscillation)
    bound = {oracle.SOLID_SCALE: 0.0, oracle.SOLID_DARCY: 1e-5, oracle.SOLID_PBB: 1e-2}[model]
    assert np.max(speed[deep]) <= bound * speed.max()
