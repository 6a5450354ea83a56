"""Sec. 3.1 at the paper's own parameters, on the GPU: one-phase conduction
melting with Ste = 0.01, alpha = 1/6, dx = 1/100 (a column of 100 cells, the
hot wall being the heated bottom of a 1-D column: x periodic, flow off),
snapshot at t = 25, for k1 in {0.1, 0.5, 1.0, 1.5}, with the B-TriRT relation
of Eq. (5) and with SRT (k0 = k1 = k2).  (k1 = 2 gives a zero lattice
diffusivity and is not run.)  Each GPU run is checked against the oracle, and
the paper's claims are checked on the GPU result: with Eq. (5) the solid stays
at Tm and the interface is one cell wide; with SRT and k1 != 1 the solid is
activated ahead of the front.  The front and the liquid temperature are
compared with the Neumann solution, Eqs. (6)-(7)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import erf

import oracle
from btrirt_workloads import cavity

pytestmark = pytest.mark.gpu

STE, ALPHA, DX, T_END, NY = 0.01, 1.0 / 6.0, 0.01, 25.0, 100
K1 = [0.1, 0.5, 1.0, 1.5]


def kappa_s():
    return brentq(lambda k: STE / (math.exp(k * k) * math.erf(k)) - k * math.sqrt(math.pi), 1e-9, 5.0)


def setup(k1, srt):
    alpha_lat = (1.0 / k1 - 0.5) / 3.0
    steps = int(round(T_END * ALPHA / (alpha_lat * DX * DX)))
    kw = dict(periodic_x=1, param_mode=1, nu=0.1, alpha=alpha_lat, gbeta=0.0, latent=1.0 / STE,
              Th=1.0, Tm=0.0, heater_center=0.5, heater_width=1.0)
    if srt:
        kw.update(k0_g=1.0 / (alpha_lat * 3.0 + 0.5), k2_g=1.0 / (alpha_lat * 3.0 + 0.5))
    return cavity(1, NY, **kw), steps


@pytest.fixture(scope="module")
def P():
    import paper_1909_13086_amd as P
    return P


@pytest.mark.parametrize("srt", [False, True], ids=["btrirt", "srt"])
@pytest.mark.parametrize("k1", K1)
def test_paper_stefan_case(P, k1, srt):
    case, steps = setup(k1, srt)
    print(f"case Stefan Ste=0.01 k1={k1} {'SRT' if srt else 'B-TriRT'}: {steps} steps", flush=True)
    with P.Context(device=0, max_slots=1) as ctx:
        ctx.set_graph_chunk(1000)
        s = ctx.add(case)
        ctx.step(s, steps)
        fld = ctx.fields(s)
    oracle.set_threads(1)
    o = oracle.Oracle(oracle.case_from_dict(case)).init_solid().step(steps)
    ofl = o.fields()
    H, fl, T = fld["H"][:, 0], fld["fl"][:, 0], fld["T"][:, 0]
    # FP64 bar: 1e-10 after 2000 steps on quantities of order one; round-off
    # gathers at most linearly with the step count in this dissipative scheme,
    # and H is of order L = 100 here
    scale = max(1.0, steps / 2000)
    dT = float(np.max(np.abs(T - ofl["T"][:, 0])))
    dfl = float(np.max(np.abs(fl - ofl["fl"][:, 0])))
    dH = float(np.max(np.abs(H - ofl["H"][:, 0])))
    print(f"  GPU vs oracle: max|dT| {dT:.2e}, max|dfl| {dfl:.2e}, max|dH| {dH:.2e} (bar x{scale:.0f})", flush=True)
    assert dT <= 1e-10 * scale and dfl <= 1e-10 * scale
    assert dH <= 1e-10 * scale * 100
    y = (np.arange(NY) + 0.5) * DX
    xi = 2 * kappa_s() * math.sqrt(ALPHA * T_END)
    front = fl.sum() * DX
    ahead = y > xi + 2 * DX
    liquid = y < xi - 2 * DX
    t_an = 1.0 - erf(y / (2 * math.sqrt(ALPHA * T_END))) / math.erf(kappa_s())
    interface = int(((fl > 1e-13) & (fl < 1 - 1e-13)).sum())
    dev_solid = float(np.max(np.abs(H[ahead])))
    t_err = float(np.max(np.abs(T[liquid] - t_an[liquid])))
    print(f"  front {front:.4f} (Neumann {xi:.4f}), interface cells {interface}, "
          f"max|H - Cp Tm| ahead {dev_solid:.2e}, Linf(T) liquid {t_err:.3e}", flush=True)
    if not srt or k1 == 1.0:
        # Eq. (5) holds (SRT with k1 = 1 is also k1 + k2 = 2): the solid stays at
        # Tm, the interface is one cell, and the Neumann solution is followed
        assert dev_solid <= 1e-12
        assert interface <= 1
        assert abs(front - xi) / xi <= 0.03
        assert t_err <= 0.02
    else:
        # SRT with k1 != 1: the solid ahead of the front is activated
        assert dev_solid > 1e-3
