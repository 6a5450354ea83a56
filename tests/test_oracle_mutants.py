"""Strength of the oracle pins: plausible mistakes are planted in a copy of the
oracle's C source (on the CPU, in a temporary directory), the copy is built and
loaded in place of the oracle, and the pin checks must reject every one of
them.  The oracle itself is never modified."""
import os
import subprocess

import pytest

import oracle
from oracle import build as obuild
from tests import test_oracle_pins as pins
from tests import test_oracle_solid as solid

# (name, text in btrirt_oracle.c, replacement)
MUTANTS = [
    ("second-order force term dropped",
     "(1.0 - 0.5 * p->k2_f) * qcontract(i, sxx, sxy, syy)", "0.0 * qcontract(i, sxx, sxy, syy)"),
    ("anti-bounce-back sign",
     "gi[k] = -st->gs[(size_t)o * n + k] + 2.0 * W[i] * p->Cp * p->Th;",
     "gi[k] = st->gs[(size_t)o * n + k] + 2.0 * W[i] * p->Cp * p->Th;"),
    ("opposite directions of 5 and 6 swapped",
     "static const int OPP[OR_Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};",
     "static const int OPP[OR_Q] = {0, 3, 4, 1, 2, 8, 7, 6, 5};"),
    ("latent part missing from the rest equilibrium",
     "geq[i] = H - Cp * T + W[0] * Cp * T;", "geq[i] = W[0] * Cp * T;"),
    ("Eq. (4) without the one half",
     "p->k1_g = 1.0 / (p->alpha / CS2 + 0.5);", "p->k1_g = 1.0 / (p->alpha / CS2 + 1.0);"),
    ("Eq. (5) default replaced by k2 = 1",
     "p->k2_g = isnan(cs->k2_g) ? 2.0 - p->k1_g : cs->k2_g;", "p->k2_g = isnan(cs->k2_g) ? 1.0 : cs->k2_g;"),
    ("full force in the velocity",
     "uy = fl * (jy + 0.5 * Fy) / p->rho0;", "uy = fl * (jy + Fy) / p->rho0;"),
    ("transposed second moment",
     "m2xy += CX[j] * CY[j] * neq[j];", "m2xy += CX[j] * CX[j] * neq[j];"),
    ("heater strip one cell short",
     "double lo = ceil(xa - 0.5), hi = floor(xb - 0.5);", "double lo = ceil(xa + 0.5), hi = floor(xb - 0.5);"),
    ("mushy temperature off Tm",
     "    *fl = (H - Hs) / latent;\n    *T = Tm;", "    *fl = (H - Hs) / latent;\n    *T = H / Cp;"),
    ("first moment relaxed with k2",
     "- (k1 - k0) * W[i] * cm1 / CS2", "- (k2 - k0) * W[i] * cm1 / CS2"),
    ("second-order equilibrium term scaled wrongly",
     "cu * cu / (2.0 * CS2 * CS2)", "cu * cu / (2.0 * CS2)"),
    ("streaming pulls from downstream",
     "int sx = x - CX[i], sy = y - CY[i];", "int sx = x + CX[i], sy = y + CY[i];"),
    ("strip flux counted once per link",
     "nsum_add(&s, &c, 2.0 * (g[(size_t)i * n + (size_t)x] - W[i] * p->Cp * p->Th));",
     "nsum_add(&s, &c, 1.0 * (g[(size_t)i * n + (size_t)x] - W[i] * p->Cp * p->Th));"),
    ("buoyancy referred to Th",
     "double Fy = p->rho0 * p->gbeta * (T - p->Tm);", "double Fy = p->rho0 * p->gbeta * (T - p->Th);"),
    ("k0 term missing",
     "out[i] = p[i] - k0 * neq[i] - (k1 - k0)", "out[i] = p[i] - 0.0 * neq[i] - (k1 - k0)"),
    ("Darcy drag taken explicitly, not at the half step",
     "uy = (jy + 0.5 * Fy) / (p->rho0 * (1.0 + 0.5 * A));", "uy = (jy + 0.5 * Fy) / p->rho0;"),
    ("Carman-Kozeny factor without the square",
     "p->darcy_c * (1.0 - fl) * (1.0 - fl)", "p->darcy_c * (1.0 - fl)"),
    ("partial bounce-back with the liquid fraction as solid fraction",
     "ns = 1.0 - fl;", "ns = fl;"),
    ("partial bounce-back of the post-collision populations",
     "ns * f[OPP[i]]", "ns * fout[OPP[i]]"),
    ("max |u| from the vertical component only",
     "double u = sqrt(m[3] * m[3] + m[4] * m[4]);", "double u = fabs(m[4]);"),
    ("max |u| as the sum of the component magnitudes",
     "double u = sqrt(m[3] * m[3] + m[4] * m[4]);", "double u = fabs(m[3]) + fabs(m[4]);"),
    ("Fourier number over the cavity area",
     "out->fourier = p->alpha * (double)st->step / ((double)p->ny * (double)p->ny);",
     "out->fourier = p->alpha * (double)st->step / ((double)p->nx * (double)p->ny);"),
    ("Fourier number without the square of the height",
     "out->fourier = p->alpha * (double)st->step / ((double)p->ny * (double)p->ny);",
     "out->fourier = p->alpha * (double)st->step / (double)p->ny;"),
]

PIN_CHECKS = [
    pins.test_geq_moments_match_energy_equation,
    pins.test_feq_moments_incompressible,
    lambda: pins.test_collision_relaxes_each_moment_at_its_rate(0),
    lambda: pins.test_collision_relaxes_each_moment_at_its_rate(1),
    pins.test_liquid_cell_momentum_gains_exactly_the_force,
    pins.test_enthalpy_map_round_trip_and_continuity,
    pins.test_rate_relations_and_dimensionless_groups,
    pins.test_heater_cells_of_the_small_cavity,
    pins.test_srt_limit_equals_independent_bgk,
    pins.test_poiseuille_magic_rate_is_exact,
    pins.test_periodic_box_conserves_enthalpy_and_mass,
    pins.test_stefan_interface_temperature_and_nusselt,
    lambda: pins.test_eq5_keeps_solid_at_melting_temperature(0.5),
    pins.test_gaussian_variance_grows_at_twice_alpha_1d,
    pins.test_walled_cavity_budget_closes,
    pins.test_centred_heater_is_mirror_symmetric,
    lambda: pins.test_max_velocity_of_a_moving_cell((0.03, -0.04)),
    lambda: solid.test_darcy_velocity_is_the_mean_momentum_and_momentum_gains_the_total_force(0),
    lambda: solid.test_partial_bounce_back_mixes_free_fluid_and_full_bounce_back(0),
    lambda: solid.test_liquid_cell_is_a_free_fluid_under_every_reading(oracle.SOLID_DARCY),
    solid.test_darcy_drag_holds_the_solid_and_grows_with_the_constant,
    lambda: solid.test_cavity_budget_symmetry_and_still_solid_under_every_reading(oracle.SOLID_DARCY),
    lambda: solid.test_cavity_budget_symmetry_and_still_solid_under_every_reading(oracle.SOLID_PBB),
]


def _build_mutant(tmp_path, old, new):
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    d = tmp_path / "mut"
    d.mkdir()
    (d / "btrirt_oracle.c").write_text(src.replace(old, new))
    (d / "btrirt_oracle.h").write_text(open(os.path.join(os.path.dirname(obuild.SRC), "btrirt_oracle.h")).read())
    so = d / "libmut.so"
    subprocess.run(["gcc", *obuild.CFLAGS, str(d / "btrirt_oracle.c"), "-o", str(so), "-lm"], check=True)
    return str(so)


def test_unmutated_oracle_passes_the_pin_checks():
    for check in PIN_CHECKS:
        check()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    so = _build_mutant(tmp_path, old, new)
    saved = oracle.lib()
    oracle._LIB = oracle.load_library(so)
    try:
        caught = None
        for k, check in enumerate(PIN_CHECKS):
            try:
                check()
            except (AssertionError, ValueError, FloatingPointError) as e:
                caught = (k, type(e).__name__)
                break
        assert caught is not None, f"mutant '{name}' passed every pin check"
    finally:
        oracle._LIB = saved
