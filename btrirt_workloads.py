"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only describes problems and draws random numbers; it holds none of
the method's arithmetic (no parameter derivation, equilibria or collisions), so
both the CPU oracle and the GPU library can be fed from it without sharing code.

Problem statements follow the cavity of Sec. 3.2 (PCM initially solid at Tm, a
bottom strip held at Th, no-slip adiabatic walls) and the one-phase conduction
melting problem of Sec. 3.1.  The paper ships no data set: every input here is
synthetic.
"""
import math

import numpy as np

NAN = math.nan

# Default field values of a cavity description (dimensionless parameters, Sec. 3.2).
CASE_DEFAULTS = dict(
    periodic_x=0, periodic_y=0, param_mode=0,
    Ra=1e4, Pr=1.0, Ste=1.0, Ma=0.1,
    nu=0.0, alpha=0.0, gbeta=0.0, latent=0.0,
    Cp=1.0, Th=1.0, Tm=0.0, rho0=1.0,
    heater_center=0.5, heater_width=0.25,
    k0_g=NAN, k2_g=NAN, k0_f=NAN, k1_f=NAN,
    solid_model=0, darcy_c=NAN, darcy_eps=NAN,
)


def cavity(nx, ny, **kw):
    """A cavity description: a plain dict of problem parameters."""
    d = dict(CASE_DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise KeyError(f"unknown case fields {sorted(unknown)}")
    d.update(kw)
    d["nx"], d["ny"] = int(nx), int(ny)
    return d


# --- the five workloads -------------------------------------------------------

def small_cavity(variant="literal"):
    """128x64 cavity, Ra 1e4, Pr 1, Ste 1, heater centred with width W/4.

    variant: "literal" keeps k0 = k2 = 1 for the enthalpy populations;
    "eq6" uses the default k2 = 2 - k1; "distinct" sets k0 = 0.8 with the
    default k2, so that every projection term is active.
    """
    if variant == "literal":
        return cavity(128, 64, Ra=1e4, k0_g=1.0, k2_g=1.0)
    if variant == "eq6":
        return cavity(128, 64, Ra=1e4)
    if variant == "distinct":
        return cavity(128, 64, Ra=1e4, k0_g=0.8)
    raise ValueError(variant)


def large_cavity(nx=2048, ny=1024):
    """Single large cavity: Ra 1e8, Pr 1, Ste 1, heater centred with width W/4."""
    return cavity(nx, ny, Ra=1e8)


def batch_sweep(seed=4, n=64):
    """Batch of cavities of uneven size: nx uniform over multiples of 64 in
    [256, 1024], ny = nx/2, heater centre uniform in [0.125, 0.875], width
    nx/4, Ra log-uniform in [1e6, 1e8]."""
    rng = np.random.default_rng(seed)
    out = []
    widths = np.arange(256, 1024 + 1, 64)
    for _ in range(n):
        nx = int(rng.choice(widths))
        c = float(rng.uniform(0.125, 0.875))
        ra = float(10.0 ** rng.uniform(6.0, 8.0))
        out.append(cavity(nx, nx // 2, Ra=ra, heater_center=c, heater_width=0.25))
    return out


SERVE_SIZES = ((256, 128), (512, 256), (1024, 512), (2048, 1024))


def serving_trace(seed=5, n=256, rate=20.0, steps_lo=1000, steps_hi=50000,
                  sizes=SERVE_SIZES, fp64_share=0.5):
    """Poisson arrivals of melting solves.  Each request: arrival time (s),
    cavity description, number of steps and precision (0 = FP64, 1 = FP32
    shifted)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for _ in range(n):
        t += float(rng.exponential(1.0 / rate))
        nx, ny = sizes[int(rng.integers(len(sizes)))]
        ra = float(10.0 ** rng.uniform(6.0, 8.0))
        c = float(rng.uniform(0.125, 0.875))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        prec = 0 if rng.uniform() < fp64_share else 1
        reqs.append(dict(arrival=t, case=cavity(nx, ny, Ra=ra, heater_center=c), steps=steps,
                         precision=prec))
    return reqs


def random_planes(seed, nplanes, ny, nx):
    """Uniform [0, 1) numbers of shape (nplanes, ny, nx), float64."""
    return np.random.default_rng(seed).random((nplanes, ny, nx))
