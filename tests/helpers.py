"""Small shared helpers for the tests (no method arithmetic)."""
import math

import numpy as np

import workloads as W

KB = 1.380649e-23


def collisionless_gas():
    """Argon with a vanishing cross-section (no NTC candidates) and an enormous viscosity
    (tau >> dt, so no Shakhov relaxation): particles only stream."""
    g = W.gas()
    g["d_ref"] = 1e-30
    g["mu_ref"] = 1e30
    return g


def box_case(dim=2, n=(10, 10, 1), h=1.0, bc="outflow", **kw):
    bcs = kw.pop("bcs", None) or (bc,) * 6
    base = W._case(dim=dim, nx=n[0], ny=n[1], nz=n[2], h=(h, h if dim >= 2 else 1.0, h if dim >= 3 else 1.0),
                   bc=tuple(bcs), F_N=1.0, dt_G=1.0, T_sigma=300.0, capacity=100000)
    base.update(kw)
    return base


def rayleigh_cdf(x, RT):
    return 1.0 - np.exp(-x * x / (2.0 * RT))


def normal_speed_cdf(z, s):
    """CDF of the density proportional to z exp(-(z - s)^2) on z > 0."""
    from scipy.special import erf
    num = 0.5 * (math.exp(-s * s) - np.exp(-(z - s) ** 2)) + s * 0.5 * math.sqrt(math.pi) * (erf(z - s) + erf(s))
    den = 0.5 * math.exp(-s * s) + s * 0.5 * math.sqrt(math.pi) * (1.0 + erf(s))
    return num / den
