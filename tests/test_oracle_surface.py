"""Pins of the oracle's body surface sampling (the wall side of Step (5); Eq. 35-36).

In a free-molecular stream (mean free path ~100x the box) a convex diffuse body sees the
undisturbed drifting Maxwellian, so its wall fluxes follow from kinetic theory alone.  The
expected pressure, shear stress and heat flux of each element come from direct quadrature
of the one-sided flux integrals of the freestream Maxwellian plus the diffuse re-emission at
T_w; the drag coefficients are checked against the textbook closed forms for a cylinder and
a sphere (Bird, Molecular Gas Dynamics and the Direct Simulation of Gas Flows, 1994, Ch. 7),
which the quadrature reproduces to 1e-9.  Statistical errors come from batch means.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import workloads as W
from oracle.oracle import Oracle

K = W.K_BOLTZMANN
M = W.ARGON["m"]


def wall_fluxes(n, U, T, Tw, th):
    """Free-molecular p, tau, q on a diffuse wall element whose outward normal makes the
    polar angle th with the upstream direction -x, in a stream of speed U along +x."""
    sig = math.sqrt(K * T / M)
    un, ut = -U * math.cos(th), U * math.sin(th)
    phi = lambda c: math.exp(-0.5 * ((c - un) / sig) ** 2) / (sig * math.sqrt(2.0 * math.pi))
    lo = un - 12.0 * sig
    quad = lambda f: integrate.quad(f, lo, 0.0, epsabs=0.0, epsrel=1e-11)[0]
    flux = n * quad(lambda c: -c * phi(c))                      # molecules / (m^2 s)
    p_in = n * M * quad(lambda c: c * c * phi(c))
    e_in = n * quad(lambda c: -c * 0.5 * M * (c * c + ut * ut + 2.0 * sig * sig) * phi(c))
    p = p_in + flux * M * math.sqrt(math.pi * K * Tw / (2.0 * M))
    return p, M * flux * ut, e_in - 2.0 * K * Tw * flux


def element_means(n, U, T, Tw, nsurf, sphere):
    """Area averages of (p, tau, q) over the elements [k, k+1) pi / nsurf."""
    out = np.zeros((nsurf, 3))
    for k in range(nsurf):
        a, b = math.pi * k / nsurf, math.pi * (k + 1) / nsurf
        wgt = (lambda th: math.sin(th)) if sphere else (lambda th: 1.0)
        norm = integrate.quad(wgt, a, b)[0]
        for j in range(3):
            out[k, j] = integrate.quad(lambda th: wall_fluxes(n, U, T, Tw, th)[j] * wgt(th), a, b,
                                       epsrel=1e-9)[0] / norm
    return out


def cd_closed(s, T, Tw, sphere):
    if sphere:
        return ((2 * s * s + 1) / (math.sqrt(math.pi) * s ** 3) * math.exp(-s * s)
                + (4 * s ** 4 + 4 * s * s - 1) / (2 * s ** 4) * math.erf(s)
                + 2 * math.sqrt(math.pi) / (3 * s) * math.sqrt(Tw / T))
    z = s * s / 2
    return (math.sqrt(math.pi) * math.exp(-z) / s * ((s * s + 1.5) * special.i0(z) + (s * s + 0.5) * special.i1(z))
            + math.pi ** 1.5 / (4 * s) * math.sqrt(Tw / T))


def test_quadrature_reproduces_closed_form_drag():
    n, T, Tw = 1e13, 300.0, 500.0
    for s in (0.5, 1.0, 2.0):
        U = s * math.sqrt(2 * K * T / M)
        qd = 0.5 * n * M * U * U
        for sphere in (False, True):
            w = (lambda th: math.sin(th)) if sphere else (lambda th: 1.0)
            fx = integrate.quad(lambda th: (wall_fluxes(n, U, T, Tw, th)[0] * math.cos(th)
                                            + wall_fluxes(n, U, T, Tw, th)[1] * math.sin(th)) * w(th),
                                0.0, math.pi, epsrel=1e-10)[0]
            cd = (2 * math.pi * fx / math.pi) / qd if sphere else (2 * fx / 2) / qd
            assert abs(cd - cd_closed(s, T, Tw, sphere)) < 1e-8 * cd


def _batched(case, batches, steps):
    """Per-batch p, tau, q per element and C_D, from the raw wall sums."""
    o = Oracle(W.gas(), case)
    o.init_particles()
    ns, R = case["n_surf"], case["body_r"]
    sphere = case["body"] == "sphere"
    th = np.pi * np.arange(ns + 1) / ns
    area = 2 * np.pi * R * R * (np.cos(th[:-1]) - np.cos(th[1:])) if sphere else 2 * R * (th[1:] - th[:-1]) * 1.0
    U = case["inflow"]["u"][0]
    n = case["inflow"]["n"]
    qd = 0.5 * n * M * U * U
    aref = math.pi * R * R if sphere else 2 * R
    prev = np.zeros((ns, 7))
    rows, cds = [], []
    for b in range(batches):
        o.step(steps)
        S = o.surface_sums(0)
        d = S - prev
        prev = S
        t = steps * case["dt_G"]
        rows.append(np.stack([-d[:, 1] / (area * t), d[:, 2] / (area * t), d[:, 3] / (area * t)], axis=1))
        cds.append(d[:, 4].sum() / t / (qd * aref) if qd > 0 else 0.0)
    return o, np.array(rows), np.array(cds)


@pytest.mark.parametrize("body,s", [("cylinder", 1.0), ("sphere", 1.0)])
def test_free_molecular_wall_fluxes(body, s):
    T, Tw = 300.0, 500.0
    if body == "cylinder":
        case = W.free_molecular_body("cylinder", s=s, T=T, T_w=Tw, cells=40, ppc=20, R=0.3, n_surf=6)
        batches, steps = 8, 250
    else:
        case = W.free_molecular_body("sphere", s=s, T=T, T_w=Tw, cells=20, ppc=8, R=0.35, n_surf=4)
        batches, steps = 8, 50
    o, rows, cds = _batched(case, batches, steps)
    n, U = case["inflow"]["n"], case["inflow"]["u"][0]
    ref = element_means(n, U, T, Tw, case["n_surf"], body == "sphere")
    mean = rows.mean(axis=0)
    se = rows.std(axis=0, ddof=1) / math.sqrt(batches)
    z = np.abs(mean - ref) / se
    assert np.all(z < 5.0), (body, z, mean, ref)
    # the pressure of the upstream half is resolved to a few per cent (the test has power)
    front = np.arange(case["n_surf"]) < case["n_surf"] // 2
    assert np.all(se[front, 0] < 0.05 * np.abs(ref[front, 0]))
    cd_ref = cd_closed(s, T, Tw, body == "sphere")
    zc = abs(cds.mean() - cd_ref) / (cds.std(ddof=1) / math.sqrt(batches))
    assert zc < 5.0, (body, cds.mean(), cd_ref)
    # the oracle's own time averages equal the batch average (same sums, same normalisation)
    r = o.surface_sample(0)
    assert r["n_samples"] == batches * steps
    np.testing.assert_allclose(r["p"], mean[:, 0], rtol=1e-10)
    np.testing.assert_allclose(r["q"], mean[:, 2], rtol=1e-9, atol=1e-12 * np.abs(mean[:, 2]).max())
    assert abs(r["CD"] - cds.mean()) < 1e-9 * abs(cd_ref)
    assert abs(r["CL"]) < 0.05 * cd_ref            # no lift on a symmetric body


def test_wall_in_a_gas_at_rest_at_its_own_temperature():
    """Equilibrium: p = n k T on every element, no shear, no heat flux, no net force."""
    T = 300.0
    case = W.free_molecular_body("cylinder", s=0.0, T=T, T_w=T, cells=40, ppc=20, R=0.3, n_surf=4)
    o, rows, cds = _batched(case, 6, 200)
    n = case["inflow"]["n"]
    mean, se = rows.mean(axis=0), rows.std(axis=0, ddof=1) / math.sqrt(6)
    assert np.all(np.abs(mean[:, 0] - n * K * T) < 5 * se[:, 0])
    assert np.all(np.abs(mean[:, 1]) < 5 * se[:, 1])
    assert np.all(np.abs(mean[:, 2]) < 5 * se[:, 2])
    S = o.surface_sums(0)
    F = S[:, 4:].sum(axis=0)
    scale = np.abs(S[:, 1]).sum()
    assert np.all(np.abs(F) < 0.02 * scale)
    r = o.surface_sample(0)
    assert r["CD"] == 0.0 and r["CL"] == 0.0 and np.all(r["Cp"] == 0.0)   # no freestream speed


def test_no_sums_before_n_steady():
    case = W.free_molecular_body("cylinder", s=1.0, cells=20, ppc=10, n_surf=4)
    case["n_steady"] = 30
    o = Oracle(W.gas(), case)
    o.init_particles()
    o.step(30)
    assert np.all(o.surface_sums(0) == 0.0)
    assert o.counters(0)["wall_hits"] > 0
    o.step(5)
    assert o.surface_sums(0)[:, 0].sum() > 0
