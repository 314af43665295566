"""Pins of the oracle's gas model against numbers the paper prints and VHS closed forms."""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import oracle as O

KB = 1.380649e-23
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def paper():
    out = {}
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            out[k] = float(v)
    return out


def test_gas_constants_match_paper(gas):
    P = paper()
    for k in ("d_ref", "T_ref", "mu_ref", "omega"):
        assert gas[k] == P[k]


def test_mean_free_path_reproduces_table1_kn(gas):
    # Sec. 4.1: Kn = lambda / L_ref with L_ref = 1 m (Eq. 32-33), Table 1 densities
    P = paper()
    for i in (1, 2, 3):
        n = P["sod_rho_up%d" % i] / gas["m"]
        lam = O.mean_free_path(gas, n, P["sod_T_up"])
        assert lam / P["sod_L_ref"] == pytest.approx(P["sod_kn%d" % i], rel=1e-4)


def test_mean_free_path_reproduces_cylinder_and_sphere_kn(gas):
    P = paper()
    assert O.mean_free_path(gas, P["cyl_n_kn001"], P["cyl_T"]) == pytest.approx(1e-2, rel=1e-4)
    assert O.mean_free_path(gas, P["cyl_n_kn01"], P["cyl_T"]) == pytest.approx(1e-1, rel=1e-4)
    n_sph = P["sph_rho"] / gas["m"]
    assert O.mean_free_path(gas, n_sph, P["sph_T"]) == pytest.approx(1e-2, rel=1e-4)
    # Sec. 4.4 calls this flow Mach 10: sqrt(gamma R T) at 65 K
    a = math.sqrt(gas["gamma"] * KB / gas["m"] * P["sph_T"])
    assert P["sph_U"] / a == pytest.approx(10.0, rel=1e-3)


def test_workload_literals(gas):
    # the literal constants of the workloads module, recomputed with the oracle
    R = KB / gas["m"]
    assert O.mean_free_path(gas, W.N_INF, W.T_INF) == pytest.approx(0.01, rel=1e-12)
    assert W.U_INF == pytest.approx(10 * math.sqrt(gas["gamma"] * R * W.T_INF), rel=1e-14)
    assert W.U_PLUS_A_INF == pytest.approx(1.1 * W.U_INF, rel=1e-14)
    assert W.SOD_N_LEFT * gas["m"] == pytest.approx(paper()["sod_rho_up3"], rel=1e-12)
    assert W.SOD_A_LEFT == pytest.approx(math.sqrt(gas["gamma"] * R * 273.0), rel=1e-14)
    lam_e = O.mean_free_path(gas, W.JET_N_LAMBDA, W.JET_TE)
    assert lam_e == pytest.approx(1.0, rel=1e-12)
    assert W.JET_UE == pytest.approx(math.sqrt(gas["gamma"] * R * W.JET_TE), rel=1e-14)


def test_viscosity_power_law(gas):
    assert O.viscosity(gas, gas["T_ref"]) == pytest.approx(gas["mu_ref"], rel=1e-15)
    assert O.viscosity(gas, 2 * gas["T_ref"]) == pytest.approx(gas["mu_ref"] * 2 ** gas["omega"], rel=1e-14)


def test_dref_consistent_with_muref(gas):
    # first-approximation VHS viscosity relation (Bird): d_ref^2 =
    # 15 sqrt(m k T_ref / pi) / (2 (5 - 2w)(7 - 2w) mu_ref); the paper prints 4.17e-10 m
    m, w = gas["m"], gas["omega"]
    d2 = 15 * math.sqrt(m * KB * gas["T_ref"] / math.pi) / (2 * (5 - 2 * w) * (7 - 2 * w) * gas["mu_ref"])
    assert math.sqrt(d2) == pytest.approx(gas["d_ref"], rel=2e-3)


@pytest.mark.parametrize("T", [200.0, 273.0, 6866.7])
def test_vhs_equilibrium_collision_rate(gas, T):
    # <sigma_T c_r> over the equilibrium relative-speed distribution of two particles at T
    # (reduced mass m/2) must equal the VHS closed form 4 d^2 sqrt(pi k T_ref / m)
    # (T / T_ref)^(1 - omega).  Integrates the oracle's sigma_c.
    m = gas["m"]
    mr = m / 2
    a = mr / (2 * KB * T)

    def f(cr):
        return cr * cr * math.exp(-a * cr * cr)
    scale = math.sqrt(1 / a)
    norm = integrate.quad(f, 0, 20 * scale)[0]
    mean = integrate.quad(lambda c: O.sigma_c(gas, c) * f(c), 0, 20 * scale, limit=200)[0] / norm
    closed = 4 * gas["d_ref"] ** 2 * math.sqrt(math.pi * KB * gas["T_ref"] / m) * (T / gas["T_ref"]) ** (1 - gas["omega"])
    assert mean == pytest.approx(closed, rel=1e-7)
    if T == 273.0:
        assert closed == pytest.approx(2.9395e-16, rel=1e-4)


def test_vhs_cross_section_at_reference_speed(gas):
    # at the relative speed where 2 k T_ref / (m_r c_r^2) = 1, sigma_T = pi d^2 / Gamma(5/2 - w)
    m = gas["m"]
    cr = math.sqrt(2 * KB * gas["T_ref"] / (m / 2))
    sig = O.sigma_c(gas, cr) / cr
    assert sig == pytest.approx(math.pi * gas["d_ref"] ** 2 / math.gamma(2.5 - gas["omega"]), rel=1e-13)
    # and it scales as c_r^(1 - 2 w)
    assert O.sigma_c(gas, 2 * cr) / (2 * cr) / sig == pytest.approx(2 ** (1 - 2 * gas["omega"]), rel=1e-13)


def test_inflow_flux_limits(gas):
    R = KB / gas["m"]
    st = dict(n=1e20, u=(0.0, 0.0, 0.0), T=300.0)
    # effusion: n c_bar / 4 with c_bar = sqrt(8 R T / pi)
    assert O.inflow_flux(gas, st, (1, 0, 0)) == pytest.approx(1e20 * math.sqrt(8 * R * 300 / math.pi) / 4, rel=1e-13)
    # hypersonic limit: n U
    st2 = dict(n=1e20, u=(50 * math.sqrt(2 * R * 300), 0.0, 0.0), T=300.0)
    assert O.inflow_flux(gas, st2, (1, 0, 0)) == pytest.approx(1e20 * st2["u"][0], rel=1e-6)
    # zero against a strong outflow
    assert O.inflow_flux(gas, st2, (-1, 0, 0)) < 1e-100 * 1e20


def test_cut_cell_volume_rule():
    # a cylinder of radius R: total fluid volume of the cells -> box area minus pi R^2
    case = W.cylinder_2d(nx=80, ny=60, ppc=10)
    h = case["h"][0]
    tot = 0
    for j in range(60):
        for i in range(80):
            tot += O.cut_count(case, i, j, 0)
    area = tot / 256 * h * h
    assert area == pytest.approx(48.0 - math.pi * 0.25, rel=1e-3)
    # far cells are full, the centre cell is empty
    assert O.cut_count(case, 0, 0, 0) == 256
    assert O.cut_count(case, 25, 30, 0) == 0
