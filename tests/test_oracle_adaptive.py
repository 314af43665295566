"""Pins of the oracle's adaptive global step (Eq. 26: the minimum over cells of the Eq. 25
local step, taken from the previous step's moments) and of the ratio-of-DSMC field
(Eq. 27's Dt_DSMC / Dt_G from the time-averaged moments)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from riemann import sample
from helpers import KB, box_case, collisionless_gas


def test_fixed_step_unchanged_by_the_option_off():
    g = W.gas()
    c = W.cylinder_2d(nx=40, ny=30, ppc=8, n_surf=0)
    o = Oracle(g, c)
    o.init_particles()
    o.step(3)
    assert o.step_dt(0)[0] == c["dt_G"]


def test_adaptive_step_is_the_minimum_over_cells_of_eq25():
    """Two regions at different temperatures and drifts: after a step the next global step
    is min over the active cells of L / (|U| + sqrt(gamma R T)) of that step's moments
    (which the Eq. 19 rescale leaves in place, so the post-step estimators give them)."""
    g = W.gas()
    R = KB / g["m"]
    n0, h = 1e20, 1e-3
    hot = dict(n=n0, u=(150.0, 0.0, 0.0), T=900.0)
    cold = dict(n=n0, u=(0.0, -80.0, 0.0), T=250.0)
    c = box_case(dim=2, n=(12, 8, 1), h=h, bc="specular",
                 regions=[((0, 0, 0, 6 * h, 8 * h, 1), hot), ((6 * h, 0, 0, 12 * h, 8 * h, 1), cold)],
                 F_N=n0 * h * h / 60, dt_G=1e-7, capacity=20000, adapt_dt=True)
    o = Oracle(g, c)
    o.init_particles()
    assert o.step_dt(0)[0] == 1e-7
    for _ in range(3):
        o.step(1)
        m = o.sample_moments(0, 1)
        act = m["T"] > 0
        um = np.sqrt((m["u"][act] ** 2).sum(1))
        want = np.min(h / (um + np.sqrt(g["gamma"] * R * m["T"][act])))
        assert o.step_dt(0)[0] == pytest.approx(want, rel=1e-11)
    # the hot, fast region sets it: close to h / (U + a) of its nominal state
    nominal = h / (150.0 + math.sqrt(g["gamma"] * R * 900.0))
    assert 0.6 * nominal < o.step_dt(0)[0] < nominal


def test_open_box_keeps_its_state_with_an_adapted_step():
    """Inflow counts scale with the step: a collisionless box fed on every face by a
    drifting Maxwellian keeps it while the step adapts (from a start 3x too small)."""
    g = collisionless_gas()
    R = KB / g["m"]
    T, n0 = 300.0, 1e15
    a = math.sqrt(2 * R * T)
    st = dict(n=n0, u=(0.3 * a, -0.2 * a, 0.0), T=T)
    nb, h = 12, 1.0
    c = box_case(dim=2, n=(nb, nb, 1), h=h, bc="inflow", inflow=st,
                 regions=[((0, 0, 0, nb, nb, 1), st)], F_N=n0 * h * h / 150,
                 dt_G=0.1 * h / a, capacity=60000, adapt_dt=True)
    o = Oracle(g, c)
    o.init_particles()
    o.step(10)
    dts, ns, us, Ts = [], [], [], []
    for _ in range(80):
        dts.append(o.step_dt(0)[0])
        o.step(1)
        m = o.sample_moments(0, 1)
        ns.append(m["n"]); us.append(m["u"]); Ts.append(m["T"])
    dts = np.array(dts)
    nominal = h / (math.hypot(*st["u"][:2]) + math.sqrt(g["gamma"] * R * T))
    assert np.all(dts > 0.5 * nominal) and np.all(dts < nominal)
    assert dts.std() > 0                               # it does follow the moments
    ns, us, Ts = np.array(ns), np.array(us), np.array(Ts)
    assert abs(ns.mean() / n0 - 1) < 0.01
    assert us[..., 0].mean() == pytest.approx(st["u"][0], rel=0.01)
    assert us[..., 1].mean() == pytest.approx(st["u"][1], rel=0.015)
    assert Ts.mean() == pytest.approx(T, rel=0.012)


def test_sod_with_the_adapted_step_matches_exact_riemann(gas):
    """The Kn = 1e-4 Sod tube advanced with Eq. 26 steps (set by the fastest cell, about
    the fixed step here) still reproduces the Euler solution on the plateaus at
    t = 0.2 L / a_L."""
    reps = 4
    cases = []
    for s in range(reps):
        c = W.sod_1d(seed=s + 1)
        c["adapt_dt"] = True
        cases.append(c)
    o = Oracle(gas, cases)
    o.init_particles()
    t_end = W.sod_steps() * cases[0]["dt_G"]
    t = 0.0
    while t + o.step_dt(0)[0] <= t_end:
        t += o.step_dt(0)[0]
        o.step(1)
    nc = cases[0]["nx"]
    xs = (np.arange(nc) + 0.5) / nc
    rho = np.zeros(nc); T = np.zeros(nc)
    for k in range(reps):
        m = o.sample_moments(k, 1)
        rho += m["n"] / reps; T += m["T"] / reps
        assert o.step_dt(k)[0] != cases[0]["dt_G"]
        assert 0.5 * cases[0]["dt_G"] < o.step_dt(k)[0] < 2.0 * cases[0]["dt_G"]
    m_ = gas["m"]
    R = KB / m_
    rl, rr = W.SOD_N_LEFT * m_, W.SOD_N_RIGHT * m_
    pl, pr = rl * R * W.SOD_T_LEFT, rr * R * W.SOD_T_RIGHT
    ex = sample(xs, t, 0.5, rl, 0.0, pl, rr, 0.0, pr, gas["gamma"])
    for lo, hi in [(0.485, 0.565), (0.675, 0.775), (0.05, 0.25), (0.85, 0.98)]:
        sel = (xs > lo) & (xs < hi)
        assert np.mean(rho[sel] * m_) == pytest.approx(np.mean(ex[sel, 0]), rel=0.05), (lo, hi)
        Tex = np.mean(ex[sel, 2] / (ex[sel, 0] * R))
        assert np.mean(T[sel]) == pytest.approx(Tex, rel=0.05), (lo, hi)


def test_dsmc_ratio_of_homogeneous_cells(gas):
    """0-D cells with Dt_c = r tau_0 and the gas at the nominal state: the ratio of DSMC is
    min(1, 1/r) (T and n, hence tau, stay at their nominal values)."""
    ncells = 48
    c = W.relax_0d(ncells=ncells, ppc=1000, n_steady=0)
    r = np.geomspace(0.05, 20.0, ncells)
    c["dt_over_tau"] = r
    v0, cell, ids = W.relax_0d_state(c, ppc=1000, tx_over_t=1.0, skew=0.0)
    o = Oracle(gas, c)
    o.set_state(0, None, v0, cell, ids, len(ids), 0)
    o.step(4)
    ratio = o.dsmc_ratio(0)
    want = np.minimum(1.0, 1.0 / r)
    # tau ~ T^(omega - 1): the sampled T is within ~0.3 % of nominal
    np.testing.assert_allclose(ratio, want, rtol=0.01)
    assert np.all(ratio[r <= 0.9] == 1.0)


def test_dsmc_ratio_in_the_cylinder_freestream(gas):
    """Ma 10 freestream at Kn 0.01 on D: Dt_c / tau = 0.068 at h = lambda, 0.68 on this
    10x coarser grid, so DSMC only (ratio 1) upstream of the bow shock, up to the noise of
    a few samples of 10-particle cells."""
    c = W.cylinder_2d(nx=80, ny=60, ppc=10, n_steady=0, n_surf=0)
    o = Oracle(gas, c)
    o.init_particles()
    o.step(4)
    ratio = o.dsmc_ratio(0).reshape(60, 80)
    up = ratio[5:55, 1:8]
    assert np.median(up) == 1.0 and np.mean(up == 1.0) > 0.9 and up.min() > 0.8
    assert np.all((ratio >= 0.0) & (ratio <= 1.0))
