"""Pins of the oracle's Step (3)-(5): moments, time split, NTC DSMC, SP-Shakhov,
conservation rescale and sampling."""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import oracle as O
from oracle.oracle import Oracle
from helpers import KB, collisionless_gas


def test_moments_hand_built(gas):
    m = gas["m"]
    v = np.array([[1.0, 2.0, 3.0], [3.0, 2.0, 1.0], [2.0, 2.0, 5.0]])
    FN, V = 1e10, 2.0
    U, T, Q = O.cell_moments(gas, v, FN, V)
    assert np.allclose(U, [2.0, 2.0, 3.0], rtol=0, atol=1e-15)
    # C = (-1,0,0), (1,0,-2), (0,0,2); sum |C|^2 = 10; estimator divides by N - 1 = 2
    assert T == pytest.approx(m * 10 / (3 * KB * 2), rel=1e-15)
    # sum |C|^2 C = (4, 0, -2); Q = n N/((N-1)(N-2)) * m/2 * that, n = N F_N / V
    n = 3 * FN / V
    assert np.allclose(Q, n * 3 / 2 * 0.5 * m * np.array([4.0, 0.0, -2.0]), rtol=1e-15, atol=0)
    # N = 2: no heat flux; N = 1: no temperature
    U2, T2, Q2 = O.cell_moments(gas, v[:2], FN, V)
    # C = (-1,0,1), (1,0,-1): sum |C|^2 = 4 over N - 1 = 1
    assert T2 == pytest.approx(m * 4 / (3 * KB), rel=1e-15) and np.all(Q2 == 0)
    U1, T1, Q1 = O.cell_moments(gas, v[:1], FN, V)
    assert T1 == 0 and np.all(U1 == v[0])


@pytest.mark.parametrize("N", [3, 5, 10])
def test_moment_estimators_unbiased(gas, N):
    rng = np.random.default_rng(N)
    R = KB / gas["m"]
    T = 300.0
    cells = 4000
    Ts, Qs = np.empty(cells), np.empty((cells, 3))
    for k in range(cells):
        v = rng.standard_normal((N, 3)) * math.sqrt(R * T) + [100.0, -50.0, 0.0]
        _, Ts[k], Qs[k] = O.cell_moments(gas, v, 1.0, 1.0)
    assert abs(Ts.mean() - T) < 3.5 * Ts.std() / math.sqrt(cells)
    z = Qs.mean(axis=0) / (Qs.std(axis=0) / math.sqrt(cells))
    assert np.all(np.abs(z) < 3.5)


def test_heat_flux_of_skewed_gaussian(gas):
    # q_x = 1/2 rho (R T_x)^{3/2} (6 s + 8 s^3) / (1 + 2 s^2)^{3/2} for
    # v_x = sqrt(R T_x) (x + s (x^2 - 1)) / sqrt(1 + 2 s^2), x ~ N(0, 1)
    rng = np.random.default_rng(1)
    R = KB / gas["m"]
    Tx, s, N = 400.0, 0.2, 400000
    x = rng.standard_normal(N)
    vx = math.sqrt(R * Tx) * (x + s * (x * x - 1)) / math.sqrt(1 + 2 * s * s)
    v = np.stack([vx, rng.standard_normal(N) * 10, rng.standard_normal(N) * 10], 1)
    FN, V = 1e12, 1.0
    U, T, Q = O.cell_moments(gas, v, FN, V)
    rho = N * FN / V * gas["m"]
    closed = 0.5 * rho * (R * Tx) ** 1.5 * (6 * s + 8 * s ** 3) / (1 + 2 * s * s) ** 1.5
    # sample noise of <C_x^3>: sqrt(15 / N) (R T_x)^{3/2} relative to the closed form's scale
    tol = 3.5 * math.sqrt(15.0 / N) * 0.5 * rho * (R * Tx) ** 1.5
    assert abs(Q[0] - closed) < tol


def test_split_identities():
    rng = np.random.default_rng(2)
    for _ in range(2000):
        tau = 10 ** rng.uniform(-8, -3)
        dtc = tau * 10 ** rng.uniform(-2, 2)
        dtG = dtc * rng.uniform(0.05, 1.0)
        dD, dS = O.split(dtc, tau, dtG)
        assert dD + dS == pytest.approx(dtG, rel=2.3e-16)   # exact up to the rounding of dt_G - dt_D
        assert dD / dtG == pytest.approx(min(1.0, tau / dtc), rel=1e-15)
        P = 0.0 if dtc <= tau else 1 - tau / dtc          # Eq. 24
        assert dS / dtG == pytest.approx(P, rel=1e-12, abs=1e-15)


def _relax_oracle(gas, ncells, ppc=1000, tx=1.5, skew=0.05, r=None, seed=2, trace=True, state_seed=11):
    c = W.relax_0d(ncells=ncells, ppc=ppc, seed=seed)
    if r is not None:
        c["dt_over_tau"] = np.asarray(r, dtype=np.float64)
    v, cell, ids = W.relax_0d_state(c, ppc=ppc, tx_over_t=tx, skew=skew, state_seed=state_seed)
    o = Oracle(gas, c, trace=trace)
    o.set_state(0, None, v, cell, ids, len(ids), 0)
    return c, o, v


def test_collision_conserves_and_scatters_isotropically(gas):
    # two-particle cells: after one accepted NTC pair (and no relaxation) |g'| = |g|, the
    # centre of mass is unchanged and g' points uniformly over the sphere (Eq. 7-9)
    ncells = 6000
    c, o, v0 = _relax_oracle(gas, ncells, ppc=2, tx=1.0, skew=0.0, r=np.full(ncells, 0.9))
    # raise F_N so that about one candidate is drawn per cell per step
    o.step(1)
    tr = o.trace(0)
    s = o.get_state(0)
    v1 = s["v"].reshape(ncells, 2, 3)
    v0 = v0.reshape(ncells, 2, 3)
    sel = (tr["nacc"] == 1) & (tr["nrelax"] == 0)
    assert sel.sum() > 200
    g0 = v0[sel, 0] - v0[sel, 1]
    g1 = v1[sel, 0] - v1[sel, 1]
    assert np.allclose(np.linalg.norm(g1, axis=1), np.linalg.norm(g0, axis=1), rtol=1e-12)
    assert np.allclose(v1[sel].sum(1), v0[sel].sum(1), rtol=1e-12, atol=1e-9)
    ghat = g1 / np.linalg.norm(g1, axis=1, keepdims=True)
    for a in range(3):
        assert stats.kstest((ghat[:, a] + 1) / 2, "uniform").pvalue > 1e-3
    # untouched cells keep their velocities (rescale is the identity up to rounding)
    idle = (tr["nacc"] == 0) & (tr["nrelax"] == 0)
    assert np.allclose(v1[idle], v0[idle], rtol=1e-13, atol=1e-10)


def test_equilibrium_collision_rate_matches_vhs(gas):
    # Maxwellian cells in the pure-DSMC range (dt <= tau): accepted pairs per step
    # = 1/2 N (N-1) (F_N / V) <sigma_T c_r>(T) dt with the VHS closed form <sigma c>
    ncells = 96
    rng = np.random.default_rng(4)
    r = 10 ** rng.uniform(-1.0, np.log10(0.8), ncells)
    c, o, _ = _relax_oracle(gas, ncells, tx=1.0, skew=0.0, r=r)
    m, d, Tr, w = gas["m"], gas["d_ref"], gas["T_ref"], gas["omega"]
    obs = exp = 0.0
    for _ in range(3):
        o.step(1)
        tr = o.trace(0)
        assert np.all(tr["p_relax"] == 0)
        sc = 4 * d * d * math.sqrt(math.pi * KB * Tr / m) * (tr["T"] / Tr) ** (1 - w)
        N = tr["n"].astype(float)
        exp += np.sum(0.5 * N * (N - 1) * c["F_N"] / 1.0 * sc * tr["dt_dsmc"])
        obs += tr["nacc"].sum()
    assert abs(obs - exp) < 3 * math.sqrt(exp), (obs, exp)


@pytest.mark.parametrize("qt", [0.05, 0.3])
def test_shakhov_sampling_moments(gas, qt):
    # accepted draws have zero mean, temperature T, heat flux (1 - Pr) Q and are accepted
    # once per A_max attempts on average (E_fM[A] = 1)
    R = KB / gas["m"]
    T, n = 300.0, 1e20
    p = n * KB * T
    Q = np.array([qt * p * math.sqrt(R * T), 0.0, 0.0])
    a_max = 1 + 20 * (1 - gas["Pr"]) * qt
    rng = np.random.default_rng(int(qt * 100))
    ns = 150000
    Cs = np.empty((ns, 3))
    att = 0
    for i in range(ns):
        w = rng.integers(0, 2 ** 32, 5 * 64, dtype=np.uint64).astype(np.uint32)
        r, Cs[i] = O.shakhov_sample(gas, T, p, Q, a_max, w)
        assert r > 0
        att += r
    sRT = math.sqrt(R * T)
    x = Cs / sRT
    assert np.all(np.abs(x.mean(0)) < 3.5 / math.sqrt(ns) * 1.05)
    assert (x * x).sum(1).mean() / 3 == pytest.approx(1.0, abs=3.5 * math.sqrt(2 / 3 / ns) * 1.5)
    qx = x[:, 0] * (x * x).sum(1)
    target = 2 * (1 - gas["Pr"]) * qt                 # <C_x C^2> / (RT)^{3/2} = 2 q / (rho (RT)^{3/2})
    assert abs(qx.mean() - target) < 3.5 * qx.std() / math.sqrt(ns)
    assert att / ns == pytest.approx(a_max, rel=0.02)


def test_shakhov_reduces_to_maxwellian(gas):
    g = dict(gas)
    g["Pr"] = 1.0
    rng = np.random.default_rng(9)
    for _ in range(200):
        w = rng.integers(0, 2 ** 32, 5 * 4, dtype=np.uint64).astype(np.uint32)
        r, _ = O.shakhov_sample(g, 300.0, 1.0, [5.0, 1.0, 0.0], 1.0, w)
        assert r == 1
        r, _ = O.shakhov_sample(gas, 300.0, 1.0, [0.0, 0.0, 0.0], 1.0, w)
        assert r == 1


def test_relaxed_fraction_and_exact_conservation(gas):
    ncells = 64
    rng = np.random.default_rng(8)
    r = 10 ** rng.uniform(-2, 2, ncells)
    c, o, v0 = _relax_oracle(gas, ncells, r=r)
    o.step(1)
    tr = o.trace(0)
    act = tr["n"] >= 2
    # Bernoulli relaxation: sum over cells of N P has binomial spread
    e = np.sum(tr["n"] * tr["p_relax"])
    var = np.sum(tr["n"] * tr["p_relax"] * (1 - tr["p_relax"]))
    assert abs(tr["nrelax"].sum() - e) < 4 * math.sqrt(var) + 1
    # Eq. 19: mean velocity and energy of each cell restored to round-off
    pre, post = tr["pre_sum"][act], tr["post_sum"][act]
    N = tr["n"][act][:, None]
    cref = np.sqrt(pre[:, 3:4] / N)
    assert np.all(np.abs(post[:, :3] - pre[:, :3]) / (N * cref) < 1e-12)
    assert np.all(np.abs(post[:, 3] - pre[:, 3]) / pre[:, 3] < 1e-12)


def test_pure_dsmc_limit_has_no_relaxation(gas):
    # rarefied cylinder (Kn = 1): dt_c <= tau everywhere -> the hybrid is pure NTC DSMC
    c = W.cylinder_2d(nx=40, ny=30, ppc=6)
    c["inflow"] = dict(c["inflow"], n=c["inflow"]["n"] / 100)
    c["regions"] = [(c["regions"][0][0], c["inflow"])]
    c["F_N"] /= 100
    o = Oracle(gas, c, trace=True)
    o.init_particles()
    o.step(5)
    tr = o.trace(0)
    assert np.all(tr["p_relax"] == 0) and tr["nrelax"].sum() == 0
    assert o.counters()["relaxed"] == 0


def test_sampling_accumulators_and_finalize(gas):
    g = collisionless_gas()
    c = W.relax_0d(ncells=3, ppc=50, n_steady=2)
    c["dt_over_tau"] = np.full(3, 0.01)
    v, cell, ids = W.relax_0d_state(c, ppc=50, state_seed=3)
    v += np.array([300.0, -20.0, 5.0])
    o = Oracle(g, c)
    o.set_state(0, None, v, cell, ids, len(ids), 0)
    o.step(5)      # steps 0..4, sampled at 2, 3, 4
    cells = o.get_cells(0)
    assert cells["n_samples"] == 3
    s = o.get_state(0)
    vv = s["v"].reshape(3, 50, 3)
    acc = cells["acc"]
    assert np.allclose(acc[:, 0], 150)
    assert np.allclose(acc[:, 1:4], 3 * vv.sum(1), rtol=1e-10)
    m = o.sample_moments(0, 0)
    U = vv.mean(1)
    Cc = vv - U[:, None, :]
    Tb = gas["m"] / (3 * KB) * (Cc ** 2).sum(2).mean(1)
    n = c["F_N"] * 50 / 1.0
    qb = 0.5 * gas["m"] * n * (Cc * (Cc ** 2).sum(2, keepdims=True)).mean(1)
    assert np.allclose(m["n"], n, rtol=1e-13)
    assert np.allclose(m["u"], U, rtol=1e-10)
    assert np.allclose(m["T"], Tb, rtol=1e-9)
    assert np.allclose(m["q"], qb, rtol=1e-6, atol=1e-9 * np.abs(qb).max())
