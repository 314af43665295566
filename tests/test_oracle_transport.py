"""Pins of the oracle's Step (2)-(3): free transport, walls, inflow, stable indexing."""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import erf

import workloads as W
from oracle import oracle as O
from oracle.oracle import Oracle
from helpers import KB, box_case, collisionless_gas, normal_speed_cdf, rayleigh_cdf


def test_free_transport_exact():
    g = collisionless_gas()
    c = box_case(dim=2, dt_G=0.5)
    o = Oracle(g, c)
    x = np.array([[1.5, 1.5, 0], [3.2, 7.7, 0], [8.9, 0.1, 0], [5.0, 5.0, 0]])
    v = np.array([[2.0, 0.0, 3.0], [-1.0, 2.0, 0.0], [0.5, 3.0, -1.0], [0.0, 0.0, 9.0]])
    cell = (np.floor(x[:, 0]) + 10 * np.floor(x[:, 1])).astype(np.int32)
    o.set_state(0, x, v, cell, np.arange(4), 4, 0)
    o.step(1)
    s = o.get_state(0)
    order = np.argsort(s["id"])
    xe = x + v * 0.5
    assert np.array_equal(s["x"][order][:, :2], xe[:, :2])
    assert np.array_equal(s["v"][order], v)           # single-particle cells: no collisions
    assert np.array_equal(s["cell"][order], (np.floor(xe[:, 0]) + 10 * np.floor(xe[:, 1])).astype(np.int32))


def test_specular_walls_reflect_exactly_and_conserve():
    g = collisionless_gas()
    c = box_case(dim=1, n=(4, 1, 1), bc="specular", dt_G=0.3)
    o = Oracle(g, c)
    x = np.array([[0.1, 0, 0], [3.95, 0, 0]])
    v = np.array([[-1.0, 0.2, 0.0], [0.5, 0.0, 0.1]])
    o.set_state(0, x, v, np.array([0, 3], np.int32), np.arange(2), 2, 0)
    o.step(1)
    s = o.get_state(0)
    assert s["x"][0, 0] == pytest.approx(0.2, abs=1e-15) and s["v"][0, 0] == 1.0
    assert s["x"][1, 0] == pytest.approx(2 * 4.0 - 4.1, abs=1e-15) and s["v"][1, 0] == -0.5
    assert list(s["cell"]) == [0, 3]


def test_outflow_removes():
    g = collisionless_gas()
    c = box_case(dim=2, dt_G=1.0)
    o = Oracle(g, c)
    x = np.array([[0.5, 5.5, 0], [9.5, 5.5, 0], [5.5, 9.5, 0], [5.5, 5.5, 0]])
    v = np.array([[-1.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0.2, 0.2, 0]])
    cell = (np.floor(x[:, 0]) + 10 * np.floor(x[:, 1])).astype(np.int32)
    o.set_state(0, x, v, cell, np.arange(4), 4, 0)
    o.step(1)
    s = o.get_state(0)
    assert list(s["id"]) == [3]
    assert o.counters()["removed"] == 3


def _ring_shot(g, body, n=4000, v0=100.0, Tw=500.0):
    """Particles on a ring of radius 0.6 around the body centre, moving radially inward
    at v0 for dt = 0.2 / v0: each hits the surface after 0.1 / v0."""
    if body == "cylinder":
        c = box_case(dim=2, n=(40, 40, 1), h=0.1, body="cylinder", body_c=(2.0, 2.0, 0.0),
                     body_r=0.5, body_T=Tw, dt_G=0.2 / v0, capacity=2 * n)
        phi = np.random.default_rng(5).uniform(0, 2 * np.pi, n)
        nh = np.stack([np.cos(phi), np.sin(phi), np.zeros(n)], 1)
    else:
        c = box_case(dim=3, n=(40, 40, 40), h=0.1, body="sphere", body_c=(2.0, 2.0, 2.0),
                     body_r=0.5, body_T=Tw, dt_G=0.2 / v0, capacity=2 * n)
        z = np.random.default_rng(5).standard_normal((n, 3))
        nh = z / np.linalg.norm(z, axis=1, keepdims=True)
    ctr = np.array(c["body_c"])
    x = ctr + 0.6 * nh
    if body == "cylinder":
        x[:, 2] = 0.0
    v = -v0 * nh
    ijk = np.floor(x / 0.1).astype(np.int64)
    cell = ijk[:, 0] + 40 * ijk[:, 1] + (1600 * ijk[:, 2] if body == "sphere" else 0)
    o = Oracle(g, c)
    o.set_state(0, x, v, cell.astype(np.int32), np.arange(n), n, 0)
    o.step(1)
    s = o.get_state(0)
    order = np.argsort(s["id"])
    return c, nh, s["x"][order], s["v"][order], o


@pytest.mark.parametrize("body", ["cylinder", "sphere"])
def test_diffuse_wall_kinematics_and_distribution(body):
    g = collisionless_gas()
    Tw = 500.0
    c, nh, xf, vf, o = _ring_shot(g, body, Tw=Tw)
    R = KB / g["m"]
    ctr = np.array(c["body_c"])
    n = len(nh)
    assert o.counters()["wall_hits"] == n
    xh = ctr + 0.5 * nh
    dt_rem = c["dt_G"] - 0.1 / 100.0
    na = 2 if body == "cylinder" else 3
    assert np.allclose(xf[:, :na], (xh + vf * dt_rem)[:, :na], rtol=0, atol=1e-12)
    cn = np.sum(vf * nh, axis=1)
    assert np.all(cn > 0)
    assert stats.kstest(cn, lambda x: rayleigh_cdf(x, R * Tw)).pvalue > 1e-3
    assert np.mean(cn) == pytest.approx(math.sqrt(math.pi * R * Tw / 2), rel=0.03)
    tang = vf - cn[:, None] * nh
    # tangential components: two independent N(0, R Tw) directions -> |c_t|^2 ~ R Tw chi2(2)
    t2 = np.sum(tang * tang, axis=1) / (R * Tw)
    assert stats.kstest(t2, stats.chi2(2).cdf).pvalue > 1e-3


@pytest.mark.parametrize("s", [-2.0, -0.5, 0.0, 0.4, 1.5, 9.13])
def test_inflow_normal_speed_distribution(s):
    rng = np.random.default_rng(int(abs(s) * 100) + 1)
    n = 20000
    zs = np.empty(n)
    used_tot = 0
    for i in range(n):
        w = rng.integers(0, 2 ** 32, 4 * 64, dtype=np.uint64).astype(np.uint32)
        zs[i], used = O.sample_normal_speed(s, w)
        assert used > 0
        used_tot += used
    assert stats.kstest(zs, lambda z: normal_speed_cdf(z, s)).pvalue > 1e-3
    # mean: [s e^{-s^2} + sqrt(pi)/2 (1 + 2 s^2)(1 + erf s)] / [e^{-s^2} + sqrt(pi) s (1 + erf s)]
    mean = (s * math.exp(-s * s) + 0.5 * math.sqrt(math.pi) * (1 + 2 * s * s) * (1 + erf(s))) / \
           (math.exp(-s * s) + math.sqrt(math.pi) * s * (1 + erf(s)))
    assert np.mean(zs) == pytest.approx(mean, rel=0.02)


def test_inflow_counts_match_flux():
    g = collisionless_gas()
    R = KB / g["m"]
    T, n0 = 300.0, 1e15
    U = (0.4 * math.sqrt(2 * R * T), 0.0, 0.0)
    st = dict(n=n0, u=U, T=T)
    c = box_case(dim=2, n=(6, 4, 1), h=0.5, bcs=("inflow", "inflow", "inflow", "outflow", "outflow", "outflow"),
                 inflow=st, F_N=1e12, dt_G=1e-4, capacity=200000)
    o = Oracle(g, c)
    f = o.faces()
    assert list(f["side"]) == [0] * 4 + [1] * 4 + [2] * 6
    # one-way flux through a face of area h * 1 m with inward normal +x, -x, +y
    beta = 1 / math.sqrt(2 * R * T)

    def flux(s):
        return n0 * (math.exp(-s * s) + math.sqrt(math.pi) * s * (1 + erf(s))) / (2 * beta * math.sqrt(math.pi))
    lam = [flux(U[0] * beta), flux(-U[0] * beta), flux(0.0)]
    for side, l in enumerate(lam):
        assert np.allclose(f["lam"][f["side"] == side], l * 0.5 * 1e-4 / 1e12, rtol=1e-13)
    steps = 30
    o.step(steps)
    inj = o.counters()["injected"]
    expect = steps * f["lam"].sum()
    assert abs(inj - expect) < 4 * math.sqrt(steps * len(f["lam"]) * 0.25) + 1


def test_open_box_flux_balance():
    """A collisionless box whose faces all feed the same drifting Maxwellian and remove
    what leaves stays at that state: density, drift and temperature everywhere."""
    g = collisionless_gas()
    R = KB / g["m"]
    T, n0 = 300.0, 1e15
    a = math.sqrt(2 * R * T)
    st = dict(n=n0, u=(0.3 * a, -0.2 * a, 0.0), T=T)
    h = 1.0
    nb = 12
    c = box_case(dim=2, n=(nb, nb, 1), h=h, bc="inflow", inflow=st,
                 regions=[((0, 0, 0, nb, nb, 1), st)], F_N=n0 * h * h / 150, dt_G=0.5 * h / a,
                 capacity=60000)
    o = Oracle(g, c)
    o.init_particles()
    o.step(10)
    ns, us, Ts = [], [], []
    for _ in range(80):
        o.step(1)
        m = o.sample_moments(0, 1)
        ns.append(m["n"]); us.append(m["u"]); Ts.append(m["T"])
    ns, us, Ts = np.array(ns), np.array(us), np.array(Ts)
    nmean = ns.mean(axis=0).reshape(nb, nb)
    # the box average is strongly autocorrelated in time (slow particles stay many
    # steps): ~0.4% noise on n and T over this window
    assert abs(nmean.mean() / n0 - 1) < 0.01
    edge = np.concatenate([nmean[0], nmean[-1], nmean[1:-1, 0], nmean[1:-1, -1]])
    assert abs(edge.mean() / n0 - 1) < 0.015
    assert np.all(np.abs(nmean / n0 - 1) < 0.1)
    assert us[..., 0].mean() == pytest.approx(st["u"][0], rel=0.01)
    assert us[..., 1].mean() == pytest.approx(st["u"][1], rel=0.015)
    assert Ts.mean() == pytest.approx(T, rel=0.012)


def test_stable_sort_order_and_bijection():
    g = W.gas()
    c = W.cylinder_2d(nx=40, ny=30, ppc=8)
    o = Oracle(g, c)
    o.init_particles()
    o.step(3)
    before = o.get_state(0)
    cnt0 = o.counters()
    pos_before = {int(i): k for k, i in enumerate(before["id"])}
    o.step(1)
    after = o.get_state(0)
    cnt1 = o.counters()
    cells = after["cell"]
    assert np.all(np.diff(cells) >= 0)
    ids = after["id"]
    assert len(np.unique(ids)) == len(ids)
    injected = cnt1["injected"] - cnt0["injected"]
    removed = cnt1["removed"] - cnt0["removed"]
    assert injected > 0 and removed > 0
    # the live count after one step: survivors plus the particles injected in it
    assert len(ids) == len(before["id"]) + injected - removed
    old = np.array([int(i) in pos_before for i in ids])
    assert (~old).sum() == injected
    for k in np.unique(cells):
        sel = np.where(cells == k)[0]
        o_idx = [pos_before[int(i)] for i in ids[sel] if int(i) in pos_before]
        assert o_idx == sorted(o_idx)                   # ties keep the previous order
        new = [int(i) for i in ids[sel] if int(i) not in pos_before]
        assert new == sorted(new)                       # injected ones last, by id
        if new and o_idx:
            assert all(int(i) in pos_before for i in ids[sel][: len(o_idx)])
    # brute force: the array before the sort holds the survivors in their previous order,
    # then the injected particles in injection (= id) order; a stable argsort of their new
    # cells must give the oracle's order exactly
    cell_of = {int(i): int(cl) for i, cl in zip(ids, cells)}
    pre_ids = [int(i) for i in before["id"] if int(i) in cell_of]
    pre_ids += sorted(int(i) for i in ids if int(i) not in pos_before)
    pre_cells = np.array([cell_of[i] for i in pre_ids])
    perm = np.argsort(pre_cells, kind="stable")
    assert np.array_equal(np.array(pre_ids)[perm], ids)


def test_closed_box_conserves_particles_momentum_energy():
    g = W.gas()
    c = W.sod_1d(ncells=40, ppc_left=40)
    o = Oracle(g, c, trace=True)
    o.init_particles()
    n0 = o.num_particles()
    s0 = o.get_state(0)
    E0 = np.sum(s0["v"] ** 2)
    o.step(10)
    s1 = o.get_state(0)
    assert o.num_particles() == n0
    # walls flip x-momentum, so only y/z momentum and energy are invariants
    assert np.sum(s1["v"][:, 1:], axis=0) == pytest.approx(np.sum(s0["v"][:, 1:], axis=0), abs=1e-9 * math.sqrt(E0))
    assert np.sum(s1["v"] ** 2) == pytest.approx(E0, rel=1e-12)
