"""Hexahedral meshes on the GPU (gfx950) against the FP64 oracle, through the C ABI.

FP64 from the same initial state and RNG streams: bit-exact ids, cells, counters and
per-cell collision records; positions within 1e-12 of the domain size (kept relative to each
cell's first node), velocities within 1e-12 relative; wall sums within 1e-9.  Cases: a box of
hexahedra (inflow, specular and outflow faces), one with jittered node planes (closed
specular box), a small spherical shell (wall, inflow, collapsed pole faces, surface sampling)
and the Sec. 4.4 sphere shell at its full cell count; in FP32-mixed the oracle's
free-molecular drag and equilibrium pins.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from gpu_util import assert_dsmc_ratio_close, vel_rel_err
from test_gpu_parity import _compare_trace
from test_oracle_surface import cd_closed

pytestmark = pytest.mark.gpu


def _sim(gas, cases, **kw):
    from paper_2506_23917_amd.hs import Sim
    return Sim(gas, cases, **kw)


def hex_abs(case, st):
    m = case["mesh"]
    return m["xy"][m["quad"][st["cell"], 0]] + st["pos"].astype(np.float64)


def extent(case):
    xy = case["mesh"]["xy"]
    return float((xy.max(axis=0) - xy.min(axis=0)).max())


def _box(seed=3):
    st = dict(n=1e20, u=(800.0, 100.0, -50.0), T=300.0)
    return W._case(dim=3, nx=6, ny=5, nz=4, h=(0.05, 0.05, 0.05),
                   bc=("inflow", "outflow", "specular", "outflow", "outflow", "specular"), inflow=st,
                   regions=[((0, 0, 0, 0.3, 0.25, 0.2), st)], F_N=1e20 * 0.05 ** 3 / 30,
                   dt_G=0.5 * 0.05 / 1100.0, T_sigma=600.0, seed=seed, n_steady=2, capacity=40000)


def hex_cases():
    box = W.mesh_twin_3d(_box())
    closed = _box(seed=4)
    closed["bc"] = ("specular",) * 6
    jit = W.mesh_twin_3d(closed, jitter=0.2)
    shell = W.sphere_hex(n_phi=16, n_theta=8, n_r=6, r_out=2.0, growth=1.2, ppc_outer=40, seed=7, n_steady=2,
                         n_surf=8)
    return dict(box=box, jitter=jit, shell=shell)


def _compare(gas, case, g, o, vtol=1e-12, label=""):
    assert len(g["id"]) == len(o["id"]), (label, len(g["id"]), len(o["id"]))
    assert np.array_equal(g["id"], o["id"]), label
    assert np.array_equal(g["cell"], o["cell"]), label
    assert g["next_id"] == o["next_id"], label
    err = vel_rel_err(g["vel"], o["v"], gas)
    assert err < vtol, (label, err)
    if len(o["x"]):
        perr = np.abs(hex_abs(case, g) - o["x"]).max() / extent(case)
        assert perr < 1e-12, (label, perr)


@pytest.mark.parametrize("name", ["box", "jitter", "shell"])
def test_hex_init_matches_oracle(gas, name):
    case = hex_cases()[name]
    sim = _sim(gas, case, precision="fp64")
    ora = Oracle(gas, case)
    ora.init_particles()
    _compare(gas, case, sim.export_state(0), ora.get_state(0), vtol=1e-14, label="init " + name)
    np.testing.assert_allclose(sim.sample_moments(0, 1)["n"], ora.sample_moments(0, 1)["n"], rtol=1e-12)


@pytest.mark.parametrize("name,steps", [("box", 6), ("jitter", 6), ("shell", 8)])
def test_hex_fp64_steps_match_oracle(gas, name, steps):
    case = hex_cases()[name]
    sim = _sim(gas, case, precision="fp64", trace=True)
    ora = Oracle(gas, case, trace=True)
    ora.init_particles()
    for s in range(steps):
        sim.step(1)
        ora.step(1)
        lab = "%s step %d" % (name, s + 1)
        _compare(gas, case, sim.export_state(0), ora.get_state(0), label=lab)
        _compare_trace(sim.trace(0), ora.trace(0), label=lab)
    assert sim.counters(0) == ora.counters(0)
    if name == "shell":
        assert ora.counters(0)["wall_hits"] > 0 and ora.counters(0)["injected"] > 0
        sg, so = sim.surface_sums(0), ora.surface_sums(0)
        assert np.array_equal(sg[:, 0], so[:, 0])
        np.testing.assert_allclose(sg, so, rtol=1e-9, atol=1e-9 * np.abs(so).max())
    np.testing.assert_allclose(sim.sample_moments(0, 0)["n"], ora.sample_moments(0, 0)["n"], rtol=1e-11)
    assert_dsmc_ratio_close(sim.dsmc_ratio(0), ora.dsmc_ratio(0), ora.get_cells(0)["acc"], rtol=1e-9, atol=1e-12)


def test_hex_full_size_sphere_steps(gas):
    """The Sec. 4.4 sphere on a 72 x 36 x 76 hexahedral shell (196,992 cells): initial state
    and two FP64 steps, every particle against the oracle, then the FP32-mixed path and a
    graph-replayed run agree with a plain run."""
    case = W.sphere_hex(ppc_outer=20, n_steady=0)
    sim = _sim(gas, case, precision="fp64")
    ora = Oracle(gas, case)
    ora.init_particles()
    _compare(gas, case, sim.export_state(0), ora.get_state(0), vtol=1e-14, label="full init")
    for s in range(2):
        sim.step(1)
        ora.step(1)
        _compare(gas, case, sim.export_state(0), ora.get_state(0), label="full step %d" % (s + 1))
    assert sim.counters(0) == ora.counters(0)
    from test_gpu_properties import _same
    a = _sim(gas, case, precision="fp32")
    b = _sim(gas, case, precision="fp32", graph=True)
    a.step(4)
    b.step(4)
    _same(a.export_state(0), b.export_state(0), "hex graph")


def test_hex_fp32_free_molecular_sphere_drag(gas):
    T, Tw, s = 300.0, 500.0, 1.0
    case = W.free_molecular_sphere_mesh(s=s, T=T, T_w=Tw, total=60000)
    sim = _sim(gas, case, precision="fp32")
    R = case["body_r"]
    n, U = case["inflow"]["n"], case["inflow"]["u"][0]
    qd = 0.5 * n * W.ARGON["m"] * U * U
    prev, cds = np.zeros((case["n_surf"], 7)), []
    for _ in range(8):
        sim.step(100)
        S = sim.surface_sums(0)
        d, prev = S - prev, S
        cds.append(d[:, 4].sum() / (100 * case["dt_G"]) / (qd * np.pi * R * R))
    cds = np.array(cds)
    ref = cd_closed(s, T, Tw, True)
    assert abs(cds.mean() - ref) < 5.0 * cds.std(ddof=1) / math.sqrt(8) + 0.03 * ref, (cds.mean(), ref)


def test_hex_fp32_gas_at_rest_stays_uniform(gas):
    T = 300.0
    case = W.free_molecular_sphere_mesh(s=0.0, T=T, T_w=T, n_surf=2, total=60000)
    sim = _sim(gas, case, precision="fp32")
    sim.step(600)
    m = sim.sample_moments(0, 0)
    vol = Oracle(gas, case).get_cells(0)["vol"]
    per = 12 * 24
    n_sh = (m["n"] * vol).reshape(-1, per).sum(axis=1) / vol.reshape(-1, per).sum(axis=1)
    n0 = case["inflow"]["n"]
    assert np.all(np.abs(n_sh[1:] / n0 - 1.0) < 0.03), n_sh / n0


def test_hex_adaptive_step_and_batch_with_grid_and_quad_cases(gas):
    """Eq. 26 with the hexahedra's L_cell, in one batch with a grid case and a quad-mesh case."""
    shell = hex_cases()["shell"]
    shell["adapt_dt"] = True
    grid = W.cylinder_2d(nx=40, ny=30, ppc=8, seed=11, n_surf=6, n_steady=0)
    og = W.cylinder_ogrid(n_theta=48, first=0.02, growth=1.15, r_out=2.0, ppc_outer=60, seed=12, n_surf=4)
    cases = [grid, shell, og]
    sim = _sim(gas, cases, precision="fp64")
    ora = Oracle(gas, cases)
    ora.init_particles()
    for s in range(4):
        sim.step(1)
        ora.step(1)
        _compare(gas, shell, sim.export_state(1), ora.get_state(1), label="hex adaptive step %d" % (s + 1))
        dg, do = sim.step_dt(1), ora.step_dt(1)
        assert abs(dg[0] - do[0]) <= 1e-12 * do[0]
    assert ora.step_dt(1)[0] != shell["dt_G"]
    for c in (0, 2):
        g0, o0 = sim.export_state(c), ora.get_state(c)
        assert np.array_equal(g0["id"], o0["id"]) and np.array_equal(g0["cell"], o0["cell"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hex_time_averages_agree_with_the_oracle(gas, prec):
    """Small hexahedral sphere shell from the impulsive start, sampled over 300 steps: the
    GPU's time-averaged n and T per cell against the oracle's pooled estimates, in units of
    the standard error of a difference (10 batch means of the oracle's run); cells with at
    least 20 samples in every batch.  z follows Student's t with 9 degrees of freedom."""
    case = W.sphere_hex(n_phi=16, n_theta=8, n_r=6, r_out=2.0, growth=1.2, ppc_outer=80, seed=23,
                        n_steady=60, n_surf=0)
    ora = Oracle(gas, case)
    ora.init_particles()
    ora.step(60)
    batches, prev = [], None
    for _ in range(10):
        ora.step(30)
        acc = ora.get_cells(0)["acc"].copy()
        batches.append(acc - (prev if prev is not None else 0.0))
        prev = acc
    vol = ora.get_cells(0)["vol"]
    m = gas["m"]

    def n_T(acc, nsamp):
        N = acc[:, 0]
        ok = N > 0
        Ns = np.where(ok, N, 1.0)
        n = np.where(ok, case["F_N"] * N / (nsamp * vol), 0.0)
        cc = (acc[:, 4] + acc[:, 5] + acc[:, 6]) / Ns
        uu = (acc[:, 1] ** 2 + acc[:, 2] ** 2 + acc[:, 3] ** 2) / Ns ** 2
        return n, np.where(ok, m / (3 * W.K_BOLTZMANN) * (cc - uu), 0.0)

    bn, bT = (np.array(x) for x in zip(*[n_T(a, 30) for a in batches]))
    on, oT = n_T(prev, 300)
    se_n = bn.std(0, ddof=1) / np.sqrt(10) * np.sqrt(2)
    se_T = bT.std(0, ddof=1) / np.sqrt(10) * np.sqrt(2)
    sim = _sim(gas, case, precision=prec)
    sim.step(360)
    g = sim.sample_moments(0, mode=0)
    assert g["n_samples"] == 300
    nb_min = np.min([b[:, 0] for b in batches], axis=0)
    sel = (nb_min >= 20) & (se_n > 0) & (se_T > 0)
    assert sel.sum() > 0.3 * len(sel)
    zn = (g["n"][sel] - on[sel]) / se_n[sel]
    zT = (g["T"][sel] - oT[sel]) / se_T[sel]
    print(prec, "cells %d mean z^2 n %.3f T %.3f" % (sel.sum(), (zn ** 2).mean(), (zT ** 2).mean()))
    for z in (zn, zT):
        assert (z ** 2).mean() < 2.0
        assert (abs(z) > 4).mean() < 0.02
