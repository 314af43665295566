"""Pins of the oracle's hexahedral meshes (3-D face-to-face tracking through planar faces).

* A box meshed as hexahedra is the 3-D grid case it was made from, step after step.
* On a mesh with jittered node planes the tracked position is the straight flight, its cell
  the one a brute-force point location finds, and a closed specular box keeps every particle
  and the energy.
* A free-molecular stream past a diffuse sphere on a spherical shell of hexahedra (poles
  with collapsed faces) gives the kinetic-theory wall fluxes and the closed-form drag; a gas
  at rest there stays uniform shell by shell.
* Non-planar faces and inverted cells are rejected.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle, OracleError
from test_oracle_surface import cd_closed, element_means

GAS = W.gas()
HF = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]


def _base(seed=3):
    st = dict(n=1e20, u=(800.0, 100.0, -50.0), T=300.0)
    return W._case(dim=3, nx=6, ny=5, nz=4, h=(0.05, 0.05, 0.05),
                   bc=("inflow", "outflow", "specular", "outflow", "outflow", "specular"), inflow=st,
                   regions=[((0, 0, 0, 0.3, 0.25, 0.2), st)], F_N=1e20 * 0.05 ** 3 / 30,
                   dt_G=0.5 * 0.05 / 1100.0, T_sigma=600.0, seed=seed, n_steady=2, capacity=40000)


def _inside(mesh, cells, x, tol=1e-12):
    P = mesh["xy"][mesh["quad"][cells]]                  # (n, 8, 3)
    ok = np.ones(len(cells), bool)
    for fn in HF:
        A = P[:, fn[0]]
        nf = np.cross(P[:, fn[2]] - P[:, fn[0]], P[:, fn[3]] - P[:, fn[1]])
        ln = np.linalg.norm(nf, axis=1)
        sd = np.einsum("ij,ij->i", A - x, nf) / np.where(ln > 0, ln, 1.0)
        ok &= (ln == 0) | (sd > -tol)
    return ok


def test_meshed_box_is_the_3d_grid_case():
    base = _base()
    A, B = Oracle(GAS, base), Oracle(GAS, W.mesh_twin_3d(base))
    A.init_particles()
    B.init_particles()
    for _ in range(6):
        A.step(1)
        B.step(1)
        sa, sb = A.get_state(), B.get_state()
        assert np.array_equal(sa["id"], sb["id"]) and np.array_equal(sa["cell"], sb["cell"])
        np.testing.assert_allclose(sb["x"], sa["x"], rtol=0, atol=1e-12)
        np.testing.assert_allclose(sb["v"], sa["v"], rtol=1e-12, atol=1e-9)
    ca, cb = A.counters(0), B.counters(0)
    assert ca == cb and ca["injected"] > 0 and ca["removed"] > 0 and ca["accepted"] > 0
    np.testing.assert_allclose(B.get_cells(0)["vol"], A.get_cells(0)["vol"], rtol=1e-12)
    np.testing.assert_allclose(B.sample_moments(0, 0)["T"], A.sample_moments(0, 0)["T"], rtol=1e-10)


def test_tracking_in_jittered_hexahedra_is_straight_flight():
    case = _base(seed=4)
    case["bc"] = ("specular",) * 6
    mc = W.mesh_twin_3d(case, jitter=0.2)
    o = Oracle(GAS, mc)
    o.init_particles()
    s0 = o.get_state()
    assert np.all(_inside(mc["mesh"], s0["cell"], s0["x"]))
    e0 = (s0["v"] ** 2).sum()
    ncell = len(mc["mesh"]["quad"])
    hi = np.array([0.3, 0.25, 0.2])
    for _ in range(5):
        s0 = o.get_state()
        o.step(1)
        s1 = o.get_state()
        assert len(s1["id"]) == len(s0["id"])
        assert np.all(_inside(mc["mesh"], s1["cell"], s1["x"]))
        pos = dict(zip(s1["id"], range(len(s1["id"]))))
        j = np.array([pos[i] for i in s0["id"]])
        free = s0["x"] + s0["v"] * case["dt_G"]
        far = np.all((free > 1e-9) & (free < hi - 1e-9), axis=1)
        assert far.mean() > 0.7
        np.testing.assert_allclose(s1["x"][j[far]], free[far], rtol=0, atol=1e-13)
        for i in np.flatnonzero(far)[:150]:
            ins = _inside(mc["mesh"], np.arange(ncell), np.repeat(free[i:i + 1], ncell, axis=0), tol=-1e-12)
            assert ins[s1["cell"][j[i]]] and ins.sum() == 1
    assert abs((o.get_state()["v"] ** 2).sum() - e0) < 1e-9 * e0


def test_free_molecular_sphere_on_a_hexahedral_shell():
    T, Tw, s = 300.0, 500.0, 1.0
    case = W.free_molecular_sphere_mesh(s=s, T=T, T_w=Tw)
    o = Oracle(GAS, case)
    o.init_particles()
    ns, R = case["n_surf"], case["body_r"]
    th = np.pi * np.arange(ns + 1) / ns
    area = 2 * np.pi * R * R * (np.cos(th[:-1]) - np.cos(th[1:]))
    n, U = case["inflow"]["n"], case["inflow"]["u"][0]
    qd = 0.5 * n * W.ARGON["m"] * U * U
    prev, rows, cds = np.zeros((ns, 7)), [], []
    batches, steps = 8, 60
    for _ in range(batches):
        o.step(steps)
        S = o.surface_sums(0)
        d, prev = S - prev, S
        t = steps * case["dt_G"]
        rows.append(np.stack([-d[:, 1] / (area * t), d[:, 2] / (area * t), d[:, 3] / (area * t)], axis=1))
        cds.append(d[:, 4].sum() / t / (qd * np.pi * R * R))
    rows, cds = np.array(rows), np.array(cds)
    ref = element_means(n, U, T, Tw, ns, True)
    mean, se = rows.mean(axis=0), rows.std(axis=0, ddof=1) / math.sqrt(batches)
    # the inscribed polyhedron stands for the sphere: a bias of O((pi / n_theta)^2)
    assert np.all(np.abs(mean - ref) < 5.0 * se + 0.03 * np.abs(ref).max(axis=0)), (mean, ref)
    cd_ref = cd_closed(s, T, Tw, True)
    assert abs(cds.mean() - cd_ref) < 5.0 * cds.std(ddof=1) / math.sqrt(batches) + 0.03 * cd_ref, (cds.mean(), cd_ref)


def test_gas_at_rest_in_a_hexahedral_shell_stays_uniform():
    T = 300.0
    case = W.free_molecular_sphere_mesh(s=0.0, T=T, T_w=T, n_surf=2, total=30000)
    o = Oracle(GAS, case)
    o.init_particles()
    o.step(600)
    m = o.sample_moments(0, 0)
    vol = o.get_cells(0)["vol"]
    per = 12 * 24
    n_sh = (m["n"] * vol).reshape(-1, per).sum(axis=1) / vol.reshape(-1, per).sum(axis=1)
    n0 = case["inflow"]["n"]
    assert np.all(np.abs(n_sh[1:] / n0 - 1.0) < 0.03), n_sh / n0
    assert abs((m["n"] * vol).sum() / vol.sum() / n0 - 1.0) < 0.01
    r = o.surface_sample(0)
    assert np.all(np.abs(r["p"] / (n0 * W.K_BOLTZMANN * T) - 1.0) < 0.06)


@pytest.mark.parametrize("what", ["nonplanar", "inverted", "nbr", "cylinder"])
def test_bad_hexahedra_are_rejected(what):
    case = W.mesh_twin_3d(_base())
    m = {k: np.array(v, copy=True) for k, v in case["mesh"].items()}
    if what == "nonplanar":
        c = m["quad"][13]
        m["xy"][c[6]] = m["xy"][c[6]] + np.array([0.0, 0.0, 0.01])   # bends faces of its cells
    elif what == "inverted":
        m["quad"][7] = m["quad"][7][[4, 5, 6, 7, 0, 1, 2, 3]]
    elif what == "nbr":
        m["nbr"][0, 3] = 9
    else:
        case["body"] = "cylinder"
    case["mesh"] = m
    with pytest.raises(OracleError):
        Oracle(GAS, case)
