"""Pins of the oracle's body-fitted quadrilateral meshes (free transport by face-to-face
tracking, uniform placement in a quad, inflow through arbitrary edges, wall edges).

* A box meshed as quads is the grid case it was made from: same initial particles, same
  injections, same moves, cells, collisions and samples (the grid path is pinned on its
  own), step after step.
* On a jittered mesh the tracked position is the straight flight x + c dt, its cell is the
  one a brute-force point location finds, and a closed specular box keeps every particle
  and the total energy.
* Initial positions are uniform in a strongly trapezoidal quad (chi-square against the
  area shares of a sub-division).
* A free-molecular stream past a diffuse cylinder on an O-grid gives the kinetic-theory wall
  fluxes and drag (closed forms of the surface-sampling pins), and the undisturbed density
  in the cells upstream of the body: the oblique inflow edges inject the right flux.
"""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle.oracle import Oracle, OracleError
from test_oracle_surface import cd_closed, element_means

GAS = W.gas()


def _base(seed=3, jitter_ok=True):
    st = dict(n=1e20, u=(800.0, 100.0, 0.0), T=300.0)
    return W._case(dim=2, nx=12, ny=8, h=(0.05, 0.05, 1.0),
                   bc=("inflow", "outflow", "specular", "outflow", "outflow", "outflow"), inflow=st,
                   regions=[((0.0, 0.0, 0.0, 0.6, 0.4, 1.0), st)], F_N=1e20 * 0.0025 / 40,
                   dt_G=0.5 * 0.05 / 1100.0, T_sigma=600.0, seed=seed, n_steady=2, capacity=20000)


def _inside(mesh, cell, x, tol=1e-12):
    """Signed distances of x to the four edges of its cell (positive inside) > -tol."""
    xy, quad = mesh["xy"], mesh["quad"]
    P = xy[quad[cell]]                                   # (n, 4, 2)
    ok = np.ones(len(cell), bool)
    for j in range(4):
        A, B = P[:, j], P[:, (j + 1) % 4]
        e = B - A
        cr = e[:, 0] * (x[:, 1] - A[:, 1]) - e[:, 1] * (x[:, 0] - A[:, 0])
        ok &= cr / np.hypot(e[:, 0], e[:, 1]) > -tol
    return ok


def test_meshed_box_is_the_grid_case():
    base = _base()
    A, B = Oracle(GAS, base), Oracle(GAS, W.mesh_twin(base))
    A.init_particles()
    B.init_particles()
    for _ in range(8):
        A.step(1)
        B.step(1)
        sa, sb = A.get_state(), B.get_state()
        assert np.array_equal(sa["id"], sb["id"]) and np.array_equal(sa["cell"], sb["cell"])
        np.testing.assert_allclose(sb["x"], sa["x"], rtol=0, atol=1e-12)
        np.testing.assert_allclose(sb["v"], sa["v"], rtol=1e-12, atol=1e-9)
    ca, cb = A.counters(0), B.counters(0)
    assert ca == cb and ca["injected"] > 0 and ca["removed"] > 0 and ca["accepted"] > 0
    np.testing.assert_allclose(B.get_cells(0)["vol"], A.get_cells(0)["vol"], rtol=1e-12)
    ma, mb = A.sample_moments(0, 0), B.sample_moments(0, 0)
    for k in ("n", "T"):
        np.testing.assert_allclose(mb[k], ma[k], rtol=1e-10)
    np.testing.assert_allclose(B.dsmc_ratio(0), A.dsmc_ratio(0), rtol=1e-10)


def test_tracking_on_a_jittered_mesh_is_straight_flight():
    case = _base(seed=4)
    case["bc"] = ("specular",) * 4 + ("outflow",) * 2
    mc = W.mesh_twin(case, jitter=0.2)
    o = Oracle(GAS, mc)
    o.init_particles()
    s0 = o.get_state()
    assert np.all(_inside(mc["mesh"], s0["cell"], s0["x"]))
    e0 = (s0["v"] ** 2).sum()
    for step in range(6):
        s0 = o.get_state()
        o.step(1)
        s1 = o.get_state()
        assert len(s1["id"]) == len(s0["id"])               # closed box: nobody leaves
        assert np.all(_inside(mc["mesh"], s1["cell"], s1["x"]))
        # particles whose straight path stays inside the box moved along it
        pos = dict(zip(s1["id"], range(len(s1["id"]))))
        j = np.array([pos[i] for i in s0["id"]])
        free = s0["x"][:, :2] + s0["v"][:, :2] * case["dt_G"]
        far = np.all((free > 1e-9) & (free < np.array([0.6, 0.4]) - 1e-9), axis=1)
        assert far.mean() > 0.8
        np.testing.assert_allclose(s1["x"][j[far], :2], free[far], rtol=0, atol=1e-13)
        # the tracked cell is the cell that contains the point (brute force over all cells)
        for i in np.flatnonzero(far)[:200]:
            k = s1["cell"][j[i]]
            ins = _inside(mc["mesh"], np.arange(96), np.repeat(free[i:i + 1], 96, axis=0), tol=-1e-12)
            assert ins[k] and ins.sum() == 1
    # specular edges and collisions keep the kinetic energy
    e1 = (o.get_state()["v"] ** 2).sum()
    assert abs(e1 - e0) < 1e-9 * e0


def test_uniform_placement_in_a_trapezoid():
    # one strongly trapezoidal cell: nodes (0,0), (1,0), (0.8,1), (0.2,0.3)
    mesh = dict(xy=np.array([[0.0, 0.0], [1.0, 0.0], [0.8, 1.0], [0.2, 0.3]]),
                quad=np.array([[0, 1, 2, 3]], np.int32),
                nbr=np.array([["specular"] * 4], dtype=object))
    st = dict(n=1e20, u=(0.0, 0.0, 0.0), T=300.0)
    case = W._case(dim=2, h=(1.0, 1.0, 1.0), regions=[((-1, -1, 0, 2, 2, 1), st)], F_N=1e20 * 0.47 / 40000,
                   dt_G=1e-6, T_sigma=300.0, seed=12, capacity=50000, mesh=mesh)
    o = Oracle(GAS, case)
    o.init_particles()
    x = o.get_state()["x"][:, :2]
    d1, d2 = mesh["xy"][2] - mesh["xy"][0], mesh["xy"][3] - mesh["xy"][1]
    area = 0.5 * abs(d1[0] * d2[1] - d1[1] * d2[0])
    assert abs(o.get_cells(0)["vol"][0] - area) < 1e-15
    assert abs(len(x) - 1e20 * area / case["F_N"]) <= 1.0
    # counts in an 8 x 8 box grid against the area of the quad inside each box (by a fine
    # point lattice), chi-square
    g = np.linspace(0.0, 1.0, 2001)
    gx, gy = np.meshgrid(0.5 * (g[1:] + g[:-1]), 0.5 * (g[1:] + g[:-1]))
    pts = np.stack([gx.ravel(), gy.ravel()], axis=1)
    inside = _inside(mesh, np.zeros(len(pts), np.int64), pts, tol=0.0)
    bins = np.linspace(0, 1, 9)
    ref, _, _ = np.histogram2d(pts[inside, 0], pts[inside, 1], bins=[bins, bins])
    obs, _, _ = np.histogram2d(x[:, 0], x[:, 1], bins=[bins, bins])
    keep = ref > 0.02 * ref.max()
    exp = ref[keep] / ref[keep].sum() * obs[keep].sum()
    chi2 = ((obs[keep] - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3, chi2
    assert obs[~keep].sum() <= 0.03 * len(x)


def test_free_molecular_cylinder_on_an_o_grid():
    T, Tw, s = 300.0, 500.0, 1.0
    case = W.free_molecular_ogrid(s=s, T=T, T_w=Tw)
    o = Oracle(GAS, case)
    o.init_particles()
    ns, R = case["n_surf"], case["body_r"]
    th = np.pi * np.arange(ns + 1) / ns
    area = 2 * R * (th[1:] - th[:-1])
    n, U = case["inflow"]["n"], case["inflow"]["u"][0]
    qd = 0.5 * n * W.ARGON["m"] * U * U
    prev = np.zeros((ns, 7))
    rows, cds = [], []
    batches, steps = 8, 250
    for _ in range(batches):
        o.step(steps)
        S = o.surface_sums(0)
        d, prev = S - prev, S
        t = steps * case["dt_G"]
        rows.append(np.stack([-d[:, 1] / (area * t), d[:, 2] / (area * t), d[:, 3] / (area * t)], axis=1))
        cds.append(d[:, 4].sum() / t / (qd * 2 * R))
    rows, cds = np.array(rows), np.array(cds)
    ref = element_means(n, U, T, Tw, ns, False)
    mean, se = rows.mean(axis=0), rows.std(axis=0, ddof=1) / math.sqrt(batches)
    # the polygon's facets stand for the circle: a bias of O((pi / n_theta)^2), below the noise
    assert np.all(np.abs(mean - ref) < 5.0 * se + 5e-3 * np.abs(ref)), (mean, ref)
    assert np.all(se[:3, 0] < 0.05 * ref[:3, 0])
    cd_ref = cd_closed(s, T, Tw, False)
    assert abs(cds.mean() - cd_ref) < 5.0 * cds.std(ddof=1) / math.sqrt(batches) + 5e-3 * cd_ref


def test_gas_at_rest_on_an_o_grid_stays_uniform():
    """A gas at rest around a wall at its own temperature is in equilibrium: the oblique
    inflow edges of the outer circle must feed exactly the one-way flux that leaves, so the
    density and temperature stay those of the gas in every ring of cells, and the wall
    feels p = n k T with no shear or heat flux."""
    T = 300.0
    case = W.free_molecular_ogrid(s=0.0, T=T, T_w=T, n_surf=4)
    o = Oracle(GAS, case)
    o.init_particles()
    o.step(1500)
    m = o.sample_moments(0, 0)
    vol = o.get_cells(0)["vol"]
    n_ring = (m["n"] * vol).reshape(-1, 72).sum(axis=1) / vol.reshape(-1, 72).sum(axis=1)
    T_ring = (m["T"] * m["n"] * vol).reshape(-1, 72).sum(axis=1) / (m["n"] * vol).reshape(-1, 72).sum(axis=1)
    n0 = case["inflow"]["n"]
    assert np.all(np.abs(n_ring[4:] / n0 - 1.0) < 0.02), n_ring / n0
    assert abs((m["n"] * vol).sum() / vol.sum() / n0 - 1.0) < 0.005
    assert np.all(np.abs(T_ring[4:] / T - 1.0) < 0.02), T_ring / T
    r = o.surface_sample(0)
    p0 = n0 * W.K_BOLTZMANN * T
    assert np.all(np.abs(r["p"] / p0 - 1.0) < 0.05), r["p"] / p0
    assert np.all(np.abs(r["tau"]) < 0.05 * p0)


@pytest.mark.parametrize("what", ["clockwise", "node", "nbr", "code", "sphere"])
def test_bad_meshes_are_rejected(what):
    case = W.mesh_twin(_base())
    m = {k: np.array(v, copy=True) for k, v in case["mesh"].items()}
    if what == "clockwise":
        m["quad"][5] = m["quad"][5][::-1]
    elif what == "node":
        m["quad"][2, 1] = len(m["xy"]) + 3
    elif what == "nbr":
        m["nbr"][0, 1] = 7                       # not a neighbour of cell 0 across edge 1
    elif what == "code":
        m["nbr"][0, 0] = -9
    else:
        case["body"] = "sphere"
    case["mesh"] = m
    with pytest.raises(OracleError):
        Oracle(GAS, case)


def test_mesh_cell_length_sets_the_adaptive_step():
    """Eq. 25-26 on a jittered mesh: the next global step is the smallest L_k / (|U_k| +
    sqrt(gamma R T_k)) over the cells with N >= 2, where L_k is the quad's area over its
    longest edge computed here from the node coordinates, and U_k, T_k are the cells' Step 3
    moments (the trace's pre-collision sums and temperature)."""
    case = _base(seed=6)
    case["bc"] = ("specular",) * 4 + ("outflow",) * 2
    mc = W.mesh_twin(case, jitter=0.2)
    mc["adapt_dt"] = True
    o = Oracle(GAS, mc, trace=True)
    o.init_particles()
    o.step(1)
    tr = o.trace(0)
    xy, quad = mc["mesh"]["xy"], mc["mesh"]["quad"]
    P = xy[quad]                                           # (cells, 4, 2)
    e = np.roll(P, -1, axis=1) - P
    longest = np.hypot(e[..., 0], e[..., 1]).max(axis=1)
    d1, d2 = P[:, 2] - P[:, 0], P[:, 3] - P[:, 1]
    area = 0.5 * np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    np.testing.assert_allclose(o.get_cells(0)["vol"], area * mc["h"][2], rtol=1e-12)
    act = (tr["n"] >= 2) & (tr["T"] > 0)
    U = tr["pre_sum"][act, :3] / tr["n"][act, None]
    R = W.K_BOLTZMANN / W.ARGON["m"]
    dtc = (area / longest)[act] / (np.linalg.norm(U, axis=1) + np.sqrt(W.ARGON["gamma"] * R * tr["T"][act]))
    assert abs(o.step_dt(0)[0] / dtc.min() - 1.0) < 1e-12
