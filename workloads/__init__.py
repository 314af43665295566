"""Synthetic workloads shaped like the paper's test cases (Sec. 4), as plain parameters.

This module is the only code shared by the GPU product path, the CPU oracle and the
tests.  It holds inputs only -- case parameters written as numbers, and seeded numpy
generators for imported initial states -- and none of the method's arithmetic.

Derived constants are written out as literals; the comments say how they follow from the
paper's gas model (Sec. 4: argon VHS, d_ref = 4.17e-10 m, T_ref = 273 K, omega = 0.81,
mu_ref = 2.117e-5 Pa s) and mean free path (Eq. 33).  The pin tests recompute them with
the oracle's own gas functions.

Case dictionaries use string codes ("outflow", "specular", "inflow"; body "none",
"cylinder", "sphere"); each binding maps them onto its own enums.
"""
from __future__ import annotations

import math

import numpy as np

K_BOLTZMANN = 1.380649e-23

# Argon VHS gas of Sec. 4.  The paper gives no molecular mass; 6.63e-26 kg is argon's.
ARGON = dict(m=6.63e-26, d_ref=4.17e-10, T_ref=273.0, omega=0.81, mu_ref=2.117e-5,
             Pr=2.0 / 3.0, gamma=5.0 / 3.0)
R_ARGON = K_BOLTZMANN / ARGON["m"]          # 208.2426847662142 J/(kg K)

# Hypersonic freestream used by the cylinder and sphere workloads: Ma 10 at 200 K.
#   a_inf = sqrt(gamma R T) = 263.4658009218744 m/s, U_inf = 10 a_inf
#   n_inf from Eq. 33 with lambda = 0.01 m (Kn = 0.01 on D = 1 m) at 200 K
T_INF = 200.0
U_INF = 2634.658009218744
N_INF = 1.1753626818345325e20
U_PLUS_A_INF = 2898.1238101406184          # U_inf + a_inf, sets dt_G = dx / (U + a)
T_STAG = 6866.666666666667                 # T_inf (1 + (gamma-1)/2 Ma^2)

# Sod tube, Table 1 row Kn = 1e-4: rho_up = 8.58174e-4, rho_down = 1.07272e-4 kg/m^3
SOD_N_LEFT = 1.2943800904977375e22         # rho / m
SOD_N_RIGHT = 1.617978883861237e21
SOD_T_LEFT, SOD_T_RIGHT = 273.0, 218.4
SOD_A_LEFT = 307.81556420789946            # sqrt(gamma R T_left)

# 0-D relaxation batch state (the cylinder case of Sec. 4.2 at 273 K)
RELAX_N, RELAX_T = 1.29438e20, 273.0

# Planar jets: exit Mach 1 from T0 = 300 K -> T_e = 225 K, U_e = a_e.
JET_T0, JET_TE = 300.0, 225.0
JET_UE = 279.4476816639035
JET_N_LAMBDA = 1.2190715036564413e18       # n * lambda at T_e from Eq. 33 (m^-2)


def _case(**kw):
    base = dict(dim=2, nx=1, ny=1, nz=1, lo=(0.0, 0.0, 0.0), h=(1.0, 1.0, 1.0),
                bc=("outflow",) * 6, inflow=dict(n=0.0, u=(0.0, 0.0, 0.0), T=1.0),
                slot_lo=(0.0, 0.0, 0.0), slot_hi=(0.0, 0.0, 0.0),
                body="none", body_c=(0.0, 0.0, 0.0), body_r=0.0, body_T=0.0,
                regions=[], F_N=1.0, dt_G=0.0, T_sigma=273.0, dt_over_tau=None,
                seed=1, n_steady=1 << 40, capacity=0, n_surf=0)
    base.update(kw)
    return base


def gas():
    return dict(ARGON)


def sod_1d(seed=1, ncells=200, ppc_left=160, n_steady=1 << 40):
    """1-D Sod tube on [0, 1] m: left state of Table 1 (Kn = 1e-4), right state with
    rho ratio 8 and T ratio 1.25; specular end walls; dt = 0.5 dx / a_left."""
    h = 1.0 / ncells
    fn = SOD_N_LEFT * h / ppc_left          # V_cell = h * 1 m^2
    dt = 0.5 * h / SOD_A_LEFT
    regions = [((0.0, 0.0, 0.0, 0.5, 1.0, 1.0), dict(n=SOD_N_LEFT, u=(0.0, 0.0, 0.0), T=SOD_T_LEFT)),
               ((0.5, 0.0, 0.0, 1.0, 1.0, 1.0), dict(n=SOD_N_RIGHT, u=(0.0, 0.0, 0.0), T=SOD_T_RIGHT))]
    n_est = ncells // 2 * ppc_left + ncells // 2 * (ppc_left // 8)
    return _case(dim=1, nx=ncells, h=(h, 1.0, 1.0),
                 bc=("specular", "specular", "outflow", "outflow", "outflow", "outflow"),
                 regions=regions, F_N=fn, dt_G=dt, T_sigma=SOD_T_LEFT, seed=seed,
                 n_steady=n_steady, capacity=int(n_est * 1.1) + 64)


def sod_steps(ncells=200):
    """Steps to t = 0.2 L / a_left at dt = 0.5 dx / a_left."""
    return int(round(0.2 / (0.5 / ncells)))


def relax_0d(ncells=4096, ppc=1000, seed=2, r_seed=7, n_steady=1 << 40):
    """0-D batch: independent homogeneous cells, each with its own dt/tau drawn
    log-uniform in [0.01, 100]."""
    rng = np.random.default_rng(r_seed)
    r = 10.0 ** (-2.0 + 4.0 * rng.random(ncells))
    return _case(dim=0, nx=ncells, h=(1.0, 1.0, 1.0),
                 regions=[((0, 0, 0, 0, 0, 0), dict(n=RELAX_N, u=(0.0, 0.0, 0.0), T=RELAX_T))],
                 F_N=RELAX_N * 1.0 / ppc, T_sigma=1.5 * RELAX_T, dt_over_tau=r, seed=seed,
                 n_steady=n_steady, capacity=ncells * ppc)


def relax_0d_state(case, ppc=1000, tx_over_t=1.5, skew=0.05, state_seed=11):
    """Initial 0-D state: bi-Maxwellian with T_x = 2 T_y = 2 T_z (mean T kept) and a
    cubic skew in v_x, v_x = sqrt(R T_x) (x + s (x^2 - 1)) / sqrt(1 + 2 s^2), x ~ N(0,1);
    per-cell mean velocity removed.  Returns (v[N,3], cell[N], id[N])."""
    rng = np.random.default_rng(state_seed)
    nc = case["nx"]
    T = RELAX_T
    tx = tx_over_t * T
    ty = (3.0 * T - tx) / 2.0
    x = rng.standard_normal((nc, ppc))
    vx = math.sqrt(R_ARGON * tx) * (x + skew * (x * x - 1.0)) / math.sqrt(1.0 + 2.0 * skew * skew)
    vy = math.sqrt(R_ARGON * ty) * rng.standard_normal((nc, ppc))
    vz = math.sqrt(R_ARGON * ty) * rng.standard_normal((nc, ppc))
    v = np.stack([vx, vy, vz], axis=-1)
    v -= v.mean(axis=1, keepdims=True)
    cell = np.repeat(np.arange(nc, dtype=np.int32), ppc)
    ids = np.arange(nc * ppc, dtype=np.int64)
    return v.reshape(-1, 3).copy(), cell, ids


def cylinder_2d(nx=800, ny=600, ppc=30, seed=1, n_steady=10000, cap_factor=1.6, n_surf=90):
    """Ma 10 argon flow over a cylinder of diameter D = 1 m at (2.5, 3) in an 8 x 6 m box;
    diffuse wall at 500 K; freestream inflow on -x, -y, +y; vacuum outflow on +x; the wall
    sampled in n_surf elements of polar angle (2 degrees each by default)."""
    h = 8.0 / nx
    assert abs(6.0 / ny - h) < 1e-12
    fn = N_INF * h * h / ppc
    st = dict(n=N_INF, u=(U_INF, 0.0, 0.0), T=T_INF)
    return _case(dim=2, nx=nx, ny=ny, h=(h, h, 1.0),
                 bc=("inflow", "outflow", "inflow", "inflow", "outflow", "outflow"),
                 inflow=st, body="cylinder", body_c=(2.5, 3.0, 0.0), body_r=0.5, body_T=500.0,
                 regions=[((0.0, 0.0, 0.0, 8.0, 6.0, 1.0), st)], F_N=fn,
                 dt_G=h / U_PLUS_A_INF, T_sigma=T_STAG, seed=seed, n_steady=n_steady,
                 capacity=int(nx * ny * ppc * cap_factor) + 4096, n_surf=n_surf)


def sphere_3d(nx=240, ny=160, nz=160, ppc=15, seed=1, n_steady=5000, cap_factor=1.6, n_surf=45):
    """Ma 10 argon flow over a sphere of diameter D = 1 m at (2, 2, 2) in a 6 x 4 x 4 m
    box; diffuse wall at 500 K; inflow on -x and the four lateral faces; outflow +x; the
    wall sampled in n_surf zones of polar angle (4 degrees each by default)."""
    h = 6.0 / nx
    assert abs(4.0 / ny - h) < 1e-12 and abs(4.0 / nz - h) < 1e-12
    fn = N_INF * h ** 3 / ppc
    st = dict(n=N_INF, u=(U_INF, 0.0, 0.0), T=T_INF)
    return _case(dim=3, nx=nx, ny=ny, nz=nz, h=(h, h, h),
                 bc=("inflow", "outflow", "inflow", "inflow", "inflow", "inflow"),
                 inflow=st, body="sphere", body_c=(2.0, 2.0, 2.0), body_r=0.5, body_T=500.0,
                 regions=[((0.0, 0.0, 0.0, 6.0, 4.0, 4.0), st)], F_N=fn,
                 dt_G=h / U_PLUS_A_INF, T_sigma=T_STAG, seed=seed, n_steady=n_steady,
                 capacity=int(nx * ny * nz * ppc * cap_factor) + 4096, n_surf=n_surf)


def free_molecular_body(body="cylinder", s=1.0, T=300.0, T_w=500.0, n=1.0e13, cells=40, ppc=20,
                        R=0.3, n_surf=12, seed=7):
    """A drifting argon stream past a diffuse body at T_w with (practically) no collisions:
    at n = 1e13 m^-3 the mean free path is ~130 m against a 2 m box, so the wall sees the
    undisturbed freestream (free-molecular flow).  Box [0,2]^dim with `cells` cells per
    axis, body of radius R at the centre, stream along +x with speed ratio
    s = U / sqrt(2 k T / m); every face is a freestream face (it injects the stream's
    one-way flux and removes leaving particles), so the box holds the undisturbed stream
    everywhere; the box starts at the freestream state and every step is sampled."""
    dim = 2 if body == "cylinder" else 3
    h = 2.0 / cells
    U = s * math.sqrt(2.0 * R_ARGON * T)
    st = dict(n=n, u=(U, 0.0, 0.0), T=T)
    vol = h ** dim
    bc = ("inflow",) * 4 + (("inflow", "inflow") if dim == 3 else ("outflow", "outflow"))
    return _case(dim=dim, nx=cells, ny=cells, nz=cells if dim == 3 else 1, h=(h, h, h if dim == 3 else 1.0),
                 bc=bc, inflow=st, body=body, body_c=(1.0, 1.0, 1.0 if dim == 3 else 0.0), body_r=R,
                 body_T=T_w, regions=[((0.0, 0.0, 0.0, 2.0, 2.0, 2.0 if dim == 3 else 1.0), st)],
                 F_N=n * vol / ppc, dt_G=0.5 * h / (U + 3.0 * math.sqrt(R_ARGON * T)), T_sigma=T,
                 seed=seed, n_steady=0, capacity=int(cells ** dim * ppc * 2) + 4096, n_surf=n_surf)


def jets_2d(n_jets=32, grids=((200, 100), (400, 200), (800, 400)), batch_seed=2026,
            seed0=100, n_steady=2500, cap_factor=0.5):
    """Ragged batch of planar jets into vacuum: exit Mach 1 slot of height H/5 centred
    on the left wall of a 2H x H box (H = 1 m), exit Kn log-uniform in [1e-3, 1e-1] on
    the slot height, 20-40 particles per cell at the exit density; all other walls
    vacuum outflow; the box starts empty."""
    rng = np.random.default_rng(batch_seed)
    cases = []
    for j in range(n_jets):
        nx, ny = grids[int(rng.integers(len(grids)))]
        kn = 10.0 ** rng.uniform(-3.0, -1.0)
        ppc = int(rng.integers(20, 41))
        H = 1.0
        h = H / ny
        hs = H / 5.0
        ne = JET_N_LAMBDA / (kn * hs)
        st = dict(n=ne, u=(JET_UE, 0.0, 0.0), T=JET_TE)
        cases.append(_case(dim=2, nx=nx, ny=ny, h=(h, h, 1.0),
                           bc=("inflow", "outflow", "outflow", "outflow", "outflow", "outflow"),
                           inflow=st, slot_lo=(0.0, 0.4 * H, 0.0), slot_hi=(0.0, 0.6 * H, 0.0),
                           F_N=ne * h * h / ppc, dt_G=h / (2.0 * JET_UE), T_sigma=JET_T0,
                           seed=seed0 + j, n_steady=n_steady,
                           capacity=int(nx * ny * ppc * cap_factor) + 4096))
    return cases


# ------------------------------------------------------------------------------------
# Body-fitted quadrilateral meshes (2-D).  A mesh is a dict of numpy arrays: xy (nodes, 2),
# quad (cells, 4) node ids counter-clockwise, nbr (cells, 4) the cell across edge j
# (node j -> node j+1) or an edge code string ("outflow", "inflow", "wall", "specular")
# that each binding maps onto its own enum.
# ------------------------------------------------------------------------------------

# Ma 5 argon cylinder of Sec. 4.2: R = 1 m, T = 273 K, U = 1537.44 m/s, wall at 273 K,
# n = 1.29438e20 m^-3 (Kn = 0.01) or 1.29438e19 m^-3 (Kn = 0.1).
CYL5_N = 1.29438e20
CYL5_T = 273.0
CYL5_U = 1537.44
CYL5_A = 307.81556420789946       # sqrt(gamma R T) at 273 K


def _edge_codes(nbr_int, codes):
    """Object array of neighbours with the boundary entries replaced by their code names."""
    out = np.empty(nbr_int.shape, dtype=object)
    for idx, v in np.ndenumerate(nbr_int):
        out[idx] = int(v) if v >= 0 else codes[int(v)]
    return out


def quad_box_mesh(nx, ny, lo=(0.0, 0.0), h=(1.0, 1.0), sides=("outflow",) * 4, jitter=0.0,
                  jitter_seed=5):
    """Structured quads of the box lo + [0, nx h0] x [0, ny h1], cells x-fastest like the
    grid's, nodes at lo + (i h0, j h1); sides = codes of the -x, +x, -y, +y boundaries.
    jitter > 0 moves every interior node by a seeded uniform offset of up to jitter * h
    per axis (kept below 0.25 so every quad stays convex)."""
    assert 0.0 <= jitter < 0.25
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    x = lo[0] + ii * h[0]
    y = lo[1] + jj * h[1]
    if jitter > 0.0:
        rng = np.random.default_rng(jitter_seed)
        inner = (ii > 0) & (ii < nx) & (jj > 0) & (jj < ny)
        x = np.where(inner, x + jitter * h[0] * rng.uniform(-1.0, 1.0, x.shape), x)
        y = np.where(inner, y + jitter * h[1] * rng.uniform(-1.0, 1.0, y.shape), y)
    xy = np.stack([x.reshape(-1), y.reshape(-1)], axis=1)
    node = lambda i, j: i + (nx + 1) * j
    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ci, cj = ci.reshape(-1), cj.reshape(-1)
    quad = np.stack([node(ci, cj), node(ci + 1, cj), node(ci + 1, cj + 1), node(ci, cj + 1)], axis=1)
    cell = lambda i, j: i + nx * j
    nbr = np.stack([np.where(cj > 0, cell(ci, cj - 1), -3),
                    np.where(ci < nx - 1, cell(ci + 1, cj), -2),
                    np.where(cj < ny - 1, cell(ci, cj + 1), -4),
                    np.where(ci > 0, cell(ci - 1, cj), -1)], axis=1)
    codes = {-1: sides[0], -2: sides[1], -3: sides[2], -4: sides[3]}
    return dict(xy=xy, quad=quad.astype(np.int32), nbr=_edge_codes(nbr, codes))


def o_grid_mesh(n_theta=180, R=1.0, first=0.001, growth=1.1, r_out=3.0, inner="wall",
                outer="inflow"):
    """O-grid around a circle of radius R at the origin (Sec. 4.2: uniform circumferential
    nodes, first layer `first`, radial growth `growth`): layers are added until the
    outer radius reaches r_out.  Cell (i, j) lies between angles 2 pi i / n_theta and
    2 pi (i + 1) / n_theta and radii r_j, r_j+1; cells angle-fastest.  Edge 0 is the ray
    at angle i, edge 1 the outer arc, edge 2 the ray at i + 1, edge 3 the inner arc."""
    r = [R]
    d = first
    while r[-1] < r_out:
        r.append(r[-1] + d)
        d *= growth
    r = np.asarray(r)
    nr = len(r) - 1
    th = 2.0 * np.pi * np.arange(n_theta) / n_theta
    xy = np.stack([np.outer(r, np.cos(th)).reshape(-1), np.outer(r, np.sin(th)).reshape(-1)], axis=1)
    node = lambda i, j: (i % n_theta) + n_theta * j
    ci, cj = np.meshgrid(np.arange(n_theta), np.arange(nr), indexing="xy")
    ci, cj = ci.reshape(-1), cj.reshape(-1)
    quad = np.stack([node(ci, cj), node(ci, cj + 1), node(ci + 1, cj + 1), node(ci + 1, cj)], axis=1)
    cell = lambda i, j: (i % n_theta) + n_theta * j
    nbr = np.stack([cell(ci - 1 + n_theta, cj),
                    np.where(cj < nr - 1, cell(ci, cj + 1), -2),
                    cell(ci + 1, cj),
                    np.where(cj > 0, cell(ci, cj - 1), -1)], axis=1)
    codes = {-1: inner, -2: outer}
    return dict(xy=xy, quad=quad.astype(np.int32), nbr=_edge_codes(nbr, codes), radii=r)


def mesh_twin(case, jitter=0.0):
    """The 2-D grid case `case` (no body) as a body-fitted quad mesh of the same cells,
    boundaries and parameters."""
    assert case["dim"] == 2 and case["body"] == "none"
    m = quad_box_mesh(case["nx"], case["ny"], lo=case["lo"][:2], h=case["h"][:2],
                      sides=tuple(case["bc"][:4]), jitter=jitter)
    out = dict(case)
    out["mesh"] = m
    return out


def cylinder_ogrid(n_theta=180, first=0.001, growth=1.1, r_out=3.0, kn=0.01, ppc_outer=500,
                   seed=1, n_steady=1 << 40, cap_factor=1.5, n_surf=90, adapt_dt=False):
    """Ma 5 argon flow past the unit cylinder of Sec. 4.2 on its O-grid (wall at 273 K,
    freestream on the outer circle); F_N puts ppc_outer particles in the outermost cells at
    the freestream density; dt_G = first / (U + a) (the Eq. 26 value at freestream).  The
    wall is sampled in n_surf bands of polar angle."""
    m = o_grid_mesh(n_theta=n_theta, first=first, growth=growth, r_out=r_out)
    r = m["radii"]
    n = CYL5_N * (0.01 / kn)
    st = dict(n=n, u=(CYL5_U, 0.0, 0.0), T=CYL5_T)
    outer_area = 0.5 * (r[-1] ** 2 - r[-2] ** 2) * (2.0 * np.pi / n_theta)
    fn = n * outer_area / ppc_outer
    total = n * np.pi * (r[-1] ** 2 - r[0] ** 2) / fn
    big = r[-1] + 1.0
    return _case(dim=2, h=(1.0, 1.0, 1.0), inflow=st, body="cylinder", body_c=(0.0, 0.0, 0.0),
                 body_r=1.0, body_T=CYL5_T, regions=[((-big, -big, 0.0, big, big, 1.0), st)],
                 F_N=fn, dt_G=first / (CYL5_U + CYL5_A), T_sigma=CYL5_T * (1.0 + 25.0 / 3.0), seed=seed,
                 n_steady=n_steady, capacity=int(total * cap_factor) + 4096, n_surf=n_surf,
                 adapt_dt=adapt_dt, mesh=m)


def free_molecular_ogrid(s=1.0, T=300.0, T_w=500.0, n=1.0e13, R=0.3, r_out=1.0, n_theta=72,
                         first=0.02, growth=1.1, total=16000, n_surf=6, seed=9):
    """free_molecular_body's cylinder on a body-fitted O-grid: a diffuse cylinder of radius R
    at T_w inside a circle of radius r_out whose edges are freestream edges, filled with the
    undisturbed stream (speed ratio s along +x); about `total` particles; every step
    sampled."""
    m = o_grid_mesh(n_theta=n_theta, R=R, first=first, growth=growth, r_out=r_out)
    r = m["radii"]
    U = s * math.sqrt(2.0 * R_ARGON * T)
    st = dict(n=n, u=(U, 0.0, 0.0), T=T)
    fn = n * math.pi * (r[-1] ** 2 - r[0] ** 2) / total
    big = r[-1] + 1.0
    return _case(dim=2, h=(1.0, 1.0, 1.0), inflow=st, body="cylinder", body_c=(0.0, 0.0, 0.0),
                 body_r=R, body_T=T_w, regions=[((-big, -big, 0.0, big, big, 1.0), st)], F_N=fn,
                 dt_G=0.5 * first / (U + 3.0 * math.sqrt(R_ARGON * T)), T_sigma=T, seed=seed,
                 n_steady=0, capacity=int(2 * total) + 4096, n_surf=n_surf, mesh=m)


def ogrid_batch(n_cases=12, seed0=300):
    """The three O-grid runs of Sec. 4.2, repeated with different seeds: mesh1 (first layer
    1 mm, growth 1.1) at Kn 0.01, mesh2 (growth 1.05) at Kn 0.01 and mesh1 at Kn 0.1, all
    with outer radius 3 R; cases cycle through the three."""
    kinds = [dict(growth=1.1, kn=0.01), dict(growth=1.05, kn=0.01), dict(growth=1.1, kn=0.1)]
    return [cylinder_ogrid(seed=seed0 + i, **kinds[i % 3]) for i in range(n_cases)]


def hex_box_mesh(nx, ny, nz, lo=(0.0, 0.0, 0.0), h=(1.0, 1.0, 1.0), sides=("outflow",) * 6, jitter=0.0,
                 jitter_seed=5):
    """Structured hexahedra of the box lo + [0, nx h0] x [0, ny h1] x [0, nz h2], cells
    x-fastest like the grid's; sides = codes of the -x, +x, -y, +y, -z, +z boundaries.  Nodes
    0-3 of a cell are its bottom (-z) face counter-clockwise seen from above, 4-7 the top.
    jitter > 0 shifts interior node planes (whole i, j or k planes by up to jitter * h, so
    every face stays planar)."""
    assert 0.0 <= jitter < 0.25
    rng = np.random.default_rng(jitter_seed)
    coords = []
    for n, l0, hh in ((nx, lo[0], h[0]), (ny, lo[1], h[1]), (nz, lo[2], h[2])):
        c = l0 + np.arange(n + 1) * hh
        if jitter > 0.0:
            c[1:-1] += jitter * hh * rng.uniform(-1.0, 1.0, n - 1)
        coords.append(c)
    X, Y, Z = np.meshgrid(coords[0], coords[1], coords[2], indexing="ij")
    node = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
    xy = np.zeros(((nx + 1) * (ny + 1) * (nz + 1), 3))
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    xy[node(ii, jj, kk).reshape(-1)] = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = (a.transpose(2, 1, 0).reshape(-1) for a in (ci, cj, ck))      # x-fastest
    quad = np.stack([node(ci, cj, ck), node(ci + 1, cj, ck), node(ci + 1, cj + 1, ck), node(ci, cj + 1, ck),
                     node(ci, cj, ck + 1), node(ci + 1, cj, ck + 1), node(ci + 1, cj + 1, ck + 1),
                     node(ci, cj + 1, ck + 1)], axis=1)
    cell = lambda i, j, k: i + nx * (j + ny * k)
    # faces: bottom (-z), top (+z), -y, +x, +y, -x
    nbr = np.stack([np.where(ck > 0, cell(ci, cj, ck - 1), -15),
                    np.where(ck < nz - 1, cell(ci, cj, ck + 1), -16),
                    np.where(cj > 0, cell(ci, cj - 1, ck), -13),
                    np.where(ci < nx - 1, cell(ci + 1, cj, ck), -12),
                    np.where(cj < ny - 1, cell(ci, cj + 1, ck), -14),
                    np.where(ci > 0, cell(ci - 1, cj, ck), -11)], axis=1)
    codes = {-11: sides[0], -12: sides[1], -13: sides[2], -14: sides[3], -15: sides[4], -16: sides[5]}
    return dict(xy=xy, quad=quad.astype(np.int32), nbr=_edge_codes(nbr, codes))


def mesh_twin_3d(case, jitter=0.0):
    """The 3-D grid case `case` (no body) as a hexahedral mesh of the same cells."""
    assert case["dim"] == 3 and case["body"] == "none"
    m = hex_box_mesh(case["nx"], case["ny"], case["nz"], lo=case["lo"], h=case["h"], sides=tuple(case["bc"]),
                     jitter=jitter)
    out = dict(case)
    out["mesh"] = m
    return out


def sphere_shell_mesh(R=1.0, r_out=3.0, n_r=20, growth=1.1, n_theta=18, n_phi=36, inner="wall",
                      outer="inflow", axis="pole_z"):
    """Hexahedra between spheres of radius R and r_out: radii growing by `growth` from the
    wall, n_theta bands of polar angle from the +z axis and n_phi of azimuth.  The faces of
    such cells are planar (equal-radius chords at two latitudes are parallel).  Cells touching
    a pole collapse one face to a segment; that face is marked specular and is never crossed.
    Cells: azimuth fastest, then polar band, then radius."""
    q = growth ** np.arange(n_r)
    r = R + (r_out - R) * np.concatenate([[0.0], np.cumsum(q) / q.sum()])
    th = np.pi * np.arange(n_theta + 1) / n_theta
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    # nodes: one per (r, theta, phi), the poles shared
    ids = {}
    xyz = []
    def nid(kr, kt, kp):
        key = (kr, kt, 0 if kt in (0, n_theta) else kp % n_phi)
        if key not in ids:
            ids[key] = len(xyz)
            rr, t, p = r[kr], th[kt], ph[key[2]]
            xyz.append((rr * np.sin(t) * np.cos(p), rr * np.sin(t) * np.sin(p), rr * np.cos(t)))
        return ids[key]
    quad, cells = [], {}
    for kr in range(n_r):
        for kt in range(n_theta):
            for kp in range(n_phi):
                cells[(kr, kt, kp)] = len(quad)
                # bottom face = inner radius, counter-clockwise seen from outside the sphere
                # (from larger r): (t, p), (t, p+1), (t+1, p+1), (t+1, p) ... oriented below
                a = [nid(kr, kt, kp), nid(kr, kt + 1, kp), nid(kr, kt + 1, kp + 1), nid(kr, kt, kp + 1)]
                b = [nid(kr + 1, kt, kp), nid(kr + 1, kt + 1, kp), nid(kr + 1, kt + 1, kp + 1), nid(kr + 1, kt, kp + 1)]
                quad.append(a + b)
    # neighbours per face from shared node sets
    face_nodes = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]
    owner = {}
    nbr = np.zeros((len(quad), 6), dtype=object)
    for c, nodes in enumerate(quad):
        for f, fn in enumerate(face_nodes):
            key = frozenset(nodes[j] for j in fn)
            if len(key) < 3:
                nbr[c, f] = "specular"          # collapsed at a pole
                continue
            if key in owner:
                c2, f2 = owner.pop(key)
                nbr[c, f] = c2
                nbr[c2, f2] = c
            else:
                owner[key] = (c, f)
    for (c, f) in owner.values():
        kr = c // (n_theta * n_phi)
        nbr[c, f] = inner if (f == 0 and kr == 0) else outer
    return dict(xy=np.array(xyz), quad=np.array(quad, dtype=np.int32), nbr=nbr, radii=r)


def free_molecular_sphere_mesh(s=1.0, T=300.0, T_w=500.0, n=1.0e13, R=0.35, r_out=1.0, n_r=8, n_theta=12,
                               n_phi=24, total=20000, n_surf=4, seed=13):
    """free_molecular_body's sphere on a body-fitted hexahedral shell (planar faces; poles on
    the z axis, the stream along +x): every outer face a freestream face, every step sampled."""
    m = sphere_shell_mesh(R=R, r_out=r_out, n_r=n_r, n_theta=n_theta, n_phi=n_phi)
    U = s * math.sqrt(2.0 * R_ARGON * T)
    st = dict(n=n, u=(U, 0.0, 0.0), T=T)
    fn = n * 4.0 / 3.0 * math.pi * (r_out ** 3 - R ** 3) / total
    dr = m["radii"][1] - m["radii"][0]
    big = r_out + 1.0
    return _case(dim=3, h=(1.0, 1.0, 1.0), inflow=st, body="sphere", body_r=R, body_T=T_w,
                 regions=[((-big, -big, -big, big, big, big), st)], F_N=fn,
                 dt_G=0.5 * dr / (U + 3.0 * math.sqrt(R_ARGON * T)), T_sigma=T, seed=seed, n_steady=0,
                 capacity=int(2 * total) + 4096, n_surf=n_surf, mesh=m)


# Ma 10 argon sphere of Sec. 4.4: R = 1 m, rho = 5.5e-6 kg/m^3 (n = rho / m), T = 65 K,
# U = 1501.11 m/s, wall at 302 K.
SPH10_N = 5.5e-6 / 6.63e-26
SPH10_T = 65.0
SPH10_U = 1501.11
SPH10_A = 150.12329153025936               # sqrt(gamma R T) at 65 K


def sphere_hex(n_phi=72, n_theta=36, n_r=76, r_out=4.0, growth=1.05, ppc_outer=400, seed=1,
               n_steady=1 << 40, cap_factor=1.5, n_surf=36):
    """The Sec. 4.4 sphere on a body-fitted hexahedral shell: n_phi x n_theta x n_r cells
    (72 x 36 x 76 = 196,992, the paper's count is 197,248), radii from R = 1 m growing by
    `growth` to r_out; the pole axis is z, the stream along +x; diffuse wall at 302 K;
    F_N puts ppc_outer particles in an outermost equatorial cell; dt_G = first layer /
    (U + a)."""
    m = sphere_shell_mesh(R=1.0, r_out=r_out, n_r=n_r, growth=growth, n_theta=n_theta, n_phi=n_phi)
    r = m["radii"]
    st = dict(n=SPH10_N, u=(SPH10_U, 0.0, 0.0), T=SPH10_T)
    dth, dph = np.pi / n_theta, 2.0 * np.pi / n_phi
    outer = (r[-1] ** 3 - r[-2] ** 3) / 3.0 * dph * (np.cos(0.5 * np.pi - 0.5 * dth) - np.cos(0.5 * np.pi + 0.5 * dth))
    fn = SPH10_N * outer / ppc_outer
    total = SPH10_N * 4.0 / 3.0 * np.pi * (r[-1] ** 3 - r[0] ** 3) / fn
    big = r[-1] + 1.0
    return _case(dim=3, h=(1.0, 1.0, 1.0), inflow=st, body="sphere", body_r=1.0, body_T=302.0,
                 regions=[((-big, -big, -big, big, big, big), st)], F_N=fn,
                 dt_G=(r[1] - r[0]) / (SPH10_U + SPH10_A), T_sigma=SPH10_T * (1.0 + 100.0 / 3.0), seed=seed,
                 n_steady=n_steady, capacity=int(total * cap_factor) + 4096, n_surf=n_surf, mesh=m)
