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
