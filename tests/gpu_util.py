"""Helpers of the GPU parity tests: run the same cases through the HIP library and the
oracle, convert states between their layouts, compare."""
import numpy as np

import workloads as W

KB = 1.380649e-23


def ijk_of(case, cell):
    cell = np.asarray(cell, np.int64)
    nx, ny = case["nx"], case["ny"]
    if case["dim"] == 0:
        return cell, np.zeros_like(cell), np.zeros_like(cell)
    i = cell % nx
    j = (cell // nx) % ny if case["dim"] >= 2 else np.zeros_like(cell)
    k = cell // (nx * ny) if case["dim"] >= 3 else np.zeros_like(cell)
    return i, j, k


def gpu_to_abs(case, st):
    """Absolute positions lo + (ijk + xr) h of an exported GPU state."""
    ijk = ijk_of(case, st["cell"])
    x = np.zeros((len(st["cell"]), 3))
    for a in range(case["dim"]):
        x[:, a] = case["lo"][a] + (ijk[a] + st["pos"][:, a].astype(np.float64)) * case["h"][a]
    return x


def abs_to_rel(case, x, cell):
    ijk = ijk_of(case, cell)
    r = np.zeros((len(cell), 3))
    for a in range(case["dim"]):
        r[:, a] = (x[:, a] - case["lo"][a]) / case["h"][a] - ijk[a]
    return r


def oracle_state_to_gpu(case, o, sigc, acc=None, n_samples=0):
    return dict(pos=abs_to_rel(case, o["x"], o["cell"]), vel=o["v"], cell=o["cell"], id=o["id"],
                next_id=o["next_id"], step=o["step"], sigc_max=sigc,
                acc=acc if acc is not None else np.zeros((len(sigc), 13)), n_samples=n_samples)


def vel_rel_err(gpu_v, ora_v, gas, T=300.0):
    cref = np.sqrt(KB * T / gas["m"])
    scale = np.maximum(np.linalg.norm(ora_v, axis=1), cref)
    return float(np.max(np.linalg.norm(gpu_v.astype(np.float64) - ora_v, axis=1) / scale)) if len(ora_v) else 0.0


def case_extent(case):
    return max(case["h"][a] * [case["nx"], case["ny"], case["nz"]][a] for a in range(max(1, case["dim"])))


def small_cases():
    """Workload shapes of the paper's cases at sizes the oracle finishes in seconds."""
    c1 = W.sod_1d(ncells=60, ppc_left=320)             # left cells > 256: block kernel path
    c3 = W.cylinder_2d(nx=80, ny=60, ppc=10)
    jets = W.jets_2d(n_jets=3, grids=((40, 20), (80, 40), (60, 30)), cap_factor=4.0)
    for j in jets:
        j["F_N"] *= 0.5     # denser exit, so the jets hold particles within a few steps
    c5 = W.sphere_3d(nx=24, ny=16, nz=16, ppc=8)
    return dict(sod=[c1], cylinder=[c3], jets=jets, sphere=[c5])


def assert_dsmc_ratio_close(rg, ro, acc, rtol, atol):
    """Ratio of DSMC (Eq. 27 from the time-averaged n, U, T) of the GPU against the oracle.
    Where the sampled T is zero in exact arithmetic (one particle with one velocity in every
    sampled step) its computed sign is decided by the rounding of the Step 5 sums, and with it
    whether the ratio is 0 (no T) or 1; those cells only need a valid ratio.  Elsewhere, where
    the peculiar energy stands above the sums' rounding, the ratios agree to rtol / atol."""
    acc = np.asarray(acc, np.float64)
    a0 = np.where(acc[:, 0] > 0, acc[:, 0], 1.0)
    cc = (acc[:, 4] + acc[:, 5] + acc[:, 6]) / a0
    uu = (acc[:, 1] ** 2 + acc[:, 2] ** 2 + acc[:, 3] ** 2) / a0 ** 2
    resolved = (acc[:, 0] > 0) & (cc - uu > 1e-9 * cc)
    np.testing.assert_allclose(rg[resolved], ro[resolved], rtol=rtol, atol=atol)
    assert np.all((rg >= 0) & (rg <= 1)) and np.all(rg[acc[:, 0] == 0] == 0)
    return resolved
