"""Cells denser than the tile kernel takes, on the GPU against the FP64 oracle.

A 0-D batch whose cells hold 150 (tile kernel), 700 and 2100 (block-per-cell kernel in LDS),
4000 (the largest LDS class) and 4500 and 9000 particles (the class that keeps its cell in
device memory), dt / tau from 0.05 to 20 so both collision sub-steps run: FP64 one sampled
step equals the oracle's (ids in order, NTC pair and relaxation counts, accepted-pair hash
bit-exact; velocities 1e-12; the 13 sums 1e-12); FP32-mixed runs it without error and
conserves each cell's momentum and energy to 1e-12 before rounding (the trace's sums).
No cell of a case is too dense: there is no per-cell particle limit."""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from gpu_util import vel_rel_err
from test_gpu_parity import _compare_trace
from test_gpu_sampling import compare_sums

pytestmark = pytest.mark.gpu

COUNTS = [150, 700, 2100, 4000, 4500, 9000]


def _dense_batch():
    case = W.relax_0d(ncells=len(COUNTS), ppc=1000, n_steady=0)
    case["dt_over_tau"] = np.array([0.05, 0.5, 2.0, 20.0, 1.0, 5.0])
    rng = np.random.default_rng(17)
    cell = np.repeat(np.arange(len(COUNTS), dtype=np.int32), COUNTS)
    R = W.R_ARGON
    T = np.array([273.0, 400.0, 300.0, 250.0, 600.0, 350.0])[cell]
    v = rng.standard_normal((len(cell), 3)) * np.sqrt(R * T)[:, None]
    v[:, 0] += 0.3 * np.sqrt(R * T) * (rng.standard_normal(len(cell)) ** 2 - 1.0)   # heat flux
    ids = np.arange(len(cell), dtype=np.int64)
    case["capacity"] = len(cell)
    return case, v, cell, ids


def _sim(gas, case, prec):
    from paper_2506_23917_amd.hs import Sim
    return Sim(gas, case, precision=prec, trace=True, no_particles=True)


def test_dense_cells_fp64_match_oracle(gas):
    case, v, cell, ids = _dense_batch()
    ora = Oracle(gas, case, trace=True)
    ora.set_state(0, None, v, cell, ids, len(ids), 0)
    cells = ora.get_cells(0)
    sim = _sim(gas, case, "fp64")
    sim.import_state(0, dict(pos=np.zeros((len(ids), 3)), vel=v, cell=cell, id=ids, next_id=len(ids),
                             step=0, sigc_max=cells["sigc_max"]))
    sim.step(1)
    ora.step(1)
    g, o = sim.export_state(0), ora.get_state(0)
    assert np.array_equal(g["cell"], o["cell"]) and np.array_equal(g["id"], o["id"])
    assert vel_rel_err(g["vel"], o["v"], gas) < 1e-12
    tg, to = sim.trace(0), ora.trace(0)
    _compare_trace(tg, to, label="dense")
    assert np.array_equal(to["n"], COUNTS)
    assert to["nacc"].sum() > 0 and to["nrelax"].sum() > 0
    compare_sums(g["acc"], ora.get_cells(0)["acc"], label="dense")


def test_dense_cells_fp32_conserve(gas):
    case, v, cell, ids = _dense_batch()
    sc = Oracle(gas, case).get_cells(0)["sigc_max"]
    sim = _sim(gas, case, "fp32")
    sim.import_state(0, dict(pos=np.zeros((len(ids), 3)), vel=v, cell=cell, id=ids, next_id=len(ids),
                             step=0, sigc_max=sc))
    for _ in range(3):
        sim.step(1)
        sim.sync()
        tr = sim.trace(0)
        assert np.array_equal(tr["n"], COUNTS)
        pre, post = tr["pre_sum"], tr["post_sum"]
        N = tr["n"][:, None].astype(np.float64)
        cref = np.sqrt(pre[:, 3:4] / N - (pre[:, :3] ** 2).sum(1, keepdims=True) / N ** 2)
        assert np.max(np.abs(post[:, :3] - pre[:, :3]) / (N * cref)) < 1e-12
        assert np.max(np.abs(post[:, 3] - pre[:, 3]) / pre[:, 3]) < 1e-12
    g = sim.export_state(0)
    assert np.array_equal(np.bincount(g["cell"]), COUNTS)
