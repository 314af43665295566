"""GPU (gfx950) against the FP64 oracle, through the C ABI.

FP64 path from an identical state and RNG stream: bit-exact particle counts per cell,
sort permutation (ids in order), NTC candidates / accepted pairs (with an
order-independent hash of the accepted candidate indices), relaxations and Shakhov
attempts; velocities within 1e-12 relative; positions within 1e-12 of the domain size.
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle
from gpu_util import (assert_dsmc_ratio_close, gpu_to_abs, oracle_state_to_gpu, small_cases, vel_rel_err,
                      case_extent)

pytestmark = pytest.mark.gpu


def _sim(gas, cases, **kw):
    from paper_2506_23917_amd.hs import Sim
    return Sim(gas, cases, **kw)


def _compare(gas, case, g, o, vtol=1e-12, label=""):
    assert len(g["id"]) == len(o["id"]), (label, len(g["id"]), len(o["id"]))
    assert np.array_equal(g["cell"], o["cell"]), label
    assert np.array_equal(g["id"], o["id"]), label
    assert g["next_id"] == o["next_id"], label
    err = vel_rel_err(g["vel"], o["v"], gas)
    assert err < vtol, (label, err)
    if case["dim"] > 0:
        xg = gpu_to_abs(case, g)
        perr = np.abs(xg - o["x"]).max() / case_extent(case) if len(xg) else 0.0
        assert perr < 1e-12, (label, perr)
    return err


def _compare_trace(tg, to, label=""):
    for f in ("n", "ncol", "nacc", "nrelax", "ar_attempts", "ar_cap", "acc_hash"):
        assert np.array_equal(tg[f], to[f]), (label, f, np.where(tg[f] != to[f])[0][:5])
    act = to["n"] >= 2
    for f in ("T", "tau", "dt_dsmc"):
        a, b = tg[f][act], to[f][act]
        assert np.allclose(a, b, rtol=1e-12, atol=0), (label, f)
    # P = -expm1(-(dt_G - dt_D) / tau): the difference cancels when dt_D ~ dt_G, so the
    # probability is compared absolutely
    assert np.allclose(tg["p_relax"][act], to["p_relax"][act], rtol=0, atol=1e-13), (label, "p_relax")


def test_philox_matches_oracle():
    from paper_2506_23917_amd.hs import debug_philox
    from oracle import oracle as O
    for (seed, stream, e0, step, d) in [(1, 0, 0, 0, 0), (0xDEADBEEF12345678, 1, (1 << 33) + 7, 99, 5),
                                         (42, 2, 1000, 7, 300), (3, 3, (1 << 59) - 10, 2 ** 31, 2 ** 32 - 1)]:
        n = 257
        w = debug_philox(seed, stream, e0, step, d, n)
        for i in (0, 1, 100, 256):
            assert tuple(int(x) for x in w[i]) == O.draw(seed, stream, e0 + i, step, d)


def test_philox_known_answers_on_gpu():
    # the published Philox4x32-10 known answers (tests/golden/philox4x32_10_kat.txt) through
    # the GPU generator's counter layout
    from paper_2506_23917_amd.hs import debug_philox
    from test_oracle_rng import _kat_vectors, kat_as_draw
    for ctr, key, out in _kat_vectors():
        seed, stream, entity, step, d = kat_as_draw(ctr, key)
        w = debug_philox(seed, stream, entity, step, d, 1)
        assert [int(x) for x in w[0]] == out


@pytest.mark.parametrize("name", ["sod", "cylinder", "jets", "sphere"])
def test_init_matches_oracle(gas, name):
    cases = small_cases()[name]
    sim = _sim(gas, cases, precision="fp64")
    ora = Oracle(gas, cases)
    ora.init_particles()
    for c, case in enumerate(cases):
        g = sim.export_state(c)
        o = ora.get_state(c)
        _compare(gas, case, g, o, vtol=1e-14, label="init " + name)
        oc = ora.get_cells(c)
        assert np.array_equal(g["sigc_max"], oc["sigc_max"])


@pytest.mark.parametrize("name,steps", [("sod", 1), ("sod", 4), ("cylinder", 1), ("cylinder", 3),
                                        ("jets", 6), ("sphere", 2)])
def test_fp64_steps_match_oracle(gas, name, steps):
    cases = small_cases()[name]
    sim = _sim(gas, cases, precision="fp64", trace=True)
    ora = Oracle(gas, cases, trace=True)
    ora.init_particles()
    for s in range(steps):
        sim.step(1)
        ora.step(1)
    for c, case in enumerate(cases):
        g = sim.export_state(c)
        o = ora.get_state(c)
        _compare(gas, case, g, o, label="%s case %d" % (name, c))
        _compare_trace(sim.trace(c), ora.trace(c), label=name)
        gc, oc = sim.counters(c), ora.counters(c)
        for k in ("injected", "removed", "wall_hits", "candidates", "accepted", "relaxed", "ar_attempts"):
            assert gc[k] == oc[k], (name, k, gc[k], oc[k])
        cells = ora.get_cells(c)
        assert np.allclose(g["sigc_max"], cells["sigc_max"], rtol=1e-12)


def test_fp64_0d_batch_matches_oracle(gas):
    case = W.relax_0d(ncells=48, ppc=300)
    rng = np.random.default_rng(3)
    case["dt_over_tau"] = 10 ** rng.uniform(-2, 2, 48)
    v, cell, ids = W.relax_0d_state(case, ppc=300)
    ora = Oracle(gas, case, trace=True)
    ora.set_state(0, None, v, cell, ids, len(ids), 0)
    sim = _sim(gas, case, precision="fp64", trace=True, no_particles=True)
    cells = ora.get_cells(0)
    sim.import_state(0, dict(pos=np.zeros((len(ids), 3)), vel=v, cell=cell, id=ids, next_id=len(ids),
                             step=0, sigc_max=cells["sigc_max"]))
    for _ in range(3):
        sim.step(1)
        ora.step(1)
    _compare(gas, case, sim.export_state(0), ora.get_state(0), label="0d")
    _compare_trace(sim.trace(0), ora.trace(0), label="0d")


def test_fp64_from_imported_midrun_state(gas):
    # a developed cylinder state (oracle after 12 steps) imported into the GPU
    case = W.cylinder_2d(nx=80, ny=60, ppc=10)
    ora = Oracle(gas, case, trace=True)
    ora.init_particles()
    ora.step(12)
    o = ora.get_state(0)
    cells = ora.get_cells(0)
    sim = _sim(gas, case, precision="fp64", trace=True)
    sim.import_state(0, oracle_state_to_gpu(case, o, cells["sigc_max"], cells["acc"], cells["n_samples"]))
    sim.step(2)
    ora.step(2)
    _compare(gas, case, sim.export_state(0), ora.get_state(0), label="midrun")
    _compare_trace(sim.trace(0), ora.trace(0), label="midrun")


def test_conservation_fp64_and_mixed(gas):
    case = W.relax_0d(ncells=32, ppc=400)
    rng = np.random.default_rng(5)
    case["dt_over_tau"] = 10 ** rng.uniform(-2, 2, 32)
    v, cell, ids = W.relax_0d_state(case, ppc=400)
    for prec in ("fp64", "fp32"):
        sim = _sim(gas, case, precision=prec, trace=True, no_particles=True)
        sc = Oracle(gas, case).get_cells(0)["sigc_max"]
        sim.import_state(0, dict(pos=np.zeros((len(ids), 3)), vel=v, cell=cell, id=ids, next_id=len(ids),
                                 step=0, sigc_max=sc))
        sim.step(1)
        tr = sim.trace(0)
        act = tr["n"] >= 2
        pre, post = tr["pre_sum"][act], tr["post_sum"][act]
        N = tr["n"][act][:, None]
        cref = np.sqrt(pre[:, 3:4] / N)
        assert np.all(np.abs(post[:, :3] - pre[:, :3]) / (N * cref) < 1e-12), prec
        assert np.all(np.abs(post[:, 3] - pre[:, 3]) / pre[:, 3] < 1e-12), prec


def test_error_paths(gas):
    from paper_2506_23917_amd.hs import HsError
    case = W.cylinder_2d(nx=40, ny=30, ppc=6)
    bad = dict(case, capacity=1000)
    with pytest.raises(HsError) as e:
        _sim(gas, bad)
    assert e.value.code == 2
    bad2 = dict(case, dt_G=-1.0)
    with pytest.raises(HsError) as e:
        _sim(gas, bad2)
    assert e.value.code == 1
    sim = _sim(gas, case)
    st = sim.export_state(0)
    st["vel"] = st["vel"].copy()
    st["vel"][5, 1] = np.nan
    with pytest.raises(HsError) as e:
        sim.import_state(0, st)
    assert e.value.code == 3
    # capacity exhausted by inflow during the run
    tight = dict(case)
    o = Oracle(gas, case)
    o.init_particles()
    tight["capacity"] = o.num_particles() + 5
    sim = _sim(gas, tight)
    sim.step(3)
    with pytest.raises(HsError) as e:
        sim.sync()
    assert e.value.code == 2


@pytest.mark.parametrize("name", ["fm_cylinder", "fm_sphere", "cylinder"])
def test_fp64_surface_sums_match_oracle(gas, name):
    """Body wall sums (reflections exact per element, momentum and energy sums to 1e-11)
    and their Eq. 35-36 time averages, FP64 path against the oracle from the same start."""
    if name == "fm_cylinder":
        case, steps = W.free_molecular_body("cylinder", s=1.0, cells=20, ppc=10, R=0.3, n_surf=8), 30
    elif name == "fm_sphere":
        case, steps = W.free_molecular_body("sphere", s=1.0, cells=12, ppc=8, R=0.35, n_surf=6), 20
    else:
        case = dict(small_cases()["cylinder"][0])
        case.update(n_steady=0, n_surf=16)       # collisions on, the Ma 10 stream
        steps = 4
    sim = _sim(gas, [case], precision="fp64")
    ora = Oracle(gas, [case])
    ora.init_particles()
    sim.step(steps)
    ora.step(steps)
    _compare(gas, case, sim.export_state(0), ora.get_state(0), label="surface " + name)
    sg, so = sim.surface_sums(0), ora.surface_sums(0)
    assert so[:, 0].sum() > 50, so[:, 0]
    assert np.array_equal(sg[:, 0], so[:, 0]), (name, sg[:, 0], so[:, 0])
    scale = np.abs(so[:, 1:]).max(axis=0)
    assert np.allclose(sg[:, 1:], so[:, 1:], rtol=1e-11, atol=1e-12 * scale), name
    rg, ro = sim.surface_sample(0), ora.surface_sample(0)
    assert rg["n_samples"] == ro["n_samples"] == steps
    for k in ("theta", "area", "p", "tau", "q", "Cp", "Cf", "Ch"):
        s = np.abs(ro[k]).max()
        assert np.allclose(rg[k], ro[k], rtol=1e-11, atol=1e-12 * s), (name, k)
    assert np.allclose(rg["force"], ro["force"], rtol=1e-11, atol=1e-12 * np.abs(ro["force"]).max())
    for k in ("CD", "CL"):
        assert abs(rg[k] - ro[k]) <= 1e-11 * max(abs(ro["CD"]), 1e-300), (name, k)


@pytest.mark.parametrize("name,steps", [("cylinder", 5), ("sod", 6), ("jets", 8)])
def test_fp64_adaptive_step_matches_oracle(gas, name, steps):
    """Eq. 26 global step: the same step sequence (1e-12) and, step by step, the same
    particles (cells and ids exact, velocities and positions 1e-12), inflow counts
    included; then the ratio-of-DSMC field of the sampled moments."""
    cases = []
    for c in small_cases()[name]:
        c = dict(c)
        c.update(adapt_dt=True, n_steady=0, n_surf=0)
        cases.append(c)
    sim = _sim(gas, cases, precision="fp64")
    ora = Oracle(gas, cases)
    ora.init_particles()
    changed = False
    for s in range(steps):
        sim.step(1)
        ora.step(1)
        for k, case in enumerate(cases):
            dg, tg = sim.step_dt(k)
            do, to = ora.step_dt(k)
            assert dg == pytest.approx(do, rel=1e-12, abs=0), (name, s, k)
            assert tg == pytest.approx(to, rel=1e-12, abs=0), (name, s, k)
            changed = changed or do != case["dt_G"]
            _compare(gas, case, sim.export_state(k), ora.get_state(k), label="adaptive %s step %d" % (name, s))
    assert changed
    for k in range(len(cases)):
        rg, ro = sim.dsmc_ratio(k), ora.dsmc_ratio(k)
        assert_dsmc_ratio_close(rg, ro, ora.get_cells(k)["acc"], rtol=1e-11, atol=1e-14)
        assert np.any((ro > 0) & (ro <= 1))


def test_fp64_many_small_cases_match_oracle(gas):
    """A batch of 120 small Sod tubes (distinct seeds; several cases per tile walk of a
    wave, so the per-wave counter slots fill and flush): states and every counter of every
    case equal the oracle's after a few steps."""
    cases = [W.sod_1d(seed=s + 11, ncells=40, ppc_left=48, n_steady=0) for s in range(120)]
    sim = _sim(gas, cases, precision="fp64")
    ora = Oracle(gas, cases)
    ora.init_particles()
    sim.step(3)
    ora.step(3)
    for c, case in enumerate(cases):
        _compare(gas, case, sim.export_state(c), ora.get_state(c), label="case %d" % c)
        gc, oc = sim.counters(c), ora.counters(c)
        for k in oc:
            assert gc[k] == oc[k], (c, k, gc[k], oc[k])
    assert sum(ora.counters(c)["candidates"] for c in range(len(cases))) > 0
