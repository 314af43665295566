"""hs_init_particles_static (the step's scratch in the library's fixed device array, for
callers that cannot allocate) against hs_init_particles, through the C ABI: two sims made one
after the other, the second on a smaller batch, each stepped beside an ordinary sim of the
same cases; states, sums, counters and Step (6) outputs must be bit-identical."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _pair(gas, cases, precision, steps):
    from paper_2506_23917_amd.hs import Sim
    ref = Sim(gas, cases, precision=precision, trace=True)
    st = Sim(gas, cases, precision=precision, trace=True, static_scratch=True)
    assert st.ws_bytes < ref.ws_bytes
    for _ in range(steps):
        ref.step(1)
        st.step(1)
    for c in range(len(cases)):
        a, b = ref.export_state(c), st.export_state(c)
        for k in ("pos", "vel", "cell", "id", "sigc_max", "acc"):
            assert np.array_equal(a[k], b[k]), (precision, c, k)
        for k in ("next_id", "step", "n_samples"):
            assert a[k] == b[k], (precision, c, k)
        assert ref.counters(c) == st.counters(c)
        ta, tb = ref.trace(c), st.trace(c)
        assert ta.tobytes() == tb.tobytes()
        for mode in (0, 1):
            ma, mb = ref.sample_moments(c, mode), st.sample_moments(c, mode)
            for k in ("n", "u", "T", "q"):
                assert np.array_equal(ma[k], mb[k]), (precision, c, mode, k)
    st.close()
    ref.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_scratch_matches_workspace_sim(gas, precision):
    # first call: a cylinder with a dense tube batched beside it (both collide kernels,
    # wall sampling, inflow); second call: a smaller batch on the same array
    big = [W.cylinder_2d(nx=80, ny=60, ppc=10, n_steady=0, n_surf=12),
           W.sod_1d(ncells=60, ppc_left=320, n_steady=0, seed=5)]
    _pair(gas, big, precision, 4)
    small = [W.cylinder_2d(nx=40, ny=30, ppc=6, n_steady=1, seed=9, n_surf=6)]
    _pair(gas, small, precision, 3)


def test_static_scratch_rejects_a_batch_too_large(gas):
    from paper_2506_23917_amd.hs import HsError, Sim
    with pytest.raises(HsError) as e:
        Sim(gas, W.cylinder_2d(), precision="fp32", static_scratch=True)
    assert e.value.code == 2
