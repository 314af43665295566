"""The C-ABI library loads and exports every entry point declared in include/hs.h
(no GPU work)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\**\s*(hs_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_2506_23917_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    lib = ctypes.CDLL(B.LIB)
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    from paper_2506_23917_amd import hs
    assert set(hs.exported_symbols()) <= set(names)


def test_plan_validates_on_host():
    from paper_2506_23917_amd import hs
    import workloads as W
    g = W.gas()
    n = hs.plan_bytes(g, W.cylinder_2d(), hs.FP32_MIXED)
    assert n > 14_000_000 * 32
    try:
        hs.plan_bytes(g, dict(W.cylinder_2d(), nx=0))
    except hs.HsError as e:
        assert e.code == 1
    else:
        raise AssertionError("expected an argument error")
    # surface elements need a body, and at most 65536 of them
    for bad in (dict(W.sod_1d(), n_surf=4), dict(W.cylinder_2d(nx=40, ny=30), n_surf=70000)):
        try:
            hs.plan_bytes(g, bad)
        except hs.HsError as e:
            assert e.code == 1
        else:
            raise AssertionError("expected an argument error")
    # two cases with the same seed are rejected
    try:
        hs.plan_bytes(g, [W.sod_1d(seed=3), W.sod_1d(seed=3)])
    except hs.HsError as e:
        assert e.code == 1
    else:
        raise AssertionError("expected an argument error")


def test_plan_validates_meshes_on_host():
    """hs_plan accepts the O-grid and the meshed box and rejects broken meshes (no GPU)."""
    import numpy as np
    from paper_2506_23917_amd import hs
    import workloads as W
    g = W.gas()
    og = W.cylinder_ogrid()
    assert hs.plan_bytes(g, og, hs.FP32_MIXED) > og["capacity"] * 32
    st = dict(n=1e20, u=(800.0, 0.0, 0.0), T=300.0)
    box = W._case(dim=2, nx=6, ny=4, h=(0.05, 0.05, 1.0), bc=("inflow", "outflow", "specular", "outflow",
                  "outflow", "outflow"), inflow=st, regions=[((0, 0, 0, 0.3, 0.2, 1), st)], F_N=1e16,
                  dt_G=1e-5, capacity=1000)
    twin = W.mesh_twin(box)
    hs.plan_bytes(g, [twin, dict(box, seed=2)])            # a mesh beside a grid case

    def rejected(case):
        try:
            hs.plan_bytes(g, case)
        except hs.HsError as e:
            return e.code == 1
        return False

    for what in ("clockwise", "node", "nbr", "code", "sphere", "dim", "frame"):
        c = dict(twin)
        m = {k: np.array(v, copy=True) for k, v in twin["mesh"].items()}
        if what == "clockwise":
            m["quad"][3] = m["quad"][3][::-1]
        elif what == "node":
            m["quad"][1, 2] = 10_000
        elif what == "nbr":
            m["nbr"][0, 1] = 5
        elif what == "code":
            m["nbr"][0, 0] = -7
        elif what == "sphere":
            c["body"] = "sphere"
        elif what == "dim":
            c["dim"] = 3
        else:
            c["n_surf"] = 4                                 # surface elements need a cylinder frame
        c["mesh"] = m
        assert rejected(c), what


def test_plan_validates_hexahedra_on_host():
    """hs_plan accepts the sphere's hexahedral shell and rejects broken hexahedra (no GPU)."""
    import numpy as np
    from paper_2506_23917_amd import hs
    import workloads as W
    g = W.gas()
    sh = W.sphere_hex(n_phi=16, n_theta=8, n_r=6, r_out=2.0, ppc_outer=40)
    assert hs.plan_bytes(g, sh, hs.FP32_MIXED) > sh["capacity"] * 36
    st = dict(n=1e20, u=(800.0, 0.0, 0.0), T=300.0)
    box = W._case(dim=3, nx=4, ny=3, nz=3, h=(0.05, 0.05, 0.05), bc=("inflow",) + ("outflow",) * 5, inflow=st,
                  regions=[((0, 0, 0, 0.2, 0.15, 0.15), st)], F_N=1e16, dt_G=1e-5, capacity=1000)
    twin = W.mesh_twin_3d(box)
    hs.plan_bytes(g, [twin, dict(W.mesh_twin(W._case(dim=2, nx=3, ny=2, h=(0.1, 0.1, 1.0), regions=[((0, 0, 0, 1, 1, 1), st)],
                                                     F_N=1e16, dt_G=1e-5, capacity=100)), seed=5)])
    for what in ("nonplanar", "inverted", "nbr", "cylinder"):
        c = dict(twin)
        m = {k: np.array(v, copy=True) for k, v in twin["mesh"].items()}
        if what == "nonplanar":
            m["xy"][m["quad"][5][6]] += np.array([0.0, 0.0, 0.01])
        elif what == "inverted":
            m["quad"][3] = m["quad"][3][[4, 5, 6, 7, 0, 1, 2, 3]]
        elif what == "nbr":
            m["nbr"][0, 3] = 7
        else:
            c["body"] = "cylinder"
        c["mesh"] = m
        try:
            hs.plan_bytes(g, c)
        except hs.HsError as e:
            assert e.code == 1, what
        else:
            raise AssertionError("expected an argument error: " + what)


def test_plan_for_the_static_scratch_variant():
    """hs_plan with HS_FLAG_STATIC_SCRATCH sizes only the caller's data part of a small batch,
    and refuses a batch whose scratch exceeds the library's fixed array (no GPU)."""
    from paper_2506_23917_amd import hs
    import workloads as W
    g = W.gas()
    small = W.cylinder_2d(nx=80, ny=60, ppc=10)
    whole = hs.plan_bytes(g, small, hs.FP64)
    data = hs.plan_bytes(g, small, hs.FP64, flags=hs.FLAG_STATIC_SCRATCH)
    assert 0 < data < whole
    try:
        hs.plan_bytes(g, W.cylinder_2d(), hs.FP32_MIXED, flags=hs.FLAG_STATIC_SCRATCH)
    except hs.HsError as e:
        assert e.code == 2
    else:
        raise AssertionError("expected a capacity error")
