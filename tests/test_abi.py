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
