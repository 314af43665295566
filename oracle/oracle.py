"""ctypes wrapper of the FP64 CPU oracle (hs_oracle.c).  Test infrastructure only.

Marshals the plain case dictionaries of the `workloads` package into the oracle's own C
structs and exposes its entry points and building blocks to the tests.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hs_oracle.c")
_LIB = os.path.join(_HERE, "libhs_oracle.so")
_lock = threading.Lock()
_lib = None

BC = {"outflow": 0, "specular": 1, "inflow": 2}
BODY = {"none": 0, "cylinder": 1, "sphere": 2}
EDGE = {"outflow": -1, "inflow": -2, "wall": -3, "specular": -4}
ERRORS = {1: "argument", 2: "capacity", 3: "numeric", 5: "state"}


class OracleError(RuntimeError):
    pass


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, no FP contraction)."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp%d" % os.getpid()
            cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                   "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, _LIB)
    return _LIB


class Gas(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("m", "d_ref", "T_ref", "omega", "mu_ref", "Pr", "gamma")]


class State(C.Structure):
    _fields_ = [("n", C.c_double), ("u", C.c_double * 3), ("T", C.c_double)]


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_cells", C.c_int32), ("xy", C.POINTER(C.c_double)),
                ("quad", C.POINTER(C.c_int32)), ("nbr", C.POINTER(C.c_int32))]


class Case(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lo", C.c_double * 3), ("h", C.c_double * 3), ("bc", C.c_int32 * 6),
                ("inflow", State), ("slot_lo", C.c_double * 3), ("slot_hi", C.c_double * 3),
                ("body", C.c_int32), ("body_c", C.c_double * 3), ("body_r", C.c_double),
                ("body_T", C.c_double), ("n_regions", C.c_int32),
                ("region_box", C.POINTER(C.c_double)), ("region_state", C.POINTER(State)),
                ("F_N", C.c_double), ("dt_G", C.c_double), ("T_sigma", C.c_double),
                ("dt_over_tau", C.POINTER(C.c_double)), ("seed", C.c_uint64),
                ("n_steady", C.c_int64), ("capacity", C.c_int64), ("n_surf", C.c_int32),
                ("adapt_dt", C.c_int32), ("mesh", C.POINTER(Mesh))]


class Trace(C.Structure):
    _fields_ = [("n", C.c_int64), ("ncol", C.c_int64), ("nacc", C.c_int64), ("nrelax", C.c_int64),
                ("ar_attempts", C.c_int64), ("ar_cap", C.c_int64), ("acc_hash", C.c_uint64),
                ("T", C.c_double), ("tau", C.c_double), ("dt_dsmc", C.c_double),
                ("p_relax", C.c_double), ("a_max", C.c_double),
                ("pre_sum", C.c_double * 4), ("post_sum", C.c_double * 4)]


TRACE_DTYPE = np.dtype([("n", "i8"), ("ncol", "i8"), ("nacc", "i8"), ("nrelax", "i8"),
                        ("ar_attempts", "i8"), ("ar_cap", "i8"), ("acc_hash", "u8"),
                        ("T", "f8"), ("tau", "f8"), ("dt_dsmc", "f8"), ("p_relax", "f8"),
                        ("a_max", "f8"), ("pre_sum", "f8", (4,)), ("post_sum", "f8", (4,))])
assert TRACE_DTYPE.itemsize == C.sizeof(Trace)

COUNTER_NAMES = ("injected", "removed", "wall_hits", "candidates", "accepted", "relaxed",
                 "ar_attempts", "ar_cap", "bounce_cap", "inject_cap", "skipped_cells")


class Counters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in COUNTER_NAMES]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lib():
    global _lib
    if _lib is None:
        build_oracle()
        L = C.CDLL(_LIB)
        P = C.POINTER
        L.hso_create.argtypes = [P(Gas), P(Case), C.c_int, C.c_int, P(C.c_void_p)]
        L.hso_destroy.argtypes = [C.c_void_p]
        L.hso_destroy.restype = None
        L.hso_init_particles.argtypes = [C.c_void_p]
        L.hso_step.argtypes = [C.c_void_p, C.c_int64]
        L.hso_sample_moments.argtypes = [C.c_void_p, C.c_int, C.c_int, P(C.c_double), P(C.c_double),
                                         P(C.c_double), P(C.c_double), P(C.c_int64)]
        L.hso_get_surface.argtypes = [C.c_void_p, C.c_int, P(C.c_double)]
        L.hso_step_dt.argtypes = [C.c_void_p, C.c_int, P(C.c_double), P(C.c_double)]
        L.hso_set_step_dt.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
        L.hso_dsmc_ratio.argtypes = [C.c_void_p, C.c_int, P(C.c_double)]
        L.hso_set_surface.argtypes = [C.c_void_p, C.c_int, P(C.c_double)]
        L.hso_surface_sample.argtypes = [C.c_void_p, C.c_int, P(C.c_double), P(C.c_double), P(C.c_int64)]
        L.hso_num_particles.argtypes = [C.c_void_p, C.c_int]
        L.hso_num_particles.restype = C.c_int64
        L.hso_num_cells.argtypes = [C.c_void_p, C.c_int]
        L.hso_num_cells.restype = C.c_int64
        L.hso_num_faces.argtypes = [C.c_void_p, C.c_int]
        L.hso_num_faces.restype = C.c_int64
        L.hso_face_info.argtypes = [C.c_void_p, C.c_int, P(C.c_int32), P(C.c_int32), P(C.c_double)]
        L.hso_get_state.argtypes = [C.c_void_p, C.c_int, P(C.c_double), P(C.c_double), P(C.c_int32),
                                    P(C.c_int64), P(C.c_int64), P(C.c_int64)]
        L.hso_set_state.argtypes = [C.c_void_p, C.c_int, C.c_int64, P(C.c_double), P(C.c_double),
                                    P(C.c_int32), P(C.c_int64), C.c_int64, C.c_int64]
        L.hso_get_cells.argtypes = [C.c_void_p, C.c_int, P(C.c_double), P(C.c_double), P(C.c_double),
                                    P(C.c_int64)]
        L.hso_set_cells.argtypes = [C.c_void_p, C.c_int, P(C.c_double), P(C.c_double), C.c_int64]
        L.hso_get_trace.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.hso_get_counters.argtypes = [C.c_void_p, C.c_int, P(Counters)]
        L.hso_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.hso_philox4x32_10.restype = None
        L.hso_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32, P(C.c_uint32)]
        L.hso_draw.restype = None
        L.hso_uniform.argtypes = [C.c_uint32]
        L.hso_uniform.restype = C.c_double
        L.hso_index.argtypes = [C.c_uint32, C.c_uint32]
        L.hso_index.restype = C.c_uint32
        for f in ("hso_sigma_c", "hso_viscosity"):
            getattr(L, f).argtypes = [P(Gas), C.c_double]
            getattr(L, f).restype = C.c_double
        L.hso_mean_free_path.argtypes = [P(Gas), C.c_double, C.c_double]
        L.hso_mean_free_path.restype = C.c_double
        L.hso_inflow_number_flux.argtypes = [P(Gas), P(State), P(C.c_double)]
        L.hso_inflow_number_flux.restype = C.c_double
        L.hso_sample_normal_speed.argtypes = [C.c_double, P(C.c_uint32), C.c_int, P(C.c_int)]
        L.hso_sample_normal_speed.restype = C.c_double
        L.hso_cell_moments.argtypes = [P(Gas), C.c_int64, P(C.c_double), C.c_double, C.c_double,
                                       P(C.c_double), P(C.c_double), P(C.c_double)]
        L.hso_shakhov_sample.argtypes = [P(Gas), C.c_double, C.c_double, P(C.c_double), C.c_double,
                                         P(C.c_uint32), C.c_int, P(C.c_double)]
        L.hso_split.argtypes = [C.c_double, C.c_double, C.c_double, P(C.c_double), P(C.c_double)]
        L.hso_split.restype = None
        L.hso_cut_count.argtypes = [P(Case), C.c_int, C.c_int, C.c_int]
        L.hso_cut_count.restype = C.c_int64
        _lib = L
    return _lib


def make_gas(g: dict) -> Gas:
    return Gas(*(float(g[k]) for k in ("m", "d_ref", "T_ref", "omega", "mu_ref", "Pr", "gamma")))


def make_state(s: dict) -> State:
    return State(float(s["n"]), (C.c_double * 3)(*s["u"]), float(s["T"]))


class _CaseHolder:
    """Keeps the numpy/ctypes buffers a Case struct points at alive."""

    def __init__(self, d: dict):
        c = Case()
        c.dim, c.nx, c.ny, c.nz = int(d["dim"]), int(d["nx"]), int(d["ny"]), int(d["nz"])
        c.lo = (C.c_double * 3)(*d["lo"])
        c.h = (C.c_double * 3)(*d["h"])
        c.bc = (C.c_int32 * 6)(*[BC[b] for b in d["bc"]])
        c.inflow = make_state(d["inflow"])
        c.slot_lo = (C.c_double * 3)(*d["slot_lo"])
        c.slot_hi = (C.c_double * 3)(*d["slot_hi"])
        c.body = BODY[d["body"]]
        c.body_c = (C.c_double * 3)(*d["body_c"])
        c.body_r, c.body_T = float(d["body_r"]), float(d["body_T"])
        regs = d["regions"]
        c.n_regions = len(regs)
        self.box = np.ascontiguousarray(np.array([r[0] for r in regs], dtype=np.float64).reshape(-1))
        self.states = (State * max(1, len(regs)))(*[make_state(r[1]) for r in regs])
        c.region_box = _dp(self.box) if len(regs) else None
        c.region_state = self.states if len(regs) else None
        c.F_N, c.dt_G, c.T_sigma = float(d["F_N"]), float(d["dt_G"]), float(d["T_sigma"])
        self.dtt = None
        if d.get("dt_over_tau") is not None:
            self.dtt = np.ascontiguousarray(np.asarray(d["dt_over_tau"], dtype=np.float64))
            c.dt_over_tau = _dp(self.dtt)
        c.seed = int(d["seed"])
        c.n_steady = int(d["n_steady"])
        c.capacity = int(d["capacity"])
        c.n_surf = int(d.get("n_surf", 0))
        c.adapt_dt = int(bool(d.get("adapt_dt", False)))
        self.mesh = None
        if d.get("mesh") is not None:
            m = d["mesh"]
            self.mxy = np.ascontiguousarray(np.asarray(m["xy"], dtype=np.float64).reshape(-1))
            self.mquad = np.ascontiguousarray(np.asarray(m["quad"], dtype=np.int32).reshape(-1))
            self.mnbr = np.ascontiguousarray(np.array(
                [EDGE[v] if isinstance(v, str) else int(v) for v in np.asarray(m["nbr"]).reshape(-1)],
                dtype=np.int32))
            dn, vn = (3, 8) if int(d["dim"]) == 3 else (2, 4)      # coordinates, nodes per cell
            self.mesh = Mesh(self.mxy.size // dn, self.mquad.size // vn, _dp(self.mxy),
                             self.mquad.ctypes.data_as(C.POINTER(C.c_int32)),
                             self.mnbr.ctypes.data_as(C.POINTER(C.c_int32)))
            c.mesh = C.pointer(self.mesh)
        self.c = c


def _check(rc, what):
    if rc != 0:
        raise OracleError("%s failed: %s error (%d)" % (what, ERRORS.get(rc, "?"), rc))


class Oracle:
    """The FP64 CPU oracle for a batch of cases."""

    def __init__(self, gas: dict, cases, trace: bool = False):
        if isinstance(cases, dict):
            cases = [cases]
        self.L = lib()
        self.case_dicts = list(cases)
        self.holders = [_CaseHolder(d) for d in cases]
        arr = (Case * len(cases))(*[h.c for h in self.holders])
        self._arr = arr
        self.gas = make_gas(gas)
        h = C.c_void_p()
        _check(self.L.hso_create(C.byref(self.gas), arr, len(cases), int(trace), C.byref(h)), "create")
        self.h = h
        self.trace_on = trace

    def close(self):
        if self.h:
            self.L.hso_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_particles(self):
        _check(self.L.hso_init_particles(self.h), "init_particles")

    def step(self, n: int = 1):
        _check(self.L.hso_step(self.h, int(n)), "step")

    def num_particles(self, c=0) -> int:
        return int(self.L.hso_num_particles(self.h, c))

    def num_cells(self, c=0) -> int:
        return int(self.L.hso_num_cells(self.h, c))

    def faces(self, c=0):
        nf = int(self.L.hso_num_faces(self.h, c))
        cell = np.zeros(nf, np.int32)
        side = np.zeros(nf, np.int32)
        lam = np.zeros(nf)
        _check(self.L.hso_face_info(self.h, c, cell.ctypes.data_as(C.POINTER(C.c_int32)),
                                    side.ctypes.data_as(C.POINTER(C.c_int32)), _dp(lam)), "faces")
        return dict(cell=cell, side=side, lam=lam)

    def get_state(self, c=0) -> dict:
        n = self.num_particles(c)
        x = np.zeros((n, 3))
        v = np.zeros((n, 3))
        cell = np.zeros(n, np.int32)
        ids = np.zeros(n, np.int64)
        nid, st = C.c_int64(), C.c_int64()
        _check(self.L.hso_get_state(self.h, c, _dp(x), _dp(v), cell.ctypes.data_as(C.POINTER(C.c_int32)),
                                    ids.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(nid), C.byref(st)),
               "get_state")
        return dict(x=x, v=v, cell=cell, id=ids, next_id=nid.value, step=st.value)

    def set_state(self, c, x, v, cell, ids, next_id, step):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
        n = v.shape[0]
        xp = None
        if x is not None:
            x = np.ascontiguousarray(x, dtype=np.float64).reshape(n, 3)
            xp = _dp(x)
        cell = np.ascontiguousarray(cell, dtype=np.int32)
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        _check(self.L.hso_set_state(self.h, c, n, xp, _dp(v), cell.ctypes.data_as(C.POINTER(C.c_int32)),
                                    ids.ctypes.data_as(C.POINTER(C.c_int64)), int(next_id), int(step)),
               "set_state")

    def get_cells(self, c=0) -> dict:
        nc = self.num_cells(c)
        vol, scm, acc = np.zeros(nc), np.zeros(nc), np.zeros((nc, 13))
        ns = C.c_int64()
        _check(self.L.hso_get_cells(self.h, c, _dp(vol), _dp(scm), _dp(acc), C.byref(ns)), "get_cells")
        return dict(vol=vol, sigc_max=scm, acc=acc, n_samples=ns.value)

    def set_cells(self, c, sigc_max=None, acc=None, n_samples=0):
        sp = ap = None
        if sigc_max is not None:
            sigc_max = np.ascontiguousarray(sigc_max, dtype=np.float64)
            sp = _dp(sigc_max)
        if acc is not None:
            acc = np.ascontiguousarray(acc, dtype=np.float64)
            ap = _dp(acc)
        _check(self.L.hso_set_cells(self.h, c, sp, ap, int(n_samples)), "set_cells")

    def step_dt(self, c=0):
        """(global step of the next step, sampled time so far)."""
        dt, ts = C.c_double(), C.c_double()
        _check(self.L.hso_step_dt(self.h, c, C.byref(dt), C.byref(ts)), "step_dt")
        return dt.value, ts.value

    def set_step_dt(self, c, dt, t_sampled=0.0):
        _check(self.L.hso_set_step_dt(self.h, c, float(dt), float(t_sampled)), "set_step_dt")

    def dsmc_ratio(self, c=0) -> np.ndarray:
        """Ratio of DSMC (Dt_DSMC / Dt_G) per cell from the time-averaged moments."""
        out = np.zeros(self.num_cells(c))
        _check(self.L.hso_dsmc_ratio(self.h, c, _dp(out)), "dsmc_ratio")
        return out

    def surface_sums(self, c=0) -> np.ndarray:
        """Raw wall sums, (n_surf, 7): reflections, sum dP.n, sum dP.t, sum dE, sum dP."""
        out = np.zeros((int(self.case_dicts[c].get("n_surf", 0)), 7))
        _check(self.L.hso_get_surface(self.h, c, _dp(out)), "get_surface")
        return out

    def set_surface_sums(self, c, sums):
        sums = np.ascontiguousarray(sums, dtype=np.float64)
        _check(self.L.hso_set_surface(self.h, c, _dp(sums)), "set_surface")

    def surface_sample(self, c=0) -> dict:
        """Eq. 35-36 time averages of the wall sums: per element theta (mid), area, p, tau,
        q, Cp, Cf, Ch; per case the force per unit time and CD, CL."""
        ns = int(self.case_dicts[c].get("n_surf", 0))
        e, b = np.zeros((ns, 8)), np.zeros(5)
        k = C.c_int64()
        _check(self.L.hso_surface_sample(self.h, c, _dp(e), _dp(b), C.byref(k)), "surface_sample")
        out = {n: e[:, i].copy() for i, n in enumerate(("theta", "area", "p", "tau", "q", "Cp", "Cf", "Ch"))}
        out.update(force=b[:3].copy(), CD=float(b[3]), CL=float(b[4]), n_samples=k.value)
        return out

    def trace(self, c=0) -> np.ndarray:
        out = np.zeros(self.num_cells(c), dtype=TRACE_DTYPE)
        _check(self.L.hso_get_trace(self.h, c, out.ctypes.data), "trace")
        return out

    def counters(self, c=0) -> dict:
        k = Counters()
        _check(self.L.hso_get_counters(self.h, c, C.byref(k)), "counters")
        return {n: getattr(k, n) for n in COUNTER_NAMES}

    def sample_moments(self, c=0, mode=0) -> dict:
        nc = self.num_cells(c)
        n, T = np.zeros(nc), np.zeros(nc)
        u, q = np.zeros((nc, 3)), np.zeros((nc, 3))
        ns = C.c_int64()
        _check(self.L.hso_sample_moments(self.h, c, mode, _dp(n), _dp(u), _dp(T), _dp(q), C.byref(ns)),
               "sample_moments")
        return dict(n=n, u=u, T=T, q=q, n_samples=ns.value)


# ---- building blocks -------------------------------------------------------------------

def philox(ctr, key):
    L = lib()
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    L.hso_philox4x32_10(c, k, o)
    return tuple(o)


def draw(seed, stream, entity, step, d):
    o = (C.c_uint32 * 4)()
    lib().hso_draw(seed, stream, entity, step, d, o)
    return tuple(o)


def uniform(w):
    return lib().hso_uniform(w)


def index(w, n):
    return lib().hso_index(w, n)


def sigma_c(gas: dict, cr):
    return lib().hso_sigma_c(C.byref(make_gas(gas)), cr)


def viscosity(gas: dict, T):
    return lib().hso_viscosity(C.byref(make_gas(gas)), T)


def mean_free_path(gas: dict, n, T):
    return lib().hso_mean_free_path(C.byref(make_gas(gas)), n, T)


def inflow_flux(gas: dict, state: dict, nrm):
    nv = (C.c_double * 3)(*nrm)
    return lib().hso_inflow_number_flux(C.byref(make_gas(gas)), C.byref(make_state(state)), nv)


def sample_normal_speed(s, words):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    used = C.c_int()
    z = lib().hso_sample_normal_speed(s, w.ctypes.data_as(C.POINTER(C.c_uint32)), len(w) // 4, C.byref(used))
    return z, used.value


def cell_moments(gas: dict, v, F_N, vol):
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    U, T, Q = (C.c_double * 3)(), C.c_double(), (C.c_double * 3)()
    lib().hso_cell_moments(C.byref(make_gas(gas)), v.shape[0], _dp(v), F_N, vol, U, C.byref(T), Q)
    return np.array(U), T.value, np.array(Q)


def shakhov_sample(gas: dict, T, p, Q, a_max, words):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    out = (C.c_double * 3)()
    q = (C.c_double * 3)(*Q)
    r = lib().hso_shakhov_sample(C.byref(make_gas(gas)), T, p, q, a_max,
                                 w.ctypes.data_as(C.POINTER(C.c_uint32)), len(w) // 5, out)
    return r, np.array(out)


def split(dt_c, tau, dt_G):
    a, b = C.c_double(), C.c_double()
    lib().hso_split(dt_c, tau, dt_G, C.byref(a), C.byref(b))
    return a.value, b.value


def cut_count(case: dict, i, j, k):
    h = _CaseHolder(case)
    return lib().hso_cut_count(C.byref(h.c), i, j, k)
