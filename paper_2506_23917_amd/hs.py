"""Python binding of the gfx950 hybrid SP-Shakhov / DSMC library (include/hs.h).

Argument marshalling only: every step of the particle update runs in the HIP kernels of
libhs.so.  PyTorch provides the device workspace and the stream.  If the library is not
built, importing the binding raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhs.so")

FP64, FP32_MIXED = 0, 1
BC = {"outflow": 0, "specular": 1, "inflow": 2}
BODY = {"none": 0, "cylinder": 1, "sphere": 2}
EDGE = {"outflow": -1, "inflow": -2, "wall": -3, "specular": -4}
FLAG_TRACE, FLAG_NO_PARTICLES, FLAG_GRAPH, FLAG_STATIC_SCRATCH = 1, 2, 4, 8
KERNELS = {"inject": 0, "move": 1, "scan": 2, "scatter": 3, "gather": 4, "scalars": 5, "collide": 6,
           "dense": 7, "step": 8}


class HsTuneReport(C.Structure):
    _fields_ = [("grid", C.c_int32 * len(KERNELS)), ("ms", C.c_double * len(KERNELS)), ("steps", C.c_int64)]
COUNTERS = ("injected", "removed", "wall_hits", "candidates", "accepted", "relaxed",
            "ar_attempts", "ar_cap", "bounce_cap", "inject_cap", "skipped_cells")
STATUS = {0: "ok", 1: "argument", 2: "capacity", 3: "numeric", 4: "device", 5: "state"}
MAGIC = 0x48534331


class HsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hs error %d (%s): %s" % (code, STATUS.get(code, "?"), msg))
        self.code = code


class HsGas(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("m", "d_ref", "T_ref", "omega", "mu_ref", "Pr", "gamma")]


class HsState(C.Structure):
    _fields_ = [("n", C.c_double), ("u", C.c_double * 3), ("T", C.c_double)]


class HsMesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_cells", C.c_int32), ("xy", C.POINTER(C.c_double)),
                ("quad", C.POINTER(C.c_int32)), ("nbr", C.POINTER(C.c_int32))]


class HsCase(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lo", C.c_double * 3), ("h", C.c_double * 3), ("bc", C.c_int32 * 6),
                ("inflow", HsState), ("slot_lo", C.c_double * 3), ("slot_hi", C.c_double * 3),
                ("body", C.c_int32), ("body_c", C.c_double * 3), ("body_r", C.c_double),
                ("body_T", C.c_double), ("n_regions", C.c_int32),
                ("region_box", C.POINTER(C.c_double)), ("region_state", C.POINTER(HsState)),
                ("F_N", C.c_double), ("dt_G", C.c_double), ("T_sigma", C.c_double),
                ("dt_over_tau", C.POINTER(C.c_double)), ("seed", C.c_uint64),
                ("n_steady", C.c_int64), ("capacity", C.c_int64), ("n_surf", C.c_int32),
                ("adapt_dt", C.c_int32), ("mesh", C.POINTER(HsMesh))]


class HsStateHeader(C.Structure):
    _fields_ = [("magic", C.c_uint32), ("version", C.c_uint32), ("precision", C.c_uint32),
                ("dim", C.c_uint32), ("np", C.c_int64), ("ncells", C.c_int64),
                ("next_id", C.c_int64), ("step", C.c_int64), ("n_samples", C.c_int64),
                ("dt_next", C.c_double), ("t_sampled", C.c_double)]


TRACE_DTYPE = np.dtype([("n", "i8"), ("ncol", "i8"), ("nacc", "i8"), ("nrelax", "i8"),
                        ("ar_attempts", "i8"), ("ar_cap", "i8"), ("acc_hash", "u8"),
                        ("T", "f8"), ("tau", "f8"), ("dt_dsmc", "f8"), ("p_relax", "f8"),
                        ("a_max", "f8"), ("pre_sum", "f8", (4,)), ("post_sum", "f8", (4,))])

_lib = None


def lib():
    """Load libhs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhs.so is not built; run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P, V = C.POINTER, C.c_void_p
        sig = {
            "hs_plan": ([P(HsGas), P(HsCase), C.c_int, C.c_int, C.c_uint32, P(C.c_size_t)], C.c_int),
            "hs_init_particles": ([P(HsGas), P(HsCase), C.c_int, C.c_int, C.c_uint32, V, C.c_size_t, V, P(V)], C.c_int),
            "hs_init_particles_static": ([P(HsGas), P(HsCase), C.c_int, C.c_int, C.c_uint32, V, C.c_size_t, V,
                                          P(V)], C.c_int),
            "hs_step": ([V, C.c_int64], C.c_int),
            "hs_sync": ([V], C.c_int),
            "hs_sample_moments": ([V, C.c_int, C.c_int, P(C.c_double), P(C.c_double), P(C.c_double),
                                   P(C.c_double), P(C.c_int64)], C.c_int),
            "hs_state_bytes": ([V, C.c_int], C.c_size_t),
            "hs_export_state": ([V, C.c_int, V, C.c_size_t], C.c_int),
            "hs_import_state": ([V, C.c_int, V, C.c_size_t], C.c_int),
            "hs_last_trace": ([V, C.c_int, V], C.c_int),
            "hs_counters": ([V, C.c_int, P(C.c_int64)], C.c_int),
            "hs_num_cells": ([V, C.c_int], C.c_int64),
            "hs_num_particles": ([V, C.c_int], C.c_int64),
            "hs_set_timing": ([V, C.c_uint32], C.c_int),
            "hs_set_timing_period": ([V, C.c_int], C.c_int),
            "hs_kernel_timing": ([V, C.c_int, P(C.c_double), P(C.c_int64)], C.c_int),
            "hs_clear_timing": ([V], C.c_int),
            "hs_autotune": ([V, C.c_int, P(HsTuneReport)], C.c_int),
            "hs_set_grid": ([V, C.c_int, C.c_int32], C.c_int),
            "hs_surface_sums": ([V, C.c_int, P(C.c_double)], C.c_int),
            "hs_step_dt": ([V, C.c_int, P(C.c_double), P(C.c_double)], C.c_int),
            "hs_dsmc_ratio": ([V, C.c_int, P(C.c_double)], C.c_int),
            "hs_surface_sample": ([V, C.c_int, P(C.c_double), P(C.c_double), P(C.c_int64)], C.c_int),
            "hs_error_string": ([V], C.c_char_p),
            "hs_destroy": ([V], None),
            "hs_debug_philox": ([C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int64, V, V], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return ["hs_plan", "hs_init_particles", "hs_init_particles_static", "hs_step", "hs_sync", "hs_sample_moments", "hs_state_bytes",
            "hs_export_state", "hs_import_state", "hs_last_trace", "hs_counters", "hs_num_cells",
            "hs_num_particles", "hs_set_timing", "hs_set_timing_period", "hs_kernel_timing", "hs_clear_timing", "hs_autotune", "hs_set_grid",
            "hs_surface_sums", "hs_surface_sample", "hs_step_dt", "hs_dsmc_ratio", "hs_error_string", "hs_destroy",
            "hs_debug_philox"]


def make_gas(g: dict) -> HsGas:
    return HsGas(*(float(g[k]) for k in ("m", "d_ref", "T_ref", "omega", "mu_ref", "Pr", "gamma")))


def _state(s: dict) -> HsState:
    return HsState(float(s["n"]), (C.c_double * 3)(*s["u"]), float(s["T"]))


class _Cases:
    """ctypes array of HsCase plus the buffers its pointers refer to."""

    def __init__(self, cases):
        self.keep = []
        arr = (HsCase * len(cases))()
        for i, d in enumerate(cases):
            c = arr[i]
            c.dim, c.nx, c.ny, c.nz = int(d["dim"]), int(d["nx"]), int(d["ny"]), int(d["nz"])
            c.lo = (C.c_double * 3)(*d["lo"])
            c.h = (C.c_double * 3)(*d["h"])
            c.bc = (C.c_int32 * 6)(*[BC[b] for b in d["bc"]])
            c.inflow = _state(d["inflow"])
            c.slot_lo = (C.c_double * 3)(*d["slot_lo"])
            c.slot_hi = (C.c_double * 3)(*d["slot_hi"])
            c.body = BODY[d["body"]]
            c.body_c = (C.c_double * 3)(*d["body_c"])
            c.body_r, c.body_T = float(d["body_r"]), float(d["body_T"])
            regs = d["regions"]
            c.n_regions = len(regs)
            if regs:
                box = np.ascontiguousarray(np.array([r[0] for r in regs], np.float64).reshape(-1))
                sts = (HsState * len(regs))(*[_state(r[1]) for r in regs])
                self.keep += [box, sts]
                c.region_box = box.ctypes.data_as(C.POINTER(C.c_double))
                c.region_state = sts
            c.F_N, c.dt_G, c.T_sigma = float(d["F_N"]), float(d["dt_G"]), float(d["T_sigma"])
            if d.get("dt_over_tau") is not None:
                r = np.ascontiguousarray(np.asarray(d["dt_over_tau"], np.float64))
                self.keep.append(r)
                c.dt_over_tau = r.ctypes.data_as(C.POINTER(C.c_double))
            c.seed = int(d["seed"])
            c.n_steady = int(d["n_steady"])
            c.capacity = int(d["capacity"])
            c.n_surf = int(d.get("n_surf", 0))
            c.adapt_dt = int(bool(d.get("adapt_dt", False)))
            if d.get("mesh") is not None:
                m = d["mesh"]
                xy = np.ascontiguousarray(np.asarray(m["xy"], np.float64).reshape(-1))
                quad = np.ascontiguousarray(np.asarray(m["quad"], np.int32).reshape(-1))
                nbr = np.ascontiguousarray(np.array(
                    [EDGE[v] if isinstance(v, str) else int(v) for v in np.asarray(m["nbr"]).reshape(-1)],
                    np.int32))
                dn, vn = (3, 8) if int(d["dim"]) == 3 else (2, 4)   # coordinates, nodes per cell
                hm = HsMesh(xy.size // dn, quad.size // vn, xy.ctypes.data_as(C.POINTER(C.c_double)),
                            quad.ctypes.data_as(C.POINTER(C.c_int32)), nbr.ctypes.data_as(C.POINTER(C.c_int32)))
                self.keep += [xy, quad, nbr, hm]
                c.mesh = C.pointer(hm)
        self.arr = arr
        self.n = len(cases)


def plan_bytes(gas: dict, cases, precision=FP64, flags=0) -> int:
    cs = _Cases(cases if isinstance(cases, (list, tuple)) else [cases])
    g = make_gas(gas)
    nb = C.c_size_t()
    rc = lib().hs_plan(C.byref(g), cs.arr, cs.n, precision, flags, C.byref(nb))
    if rc:
        raise HsError(rc, "hs_plan")
    return nb.value


class Sim:
    """A batch of flow cases on one GPU.  `precision` is "fp64" or "fp32" (FP32-mixed)."""

    def __init__(self, gas: dict, cases, precision="fp64", trace=False, graph=False,
                 no_particles=False, device="cuda:0", static_scratch=False):
        """static_scratch: make the sim with hs_init_particles_static (the step's scratch in
        the library's fixed device array; this binding then allocates only the data part)."""
        import torch
        if isinstance(cases, dict):
            cases = [cases]
        self.L = lib()
        self.torch = torch
        self.device = torch.device(device)
        self.prec = FP64 if precision in ("fp64", FP64) else FP32_MIXED
        self.es = 8 if self.prec == FP64 else 4
        self.rdt = np.float64 if self.prec == FP64 else np.float32
        self.flags = (FLAG_TRACE if trace else 0) | (FLAG_GRAPH if graph else 0) | \
                     (FLAG_NO_PARTICLES if no_particles else 0)
        self.cases = list(cases)
        self._cs = _Cases(self.cases)
        self._gas = make_gas(gas)
        nb = C.c_size_t()
        plan_flags = self.flags | (FLAG_STATIC_SCRATCH if static_scratch else 0)
        rc = self.L.hs_plan(C.byref(self._gas), self._cs.arr, self._cs.n, self.prec, plan_flags, C.byref(nb))
        if rc:
            raise HsError(rc, "hs_plan rejected the cases")
        self.ws_bytes = nb.value
        with torch.cuda.device(self.device):
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            # a stream of its own (default priority): graph capture is not allowed on the
            # legacy default stream
            self.stream = torch.cuda.Stream(device=self.device)
            torch.cuda.current_stream(self.device).synchronize()
        h = C.c_void_p()
        init = self.L.hs_init_particles_static if static_scratch else self.L.hs_init_particles
        rc = init(C.byref(self._gas), self._cs.arr, self._cs.n, self.prec, self.flags,
                  C.c_void_p(self.ws.data_ptr()), self.ws_bytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self.h = h
        if rc:
            msg = self.error() if h.value else "hs_init_particles"
            raise HsError(rc, msg)

    # -- lifecycle ------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.L.hs_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return self.L.hs_error_string(self.h).decode()

    def _check(self, rc, what):
        if rc:
            raise HsError(rc, "%s: %s" % (what, self.error()))

    # -- the step ---------------------------------------------------------------------
    def step(self, n: int = 1):
        self._check(self.L.hs_step(self.h, int(n)), "hs_step")

    def sync(self):
        self._check(self.L.hs_sync(self.h), "hs_sync")

    # -- output -----------------------------------------------------------------------
    def num_cells(self, c=0) -> int:
        return int(self.L.hs_num_cells(self.h, c))

    def num_particles(self, c=0) -> int:
        n = int(self.L.hs_num_particles(self.h, c))
        if n < 0:
            self._check(self.L.hs_sync(self.h) or 5, "hs_num_particles")
        return n

    def sample_moments(self, c=0, mode=0) -> dict:
        nc = self.num_cells(c)
        n, T = np.zeros(nc), np.zeros(nc)
        u, q = np.zeros((nc, 3)), np.zeros((nc, 3))
        ns = C.c_int64()
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(self.L.hs_sample_moments(self.h, c, mode, dp(n), dp(u), dp(T), dp(q), C.byref(ns)),
                    "hs_sample_moments")
        return dict(n=n, u=u, T=T, q=q, n_samples=ns.value)

    def _n_surf(self, c):
        return int(self.cases[c].get("n_surf", 0))

    def step_dt(self, c=0):
        """(global step the next step of case c will use, sampled time so far)."""
        dt, ts = C.c_double(), C.c_double()
        self._check(self.L.hs_step_dt(self.h, c, C.byref(dt), C.byref(ts)), "hs_step_dt")
        return dt.value, ts.value

    def dsmc_ratio(self, c=0) -> np.ndarray:
        """Ratio of DSMC (Dt_DSMC / Dt_G) per cell from the time-averaged moments."""
        out = np.zeros(self.num_cells(c))
        self._check(self.L.hs_dsmc_ratio(self.h, c, out.ctypes.data_as(C.POINTER(C.c_double))), "hs_dsmc_ratio")
        return out

    def surface_sums(self, c=0) -> np.ndarray:
        """Raw body wall sums of case c, (n_surf, 7): reflections, sum dP.n, sum dP.t, sum dE,
        sum dP (x, y, z)."""
        out = np.zeros((self._n_surf(c), 7))
        self._check(self.L.hs_surface_sums(self.h, c, out.ctypes.data_as(C.POINTER(C.c_double))),
                    "hs_surface_sums")
        return out

    def surface_sample(self, c=0) -> dict:
        """Time-averaged wall quantities (Eq. 35-36): per element theta (mid), area, p, tau, q,
        Cp, Cf, Ch; for the body the force per unit time and CD, CL."""
        e, b = np.zeros((self._n_surf(c), 8)), np.zeros(5)
        k = C.c_int64()
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(self.L.hs_surface_sample(self.h, c, dp(e), dp(b), C.byref(k)), "hs_surface_sample")
        out = {n: e[:, i].copy() for i, n in enumerate(("theta", "area", "p", "tau", "q", "Cp", "Cf", "Ch"))}
        out.update(force=b[:3].copy(), CD=float(b[3]), CL=float(b[4]), n_samples=k.value)
        return out

    def trace(self, c=0) -> np.ndarray:
        out = np.zeros(self.num_cells(c), dtype=TRACE_DTYPE)
        self._check(self.L.hs_last_trace(self.h, c, out.ctypes.data), "hs_last_trace")
        return out

    def counters(self, c=0) -> dict:
        out = (C.c_int64 * len(COUNTERS))()
        self._check(self.L.hs_counters(self.h, c, out), "hs_counters")
        return {k: int(v) for k, v in zip(COUNTERS, out)}

    # -- checkpoints ----------------------------------------------------------------------
    def export_raw(self, c=0) -> bytes:
        nb = int(self.L.hs_state_bytes(self.h, c))
        if nb == 0:
            self._check(self.L.hs_sync(self.h) or 5, "hs_state_bytes")
        buf = C.create_string_buffer(nb)
        self._check(self.L.hs_export_state(self.h, c, buf, nb), "hs_export_state")
        return buf.raw

    def export_state(self, c=0) -> dict:
        raw = self.export_raw(c)
        hd = HsStateHeader.from_buffer_copy(raw[:C.sizeof(HsStateHeader)])
        np_, nc = hd.np, hd.ncells
        o = C.sizeof(HsStateHeader)
        rdt = np.float64 if hd.precision == FP64 else np.float32
        es = np.dtype(rdt).itemsize
        pos = np.frombuffer(raw, rdt, 3 * np_, o).reshape(3, np_).T.copy(); o += 3 * es * np_
        vel = np.frombuffer(raw, rdt, 3 * np_, o).reshape(3, np_).T.copy(); o += 3 * es * np_
        cell = np.frombuffer(raw, np.int32, np_, o).copy(); o += 4 * np_
        ids = np.frombuffer(raw, np.int64, np_, o).copy(); o += 8 * np_
        sigc = np.frombuffer(raw, np.float64, nc, o).copy(); o += 8 * nc
        acc = np.frombuffer(raw, np.float64, 13 * nc, o).reshape(nc, 13).copy()
        return dict(pos=pos, vel=vel, cell=cell, id=ids, sigc_max=sigc, acc=acc, next_id=hd.next_id,
                    step=hd.step, n_samples=hd.n_samples, dim=hd.dim, precision=hd.precision,
                    dt_next=hd.dt_next, t_sampled=hd.t_sampled)

    def import_state(self, c, st: dict):
        rdt = self.rdt
        pos = np.asarray(st["pos"], rdt).reshape(-1, 3)
        if rdt == np.float32 and self.cases[c].get("mesh") is None:
            # an FP64 offset just below 1 rounds to 1.0f: keep it inside its cell
            pos = np.minimum(pos, np.nextafter(np.float32(1.0), np.float32(0.0)))
        vel = np.asarray(st["vel"], rdt).reshape(-1, 3)
        np_ = vel.shape[0]
        nc = self.num_cells(c)
        ns = int(st.get("n_samples", 0))
        dt0 = float(self.cases[c]["dt_G"])
        hd = HsStateHeader(MAGIC, 2, self.prec, int(self.cases[c]["dim"]), np_, nc, int(st["next_id"]),
                           int(st["step"]), ns, float(st.get("dt_next", dt0)),
                           float(st.get("t_sampled", ns * dt0)))
        sigc = np.asarray(st["sigc_max"], np.float64).reshape(nc)
        acc = np.asarray(st.get("acc", np.zeros((nc, 13))), np.float64).reshape(nc, 13)
        parts = [bytes(hd), np.ascontiguousarray(pos.T).tobytes(), np.ascontiguousarray(vel.T).tobytes(),
                 np.asarray(st["cell"], np.int32).tobytes(), np.asarray(st["id"], np.int64).tobytes(),
                 sigc.tobytes(), acc.tobytes()]
        raw = b"".join(parts)
        buf = C.create_string_buffer(raw, len(raw))
        self._check(self.L.hs_import_state(self.h, c, buf, len(raw)), "hs_import_state")

    # -- timing -------------------------------------------------------------------------
    def set_timing(self, groups=True, period=1):
        """Time kernel groups with HIP events: True = all, False/None = off, or an iterable
        of names from KERNELS; with period k the events are recorded in every k-th step."""
        if groups is True:
            mask = (1 << len(KERNELS)) - 1
        elif not groups:
            mask = 0
        else:
            mask = 0
            for g in groups:
                mask |= 1 << KERNELS[g]
        self._check(self.L.hs_set_timing(self.h, mask), "hs_set_timing")
        self._check(self.L.hs_set_timing_period(self.h, int(period)), "hs_set_timing_period")

    def kernel_timing(self, which="collide"):
        ms, n = C.c_double(), C.c_int64()
        self._check(self.L.hs_kernel_timing(self.h, KERNELS[which], C.byref(ms), C.byref(n)), "hs_kernel_timing")
        return ms.value, n.value

    def clear_timing(self):
        self._check(self.L.hs_clear_timing(self.h), "hs_clear_timing")

    # -- launch shapes --------------------------------------------------------------------
    def autotune(self, steps_per_trial=10) -> dict:
        """Pick the grid size of each tunable kernel group by timing candidates on the live
        run (the simulation advances by the returned `steps`; results do not depend on it)."""
        r = HsTuneReport()
        self._check(self.L.hs_autotune(self.h, int(steps_per_trial), C.byref(r)), "hs_autotune")
        out = {k: (int(r.grid[i]), float(r.ms[i])) for k, i in KERNELS.items() if r.grid[i] > 0}
        return dict(grids=out, steps=int(r.steps))

    def set_grid(self, which, blocks):
        self._check(self.L.hs_set_grid(self.h, KERNELS[which], int(blocks)), "hs_set_grid")


def debug_philox(seed, stream, first, step, draw, n, device="cuda:0") -> np.ndarray:
    """Philox4x32-10 words computed by the GPU for entities first..first+n-1."""
    import torch
    out = torch.empty(4 * n, dtype=torch.int32, device=device)
    s = torch.cuda.current_stream(torch.device(device))
    rc = lib().hs_debug_philox(seed, stream, first, step, draw, n, C.c_void_p(out.data_ptr()),
                               C.c_void_p(s.cuda_stream))
    if rc:
        raise HsError(rc, "hs_debug_philox")
    return out.cpu().numpy().view(np.uint32).reshape(n, 4)
