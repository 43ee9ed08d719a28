"""Python binding of the C ABI in ``include/swe_dg.h`` (argument marshalling only).

Every computation runs in ``libswe_hip.so`` on the GPU.  There is no CPU
fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libswe_hip.so")

SWE_OK, SWE_EINVAL, SWE_ENOMEM, SWE_EDEVICE, SWE_ESTATE, SWE_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SWE_FP64, SWE_FP32_WB = 0, 1
SWE_NQP = 36
K_OF_P = (1, 3, 6, 10)
_NAMES = {0: "SWE_OK", -1: "SWE_EINVAL", -2: "SWE_ENOMEM", -3: "SWE_EDEVICE", -4: "SWE_ESTATE",
          -5: "SWE_EUNSUPPORTED"}


class SweError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class swe_config(C.Structure):
    _fields_ = [("precision", C.c_int), ("p_base", C.c_int), ("p_max", C.c_int),
                ("g", C.c_double), ("f_coriolis", C.c_double), ("friction", C.c_int),
                ("friction_coef", C.c_double), ("adapt", C.c_int), ("adapt_tau", C.c_double),
                ("separate", C.c_int), ("stream_base", C.c_void_p), ("stream_corr", C.c_void_p),
                ("step_graph", C.c_int), ("hetero", C.c_int), ("host_threads", C.c_int),
                ("h_min", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load the HIP library (built by ``paper_2311_11348_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_11348_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, dp, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    i8p, i32p = C.POINTER(C.c_int8), C.POINTER(C.c_int32)
    pp = C.POINTER(C.c_void_p)
    sig = {
        "swe_config_default": (None, [C.POINTER(swe_config)]),
        "swe_create": (C.c_int, [C.POINTER(swe_config), pp]),
        "swe_set_mesh": (C.c_int, [vp, i64, dp, i64, i32p, i8p]),
        "swe_set_bathymetry": (C.c_int, [vp, dp]),
        "swe_set_order": (C.c_int, [vp, i8p]),
        "swe_get_order": (C.c_int, [vp, i8p]),
        "swe_set_open_boundary": (C.c_int, [vp, C.c_int, dp, dp, dp]),
        "swe_set_state": (C.c_int, [vp, C.c_double, dp]),
        "swe_project_points": (C.c_int, [vp, dp]),
        "swe_set_state_points": (C.c_int, [vp, C.c_double, dp]),
        "swe_set_source": (C.c_int, [vp, dp]),
        "swe_step": (C.c_int, [vp, i64, C.c_double]),
        "swe_sync": (C.c_int, [vp]),
        "swe_get_state": (C.c_int, [vp, dp, dp]),
        "swe_mass": (C.c_int, [vp, dp]),
        "swe_mass_noalloc": (C.c_int, [vp, vp]),
        "swe_rhs": (C.c_int, [vp, C.c_double, dp, dp]),
        "swe_usolve": (C.c_int, [vp, dp, dp]),
        "swe_rhs_split": (C.c_int, [vp, C.c_double, dp, dp, dp]),
        "swe_indicator": (C.c_int, [vp, C.c_double, dp, dp]),
        "swe_last_error": (C.c_char_p, [vp]),
        "swe_footprint_bytes": (C.c_int64, [i64, C.c_int, C.c_int]),
        "swe_destroy": (None, [vp]),
        "swe_num_elements": (C.c_int64, [vp]),
        "swe_num_modes": (C.c_int, [vp]),
        "swe_batch_create": (C.c_int, [C.POINTER(swe_config), i64, C.c_int, pp]),
        "swe_batch_admit": (C.c_int, [vp, vp, i64, C.c_double, C.POINTER(C.c_int32)]),
        "swe_batch_tick": (C.c_int, [vp, i64]),
        "swe_batch_sync": (C.c_int, [vp]),
        "swe_batch_query": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int64), dp, C.POINTER(C.c_int)]),
        "swe_batch_retire": (C.c_int, [vp, C.c_int32]),
        "swe_batch_tune": (C.c_int, [vp, C.c_int]),
        "swe_batch_set_tile": (C.c_int, [vp, C.c_int, C.c_int, C.c_int]),
        "swe_batch_tile_config": (C.c_int, [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                            C.POINTER(C.c_int)]),
        "swe_batch_free_bytes": (C.c_int64, [vp]),
        "swe_batch_resident": (C.c_int, [vp]),
        "swe_batch_last_error": (C.c_char_p, [vp]),
        "swe_batch_destroy": (None, [vp]),
        "swe_batch_poll": (C.c_int, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def swe_footprint_bytes(ne: int, p_max: int, precision: int) -> int:
    return int(lib().swe_footprint_bytes(int(ne), int(p_max), int(precision)))


@dataclass
class Config:
    precision: int = SWE_FP64
    p_base: int = 1
    p_max: int = 1
    g: float = 9.81
    f_coriolis: float = 0.0
    friction: int = 0
    friction_coef: float = 0.0
    adapt: int = 0
    adapt_tau: float = 1e-3
    separate: int = 0
    stream_base: Optional[int] = None
    stream_corr: Optional[int] = None
    step_graph: int = 1          # 1: graph for separated steps, 2: always, 0: never
    hetero: int = 0              # 1: correction on the host's cores beside the GPU base pass
    host_threads: int = 0        # threads of that correction (0: every usable core)
    h_min: float = 0.0           # minimum depth control after every stage (0: off)

    def to_c(self) -> swe_config:
        c = swe_config()
        lib().swe_config_default(C.byref(c))
        for k in ("precision", "p_base", "p_max", "g", "f_coriolis", "friction", "friction_coef",
                  "adapt", "adapt_tau", "separate", "step_graph", "hetero", "host_threads", "h_min"):
            setattr(c, k, getattr(self, k))
        c.stream_base = self.stream_base
        c.stream_corr = self.stream_corr
        return c


class Context:
    """One solve instance: a thin owner of a ``swe_ctx*``."""

    def __init__(self, cfg: Config):
        self.L = lib()
        self.cfg = cfg
        self._c = cfg.to_c()
        h = C.c_void_p()
        st = self.L.swe_create(C.byref(self._c), C.byref(h))
        if st != SWE_OK:
            raise SweError(st, "swe_create failed")
        self.h = h
        self.ne = 0
        self.K = K_OF_P[cfg.p_max]

    def _check(self, st: int):
        if st != SWE_OK:
            raise SweError(st, self.L.swe_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.L.swe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- setup
    def set_mesh(self, vxy, tri, tag=None):
        vxy = np.ascontiguousarray(vxy, np.float64)
        tri = np.ascontiguousarray(tri, np.int32)
        tagp = None
        if tag is not None:
            tag = np.ascontiguousarray(tag, np.int8)
            tagp = tag.ctypes.data_as(C.POINTER(C.c_int8))
        self._check(self.L.swe_set_mesh(self.h, vxy.shape[0], _d(vxy), tri.shape[0],
                                        tri.ctypes.data_as(C.POINTER(C.c_int32)), tagp))
        self.ne = tri.shape[0]

    def set_bathymetry(self, hb):
        hb = np.ascontiguousarray(hb, np.float64)
        self._check(self.L.swe_set_bathymetry(self.h, _d(hb)))

    def set_order(self, p):
        p = np.ascontiguousarray(p, np.int8)
        self._check(self.L.swe_set_order(self.h, p.ctypes.data_as(C.POINTER(C.c_int8))))

    def order(self):
        p = np.zeros(self.ne, np.int8)
        self._check(self.L.swe_get_order(self.h, p.ctypes.data_as(C.POINTER(C.c_int8))))
        return p

    def set_open_boundary(self, amp, omega, phase):
        a = np.ascontiguousarray(amp, np.float64)
        w = np.ascontiguousarray(omega, np.float64)
        ph = np.ascontiguousarray(phase, np.float64)
        self._check(self.L.swe_set_open_boundary(self.h, len(a), _d(a), _d(w), _d(ph)))

    def set_state(self, coef, t0=0.0):
        coef = np.ascontiguousarray(coef, np.float64)
        assert coef.shape == (self.ne, 3, self.K), coef.shape
        self._check(self.L.swe_set_state(self.h, float(t0), _d(coef)))

    def project_points(self):
        xy = np.zeros((self.ne, SWE_NQP, 2))
        self._check(self.L.swe_project_points(self.h, _d(xy)))
        return xy

    def set_state_fn(self, fn, t0=0.0):
        xy = self.project_points()
        xi, U, V = fn(xy[..., 0], xy[..., 1])
        vals = np.ascontiguousarray(np.stack([xi, U, V], -1), np.float64)
        self._check(self.L.swe_set_state_points(self.h, float(t0), _d(vals)))

    def set_source(self, coef):
        if coef is None:
            self._check(self.L.swe_set_source(self.h, None))
        else:
            coef = np.ascontiguousarray(coef, np.float64)
            self._check(self.L.swe_set_source(self.h, _d(coef)))

    # -- run
    def step(self, nsteps, dt):
        self._check(self.L.swe_step(self.h, int(nsteps), float(dt)))

    def sync(self):
        self._check(self.L.swe_sync(self.h))

    def state(self):
        c = np.zeros((self.ne, 3, self.K))
        t = C.c_double()
        self._check(self.L.swe_get_state(self.h, _d(c), C.byref(t)))
        return c, t.value

    def mass(self):
        m = C.c_double()
        self._check(self.L.swe_mass(self.h, C.byref(m)))
        return m.value

    def mass_noalloc(self, d_out: int):
        """Enqueue the mass reduction without allocating; the result lands in
        the device double at address d_out once the context's stream gets there."""
        self._check(self.L.swe_mass_noalloc(self.h, C.c_void_p(int(d_out))))

    # -- test hooks
    def rhs(self, t, coef):
        coef = np.ascontiguousarray(coef, np.float64)
        out = np.zeros_like(coef)
        self._check(self.L.swe_rhs(self.h, float(t), _d(coef), _d(out)))
        return out

    def rhs_split(self, t, coef):
        coef = np.ascontiguousarray(coef, np.float64)
        b, c = np.zeros_like(coef), np.zeros_like(coef)
        self._check(self.L.swe_rhs_split(self.h, float(t), _d(coef), _d(b), _d(c)))
        return b, c

    def usolve(self, coef):
        coef = np.ascontiguousarray(coef, np.float64)
        u = np.zeros((self.ne, 2, self.K))
        self._check(self.L.swe_usolve(self.h, _d(coef), _d(u)))
        return u

    def indicator(self, t, coef):
        coef = np.ascontiguousarray(coef, np.float64)
        I = np.zeros(self.ne)
        self._check(self.L.swe_indicator(self.h, float(t), _d(coef), _d(I)))
        return I


def context_for(problem, precision=SWE_FP64, separate=0, stream_base=None, stream_corr=None,
                step_graph=1, hetero=0, host_threads=0, h_min=None) -> Context:
    """Build a context from an ``inputs.Problem`` (mesh, bathymetry, forcing, orders)."""
    cfg = Config(precision=precision, p_base=problem.p_base, p_max=problem.p_max, g=problem.g,
                 f_coriolis=problem.f_coriolis, friction=problem.friction,
                 friction_coef=problem.friction_coef, adapt=problem.adapt,
                 adapt_tau=problem.adapt_tau, separate=separate, stream_base=stream_base,
                 stream_corr=stream_corr, step_graph=step_graph, hetero=hetero, host_threads=host_threads,
                 h_min=getattr(problem, "h_min", 0.0) if h_min is None else h_min)
    ctx = Context(cfg)
    ctx.set_mesh(problem.mesh.vxy, problem.mesh.tri, problem.mesh.tag)
    ctx.set_bathymetry(problem.hb_vertex)
    if problem.forcing is not None and len(problem.forcing.amp):
        ctx.set_open_boundary(problem.forcing.amp, problem.forcing.omega, problem.forcing.phase)
    # separated contexts start at p_base, unseparated ones at p_max
    if separate or np.any(problem.p != problem.p_max):
        ctx.set_order(problem.p)
    return ctx


class Batch:
    """Many independent instances advanced together (see swe_batch_* in the header)."""

    def __init__(self, precision=SWE_FP64, budget_bytes=64 << 30, max_instances=1024, stream=None):
        self.L = lib()
        cfg = Config(precision=precision, stream_base=stream)
        self._c = cfg.to_c()
        h = C.c_void_p()
        st = self.L.swe_batch_create(C.byref(self._c), int(budget_bytes), int(max_instances), C.byref(h))
        if st != SWE_OK:
            raise SweError(st, "swe_batch_create failed")
        self.h = h
        self.members = {}

    def _check(self, st):
        if st != SWE_OK:
            raise SweError(st, self.L.swe_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.L.swe_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def admit(self, ctx: Context, nsteps: int, dt: float) -> int:
        slot = C.c_int32()
        self._check(self.L.swe_batch_admit(self.h, ctx.h, int(nsteps), float(dt), C.byref(slot)))
        self.members[slot.value] = ctx
        return slot.value

    def tick(self, nsteps: int):
        self._check(self.L.swe_batch_tick(self.h, int(nsteps)))

    def sync(self):
        self._check(self.L.swe_batch_sync(self.h))

    def query(self, slot: int):
        left, t, failed = C.c_int64(), C.c_double(), C.c_int()
        self._check(self.L.swe_batch_query(self.h, int(slot), C.byref(left), C.byref(t), C.byref(failed)))
        return left.value, t.value, bool(failed.value)

    def poll(self, max_slots: int = 4096):
        """Slots that are done or failed: list of (slot, failed)."""
        slots = (C.c_int32 * max_slots)()
        failed = (C.c_int32 * max_slots)()
        n = C.c_int()
        self._check(self.L.swe_batch_poll(self.h, slots, failed, max_slots, C.byref(n)))
        return [(slots[i], bool(failed[i])) for i in range(n.value)]

    def retire(self, slot: int) -> Context:
        self._check(self.L.swe_batch_retire(self.h, int(slot)))
        return self.members.pop(slot)

    def tune(self, reps: int = 3):
        self._check(self.L.swe_batch_tune(self.h, int(reps)))

    def set_tile(self, p: int, tile: int, shared: bool = False):
        """Pick order p's kernel by hand (instead of tune())."""
        self._check(self.L.swe_batch_set_tile(self.h, int(p), int(tile), 1 if shared else 0))

    def tile_config(self, p: int):
        """(tile size, grid, shared-flux kernel) of order p."""
        t, g, sh = C.c_int(), C.c_int(), C.c_int()
        self._check(self.L.swe_batch_tile_config(self.h, int(p), C.byref(t), C.byref(g), C.byref(sh)))
        return t.value, g.value, bool(sh.value)

    def free_bytes(self) -> int:
        return int(self.L.swe_batch_free_bytes(self.h))

    def resident(self) -> int:
        return int(self.L.swe_batch_resident(self.h))
