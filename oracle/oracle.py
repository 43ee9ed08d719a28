"""ctypes wrapper of the plain FP64 CPU oracle (``swe_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check
and by the CPU-baseline leg of ``bench.py``.  The product path never imports it.

Coefficient arrays use the layout ``[element][component (xi, U, V)][mode]``
with ``K(p_max)`` modes in the physical orthonormal basis, element order as
given by the caller.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "swe_oracle.c")
LIB = os.path.join(HERE, "_build", "liboracle.so")
K_OF_P = (1, 3, 6, 10)

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, no fast-math)."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-fPIC", "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.c_int, dp, dp, C.c_int, ip, C.POINTER(C.c_byte), C.c_int]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_physics.argtypes = [vp, C.c_double, C.c_double, C.c_int, C.c_double]
        L.orc_set_open.argtypes = [vp, C.c_int, dp, dp, dp]
        L.orc_set_order.argtypes = [vp, ip]
        L.orc_get_order.argtypes = [vp, ip]
        L.orc_set_source.argtypes = [vp, dp]
        L.orc_set_exact_H.argtypes = [vp, C.c_int]
        L.orc_usolve.argtypes = [vp, dp, dp]
        L.orc_rhs.argtypes = [vp, C.c_double, dp, dp]
        L.orc_step.argtypes = [vp, C.c_int, C.c_double, C.c_double, dp, C.c_int, C.c_double,
                               C.c_int, C.c_int]
        L.orc_mass.restype = C.c_double
        L.orc_mass.argtypes = [vp, dp]
        L.orc_indicator.argtypes = [vp, C.c_double, dp, dp]
        L.orc_adapt.argtypes = [vp, C.c_double, dp, C.c_double, C.c_int, C.c_int]
        L.orc_quad_points.argtypes = [vp, C.c_int, dp]
        L.orc_project.argtypes = [vp, C.c_int, dp, dp]
        L.orc_eval.argtypes = [vp, dp, C.c_int, C.c_double, C.c_double, dp]
        L.orc_basis.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp]
        L.orc_basis_coeffs.argtypes = [dp]
        L.orc_neighbours.argtypes = [vp, ip, ip]
        L.orc_depth_limit.argtypes = [vp, dp, C.c_double]
        L.orc_set_depth_limit.argtypes = [vp, C.c_double]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def basis(K: int, x: float, y: float):
    """Values and reference gradients of the first K oracle basis functions."""
    phi, dx, dy = np.zeros(10), np.zeros(10), np.zeros(10)
    lib().orc_basis(K, x, y, _d(phi), _d(dx), _d(dy))
    return phi[:K], dx[:K], dy[:K]


class Oracle:
    """One discretised problem: mesh, bathymetry, physics, forcing, orders."""

    def __init__(self, vxy, hb_vertex, tri, tag, p_max, *, g=9.81, f_coriolis=0.0,
                 friction=0, friction_coef=0.0, forcing=None, order=None):
        self.L = lib()
        self.vxy = np.ascontiguousarray(vxy, np.float64)
        self.hb = np.ascontiguousarray(hb_vertex, np.float64)
        self.tri = np.ascontiguousarray(tri, np.int32)
        self.tag = np.ascontiguousarray(tag, np.int8)
        self.ne = self.tri.shape[0]
        self.p_max = int(p_max)
        self.K = K_OF_P[self.p_max]
        h = self.L.orc_create(self.vxy.shape[0], _d(self.vxy), _d(self.hb), self.ne, _i(self.tri),
                              self.tag.ctypes.data_as(C.POINTER(C.c_byte)), self.p_max)
        if not h:
            raise ValueError("oracle rejected the mesh")
        self.h = C.c_void_p(h)
        if self.L.orc_set_physics(self.h, g, f_coriolis, friction, friction_coef) != 0:
            raise ValueError("bad physics parameters")
        if forcing is not None and len(forcing.amp):
            a = np.asarray(forcing.amp, np.float64)
            w = np.asarray(forcing.omega, np.float64)
            ph = np.asarray(forcing.phase, np.float64)
            self.L.orc_set_open(self.h, len(a), _d(a), _d(w), _d(ph))
        if order is not None:
            self.set_order(order)

    @classmethod
    def from_problem(cls, prob):
        o = cls(prob.mesh.vxy, prob.hb_vertex, prob.mesh.tri, prob.mesh.tag, prob.p_max,
                g=prob.g, f_coriolis=prob.f_coriolis, friction=prob.friction,
                friction_coef=prob.friction_coef, forcing=prob.forcing, order=prob.p)
        if getattr(prob, "h_min", 0.0) > 0.0:
            o.set_depth_limit(prob.h_min)
        return o

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.L.orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # -- configuration
    def set_order(self, p):
        p = np.ascontiguousarray(p, np.int32)
        if self.L.orc_set_order(self.h, _i(p)) != 0:
            raise ValueError("order out of range")

    def order(self):
        p = np.zeros(self.ne, np.int32)
        self.L.orc_get_order(self.h, _i(p))
        return p

    def set_source(self, src):
        if src is None:
            self.L.orc_set_source(self.h, None)
        else:
            s = np.ascontiguousarray(src, np.float64)
            self.L.orc_set_source(self.h, _d(s))

    def set_exact_H(self, on: bool):
        self.L.orc_set_exact_H(self.h, int(bool(on)))

    def _c(self, c):
        c = np.ascontiguousarray(c, np.float64)
        assert c.shape == (self.ne, 3, self.K), c.shape
        return c

    # -- the method
    def usolve(self, c):
        c = self._c(c)
        u = np.zeros((self.ne, 2, self.K))
        rc = self.L.orc_usolve(self.h, _d(c), _d(u))
        if rc:
            raise FloatingPointError(f"u-solve failed ({rc})")
        return u

    def rhs(self, t, c):
        c = self._c(c)
        L = np.zeros_like(c)
        rc = self.L.orc_rhs(self.h, float(t), _d(c), _d(L))
        if rc:
            raise FloatingPointError(f"rhs failed ({rc})")
        return L

    def step(self, c, nsteps, dt, t0=0.0, adapt=False, tau=1e-3, p_lo=1, p_hi=3):
        c = self._c(c).copy()
        rc = self.L.orc_step(self.h, int(nsteps), float(dt), float(t0), _d(c), int(bool(adapt)),
                             float(tau), int(p_lo), int(p_hi))
        if rc:
            raise FloatingPointError(f"step failed ({rc})")
        return c

    def mass(self, c):
        return float(self.L.orc_mass(self.h, _d(self._c(c))))

    def set_depth_limit(self, h_min):
        """Minimum depth control after every stage of ``step`` (0: off)."""
        if self.L.orc_set_depth_limit(self.h, float(h_min)) != 0:
            raise ValueError("h_min must be finite and >= 0")

    def depth_limit(self, c, h_min):
        """The minimum depth control applied once: (new state, elements changed)."""
        c = self._c(c).copy()
        n = self.L.orc_depth_limit(self.h, _d(c), float(h_min))
        return c, int(n)

    def indicator(self, t, c):
        I = np.zeros(self.ne)
        self.L.orc_indicator(self.h, float(t), _d(self._c(c)), _d(I))
        return I

    def adapt(self, t, c, tau, p_lo, p_hi):
        c = self._c(c).copy()
        self.L.orc_adapt(self.h, float(t), _d(c), float(tau), int(p_lo), int(p_hi))
        return c

    # -- input preparation
    def quad_points(self, n1=8):
        xy = np.zeros((self.ne, n1 * n1, 2))
        self.L.orc_quad_points(self.h, n1, _d(xy))
        return xy

    def project(self, fn, n1=8):
        """L2-project point function fn(x, y) -> (xi, U, V) onto each element's space."""
        xy = self.quad_points(n1)
        xi, U, V = fn(xy[..., 0], xy[..., 1])
        vals = np.ascontiguousarray(np.stack([xi, U, V], axis=-1), np.float64)
        c = np.zeros((self.ne, 3, self.K))
        self.L.orc_project(self.h, n1, _d(vals), _d(c))
        return c

    def project_values(self, vals, n1=8):
        vals = np.ascontiguousarray(vals, np.float64)
        c = np.zeros((self.ne, 3, self.K))
        self.L.orc_project(self.h, n1, _d(vals), _d(c))
        return c

    def eval(self, c, e, x, y):
        """Point values (xi, U, V, u, v) of element e; u, v from the last u-solve."""
        out = np.zeros(5)
        self.L.orc_eval(self.h, _d(self._c(c)), int(e), float(x), float(y), _d(out))
        return out

    def neighbours(self):
        nb = np.zeros((self.ne, 3), np.int32)
        bt = np.zeros((self.ne, 3), np.int32)
        self.L.orc_neighbours(self.h, _i(nb), _i(bt))
        return nb, bt
