"""ctypes wrapper of the one-dimensional D1Q3 CPU oracle (dugks_oracle1d.c):
B(phi, x, t) = b(x, t) phi with b = (p0 + p1 t) x + q0 exp(q1 t + q2 t^2),
D = (r0 + r1 t) phi, C = 0, R_i = w_i c_i dB/dt / c_s^2 (Remark 3).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .oracle import build, library_path1

_LIB = None
_d = C.POINTER(C.c_double)
_i = C.POINTER(C.c_int)


def _lib():
    global _LIB
    if _LIB is None:
        path = library_path1(False)
        if not os.path.exists(path):
            build()
        lib = C.CDLL(path)
        lib.or1_create.restype = C.c_void_p
        lib.or1_create.argtypes = [C.c_int, _d, C.c_double, C.c_double, C.c_double, C.c_int, _d]
        lib.or1_destroy.argtypes = [C.c_void_p]
        lib.or1_constants.argtypes = [C.c_void_p, _d]
        lib.or1_time.restype = C.c_double
        lib.or1_time.argtypes = [C.c_void_p]
        lib.or1_set_time.argtypes = [C.c_void_p, C.c_double]
        lib.or1_feq.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, _d]
        lib.or1_rdist.argtypes = [C.c_void_p, C.c_double, _d]
        lib.or1_set_phi.argtypes = [C.c_void_p, _d]
        lib.or1_set_state.argtypes = [C.c_void_p, _d, _d]
        lib.or1_get_f.argtypes = [C.c_void_p, _d]
        lib.or1_get_phi_prev.argtypes = [C.c_void_p, _d]
        lib.or1_get_phi.argtypes = [C.c_void_p, _d]
        lib.or1_step.argtypes = [C.c_void_p, C.c_int, _d]
        lib.or1_step_cells.argtypes = [C.c_void_p, C.c_int, _i, _d, _d]
        lib.or1_errors.argtypes = [C.c_void_p, _d, _d, _d]
        lib.or1_mass.restype = C.c_double
        lib.or1_mass.argtypes = [C.c_void_p]
        _LIB = lib
    return _LIB


def _p(a):
    return a.ctypes.data_as(_d)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle1D:
    """One D1Q3 instance advanced by the plain CPU oracle.

    problem: an object with xf, c, cfl, alpha, bc (0 periodic, 1 Dirichlet),
    coef (p0, p1, q0, q1, q2, r0, r1), t0, phi0 [nx] (or None) and, for
    Dirichlet walls, ghost(t) -> (phi at the left ghost centre, right)."""

    def __init__(self, problem):
        self.lib = _lib()
        self.problem = problem
        self.xf = _f64(problem.xf)
        self.nx = len(self.xf) - 1
        self._coef = _f64(problem.coef)
        self.h = self.lib.or1_create(self.nx, _p(self.xf), problem.c, problem.cfl, problem.alpha,
                                     int(problem.bc), _p(self._coef))
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.lib.or1_set_time(self.h, float(getattr(problem, "t0", 0.0)))
        if problem.phi0 is not None:
            self.set_phi(problem.phi0)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.or1_destroy(self.h)
            self.h = None

    @property
    def constants(self) -> dict:
        out = np.zeros(4)
        self.lib.or1_constants(self.h, _p(out))
        return dict(zip(["lambda", "dt", "h", "cs2"], out.tolist()))

    @property
    def dt(self) -> float:
        return self.constants["dt"]

    @property
    def time(self) -> float:
        return self.lib.or1_time(self.h)

    def feq(self, phi, x, t) -> np.ndarray:
        out = np.zeros(3)
        self.lib.or1_feq(self.h, float(phi), float(x), float(t), _p(out))
        return out

    def rdist(self, dB) -> np.ndarray:
        out = np.zeros(3)
        self.lib.or1_rdist(self.h, float(dB), _p(out))
        return out

    def set_phi(self, phi):
        self._tmp = _f64(phi).reshape(self.nx)
        self.lib.or1_set_phi(self.h, _p(self._tmp))

    def set_state(self, f, phi_prev):
        f = _f64(f).reshape(3, self.nx)
        pp = _f64(phi_prev).reshape(self.nx)
        self.lib.or1_set_state(self.h, _p(f), _p(pp))

    def get_f(self) -> np.ndarray:
        out = np.zeros((3, self.nx))
        self.lib.or1_get_f(self.h, _p(out))
        return out

    def get_phi(self) -> np.ndarray:
        out = np.zeros(self.nx)
        self.lib.or1_get_phi(self.h, _p(out))
        return out

    def get_phi_prev(self) -> np.ndarray:
        out = np.zeros(self.nx)
        self.lib.or1_get_phi_prev(self.h, _p(out))
        return out

    def _ghosts(self, nsteps):
        g = np.zeros(2 * max(nsteps, 1))
        if int(self.problem.bc) == 1:
            t0, dt = self.time, self.dt
            for s in range(nsteps):
                g[2 * s:2 * s + 2] = self.problem.ghost(t0 + s * dt)
        return g

    def step(self, nsteps: int = 1):
        g = self._ghosts(nsteps)
        self.lib.or1_step(self.h, int(nsteps), _p(g))

    def step_cells(self, cells) -> np.ndarray:
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        out = np.zeros((len(cells), 3))
        g = self._ghosts(1)
        self.lib.or1_step_cells(self.h, len(cells), cells.ctypes.data_as(_i), _p(g), _p(out))
        return out

    def errors(self, phi_a):
        phi_a = _f64(phi_a).reshape(self.nx)
        gre, l2 = C.c_double(), C.c_double()
        self.lib.or1_errors(self.h, _p(phi_a), C.byref(gre), C.byref(l2))
        return gre.value, l2.value

    def mass(self) -> float:
        return self.lib.or1_mass(self.h)
