"""ctypes wrapper of the three-dimensional CPU oracle (dugks_oracle3d.c).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .oracle import build, library_path3

_LIBS = {}
_d = C.POINTER(C.c_double)
_i = C.POINTER(C.c_int)


def _lib(openmp: bool = False):
    if openmp not in _LIBS:
        path = library_path3(openmp)
        if not os.path.exists(path):
            build()
        lib = C.CDLL(path)
        lib.or3_create.restype = C.c_void_p
        lib.or3_create.argtypes = [C.c_int, C.c_int, C.c_int, _d, _d, _d, C.c_int, C.c_double,
                                   C.c_double, C.c_double, C.c_int, C.c_int, C.c_int]
        lib.or3_destroy.argtypes = [C.c_void_p]
        lib.or3_set_B.argtypes = [C.c_void_p, C.c_int, _d]
        lib.or3_set_D.argtypes = [C.c_void_p, C.c_int, _d]
        lib.or3_constants.argtypes = [C.c_void_p, _d]
        lib.or3_feq.argtypes = [C.c_void_p, C.c_double, _d]
        lib.or3_set_phi.argtypes = [C.c_void_p, _d]
        lib.or3_set_f.argtypes = [C.c_void_p, _d]
        lib.or3_get_f.argtypes = [C.c_void_p, _d]
        lib.or3_get_phi.argtypes = [C.c_void_p, _d]
        lib.or3_time.restype = C.c_double
        lib.or3_time.argtypes = [C.c_void_p]
        lib.or3_step.argtypes = [C.c_void_p, C.c_int, _d]
        lib.or3_step_cells.argtypes = [C.c_void_p, C.c_int, _i, _d, _d]
        lib.or3_set_source_terms.argtypes = [C.c_void_p, C.c_int, _d, _i, _d]
        lib.or3_threads.restype = C.c_int
        lib.or3_threads.argtypes = [C.c_int]
        lib.or3_shell_len.restype = C.c_size_t
        lib.or3_shell_len.argtypes = [C.c_void_p]
        lib.or3_errors.argtypes = [C.c_void_p, _d, _d, _d]
        lib.or3_mass.restype = C.c_double
        lib.or3_mass.argtypes = [C.c_void_p]
        _LIBS[openmp] = lib
    return _LIBS[openmp]


def threads(n: int = 0, openmp: bool = True) -> int:
    """Threads of the 3-D oracle's OpenMP build (n > 0 sets them); the serial build uses 1."""
    return int(_lib(openmp).or3_threads(int(n)))


def _p(a):
    return a.ctypes.data_as(_d)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _pad(v, n):
    out = np.zeros(n)
    out[:len(v)] = v
    return out


class Oracle3D:
    """One three-dimensional DUGKS instance advanced by the plain CPU oracle.

    problem: an object with xf, yf, zf, q, c, cfl, alpha, bc (3), b (3 tuples:
    B_x, B_y, B_z coefficients), d (6 tuples: D_xx, D_yy, D_zz, D_xy, D_xz, D_yz)
    and phi0 [nz][ny][nx] (or None)."""

    def __init__(self, problem, openmp=False):
        self.lib = _lib(openmp)
        self.xf, self.yf, self.zf = _f64(problem.xf), _f64(problem.yf), _f64(problem.zf)
        self.nx, self.ny, self.nz = len(self.xf) - 1, len(self.yf) - 1, len(self.zf) - 1
        self.q = problem.q
        bc = problem.bc
        self.h = self.lib.or3_create(self.nx, self.ny, self.nz, _p(self.xf), _p(self.yf),
                                     _p(self.zf), self.q, problem.c, problem.cfl, problem.alpha,
                                     bc[0], bc[1], bc[2])
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        deg = max(len(v) for v in problem.b) - 1
        b = np.concatenate([_pad(v, deg + 1) for v in problem.b])
        if self.lib.or3_set_B(self.h, deg, _p(b)) != 0:
            raise ValueError("B degree out of range")
        deg = max(len(v) for v in problem.d) - 1
        d = np.concatenate([_pad(v, deg + 1) for v in problem.d])
        if self.lib.or3_set_D(self.h, deg, _p(d)) != 0:
            raise ValueError("D degree out of range")
        terms = getattr(problem, "src_terms", None)
        if terms:
            self.set_source_terms(terms)
        if problem.phi0 is not None:
            self.set_phi(problem.phi0)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.or3_destroy(self.h)
            self.h = None

    @property
    def constants(self) -> dict:
        out = np.zeros(10)
        self.lib.or3_constants(self.h, _p(out))
        keys = ["lambda", "dt", "h", "a1", "b1", "a2", "b2", "a3", "b3", "cs2"]
        return dict(zip(keys, out.tolist()))

    @property
    def dt(self) -> float:
        return self.constants["dt"]

    @property
    def time(self) -> float:
        return self.lib.or3_time(self.h)

    def feq(self, phi: float) -> np.ndarray:
        out = np.zeros(self.q)
        self.lib.or3_feq(self.h, float(phi), _p(out))
        return out

    def set_phi(self, phi):
        self._tmp = _f64(phi).reshape(self.nz, self.ny, self.nx)
        self.lib.or3_set_phi(self.h, _p(self._tmp))

    def set_f(self, f):
        self._tmp = _f64(f).reshape(self.q, self.nz, self.ny, self.nx)
        self.lib.or3_set_f(self.h, _p(self._tmp))

    def get_f(self) -> np.ndarray:
        out = np.zeros((self.q, self.nz, self.ny, self.nx))
        self.lib.or3_get_f(self.h, _p(out))
        return out

    def get_phi(self) -> np.ndarray:
        out = np.zeros((self.nz, self.ny, self.nx))
        self.lib.or3_get_phi(self.h, _p(out))
        return out

    def set_source_terms(self, terms):
        """F(x, t, phi) = sum_j exp(gamma_j t) phi^k_j G_j(x): terms as (k_j,
        gamma_j, G_j [nz][ny][nx]); an empty list removes the source.  Call
        before set_phi (the initial state depends on the source)."""
        n = len(terms)
        g = _f64(np.stack([np.asarray(G, dtype=np.float64).reshape(self.nz, self.ny, self.nx)
                           for _, _, G in terms])) if n else np.zeros(1)
        pw = np.ascontiguousarray([int(k) for k, _, _ in terms] or [0], dtype=np.int32)
        gm = _f64([float(gam) for _, gam, _ in terms] or [0.0])
        self._src = g
        if self.lib.or3_set_source_terms(self.h, n, _p(g), pw.ctypes.data_as(_i), _p(gm)) != 0:
            raise ValueError("bad source terms")

    def shell_len(self) -> int:
        """Boundary values of one step (the ghost shell, Dirichlet walls)."""
        return int(self.lib.or3_shell_len(self.h))

    def step(self, nsteps: int = 1, rings=None):
        """Advance nsteps; rings: [nsteps][shell_len] boundary values at the
        ghost centres, step by step (needed with Dirichlet walls)."""
        if rings is not None:
            rings = _f64(rings).reshape(nsteps, -1)
            assert rings.shape[1] == self.shell_len()
        self.lib.or3_step(self.h, int(nsteps), _p(rings) if rings is not None else None)

    def step_cells(self, cells, ring=None) -> np.ndarray:
        """One step evaluated at the listed (i, j, k) cells; the state is unchanged."""
        cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 3)
        out = np.zeros((len(cells), self.q))
        r = _f64(ring) if ring is not None else None
        self.lib.or3_step_cells(self.h, len(cells), cells.ctypes.data_as(_i),
                                _p(r) if r is not None else None, _p(out))
        return out

    def errors(self, phi_a):
        phi_a = _f64(phi_a).reshape(self.nz, self.ny, self.nx)
        gre, l2 = C.c_double(), C.c_double()
        self.lib.or3_errors(self.h, _p(phi_a), C.byref(gre), C.byref(l2))
        return gre.value, l2.value

    def mass(self) -> float:
        return self.lib.or3_mass(self.h)
