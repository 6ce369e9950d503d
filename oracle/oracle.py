"""ctypes wrapper around the plain C oracle ``dugks_oracle.c``.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the
benchmark's CPU baseline.  Shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dugks_oracle.c")


def library_path(openmp: bool = False) -> str:
    return os.path.join(HERE, "liboracle_omp.so" if openmp else "liboracle.so")


SRC3 = os.path.join(HERE, "dugks_oracle3d.c")


def library_path3(openmp: bool = False) -> str:
    return os.path.join(HERE, "liboracle3d_omp.so" if openmp else "liboracle3d.so")


SRC1 = os.path.join(HERE, "dugks_oracle1d.c")


def library_path1(openmp: bool = False) -> str:
    return os.path.join(HERE, "liboracle1d_omp.so" if openmp else "liboracle1d.so")


def build(verbose: bool = False) -> None:
    """Compile the oracles (1-D, 2-D, 3-D): plain -O2, no FMA contraction, no fast-math."""
    for src, path in ((SRC, library_path), (SRC3, library_path3), (SRC1, library_path1)):
        for omp in (False, True):
            cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC",
                   "-shared", "-o", path(omp) + ".tmp", src, "-lm"]
            if omp:
                cmd.insert(1, "-fopenmp")
            if verbose:
                print(" ".join(cmd))
            subprocess.check_call(cmd)
            os.replace(path(omp) + ".tmp", path(omp))


_LIBS = {}
_d = C.POINTER(C.c_double)
_i = C.POINTER(C.c_int)


def _lib(openmp: bool = False):
    if openmp not in _LIBS:
        path = library_path(openmp)
        if not os.path.exists(path):
            build()
        lib = C.CDLL(path)
        lib.or_create.restype = C.c_void_p
        lib.or_create.argtypes = [C.c_int, C.c_int, _d, _d, C.c_int, C.c_double, C.c_double,
                                  C.c_double, C.c_int, C.c_int]
        lib.or_destroy.argtypes = [C.c_void_p]
        lib.or_set_B.argtypes = [C.c_void_p, C.c_int, _d, _d]
        lib.or_set_D.argtypes = [C.c_void_p, C.c_int, _d, _d, _d]
        lib.or_set_source.argtypes = [C.c_void_p, _d, C.c_double]
        lib.or_set_source_terms.argtypes = [C.c_void_p, C.c_int, _d, C.POINTER(C.c_int), _d]
        lib.or_constants.argtypes = [C.c_void_p, _d]
        lib.or_threads.restype = C.c_int
        lib.or_threads.argtypes = [C.c_int]
        lib.or_geometry.argtypes = [C.c_void_p, _d, _d, _d, _d]
        lib.or_feq.argtypes = [C.c_void_p, C.c_double, _d]
        lib.or_set_phi.argtypes = [C.c_void_p, _d]
        lib.or_set_f.argtypes = [C.c_void_p, _d]
        lib.or_get_f.argtypes = [C.c_void_p, _d]
        lib.or_get_phi.argtypes = [C.c_void_p, _d]
        lib.or_set_clock.argtypes = [C.c_void_p, C.c_long, C.c_double]
        lib.or_step_index.restype = C.c_long
        lib.or_step_index.argtypes = [C.c_void_p]
        lib.or_time.restype = C.c_double
        lib.or_time.argtypes = [C.c_void_p]
        lib.or_step.argtypes = [C.c_void_p, C.c_int, _d]
        lib.or_step_cells.argtypes = [C.c_void_p, C.c_int, _i, _d, _d]
        lib.or_fbar_plus_all.argtypes = [C.c_void_p, _d, _d]
        lib.or_errors.argtypes = [C.c_void_p, _d, _d, _d]
        lib.or_mass.restype = C.c_double
        lib.or_mass.argtypes = [C.c_void_p]
        _LIBS[openmp] = lib
    return _LIBS[openmp]


def threads(n: int = 0, openmp: bool = True) -> int:
    """Threads of the oracle's OpenMP build (n > 0 sets them); the serial build uses 1."""
    return int(_lib(openmp).or_threads(int(n)))


def _p(a):
    return a.ctypes.data_as(_d)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One DUGKS instance advanced by the plain CPU oracle."""

    def __init__(self, problem=None, *, xf=None, yf=None, q=9, c=1.0, cfl=0.5, alpha=1e-3,
                 bcx=0, bcy=0, bx=(0.0,), by=(0.0,), dxx=(0.0, 1.0), dxy=(0.0, 0.0),
                 dyy=(0.0, 1.0), openmp=False):
        if problem is not None:
            xf, yf, q, c, cfl, alpha = (problem.xf, problem.yf, problem.q, problem.c,
                                        problem.cfl, problem.alpha)
            bcx, bcy = problem.bcx, problem.bcy
            bx, by, dxx, dxy, dyy = problem.bx, problem.by, problem.dxx, problem.dxy, problem.dyy
        self.lib = _lib(openmp)
        self.xf, self.yf = _f64(xf), _f64(yf)
        self.nx, self.ny, self.q = len(self.xf) - 1, len(self.yf) - 1, q
        self.h = self.lib.or_create(self.nx, self.ny, _p(self.xf), _p(self.yf), q, c, cfl,
                                    alpha, bcx, bcy)
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.set_B(bx, by)
        self.set_D(dxx, dxy, dyy)
        if problem is not None and getattr(problem, "src_g", None) is not None:
            self.set_source(problem.src_g, problem.src_gamma)
        if problem is not None and getattr(problem, "src_terms", None):
            self.set_source_terms(problem.src_terms)
        if problem is not None and problem.phi0 is not None:
            self.set_phi(problem.phi0)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.or_destroy(self.h)
            self.h = None

    def set_B(self, bx, by):
        deg = max(len(bx), len(by)) - 1
        a = np.zeros(deg + 1); a[:len(bx)] = bx
        b = np.zeros(deg + 1); b[:len(by)] = by
        if self.lib.or_set_B(self.h, deg, _p(a), _p(b)) != 0:
            raise ValueError("B degree out of range")

    def set_D(self, dxx, dxy, dyy):
        deg = max(len(dxx), len(dxy), len(dyy)) - 1
        arrs = []
        for v in (dxx, dxy, dyy):
            a = np.zeros(deg + 1); a[:len(v)] = v
            arrs.append(a)
        if self.lib.or_set_D(self.h, deg, *[_p(a) for a in arrs]) != 0:
            raise ValueError("D degree out of range")

    def set_source(self, g, gamma: float = 0.0):
        """F(x, t) = exp(gamma t) g(x), g [ny][nx] at the cell centres; None removes it.
        Takes effect for the next set_phi (initialisation) and step."""
        if g is None:
            self.lib.or_set_source(self.h, None, 0.0)
            return
        self._src = _f64(g).reshape(self.ny, self.nx)
        self.lib.or_set_source(self.h, _p(self._src), float(gamma))

    def set_source_terms(self, terms):
        """F(x, t, phi) = sum over terms (k, gamma, G) of exp(gamma t) phi^k G(x),
        G [ny][nx] at the cell centres, k in 0..3, at most 8 terms; an empty list
        removes the source.  Takes effect for the next set_phi and step."""
        n = len(terms)
        if n == 0:
            self.lib.or_set_source_terms(self.h, 0, None, None, None)
            return
        self._src = np.ascontiguousarray(
            np.stack([_f64(g).reshape(self.ny, self.nx) for _, _, g in terms]))
        self._pow = (C.c_int * n)(*[int(k) for k, _, _ in terms])
        self._gam = np.array([float(gm) for _, gm, _ in terms])
        if self.lib.or_set_source_terms(self.h, n, _p(self._src), self._pow, _p(self._gam)) != 0:
            raise ValueError("at most 8 source terms, powers of phi 0..3")

    @property
    def constants(self) -> dict:
        out = np.zeros(10)
        self.lib.or_constants(self.h, _p(out))
        keys = ["lambda", "dt", "h", "a1", "b1", "a2", "b2", "a3", "b3", "cs2"]
        return dict(zip(keys, out.tolist()))

    @property
    def dt(self) -> float:
        return self.constants["dt"]

    def geometry(self):
        wx, xc = np.zeros(self.nx + 2), np.zeros(self.nx + 2)
        wy, yc = np.zeros(self.ny + 2), np.zeros(self.ny + 2)
        self.lib.or_geometry(self.h, _p(wx), _p(xc), _p(wy), _p(yc))
        return wx, xc, wy, yc

    def feq(self, phi: float) -> np.ndarray:
        out = np.zeros(self.q)
        self.lib.or_feq(self.h, float(phi), _p(out))
        return out

    def set_phi(self, phi):
        phi = _f64(phi).reshape(self.ny, self.nx)
        self.lib.or_set_phi(self.h, _p(phi))

    def set_f(self, f):
        f = _f64(f).reshape(self.q, self.ny, self.nx)
        self.lib.or_set_f(self.h, _p(f))

    def get_f(self) -> np.ndarray:
        out = np.zeros((self.q, self.ny, self.nx))
        self.lib.or_get_f(self.h, _p(out))
        return out

    def get_phi(self) -> np.ndarray:
        out = np.zeros((self.ny, self.nx))
        self.lib.or_get_phi(self.h, _p(out))
        return out

    def set_clock(self, step: int, t: float):
        self.lib.or_set_clock(self.h, int(step), float(t))

    @property
    def step_index(self) -> int:
        return self.lib.or_step_index(self.h)

    @property
    def time(self) -> float:
        return self.lib.or_time(self.h)

    def step(self, nsteps: int = 1, rings=None):
        if rings is not None:
            rings = _f64(rings).reshape(nsteps, -1)
            assert rings.shape[1] == 2 * (self.nx + self.ny) + 4
        self.lib.or_step(self.h, int(nsteps), _p(rings) if rings is not None else None)

    def step_cells(self, cells, ring=None) -> np.ndarray:
        """One step evaluated at the listed (i, j) cells; the state is unchanged."""
        cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 2)
        out = np.zeros((len(cells), self.q))
        r = _f64(ring) if ring is not None else None
        self.lib.or_step_cells(self.h, len(cells), cells.ctypes.data_as(_i),
                               _p(r) if r is not None else None, _p(out))
        return out

    def fbar_plus_all(self, ring=None) -> np.ndarray:
        out = np.zeros((self.ny + 2, self.nx + 2, self.q))
        r = _f64(ring) if ring is not None else None
        self.lib.or_fbar_plus_all(self.h, _p(r) if r is not None else None, _p(out))
        return out

    def errors(self, phi_a):
        phi_a = _f64(phi_a).reshape(self.ny, self.nx)
        gre, l2 = C.c_double(), C.c_double()
        self.lib.or_errors(self.h, _p(phi_a), C.byref(gre), C.byref(l2))
        return gre.value, l2.value

    def mass(self) -> float:
        return self.lib.or_mass(self.h)
