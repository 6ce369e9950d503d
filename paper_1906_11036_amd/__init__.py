"""DUGKS for nonlinear convection-diffusion equations on MI355X.

Thin binding over libdugks.so (include/dugks.h): argument marshalling only.
PyTorch provides the device workspace and the stream; every step of the
method runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L
from ._lib import (BC_DIRICHLET, BC_MIRROR, BC_PERIODIC, BF16NEQ, F16NEQ, F32, F64,  # noqa: F401
                   KERNEL_FUSED, KERNEL_PLAIN, SCHED_GRID, SCHED_PERSISTENT, STORAGE, DugksError)

__all__ = ["Solver", "Batch", "Solver3D", "Batch3D", "Solver1D", "DugksError", "F64", "F32", "F16NEQ", "BF16NEQ"]


def _torch():
    import torch
    return torch


def _stream_handle(device):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _poly(v, n=None):
    v = [float(x) for x in v]
    if n is not None:
        v = v + [0.0] * (n - len(v))
    return v


def _params(problem, storage, kernel):
    p = L.Params()
    p.abi_version = L.ABI_VERSION
    p.storage = storage
    p.bc[0] = p.bc[1] = int(problem.bcx)
    p.bc[2] = p.bc[3] = int(problem.bcy)
    p.kernel = kernel
    p.c, p.cfl, p.alpha = float(problem.c), float(problem.cfl), float(problem.alpha)
    return p


def _terms_args(terms, ny, nx, device):
    """(device array [n][ny][nx], host powers, host rates) of source terms (k, gamma,
    G), or Nones for no terms; the caller keeps the three alive."""
    torch = _torch()
    n = len(terms)
    if n == 0:
        return None, None, None
    g = np.ascontiguousarray(np.stack([np.asarray(G, dtype=np.float64).reshape(ny, nx)
                                       for _, _, G in terms]))
    t = torch.from_numpy(g).to(device)
    pw = (C.c_int * n)(*[int(k) for k, _, _ in terms])
    gm = np.array([float(gam) for _, gam, _ in terms], dtype=np.float64)
    return t, pw, gm


def _terms_ptrs(t, pw, gm):
    if t is None:
        return None, None, None
    return C.c_void_p(t.data_ptr()), pw, _dptr(gm)


def _storage_code(storage):
    return L.STORAGE[storage] if isinstance(storage, str) else int(storage)


class Solver:
    """One instance (``dugks_ctx``).

    ``problem`` is any object with the fields of ``workloads.Problem`` (mesh
    faces, q, c, cfl, alpha, bcx, bcy, B and D coefficients).
    """

    def __init__(self, problem, storage="f64", kernel=KERNEL_FUSED, device="cuda:0",
                 launch: Optional[Sequence[int]] = None):
        torch = _torch()
        self.lib = L.lib()
        self.device = torch.device(device)
        self.problem = problem
        self.storage = _storage_code(storage)
        self.xf = np.ascontiguousarray(problem.xf, dtype=np.float64)
        self.yf = np.ascontiguousarray(problem.yf, dtype=np.float64)
        self.nx, self.ny, self.q = len(self.xf) - 1, len(self.yf) - 1, int(problem.q)
        h = C.c_void_p()
        p = _params(problem, self.storage, kernel)
        rc = self.lib.dugks_create(C.byref(h), self.nx, self.ny, _dptr(self.xf), _dptr(self.yf),
                                   self.q, C.byref(p))
        self.h = h
        L.check(rc, h, "dugks_create")
        self.set_B(problem.bx, problem.by)
        self.set_D(problem.dxx, problem.dxy, problem.dyy)
        if launch is not None:
            self.set_launch(*launch)
        nbytes = self.lib.dugks_workspace_bytes(self.h)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) & ~255
            L.check(self.lib.dugks_bind(self.h, C.c_void_p(self._ws_ptr), nbytes,
                                        _stream_handle(self.device)), self.h, "dugks_bind")
        self._ring = None
        self._src = None
        if getattr(problem, "src_g", None) is not None:
            self.set_source(problem.src_g, problem.src_gamma)
        if getattr(problem, "src_terms", None):
            self.set_source_terms(problem.src_terms)

    # -- coefficients
    def set_B(self, bx, by):
        deg = max(len(bx), len(by)) - 1
        a, b = np.array(_poly(bx, deg + 1)), np.array(_poly(by, deg + 1))
        L.check(self.lib.dugks_set_B(self.h, deg, _dptr(a), _dptr(b)), self.h, "dugks_set_B")

    def set_D(self, dxx, dxy, dyy):
        deg = max(len(dxx), len(dxy), len(dyy)) - 1
        arrs = [np.array(_poly(v, deg + 1)) for v in (dxx, dxy, dyy)]
        L.check(self.lib.dugks_set_D(self.h, deg, *[_dptr(a) for a in arrs]), self.h, "dugks_set_D")

    def set_dirichlet(self, rings):
        """rings: [nsteps][2(nx+ny)+4] binary64 (numpy or device tensor); kept alive here."""
        torch = _torch()
        t = torch.as_tensor(np.asarray(rings, dtype=np.float64) if not torch.is_tensor(rings)
                            else rings, dtype=torch.float64, device=self.device).contiguous()
        self._ring = t
        L.check(self.lib.dugks_set_dirichlet(self.h, C.c_void_p(t.data_ptr()), int(t.shape[0])),
                self.h, "dugks_set_dirichlet")

    def set_source(self, g, gamma=0.0):
        """F(x, t) = exp(gamma t) g(x), g [ny][nx] at the cell centres (kept alive
        here); None removes it.  Call before set_phi."""
        if g is None:
            self._src = None
            L.check(self.lib.dugks_set_source(self.h, None, 0.0), self.h, "dugks_set_source")
            return
        t = self._dev64(g, (self.ny, self.nx))
        L.check(self.lib.dugks_set_source(self.h, C.c_void_p(t.data_ptr()), float(gamma)), self.h,
                "dugks_set_source")
        self._src = t

    def set_source_terms(self, terms):
        """F(x, t, phi) = sum over terms (k, gamma, G) of exp(gamma t) phi^k G(x), G
        [ny][nx] at the cell centres, k in 0..3 (the G are kept alive here); an
        empty list removes the source.  Call before set_phi."""
        keep = _terms_args(terms, self.ny, self.nx, self.device)
        L.check(self.lib.dugks_set_source_terms(self.h, len(terms), *_terms_ptrs(*keep)), self.h,
                "dugks_set_source_terms")
        self._src = keep if terms else None

    # -- state
    def _dev64(self, a, shape):
        torch = _torch()
        if torch.is_tensor(a):
            t = a.to(device=self.device, dtype=torch.float64).contiguous()
        else:
            t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
        return t.reshape(shape)

    def set_phi(self, phi):
        t = self._dev64(phi, (self.ny, self.nx))
        L.check(self.lib.dugks_set_phi(self.h, C.c_void_p(t.data_ptr()), 1), self.h, "dugks_set_phi")

    def set_f(self, f):
        t = self._dev64(f, (self.q, self.ny, self.nx))
        L.check(self.lib.dugks_set_f(self.h, C.c_void_p(t.data_ptr()), 1), self.h, "dugks_set_f")

    def step(self, nsteps=1):
        L.check(self.lib.dugks_step(self.h, int(nsteps)), self.h, "dugks_step")

    def time_steps(self, nsteps):
        ms = C.c_float()
        L.check(self.lib.dugks_time_steps(self.h, int(nsteps), C.byref(ms)), self.h, "dugks_time_steps")
        return ms.value

    def phi_tensor(self):
        torch = _torch()
        out = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        L.check(self.lib.dugks_get_phi(self.h, C.c_void_p(out.data_ptr()), 1), self.h, "dugks_get_phi")
        return out

    def get_phi(self) -> np.ndarray:
        return self.phi_tensor().cpu().numpy()

    def f_tensor(self):
        """f~ decoded to binary64 [q][ny][nx], a device tensor."""
        torch = _torch()
        out = torch.empty((self.q, self.ny, self.nx), dtype=torch.float64, device=self.device)
        L.check(self.lib.dugks_get_f(self.h, C.c_void_p(out.data_ptr()), 1), self.h, "dugks_get_f")
        return out

    def get_f(self) -> np.ndarray:
        return self.f_tensor().cpu().numpy()

    def diag(self, check=True) -> dict:
        d = L.Diag()
        rc = self.lib.dugks_get_diag(self.h, C.byref(d))
        if check:
            L.check(rc, self.h, "dugks_get_diag")
        return {"step": d.step, "t": d.t, "dt": d.dt, "mass": d.mass, "max_neq": d.max_neq,
                "scale": d.scale, "flags": d.flags, "rc": rc}

    def error_norms(self, ref):
        t = self._dev64(ref, (self.ny, self.nx))
        l2, gre = C.c_double(), C.c_double()
        L.check(self.lib.dugks_error_norms(self.h, C.c_void_p(t.data_ptr()), C.byref(l2), C.byref(gre)),
                self.h, "dugks_error_norms")
        return gre.value, l2.value

    def checkpoint(self) -> bytes:
        n = C.c_size_t()
        L.check(self.lib.dugks_checkpoint(self.h, None, C.byref(n)), self.h, "dugks_checkpoint")
        buf = (C.c_char * n.value)()
        L.check(self.lib.dugks_checkpoint(self.h, buf, C.byref(n)), self.h, "dugks_checkpoint")
        return bytes(buf[:n.value])

    def restore(self, blob: bytes):
        buf = (C.c_char * len(blob)).from_buffer_copy(blob)
        L.check(self.lib.dugks_restore(self.h, buf, len(blob)), self.h, "dugks_restore")

    def set_launch(self, rows_per_wave=64, waves_per_block=4, schedule=SCHED_GRID, xcd_remap=1):
        L.check(self.lib.dugks_set_launch(self.h, rows_per_wave, waves_per_block, schedule, xcd_remap),
                self.h, "dugks_set_launch")

    def autotune(self, trial_steps=5):
        L.check(self.lib.dugks_autotune(self.h, trial_steps), self.h, "dugks_autotune")

    def info(self) -> dict:
        i = L.Info()
        L.check(self.lib.dugks_get_info(self.h, C.byref(i)), self.h, "dugks_get_info")
        return {k: getattr(i, k) for k, _ in L.Info._fields_}

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.dugks_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent instances advanced by one launch per step (``dugks_batch``)."""

    def __init__(self, problems, storage="f32", device="cuda:0", launch=None):
        torch = _torch()
        self.lib = L.lib()
        self.device = torch.device(device)
        self.problems = list(problems)
        self.storage = _storage_code(storage)
        n = len(self.problems)
        descs = (L.InstanceDesc * n)()
        self._faces = []
        for k, pb in enumerate(self.problems):
            xf = np.ascontiguousarray(pb.xf, dtype=np.float64)
            yf = np.ascontiguousarray(pb.yf, dtype=np.float64)
            self._faces.append((xf, yf))
            d = descs[k]
            d.nx, d.ny, d.q = len(xf) - 1, len(yf) - 1, int(pb.q)
            d.xf, d.yf = _dptr(xf), _dptr(yf)
            d.p = _params(pb, self.storage, KERNEL_FUSED)
            bdeg = max(len(pb.bx), len(pb.by)) - 1
            ddeg = max(len(pb.dxx), len(pb.dxy), len(pb.dyy)) - 1
            d.b_deg, d.d_deg = bdeg, ddeg
            for name, v in (("bx", pb.bx), ("by", pb.by), ("dxx", pb.dxx), ("dxy", pb.dxy),
                            ("dyy", pb.dyy)):
                arr = getattr(d, name)
                for i, x in enumerate(_poly(v, L.MAX_DEG + 1)):
                    arr[i] = x
        h = C.c_void_p()
        rc = self.lib.dugks_batch_create(C.byref(h), n, descs, self.storage)
        self.h = h
        L.check(rc, h, "dugks_batch_create")
        if launch is not None:
            L.check(self.lib.dugks_batch_set_launch(self.h, *launch), self.h, "set_launch")
        nbytes = self.lib.dugks_batch_workspace_bytes(self.h)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self._ws_ptr = (self.workspace.data_ptr() + 255) & ~255
            L.check(self.lib.dugks_batch_bind(self.h, C.c_void_p(self._ws_ptr), nbytes,
                                              _stream_handle(self.device)), self.h, "dugks_batch_bind")
        self._src = {}
        for k, pb in enumerate(self.problems):
            if getattr(pb, "src_g", None) is not None:
                self.set_source(k, pb.src_g, pb.src_gamma)
            if getattr(pb, "src_terms", None):
                self.set_source_terms(k, pb.src_terms)

    def __len__(self):
        return len(self.problems)

    def set_phi(self, i, phi):
        torch = _torch()
        pb = self.problems[i]
        t = torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float64)).to(self.device)
        L.check(self.lib.dugks_batch_set_phi(self.h, i, C.c_void_p(t.data_ptr()), 1), self.h,
                "dugks_batch_set_phi")
        del pb

    def set_source(self, i, g, gamma=0.0):
        """Source of instance i (see Solver.set_source); None removes it."""
        torch = _torch()
        if g is None:
            self._src.pop(i, None)
            L.check(self.lib.dugks_batch_set_source(self.h, i, None, 0.0), self.h,
                    "dugks_batch_set_source")
            return
        t = torch.from_numpy(np.ascontiguousarray(g, dtype=np.float64)).to(self.device).contiguous()
        L.check(self.lib.dugks_batch_set_source(self.h, i, C.c_void_p(t.data_ptr()), float(gamma)),
                self.h, "dugks_batch_set_source")
        self._src[i] = t

    def set_source_terms(self, i, terms):
        """Source terms (k, gamma, G) of instance i (see Solver.set_source_terms)."""
        pb = self.problems[i]
        keep = _terms_args(terms, pb.ny, pb.nx, self.device)
        L.check(self.lib.dugks_batch_set_source_terms(self.h, i, len(terms), *_terms_ptrs(*keep)),
                self.h, "dugks_batch_set_source_terms")
        if terms:
            self._src[i] = keep
        else:
            self._src.pop(i, None)

    def set_all_phi(self):
        for i, pb in enumerate(self.problems):
            self.set_phi(i, pb.phi0)

    def step(self, nsteps=1):
        L.check(self.lib.dugks_batch_step(self.h, int(nsteps)), self.h, "dugks_batch_step")

    def time_steps(self, nsteps):
        ms = C.c_float()
        L.check(self.lib.dugks_batch_time_steps(self.h, int(nsteps), C.byref(ms)), self.h,
                "dugks_batch_time_steps")
        return ms.value

    def get_phi(self, i) -> np.ndarray:
        torch = _torch()
        pb = self.problems[i]
        out = torch.empty((pb.ny, pb.nx), dtype=torch.float64, device=self.device)
        L.check(self.lib.dugks_batch_get_phi(self.h, i, C.c_void_p(out.data_ptr()), 1), self.h,
                "dugks_batch_get_phi")
        return out.cpu().numpy()

    def set_launch(self, rows_per_wave=64, waves_per_block=4, schedule=SCHED_GRID, xcd_remap=1):
        L.check(self.lib.dugks_batch_set_launch(self.h, rows_per_wave, waves_per_block, schedule,
                                                xcd_remap), self.h, "dugks_batch_set_launch")

    def autotune(self, trial_steps=3):
        L.check(self.lib.dugks_batch_autotune(self.h, trial_steps), self.h, "dugks_batch_autotune")

    def info(self, i=0) -> dict:
        inf = L.Info()
        L.check(self.lib.dugks_batch_get_info(self.h, i, C.byref(inf)), self.h, "info")
        return {k: getattr(inf, k) for k, _ in L.Info._fields_}

    def totals(self):
        cells, sb = C.c_longlong(), C.c_size_t()
        L.check(self.lib.dugks_batch_totals(self.h, C.byref(cells), C.byref(sb)), self.h, "totals")
        return cells.value, sb.value

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.dugks_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver3D:
    """One three-dimensional instance (``dugks3_ctx``: D3Q15, D3Q19 or D3Q7).

    ``problem`` has the fields of ``workloads.Problem3D`` (faces xf, yf, zf, q,
    c, cfl, alpha, bc per axis, b = (B_x, B_y, B_z) and d = (D_xx, D_yy, D_zz,
    D_xy, D_xz, D_yz) coefficient tuples)."""

    def __init__(self, problem, storage="f64", device="cuda:0", launch=None):
        torch = _torch()
        self.lib = L.lib()
        self.device = torch.device(device)
        self.problem = problem
        self.storage = _storage_code(storage)
        self.faces = [np.ascontiguousarray(f, dtype=np.float64) for f in (problem.xf, problem.yf, problem.zf)]
        self.nx, self.ny, self.nz = (len(f) - 1 for f in self.faces)
        self.q = int(problem.q)
        p = L.Params3()
        p.abi_version = L.ABI3_VERSION
        p.storage = self.storage
        for i, b in enumerate(problem.bc):
            p.bc[i] = int(b)
        p.c, p.cfl, p.alpha = float(problem.c), float(problem.cfl), float(problem.alpha)
        h = C.c_void_p()
        rc = self.lib.dugks3_create(C.byref(h), self.nx, self.ny, self.nz, *[_dptr(f) for f in self.faces],
                                    self.q, C.byref(p))
        self.h = h
        L.check3(rc, h, "dugks3_create")
        deg = max(len(v) for v in problem.b) - 1
        b = np.concatenate([np.array(_poly(v, deg + 1)) for v in problem.b])
        L.check3(self.lib.dugks3_set_B(self.h, deg, _dptr(b)), self.h, "dugks3_set_B")
        deg = max(len(v) for v in problem.d) - 1
        d = np.concatenate([np.array(_poly(v, deg + 1)) for v in problem.d])
        L.check3(self.lib.dugks3_set_D(self.h, deg, _dptr(d)), self.h, "dugks3_set_D")
        nbytes = self.lib.dugks3_workspace_bytes(self.h)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self._ws_ptr = (self.workspace.data_ptr() + 255) & ~255
            L.check3(self.lib.dugks3_bind(self.h, C.c_void_p(self._ws_ptr), nbytes,
                                          _stream_handle(self.device)), self.h, "dugks3_bind")
        if launch is not None:
            self.set_launch(*launch)
        if getattr(problem, "src_terms", None):
            self.set_source_terms(problem.src_terms)

    def _dev64(self, a, shape):
        torch = _torch()
        if torch.is_tensor(a):
            t = a.to(device=self.device, dtype=torch.float64).contiguous()
        else:
            t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
        return t.reshape(shape)

    def set_phi(self, phi):
        t = self._dev64(phi, (self.nz, self.ny, self.nx))
        L.check3(self.lib.dugks3_set_phi(self.h, C.c_void_p(t.data_ptr()), 1), self.h, "dugks3_set_phi")

    def set_f(self, f):
        t = self._dev64(f, (self.q, self.nz, self.ny, self.nx))
        L.check3(self.lib.dugks3_set_f(self.h, C.c_void_p(t.data_ptr()), 1), self.h, "dugks3_set_f")

    def set_source_terms(self, terms):
        """F(x, t, phi) = sum_j exp(gamma_j t) phi^k_j G_j(x), terms as (k_j,
        gamma_j, G_j [nz][ny][nx]); an empty list removes the source.  Set
        before set_phi.  The G_j (and, for D3Q7's three-pass step, its scratch)
        stay on the device while this solver lives."""
        torch = _torch()
        n = len(terms)
        if n == 0:
            L.check3(self.lib.dugks3_set_source_terms(self.h, 0, None, None, None, None, 0), self.h,
                     "dugks3_set_source_terms")
            self._src = None
            return
        g = np.stack([np.asarray(G, dtype=np.float64).reshape(self.nz, self.ny, self.nx) for _, _, G in terms])
        self._src_g = torch.from_numpy(np.ascontiguousarray(g)).to(self.device)
        nb = self.lib.dugks3_source_scratch_bytes(self.h)   # 0: the fused step needs none
        self._scratch = torch.empty(nb + 256, dtype=torch.uint8, device=self.device) if nb else None
        sp = (self._scratch.data_ptr() + 255) & ~255 if nb else None
        pw = (C.c_int * n)(*[int(k) for k, _, _ in terms])
        gm = (C.c_double * n)(*[float(gam) for _, gam, _ in terms])
        L.check3(self.lib.dugks3_set_source_terms(self.h, n, C.c_void_p(self._src_g.data_ptr()), pw, gm,
                                                  C.c_void_p(sp), nb), self.h, "dugks3_set_source_terms")

    def set_dirichlet(self, rings):
        """Dirichlet data, [nsteps][shell length] (workloads.Problem3D.rings),
        kept on the device while this solver lives."""
        torch = _torch()
        t = rings if torch.is_tensor(rings) else torch.from_numpy(np.ascontiguousarray(rings, dtype=np.float64))
        self._rings = t.to(device=self.device, dtype=torch.float64).contiguous()
        n = int(self._rings.shape[0]) if self._rings.dim() > 1 else 1
        L.check3(self.lib.dugks3_set_dirichlet(self.h, C.c_void_p(self._rings.data_ptr()), n), self.h,
                 "dugks3_set_dirichlet")

    def step(self, nsteps=1):
        L.check3(self.lib.dugks3_step(self.h, int(nsteps)), self.h, "dugks3_step")

    def time_steps(self, nsteps):
        ms = C.c_float()
        L.check3(self.lib.dugks3_time_steps(self.h, int(nsteps), C.byref(ms)), self.h, "dugks3_time_steps")
        return ms.value

    def get_phi(self) -> np.ndarray:
        out = np.zeros((self.nz, self.ny, self.nx))
        L.check3(self.lib.dugks3_get_phi(self.h, _dptr(out), 0), self.h, "dugks3_get_phi")
        return out

    def get_f(self) -> np.ndarray:
        out = np.zeros((self.q, self.nz, self.ny, self.nx))
        L.check3(self.lib.dugks3_get_f(self.h, _dptr(out), 0), self.h, "dugks3_get_f")
        return out

    def reduce(self, ref=None) -> dict:
        """mass, and with a reference field [nz][ny][nx] the GRE (eq. 4.1) and rel-L2."""
        m, g, l2 = C.c_double(), C.c_double(), C.c_double()
        t = self._dev64(ref, (self.nz, self.ny, self.nx)) if ref is not None else None
        L.check3(self.lib.dugks3_reduce(self.h, C.c_void_p(t.data_ptr()) if t is not None else None,
                                        C.byref(m), C.byref(g), C.byref(l2)), self.h, "dugks3_reduce")
        return {"mass": m.value, "gre": g.value, "rel_l2": l2.value}

    def set_launch(self, rows_per_block=4, planes_per_block=64):
        L.check3(self.lib.dugks3_set_launch(self.h, int(rows_per_block), int(planes_per_block)), self.h,
                 "dugks3_set_launch")

    def autotune(self, trial_steps=3):
        """Keep the fastest launch shape (dugks3_autotune; the state is unchanged)."""
        L.check3(self.lib.dugks3_autotune(self.h, int(trial_steps)), self.h, "dugks3_autotune")

    def info(self) -> dict:
        inf = L.Info3()
        L.check3(self.lib.dugks3_get_info(self.h, C.byref(inf)), self.h, "dugks3_get_info")
        return {k: getattr(inf, k) for k, _ in L.Info3._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.dugks3_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch3D:
    """Many D3Q15 or D3Q19 instances stepped by one launch per step
    (``dugks3_batch``): ``solvers`` are ``Solver3D`` objects of one lattice and
    storage, set up and given their states; they stay alive and bound while the
    batch lives, and their own accessors read the results."""

    def __init__(self, solvers, launch=None):
        torch = _torch()
        self.lib = L.lib()
        self.solvers = list(solvers)
        self.device = self.solvers[0].device
        self.h = C.c_void_p()
        arr = (C.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        rc = self.lib.dugks3_batch_create(C.byref(self.h), len(self.solvers), arr)
        L.check_b3(rc, self.h, "dugks3_batch_create")
        nbytes = self.lib.dugks3_batch_workspace_bytes(self.h)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            ptr = (self.workspace.data_ptr() + 255) & ~255
            L.check_b3(self.lib.dugks3_batch_bind(self.h, C.c_void_p(ptr), nbytes, _stream_handle(self.device)),
                       self.h, "dugks3_batch_bind")
        if launch is not None:
            self.set_launch(*launch)

    def set_launch(self, rows_per_block, planes_per_block):
        L.check_b3(self.lib.dugks3_batch_set_launch(self.h, int(rows_per_block), int(planes_per_block)), self.h,
                   "dugks3_batch_set_launch")

    def step(self, nsteps=1):
        L.check_b3(self.lib.dugks3_batch_step(self.h, int(nsteps)), self.h, "dugks3_batch_step")

    def time_steps(self, nsteps):
        ms = C.c_float()
        L.check_b3(self.lib.dugks3_batch_time_steps(self.h, int(nsteps), C.byref(ms)), self.h,
                   "dugks3_batch_time_steps")
        return ms.value

    def info(self) -> dict:
        r, p, b, c = C.c_int(), C.c_int(), C.c_longlong(), C.c_longlong()
        L.check_b3(self.lib.dugks3_batch_get_info(self.h, C.byref(r), C.byref(p), C.byref(b), C.byref(c)), self.h,
                   "dugks3_batch_get_info")
        return {"rows_per_block": r.value, "planes_per_block": p.value, "blocks": b.value, "cells": c.value}

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.dugks3_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver1D:
    """One D1Q3 instance on the GPU through include/dugks1d.h: B = b(x, t) phi with
    b = (p0 + p1 t) x + q0 exp(q1 t + q2 t^2), D = (r0 + r1 t) phi, C = 0, R from
    dB/dt (Remark 3).

    ``problem`` has the fields of ``workloads.Problem1D`` (faces xf, coef, c, cfl,
    alpha, bc, t0 and, for Dirichlet walls, ghost(t))."""

    def __init__(self, problem, storage="f64", device="cuda:0"):
        torch = _torch()
        self.lib = L.lib()
        self.device = torch.device(device)
        self.problem = problem
        self.storage = _storage_code(storage)
        self.xf = np.ascontiguousarray(problem.xf, dtype=np.float64)
        self.nx = len(self.xf) - 1
        p = L.Params1()
        p.abi_version = L.ABI1_VERSION
        p.storage = self.storage
        p.bc = int(problem.bc)
        p.c, p.cfl, p.alpha = float(problem.c), float(problem.cfl), float(problem.alpha)
        for k in range(7):
            p.coef[k] = float(problem.coef[k])
        p.t0 = float(getattr(problem, "t0", 0.0))
        h = C.c_void_p()
        rc = self.lib.dugks1_create(C.byref(h), self.nx, _dptr(self.xf), C.byref(p))
        self.h = h
        L.check1(rc, h, "dugks1_create")
        nbytes = self.lib.dugks1_workspace_bytes(self.h)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self._ws_ptr = (self.workspace.data_ptr() + 255) & ~255
            L.check1(self.lib.dugks1_bind(self.h, C.c_void_p(self._ws_ptr), nbytes,
                                          _stream_handle(self.device)), self.h, "dugks1_bind")
        self._ghosts = None

    def _dev64(self, a, shape):
        torch = _torch()
        if torch.is_tensor(a):
            t = a.to(device=self.device, dtype=torch.float64).contiguous()
        else:
            t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
        return t.reshape(shape)

    def info(self) -> dict:
        inf = L.Info1()
        L.check1(self.lib.dugks1_get_info(self.h, C.byref(inf)), self.h, "dugks1_get_info")
        return {k: getattr(inf, k) for k, _ in L.Info1._fields_}

    def set_phi(self, phi):
        t = self._dev64(phi, (self.nx,))
        L.check1(self.lib.dugks1_set_phi(self.h, C.c_void_p(t.data_ptr()), 1), self.h, "dugks1_set_phi")

    def set_state(self, f, phi_prev):
        tf = self._dev64(f, (3, self.nx))
        tp = self._dev64(phi_prev, (self.nx,))
        L.check1(self.lib.dugks1_set_state(self.h, C.c_void_p(tf.data_ptr()), C.c_void_p(tp.data_ptr()), 1),
                 self.h, "dugks1_set_state")

    def set_dirichlet(self, ghosts):
        """ghosts: [nsteps][2] phi at the two ghost centres for the next steps."""
        g = np.ascontiguousarray(ghosts, dtype=np.float64).reshape(-1, 2)
        old = self._ghosts          # the library may still read its last pair
        self._ghosts = self._dev64(g, (g.shape[0] * 2,))   # kept alive while stepping
        L.check1(self.lib.dugks1_set_dirichlet(self.h, C.c_void_p(self._ghosts.data_ptr()), g.shape[0]),
                 self.h, "dugks1_set_dirichlet")
        del old

    def ghost_table(self, nsteps):
        """Ghost data of the problem for the next nsteps steps (Dirichlet walls)."""
        inf = self.info()
        t0, dt = inf["time"], inf["dt"]
        return np.array([self.problem.ghost(t0 + s * dt) for s in range(nsteps)], dtype=np.float64)

    def step(self, nsteps=1, auto_ghosts=True):
        if int(self.problem.bc) == 1 and auto_ghosts and nsteps > 0:
            self.set_dirichlet(self.ghost_table(nsteps))
        L.check1(self.lib.dugks1_step(self.h, int(nsteps)), self.h, "dugks1_step")

    def time_steps(self, nsteps):
        if int(self.problem.bc) == 1 and nsteps > 0:
            self.set_dirichlet(self.ghost_table(nsteps))
        ms = C.c_float()
        L.check1(self.lib.dugks1_time_steps(self.h, int(nsteps), C.byref(ms)), self.h, "dugks1_time_steps")
        return ms.value

    def _read(self, fn, shape):
        out = np.zeros(shape)
        L.check1(fn(self.h, _dptr(out), 0), self.h, "dugks1 read-out")
        return out

    def get_phi(self) -> np.ndarray:
        return self._read(self.lib.dugks1_get_phi, (self.nx,))

    def get_f(self) -> np.ndarray:
        return self._read(self.lib.dugks1_get_f, (3, self.nx))

    def get_phi_prev(self) -> np.ndarray:
        return self._read(self.lib.dugks1_get_phi_prev, (self.nx,))

    def reduce(self, ref=None) -> dict:
        m, g, l2 = C.c_double(), C.c_double(), C.c_double()
        t = self._dev64(ref, (self.nx,)) if ref is not None else None
        L.check1(self.lib.dugks1_reduce(self.h, C.c_void_p(t.data_ptr()) if t is not None else None,
                                        C.byref(m), C.byref(g), C.byref(l2)), self.h, "dugks1_reduce")
        return {"mass": m.value, "gre": g.value, "rel_l2": l2.value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.dugks1_destroy(self.h)
            self.h = None
        self.workspace = None
        self._ghosts = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
