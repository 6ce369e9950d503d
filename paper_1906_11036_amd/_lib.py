"""ctypes declarations of the C ABI in include/dugks.h and include/dugks3d.h.

Loading fails loudly when libdugks.so is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdugks.so")

ABI_VERSION = 4
ABI3_VERSION = 1
ABI1_VERSION = 1
MAX_DEG = 4
OK, E_ARG, E_STATE, E_HIP, E_UNSTABLE, E_UNSUPPORTED, E_NOMEM, E_FORMAT = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32, F16NEQ, BF16NEQ = 0, 1, 2, 3
BC_PERIODIC, BC_DIRICHLET, BC_MIRROR = 0, 1, 2
KERNEL_FUSED, KERNEL_PLAIN = 0, 1
SCHED_GRID, SCHED_PERSISTENT = 0, 1
FLAG_NONFINITE, FLAG_OVERFLOW = 1, 2

ERROR_NAMES = {E_ARG: "E_ARG", E_STATE: "E_STATE", E_HIP: "E_HIP", E_UNSTABLE: "E_UNSTABLE",
               E_UNSUPPORTED: "E_UNSUPPORTED", E_NOMEM: "E_NOMEM", E_FORMAT: "E_FORMAT"}
STORAGE = {"f64": F64, "f32": F32, "f16neq": F16NEQ, "bf16neq": BF16NEQ}


class Params(C.Structure):
    _fields_ = [("abi_version", C.c_int), ("storage", C.c_int), ("bc", C.c_int * 4),
                ("kernel", C.c_int), ("c", C.c_double), ("cfl", C.c_double), ("alpha", C.c_double)]


class Info(C.Structure):
    _fields_ = [("dt", C.c_double), ("h", C.c_double), ("lambda_", C.c_double), ("cs2", C.c_double),
                ("a1", C.c_double), ("b1", C.c_double), ("a2", C.c_double), ("b2", C.c_double),
                ("a3", C.c_double), ("b3", C.c_double), ("nx", C.c_int), ("ny", C.c_int),
                ("q", C.c_int), ("storage", C.c_int), ("pitch", C.c_int), ("eq_degree", C.c_int),
                ("rows_per_wave", C.c_int), ("waves_per_block", C.c_int), ("schedule", C.c_int),
                ("xcd_remap", C.c_int), ("work_items", C.c_longlong), ("state_bytes", C.c_size_t),
                ("graph_steps", C.c_longlong), ("eager_steps", C.c_longlong), ("xy_symmetric", C.c_int)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_longlong), ("t", C.c_double), ("dt", C.c_double), ("mass", C.c_double),
                ("max_neq", C.c_double), ("scale", C.c_double), ("flags", C.c_int)]


class Params3(C.Structure):
    _fields_ = [("abi_version", C.c_int), ("storage", C.c_int), ("bc", C.c_int * 3),
                ("c", C.c_double), ("cfl", C.c_double), ("alpha", C.c_double)]


class Info3(C.Structure):
    _fields_ = [("dt", C.c_double), ("h", C.c_double), ("lambda_", C.c_double), ("cs2", C.c_double),
                ("a1", C.c_double), ("b1", C.c_double), ("a2", C.c_double), ("b2", C.c_double),
                ("a3", C.c_double), ("b3", C.c_double), ("nx", C.c_int), ("ny", C.c_int),
                ("nz", C.c_int), ("q", C.c_int), ("storage", C.c_int), ("pitch", C.c_int),
                ("eq_degree", C.c_int), ("rows_per_block", C.c_int), ("planes_per_block", C.c_int),
                ("blocks", C.c_longlong), ("state_bytes", C.c_size_t)]


class Params1(C.Structure):
    _fields_ = [("abi_version", C.c_int), ("storage", C.c_int), ("bc", C.c_int),
                ("c", C.c_double), ("cfl", C.c_double), ("alpha", C.c_double),
                ("coef", C.c_double * 7), ("t0", C.c_double)]


class Info1(C.Structure):
    _fields_ = [("dt", C.c_double), ("h", C.c_double), ("lambda_", C.c_double), ("cs2", C.c_double),
                ("time", C.c_double), ("steps", C.c_longlong), ("nx", C.c_int), ("storage", C.c_int),
                ("bc", C.c_int), ("dirichlet_left", C.c_int), ("state_bytes", C.c_size_t)]


_D5 = C.c_double * (MAX_DEG + 1)


class InstanceDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("q", C.c_int),
                ("xf", C.POINTER(C.c_double)), ("yf", C.POINTER(C.c_double)),
                ("p", Params), ("b_deg", C.c_int), ("bx", _D5), ("by", _D5),
                ("d_deg", C.c_int), ("dxx", _D5), ("dxy", _D5), ("dyy", _D5)]


_vp, _dp, _int, _sz = C.c_void_p, C.POINTER(C.c_double), C.c_int, C.c_size_t

# name -> (restype, argtypes); every function declared in include/dugks.h
SIGNATURES = {
    "dugks_create": (_int, [C.POINTER(_vp), _int, _int, _dp, _dp, _int, C.POINTER(Params)]),
    "dugks_workspace_bytes": (_sz, [_vp]),
    "dugks_bind": (_int, [_vp, _vp, _sz, _vp]),
    "dugks_set_B": (_int, [_vp, _int, _dp, _dp]),
    "dugks_set_D": (_int, [_vp, _int, _dp, _dp, _dp]),
    "dugks_set_source": (_int, [_vp, _vp, C.c_double]),
    "dugks_set_source_terms": (_int, [_vp, _int, _vp, C.POINTER(C.c_int), _dp]),
    "dugks_set_dirichlet": (_int, [_vp, _vp, _int]),
    "dugks_set_phi": (_int, [_vp, _vp, _int]),
    "dugks_set_f": (_int, [_vp, _vp, _int]),
    "dugks_step": (_int, [_vp, _int]),
    "dugks_get_phi": (_int, [_vp, _vp, _int]),
    "dugks_get_f": (_int, [_vp, _vp, _int]),
    "dugks_get_diag": (_int, [_vp, C.POINTER(Diag)]),
    "dugks_error_norms": (_int, [_vp, _vp, _dp, _dp]),
    "dugks_error_norms_noalloc": (_int, [_vp, _vp, _vp]),
    "dugks_checkpoint": (_int, [_vp, _vp, C.POINTER(_sz)]),
    "dugks_restore": (_int, [_vp, _vp, _sz]),
    "dugks_set_launch": (_int, [_vp, _int, _int, _int, _int]),
    "dugks_autotune": (_int, [_vp, _int]),
    "dugks_get_info": (_int, [_vp, C.POINTER(Info)]),
    "dugks_time_steps": (_int, [_vp, _int, C.POINTER(C.c_float)]),
    "dugks_batch_create": (_int, [C.POINTER(_vp), _int, C.POINTER(InstanceDesc), _int]),
    "dugks_batch_workspace_bytes": (_sz, [_vp]),
    "dugks_batch_bind": (_int, [_vp, _vp, _sz, _vp]),
    "dugks_batch_set_phi": (_int, [_vp, _int, _vp, _int]),
    "dugks_batch_set_source": (_int, [_vp, _int, _vp, C.c_double]),
    "dugks_batch_set_source_terms": (_int, [_vp, _int, _int, _vp, C.POINTER(C.c_int), _dp]),
    "dugks_batch_autotune": (_int, [_vp, _int]),
    "dugks_batch_set_launch": (_int, [_vp, _int, _int, _int, _int]),
    "dugks_batch_step": (_int, [_vp, _int]),
    "dugks_batch_get_phi": (_int, [_vp, _int, _vp, _int]),
    "dugks_batch_get_info": (_int, [_vp, _int, C.POINTER(Info)]),
    "dugks_batch_totals": (_int, [_vp, C.POINTER(C.c_longlong), C.POINTER(_sz)]),
    "dugks_batch_time_steps": (_int, [_vp, _int, C.POINTER(C.c_float)]),
    "dugks_last_error": (C.c_char_p, [_vp]),
    "dugks_destroy": (None, [_vp]),
    # three dimensions (include/dugks3d.h)
    "dugks3_create": (_int, [C.POINTER(_vp), _int, _int, _int, _dp, _dp, _dp, _int, C.POINTER(Params3)]),
    "dugks3_workspace_bytes": (_sz, [_vp]),
    "dugks3_bind": (_int, [_vp, _vp, _sz, _vp]),
    "dugks3_set_B": (_int, [_vp, _int, _dp]),
    "dugks3_set_D": (_int, [_vp, _int, _dp]),
    "dugks3_set_phi": (_int, [_vp, _vp, _int]),
    "dugks3_set_f": (_int, [_vp, _vp, _int]),
    "dugks3_step": (_int, [_vp, _int]),
    "dugks3_set_dirichlet": (_int, [_vp, _vp, _int]),
    "dugks3_source_scratch_bytes": (_sz, [_vp]),
    "dugks3_set_source_terms": (_int, [_vp, _int, _vp, C.POINTER(_int), C.POINTER(C.c_double), _vp, _sz]),
    "dugks3_get_phi": (_int, [_vp, _vp, _int]),
    "dugks3_get_f": (_int, [_vp, _vp, _int]),
    "dugks3_reduce": (_int, [_vp, _vp, _dp, _dp, _dp]),
    "dugks3_set_launch": (_int, [_vp, _int, _int]),
    "dugks3_time_steps": (_int, [_vp, _int, C.POINTER(C.c_float)]),
    "dugks3_autotune": (_int, [_vp, _int]),
    "dugks3_batch_create": (_int, [C.POINTER(_vp), _int, C.POINTER(_vp)]),
    "dugks3_batch_workspace_bytes": (C.c_size_t, [_vp]),
    "dugks3_batch_bind": (_int, [_vp, _vp, C.c_size_t, _vp]),
    "dugks3_batch_set_launch": (_int, [_vp, _int, _int]),
    "dugks3_batch_step": (_int, [_vp, _int]),
    "dugks3_batch_time_steps": (_int, [_vp, _int, C.POINTER(C.c_float)]),
    "dugks3_batch_get_info": (_int, [_vp, C.POINTER(_int), C.POINTER(_int), C.POINTER(C.c_longlong),
                                     C.POINTER(C.c_longlong)]),
    "dugks3_batch_last_error": (C.c_char_p, [_vp]),
    "dugks3_batch_destroy": (None, [_vp]),
    "dugks3_get_info": (_int, [_vp, C.POINTER(Info3)]),
    "dugks3_last_error": (C.c_char_p, [_vp]),
    "dugks3_destroy": (None, [_vp]),
    "dugks1_create": (_int, [C.POINTER(_vp), _int, _dp, C.POINTER(Params1)]),
    "dugks1_workspace_bytes": (_sz, [_vp]),
    "dugks1_bind": (_int, [_vp, _vp, _sz, _vp]),
    "dugks1_set_phi": (_int, [_vp, _vp, _int]),
    "dugks1_set_state": (_int, [_vp, _vp, _vp, _int]),
    "dugks1_set_dirichlet": (_int, [_vp, _vp, _int]),
    "dugks1_step": (_int, [_vp, _int]),
    "dugks1_get_phi": (_int, [_vp, _vp, _int]),
    "dugks1_get_f": (_int, [_vp, _vp, _int]),
    "dugks1_get_phi_prev": (_int, [_vp, _vp, _int]),
    "dugks1_reduce": (_int, [_vp, _vp, _dp, _dp, _dp]),
    "dugks1_time_steps": (_int, [_vp, _int, C.POINTER(C.c_float)]),
    "dugks1_get_info": (_int, [_vp, C.POINTER(Info1)]),
    "dugks1_last_error": (C.c_char_p, [_vp]),
    "dugks1_destroy": (None, [_vp]),
}

_LIB = None


def lib():
    """The loaded libdugks.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; "
                "g.build()'); there is no fallback implementation")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = h
    return _LIB


class DugksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc, handle, what=""):
    if rc != OK:
        msg = lib().dugks_last_error(handle).decode() if handle else ""
        raise DugksError(rc, f"{what}: {msg}" if what else msg)
    return rc


def check1(rc, handle, what=""):
    """check() for a one-dimensional handle."""
    if rc != OK:
        msg = lib().dugks1_last_error(handle).decode() if handle else ""
        raise DugksError(rc, f"{what}: {msg}" if what else msg)
    return rc


def check_b3(rc, handle, what=""):
    """check() for a three-dimensional batch handle."""
    if rc != OK:
        msg = lib().dugks3_batch_last_error(handle).decode() if handle else ""
        raise DugksError(rc, f"{what}: {msg}" if what else msg)
    return rc


def check3(rc, handle, what=""):
    """check() for a three-dimensional handle."""
    if rc != OK:
        msg = lib().dugks3_last_error(handle).decode() if handle else ""
        raise DugksError(rc, f"{what}: {msg}" if what else msg)
    return rc
