"""Host-only checks of the C ABI: the library loads, exports every function of
include/dugks.h, include/dugks3d.h and include/dugks1d.h, and validates
arguments without touching a device."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_1906_11036_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", n) for n in ("dugks.h", "dugks3d.h", "dugks1d.h")]


def header_functions():
    names = set()
    for path in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names |= set(re.findall(r"\b(dugks[13]?_[A-Za-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = header_functions()
    for must in ("dugks_create", "dugks_bind", "dugks_set_B", "dugks_set_D", "dugks_set_source",
                 "dugks_set_phi", "dugks_step", "dugks_get_phi", "dugks_batch_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = header_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(L.SIGNATURES), set(names) ^ set(L.SIGNATURES)


def _params(**kw):
    p = L.Params()
    p.abi_version = L.ABI_VERSION
    p.storage = kw.get("storage", L.F64)
    for i, b in enumerate(kw.get("bc", (0, 0, 0, 0))):
        p.bc[i] = b
    p.kernel = kw.get("kernel", L.KERNEL_FUSED)
    p.c, p.cfl, p.alpha = kw.get("c", 1.0), kw.get("cfl", 0.5), kw.get("alpha", 1e-3)
    return p


def _create(nx=8, ny=6, q=9, xf=None, yf=None, **kw):
    lib = L.lib()
    xf = np.linspace(0, 1, nx + 1) if xf is None else np.asarray(xf, float)
    yf = np.linspace(0, 1, ny + 1) if yf is None else np.asarray(yf, float)
    h = C.c_void_p()
    p = _params(**kw)
    rc = lib.dugks_create(C.byref(h), nx, ny, xf.ctypes.data_as(C.POINTER(C.c_double)),
                          yf.ctypes.data_as(C.POINTER(C.c_double)), q, C.byref(p))
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(cfl=1.0), L.E_ARG), (dict(cfl=0.0), L.E_ARG), (dict(alpha=0.0), L.E_ARG),
    (dict(c=-1.0), L.E_ARG), (dict(nx=0), L.E_ARG), (dict(q=7), L.E_UNSUPPORTED),
    (dict(storage=9), L.E_UNSUPPORTED), (dict(bc=(0, 1, 0, 0)), L.E_UNSUPPORTED),
    (dict(bc=(1, 2, 0, 0)), L.E_UNSUPPORTED),   # two kinds on one axis
    (dict(kernel=L.KERNEL_PLAIN, storage=L.F32), L.E_UNSUPPORTED),
    (dict(xf=[0, 0.5, 0.4, 1.0], nx=3), L.E_ARG),
])
def test_create_rejects_bad_arguments(kw, code):
    rc, h = _create(**kw)
    assert rc == code
    assert L.lib().dugks_last_error(h).decode()
    L.lib().dugks_destroy(h)


def test_create_and_workspace_size():
    lib = L.lib()
    for storage, per in ((L.F64, 8 * 9), (L.F32, 4 * 9), (L.F16NEQ, 4 + 2 * 8), (L.BF16NEQ, 4 + 2 * 8)):
        rc, h = _create(nx=100, ny=30, storage=storage)
        assert rc == L.OK
        n = lib.dugks_workspace_bytes(h)
        assert n >= 2 * per * 128 * 30   # two buffers of padded rows
        info = L.Info()
        assert lib.dugks_get_info(h, C.byref(info)) == L.OK
        assert info.pitch == 128 and info.state_bytes == per * 128 * 30
        lib.dugks_destroy(h)


def test_calls_before_bind_report_state_errors():
    lib = L.lib()
    rc, h = _create()
    assert rc == L.OK
    assert lib.dugks_step(h, 1) == L.E_STATE
    assert lib.dugks_set_phi(h, None, 0) == L.E_STATE
    assert lib.dugks_set_source(h, None, 0.0) == L.OK
    assert lib.dugks_set_source(h, C.c_void_p(8), float("nan")) == L.E_ARG
    assert lib.dugks_set_launch(h, 0, 4, 0, 1) == L.E_ARG
    assert lib.dugks_set_launch(h, 32, 3, 0, 1) == L.E_ARG
    assert lib.dugks_set_launch(h, 32, 2, 1, 0) == L.OK
    assert lib.dugks_set_launch(h, 32, 16, 0, 1) == L.E_ARG
    n = C.c_size_t()
    assert lib.dugks_checkpoint(h, None, C.byref(n)) == L.OK and n.value > 0
    assert lib.dugks_restore(h, b"short", 5) == L.E_FORMAT
    lib.dugks_destroy(h)


def test_d2q5_accepts_only_identity_diffusion():
    lib = L.lib()
    rc, h = _create(q=5)
    assert rc == L.OK
    d = np.array([0.0, 1.0]); z = np.zeros(2)
    P = C.POINTER(C.c_double)
    assert lib.dugks_set_D(h, 1, d.ctypes.data_as(P), z.ctypes.data_as(P), d.ctypes.data_as(P)) == L.OK
    d2 = np.array([0.0, 2.0])
    assert lib.dugks_set_D(h, 1, d2.ctypes.data_as(P), z.ctypes.data_as(P), d.ctypes.data_as(P)) \
        == L.E_UNSUPPORTED
    lib.dugks_destroy(h)


def test_degree_limits():
    lib = L.lib()
    rc, h = _create()
    a = np.zeros(6)
    P = C.POINTER(C.c_double)
    assert lib.dugks_set_B(h, 5, a.ctypes.data_as(P), a.ctypes.data_as(P)) == L.E_ARG
    assert lib.dugks_set_B(h, 4, a.ctypes.data_as(P), a.ctypes.data_as(P)) == L.OK
    lib.dugks_destroy(h)


def test_invalid_handles():
    lib = L.lib()
    assert lib.dugks_step(None, 1) == L.E_ARG
    assert lib.dugks_last_error(None) == b"invalid handle"
    lib.dugks_destroy(None)


def test_source_is_refused_where_it_is_not_built():
    """Sources run in binary64 / binary32 storage with the fused kernel; the
    host refuses the other combinations before any device work."""
    lib = L.lib()
    for kw in (dict(storage=L.F16NEQ), dict(storage=L.BF16NEQ),
               dict(storage=L.F64, kernel=L.KERNEL_PLAIN)):
        rc, h = _create(**kw)
        assert rc == L.OK
        assert lib.dugks_set_source(h, C.c_void_p(8), 0.5) == L.E_UNSUPPORTED
        assert "source" in lib.dugks_last_error(h).decode()
        assert lib.dugks_set_source(h, None, 0.0) == L.OK
        lib.dugks_destroy(h)


def test_dirichlet_axis_beside_mirror_axis_is_accepted():
    for bc in ((1, 1, 2, 2), (2, 2, 1, 1)):
        rc, h = _create(bc=bc)
        assert rc == L.OK, L.lib().dugks_last_error(h).decode()
        L.lib().dugks_destroy(h)


def _create3(nx=8, ny=6, nz=5, q=19, **kw):
    lib = L.lib()
    f = [np.linspace(0, 1, n + 1) for n in (nx, ny, nz)]
    p = L.Params3()
    p.abi_version = kw.get("abi", L.ABI3_VERSION)
    p.storage = kw.get("storage", L.F64)
    for i, b in enumerate(kw.get("bc", (0, 0, 0))):
        p.bc[i] = b
    p.c, p.cfl, p.alpha = kw.get("c", 1.0), kw.get("cfl", 0.5), kw.get("alpha", 1e-3)
    h = C.c_void_p()
    P = C.POINTER(C.c_double)
    rc = lib.dugks3_create(C.byref(h), nx, ny, nz, f[0].ctypes.data_as(P), f[1].ctypes.data_as(P),
                           f[2].ctypes.data_as(P), q, C.byref(p))
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(q=9), L.E_UNSUPPORTED), (dict(storage=L.F16NEQ), L.E_UNSUPPORTED),
    (dict(bc=(3, 0, 0)), L.E_ARG), (dict(cfl=1.0), L.E_ARG), (dict(nz=0), L.E_ARG),
    (dict(abi=99), L.E_ARG),
])
def test_create3_rejects_bad_arguments(kw, code):
    rc, h = _create3(**kw)
    assert rc == code
    assert L.lib().dugks3_last_error(h).decode()
    L.lib().dugks3_destroy(h)


def test_3d_sizes_and_state_errors():
    lib = L.lib()
    for storage, per in ((L.F64, 8 * 19), (L.F32, 4 * 19)):
        rc, h = _create3(nx=100, ny=6, nz=5, storage=storage)
        assert rc == L.OK
        info = L.Info3()
        assert lib.dugks3_get_info(h, C.byref(info)) == L.OK
        assert info.pitch == 128 and info.state_bytes == per * 128 * 6 * 5
        assert info.nz == 5 and info.q == 19
        assert lib.dugks3_workspace_bytes(h) >= 2 * info.state_bytes
        assert lib.dugks3_step(h, 1) == L.E_STATE
        assert lib.dugks3_autotune(h, 2) == L.E_STATE      # not bound: no trial step
        # rows per block: binary64 1..2 interior rows, binary32 2..4 rows
        bad, good = ((3, 0), (1, 2)) if storage == L.F64 else ((5, 1), (2, 4))
        for rows in bad:
            assert lib.dugks3_set_launch(h, rows, 8) == L.E_ARG
        assert lib.dugks3_set_launch(h, good[0], 0) == L.E_ARG
        for rows in good:
            assert lib.dugks3_set_launch(h, rows, 16) == L.OK
        lib.dugks3_destroy(h)


def test_3d_dirichlet_data_arguments():
    """Dirichlet walls are accepted; their data is checked (no device work)."""
    lib = L.lib()
    rc, h = _create3(bc=(1, 2, 0))
    assert rc == L.OK
    P = C.POINTER(C.c_double)
    assert lib.dugks3_set_dirichlet(h, None, 3) == L.E_ARG
    assert lib.dugks3_set_dirichlet(h, C.cast(C.c_void_p(256), P), -1) == L.E_ARG
    assert lib.dugks3_set_dirichlet(h, None, 0) == L.OK
    assert lib.dugks3_step(h, 1) == L.E_STATE        # not bound
    lib.dugks3_destroy(h)


def test_3d_source_term_arguments():
    """Every lattice takes the source in the fused step: no scratch; the terms are checked."""
    lib = L.lib()
    g = C.c_void_p(256)
    pw = (C.c_int * 2)(0, 3)
    gm = (C.c_double * 2)(0.1, -0.2)
    for q in (19, 15, 7):
        rc, h = _create3(q=q, bc=(0, 2, 1))
        assert rc == L.OK
        assert lib.dugks3_source_scratch_bytes(h) == 0
        assert lib.dugks3_set_source_terms(h, 7, g, pw, gm, None, 0) == L.E_ARG      # too many terms
        bad = (C.c_int * 2)(0, 4)
        assert lib.dugks3_set_source_terms(h, 2, g, bad, gm, None, 0) == L.E_ARG     # power
        nan = (C.c_double * 2)(0.1, float("nan"))
        assert lib.dugks3_set_source_terms(h, 2, g, pw, nan, None, 0) == L.E_ARG     # rate
        assert lib.dugks3_set_source_terms(h, 2, None, pw, gm, None, 0) == L.E_ARG   # no G
        assert lib.dugks3_set_source_terms(h, 2, g, pw, gm, None, 0) == L.OK
        assert lib.dugks3_set_source_terms(h, 0, None, None, None, None, 0) == L.OK
        lib.dugks3_destroy(h)


def test_3d_batch_arguments():
    """Batch creation and binding are checked on the host, with no device work."""
    lib = L.lib()
    P = C.c_void_p
    hs = [_create3(nx=20 + k, q=19)[1] for k in range(2)]
    h15 = _create3(q=15)[1]
    h7 = _create3(q=7)[1]
    h32 = _create3(q=19, storage=L.F32)[1]
    b = P()
    assert lib.dugks3_batch_create(C.byref(b), 0, (P * 1)(hs[0])) == L.E_ARG
    lib.dugks3_batch_destroy(b)
    assert lib.dugks3_batch_create(C.byref(b), 2, (P * 2)(hs[0], h15)) == L.E_ARG        # lattices
    lib.dugks3_batch_destroy(b)
    assert lib.dugks3_batch_create(C.byref(b), 2, (P * 2)(hs[0], h32)) == L.E_ARG        # storages
    lib.dugks3_batch_destroy(b)
    assert lib.dugks3_batch_create(C.byref(b), 1, (P * 1)(h7)) == L.E_UNSUPPORTED         # D3Q7
    lib.dugks3_batch_destroy(b)
    assert lib.dugks3_batch_create(C.byref(b), 2, (P * 2)(*hs)) == L.OK
    nb = lib.dugks3_batch_workspace_bytes(b)
    assert nb >= 2 * 8 + 3 * 8
    assert lib.dugks3_batch_step(b, 1) == L.E_STATE                                       # not bound
    assert lib.dugks3_batch_bind(b, P(4096), nb, None) == L.E_STATE                        # instances unbound
    assert lib.dugks3_batch_bind(b, P(4100), nb, None) == L.E_ARG                          # alignment
    assert lib.dugks3_batch_bind(b, P(4096), nb - 1, None) == L.E_NOMEM
    assert lib.dugks3_batch_set_launch(b, 3, 8) == L.E_ARG                                 # binary64 rows
    assert lib.dugks3_batch_set_launch(b, 2, 0) == L.E_ARG
    assert lib.dugks3_batch_set_launch(b, 1, 16) == L.OK
    rows, planes, blocks, cells = C.c_int(), C.c_int(), C.c_longlong(), C.c_longlong()
    assert lib.dugks3_batch_get_info(b, C.byref(rows), C.byref(planes), C.byref(blocks), C.byref(cells)) == L.OK
    assert (rows.value, planes.value, cells.value) == (1, 16, (20 + 21) * 6 * 5)
    assert blocks.value == sum(((20 + k + 61) // 62) * 6 * 1 for k in range(2))
    assert lib.dugks3_batch_last_error(b).decode()
    lib.dugks3_batch_destroy(b)
    for h in hs + [h15, h7, h32]:
        lib.dugks3_destroy(h)


def test_d3q7_accepts_only_identity_diffusion():
    lib = L.lib()
    rc, h = _create3(q=7)
    assert rc == L.OK
    P = C.POINTER(C.c_double)
    eye = np.array([0, 1, 0, 1, 0, 1, 0, 0, 0, 0, 0, 0], dtype=float)
    assert lib.dugks3_set_D(h, 1, eye.ctypes.data_as(P)) == L.OK
    bad = eye.copy(); bad[1] = 2.0
    assert lib.dugks3_set_D(h, 1, bad.ctypes.data_as(P)) == L.E_UNSUPPORTED
    lib.dugks3_destroy(h)


def _create1(nx=10, **kw):
    lib = L.lib()
    xf = kw.get("xf", np.linspace(0, 1, nx + 1))
    p = L.Params1()
    p.abi_version = kw.get("abi", L.ABI1_VERSION)
    p.storage = kw.get("storage", L.F64)
    p.bc = kw.get("bc", 1)
    p.c, p.cfl, p.alpha = kw.get("c", 1.0), kw.get("cfl", 0.5), kw.get("alpha", 1e-3)
    for k, v in enumerate(kw.get("coef", (0.1, 0.2, 1.0, 0.5, 0.1, 1.0, 0.3))):
        p.coef[k] = v
    p.t0 = kw.get("t0", 0.0)
    h = C.c_void_p()
    rc = lib.dugks1_create(C.byref(h), nx, np.ascontiguousarray(xf, dtype=np.float64).ctypes.data_as(
        C.POINTER(C.c_double)), C.byref(p))
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(storage=L.F16NEQ), L.E_UNSUPPORTED), (dict(bc=2), L.E_UNSUPPORTED), (dict(cfl=1.0), L.E_ARG),
    (dict(nx=0), L.E_ARG), (dict(abi=99), L.E_ARG), (dict(c=-1.0), L.E_ARG), (dict(alpha=0.0), L.E_ARG),
    (dict(bc=0), L.E_ARG),                       # periodic walls with an x-dependent b
    (dict(xf=np.array([0, 0.5, 0.4, 1.0]), nx=3), L.E_ARG),
    (dict(coef=(0, 0, float("nan"), 0, 0, 1, 0)), L.E_ARG),
])
def test_create1_rejects_bad_arguments(kw, code):
    rc, h = _create1(**kw)
    assert rc == code
    assert L.lib().dugks1_last_error(h).decode()
    L.lib().dugks1_destroy(h)


def test_1d_sizes_and_state_errors():
    lib = L.lib()
    for storage, per in ((L.F64, 8), (L.F32, 4)):
        rc, h = _create1(nx=100, storage=storage)
        assert rc == L.OK
        info = L.Info1()
        assert lib.dugks1_get_info(h, C.byref(info)) == L.OK
        assert info.nx == 100 and info.state_bytes == 4 * 128 * per
        assert math.isclose(info.dt, 0.5 * 0.01 / 1.0) and math.isclose(info.lambda_, 1e-3 * 3.0)
        assert lib.dugks1_workspace_bytes(h) >= 2 * info.state_bytes
        assert lib.dugks1_step(h, 1) == L.E_STATE
        assert lib.dugks1_set_dirichlet(h, None, 3) == L.E_ARG
        lib.dugks1_destroy(h)
    rc, h = _create1(nx=16, bc=0, coef=(0, 0, 1.0, 0.5, 0.1, 1.0, 0.3))
    assert rc == L.OK
    g = np.zeros(4)
    assert lib.dugks1_set_dirichlet(h, g.ctypes.data_as(C.POINTER(C.c_double)), 2) == L.E_STATE
    lib.dugks1_destroy(h)


def test_eight_wave_blocks_only_at_two_waves_per_simd():
    """8-wave blocks: binary32 / 16-bit storage without a source; binary64 and
    the source path (one wave per SIMD) refuse them, and a source set later
    turns an 8 into 4."""
    lib = L.lib()
    for storage, ok in ((L.F64, False), (L.F32, True), (L.BF16NEQ, True)):
        rc, h = _create(storage=storage)
        assert rc == L.OK
        assert (lib.dugks_set_launch(h, 8, 8, 0, 1) == L.OK) == ok
        if storage == L.F32:
            assert lib.dugks_set_source(h, C.c_void_p(256), 0.0) == L.OK
            info = L.Info()
            assert lib.dugks_get_info(h, C.byref(info)) == L.OK
            assert info.waves_per_block == 4
            assert lib.dugks_set_launch(h, 8, 8, 0, 1) == L.E_ARG
        lib.dugks_destroy(h)


def _lds3(q, f32, rows, walls):
    """LDS bytes of a D3Q15/D3Q19 block as the launch documentation states
    them: g of 3 planes of rows + 2 rows; staged f~ of 1 or 2 planes (rows + 2
    rows with two waves a row, the rows alone with four, whose halo rows go
    through registers); 4 face sums per row and wave; with the halo rows in
    registers 2 x 4 x 64 binary64 phi sums.  Binary32 takes one slot where that
    alone brings the block within 80 KiB, binary64 always one."""
    e = 4 if f32 else 8
    four = (q == 19 or not walls) and ((f32 and rows >= 3) or (not f32 and rows == 2))
    parts = 4 if four else 2
    staged = rows if four else rows + 2
    hs = 2 * 4 * 64 * 8 if four else 0
    def size(ns):
        return 3 * (rows + 2) * q * 64 * e + ns * staged * q * 64 * e + 4 * rows * parts * 64 * e + hs
    if not f32:
        return size(1)
    return size(1) if size(2) > 81920 and size(1) <= 81920 else size(2)


def _default_launch3(nx, ny, nz, q, f32, walls):
    """The default launch as documented: rows 2 (binary64) or 4 (binary32;
    D3Q15 with walls 2); planes for D3Q15/19 the power of two in 4..128
    minimising (rounds of blocks over 256 CUs x blocks a CU) x (planes + 3),
    the longer on a tie; D3Q7 32 halved down to 4 while under 512 blocks."""
    rows = 2 if not f32 or (q == 15 and walls) else 4
    strips, tiles = -(-nx // 62), -(-ny // rows)
    if q == 7:
        planes = 32
        while planes > 4 and strips * tiles * -(-nz // planes) < 512:
            planes //= 2
    else:
        slots = 256 * max(1, 163840 // _lds3(q, f32, rows, walls))
        best = None
        for pl in (128, 64, 32, 16, 8, 4):
            cost = -(-(strips * tiles * -(-nz // pl)) // slots) * (pl + 3)
            if best is None or cost < best[0]:
                best = (cost, pl)
        planes = best[1]
    return rows, planes, strips * tiles * -(-nz // planes)


@pytest.mark.parametrize("q", [19, 15, 7])
@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("bc", [(0, 0, 0), (2, 0, 2)])
def test_3d_default_launch_follows_the_documented_model(q, storage, bc):
    """Host logic only (no device work): the default rows, chunk length and
    block count of dugks3_create against the rule the header documents, on
    cubes and ragged boxes, unchanged by source terms; at 256^3 the measured
    best (64 planes binary32, 128 binary64 for D3Q19)."""
    lib = L.lib()
    f32 = storage == "f32"
    walls = any(b != 0 for b in bc)
    for nx, ny, nz in ((48, 48, 48), (64, 64, 64), (128, 128, 128), (192, 192, 192), (256, 256, 256),
                       (100, 37, 211), (31, 5, 300), (300, 200, 150), (1, 1, 1), (700, 3, 9)):
        rc, h = _create3(nx=nx, ny=ny, nz=nz, q=q, storage=L.F32 if f32 else L.F64, bc=bc)
        assert rc == L.OK, lib.dugks3_last_error(h)
        info = L.Info3()
        assert lib.dugks3_get_info(h, C.byref(info)) == L.OK
        got = (info.rows_per_block, info.planes_per_block, info.blocks)
        # a source keeps the default launch (unbound: the terms are only recorded)
        pw, gm = (C.c_int * 2)(0, 1), (C.c_double * 2)(0.0, 0.3)
        assert lib.dugks3_set_source_terms(h, 2, C.c_void_p(256), pw, gm, None, 0) == L.OK
        assert lib.dugks3_get_info(h, C.byref(info)) == L.OK
        assert (info.rows_per_block, info.planes_per_block, info.blocks) == got, (nx, ny, nz)
        lib.dugks3_destroy(h)
        assert got == _default_launch3(nx, ny, nz, q, f32, walls), (nx, ny, nz)
        if (nx, ny, nz) == (256, 256, 256) and q == 19:
            assert got[1] == (64 if f32 else 128)


def test_source_terms_validation_without_a_device():
    """dugks_set_source_terms checks its arguments before any device work."""
    lib = L.lib()
    rc, h = _create(nx=10, ny=8)
    assert rc == L.OK
    g = C.c_void_p(0x1000)          # never dereferenced on these paths
    pw = (C.c_int * 7)(*([0] * 7))
    gm = np.zeros(7)
    gmp = gm.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.dugks_set_source_terms(h, 7, g, pw, gmp) == L.E_ARG          # more than 6 terms
    pw[0] = 4
    assert lib.dugks_set_source_terms(h, 1, g, pw, gmp) == L.E_ARG          # power above 3
    pw[0] = 2
    gm[0] = float("inf")
    assert lib.dugks_set_source_terms(h, 1, g, pw, gmp) == L.E_ARG          # rate not finite
    gm[0] = -1.0
    assert lib.dugks_set_source_terms(h, 1, None, pw, gmp) == L.E_ARG       # no G
    assert lib.dugks_set_source_terms(h, 1, g, pw, gmp) == L.OK             # not bound: kept
    assert lib.dugks_set_source_terms(h, 0, None, None, None) == L.OK       # removed
    lib.dugks_destroy(h)
    for storage in (L.F16NEQ, L.BF16NEQ):
        rc, h = _create(nx=10, ny=8, storage=storage)
        assert lib.dugks_set_source_terms(h, 1, g, pw, gmp) == L.E_UNSUPPORTED
        lib.dugks_destroy(h)
    rc, h = _create(nx=10, ny=8, kernel=L.KERNEL_PLAIN)
    assert lib.dugks_set_source_terms(h, 1, g, pw, gmp) == L.E_UNSUPPORTED
    lib.dugks_destroy(h)
