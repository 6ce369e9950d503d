"""The allocation-free norms entry point (dugks_error_norms_noalloc) against
dugks_error_norms, through the C ABI: two calls in a row, the second on a
smaller instance, each compared with the allocating entry point's result."""
import ctypes as C

import numpy as np
import pytest

import paper_1906_11036_amd as dg
from paper_1906_11036_amd import _lib as L
from paper_1906_11036_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def norms_both(s, ref):
    """(rel_l2, gre) from dugks_error_norms and from the allocation-free variant."""
    import torch
    lib = L.lib()
    r = torch.from_numpy(np.ascontiguousarray(ref, dtype=np.float64)).to(s.device)
    l2, gre = C.c_double(), C.c_double()
    L.check(lib.dugks_error_norms(s.h, C.c_void_p(r.data_ptr()), C.byref(l2), C.byref(gre)), s.h,
            "dugks_error_norms")
    out = torch.full((2,), float("nan"), dtype=torch.float64, device=s.device)
    L.check(lib.dugks_error_norms_noalloc(s.h, C.c_void_p(r.data_ptr()), C.c_void_p(out.data_ptr())),
            s.h, "dugks_error_norms_noalloc")
    torch.cuda.current_stream(s.device).synchronize()
    o = out.cpu().numpy()
    return (l2.value, gre.value), (float(o[0]), float(o[1]))


def check_pair(a, b):
    # same partial sums in the same order; the final division and square root
    # run on the device in one case and on the host in the other
    for x, y in zip(a, b):
        assert abs(x - y) <= 4 * np.finfo(np.float64).eps * abs(x), (a, b)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16neq"])
def test_noalloc_norms_match_allocating_entry_point(storage):
    big = W.gaussian_hill_problem(300, u=(0.05, 0.02), D=1e-3, sigma0=0.1, steps=20)
    small = W.random_problem(41, 37, 23, bdeg=2, ddeg=2)
    results = []
    for p, steps in ((big, 20), (small, 5)):
        say(f"case noalloc norms storage={storage} n={p.nx}x{p.ny}")
        s = dg.Solver(p, storage=storage)
        s.set_phi(p.phi0)
        s.step(steps)
        X, Y = p.mesh()
        ref = p.exact(X, Y, steps * s.info()["dt"])
        alloc, noalloc = norms_both(s, ref)
        say(f"  alloc {alloc} noalloc {noalloc}")
        check_pair(alloc, noalloc)
        assert alloc[0] > 0 and alloc[1] > 0
        results.append(noalloc)
        s.close()
    # the second, smaller call did not see the first one's partial sums
    assert results[0] != results[1]


def test_noalloc_norms_refuse_without_state():
    p = W.random_problem(42, 20, 10)
    s = dg.Solver(p, storage="f64")
    import torch
    r = torch.zeros((p.ny, p.nx), dtype=torch.float64, device=s.device)
    out = torch.zeros(2, dtype=torch.float64, device=s.device)
    rc = L.lib().dugks_error_norms_noalloc(s.h, C.c_void_p(r.data_ptr()), C.c_void_p(out.data_ptr()))
    assert rc == L.E_STATE
    rc = L.lib().dugks_error_norms_noalloc(s.h, None, C.c_void_p(out.data_ptr()))
    assert rc == L.E_ARG
