"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Binary64 storage must match to 1e-12 (max-norm, relative to max |f~|); the
reduced-precision storages meet the per-format bounds stated in the tests.
"""
import math

import numpy as np
import pytest

import paper_1906_11036_amd as dg
from oracle import Oracle
from paper_1906_11036_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def say(*a):
    print(*a, flush=True)


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def run_gpu(p, steps, storage="f64", kernel=dg.KERNEL_FUSED, launch=None, f0=None):
    s = dg.Solver(p, storage=storage, kernel=kernel, launch=launch)
    if f0 is not None:
        s.set_f(f0)
    else:
        s.set_phi(p.phi0)
    rings = p.rings(steps) if steps else None
    if rings is not None:
        s.set_dirichlet(rings)
    s.step(steps)
    return s


def run_oracle(p, steps, f0=None):
    o = Oracle(p)
    if f0 is not None:
        o.set_f(f0)
    o.step(steps, p.rings(steps) if steps else None)
    return o


SIZES = [(1, 1), (2, 3), (5, 4), (61, 7), (62, 9), (63, 5), (64, 6), (65, 3), (124, 4), (125, 11),
         (130, 17), (17, 70)]


@pytest.mark.parametrize("nx,ny", SIZES)
@pytest.mark.parametrize("bc", [W.PERIODIC, W.DIRICHLET, W.MIRROR])
def test_fp64_fused_random_problems(nx, ny, bc):
    if bc != W.PERIODIC and (nx < 2 or ny < 2):
        pytest.skip("walls need two cells per axis for distinct ghosts")
    p = W.random_problem(100 + nx * 7 + ny, nx, ny, bcx=bc, bcy=bc, stretched=(bc == W.MIRROR),
                         bdeg=2, ddeg=2)
    if bc == W.MIRROR:
        p.bx, p.by = (0.0,), (0.0,)
    say(f"case fp64 fused nx={nx} ny={ny} bc={bc}")
    s = run_gpu(p, 4)
    o = run_oracle(p, 4)
    assert rel_max(s.get_f(), o.get_f()) <= TOL64


@pytest.mark.parametrize("q", [9, 5])
@pytest.mark.parametrize("bcx,bcy", [(W.PERIODIC, W.DIRICHLET), (W.DIRICHLET, W.PERIODIC),
                                     (W.PERIODIC, W.MIRROR), (W.MIRROR, W.PERIODIC),
                                     (W.DIRICHLET, W.MIRROR), (W.MIRROR, W.DIRICHLET)])
def test_fp64_mixed_axes_and_d2q5(q, bcx, bcy):
    p = W.random_problem(7 + q + 3 * bcx + bcy, 70, 23, q=q, bcx=bcx, bcy=bcy, stretched=True,
                         bdeg=3, ddeg=1)
    if W.MIRROR in (bcx, bcy):
        p.bx, p.by = (0.0, 0.1, 0.2), (0.0, 0.1, 0.2)
    say(f"case mixed q={q} bcx={bcx} bcy={bcy}")
    s = run_gpu(p, 3)
    o = run_oracle(p, 3)
    assert rel_max(s.get_f(), o.get_f()) <= TOL64


@pytest.mark.parametrize("deg", [(1, 1), (2, 3), (4, 4)])
def test_fp64_polynomial_degrees(deg):
    p = W.random_problem(55 + deg[0], 40, 33, bdeg=deg[0], ddeg=deg[1])
    say(f"case degrees {deg}")
    s = run_gpu(p, 3)
    o = run_oracle(p, 3)
    assert rel_max(s.get_f(), o.get_f()) <= TOL64


@pytest.mark.parametrize("kernel", [dg.KERNEL_FUSED, dg.KERNEL_PLAIN])
def test_gaussian_hill_128_full_run(kernel):
    """Linear CDE, Gaussian hill, 128^2 periodic, 500 steps, FP64."""
    p = W.gaussian_hill_problem(128, steps=500)
    say(f"case gaussian hill 128 kernel={kernel}")
    s = run_gpu(p, 500, kernel=kernel)
    o = run_oracle(p, 500)
    assert rel_max(s.get_f(), o.get_f()) <= TOL64
    phi = s.get_phi()
    assert rel_max(phi, o.get_phi()) <= TOL64
    X, Y = p.mesh()
    gre, l2 = s.error_norms(p.exact(X, Y, o.time))
    gre_o, l2_o = o.errors(p.exact(X, Y, o.time))
    assert abs(gre - gre_o) <= 1e-10 * gre_o and abs(l2 - l2_o) <= 1e-10 * l2_o


def test_burgers_dirichlet_128():
    """Burgers front with NEE walls, 128^2, 300 steps, FP64 fused and plain."""
    p = W.burgers_problem(128, steps=300)
    say("case burgers 128")
    o = run_oracle(p, 300)
    for kernel in (dg.KERNEL_FUSED, dg.KERNEL_PLAIN):
        s = run_gpu(p, 300, kernel=kernel)
        assert rel_max(s.get_f(), o.get_f()) <= TOL64


def test_nonlinear_diffusion_stretched_128():
    p = W.nonlinear_diffusion_problem(128, steps=200)
    say("case nonlinear diffusion 128")
    o = run_oracle(p, 200)
    s = run_gpu(p, 200)
    assert rel_max(s.get_f(), o.get_f()) <= TOL64
    s32 = run_gpu(p, 200, storage="f32")
    err = rel_max(s32.get_phi(), o.get_phi())
    say(f"  f32 max rel err {err:.2e}")
    # each binary32 step rounds every stored value and the arithmetic before it
    # (a few ulp); over n steps these add at worst linearly: 2 n eps32
    assert err <= 2 * 200 * np.finfo(np.float32).eps


@pytest.mark.parametrize("name,n,storage,tol", [
    ("burgers", 512, "f64", TOL64), ("nonlinear_diffusion", 1024, "f64", TOL64),
    ("gaussian_hill", 4096, "f32", 2e-6), ("burgers", 512, "f32", 2e-6)])
def test_full_size_one_step_sampled(name, n, storage, tol):
    """Full-size grids in the launch configuration of the benchmark: one step
    from a seeded non-equilibrium state, checked at sampled cells (edges,
    corners, strip seams and random interior cells) against the oracle."""
    if name == "burgers":
        p = W.burgers_problem(n, steps=1)
    elif name == "nonlinear_diffusion":
        p = W.nonlinear_diffusion_problem(n, steps=1)
    else:
        p = W.gaussian_hill_problem(n, u=(0.05, 0.02), D=1e-4, steps=1)
    say(f"case full size {name} {n} {storage}")
    f0 = W.random_distributions(9000 + n, p.q, p.ny, p.nx)
    s = run_gpu(p, 1, storage=storage, f0=f0)
    gpu = s.get_f()
    del s
    o = Oracle(p)
    o.set_f(f0)
    rng = np.random.default_rng(n)
    pts = set()
    for i in (0, 1, 61, 62, 63, 123, 124, n - 2, n - 1):
        for j in (0, 1, 63, 64, n - 1, n // 2):
            pts.add((i, j))
    for _ in range(600):
        pts.add((int(rng.integers(0, n)), int(rng.integers(0, n))))
    cells = np.array(sorted(pts))
    ring = p.rings(1)
    ref = o.step_cells(cells, ring[0] if ring is not None else None)
    got = gpu[:, cells[:, 1], cells[:, 0]].T
    err = float(np.abs(got - ref).max() / np.abs(f0).max())
    say(f"  sampled max rel err {err:.2e}")
    assert err <= tol


def test_launch_shape_invariance_bitwise():
    """FP64 results do not depend on rows per wave, waves per block, schedule
    or the XCD remap: every cell's arithmetic is the same in each tiling."""
    p = W.random_problem(321, 150, 97, bcx=W.PERIODIC, bcy=W.DIRICHLET, bdeg=2, ddeg=2)
    say("case launch invariance")
    ref = None
    for launch in ((64, 2, dg.SCHED_GRID, 1), (1, 1, dg.SCHED_GRID, 0), (7, 2, dg.SCHED_PERSISTENT, 1),
                   (97, 1, dg.SCHED_PERSISTENT, 0), (150, 1, dg.SCHED_GRID, 1), (33, 2, dg.SCHED_GRID, 1),
                   (3, 4, dg.SCHED_GRID, 1)):
        s = run_gpu(p, 6, launch=launch)
        f = s.get_f()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f, ref), launch


@pytest.mark.parametrize("storage", ["f32", "bf16neq"])
def test_eight_wave_blocks_bitwise(storage):
    """Binary32 and 16-bit storage: 8-wave blocks give the 4-wave results bit for
    bit (every wave runs its own work item), grid and persistent schedules."""
    p = W.random_problem(322, 150, 97, bcx=W.PERIODIC, bcy=W.DIRICHLET, bdeg=2, ddeg=2)
    ref = run_gpu(p, 5, storage=storage, launch=(8, 4, dg.SCHED_GRID, 1)).get_f()
    for launch in ((8, 8, dg.SCHED_GRID, 1), (3, 8, dg.SCHED_PERSISTENT, 1), (16, 8, dg.SCHED_GRID, 0)):
        assert np.array_equal(run_gpu(p, 5, storage=storage, launch=launch).get_f(), ref), launch


def test_checkpoint_round_trip_bitwise():
    p = W.random_problem(77, 90, 40, bdeg=2, ddeg=2)
    say("case checkpoint")
    for storage in ("f64", "f32", "f16neq", "bf16neq"):
        a = run_gpu(p, 10, storage=storage)
        a.step(7)
        full = a.get_f()
        b = run_gpu(p, 10, storage=storage)
        blob = b.checkpoint()
        c = dg.Solver(p, storage=storage)
        c.restore(blob)
        c.step(7)
        assert np.array_equal(c.get_f(), full), storage
        bad = bytearray(blob)
        bad[-1] ^= 1
        with pytest.raises(dg.DugksError):
            c.restore(bytes(bad))


def test_mass_conservation_and_diag():
    p = W.random_problem(12, 200, 130, bdeg=3, ddeg=3)
    say("case mass")
    s = run_gpu(p, 0)
    m0 = s.diag()["mass"]
    s.step(1000)
    d = s.diag()
    assert d["step"] == 1000 and abs(d["t"] - 1000 * d["dt"]) < 1e-12
    assert abs(d["mass"] - m0) <= 1e-12 * abs(m0)


def test_nonfinite_input_is_reported():
    p = W.random_problem(13, 70, 20)
    phi = p.phi0.copy()
    phi[5, 7] = np.nan
    s = dg.Solver(p, storage="f32")
    s.set_phi(phi)
    s.step(3)
    d = s.diag(check=False)
    assert d["rc"] == dg._lib.E_UNSTABLE and d["flags"] & dg._lib.FLAG_NONFINITE


def test_dirichlet_data_must_cover_steps():
    p = W.burgers_problem(64, steps=5)
    s = dg.Solver(p, storage="f64")
    s.set_phi(p.phi0)
    s.set_dirichlet(p.rings(5))
    s.step(5)
    with pytest.raises(dg.DugksError):
        s.step(1)


def test_autotune_refuses_exhausted_dirichlet_data():
    """Autotune's trial steps read the current step's ghost data: once the data
    is used up they are refused (no kernel reads past the caller's array)."""
    p = W.burgers_problem(64, steps=5)
    s = dg.Solver(p, storage="f64")
    s.set_phi(p.phi0)
    s.set_dirichlet(p.rings(5))
    s.autotune(1)              # data for step 0 is there
    s.step(5)
    with pytest.raises(dg.DugksError) as ei:
        s.autotune(1)
    assert ei.value.code == dg._lib.E_STATE


def test_error_norms_of_a_nonfinite_state_are_refused():
    """A state with a non-finite cell has no error norm: E_UNSTABLE (and NaN from
    the allocation-free variant), not the norm of the finite cells."""
    import ctypes as C

    import torch
    p = W.random_problem(14, 40, 30)
    phi = p.phi0.copy()
    phi[3, 4] = np.inf
    s = dg.Solver(p, storage="f64")
    s.set_phi(phi)
    with pytest.raises(dg.DugksError) as ei:
        s.error_norms(p.phi0)
    assert ei.value.code == dg._lib.E_UNSTABLE
    r = torch.from_numpy(p.phi0).to(s.device)
    out = torch.zeros(2, dtype=torch.float64, device=s.device)
    assert dg._lib.lib().dugks_error_norms_noalloc(s.h, C.c_void_p(r.data_ptr()),
                                                   C.c_void_p(out.data_ptr())) == 0
    torch.cuda.synchronize()
    assert np.isnan(out.cpu().numpy()).all()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_graph_replay_with_dirichlet_data_and_sources(storage):
    """Captured graphs take their step index from a base written before each
    replay, so runs with Dirichlet data (the ring of each step) and with
    time-dependent sources replay graphs too: bit for bit the eager steps."""
    p = W.burgers_problem(100, steps=80)
    q = W.random_problem(611, 90, 70, bdeg=2, ddeg=2)
    q.cfl = 0.4   # as drawn (0.79) this problem is unstable within 150 steps, oracle included
    q.src_terms = W.random_source_terms(612, q, nterms=4, amp=1.0)
    for prob in (p, q):
        a = dg.Solver(prob, storage=storage)
        e = dg.Solver(prob, storage=storage)
        for s in (a, e):
            s.set_phi(prob.phi0)
            if prob.rings(1) is not None:
                s.set_dirichlet(prob.rings(80))
        for n in (36, 4, 3, 9, 28):
            a.step(n)
            for _ in range(n):
                e.step(1)
        assert a.info()["graph_steps"] >= 36 + 4 + 4 + 28
        fa = a.get_f()
        assert np.isfinite(fa).all()
        assert np.array_equal(fa, e.get_f()), prob.name
