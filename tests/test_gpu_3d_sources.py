"""Three-dimensional sources F(x, t, phi) = sum_j exp(gamma_j t) phi^k_j G_j(x)
on the GPU (the fused source step, through the C ABI of include/dugks3d.h)
against the 3-D CPU oracle: binary64 to 1e-12 (max-norm relative to max |f~|)
on all three lattices and every wall kind; binary32 within 2 n eps32 (relative
L2 of phi); a uniform field follows the implicit trapezoidal rule; with all
G_j = 0 the source step equals the fused source-free step to 1e-12."""
import math

import numpy as np
import pytest

import paper_1906_11036_amd as dg
from oracle import Oracle3D
from paper_1906_11036_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)
P, M, D = W.PERIODIC, W.MIRROR, W.DIRICHLET


def say(*a):
    print(*a, flush=True)


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def run_pair(p, steps, storage="f64"):
    rings = p.rings(steps)
    s = dg.Solver3D(p, storage=storage)
    s.set_phi(p.phi0)
    if rings is not None:
        s.set_dirichlet(rings)
    s.step(steps)
    o = Oracle3D(p, openmp=True)
    o.step(steps, rings)
    return s, o


CASES = [(1, 1, 1, 19, (P, P, P)), (9, 7, 6, 19, (P, P, P)), (17, 5, 4, 19, (D, M, P)),
         (66, 6, 5, 19, (M, D, D)), (10, 9, 8, 15, (P, M, D)), (33, 4, 7, 15, (D, D, D)),
         (12, 11, 5, 7, (P, P, M)), (20, 6, 9, 7, (D, P, M))]


@pytest.mark.parametrize("nx,ny,nz,q,bc", CASES)
def test_fp64_sources_match_oracle(nx, ny, nz, q, bc):
    p = W.random_problem3d(500 + nx + 3 * ny + 7 * nz, nx, ny, nz, q=q, bc=bc, stretched=True, bdeg=2,
                           ddeg=2)
    p.src_terms = W.random_source_terms3d(600 + nx, p, nterms=5, amp=1.2)
    say(f"case 3d source f64 {nx}x{ny}x{nz} q={q} bc={bc} powers {[k for k, _, _ in p.src_terms]}")
    s, o = run_pair(p, 5)
    assert rel_max(s.get_f(), o.get_f()) <= 1e-12
    assert rel_max(s.get_phi(), o.get_phi()) <= 1e-12
    r = s.reduce()
    assert abs(r["mass"] - o.mass()) <= 1e-12 * abs(o.mass())


@pytest.mark.parametrize("q", [19, 15, 7])
def test_fp32_sources_against_oracle(q):
    p = W.random_problem3d(700 + q, 40, 12, 10, q=q, bc=(P, M, D), stretched=True, bdeg=2)
    p.src_terms = W.random_source_terms3d(701, p, nterms=4)
    steps = 30
    s, o = run_pair(p, steps, storage="f32")
    ref = o.get_phi()
    err = float(np.sqrt(((s.get_phi() - ref) ** 2).sum() / (ref ** 2).sum()))
    say(f"  3d f32 source q={q}: rel-L2 {err:.2e} (bound {2 * steps * EPS32:.2e})")
    assert err <= 2 * steps * EPS32


def test_uniform_logistic_field_3d():
    from scipy.optimize import brentq
    f = W.uniform_faces(6, 0.0, 1.0)
    p = W.Problem3D(name="uniform", xf=f, yf=f, zf=f, q=19, c=2.0, cfl=0.6, alpha=3e-3,
                    b=((0.0, 0.0, 0.3), (0.0, -0.2), (0.0, 0.1)),
                    d=((0.0, 1.0, 0.2), (0.0, 0.8), (0.0, 1.1), (0.0,), (0.0,), (0.0,)))
    one = np.ones((6, 6, 6))
    p.src_terms = [(1, 0.0, 1.5 * one), (3, 0.0, -2.0 * one), (0, 0.7, 0.3 * one)]
    p.phi0 = np.full((6, 6, 6), 0.4)
    s = dg.Solver3D(p, storage="f64")
    s.set_phi(p.phi0)
    dt = s.info()["dt"]

    def F(t, v):
        return 1.5 * v - 2.0 * v ** 3 + 0.3 * math.exp(0.7 * t)

    v, t = 0.4, 0.0
    for _ in range(20):
        s.step(1)
        rhs = v + 0.5 * dt * F(t, v)
        v = brentq(lambda w: w - 0.5 * dt * F(t + dt, w) - rhs, v - 1.0, v + 1.0, xtol=1e-16, rtol=1e-15)
        t += dt
        assert np.abs(s.get_phi() - v).max() <= 1e-14 * abs(v)


@pytest.mark.parametrize("q", [19, 7])
def test_zero_source_equals_fused_step(q):
    p = W.random_problem3d(800 + q, 70, 9, 8, q=q, bc=(D, M, P), stretched=True, bdeg=2)
    rings = p.rings(4)
    a = dg.Solver3D(p, storage="f64")
    a.set_phi(p.phi0)
    a.set_dirichlet(rings)
    a.step(4)
    p.src_terms = [(1, 0.5, np.zeros((p.nz, p.ny, p.nx)))]
    b = dg.Solver3D(p, storage="f64")
    b.set_phi(p.phi0)
    b.set_dirichlet(rings)
    b.step(4)
    assert rel_max(b.get_f(), a.get_f()) <= 1e-12


def test_full_size_source_step_sampled():
    """The 256^3 D3Q19 mesh with two source terms (one depending on phi), binary64: one step of
    the fused source step from a seeded non-equilibrium state, checked at sampled cells
    (faces, edges, corners, strip seams and random interior cells) against the oracle's per-cell
    step, in the default launch."""
    p = W.workload3d("gaussian_hill3d_256")
    n = p.nx
    X, Y, Z = p.mesh()
    p.src_terms = [(1, 0.2, 0.3 * np.cos(np.pi * X) * np.sin(np.pi * Y)), (0, -0.4, 0.1 + 0.05 * Z)]
    del X, Y, Z
    say(f"case full size 3-D source step {n}^3 f64")
    f0 = W.random_distributions3d(4343, p.q, p.nz, p.ny, p.nx)
    s = dg.Solver3D(p, storage="f64")
    s.set_f(f0)
    s.step(1)
    gpu = s.get_f()
    s.close()
    o = Oracle3D(p)
    o.set_f(f0)
    del f0
    rng = np.random.default_rng(n + 1)
    pts = set()
    for i in (0, 1, 61, 62, 63, 64, n - 2, n - 1):
        for j in (0, 1, n // 2, n - 1):
            for k in (0, 1, n - 2, n - 1):
                pts.add((i, j, k))
    for _ in range(300):
        pts.add(tuple(int(v) for v in rng.integers(0, n, size=3)))
    cells = np.array(sorted(pts))
    ref = o.step_cells(cells)
    got = gpu[:, cells[:, 2], cells[:, 1], cells[:, 0]].T
    err = rel_max(got, ref)
    say(f"  sampled max rel err {err:.2e} over {len(cells)} cells")
    assert err <= 1e-12


@pytest.mark.parametrize("storage,launches", [("f32", [(2, 1), (3, 5), (4, 2), (2, 32)]),
                                              ("f64", [(1, 3), (2, 1), (2, 32)])])
@pytest.mark.parametrize("q,bc", [(19, (P, P, P)), (15, (M, D, P))])
def test_fused_source_launch_shapes_give_identical_results(storage, launches, q, bc):
    """The fused source step: tiles of 1 to 4 rows and chunks of 1 to 32 planes give bitwise the
    same state (ragged strips, tiles and chunks; walls of every kind)."""
    p = W.random_problem3d(950 + q, 67, 7, 9, q=q, bc=bc, stretched=True, bdeg=2)
    p.src_terms = W.random_source_terms3d(960 + q, p, nterms=3, amp=1.0)
    say(f"case 3d fused source launch shapes {storage} q={q} bc={bc}")
    out = []
    for ln in launches:
        s = dg.Solver3D(p, storage=storage)
        try:
            s.set_launch(*ln)
        except dg.DugksError as e:
            pytest.skip(f"launch {ln} not available on this device: {e}")
        s.set_phi(p.phi0)
        if D in bc:
            s.set_dirichlet(p.rings(4))
        s.step(4)
        out.append(s.get_f())
        s.close()
    for f in out[1:]:
        assert np.array_equal(f, out[0])


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_fused_source_autotune_keeps_state(storage):
    """dugks3_autotune with a source: the state is unchanged and later steps equal a run
    without it, bitwise."""
    p = W.random_problem3d(970, 70, 9, 7, q=19, bc=(P, M, P), bdeg=2)
    p.src_terms = W.random_source_terms3d(971, p, nterms=2, amp=0.8)
    say(f"case 3d fused source autotune {storage}")
    ref = dg.Solver3D(p, storage=storage)
    ref.set_phi(p.phi0)
    ref.step(5)
    s = dg.Solver3D(p, storage=storage)
    s.set_phi(p.phi0)
    s.step(2)
    f0 = s.get_f()
    s.autotune(2)
    assert np.array_equal(s.get_f(), f0)
    s.step(3)
    assert np.array_equal(s.get_f(), ref.get_f())
