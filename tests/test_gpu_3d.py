"""GPU parity of the three-dimensional path (D3Q15, D3Q19, D3Q7) against the
3-D CPU oracle, through the C ABI of include/dugks3d.h."""
import math

import numpy as np
import pytest

import paper_1906_11036_amd as dg
from oracle import Oracle3D
from paper_1906_11036_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)
P, M = W.PERIODIC, W.MIRROR


def say(*a):
    print(*a, flush=True)


def solver(p, storage, launch=None):
    s = dg.Solver3D(p, storage=storage)
    if launch is not None:
        try:
            s.set_launch(*launch)
        except dg.DugksError as e:
            pytest.skip(f"launch {launch} not available on this device: {e}")
    return s


CASES = [
    (1, 1, 1, 19, (P, P, P)), (5, 4, 3, 19, (P, P, P)), (62, 3, 4, 19, (M, P, M)),
    (63, 5, 2, 19, (P, M, P)), (64, 2, 7, 15, (P, P, P)), (65, 4, 5, 15, (M, M, M)),
    (130, 3, 3, 19, (P, P, P)), (17, 9, 11, 19, (M, P, P)), (9, 7, 6, 7, (P, M, P)),
    (70, 6, 4, 7, (M, M, M)), (33, 5, 4, 7, (P, P, P)),
]


@pytest.mark.parametrize("nx,ny,nz,q,bc", CASES)
def test_fp64_matches_oracle(nx, ny, nz, q, bc):
    p = W.random_problem3d(600 + nx + 3 * ny + 7 * nz, nx, ny, nz, q=q, bc=bc,
                           stretched=any(v == M for v in bc), bdeg=2, ddeg=2)
    say(f"case 3d f64 {nx}x{ny}x{nz} q={q} bc={bc}")
    s = solver(p, "f64", (2, 3))
    s.set_phi(p.phi0)
    s.step(3)
    o = Oracle3D(p)
    o.step(3)
    f, fo = s.get_f(), o.get_f()
    assert np.abs(f - fo).max() <= 1e-12 * np.abs(fo).max()
    r = s.reduce()
    assert abs(r["mass"] - o.mass()) <= 1e-12 * abs(o.mass())


D = W.DIRICHLET
DCASES = [
    (1, 1, 1, 19, (D, D, D)), (5, 4, 3, 19, (D, D, D)), (62, 3, 4, 19, (D, P, M)),
    (63, 5, 2, 19, (P, D, P)), (64, 2, 7, 15, (M, P, D)), (65, 4, 5, 15, (D, M, D)),
    (130, 3, 3, 19, (D, D, P)), (17, 9, 11, 19, (P, P, D)), (9, 7, 6, 7, (D, M, P)),
    (70, 6, 4, 7, (D, D, D)), (130, 67, 20, 19, (D, D, D)),
]


@pytest.mark.parametrize("launch", [(2, 3), (1, 2)])
@pytest.mark.parametrize("nx,ny,nz,q,bc", DCASES)
def test_fp64_dirichlet_walls_match_oracle(nx, ny, nz, q, bc, launch):
    """Dirichlet walls (non-equilibrium extrapolation, data per step on the
    ghost shell) alone and beside mirror and periodic axes: binary64 equals
    the oracle to 1e-12, in tiles of 2 and 1 interior rows."""
    p = W.random_problem3d(900 + nx + 3 * ny + 7 * nz, nx, ny, nz, q=q, bc=bc, stretched=True,
                           bdeg=2, ddeg=2)
    steps = 4
    rings = p.rings(steps)
    say(f"case 3d dirichlet f64 {nx}x{ny}x{nz} q={q} bc={bc} launch={launch}")
    s = solver(p, "f64", launch)
    s.set_phi(p.phi0)
    s.set_dirichlet(rings)
    s.step(steps)
    o = Oracle3D(p, openmp=True)
    o.step(steps, rings)
    f, fo = s.get_f(), o.get_f()
    assert np.abs(f - fo).max() <= 1e-12 * np.abs(fo).max()


@pytest.mark.parametrize("q", [19, 15, 7])
def test_fp32_dirichlet_walls(q):
    """binary32 with Dirichlet walls: launch shapes bitwise the same, and the
    oracle within 2 n eps32 (relative L2 of phi)."""
    bc = (D, M, D) if q != 19 else (D, D, D)
    p = W.random_problem3d(950 + q, 70, 9, 8, q=q, bc=bc, stretched=True, bdeg=2)
    steps = 20
    rings = p.rings(steps)
    say(f"case 3d dirichlet f32 q={q} bc={bc}")
    out = []
    for launch in ((4, 32), (2, 1), (3, 7), (4, 3)):
        s = solver(p, "f32", launch)
        s.set_phi(p.phi0)
        s.set_dirichlet(rings)
        s.step(steps)
        out.append(s.get_f())
        if len(out) == 1:
            phi = s.get_phi()
    for f in out[1:]:
        assert np.array_equal(f, out[0])
    o = Oracle3D(p, openmp=True)
    o.step(steps, rings)
    ref = o.get_phi()
    err = float(np.sqrt(((phi - ref) ** 2).sum() / (ref ** 2).sum()))
    say(f"  rel-L2 {err:.2e} (bound {2 * steps * EPS32:.2e})")
    assert err <= 2 * steps * EPS32


def test_dirichlet_data_must_cover_every_step():
    p = W.random_problem3d(960, 10, 6, 5, q=19, bc=(D, P, P))
    s = solver(p, "f64")
    s.set_phi(p.phi0)
    with pytest.raises(dg.DugksError):
        s.step(1)                      # no data yet
    s.set_dirichlet(p.rings(3))
    s.step(3)
    with pytest.raises(dg.DugksError):
        s.step(1)                      # past the data
    s.set_phi(p.phi0)                  # the clock restarts at step 0
    s.step(2)


@pytest.mark.parametrize("launch", [(2, 1), (2, 5), (3, 2), (3, 7), (4, 1), (4, 3), (2, 32)])
def test_launch_shapes_give_identical_results(launch):
    """Tiles of 2 to 4 rows and chunks of 1..32 planes: bitwise the same (binary32)."""
    p = W.random_problem3d(77, 70, 7, 9, q=19, bc=(P, M, P), stretched=True, bdeg=2)
    ref = solver(p, "f32", (4, 32))
    ref.set_phi(p.phi0)
    ref.step(4)
    s = solver(p, "f32", launch)
    s.set_phi(p.phi0)
    s.step(4)
    assert np.array_equal(s.get_f(), ref.get_f())


@pytest.mark.parametrize("storage,launch", [("f32", (2, 1)), ("f32", (3, 7)), ("f32", (4, 3)),
                                            ("f64", (1, 4)), ("f64", (2, 5))])
@pytest.mark.parametrize("q", [19, 15, 7])
def test_periodic_launch_shapes_give_identical_results(storage, launch, q):
    """All axes periodic (the instantiation without mirror code): launch shapes bitwise the same."""
    p = W.random_problem3d(79, 67, 7, 9, q=q, bc=(P, P, P), bdeg=2)
    ref = solver(p, storage, (4, 32) if storage == "f32" else (2, 32))
    ref.set_phi(p.phi0)
    ref.step(3)
    s = solver(p, storage, launch)
    s.set_phi(p.phi0)
    s.step(3)
    assert np.array_equal(s.get_f(), ref.get_f())


@pytest.mark.parametrize("q", [15, 19, 7])
@pytest.mark.parametrize("launch", [(1, 1), (1, 4), (2, 2), (2, 32)])
def test_fp64_launch_shapes_give_identical_results(launch, q):
    """binary64: tiles of 1 or 2 interior rows and chunks of 1..32 planes, bitwise the same."""
    p = W.random_problem3d(78, 66, 5, 7, q=q, bc=(M, P, M), stretched=True, bdeg=2)
    ref = solver(p, "f64", (2, 32))
    ref.set_phi(p.phi0)
    ref.step(3)
    s = solver(p, "f64", launch)
    s.set_phi(p.phi0)
    s.step(3)
    assert np.array_equal(s.get_f(), ref.get_f())


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("q,bc", [(19, (P, P, P)), (15, (M, P, D)), (7, (D, M, P))])
def test_autotune_keeps_state_and_results(storage, q, bc):
    """dugks3_autotune after some steps: the state is unchanged, the launch it keeps is a
    valid shape, and later steps equal bitwise those of a run without it (with
    Dirichlet walls, the trials read the current step's data only)."""
    p = W.random_problem3d(83, 70, 9, 7, q=q, bc=bc, bdeg=2)
    say(f"case 3d autotune {storage} q={q} bc={bc}")
    ref = solver(p, storage)
    ref.set_phi(p.phi0)
    s = solver(p, storage)
    s.set_phi(p.phi0)
    if D in bc:
        ref.set_dirichlet(p.rings(5))
        s.set_dirichlet(p.rings(5))
    ref.step(5)
    s.step(2)
    f0 = s.get_f()
    s.autotune(2)
    assert np.array_equal(s.get_f(), f0)
    inf = s.info()
    assert inf["rows_per_block"] in ((1, 2) if storage == "f64" else (2, 3, 4))
    assert inf["planes_per_block"] in (4, 8, 16, 32, 64, 128)
    s.step(3)
    assert np.array_equal(s.get_f(), ref.get_f())


def test_autotune_needs_the_current_steps_dirichlet_data():
    p = W.random_problem3d(84, 12, 6, 5, q=19, bc=(D, P, P))
    s = solver(p, "f64")
    s.set_phi(p.phi0)
    s.set_dirichlet(p.rings(2))
    s.step(2)
    with pytest.raises(dg.DugksError):
        s.autotune(1)                  # the data ends at the current step: no trial is launched


@pytest.mark.parametrize("q", [19, 15, 7])
def test_fp32_against_oracle(q):
    p = W.random_problem3d(88 + q, 40, 12, 10, q=q, bc=(P, P, M), bdeg=2)
    steps = 40
    s = solver(p, "f32")
    s.set_phi(p.phi0)
    s.step(steps)
    o = Oracle3D(p, openmp=True)
    o.step(steps)
    ref = o.get_phi()
    err = float(np.sqrt(((s.get_phi() - ref) ** 2).sum() / (ref ** 2).sum()))
    say(f"  3d f32 q={q}: rel-L2 {err:.2e} (bound {2 * steps * EPS32:.2e})")
    assert err <= 2 * steps * EPS32


@pytest.mark.parametrize("q", [19, 15, 7])
def test_high_degree_3d(q):
    """B of degree 4 (so C of degree 7: eight coefficients per equilibrium
    polynomial), mirror walls on x and z, stretched mesh: binary64 to 1e-12 and
    binary32 within the rounding bound, against the oracle."""
    p = W.random_problem3d(950 + q, 67, 6, 5, q=q, bc=(M, P, M), stretched=True, bdeg=4, ddeg=3)
    steps = 10
    say(f"case 3d degree 4 q={q}")
    o = Oracle3D(p)
    o.step(steps)
    fo = o.get_f()
    s = solver(p, "f64")
    s.set_phi(p.phi0)
    s.step(steps)
    assert np.abs(s.get_f() - fo).max() <= 1e-12 * np.abs(fo).max()
    s.close()
    s = solver(p, "f32")
    s.set_phi(p.phi0)
    s.step(steps)
    ref = o.get_phi()
    err = float(np.sqrt(((s.get_phi() - ref) ** 2).sum() / (ref ** 2).sum()))
    say(f"  binary32 rel-L2 {err:.2e} (bound {2 * steps * EPS32:.2e})")
    assert err <= 2 * steps * EPS32


def test_gaussian_hill_3d_on_gpu():
    """Anisotropic 3-D Gaussian hill, 48^3, binary64: GRE equal to the oracle's."""
    K = [[1.0e-3, 2e-4, 1e-4], [2e-4, 1.5e-3, -1e-4], [1e-4, -1e-4, 0.8e-3]]
    p = W.gaussian_hill3d_problem(48, q=19, K=K, D=1e-3, c=5.0, sigma0=0.2)
    s = solver(p, "f64")
    s.set_phi(p.phi0)
    o = Oracle3D(p, openmp=True)
    nst = int(round(0.2 / o.dt))
    s.step(nst)
    o.step(nst)
    X, Y, Z = p.mesh()
    exact = p.exact(X, Y, Z, o.time)
    gre = s.reduce(exact)["gre"]
    gre_o = o.errors(exact)[0]
    say(f"  3-D Gaussian hill 48^3: GRE gpu {gre:.4e} oracle {gre_o:.4e}")
    assert abs(gre - gre_o) <= 1e-9 * gre_o


def test_uniform_state_and_mass_3d():
    p = W.random_problem3d(3, 66, 5, 6, q=19, bc=(M, P, M), stretched=True)
    p.b = ((0.0,), (0.0,), (0.0,))
    p.d = p.d[:3] + ((0.0,), (0.0,), (0.0,))
    s = solver(p, "f64")
    s.set_phi(np.full_like(p.phi0, 0.7))
    f0 = s.get_f()
    s.step(5)
    assert np.abs(s.get_f() - f0).max() <= 1e-14
    s.set_phi(p.phi0)
    m0 = s.reduce()["mass"]
    s.step(50)
    assert abs(s.reduce()["mass"] - m0) <= 1e-12 * abs(m0)


@pytest.mark.parametrize("storage,tol", [("f32", 2e-6), ("f64", 1e-12)])
def test_full_size_one_step_sampled_3d(storage, tol):
    """The 256^3 D3Q19 benchmark mesh in its default launch: one step from a
    seeded non-equilibrium state, checked at sampled cells (faces, edges,
    corners, strip seams, tile and chunk seams, random interior cells) against
    the oracle."""
    p = W.workload3d("gaussian_hill3d_256")
    n = p.nx
    say(f"case full size 3-D {n}^3 {storage}")
    f0 = W.random_distributions3d(4242, p.q, p.nz, p.ny, p.nx)
    s = solver(p, storage)
    s.set_f(f0)
    s.step(1)
    gpu = s.get_f()
    s.close()
    o = Oracle3D(p)
    o.set_f(f0)
    del f0
    rng = np.random.default_rng(n)
    pts = set()
    edge = (0, 1, 31, 32, 61, 62, 63, 123, 124, n - 2, n - 1)
    for i in edge:
        for j in (0, 1, 2, n - 1, n // 2):
            for k in (0, 31, 32, 33, n - 1):
                pts.add((i, j, k))
    for _ in range(400):
        pts.add(tuple(int(v) for v in rng.integers(0, n, size=3)))
    cells = np.array(sorted(pts))
    ref = o.step_cells(cells)
    got = gpu[:, cells[:, 2], cells[:, 1], cells[:, 0]].T
    err = float(np.abs(got - ref).max() / np.abs(ref).max())
    say(f"  sampled max rel err {err:.2e} over {len(cells)} cells")
    assert err <= tol
