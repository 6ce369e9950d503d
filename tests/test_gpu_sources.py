"""GPU parity of the source-term path (F of eq. 2.1 with F_i and R_i of eq. 2.3
and Remark 3, through eqs. 2.24-2.27) against the CPU oracle, and Example 4.1
on the GPU against its closed form and the paper's printed GREs."""
import math
import os

import numpy as np
import pytest

import paper_1906_11036_amd as dg
from oracle import Oracle
from paper_1906_11036_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


def say(*a):
    print(*a, flush=True)


def with_source(p, seed):
    p.src_g, p.src_gamma = W.random_source(seed, p)
    return p


CASES = [(1, 1, W.PERIODIC, 9), (5, 4, W.PERIODIC, 9), (61, 7, W.PERIODIC, 9), (65, 19, W.PERIODIC, 9),
         (130, 17, W.PERIODIC, 9), (63, 33, W.MIRROR, 9), (70, 21, W.DIRICHLET, 9),
         (66, 12, W.PERIODIC, 5), (40, 41, W.MIRROR, 5)]


@pytest.mark.parametrize("nx,ny,bc,q", CASES)
def test_fp64_source_matches_oracle(nx, ny, bc, q):
    if bc != W.PERIODIC and (nx < 2 or ny < 2):
        pytest.skip("walls need two cells per axis")
    p = W.random_problem(300 + nx + 7 * ny, nx, ny, q=q, bcx=bc, bcy=bc,
                         stretched=(bc == W.MIRROR), bdeg=3 if q == 9 else 1)
    if q == 5:
        p.dxx, p.dxy, p.dyy = (0.0, 1.0), (0.0,), (0.0, 1.0)
    with_source(p, 11 + nx)
    steps = 6
    say(f"case source f64 {nx}x{ny} bc={bc} q={q}")
    s = dg.Solver(p, storage="f64")
    s.set_phi(p.phi0)
    rings = p.rings(steps)
    if rings is not None:
        s.set_dirichlet(rings)
    s.step(steps)
    o = Oracle(p)
    o.step(steps, rings)
    f, fo = s.get_f(), o.get_f()
    assert np.abs(f - fo).max() <= 1e-12 * np.abs(fo).max()
    phi, phio = s.get_phi(), o.get_phi()
    assert np.abs(phi - phio).max() <= 1e-12 * np.abs(phio).max()
    # mass read-out through the reduction includes dt F / 2 as well
    assert abs(s.diag()["mass"] - o.mass()) <= 1e-12 * abs(o.mass()) + 1e-14


def test_fp32_source_against_oracle():
    p = with_source(W.random_problem(77, 96, 80, bdeg=2), 5)
    steps = 120
    s = dg.Solver(p, storage="f32")
    s.set_phi(p.phi0)
    s.step(steps)
    o = Oracle(p)
    o.step(steps)
    ref = o.get_phi()
    err = float(np.sqrt(((s.get_phi() - ref) ** 2).sum() / (ref ** 2).sum()))
    say(f"  f32 with source: rel-L2 {err:.2e} (bound {2 * steps * EPS32:.2e})")
    assert err <= 2 * steps * EPS32


def mixed_source_batch():
    specs = [(64, 64, True), (300, 41, False), (62, 17, True), (125, 130, False), (7, 9, True),
             (129, 64, False)]
    out = []
    for k, (nx, ny, src) in enumerate(specs):
        p = W.random_problem(700 + k, nx, ny, bdeg=k % 3 + 1)
        if src:
            with_source(p, 900 + k)
        out.append(p)
    return out


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_with_sources_equals_single_instances(storage):
    """Instances with and without a source in one launch; each equals its
    single-instance run bit for bit, and the instances without a source equal
    a batch that has no source at all."""
    probs = mixed_source_batch()
    say(f"case source batch {storage}")
    b = dg.Batch(probs, storage=storage)
    b.set_all_phi()
    b.step(7)
    for i, p in enumerate(probs):
        s = dg.Solver(p, storage=storage)
        s.set_phi(p.phi0)
        s.step(7)
        assert np.array_equal(b.get_phi(i), s.get_phi()), i
    plain = [p for p in probs if p.src_g is None]
    nb = dg.Batch(plain, storage=storage)
    nb.set_all_phi()
    nb.step(7)
    k = 0
    for i, p in enumerate(probs):
        if p.src_g is None:
            assert np.array_equal(b.get_phi(i), nb.get_phi(k)), i
            k += 1


def test_source_refused_for_16bit_storage():
    p = with_source(W.random_problem(5, 16, 16), 3)
    with pytest.raises(dg.DugksError):
        dg.Solver(p, storage="f16neq")


def read_ex41():
    path = os.path.join(os.path.dirname(__file__), "golden", "ex41_source_wave_gre.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            pe, gre, tol = line.split()
            if tol != "-":
                rows.append((float(pe), float(gre), float(tol)))
    return rows


@pytest.mark.parametrize("Pe,paper_gre,tol", read_ex41())
def test_source_wave_on_gpu(Pe, paper_gre, tol):
    """Example 4.1 as printed (200^2, c = 1, CFL 0.5, t = 3), binary64 on the GPU:
    the GRE equals the oracle's and reproduces the paper's value."""
    p = W.source_wave_problem(200, Pe=Pe)
    s = dg.Solver(p, storage="f64")
    s.set_phi(p.phi0)
    s.step(p.steps)
    t = p.steps * s.info()["dt"]
    X, Y = p.mesh()
    gre, _ = s.error_norms(p.exact(X, Y, t))
    o = Oracle(p, openmp=True)
    o.step(p.steps)
    gre_o, _ = o.errors(p.exact(X, Y, o.time))
    say(f"  Pe={Pe:g}: GRE gpu {gre:.4e} oracle {gre_o:.4e} paper {paper_gre:.4e}")
    # The oracle forms fbar from f as eq. 2.27 writes it, f + h (f - E) / (2 lambda):
    # rounding of f - E grows by h / (2 lambda), about 2e6 at Pe = 1e9, so the two
    # GREs agree to 1e-5 (relative), not to the binary64 parity bound.
    assert abs(gre - gre_o) <= 1e-5 * gre_o
    assert abs(gre - paper_gre) <= tol * paper_gre
