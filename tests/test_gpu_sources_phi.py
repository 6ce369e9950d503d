"""GPU path with sources that depend on phi (F(x, t, phi) = sum_j exp(gamma_j t)
phi^k_j G_j(x); Examples 4.2 and 4.5) against the CPU oracle, through the C ABI.

Binary64 must equal the oracle to 1e-12 (max-norm relative to the largest
value); binary32 meets the 2 n eps32 bound of the other binary32 tests; batches
give each instance its single-instance result bit for bit.  Examples 4.2 and
4.5 run at the paper's sizes: their GREs equal the oracle's and are compared
with the printed values (context: the readings of boundary data, face
gradients and, for Example 4.5, the unstated velocity decide the last digits).
"""
import os

import numpy as np
import pytest

import paper_1906_11036_amd as dg
from oracle import Oracle
from paper_1906_11036_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
EPS32 = float(np.finfo(np.float32).eps)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def with_terms(p, seed, nterms=5, amp=1.5):
    p.src_terms = W.random_source_terms(seed, p, nterms=nterms, amp=amp)
    return p


def run_pair(p, steps, storage="f64"):
    rings = p.rings(steps)
    s = dg.Solver(p, storage=storage)
    s.set_phi(p.phi0)
    if rings is not None:
        s.set_dirichlet(rings)
    s.step(steps)
    o = Oracle(p)
    o.step(steps, rings)
    return s, o


CASES = [(1, 1, W.PERIODIC, 9), (5, 4, W.PERIODIC, 9), (61, 7, W.PERIODIC, 9), (65, 19, W.PERIODIC, 9),
         (130, 17, W.PERIODIC, 9), (63, 33, W.MIRROR, 9), (70, 21, W.DIRICHLET, 9), (66, 12, W.PERIODIC, 5),
         (40, 41, W.MIRROR, 5)]


@pytest.mark.parametrize("nx,ny,bc,q", CASES)
def test_fp64_phi_source_matches_oracle(nx, ny, bc, q):
    p = W.random_problem(300 + nx + 3 * ny + bc, nx, ny, q=q, bcx=bc, bcy=bc,
                         stretched=(bc == W.MIRROR), bdeg=2, ddeg=2)
    if bc == W.MIRROR:
        p.bx, p.by = (0.0,), (0.0,)
    with_terms(p, 700 + nx)
    say(f"case phi source f64 {nx}x{ny} bc={bc} q={q} powers {[k for k, _, _ in p.src_terms]}")
    s, o = run_pair(p, 6)
    assert rel_max(s.get_f(), o.get_f()) <= 1e-12
    assert rel_max(s.get_phi(), o.get_phi()) <= 1e-12
    assert abs(s.diag()["mass"] - o.mass()) <= 1e-12 * abs(o.mass())


def test_fp32_phi_source_against_oracle():
    p = with_terms(W.random_problem(401, 150, 90, bdeg=2, ddeg=2), 402)
    steps = 100
    s, o = run_pair(p, steps, storage="f32")
    ref = o.get_phi()
    l2 = float(np.sqrt(((s.get_phi() - ref) ** 2).sum() / (ref ** 2).sum()))
    say(f"  f32 with phi-dependent source: rel-L2 {l2:.2e} (bound {2 * steps * EPS32:.2e})")
    assert l2 <= 2 * steps * EPS32


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_mixing_source_kinds_equals_single_instances(storage):
    """One launch over instances with a phi-dependent source, a phi-free source
    and none: each equals its single-instance run bit for bit, and the
    instance without a source equals its run in a batch without sources."""
    a = with_terms(W.random_problem(501, 70, 40, bdeg=2, ddeg=2), 502)
    b = W.random_problem(503, 130, 17, bdeg=1, ddeg=1)
    b.src_g, b.src_gamma = W.random_source(504, b)
    c = W.random_problem(505, 64, 64, bdeg=2, ddeg=3)
    probs = [a, b, c]
    say(f"case batch mixing source kinds {storage}")
    bt = dg.Batch(probs, storage=storage)
    bt.set_all_phi()
    bt.step(7)
    for i, p in enumerate(probs):
        s = dg.Solver(p, storage=storage)
        s.set_phi(p.phi0)
        s.step(7)
        assert np.array_equal(bt.get_phi(i), s.get_phi()), i
    plain = dg.Batch([c], storage=storage)
    plain.set_all_phi()
    plain.step(7)
    assert np.array_equal(bt.get_phi(2), plain.get_phi(0))


def test_uniform_logistic_field_on_gpu():
    """A uniform field under F = 1.5 phi - 2 phi^3 + 0.3 e^{0.7 t}: no fluxes, the
    GPU follows the implicit trapezoidal rule (solved here with scipy)."""
    import math

    from scipy.optimize import brentq
    xf = W.uniform_faces(70, 0.0, 1.0)
    p = W.Problem(name="uniform", xf=xf, yf=xf.copy(), c=2.0, cfl=0.6, alpha=3e-3,
                  bx=(0.0, 0.0, 0.3), by=(0.0, -0.2), dxx=(0.0, 1.0, 0.2), dxy=(0.0,),
                  dyy=(0.0, 0.8, 0.0, 0.1))
    one = np.ones((70, 70))
    p.src_terms = [(1, 0.0, 1.5 * one), (3, 0.0, -2.0 * one), (0, 0.7, 0.3 * one)]
    p.phi0 = np.full((70, 70), 0.4)
    s = dg.Solver(p, storage="f64")
    s.set_phi(p.phi0)
    dt = s.info()["dt"]

    def F(t, v):
        return 1.5 * v - 2.0 * v ** 3 + 0.3 * math.exp(0.7 * t)

    v, t = 0.4, 0.0
    for _ in range(30):
        s.step(1)
        rhs = v + 0.5 * dt * F(t, v)
        v = brentq(lambda w: w - 0.5 * dt * F(t + dt, w) - rhs, v - 1.0, v + 1.0, xtol=1e-16,
                   rtol=1e-15)
        t += dt
        assert np.abs(s.get_phi() - v).max() <= 1e-14 * abs(v)


def read_ex42():
    rows = []
    for line in open(os.path.join(GOLDEN, "ex42_burgers_fisher_gre.txt")):
        if line.strip() and not line.startswith("#"):
            c, ny, b, gre = line.split()
            rows.append((float(c), int(ny), float(b), float(gre)))
    return rows


def gpu_gre(p):
    s = dg.Solver(p, storage="f64")
    s.set_phi(p.phi0)
    rings = p.rings(p.steps)
    if rings is not None:
        s.set_dirichlet(rings)
    s.step(p.steps)
    X, Y = p.mesh()
    t = p.steps * s.info()["dt"]
    return s, s.error_norms(p.exact(X, Y, t))[0]


def test_burgers_fisher_300_full_length_against_oracle():
    """Example 4.2 at the paper's size (300 x 150 here, b = 0.1, c = 10, 5000
    steps to t = 0.5): binary64 GPU equals the oracle."""
    p = W.burgers_fisher_problem(300, ny=150, b=0.1, c=10.0)
    s, gre = gpu_gre(p)
    o = Oracle(p, openmp=True)
    o.step(p.steps, p.rings(p.steps))
    X, Y = p.mesh()
    gre_o = o.errors(p.exact(X, Y, o.time))[0]
    err = rel_max(s.get_phi(), o.get_phi())
    say(f"  ex 4.2 300x150 b=0.1: GPU GRE {gre:.4e}, oracle {gre_o:.4e}, phi max rel diff {err:.2e}")
    assert err <= 1e-12
    assert abs(gre - gre_o) <= 1e-9 * gre_o


@pytest.mark.parametrize("c,ny,b,paper", read_ex42())
def test_burgers_fisher_paper_table(c, ny, b, paper):
    """Table 4.2.1: the GPU GRE beside the printed one."""
    p = W.burgers_fisher_problem(300, ny=ny, b=b, c=c)
    _, gre = gpu_gre(p)
    say(f"  ex 4.2 c={c:g} 300x{ny} b={b:g}: GRE {gre:.4e}, paper {paper:.4e}, ratio {gre / paper:.2f}")
    assert 0.5 * paper <= gre <= 2.0 * paper


def test_nonlinear_source_400_against_oracle_and_paper():
    """Example 4.5 at the paper's size (400^2, t = 3, Pe = 100 and 1000, u read as
    (0.1, 0.1)): binary64 GPU equals the oracle (Pe = 1000), GREs beside the
    printed ones."""
    rows = []
    for line in open(os.path.join(GOLDEN, "ex45_nonlinear_source_gre.txt")):
        if line.strip() and not line.startswith("#"):
            pe, g = line.split()
            rows.append((float(pe), float(g)))
    for Pe, paper in rows:
        p = W.nonlinear_source_problem(400, Pe=Pe)
        s, gre = gpu_gre(p)
        say(f"  ex 4.5 Pe={Pe:g}: GRE {gre:.4e}, paper {paper:.4e}, ratio {gre / paper:.2f}")
        if Pe == 1000:
            o = Oracle(p, openmp=True)
            o.step(p.steps)
            err = rel_max(s.get_phi(), o.get_phi())
            say(f"    phi max rel diff against the oracle {err:.2e}")
            assert err <= 1e-12
        assert 0.1 * paper <= gre <= 10.0 * paper
