"""Pins of the oracle's source-term path (F of eq. 2.1 with F_i and R_i of
eq. 2.3 and Remark 3, treated through eqs. 2.24-2.27) against what the
mathematics and the paper fix:

- with G = 0 the source route (f recovered from f~, then fbar and fbar+ by
  eq. 2.27, f~+ by eq. 2.25, f at the face from eq. 2.27) equals the direct
  route of eqs. 2.13, 2.21 and 2.22;
- on a periodic domain the fluxes cancel and the moments of eq. 2.7 give the
  exact discrete mass balance M(n+1) - M(n) = dt/2 [sum F(t_n)|V| + sum F(t_n+1)|V|];
- a uniform field under a uniform constant source grows by exactly dt F a step;
- Example 4.1's closed form (eq. 4.1.5): second-order convergence, and the GREs
  printed in the paper.
"""
import math
import os

import numpy as np
import pytest

from oracle import Oracle
from paper_1906_11036_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ex41_source_wave_gre.txt")


def read_ex41():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            pe, gre, tol = line.split()
            rows.append((float(pe), float(gre), None if tol == "-" else float(tol)))
    return rows


@pytest.mark.parametrize("bc,stretched,q", [(W.PERIODIC, False, 9), (W.MIRROR, True, 9),
                                            (W.DIRICHLET, False, 9), (W.PERIODIC, True, 5)])
def test_zero_source_equals_source_free_step(bc, stretched, q):
    p = W.random_problem(41, 13, 11, q=q, bcx=bc, bcy=bc, stretched=stretched)
    rings = None
    if bc == W.DIRICHLET:
        rings = np.stack([W.ring_points(p.xf, p.yf, bc, bc)[0] * 0 + 0.5 for _ in range(4)])
    a = Oracle(p)
    b = Oracle(p)
    b.set_source(np.zeros((p.ny, p.nx)), 0.7)
    b.set_phi(p.phi0)
    a.step(4, rings)
    b.step(4, rings)
    fa, fb = a.get_f(), b.get_f()
    assert np.abs(fa - fb).max() <= 1e-13 * np.abs(fa).max()


@pytest.mark.parametrize("stretched", [False, True])
def test_mass_balance_is_the_trapezoidal_rule(stretched):
    p = W.random_problem(7, 20, 17, stretched=stretched)
    g, gam = W.random_source(8, p)
    p.src_g, p.src_gamma = g, gam
    o = Oracle(p)
    wx, _, wy, _ = o.geometry()
    V = np.outer(wy[1:-1], wx[1:-1])
    dt = o.dt

    def total_source(t):
        return float((math.exp(gam * t) * g * V).sum())

    for _ in range(5):
        m0, t0 = o.mass(), o.time
        o.step(1)
        m1, t1 = o.mass(), o.time
        expect = 0.5 * dt * (total_source(t0) + total_source(t1))
        # exact up to the rounding of the two mass sums (a few hundred terms of size <= |M|)
        assert abs((m1 - m0) - expect) <= 1e-13 * abs(m0)


def test_uniform_field_grows_by_dt_F_each_step():
    xf = W.uniform_faces(8, 0.0, 1.0)
    o = Oracle(xf=xf, yf=xf, q=9, c=2.0, cfl=0.6, alpha=3e-3, bx=(0.0, 0.1, 0.3),
               by=(0.0, -0.2, 0.1), dxx=(0.0, 1.0, 0.2), dxy=(0.0, 0.1), dyy=(0.0, 0.8))
    o.set_source(np.full((8, 8), 0.7), 0.0)
    o.set_phi(np.full((8, 8), 0.3))
    dt = o.dt
    for n in range(1, 6):
        o.step(1)
        phi = o.get_phi()
        assert np.abs(phi - (0.3 + 0.7 * n * dt)).max() <= 1e-14


def test_source_wave_second_order():
    """Example 4.1 at Pe = 100 with c = 5 (lambda = 3 alpha / c^2 small, so the
    initial layer of f~ = E - dt S / 2 stays below the discretisation error):
    25^2 -> 50^2 -> 100^2 at CFL 0.5, t = 0.5."""
    errs = []
    for n in (25, 50, 100):
        p = W.source_wave_problem(n, Pe=100.0, t_end=0.5, c=5.0)
        o = Oracle(p, openmp=True)
        o.step(p.steps)
        X, Y = p.mesh()
        errs.append(o.errors(p.exact(X, Y, o.time))[0])
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(orders) >= 1.9, (errs, orders)


@pytest.mark.parametrize("Pe,paper_gre,tol", [r for r in read_ex41() if r[2] is not None])
def test_source_wave_paper_gre(Pe, paper_gre, tol):
    """Example 4.1 as printed: 200^2, c = 1, CFL 0.5, t = 3."""
    p = W.source_wave_problem(200, Pe=Pe)
    o = Oracle(p, openmp=True)
    o.step(p.steps)
    X, Y = p.mesh()
    gre = o.errors(p.exact(X, Y, o.time))[0]
    assert abs(o.time - 3.0) < 1e-9
    assert abs(gre - paper_gre) <= tol * paper_gre, gre
