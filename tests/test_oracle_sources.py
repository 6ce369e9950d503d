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


# ------------------------------------------- face time of the source term

def _read_lattice_d2q9():
    path = os.path.join(os.path.dirname(__file__), "golden", "lattices.txt")
    rows = []
    for line in open(path):
        t = line.split()
        if t and t[0] == "D2Q9":
            rows.append((int(t[2]), int(t[3]), int(t[4]) / int(t[5])))
    a = np.array(rows, dtype=float)
    return a[:, 0], a[:, 1], a[:, 2]


def source_step_symbol(kx, ky, n, L, c, alpha, cfl, u, Dm, gamma, t_n, face_time):
    """One step on a periodic uniform mesh for one Fourier mode: returns
    (G, s) with  f~^(n+1) = G f~^n + s g  for f~ = F e^{ik.x} and a source
    F(x, t) = exp(gamma t) g e^{ik.x}, built from the definitions:
      f~ = f - dt/2 (Omega + S),  fbar = f - h/2 (Omega + S)   (eqs. 2.25, 2.27)
      fbar+ = (2L-h)/(2L+h) fbar + 2h/(2L+h) E + 2Lh/(2L+h) S (eq. 2.27)
      f~+ = (2L-dt)/(2L+dt) f~ + 2dt/(2L+dt) E + 2Ldt/(2L+dt) S (eq. 2.25)
    with S_i = w_i (1 + c_i.u / c_s^2) F (eq. 2.3, Remark 3), phi = sum f~ +
    dt F / 2 in the cell at t_n, and at a face, where fbar lives at t_n + h,
    phi_b = sum fbar + h F_b / 2 with F_b the mean of the two cells' G at
    ``face_time``.  The equilibrium E = e phi solves the moment system of
    eq. 2.7 for B = u phi, D = Dm phi, C = u u^T phi."""
    cxl, cyl, w = _read_lattice_d2q9()
    cx, cy = c * cxl, c * cyl
    cs2 = c * c / 3.0
    basis = np.stack([np.ones(9), cx, cy, cx * cx, cx * cy, cy * cy], axis=1)
    A = np.array([[np.sum(w * r * basis[:, j]) for j in range(6)] for r in basis.T])
    M2 = cs2 * np.asarray(Dm) + np.outer(u, u)
    e = w * (basis @ np.linalg.solve(A, [1.0, u[0], u[1], M2[0][0], M2[0][1], M2[1][1]]))
    rho = w * (1.0 + (cx * u[0] + cy * u[1]) / cs2)
    dx = L / n
    lam = alpha / cs2
    dt = cfl * dx / c
    h = dt / 2
    one = np.ones(9)
    I = np.eye(9)
    tx, ty = kx * dx, ky * dx

    # affine maps on the vector (F, g) of length 10
    def cell(Fg):
        F, g = Fg[:9], Fg[9]
        Fc = math.exp(gamma * t_n) * g
        phi = one @ F + dt * Fc / 2
        S = rho * Fc
        f = (2 * lam * F + dt * e * phi + lam * dt * S) / (2 * lam + dt)
        fbar = f + h / (2 * lam) * (f - e * phi) - h / 2 * S
        fbp = (2 * lam - h) / (2 * lam + h) * fbar + 2 * h / (2 * lam + h) * e * phi + \
            2 * lam * h / (2 * lam + h) * S
        ftp = (2 * lam - dt) / (2 * lam + dt) * F + 2 * dt / (2 * lam + dt) * e * phi + \
            2 * lam * dt / (2 * lam + dt) * S
        return fbp, ftp

    def face(fbp, g, t_shift, Cn, Ct, tt, tn):
        # reconstruction of eq. 2.20 and the shift of eq. 2.19 on the low-side face
        Rec = (1 + np.exp(-1j * tn)) / 2 * (I - h * Ct * 1j * math.sin(tt) / dx) - \
            h * Cn * (1 - np.exp(-1j * tn)) / dx
        fb = Rec @ fbp
        Fb = math.exp(gamma * t_shift) * g * (1 + np.exp(-1j * tn)) / 2
        phib = one @ fb + h * Fb / 2
        Sb = rho * Fb
        return (2 * lam * fb + h * e * phib + lam * h * Sb) / (2 * lam + h)

    def step(Fg):
        fbp, ftp = cell(Fg)
        Cx, Cy = np.diag(cx), np.diag(cy)
        fx = face(fbp, Fg[9], face_time, Cx, Cy, ty, tx)
        fy = face(fbp, Fg[9], face_time, Cy, Cx, tx, ty)
        return ftp - dt * ((np.exp(1j * tx) - 1) / dx * cx * fx + (np.exp(1j * ty) - 1) / dx * cy * fy)

    cols = [step(np.eye(10)[j].astype(complex)) for j in range(10)]
    M = np.stack(cols, axis=1)
    return M[:, :9], M[:, 9], dt


def test_face_time_of_the_source_by_fourier_symbol():
    """The oracle's step with a source F = exp(gamma t) G(x) on one Fourier
    mode equals the symbol built from the definitions with the face source at
    t_n + h (where fbar(x_b, t_n + h) lives, eq. 2.27), to rounding; the same
    symbol with the face source at t_n differs by far more than that, so this
    pins the face time."""
    n, L = 16, 2.0
    c, alpha, cfl, u, Dm, gamma = 1.0, 2e-2, 0.7, (0.3, -0.2), [[1.0, 0.2], [0.2, 0.6]], 4.0
    xf = W.uniform_faces(n, -1.0, 1.0)
    X, Y = np.meshgrid(W.centres(xf), W.centres(xf))
    rng = np.random.default_rng(31)
    for (mx, my) in ((1, 0), (0, 1), (2, 3), (5, -7), (8, 8)):
        kx, ky = 2 * math.pi * mx / L, 2 * math.pi * my / L
        phase = np.exp(1j * (kx * X + ky * Y))
        Fh = rng.normal(size=9) + 1j * rng.normal(size=9)
        gh = complex(rng.normal(), rng.normal())
        o = Oracle(xf=xf, yf=xf, c=c, cfl=cfl, alpha=alpha, bx=(0.0, u[0]), by=(0.0, u[1]),
                   dxx=(0.0, Dm[0][0]), dxy=(0.0, Dm[0][1]), dyy=(0.0, Dm[1][1]))
        o.set_source(np.real(gh * phase), gamma)
        o.set_f(np.real(Fh[:, None, None] * phase[None]))
        t_n = 0.37
        o.set_clock(5, t_n)
        o.step(1)
        got = o.get_f()
        scale = max(np.abs(Fh).max(), abs(gh) * math.exp(gamma * t_n))
        errs = {}
        for name, ft in (("t_n + h", None), ("t_n", t_n)):
            G, s, dt = source_step_symbol(kx, ky, n, L, c, alpha, cfl, u, Dm, gamma, t_n,
                                          face_time=(t_n + 0.5 * o.dt) if ft is None else ft)
            assert math.isclose(dt, o.dt, rel_tol=1e-14)
            expect = np.real((G @ Fh + s * gh)[:, None, None] * phase[None])
            errs[name] = np.abs(got - expect).max() / scale
        assert errs["t_n + h"] <= 1e-13, (mx, my, errs)
        if (mx, my) != (n // 2, n // 2):   # at (8, 8) the face mean of G is zero on both faces
            assert errs["t_n"] >= 1e3 * max(errs["t_n + h"], 1e-16), (mx, my, errs)
