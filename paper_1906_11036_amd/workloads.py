"""Seeded synthetic inputs for the DUGKS hot path.

This module only builds inputs: meshes, coefficient sets, initial fields,
boundary data and the closed-form solutions they are sampled from.  It holds
none of the scheme's arithmetic, so both the HIP path and the CPU oracle can
take their inputs from it.

Workloads (sizes and constants are those of the benchmark plan; where the
paper fixes nothing, the choice is stated here):

* ``gaussian_hill``   -- linear convection-diffusion, Gaussian hill of
  Sec. 4, Example 4.4 (closed form eq. 4.4.3), periodic square.
* ``burgers_wave``    -- 2-D viscous Burgers with a travelling tanh front,
  Dirichlet walls fed from the exact solution.
* ``nonlinear_diffusion`` -- phi_t = div(D0 (1 + phi^2) grad phi) on a
  two-sided tanh-stretched mesh (the map of eqs. 4.3.4/4.3.5 made symmetric),
  zero-flux mirror walls, 16-mode cosine initial field.
* ``batch``           -- many independent periodic instances with log-uniform
  sizes, random nonlinear convection and diffusion coefficients and
  Fourier-mode initial fields.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

PERIODIC, DIRICHLET, MIRROR = 0, 1, 2


# ----------------------------------------------------------------- meshes

def uniform_faces(n: int, a: float, b: float) -> np.ndarray:
    """n+1 equally spaced cell faces on [a, b]."""
    return a + (b - a) * np.arange(n + 1, dtype=np.float64) / n


def tanh_faces(n: int, k: float = 2.0) -> np.ndarray:
    """Faces of a mesh on [0, 1] clustered toward both walls.

    The one-sided map x = tanh(k eta)/tanh(k) of eqs. 4.3.4/4.3.5 applied to
    eta = 2i/n - 1 in [-1, 1] and shifted onto [0, 1]; grid points are faces.
    """
    eta = 2.0 * np.arange(n + 1, dtype=np.float64) / n - 1.0
    x = 0.5 * (1.0 + np.tanh(k * eta) / math.tanh(k))
    x[0], x[-1] = 0.0, 1.0
    return x


def centres(faces: np.ndarray) -> np.ndarray:
    return 0.5 * (faces[:-1] + faces[1:])


def ghost_centres(faces: np.ndarray, bc: int) -> np.ndarray:
    """Centres of cells -1..n including the one-cell ghost ring.

    A wall ghost mirrors the adjacent interior cell's width; a periodic ghost
    takes the width of the wrapped cell.  This is the location at which the
    caller samples Dirichlet data.
    """
    w = np.diff(faces)
    c = centres(faces)
    wl = w[-1] if bc == PERIODIC else w[0]
    wr = w[0] if bc == PERIODIC else w[-1]
    return np.concatenate([[faces[0] - 0.5 * wl], c, [faces[-1] + 0.5 * wr]])


def ring_points(xf: np.ndarray, yf: np.ndarray, bcx: int, bcy: int):
    """(x, y) of the 2(nx+ny)+4 ghost centres in ring order.

    Order: bottom row j=-1 (i=-1..nx), top row j=ny (i=-1..nx), left column
    i=-1 (j=0..ny-1), right column i=nx (j=0..ny-1).
    """
    gx, gy = ghost_centres(xf, bcx), ghost_centres(yf, bcy)
    nx, ny = len(xf) - 1, len(yf) - 1
    xs = np.concatenate([gx, gx, np.full(ny, gx[0]), np.full(ny, gx[-1])])
    ys = np.concatenate([np.full(nx + 2, gy[0]), np.full(nx + 2, gy[-1]),
                         gy[1:-1], gy[1:-1]])
    return xs, ys


# ---------------------------------------------------------- closed forms

def gaussian_hill(x, y, t, u, K, sigma0, period=None):
    """Gaussian hill of eq. 4.4.3 with phi0 = 2 pi sigma0^2 (peak 1 at t = 0).

    sigma(t) = sigma0^2 I + 2 K t.  On a periodic box of side ``period`` the
    infinite-domain solution is summed over the 3x3 nearest images after
    wrapping x - u t back into the box.
    """
    s = np.array([[sigma0 ** 2 + 2 * K[0][0] * t, 2 * K[0][1] * t],
                  [2 * K[1][0] * t, sigma0 ** 2 + 2 * K[1][1] * t]])
    det = s[0, 0] * s[1, 1] - s[0, 1] * s[1, 0]
    inv = np.array([[s[1, 1], -s[0, 1]], [-s[1, 0], s[0, 0]]]) / det
    phi0 = 2 * math.pi * sigma0 ** 2
    x0 = np.asarray(x, dtype=np.float64) - u[0] * t
    y0 = np.asarray(y, dtype=np.float64) - u[1] * t
    shifts = [0.0]
    if period is not None:
        x0 = (x0 + 0.5 * period) % period - 0.5 * period
        y0 = (y0 + 0.5 * period) % period - 0.5 * period
        shifts = [-period, 0.0, period]
    out = np.zeros(np.broadcast(x0, y0).shape)
    for sx in shifts:
        for sy in shifts:
            dx, dy = x0 + sx, y0 + sy
            q = inv[0, 0] * dx * dx + 2 * inv[0, 1] * dx * dy + inv[1, 1] * dy * dy
            out += np.exp(-0.5 * q)
    return phi0 / (2 * math.pi * math.sqrt(abs(det))) * out


def burgers_front(x, y, t, nu, s0=0.5):
    """Travelling front of phi_t + d_x(phi^2/2) + d_y(phi^2/2) = nu lap(phi).

    phi = 1/2 - 1/2 tanh((x + y - t - s0) / (4 nu)); substituting
    g(xi), xi = x + y - t - s0, gives -g' + 2 g g' = 2 nu g'', which this g
    satisfies with zero integration constant.
    """
    return 0.5 - 0.5 * np.tanh((np.asarray(x) + np.asarray(y) - t - s0) / (4.0 * nu))


def cosine_decay(x, y, t, alpha, mean=1.0, amp=0.5, period=1.0, neumann=False):
    """Pure diffusion (B = 0, D = phi I) of one cosine mode.

    Periodic: phi = mean + amp cos(2 pi x / L) cos(2 pi y / L) exp(-8 pi^2 alpha t / L^2).
    Neumann on [0, L]^2: cos(pi x / L) cos(pi y / L) exp(-2 pi^2 alpha t / L^2).
    """
    kk = (math.pi if neumann else 2 * math.pi) / period
    return mean + amp * np.cos(kk * np.asarray(x)) * np.cos(kk * np.asarray(y)) * \
        math.exp(-2 * kk * kk * alpha * t)


# ------------------------------------------------------------- problems

@dataclasses.dataclass
class Problem:
    """One NCDE instance: mesh, lattice, constants, coefficients, initial field."""
    name: str
    xf: np.ndarray
    yf: np.ndarray
    q: int = 9
    c: float = 1.0
    cfl: float = 0.5
    alpha: float = 1e-3
    bcx: int = PERIODIC
    bcy: int = PERIODIC
    bx: tuple = (0.0,)
    by: tuple = (0.0,)
    dxx: tuple = (0.0, 1.0)
    dxy: tuple = (0.0, 0.0)
    dyy: tuple = (0.0, 1.0)
    phi0: Optional[np.ndarray] = None        # [ny][nx], point values at centres
    steps: int = 1
    exact: Optional[Callable] = None         # (x, y, t) -> phi, or None
    seed: Optional[int] = None
    src_g: Optional[np.ndarray] = None       # source F = exp(src_gamma t) src_g, [ny][nx]
    src_gamma: float = 0.0
    # source terms F(x, t, phi) = sum of exp(gamma t) phi^k G(x) over (k, gamma, G [ny][nx])
    src_terms: Optional[list] = None

    @property
    def nx(self) -> int:
        return len(self.xf) - 1

    @property
    def ny(self) -> int:
        return len(self.yf) - 1

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def mesh(self):
        """Cell-centre coordinates as [ny][nx] arrays."""
        return np.meshgrid(centres(self.xf), centres(self.yf))

    def dt(self) -> float:
        """Time step for the workload's own bookkeeping (end time, ring times).

        Mirrors the scheme's rule dt = cfl * min width / c so that the caller
        can sample boundary data at t_n; the solver computes its own dt.
        """
        return self.cfl * min(np.diff(self.xf).min(), np.diff(self.yf).min()) / self.c

    def rings(self, nsteps: int, start_step: int = 0) -> Optional[np.ndarray]:
        """Dirichlet data at ghost centres for steps start..start+nsteps-1."""
        if DIRICHLET not in (self.bcx, self.bcy):
            return None
        xs, ys = ring_points(self.xf, self.yf, self.bcx, self.bcy)
        dt = self.dt()
        return np.stack([self.exact(xs, ys, (start_step + n) * dt)
                         for n in range(nsteps)]).astype(np.float64)


def _poly_pad(p, n=5):
    p = list(p) + [0.0] * (n - len(p))
    return tuple(float(v) for v in p[:n])


def gaussian_hill_problem(n=128, u=(0.1, 0.1), D=1e-3, sigma0=0.05, steps=500, cfl=0.5,
                          c=1.0, K=None, q=9, name="gaussian_hill", half=1.0) -> Problem:
    """Linear CDE on [-half, half]^2 (default [-1, 1]^2), periodic: B = u phi,
    D = (K / alpha) phi."""
    K = K if K is not None else [[D, 0.0], [0.0, D]]
    alpha = D
    xf = uniform_faces(n, -half, half)
    p = Problem(name=name, xf=xf, yf=xf.copy(), q=q, c=c, cfl=cfl, alpha=alpha,
                bx=(0.0, u[0]), by=(0.0, u[1]),
                dxx=(0.0, K[0][0] / alpha), dxy=(0.0, K[0][1] / alpha),
                dyy=(0.0, K[1][1] / alpha), steps=steps)
    p.exact = lambda x, y, t: gaussian_hill(x, y, t, u, K, sigma0, period=2.0 * half)
    X, Y = p.mesh()
    p.phi0 = p.exact(X, Y, 0.0)
    return p


def gaussian_hill_4096_crop(n=1024, steps=1000, **kw) -> Problem:
    """The 4096^2 Gaussian-hill workload on an n^2 window around the hill:
    [-n/4096, n/4096]^2 (periodic) with the same cell width, dt, lambda,
    coefficients, initial hill and step count.  Over its 1000 steps the hill
    moves by u t = (0.012, 0.005) and its variance grows by 2 alpha t =
    4.9e-5 against sigma0^2 = 2.5e-3, so at n = 1024 it stays 5 sigma0 inside
    the window and every cell sees the arithmetic of the full-size run."""
    return gaussian_hill_problem(n, u=(0.05, 0.02), D=1e-4, steps=steps, half=n / 4096.0,
                                 name=f"gaussian_hill_4096_crop{n}", **kw)


def burgers_problem(n=512, nu=0.01, c=4.0, cfl=0.5, steps=2000, s0=0.5,
                    name="burgers_wave") -> Problem:
    """phi_t + div((1,1) phi^2/2) = nu lap(phi) on [0,1]^2, Dirichlet from the front."""
    xf = uniform_faces(n, 0.0, 1.0)
    p = Problem(name=name, xf=xf, yf=xf.copy(), c=c, cfl=cfl, alpha=nu,
                bcx=DIRICHLET, bcy=DIRICHLET, bx=(0.0, 0.0, 0.5), by=(0.0, 0.0, 0.5),
                steps=steps)
    p.exact = lambda x, y, t: burgers_front(x, y, t, nu, s0)
    X, Y = p.mesh()
    p.phi0 = p.exact(X, Y, 0.0)
    return p


def cosine_field(X, Y, seed, modes=4, total=0.5, wavenumber=math.pi, phases=False):
    """Sum of modes x modes products of cosines with seeded amplitudes.

    a_mn ~ U(-1, 1), rescaled so that sum |a_mn| = total; with ``phases`` each
    factor gets a seeded phase (periodic fields), otherwise the field is
    Neumann-compatible on [0, 1]^2.  X and Y are meshgrid arrays of a tensor
    mesh; each product is separable, so the field is built from 1-D factors.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=(modes, modes))
    a *= total / np.abs(a).sum()
    th = rng.uniform(0, 2 * math.pi, size=(modes, modes)) if phases else np.zeros((modes, modes))
    ps = rng.uniform(0, 2 * math.pi, size=(modes, modes)) if phases else np.zeros((modes, modes))
    x, y = np.asarray(X)[0, :], np.asarray(Y)[:, 0]
    out = np.zeros((len(y), len(x)))
    for m in range(modes):
        cx, sx = np.cos(wavenumber * m * x), np.sin(wavenumber * m * x)
        for k in range(modes):
            fx = cx * math.cos(th[m, k]) - sx * math.sin(th[m, k])
            fy = np.cos(wavenumber * k * y) * math.cos(ps[m, k]) - \
                np.sin(wavenumber * k * y) * math.sin(ps[m, k])
            out += a[m, k] * np.outer(fy, fx)
    return out


def nonlinear_diffusion_problem(n=1024, D0=0.01, k=2.0, c=1.0, cfl=0.5, steps=1000, seed=3,
                                name="nonlinear_diffusion") -> Problem:
    """phi_t = div(D0 (1 + phi^2) grad phi): B = 0, D = (phi + phi^3/3) I, mirror walls."""
    xf = tanh_faces(n, k)
    p = Problem(name=name, xf=xf, yf=xf.copy(), c=c, cfl=cfl, alpha=D0, bcx=MIRROR,
                bcy=MIRROR, dxx=(0.0, 1.0, 0.0, 1.0 / 3.0), dyy=(0.0, 1.0, 0.0, 1.0 / 3.0),
                dxy=(0.0,), steps=steps, seed=seed)
    X, Y = p.mesh()
    p.phi0 = cosine_field(X, Y, seed)
    return p


def neumann_companion_problem(n=64, alpha=0.01, k=2.0, c=1.0, cfl=0.5, steps=100,
                              name="neumann_cosine") -> Problem:
    """Pure diffusion of one Neumann cosine mode on the stretched mesh, mirror walls."""
    xf = tanh_faces(n, k)
    p = Problem(name=name, xf=xf, yf=xf.copy(), c=c, cfl=cfl, alpha=alpha, bcx=MIRROR,
                bcy=MIRROR, steps=steps)
    p.exact = lambda x, y, t: cosine_decay(x, y, t, alpha, 1.0, 0.5, 1.0, neumann=True)
    X, Y = p.mesh()
    p.phi0 = p.exact(X, Y, 0.0)
    return p


def batch_problems(count=256, seed=5, nmin=64, nmax=1024, c=2.0, cfl=0.5, steps=500,
                   max_cells=None) -> List[Problem]:
    """Independent periodic instances on [0, 1]^2.

    N = round(exp U(ln nmin, ln nmax)); B = a (1, 1) phi^2 / 2 with a ~ U(0, 1);
    D = phi I with alpha ~ logU(1e-4, 1e-2); phi0 = seeded 16-mode Fourier field
    with random phases, sum |a_mn| = 0.5.  Instance k draws its field from seed
    seed*1000 + k.
    """
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=count))).astype(int)
    avals = rng.uniform(0.0, 1.0, size=count)
    alphas = np.exp(rng.uniform(math.log(1e-4), math.log(1e-2), size=count))
    out = []
    for k in range(count):
        n = int(ns[k])
        if max_cells is not None:
            n = min(n, int(math.isqrt(max_cells)))
        xf = uniform_faces(n, 0.0, 1.0)
        p = Problem(name=f"batch{k}", xf=xf, yf=xf.copy(), c=c, cfl=cfl,
                    alpha=float(alphas[k]), bx=(0.0, 0.0, 0.5 * avals[k]),
                    by=(0.0, 0.0, 0.5 * avals[k]), steps=steps, seed=seed * 1000 + k)
        X, Y = p.mesh()
        p.phi0 = cosine_field(X, Y, seed * 1000 + k, wavenumber=2 * math.pi, phases=True)
        out.append(p)
    return out


def random_problem(seed: int, nx: int, ny: int, q: int = 9, bcx: int = PERIODIC,
                   bcy: int = PERIODIC, stretched: bool = False, bdeg: int = 2,
                   ddeg: int = 1) -> Problem:
    """A small random instance for property tests: random polynomial B and D.

    D's coefficients keep the diffusion tensor positive definite for |phi| <= 1;
    the initial field is a smooth random cosine field of amplitude <= 0.5.
    The Dirichlet data (if any) is a smooth field that moves with time.
    """
    rng = np.random.default_rng(seed)
    xf = tanh_faces(nx, 1.5) if stretched else uniform_faces(nx, 0.0, 1.0)
    yf = tanh_faces(ny, 1.5) if stretched else uniform_faces(ny, 0.0, 1.0)
    bx = [0.0] + list(rng.uniform(-0.3, 0.3, size=bdeg))
    by = [0.0] + list(rng.uniform(-0.3, 0.3, size=bdeg))
    if q == 5:
        dxx, dxy, dyy = (0.0, 1.0), (0.0,), (0.0, 1.0)
    else:
        d1 = rng.uniform(0.5, 1.5, size=2)
        dxx = [0.0, d1[0]] + list(rng.uniform(0.0, 0.2, size=max(ddeg - 1, 0)))
        dyy = [0.0, d1[1]] + list(rng.uniform(0.0, 0.2, size=max(ddeg - 1, 0)))
        dxy = [0.0, rng.uniform(-0.3, 0.3)]
    p = Problem(name=f"random{seed}", xf=xf, yf=yf, q=q, c=float(rng.uniform(1.0, 3.0)),
                cfl=float(rng.uniform(0.3, 0.8)), alpha=float(np.exp(rng.uniform(-7, -3))),
                bcx=bcx, bcy=bcy, bx=tuple(bx), by=tuple(by), dxx=tuple(dxx), dxy=tuple(dxy),
                dyy=tuple(dyy), steps=3, seed=seed)
    X, Y = p.mesh()
    wn = 2 * math.pi if bcx == PERIODIC and bcy == PERIODIC else math.pi
    p.phi0 = 0.5 + cosine_field(X, Y, seed + 17, modes=3, total=0.4, wavenumber=wn,
                                phases=(bcx == PERIODIC and bcy == PERIODIC))
    amp = float(rng.uniform(0.1, 0.3))
    p.exact = lambda x, y, t: 0.5 + amp * np.sin(2.0 * np.asarray(x) + 3.0 * np.asarray(y)
                                                 + 5.0 * t)
    return p


def source_wave_problem(n=200, Pe=100.0, u=(0.1, 0.1), L=2.0, c=1.0, cfl=0.5, t_end=3.0,
                        q=9, rate=None, name="source_wave") -> Problem:
    """Example 4.1: phi_t + div(u phi) = alpha lap(phi) + F on [0, 2]^2, periodic,
    alpha = L u_x / Pe, F = exp(g t) [sin(pi(x+y)) + pi(u_x+u_y) cos(pi(x+y))] with
    g = 1 - 2 pi^2 alpha (eq. 4.1.3), phi_0 = sin(pi(x+y)) (eq. 4.1.4), exact
    solution exp(g t) sin(pi(x+y)) (eq. 4.1.5); B = u phi, D = phi I.

    rate: another growth rate g of the same exact form; the source is then
    exp(g t) [(g + 2 pi^2 alpha) sin(pi(x+y)) + pi(u_x+u_y) cos(pi(x+y))]."""
    alpha = L * u[0] / Pe
    gam = 1.0 - 2.0 * math.pi ** 2 * alpha if rate is None else float(rate)
    xf = uniform_faces(n, 0.0, L)
    p = Problem(name=name, xf=xf, yf=xf.copy(), q=q, c=c, cfl=cfl, alpha=alpha,
                bx=(0.0, u[0]), by=(0.0, u[1]), dxx=(0.0, 1.0), dxy=(0.0, 0.0),
                dyy=(0.0, 1.0))
    p.exact = lambda x, y, t: math.exp(gam * t) * np.sin(math.pi * (np.asarray(x) + np.asarray(y)))
    X, Y = p.mesh()
    p.phi0 = p.exact(X, Y, 0.0)
    p.src_g = ((gam + 2.0 * math.pi ** 2 * alpha) * np.sin(math.pi * (X + Y))
               + math.pi * (u[0] + u[1]) * np.cos(math.pi * (X + Y)))
    p.src_gamma = gam
    p.steps = int(round(t_end / p.dt()))
    return p


def burgers_fisher(x, y, t, a, b, k, delta):
    """Travelling wave of the 2-D Burgers-Fisher equation (eq. 4.2.2):
    phi = [1/2 + 1/2 tanh(A (x + y - m t))]^(1/delta) with A = -a delta / (4 b (delta + 1))
    and m = (a^2 + 2 b k (delta + 1)^2) / (a (delta + 1)); it solves eq. 4.2.1,
    phi_t + a phi^delta phi_x = b lap(phi) + k phi (1 - phi^delta)."""
    A = -a * delta / (4.0 * b * (delta + 1.0))
    m = (a * a + 2.0 * b * k * (delta + 1.0) ** 2) / (a * (delta + 1.0))
    w = 0.5 + 0.5 * np.tanh(A * (np.asarray(x) + np.asarray(y) - m * t))
    return w ** (1.0 / delta)


def burgers_fisher_problem(n=300, ny=None, b=0.05, a=6.0, k=1.0, delta=2, c=10.0, cfl=0.1,
                           t_end=0.5, lo=-1.0, hi=2.0, name="burgers_fisher") -> Problem:
    """Example 4.2 on [lo, hi]^2 (the paper: [-1, 2]^2, 300 x 300 or 300 x 150,
    a = 6, k = 1, delta = 2, c = 10, CFL 0.1): B = (a phi^(delta+1) / (delta+1), 0),
    D = phi I, alpha = b, F = k phi - k phi^(delta+1) (two terms of powers 1 and
    delta + 1), Dirichlet walls from the closed form eq. 4.2.2, which also gives
    the initial field.  delta is 1 or 2 (powers of phi up to 3)."""
    ny = n if ny is None else ny
    if delta not in (1, 2):
        raise ValueError("delta must be 1 or 2")
    xf, yf = uniform_faces(n, lo, hi), uniform_faces(ny, lo, hi)
    bx = [0.0] * (delta + 2)
    bx[delta + 1] = a / (delta + 1.0)
    p = Problem(name=name, xf=xf, yf=yf, c=c, cfl=cfl, alpha=b, bcx=DIRICHLET, bcy=DIRICHLET,
                bx=tuple(bx), by=(0.0,), dxx=(0.0, 1.0), dxy=(0.0,), dyy=(0.0, 1.0))
    p.exact = lambda x, y, t: burgers_fisher(x, y, t, a, b, k, delta)
    X, Y = p.mesh()
    p.phi0 = p.exact(X, Y, 0.0)
    one = np.ones((ny, n))
    p.src_terms = [(1, 0.0, k * one), (delta + 1, 0.0, -k * one)]
    p.steps = int(round(t_end / p.dt()))
    return p


def nonlinear_source_terms(X, Y, A, alpha, m, nxp, nyp, u):
    """Example 4.5's source (eq. 4.5.3) as terms (k, gamma, G): with
    e = exp(-A t), C = cos(2 pi x) cos(2 pi y),
      F = e A C - 4 n_x pi^2 alpha phi^(n_x-2) [(n_x - 1) e^2 sin^2(2 pi x) cos^2(2 pi y) + e phi C]
                - 4 n_y pi^2 alpha phi^(n_y-2) [(n_y - 1) e^2 sin^2(2 pi y) cos^2(2 pi x) + e phi C]
                + 2 pi m e phi^(m-1) [u_x sin(2 pi x) cos(2 pi y) + u_y cos(2 pi x) sin(2 pi y)];
    terms with equal (k, gamma) are merged.  Needs n_x, n_y >= 2, m >= 1."""
    cx, sx = np.cos(2 * math.pi * X), np.sin(2 * math.pi * X)
    cy, sy = np.cos(2 * math.pi * Y), np.sin(2 * math.pi * Y)
    C = cx * cy
    pi2 = math.pi ** 2
    raw = [(0, -A, A * C),
           (nxp - 2, -2 * A, -4 * nxp * pi2 * alpha * (nxp - 1) * sx ** 2 * cy ** 2),
           (nxp - 1, -A, -4 * nxp * pi2 * alpha * C),
           (nyp - 2, -2 * A, -4 * nyp * pi2 * alpha * (nyp - 1) * sy ** 2 * cx ** 2),
           (nyp - 1, -A, -4 * nyp * pi2 * alpha * C),
           (m - 1, -A, 2 * math.pi * m * (u[0] * sx * cy + u[1] * cx * sy))]
    merged = {}
    for k, gam, G in raw:
        key = (int(k), float(gam))
        merged[key] = merged.get(key, 0.0) + G
    return [(k, gam, np.asarray(G, dtype=np.float64)) for (k, gam), G in merged.items()]


def nonlinear_source_problem(n=400, Pe=100.0, kappa=1.1, A=1.0, m=2, nxp=2, nyp=3, u=(0.1, 0.1),
                             c=1.0, cfl=0.5, t_end=3.0, name="nonlinear_source") -> Problem:
    """Example 4.5 on [0, 1]^2, periodic: B = phi^m u, D = diag(phi^n_x, phi^n_y),
    alpha = L u_x / Pe with L = 1, F of eq. 4.5.3, exact phi = kappa -
    exp(-A t) cos(2 pi x) cos(2 pi y) (eq. 4.5.4).  The paper states Pe but not u;
    u = (0.1, 0.1) is the velocity of its Example 4.1."""
    alpha = 1.0 * u[0] / Pe
    xf = uniform_faces(n, 0.0, 1.0)
    bx, by = [0.0] * (m + 1), [0.0] * (m + 1)
    bx[m], by[m] = u[0], u[1]
    dxx, dyy = [0.0] * (nxp + 1), [0.0] * (nyp + 1)
    dxx[nxp], dyy[nyp] = 1.0, 1.0
    p = Problem(name=name, xf=xf, yf=xf.copy(), c=c, cfl=cfl, alpha=alpha, bx=tuple(bx),
                by=tuple(by), dxx=tuple(dxx), dxy=(0.0,), dyy=tuple(dyy))
    p.exact = lambda x, y, t: kappa - math.exp(-A * t) * np.cos(2 * math.pi * np.asarray(x)) * \
        np.cos(2 * math.pi * np.asarray(y))
    X, Y = p.mesh()
    p.phi0 = p.exact(X, Y, 0.0)
    p.src_terms = nonlinear_source_terms(X, Y, A, alpha, m, nxp, nyp, u)
    p.steps = int(round(t_end / p.dt()))
    return p


def random_source_terms(seed: int, p: Problem, nterms: int = 4, amp: float = 0.5):
    """Seeded smooth source terms (k, gamma, G) with powers 0..3 for property tests."""
    rng = np.random.default_rng(seed)
    X, Y = p.mesh()
    wn = 2 * math.pi if p.bcx == PERIODIC and p.bcy == PERIODIC else math.pi
    out = []
    for j in range(nterms):
        g = amp * cosine_field(X, Y, seed + 31 * j + 7, modes=3, total=1.0, wavenumber=wn,
                               phases=(p.bcx == PERIODIC and p.bcy == PERIODIC))
        out.append((j % 4, float(rng.uniform(-1.0, 1.0)), g + float(rng.uniform(-0.2, 0.2))))
    return out


def random_source_terms3d(seed: int, p: "Problem3D", nterms: int = 4, amp: float = 0.5):
    """Seeded smooth 3-D source terms (k, gamma, G [nz][ny][nx]) with powers 0..3."""
    rng = np.random.default_rng(seed)
    X, Y, Z = p.mesh()
    out = []
    for j in range(nterms):
        kx, ky, kz = rng.integers(0, 3, size=3)
        ph = rng.uniform(0, 2 * math.pi, size=3)
        g = amp * np.cos(math.pi * kx * X + ph[0]) * np.cos(math.pi * ky * Y + ph[1]) * np.cos(math.pi * kz * Z + ph[2])
        out.append((j % 4, float(rng.uniform(-1.0, 1.0)), g + float(rng.uniform(-0.2, 0.2))))
    return out


def random_source(seed: int, p: Problem, amp: float = 0.5):
    """A smooth seeded source shape G [ny][nx] and rate gamma for property tests."""
    rng = np.random.default_rng(seed)
    X, Y = p.mesh()
    wn = 2 * math.pi if p.bcx == PERIODIC and p.bcy == PERIODIC else math.pi
    g = amp * cosine_field(X, Y, seed + 29, modes=3, total=1.0, wavenumber=wn,
                           phases=(p.bcx == PERIODIC and p.bcy == PERIODIC))
    return g + float(rng.uniform(-0.2, 0.2)), float(rng.uniform(-1.0, 1.0))


def workload(name: str, **kw):
    """The named benchmark workloads."""
    table = {
        "gaussian_hill_128": lambda: gaussian_hill_problem(128, **kw),
        "burgers_512": lambda: burgers_problem(512, **kw),
        "nonlinear_diffusion_1024": lambda: nonlinear_diffusion_problem(1024, **kw),
        "gaussian_hill_4096": lambda: gaussian_hill_problem(
            4096, u=(0.05, 0.02), D=1e-4, steps=1000, name="gaussian_hill_4096", **kw),
        "batch256": lambda: batch_problems(**kw),
        "source_wave_4096": lambda: source_wave_problem(4096, Pe=1000.0, t_end=0.05,
                                                        name="source_wave_4096", **kw),
        # the 4096^2 Gaussian hill on D2Q5 (linear equilibrium of Remark 3, D = phi I)
        "gaussian_hill_4096_d2q5": lambda: gaussian_hill_problem(
            4096, u=(0.05, 0.02), D=1e-4, steps=1000, q=5, name="gaussian_hill_4096_d2q5", **kw),
    }
    return table[name]()


def random_distributions(seed: int, q: int, ny: int, nx: int, mean: float = 0.5,
                         amp: float = 0.05) -> np.ndarray:
    """Seeded smooth distributions f~ [q][ny][nx] (any f~ is a valid step input).

    Direction k gets mean * (weight-like share) plus a smooth seeded cosine field of
    amplitude ``amp`` and a small cell-scale seeded noise (so that every
    neighbour difference is exercised).
    """
    rng = np.random.default_rng(seed)
    share = np.full(q, 1.0 / (2.0 * q))
    share[0] = 0.5
    share /= share.sum()
    y = (np.arange(ny) + 0.5) / ny
    x = (np.arange(nx) + 0.5) / nx
    X, Y = np.meshgrid(x, y)
    out = np.empty((q, ny, nx))
    for k in range(q):
        a, b, ph = rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0, 2 * math.pi, size=2)
        m, n = rng.integers(1, 4, size=2)
        out[k] = mean * share[k] + amp * share[k] * (
            a * np.cos(2 * math.pi * m * X + ph[0]) + b * np.cos(2 * math.pi * n * Y + ph[1]))
        out[k] += 1e-3 * amp * rng.standard_normal((ny, nx))
    return out


# ------------------------------------------------------------ three dimensions
@dataclasses.dataclass
class Problem3D:
    """One three-dimensional NCDE instance (D3Q15, D3Q19 or D3Q7).

    b: (B_x, B_y, B_z) coefficient tuples of B(phi) = sum_k b_k phi^k;
    d: (D_xx, D_yy, D_zz, D_xy, D_xz, D_yz) coefficient tuples of D(phi);
    bc: per axis PERIODIC, MIRROR or DIRICHLET (data from exact at the ghost centres)."""
    name: str
    xf: np.ndarray
    yf: np.ndarray
    zf: np.ndarray
    q: int = 19
    c: float = 1.0
    cfl: float = 0.5
    alpha: float = 1e-3
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    b: tuple = ((0.0,), (0.0,), (0.0,))
    d: tuple = ((0.0, 1.0), (0.0, 1.0), (0.0, 1.0), (0.0,), (0.0,), (0.0,))
    phi0: Optional[np.ndarray] = None        # [nz][ny][nx]
    steps: int = 1
    exact: Optional[Callable] = None         # (x, y, z, t) -> phi
    seed: Optional[int] = None
    src_terms: Optional[list] = None         # source F = sum exp(g t) phi^k G: (k, g, G [nz][ny][nx])

    @property
    def nx(self) -> int:
        return len(self.xf) - 1

    @property
    def ny(self) -> int:
        return len(self.yf) - 1

    @property
    def nz(self) -> int:
        return len(self.zf) - 1

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def mesh(self):
        """Cell-centre coordinates as [nz][ny][nx] arrays (X, Y, Z)."""
        Z, Y, X = np.meshgrid(centres(self.zf), centres(self.yf), centres(self.xf), indexing="ij")
        return X, Y, Z

    def dt(self) -> float:
        w = min(np.diff(self.xf).min(), np.diff(self.yf).min(), np.diff(self.zf).min())
        return self.cfl * float(w) / self.c

    def rings(self, nsteps: int, start_step: int = 0) -> Optional[np.ndarray]:
        """Dirichlet data at the ghost-shell centres for steps
        start..start+nsteps-1, [nsteps][shell length] (None without a
        Dirichlet axis)."""
        if DIRICHLET not in self.bc:
            return None
        xs, ys, zs = shell_points3d(self.xf, self.yf, self.zf, self.bc)
        dt = self.dt()
        return np.stack([self.exact(xs, ys, zs, (start_step + n) * dt)
                         for n in range(nsteps)]).astype(np.float64)


def shell_points3d(xf: np.ndarray, yf: np.ndarray, zf: np.ndarray, bc):
    """(x, y, z) of the ghost-shell centres of a 3-D mesh, in the order of one
    step's Dirichlet data: the z = -1 and z = nz planes ([ny+2][nx+2], j and i
    from -1), the y = -1 and y = ny slabs ([nz][nx+2]), then the x = -1 and
    x = nx columns ([nz][ny])."""
    gx, gy, gz = ghost_centres(xf, bc[0]), ghost_centres(yf, bc[1]), ghost_centres(zf, bc[2])
    nx, ny, nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
    parts = []
    for kk in (0, nz + 1):
        Y, X = np.meshgrid(gy, gx, indexing="ij")
        parts.append((X.ravel(), Y.ravel(), np.full(X.size, gz[kk])))
    for jj in (0, ny + 1):
        Z, X = np.meshgrid(gz[1:-1], gx, indexing="ij")
        parts.append((X.ravel(), np.full(X.size, gy[jj]), Z.ravel()))
    for ii in (0, nx + 1):
        Z, Y = np.meshgrid(gz[1:-1], gy[1:-1], indexing="ij")
        parts.append((np.full(Y.size, gx[ii]), Y.ravel(), Z.ravel()))
    return tuple(np.concatenate([p[a] for p in parts]) for a in range(3))


def gaussian_hill3d(x, y, z, t, u, K, sigma0, period=2.0, images=1):
    """Closed form of phi_t + u.grad(phi) = div(K grad(phi)) for a Gaussian of
    width sigma0 (amplitude (2 pi sigma0^2)^(3/2) normalised to peak 1 at t = 0),
    constant u and constant symmetric positive definite K, with periodic images
    on the cube [-period/2, period/2]^3."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    S = sigma0 ** 2 * np.eye(3) + 2.0 * t * np.asarray(K, dtype=np.float64)
    Si = np.linalg.inv(S)
    norm = sigma0 ** 3 / math.sqrt(np.linalg.det(S))
    out = np.zeros(np.broadcast(x, y, z).shape)
    r = range(-images, images + 1)
    for a in r:
        for b in r:
            for c in r:
                dx = x - u[0] * t - a * period
                dy = y - u[1] * t - b * period
                dz = z - u[2] * t - c * period
                qf = (Si[0, 0] * dx * dx + Si[1, 1] * dy * dy + Si[2, 2] * dz * dz
                      + 2 * (Si[0, 1] * dx * dy + Si[0, 2] * dx * dz + Si[1, 2] * dy * dz))
                out += norm * np.exp(-0.5 * qf)
    return out


def gaussian_hill3d_problem(n=64, q=19, u=(0.1, 0.05, 0.02), D=1e-3, K=None, sigma0=0.15,
                            c=1.0, cfl=0.5, steps=100, name="gaussian_hill3d",
                            images0=1) -> Problem3D:
    """Linear CDE on [-1, 1]^3, periodic: B = u phi, D = (K / alpha) phi.
    images0: periodic images summed for the initial field (0 is exact to
    rounding while sigma0 <= 0.2: the nearest image is 2 / sigma0 widths away)."""
    K = np.asarray(K if K is not None else np.eye(3) * D, dtype=np.float64)
    alpha = D
    f = uniform_faces(n, -1.0, 1.0)
    kd = K / alpha
    p = Problem3D(name=name, xf=f, yf=f.copy(), zf=f.copy(), q=q, c=c, cfl=cfl, alpha=alpha,
                  b=((0.0, u[0]), (0.0, u[1]), (0.0, u[2])),
                  d=((0.0, kd[0, 0]), (0.0, kd[1, 1]), (0.0, kd[2, 2]), (0.0, kd[0, 1]),
                     (0.0, kd[0, 2]), (0.0, kd[1, 2])), steps=steps)
    p.exact = lambda x, y, z, t: gaussian_hill3d(x, y, z, t, u, K, sigma0)
    X, Y, Z = p.mesh()
    p.phi0 = gaussian_hill3d(X, Y, Z, 0.0, u, K, sigma0, images=images0)
    return p


def workload3d(name: str, **kw) -> Problem3D:
    """The named three-dimensional benchmark workloads."""
    table = {
        # anisotropic Gaussian hill on a periodic 256^3 D3Q19 mesh (16.8 M cells)
        "gaussian_hill3d_256": lambda: gaussian_hill3d_problem(
            256, q=19, u=(0.05, 0.02, 0.01),
            K=[[1.0e-4, 2e-5, 1e-5], [2e-5, 1.5e-4, -1e-5], [1e-5, -1e-5, 0.8e-4]], D=1e-4,
            sigma0=0.15, steps=1000, name="gaussian_hill3d_256", images0=0, **kw),
        # the same mesh on D3Q15, and on D3Q7 with isotropic diffusion (D = phi I)
        "gaussian_hill3d_256_d3q15": lambda: gaussian_hill3d_problem(
            256, q=15, u=(0.05, 0.02, 0.01),
            K=[[1.0e-4, 2e-5, 1e-5], [2e-5, 1.5e-4, -1e-5], [1e-5, -1e-5, 0.8e-4]], D=1e-4,
            sigma0=0.15, steps=1000, name="gaussian_hill3d_256_d3q15", images0=0, **kw),
        "gaussian_hill3d_256_d3q7": lambda: gaussian_hill3d_problem(
            256, q=7, u=(0.05, 0.02, 0.01), D=1e-4, sigma0=0.15, steps=1000,
            name="gaussian_hill3d_256_d3q7", images0=0, **kw),
        # the D3Q19 hill with a source of two terms: 0.1 cos(pi x) cos(pi y) phi (depends on
        # phi: Newton's method in cells and faces) and 0.05 e^{0.3 t}
        "gaussian_hill3d_256_src": lambda: with_sources3d(gaussian_hill3d_problem(
            256, q=19, u=(0.05, 0.02, 0.01),
            K=[[1.0e-4, 2e-5, 1e-5], [2e-5, 1.5e-4, -1e-5], [1e-5, -1e-5, 0.8e-4]], D=1e-4,
            sigma0=0.15, steps=1000, name="gaussian_hill3d_256_src", images0=0, **kw)),
    }
    return table[name]()


def with_sources3d(p: "Problem3D") -> "Problem3D":
    """p with the source of the gaussian_hill3d_256_src workload (two terms)."""
    X, Y, Z = p.mesh()
    p.src_terms = [(1, 0.0, 0.1 * np.cos(np.pi * X) * np.cos(np.pi * Y)), (0, 0.3, np.full_like(X, 0.05))]
    return p


def random_distributions3d(seed: int, q: int, nz: int, ny: int, nx: int, mean: float = 0.5,
                           amp: float = 0.05) -> np.ndarray:
    """Seeded distributions f~ [q][nz][ny][nx]: per direction a share of ``mean``,
    a smooth seeded cosine field of amplitude ``amp`` and a small cell-scale noise."""
    rng = np.random.default_rng(seed)
    share = np.full(q, 1.0 / (2.0 * q))
    share[0] = 0.5
    share /= share.sum()
    axes = [(np.arange(n) + 0.5) / n for n in (nx, ny, nz)]
    out = np.empty((q, nz, ny, nx))
    for k in range(q):
        a = rng.uniform(-1, 1, size=3)
        ph = rng.uniform(0, 2 * math.pi, size=3)
        m = rng.integers(1, 4, size=3)
        cx, cy, cz = (a[i] * np.cos(2 * math.pi * m[i] * axes[i] + ph[i]) for i in range(3))
        out[k] = mean * share[k] + amp * share[k] * (cx[None, None, :] + cy[None, :, None] + cz[:, None, None])
        out[k] += 1e-3 * amp * rng.standard_normal((nz, ny, nx))
    return out


def random_problem3d(seed: int, nx: int, ny: int, nz: int, q: int = 19,
                     bc=(PERIODIC, PERIODIC, PERIODIC), stretched: bool = False, bdeg: int = 2,
                     ddeg: int = 1) -> Problem3D:
    """A small random 3-D instance for property tests (random polynomial B and D,
    D positive definite for |phi| <= 1, smooth random initial field)."""
    rng = np.random.default_rng(seed)
    faces = [tanh_faces(n, 1.5) if stretched else uniform_faces(n, 0.0, 1.0) for n in (nx, ny, nz)]
    b = tuple(tuple([0.0] + list(rng.uniform(-0.3, 0.3, size=bdeg))) for _ in range(3))
    if q == 7:
        d = ((0.0, 1.0), (0.0, 1.0), (0.0, 1.0), (0.0,), (0.0,), (0.0,))
    else:
        diag = [tuple([0.0, float(rng.uniform(0.6, 1.4))] + list(rng.uniform(0.0, 0.2, size=max(ddeg - 1, 0))))
                for _ in range(3)]
        off = [(0.0, float(rng.uniform(-0.2, 0.2))) for _ in range(3)]
        d = (diag[0], diag[1], diag[2], off[0], off[1], off[2])
    p = Problem3D(name=f"random3d_{seed}", xf=faces[0], yf=faces[1], zf=faces[2], q=q,
                  c=float(rng.uniform(1.0, 3.0)), cfl=float(rng.uniform(0.3, 0.7)),
                  alpha=float(np.exp(rng.uniform(-7, -3))), bc=tuple(bc), b=b, d=d, steps=3,
                  seed=seed)
    X, Y, Z = p.mesh()
    periodic = all(v == PERIODIC for v in bc)
    wn = 2 * math.pi if periodic else math.pi
    field = np.zeros_like(X)
    for m in range(4):
        a = rng.uniform(-0.1, 0.1)
        kx, ky, kz = rng.integers(0, 3, size=3)
        ph = rng.uniform(0, 2 * math.pi, size=3) if periodic else np.zeros(3)
        field += a * np.cos(wn * kx * X + ph[0]) * np.cos(wn * ky * Y + ph[1]) * np.cos(wn * kz * Z + ph[2])
    p.phi0 = 0.5 + field
    amp = float(rng.uniform(0.05, 0.2))   # Dirichlet data (any smooth field of x, y, z, t)
    p.exact = lambda x, y, z, t: 0.5 + amp * np.sin(2.0 * np.asarray(x) + 3.0 * np.asarray(y)
                                                    - 1.5 * np.asarray(z) + 5.0 * t)
    return p


# ------------------------------------------------------------- one dimension
DIRICHLET1 = 1   # one-dimensional walls: 0 periodic, 1 Dirichlet


@dataclasses.dataclass
class Problem1D:
    """One-dimensional D1Q3 problem with B(phi, x, t) = b(x, t) phi,
    b = (p0 + p1 t) x + q0 exp(q1 t + q2 t^2), and D = (r0 + r1 t) phi.

    coef: (p0, p1, q0, q1, q2, r0, r1); bc: PERIODIC or DIRICHLET1; for
    Dirichlet walls ghost(t) gives phi at the two ghost centres."""
    name: str
    xf: np.ndarray
    coef: tuple = (0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0)
    c: float = 1.0
    cfl: float = 0.5
    alpha: float = 1e-3
    bc: int = PERIODIC
    t0: float = 0.0
    phi0: Optional[np.ndarray] = None
    exact: Optional[Callable] = None          # (x, t) -> phi
    ghost: Optional[Callable] = None          # t -> (phi_left_ghost, phi_right_ghost)
    steps: int = 1
    seed: Optional[int] = None

    @property
    def nx(self) -> int:
        return len(self.xf) - 1

    @property
    def cells(self) -> int:
        return self.nx

    def centres(self) -> np.ndarray:
        return centres(self.xf)

    def ghost_centres(self):
        w0, w1 = self.xf[1] - self.xf[0], self.xf[-1] - self.xf[-2]
        return self.xf[0] - 0.5 * w0, self.xf[-1] + 0.5 * w1

    def dt(self) -> float:
        return self.cfl * float(np.diff(self.xf).min()) / self.c


def fokker_planck_exact(x, t):
    """Closed form eq. 4.6.3 of the nonlinear Fokker-Planck equation eq. 4.6.1
    (Example 4.6): a Gaussian of mean <x(t)> = exp(t + t^2/2) and variance
    2 eta(t) exp(t^2), eta = 1 - exp(-t^2)."""
    x = np.asarray(x, dtype=np.float64)
    m = math.exp(t + 0.5 * t * t)
    v = 2.0 * (1.0 - math.exp(-t * t)) * math.exp(t * t)   # 2 eta e^{t^2}
    return np.exp(-(x - m) ** 2 / (2.0 * v)) / math.sqrt(2.0 * math.pi * v)


def fokker_planck_problem(n=400, t0=0.5, c=10.0, cfl=0.5, a=-2.0, b=8.0, alpha=1.0,
                          name="fokker_planck") -> Problem1D:
    """Example 4.6 on [a, b] with n uniform cells, started from the closed form
    at t0 > 0 (eq. 4.6.3) with Dirichlet walls from the closed form:
    B = (t x + exp(t + t^2/2)) phi, alpha D = 2 t phi (alpha = 1: D = 2 t phi)."""
    f = uniform_faces(n, a, b)
    p = Problem1D(name=name, xf=f, coef=(0.0, 1.0, 1.0, 1.0, 0.5, 0.0, 2.0 / alpha), c=c, cfl=cfl,
                  alpha=alpha, bc=DIRICHLET1, t0=t0)
    p.exact = fokker_planck_exact
    gl, gr = p.ghost_centres()
    p.ghost = lambda t: (float(fokker_planck_exact(gl, t)), float(fokker_planck_exact(gr, t)))
    p.phi0 = fokker_planck_exact(p.centres(), t0)
    return p


def fokker_planck_delta_initial(p: Problem1D, x0: float = 1.0) -> np.ndarray:
    """The discrete delta of eq. 4.6.4: mass 1 at x0, held by the cell that
    contains x0, or split evenly between the two cells when x0 is a face."""
    phi = np.zeros(p.nx)
    k = int(np.searchsorted(p.xf, x0))
    w = np.diff(p.xf)
    if k < len(p.xf) and abs(p.xf[k] - x0) <= 1e-12 * max(1.0, abs(x0)) and 0 < k < p.nx:
        phi[k - 1] = 0.5 / w[k - 1]
        phi[k] = 0.5 / w[k]
    else:
        j = min(max(k - 1, 0), p.nx - 1)
        phi[j] = 1.0 / w[j]
    return phi


def random_problem1d(seed: int, n: int, bc: int = PERIODIC, stretched: bool = False) -> Problem1D:
    """A small random D1Q3 instance for property tests: random coefficients of
    b(x, t) (no x-dependence with periodic walls) and d(t), random c, CFL,
    alpha, a smooth random initial field; Dirichlet walls take a seeded smooth
    function of t."""
    rng = np.random.default_rng(seed)
    f = tanh_faces(n, 1.5) if stretched else uniform_faces(n, 0.0, 1.0)
    coef = (float(rng.uniform(-0.5, 0.5)), float(rng.uniform(-0.5, 0.5)), float(rng.uniform(-0.5, 0.5)),
            float(rng.uniform(-1, 1)), float(rng.uniform(-0.5, 0.5)), float(rng.uniform(0.5, 1.5)),
            float(rng.uniform(-0.5, 0.5)))
    if bc == PERIODIC:   # periodic walls: b must not depend on x
        coef = (0.0, 0.0) + coef[2:]
    p = Problem1D(name=f"random1d_{seed}", xf=f, coef=coef, c=float(rng.uniform(1.0, 3.0)),
                  cfl=float(rng.uniform(0.3, 0.7)), alpha=float(np.exp(rng.uniform(-6, -3))), bc=bc,
                  t0=float(rng.uniform(0.0, 0.5)), seed=seed)
    x = p.centres()
    field = 1.0 + 0.2 * np.cos(2 * math.pi * x + rng.uniform(0, 2 * math.pi))
    field += 0.05 * np.cos(6 * math.pi * x + rng.uniform(0, 2 * math.pi))
    p.phi0 = field
    if bc == DIRICHLET1:
        a0, a1, w0 = rng.uniform(0.8, 1.2), rng.uniform(0.8, 1.2), rng.uniform(0.5, 2.0)
        p.ghost = lambda t: (float(a0 + 0.1 * math.sin(w0 * t)), float(a1 + 0.1 * math.cos(w0 * t)))
    return p


def workload1d(name: str, **kw) -> Problem1D:
    """The named one-dimensional benchmark workloads."""
    table = {
        # Example 4.6 on [-2, 8] with 2^26 uniform cells, from the closed form at
        # t = 0.5; c = 50 keeps max |b| / c_s below 0.45
        "fokker_planck_64m": lambda: fokker_planck_problem(1 << 26, t0=0.5, c=50.0, cfl=0.5,
                                                           name="fokker_planck_64m", **kw),
    }
    return table[name]()
