/*
 * Plain FP64 CPU oracle for one DUGKS time step of the nonlinear
 * convection-diffusion equation (Shang, Chai, Wang, Shi, "Discrete unified gas
 * kinetic scheme for nonlinear convection-diffusion equations", arXiv
 * 1906.11036).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  It shares no code,
 * header, table or constant generator with the HIP library; neither includes
 * or links the other.
 *
 * Everything is IEEE binary64, built with -O2 -ffp-contract=off, no fast-math,
 * no intrinsics.  Sums over discrete directions run in index order 0..Q-1.
 * The step follows the one-step summary at the end of Section 2 in the paper's
 * order:
 *   phi -> f~, E  (eq. 2.3)            -> f~+, fbar+  (eqs. 2.13, 2.21)
 *   -> fbar+ at the face (eq. 2.20)    -> fbar(x_b, t+h) (eqs. 2.19, 2.26)
 *   -> phi(x_b, t+h) = sum fbar        -> f(x_b, t+h) (eq. 2.22)
 *   -> face flux J (eq. 2.9)           -> f~(t+dt) (eq. 2.24)
 *   -> phi = sum f~ (+ dt F / 2 with a source).
 *
 * Source term (eq. 2.1's F), when set: a sum of terms
 *   F(x, t, phi) = sum_j exp(gamma_j t) phi^k_j G_j(x),   k_j in 0..3,
 * with each G_j given at the cell centres (F(x, t) = exp(gamma t) G(x) is one
 * term with k = 0).  Its distributions are F_i = w_i F (eq. 2.3) and, with
 * C = int B'B'^T, R_i = w_i c_i.B'(phi) F / c_s^2 (Remark 3); they enter
 * through the shifted distributions of eqs. 2.25 and 2.27, which this file
 * applies literally: f is recovered from f~ (first line of eq. 2.25), fbar
 * and fbar+ follow from eq. 2.27, f~+ from the second line of eq. 2.25, and
 * f at the face from the first line of eq. 2.27.  Without a source the step
 * uses eqs. 2.13, 2.21 and 2.22 directly.  When F depends on phi, the
 * conserved value is implicit (the paper notes this after eq. 2.27):
 * phi = sum f~ + dt F(phi) / 2 in a cell and phi_b = sum fbar + h F_b(phi_b) / 2
 * at a face; each is solved by Newton's method from phi = sum f~ (resp.
 * sum fbar) until the update is below 1e-15 (1 + |phi|).
 *
 * Readings of points the paper leaves open (each one also listed in the
 * design notes):
 *   - 2-D face gradient: the normal derivative is the two-cell difference of
 *     eq. 2.20; the tangential derivative at the face is the mean of the two
 *     adjacent cells' central differences along the face.
 *   - Point values at cell centres stand for cell averages (eq. 2.10).
 *   - dt = cfl * (smallest cell width in x or y) / c  (Sec. 2, after eq. 2.9).
 *   - lambda = alpha / c_s^2 (Chapman-Enskog result, Sec. 3).
 *   - C = integral from 0 to phi of B'(s) B'(s)^T ds (Sec. 2 after eq. 2.3
 *     and Remark 3), integration constant zero.
 *   - D2Q9 weights 4/9, 1/9 (x4), 1/36 (x4) (the printed second group label of
 *     eq. 2.5 is a typo); D2Q5 weights 1/3, 1/6 (x4) with the linear
 *     equilibrium of Remark 3, which requires D = phi I.
 *   - Boundary ghosts, one cell wide, corners included:
 *       periodic  : wrapped cell, wrapped width;
 *       Dirichlet : non-equilibrium extrapolation,
 *                   fbar+_g = E(phi_g) + (fbar+_a - E(phi_a)), a = adjacent
 *                   interior cell (diagonal for corners), phi_g = boundary data
 *                   at the ghost centre at t_n, supplied by the caller;
 *       mirror    : specular zero-flux wall, fbar+_g,i = fbar+_a,m(i) with
 *                   m(i) the direction whose normal component is reversed;
 *       a corner where a Dirichlet axis meets a mirror axis takes the
 *       Dirichlet rule (the paper gives no corner treatment).
 *     Wall ghosts take the width of the adjacent interior cell.
 *   - With a source: the moments of eq. 2.7 (sum F_i = F, sum R_i = 0) give
 *     phi = sum f~ + dt F / 2 in a cell and phi_b = sum fbar + h F / 2 at a
 *     face (the paper's phi_b = sum fbar is the F = 0 case).  F at a face is
 *     the linear interpolation of eq. 2.20 between the two cell centres, at
 *     t_n + h; a ghost cell takes G of the cell its fbar+ comes from.  f~ is
 *     initialised as f - dt (Omega + R + F) / 2 with f = E(phi_0), i.e.
 *     E(phi_0) - dt S(phi_0, F(x, 0)) / 2.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXQ 9
#define OR_MAXDEG 4
#define OR_MAXTERMS 8       /* source terms */
#define OR_MAXPOW 3         /* highest power of phi in a source term */

enum { OR_PERIODIC = 0, OR_DIRICHLET = 1, OR_MIRROR = 2 };

typedef struct {
  int nx, ny, q;
  double c, cfl, alpha;
  int bcx, bcy;
  /* lattice */
  double cx[OR_MAXQ], cy[OR_MAXQ], w[OR_MAXQ], cs2;
  int mirx[OR_MAXQ], miry[OR_MAXQ];
  /* coefficient polynomials  B(phi) = sum_k b_k phi^k,  D(phi) = sum_k M_k phi^k */
  int bdeg, ddeg;
  double bx[OR_MAXDEG + 1], by[OR_MAXDEG + 1];
  double dxx[OR_MAXDEG + 1], dxy[OR_MAXDEG + 1], dyy[OR_MAXDEG + 1];
  /* time stepping constants */
  double lambda, dt, h;
  double a1, b1, a2, b2, a3, b3;
  /* geometry, index shifted by one so that ghost -1 sits at [0] */
  double *xf, *yf;        /* faces, nx+1 / ny+1 */
  double *wx, *wy;        /* widths of cells -1..n */
  double *xc, *yc;        /* centres of cells -1..n */
  /* source F(x, t, phi) = sum_j exp(src_gam[j] t) phi^src_pow[j] G_j(x);
     src_g holds G_j as [src_n][ny][nx]; src_n = 0: no source */
  int src_n;
  double *src_g;
  int src_pow[OR_MAXTERMS];
  double src_gam[OR_MAXTERMS];
  int src_implicit;       /* some term depends on phi */
  /* state */
  double *f;              /* f~ [q][ny][nx] */
  long step;
  double t;
  /* work arrays of one step, allocated on the first step and kept */
  double *wG, *wSY, *wSX, *wFX, *wFY, *wfn;
} Oracle;

/* ---------------------------------------------------------------- lattice */

/* D2Q9 velocities of eq. 2.5 (columns of the 2x9 matrix) and D2Q5 (the first
 * five of them, the D(2)Q(2d+1) set named in Remark 3). */
static const int LAT_CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int LAT_CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

static void set_lattice(Oracle* o) {
  int i, k;
  o->cs2 = o->c * o->c / 3.0;                   /* c_s = c / sqrt(3), eq. 2.5 */
  for (i = 0; i < o->q; ++i) {
    o->cx[i] = o->c * LAT_CX[i];
    o->cy[i] = o->c * LAT_CY[i];
    if (o->q == 9)
      o->w[i] = (i == 0) ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    else
      o->w[i] = (i == 0) ? 1.0 / 3.0 : 1.0 / 6.0;
  }
  /* mirror maps: the direction with the reversed normal component */
  for (i = 0; i < o->q; ++i) {
    o->mirx[i] = o->miry[i] = -1;
    for (k = 0; k < o->q; ++k) {
      if (LAT_CX[k] == -LAT_CX[i] && LAT_CY[k] == LAT_CY[i]) o->mirx[i] = k;
      if (LAT_CX[k] == LAT_CX[i] && LAT_CY[k] == -LAT_CY[i]) o->miry[i] = k;
    }
  }
}

/* ------------------------------------------------------------ equilibrium */

static double poly(const double* a, int deg, double x) {
  double s = 0.0, p = 1.0;
  int k;
  for (k = 0; k <= deg; ++k) { s += a[k] * p; p *= x; }
  return s;
}

/* C(phi) = int_0^phi B'(s) B'(s)^T ds, written out term by term:
 * B'(s) = sum_{k>=1} k b_k s^(k-1), so the (u,v) entry is
 * sum_{k,l>=1} k l bu_k bv_l phi^(k+l-1) / (k+l-1). */
static double c_moment(const Oracle* o, const double* bu, const double* bv, double phi) {
  double s = 0.0;
  int k, l, e, m;
  for (k = 1; k <= o->bdeg; ++k)
    for (l = 1; l <= o->bdeg; ++l) {
      double p = 1.0;
      e = k + l - 1;
      for (m = 0; m < e; ++m) p *= phi;
      s += (double)(k * l) * bu[k] * bv[l] * p / (double)e;
    }
  return s;
}

/* Equilibrium of eq. 2.3:
 * E_i = w_i [ phi + c_i.B / cs2 + (cs2 D + C - cs2 phi I):(c_i c_i - cs2 I) / (2 cs2^2) ].
 * D2Q5 uses the linear equilibrium of Remark 3: E_i = w_i (phi + c_i.B / cs2). */
static void feq(const Oracle* o, double phi, double* E) {
  int i;
  double Bx = poly(o->bx, o->bdeg, phi), By = poly(o->by, o->bdeg, phi);
  double cs2 = o->cs2;
  if (o->q == 5) {
    for (i = 0; i < o->q; ++i)
      E[i] = o->w[i] * (phi + (o->cx[i] * Bx + o->cy[i] * By) / cs2);
    return;
  }
  double Dxx = poly(o->dxx, o->ddeg, phi), Dxy = poly(o->dxy, o->ddeg, phi),
         Dyy = poly(o->dyy, o->ddeg, phi);
  double Cxx = c_moment(o, o->bx, o->bx, phi), Cxy = c_moment(o, o->bx, o->by, phi),
         Cyy = c_moment(o, o->by, o->by, phi);
  double Mxx = cs2 * Dxx + Cxx - cs2 * phi;
  double Mxy = cs2 * Dxy + Cxy;
  double Myy = cs2 * Dyy + Cyy - cs2 * phi;
  for (i = 0; i < o->q; ++i) {
    double cx = o->cx[i], cy = o->cy[i];
    double contr = Mxx * (cx * cx - cs2) + 2.0 * Mxy * cx * cy + Myy * (cy * cy - cs2);
    E[i] = o->w[i] * (phi + (cx * Bx + cy * By) / cs2 + contr / (2.0 * cs2 * cs2));
  }
}

/* ----------------------------------------------------------------- source */

/* S_i = R_i + F_i for a source value F at conserved value phi:
 * F_i = w_i F (eq. 2.3); R_i = w_i c_i.B'(phi) F / cs2 (Remark 3, C = int B'B'^T).
 * B'(phi) = sum_{k>=1} k b_k phi^(k-1). */
static void source_dist(const Oracle* o, double phi, double F, double* S) {
  double bpx = 0.0, bpy = 0.0, p = 1.0;
  int k, i;
  for (k = 1; k <= o->bdeg; ++k) {
    bpx += (double)k * o->bx[k] * p;
    bpy += (double)k * o->by[k] * p;
    p *= phi;
  }
  for (i = 0; i < o->q; ++i)
    S[i] = o->w[i] * F + o->w[i] * (o->cx[i] * bpx + o->cy[i] * bpy) * F / o->cs2;
}

/* Coefficients a_k of F as a polynomial in phi, F = sum_k a_k phi^k, at time t
 * and at a point whose G_j are a weighted mean of two cells' values:
 * G_j = (1 - r) G_j(cL) + r G_j(cR) (r = 0: the centre of cell cL). */
static void source_coefs(const Oracle* o, size_t cL, size_t cR, double r, double t, double* a) {
  size_t N = (size_t)o->nx * o->ny;
  int j, k;
  for (k = 0; k <= OR_MAXPOW; ++k) a[k] = 0.0;
  for (j = 0; j < o->src_n; ++j) {
    double gL = o->src_g[(size_t)j * N + cL], gR = o->src_g[(size_t)j * N + cR];
    a[o->src_pow[j]] += exp(o->src_gam[j] * t) * (gL + r * (gR - gL));
  }
}

static double poly3(const double* a, double phi) {
  return a[0] + phi * (a[1] + phi * (a[2] + phi * a[3]));
}

/* The conserved value phi with phi - tau F(phi) / 2 = s, F = sum_k a_k phi^k
 * (tau = dt in a cell, eq. 2.25; tau = h at a face, eq. 2.27): explicit when F
 * does not depend on phi, otherwise Newton's method from phi = s. */
static double solve_conserved(const Oracle* o, double s, double tau, const double* a) {
  double phi = s;
  int it;
  if (!o->src_implicit) return s + 0.5 * tau * a[0];
  for (it = 0; it < 60; ++it) {
    double F = poly3(a, phi);
    double dF = a[1] + phi * (2.0 * a[2] + phi * 3.0 * a[3]);
    double d = (phi - 0.5 * tau * F - s) / (1.0 - 0.5 * tau * dF);
    phi -= d;
    if (fabs(d) <= 1e-15 * (1.0 + fabs(phi))) break;
  }
  return phi;
}

/* --------------------------------------------------------------- geometry */

#define XW(o, i) ((o)->wx[(i) + 1])
#define YW(o, j) ((o)->wy[(j) + 1])
#define XC(o, i) ((o)->xc[(i) + 1])
#define YC(o, j) ((o)->yc[(j) + 1])

static void build_axis(int n, const double* f, int bc, double* w, double* c) {
  int i;
  for (i = 0; i < n; ++i) {
    w[i + 1] = f[i + 1] - f[i];
    c[i + 1] = 0.5 * (f[i] + f[i + 1]);
  }
  w[0] = (bc == OR_PERIODIC) ? w[n] : w[1];
  w[n + 1] = (bc == OR_PERIODIC) ? w[1] : w[n];
  c[0] = f[0] - 0.5 * w[0];
  c[n + 1] = f[n] + 0.5 * w[n + 1];
}

/* ------------------------------------------------------------ public API */

Oracle* or_create(int nx, int ny, const double* xf, const double* yf, int q, double c,
                  double cfl, double alpha, int bcx, int bcy) {
  Oracle* o;
  int i;
  double dmin;
  if (nx < 1 || ny < 1 || (q != 9 && q != 5) || !(c > 0) || !(cfl > 0) || !(alpha > 0))
    return NULL;
  if (bcx < 0 || bcx > 2 || bcy < 0 || bcy > 2) return NULL;
  o = (Oracle*)calloc(1, sizeof(Oracle));
  o->nx = nx; o->ny = ny; o->q = q; o->c = c; o->cfl = cfl; o->alpha = alpha;
  o->bcx = bcx; o->bcy = bcy;
  set_lattice(o);
  o->xf = (double*)malloc(sizeof(double) * (nx + 1));
  o->yf = (double*)malloc(sizeof(double) * (ny + 1));
  memcpy(o->xf, xf, sizeof(double) * (nx + 1));
  memcpy(o->yf, yf, sizeof(double) * (ny + 1));
  o->wx = (double*)malloc(sizeof(double) * (nx + 2));
  o->xc = (double*)malloc(sizeof(double) * (nx + 2));
  o->wy = (double*)malloc(sizeof(double) * (ny + 2));
  o->yc = (double*)malloc(sizeof(double) * (ny + 2));
  build_axis(nx, o->xf, bcx, o->wx, o->xc);
  build_axis(ny, o->yf, bcy, o->wy, o->yc);
  o->f = (double*)calloc((size_t)q * nx * ny, sizeof(double));
  /* B = D = 0 until set */
  /* constants (Sec. 2 and Sec. 3) */
  o->lambda = alpha / o->cs2;
  dmin = XW(o, 0);
  for (i = 0; i < nx; ++i) if (XW(o, i) < dmin) dmin = XW(o, i);
  for (i = 0; i < ny; ++i) if (YW(o, i) < dmin) dmin = YW(o, i);
  o->dt = cfl * dmin / c;
  o->h = 0.5 * o->dt;
  {
    double L = o->lambda, dt = o->dt, h = o->h;
    o->a1 = (2.0 * L - h) / (2.0 * L + dt);   /* eq. 2.21 */
    o->b1 = 3.0 * h / (2.0 * L + dt);
    o->a2 = (2.0 * L - dt) / (2.0 * L + dt);  /* eq. 2.13 */
    o->b2 = 2.0 * dt / (2.0 * L + dt);
    o->a3 = 2.0 * L / (2.0 * L + h);          /* eq. 2.22 */
    o->b3 = h / (2.0 * L + h);
  }
  return o;
}

void or_destroy(Oracle* o) {
  if (!o) return;
  free(o->xf); free(o->yf); free(o->wx); free(o->wy); free(o->xc); free(o->yc); free(o->f);
  free(o->src_g);
  free(o->wG); free(o->wSY); free(o->wSX); free(o->wFX); free(o->wFY); free(o->wfn);
  free(o);
}

int or_set_B(Oracle* o, int deg, const double* bx, const double* by) {
  int k;
  if (deg < 0 || deg > OR_MAXDEG) return -1;
  memset(o->bx, 0, sizeof(o->bx)); memset(o->by, 0, sizeof(o->by));
  for (k = 0; k <= deg; ++k) { o->bx[k] = bx[k]; o->by[k] = by[k]; }
  o->bdeg = deg;
  return 0;
}

int or_set_D(Oracle* o, int deg, const double* dxx, const double* dxy, const double* dyy) {
  int k;
  if (deg < 0 || deg > OR_MAXDEG) return -1;
  memset(o->dxx, 0, sizeof(o->dxx)); memset(o->dxy, 0, sizeof(o->dxy));
  memset(o->dyy, 0, sizeof(o->dyy));
  for (k = 0; k <= deg; ++k) { o->dxx[k] = dxx[k]; o->dxy[k] = dxy[k]; o->dyy[k] = dyy[k]; }
  o->ddeg = deg;
  return 0;
}

/* Source terms F(x, t, phi) = sum_j exp(gam[j] t) phi^pow[j] G_j(x), j < n,
 * g = G_j as [n][ny][nx] at the cell centres (copied); n == 0 or g == NULL
 * removes the source.  Returns -1 (nothing changed) for n > 8 or a power
 * outside 0..3. */
int or_set_source_terms(Oracle* o, int n, const double* g, const int* pow, const double* gam) {
  size_t N = (size_t)o->nx * o->ny;
  int j;
  if (n < 0 || n > OR_MAXTERMS) return -1;
  for (j = 0; j < n && g; ++j)
    if (pow[j] < 0 || pow[j] > OR_MAXPOW) return -1;
  free(o->src_g);
  o->src_g = NULL;
  o->src_n = 0;
  o->src_implicit = 0;
  if (n == 0 || !g) return 0;
  o->src_g = (double*)malloc(sizeof(double) * N * n);
  memcpy(o->src_g, g, sizeof(double) * N * n);
  o->src_n = n;
  for (j = 0; j < n; ++j) {
    o->src_pow[j] = pow[j];
    o->src_gam[j] = gam[j];
    if (pow[j] > 0) o->src_implicit = 1;
  }
  return 0;
}

/* Source F(x, t) = exp(gamma t) g(x) (one term independent of phi); g == NULL
 * removes it. */
void or_set_source(Oracle* o, const double* g, double gamma) {
  int zero = 0;
  or_set_source_terms(o, g ? 1 : 0, g, &zero, &gamma);
}

/* Threads of the OpenMP build: n > 0 sets them; returns the number a step
 * uses (1 in the serial build). */
int or_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* constants: lambda, dt, h, a1, b1, a2, b2, a3, b3, cs2 */
void or_constants(const Oracle* o, double* out) {
  out[0] = o->lambda; out[1] = o->dt; out[2] = o->h;
  out[3] = o->a1; out[4] = o->b1; out[5] = o->a2; out[6] = o->b2;
  out[7] = o->a3; out[8] = o->b3; out[9] = o->cs2;
}

/* geometry with ghosts: widths and centres of cells -1..n along x and y */
void or_geometry(const Oracle* o, double* wx, double* xc, double* wy, double* yc) {
  memcpy(wx, o->wx, sizeof(double) * (o->nx + 2));
  memcpy(xc, o->xc, sizeof(double) * (o->nx + 2));
  memcpy(wy, o->wy, sizeof(double) * (o->ny + 2));
  memcpy(yc, o->yc, sizeof(double) * (o->ny + 2));
}

void or_feq(const Oracle* o, double phi, double* E) { feq(o, phi, E); }

/* Initialisation of Sec. 4: f~(x, t0) = E(phi(x, t0)), point values at centres. */
void or_set_phi(Oracle* o, const double* phi) {
  int i, j, k;
  double E[OR_MAXQ], S[OR_MAXQ];
  size_t N = (size_t)o->nx * o->ny;
  for (j = 0; j < o->ny; ++j)
    for (i = 0; i < o->nx; ++i) {
      size_t c = (size_t)j * o->nx + i;
      feq(o, phi[c], E);
      for (k = 0; k < o->q; ++k) o->f[k * N + c] = E[k];
      if (o->src_n) {
        /* f = E at t = 0, Omega = 0: f~ = f - dt (R + F) / 2 (eq. 2.25) */
        double a[OR_MAXPOW + 1];
        source_coefs(o, c, c, 0.0, 0.0, a);
        source_dist(o, phi[c], poly3(a, phi[c]), S);
        for (k = 0; k < o->q; ++k) o->f[k * N + c] = E[k] - 0.5 * o->dt * S[k];
      }
    }
  o->step = 0; o->t = 0.0;
}

void or_set_f(Oracle* o, const double* f) {
  memcpy(o->f, f, sizeof(double) * o->q * o->nx * o->ny);
}
void or_get_f(const Oracle* o, double* f) {
  memcpy(f, o->f, sizeof(double) * o->q * o->nx * o->ny);
}
void or_set_clock(Oracle* o, long step, double t) { o->step = step; o->t = t; }
long or_step_index(const Oracle* o) { return o->step; }
double or_time(const Oracle* o) { return o->t; }

/* phi of cell c at the current time: sum_i f~_i (Sec. 2, after eq. 2.13); with
 * a source the root of phi = sum_i f~_i + dt F(phi) / 2 (eq. 2.25 summed with
 * the moments of eq. 2.7), and *F = F(phi) there (F may be NULL). */
static double cell_phi_F(const Oracle* o, size_t c, double* F) {
  size_t N = (size_t)o->nx * o->ny;
  double s = 0.0, a[OR_MAXPOW + 1], phi;
  int k;
  for (k = 0; k < o->q; ++k) s += o->f[k * N + c];
  if (!o->src_n) {
    if (F) *F = 0.0;
    return s;
  }
  source_coefs(o, c, c, 0.0, o->t, a);
  phi = solve_conserved(o, s, o->dt, a);
  if (F) *F = poly3(a, phi);
  return phi;
}

static double cell_phi(const Oracle* o, size_t c) { return cell_phi_F(o, c, NULL); }

void or_get_phi(const Oracle* o, double* phi) {
  size_t i, N = (size_t)o->nx * o->ny;
  for (i = 0; i < N; ++i) phi[i] = cell_phi(o, i);
}

/* ------------------------------------------------------------------- step */

static int ring_index(const Oracle* o, int i, int j) {
  if (j == -1) return i + 1;
  if (j == o->ny) return (o->nx + 2) + i + 1;
  if (i == -1) return 2 * (o->nx + 2) + j;
  return 2 * (o->nx + 2) + o->ny + j; /* i == nx */
}

static int wrap_or_clamp(int i, int n, int bc) {
  if (i >= 0 && i < n) return i;
  if (bc == OR_PERIODIC) return (i + n) % n;
  return i < 0 ? 0 : n - 1;
}

/* fbar+ at cell (i, j), i in -1..nx, j in -1..ny, from the current f~ and the
 * ghost rules.  Without a source fbar+ = a1 f~ + b1 E(phi)  (eq. 2.21); with
 * one, f from f~ (eq. 2.25), then fbar and fbar+ (eq. 2.27). */
static void fbar_plus(const Oracle* o, int i, int j, const double* ring, double* out) {
  int si = wrap_or_clamp(i, o->nx, o->bcx), sj = wrap_or_clamp(j, o->ny, o->bcy);
  size_t N = (size_t)o->nx * o->ny, c = (size_t)sj * o->nx + si;
  double ft[OR_MAXQ], E[OR_MAXQ], phi, tmp[OR_MAXQ];
  int k;
  int xwall = (i < 0 || i >= o->nx) && o->bcx != OR_PERIODIC;
  int ywall = (j < 0 || j >= o->ny) && o->bcy != OR_PERIODIC;
  double Fc;
  for (k = 0; k < o->q; ++k) ft[k] = o->f[k * N + c];
  phi = cell_phi_F(o, c, &Fc);
  feq(o, phi, E);
  if (!o->src_n) {
    for (k = 0; k < o->q; ++k) out[k] = o->a1 * ft[k] + o->b1 * E[k];
  } else {
    double S[OR_MAXQ], L = o->lambda, dt = o->dt, h = o->h;
    source_dist(o, phi, Fc, S);
    for (k = 0; k < o->q; ++k) {
      /* f~ = f - dt/2 Omega - dt/2 S with Omega = -(f - E)/lambda, solved for f */
      double f = (2.0 * L * ft[k] + dt * E[k] + L * dt * S[k]) / (2.0 * L + dt);
      /* fbar = f - h/2 Omega - h/2 S (eq. 2.27, first line) */
      double fb = f + h / (2.0 * L) * (f - E[k]) - 0.5 * h * S[k];
      /* eq. 2.27, second line */
      out[k] = (2.0 * L - h) / (2.0 * L + h) * fb + 2.0 * h / (2.0 * L + h) * E[k] +
               2.0 * L * h / (2.0 * L + h) * S[k];
    }
  }
  if (!xwall && !ywall) return;
  if ((xwall && o->bcx == OR_DIRICHLET) || (ywall && o->bcy == OR_DIRICHLET)) {
    double phig = ring[ring_index(o, i, j)], Eg[OR_MAXQ];
    feq(o, phig, Eg);
    for (k = 0; k < o->q; ++k) out[k] = Eg[k] + (out[k] - E[k]);
    return;
  }
  /* mirror walls */
  memcpy(tmp, out, sizeof(double) * (size_t)o->q);
  if (xwall) for (k = 0; k < o->q; ++k) out[k] = tmp[o->mirx[k]];
  memcpy(tmp, out, sizeof(double) * (size_t)o->q);
  if (ywall) for (k = 0; k < o->q; ++k) out[k] = tmp[o->miry[k]];
}

/* Half-step interface distribution and flux on one face.
 *   fL, fR : fbar+ at the two cells across the face (L on the low side)
 *   tL, tR : central-difference slopes of fbar+ along the face at L and R
 *   dn     : distance between the two centres, wl : face minus L centre
 *   (cn, ct) : velocity components normal / tangential to the face
 *   sL, sR : cells whose G the two sides take (ignored without a source)
 * Linear reconstruction (eq. 2.20), Taylor shift back along the
 * characteristic (eq. 2.19 in the form of eq. 2.26), interface phi (sum of
 * fbar), f = a3 fbar + b3 E(phi_b)  (eq. 2.22; with a source, the first line
 * of eq. 2.27 solved for f), flux c_n f  (eq. 2.9). */
static void face_flux(const Oracle* o, const double* cn, const double* ct, const double* fL,
                      const double* fR, const double* tL, const double* tR, double dn,
                      double wl, size_t sL, size_t sR, double* flux) {
  double fb[OR_MAXQ], E[OR_MAXQ], phib = 0.0;
  int k;
  for (k = 0; k < o->q; ++k) {
    double Gn = (fR[k] - fL[k]) / dn;
    double v = fL[k] + wl * Gn;
    double Gt = 0.5 * (tL[k] + tR[k]);
    fb[k] = v - o->h * (cn[k] * Gn + ct[k] * Gt);
  }
  for (k = 0; k < o->q; ++k) phib += fb[k];
  if (!o->src_n) {
    feq(o, phib, E);
    for (k = 0; k < o->q; ++k) flux[k] = cn[k] * (o->a3 * fb[k] + o->b3 * E[k]);
  } else {
    double S[OR_MAXQ], L = o->lambda, h = o->h, a[OR_MAXPOW + 1], Fb;
    /* F at the face at t_n + h (where fbar lives, eq. 2.27), each G_j
       interpolated linearly between the centres; phi_b = sum fbar + h F_b / 2 */
    source_coefs(o, sL, sR, wl / dn, o->t + h, a);
    phib = solve_conserved(o, phib, h, a);
    Fb = poly3(a, phib);
    feq(o, phib, E);
    source_dist(o, phib, Fb, S);
    for (k = 0; k < o->q; ++k)
      flux[k] = cn[k] * (2.0 * L * fb[k] + h * E[k] + L * h * S[k]) / (2.0 * L + h);
  }
}

/* the cell whose source G_j cell (i, j), i in -1..nx, j in -1..ny, takes: a
 * ghost takes those of the cell its fbar+ comes from */
static size_t src_g_at(const Oracle* o, int i, int j) {
  return (size_t)wrap_or_clamp(j, o->ny, o->bcy) * o->nx + wrap_or_clamp(i, o->nx, o->bcx);
}

static void slope(const Oracle* o, const double* fm, const double* fp, double dist, double* s) {
  int k;
  for (k = 0; k < o->q; ++k) s[k] = (fp[k] - fm[k]) / dist;
}

/* f~ update of eq. 2.24 on a Cartesian cell: the surface integral of eq. 2.9
 * with the midpoint rule on each of the four faces, divided by |V|. */
static void update_cell(const Oracle* o, size_t c, const double* ft_plus, const double* FW,
                        const double* FE, const double* FS, const double* FN, double dxi,
                        double dyj, double* out) {
  int k;
  (void)c;
  for (k = 0; k < o->q; ++k)
    out[k] = ft_plus[k] - o->dt * ((FE[k] - FW[k]) / dxi + (FN[k] - FS[k]) / dyj);
}

static void ftilde_plus(const Oracle* o, size_t c, double* out) {
  size_t N = (size_t)o->nx * o->ny;
  double ft[OR_MAXQ], E[OR_MAXQ], S[OR_MAXQ], phi;
  int k;
  double Fc;
  for (k = 0; k < o->q; ++k) ft[k] = o->f[k * N + c];
  phi = cell_phi_F(o, c, &Fc);
  feq(o, phi, E);
  if (!o->src_n) {
    for (k = 0; k < o->q; ++k) out[k] = o->a2 * ft[k] + o->b2 * E[k]; /* eq. 2.13 */
    return;
  }
  source_dist(o, phi, Fc, S);
  for (k = 0; k < o->q; ++k) /* eq. 2.25, second line */
    out[k] = o->a2 * ft[k] + o->b2 * E[k] + 2.0 * o->lambda * o->dt / (2.0 * o->lambda + o->dt) * S[k];
}

/* One full step over the grid, phase by phase.  ring: boundary phi at ghost
 * centres for this step (2(nx+ny)+4 values) or NULL without Dirichlet walls. */
static void step_once(Oracle* o, const double* ring) {
  const int nx = o->nx, ny = o->ny, q = o->q;
  const size_t N = (size_t)nx * ny;
  const int NX2 = nx + 2;
  double *G, *SY, *SX, *FX, *FY, *fn;
  double zx[OR_MAXQ], zy[OR_MAXQ];
  int i, j, k;
#define GP(i, j) (G + ((size_t)((j) + 1) * NX2 + ((i) + 1)) * q)
  if (!o->wG) {
    o->wG = (double*)malloc(sizeof(double) * (size_t)(nx + 2) * (ny + 2) * q);
    o->wSY = (double*)malloc(sizeof(double) * (size_t)(nx + 2) * ny * q);
    o->wSX = (double*)malloc(sizeof(double) * (size_t)nx * (ny + 2) * q);
    o->wFX = (double*)malloc(sizeof(double) * (size_t)(nx + 1) * ny * q);
    o->wFY = (double*)malloc(sizeof(double) * (size_t)nx * (ny + 1) * q);
    o->wfn = (double*)malloc(sizeof(double) * N * q);
  }
  G = o->wG; SY = o->wSY; SX = o->wSX; FX = o->wFX; FY = o->wFY; fn = o->wfn;
  for (k = 0; k < q; ++k) { zx[k] = o->cx[k]; zy[k] = o->cy[k]; }
  /* 1-2: fbar+ on interior and ghost cells */
#pragma omp parallel for private(i)
  for (j = -1; j <= ny; ++j)
    for (i = -1; i <= nx; ++i) fbar_plus(o, i, j, ring, GP(i, j));
  /* 3: slopes along y at cells -1..nx, rows 0..ny-1; along x at 0..nx-1, rows -1..ny */
#pragma omp parallel for private(i)
  for (j = 0; j < ny; ++j)
    for (i = -1; i <= nx; ++i)
      slope(o, GP(i, j - 1), GP(i, j + 1), YC(o, j + 1) - YC(o, j - 1),
            SY + ((size_t)j * NX2 + (i + 1)) * q);
#pragma omp parallel for private(i)
  for (j = -1; j <= ny; ++j)
    for (i = 0; i < nx; ++i)
      slope(o, GP(i - 1, j), GP(i + 1, j), XC(o, i + 1) - XC(o, i - 1),
            SX + ((size_t)(j + 1) * nx + i) * q);
  /* 4: x-faces between (i-1, j) and (i, j), i = 0..nx */
#pragma omp parallel for private(i)
  for (j = 0; j < ny; ++j)
    for (i = 0; i <= nx; ++i)
      face_flux(o, zx, zy, GP(i - 1, j), GP(i, j), SY + ((size_t)j * NX2 + i) * q,
                SY + ((size_t)j * NX2 + i + 1) * q, XC(o, i) - XC(o, i - 1),
                o->xf[i] - XC(o, i - 1), src_g_at(o, i - 1, j), src_g_at(o, i, j),
                FX + ((size_t)j * (nx + 1) + i) * q);
  /* y-faces between (i, j-1) and (i, j), j = 0..ny */
#pragma omp parallel for private(i)
  for (j = 0; j <= ny; ++j)
    for (i = 0; i < nx; ++i)
      face_flux(o, zy, zx, GP(i, j - 1), GP(i, j), SX + ((size_t)j * nx + i) * q,
                SX + ((size_t)(j + 1) * nx + i) * q, YC(o, j) - YC(o, j - 1),
                o->yf[j] - YC(o, j - 1), src_g_at(o, i, j - 1), src_g_at(o, i, j),
                FY + ((size_t)j * nx + i) * q);
  /* 5: update */
#pragma omp parallel for private(i)
  for (j = 0; j < ny; ++j)
    for (i = 0; i < nx; ++i) {
      size_t c = (size_t)j * nx + i;
      double ftp[OR_MAXQ], out[OR_MAXQ];
      ftilde_plus(o, c, ftp);
      update_cell(o, c, ftp, FX + ((size_t)j * (nx + 1) + i) * q,
                  FX + ((size_t)j * (nx + 1) + i + 1) * q, FY + ((size_t)j * nx + i) * q,
                  FY + ((size_t)(j + 1) * nx + i) * q, XW(o, i), YW(o, j), out);
      for (k = 0; k < q; ++k) fn[k * N + c] = out[k];
    }
#undef GP
  /* the new state becomes f~; the old array is the next step's output */
  o->wfn = o->f;
  o->f = fn;
  o->step += 1;
  o->t += o->dt;
}

/* Advance nsteps.  rings: nsteps consecutive rings (step n uses rings + n*len)
 * or NULL when no wall is Dirichlet. */
void or_step(Oracle* o, int nsteps, const double* rings) {
  int n;
  int len = 2 * (o->nx + o->ny) + 4;
  for (n = 0; n < nsteps; ++n) step_once(o, rings ? rings + (size_t)n * len : NULL);
}

/* One step evaluated only at the listed cells (pairs i, j), without changing
 * the state.  Every value is computed with the same helpers and argument order
 * as the full step, from the 3x3 neighbourhood of each cell. out: [ncells][q]. */
void or_step_cells(const Oracle* o, int ncells, const int* cells, const double* ring,
                   double* out) {
  const int q = o->q;
  double zx[OR_MAXQ], zy[OR_MAXQ];
  int n, a, b, k;
  for (k = 0; k < q; ++k) { zx[k] = o->cx[k]; zy[k] = o->cy[k]; }
  for (n = 0; n < ncells; ++n) {
    int i = cells[2 * n], j = cells[2 * n + 1];
    double g[3][3][OR_MAXQ], sy[3][OR_MAXQ], sx[3][OR_MAXQ];
    double fw[OR_MAXQ], fe[OR_MAXQ], fs[OR_MAXQ], fnn[OR_MAXQ], ftp[OR_MAXQ];
    for (b = -1; b <= 1; ++b)
      for (a = -1; a <= 1; ++a) fbar_plus(o, i + a, j + b, ring, g[b + 1][a + 1]);
    /* y-slopes at (i-1, j), (i, j), (i+1, j); x-slopes at (i, j-1), (i, j), (i, j+1) */
    for (a = -1; a <= 1; ++a)
      slope(o, g[0][a + 1], g[2][a + 1], YC(o, j + 1) - YC(o, j - 1), sy[a + 1]);
    for (b = -1; b <= 1; ++b)
      slope(o, g[b + 1][0], g[b + 1][2], XC(o, i + 1) - XC(o, i - 1), sx[b + 1]);
    face_flux(o, zx, zy, g[1][0], g[1][1], sy[0], sy[1], XC(o, i) - XC(o, i - 1),
              o->xf[i] - XC(o, i - 1), src_g_at(o, i - 1, j), src_g_at(o, i, j), fw);
    face_flux(o, zx, zy, g[1][1], g[1][2], sy[1], sy[2], XC(o, i + 1) - XC(o, i),
              o->xf[i + 1] - XC(o, i), src_g_at(o, i, j), src_g_at(o, i + 1, j), fe);
    face_flux(o, zy, zx, g[0][1], g[1][1], sx[0], sx[1], YC(o, j) - YC(o, j - 1),
              o->yf[j] - YC(o, j - 1), src_g_at(o, i, j - 1), src_g_at(o, i, j), fs);
    face_flux(o, zy, zx, g[1][1], g[2][1], sx[1], sx[2], YC(o, j + 1) - YC(o, j),
              o->yf[j + 1] - YC(o, j), src_g_at(o, i, j), src_g_at(o, i, j + 1), fnn);
    ftilde_plus(o, (size_t)j * o->nx + i, ftp);
    update_cell(o, 0, ftp, fw, fe, fs, fnn, XW(o, i), YW(o, j), out + (size_t)n * q);
  }
}

/* fbar+ on every cell including the ghost ring: out [(ny+2)][(nx+2)][q] */
void or_fbar_plus_all(const Oracle* o, const double* ring, double* out) {
  int i, j;
  for (j = -1; j <= o->ny; ++j)
    for (i = -1; i <= o->nx; ++i)
      fbar_plus(o, i, j, ring, out + ((size_t)(j + 1) * (o->nx + 2) + (i + 1)) * o->q);
}

/* GRE of eq. 4.1 (unweighted sums over cells) and the relative L2 error
 * weighted by cell area, against a reference field phi_a [ny][nx]. */
void or_errors(const Oracle* o, const double* phi_a, double* gre, double* rel_l2) {
  int i, j;
  double num = 0.0, den = 0.0, e2 = 0.0, r2 = 0.0;
  for (j = 0; j < o->ny; ++j)
    for (i = 0; i < o->nx; ++i) {
      size_t c = (size_t)j * o->nx + i;
      double phi = cell_phi(o, c), v = XW(o, i) * YW(o, j);
      num += fabs(phi_a[c] - phi);
      den += fabs(phi_a[c]);
      e2 += v * (phi - phi_a[c]) * (phi - phi_a[c]);
      r2 += v * phi_a[c] * phi_a[c];
    }
  *gre = num / den;
  *rel_l2 = sqrt(e2 / r2);
}

/* mass = sum_j phi_j |V_j| */
double or_mass(const Oracle* o) {
  int i, j;
  double m = 0.0;
  for (j = 0; j < o->ny; ++j)
    for (i = 0; i < o->nx; ++i) {
      size_t c = (size_t)j * o->nx + i;
      m += cell_phi(o, c) * XW(o, i) * YW(o, j);
    }
  return m;
}
