/*
 * Plain FP64 CPU oracle for one DUGKS time step on three-dimensional lattices
 * (D3Q15 of eq. 2.28, D3Q19 of eq. 2.6, D3Q7 of Remark 3) of the nonlinear
 * convection-diffusion equation (Shang, Chai, Wang, Shi, arXiv 1906.11036).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  It shares no code,
 * header, table or constant generator with the HIP library (nor with the
 * two-dimensional oracle); neither includes or links the other.
 *
 * IEEE binary64, built with -O2 -ffp-contract=off, no fast-math, no
 * intrinsics.  Sums over discrete directions run in index order 0..Q-1.
 * The step is the one-step summary at the end of Section 2, in the paper's
 * order, on a Cartesian mesh of nx x ny x nz cells:
 *   phi -> E (eq. 2.3) -> fbar+ (eq. 2.21), f~+ (eq. 2.13)
 *   -> fbar+ at each face (eq. 2.20) -> fbar(x_b, t+h) (eqs. 2.19, 2.26)
 *   -> phi_b = sum fbar -> f(x_b, t+h) (eq. 2.22) -> flux (eq. 2.9)
 *   -> f~(t+dt) (eq. 2.24) -> phi = sum f~.
 *
 * Readings (each also listed in the design notes):
 *   - the face gradient: the normal derivative is the two-cell difference of
 *     eq. 2.20; each tangential derivative is the mean of the two adjacent
 *     cells' central differences along that axis (the 2-D reading, per axis);
 *   - point values at cell centres stand for cell averages (eq. 2.10);
 *   - dt = cfl * (smallest cell width along any axis) / c, lambda = alpha/c_s^2;
 *   - C = int_0^phi B'(s) B'(s)^T ds (Remark 3), integration constant 0;
 *   - D3Q7: weights 0 (rest) and 1/6 (x6) with c_s^2 = c^2/3 and the linear
 *     equilibrium E_i = w_i (phi + c_i.B / c_s^2) of Remark 3 (needs D = phi I);
 *   - walls: periodic (wrapped ghost cell and width), zero-flux mirror
 *     (fbar+ of the adjacent interior cell with the wall-normal velocity
 *     component reversed, width of the adjacent cell) or Dirichlet by
 *     non-equilibrium extrapolation, per axis; a ghost shell one cell wide,
 *     edges and corners included.  A ghost with a Dirichlet wall on any of
 *     its out-of-range axes takes fbar+_g = E(phi_g) + (fbar+_a - E(phi_a)),
 *     a the nearest interior cell (clamped per axis) and phi_g the caller's
 *     boundary value at the ghost centre at t_n (the two-dimensional rule,
 *     per axis); otherwise each mirror axis reflects in turn.
 *   - sources F(x, t, phi) = sum_j exp(gamma_j t) phi^k_j G_j(x) (k_j <= 3,
 *     at most 8 terms), the two-dimensional treatment per axis: F_i = w_i F
 *     and R_i = w_i c_i.B'(phi) F / c_s^2 (eq. 2.3, Remark 3), f~ and fbar
 *     shifted by the sources (eqs. 2.25, 2.27); the conserved value solves
 *     phi = sum f~ + dt F(phi) / 2 in a cell at t_n and phi_b = sum fbar +
 *     h F(phi_b) / 2 at a face at t_n + h, each G_j interpolated linearly
 *     between the two centres; Newton's method from the explicit sum when F
 *     depends on phi (update <= 1e-15 (1 + |phi|), at most 60 updates);
 *     f~ = E(phi0) - dt S(phi0) / 2 at t = 0; a ghost takes the G_j of the
 *     cell its fbar+ comes from.
 *   - boundary values of one step: the shell in the order z = -1 plane and
 *     z = nz plane (each [ny+2][nx+2], j and i from -1), then the y = -1 and
 *     y = ny slabs (each [nz][nx+2]), then the x = -1 and x = nx columns (each
 *     [nz][ny]).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O3_MAXQ 19
#define O3_MAXDEG 4
#define O3_MAXTERMS 8
#define O3_MAXPOW 3

enum { O3_PERIODIC = 0, O3_DIRICHLET = 1, O3_MIRROR = 2 };

/* D3Q15 (eq. 2.28) and D3Q19 (eq. 2.6): the columns of the printed matrices */
static const int Q15[15][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                               {0, 0, 1},  {0, 0, -1},  {1, 1, 1},  {1, 1, -1}, {1, -1, 1},
                               {-1, 1, 1}, {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}};
static const int Q19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                               {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                               {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1},
                               {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

typedef struct {
  int n[3];               /* cells along x, y, z */
  int q;
  double c, cfl, alpha;
  int bc[3];
  int e[O3_MAXQ][3];      /* integer directions */
  double cv[O3_MAXQ][3];  /* velocities c e_i */
  double w[O3_MAXQ], cs2;
  int mir[3][O3_MAXQ];    /* direction with component a reversed */
  int bdeg, ddeg;
  double b[3][O3_MAXDEG + 1];  /* B_a(phi) = sum_k b[a][k] phi^k */
  double d[3][3][O3_MAXDEG + 1];
  double lambda, dt, h, a1, b1, a2, b2, a3, b3;
  double* fc[3];          /* faces, n+1 per axis */
  double* wd[3];          /* widths of cells -1..n (index +1) */
  double* cc[3];          /* centres of cells -1..n (index +1) */
  double* f;              /* f~ [q][nz][ny][nx] */
  long step;
  double t;
  int src_n, src_implicit;       /* source terms (0: none); some term depends on phi */
  double* src_g;                 /* G_j [src_n][nz][ny][nx] */
  int src_pow[O3_MAXTERMS];
  double src_gam[O3_MAXTERMS];
} Oracle3;

/* ------------------------------------------------------------ lattice */

static void set_lattice(Oracle3* o) {
  int i, a, k;
  o->cs2 = o->c * o->c / 3.0; /* c_s = c / sqrt(3), eqs. 2.28 and 2.6 */
  for (i = 0; i < o->q; ++i) {
    for (a = 0; a < 3; ++a) o->e[i][a] = (o->q == 19) ? Q19[i][a] : Q15[i][a];
    for (a = 0; a < 3; ++a) o->cv[i][a] = o->c * o->e[i][a];
    if (o->q == 15)
      o->w[i] = i == 0 ? 2.0 / 9.0 : (i <= 6 ? 1.0 / 9.0 : 1.0 / 72.0);
    else if (o->q == 19)
      o->w[i] = i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    else
      o->w[i] = i == 0 ? 0.0 : 1.0 / 6.0;
  }
  for (a = 0; a < 3; ++a)
    for (i = 0; i < o->q; ++i) {
      o->mir[a][i] = -1;
      for (k = 0; k < o->q; ++k) {
        int same = 1, b;
        for (b = 0; b < 3; ++b) {
          int want = (b == a) ? -o->e[i][b] : o->e[i][b];
          if (o->e[k][b] != want) same = 0;
        }
        if (same) o->mir[a][i] = k;
      }
    }
}

/* ------------------------------------------------------------ equilibrium */

static double poly(const double* p, int deg, double x) {
  double s = 0.0, m = 1.0;
  int k;
  for (k = 0; k <= deg; ++k) { s += p[k] * m; m *= x; }
  return s;
}

/* C_ab(phi) = int_0^phi B'_a B'_b ds = sum_{k,l>=1} k l b_ak b_bl phi^(k+l-1)/(k+l-1) */
static double c_moment(const Oracle3* o, int a, int b, double phi) {
  double s = 0.0;
  int k, l, m;
  for (k = 1; k <= o->bdeg; ++k)
    for (l = 1; l <= o->bdeg; ++l) {
      int e = k + l - 1;
      double p = 1.0;
      for (m = 0; m < e; ++m) p *= phi;
      s += (double)(k * l) * o->b[a][k] * o->b[b][l] * p / (double)e;
    }
  return s;
}

/* eq. 2.3: E_i = w_i [phi + c_i.B/cs2 + M:(c_i c_i - cs2 I)/(2 cs2^2)],
 * M = cs2 D + C - cs2 phi I; D3Q7 uses the linear equilibrium of Remark 3. */
static void feq(const Oracle3* o, double phi, double* E) {
  double B[3], M[3][3];
  int i, a, b;
  const double cs2 = o->cs2;
  for (a = 0; a < 3; ++a) B[a] = poly(o->b[a], o->bdeg, phi);
  if (o->q == 7) {
    for (i = 0; i < o->q; ++i) {
      double cb = 0.0;
      for (a = 0; a < 3; ++a) cb += o->cv[i][a] * B[a];
      E[i] = o->w[i] * (phi + cb / cs2);
    }
    return;
  }
  for (a = 0; a < 3; ++a)
    for (b = 0; b < 3; ++b)
      M[a][b] = cs2 * poly(o->d[a][b], o->ddeg, phi) + c_moment(o, a, b, phi) - (a == b ? cs2 * phi : 0.0);
  for (i = 0; i < o->q; ++i) {
    double cb = 0.0, contr = 0.0;
    for (a = 0; a < 3; ++a) cb += o->cv[i][a] * B[a];
    for (a = 0; a < 3; ++a)
      for (b = 0; b < 3; ++b)
        contr += M[a][b] * (o->cv[i][a] * o->cv[i][b] - (a == b ? cs2 : 0.0));
    E[i] = o->w[i] * (phi + cb / cs2 + contr / (2.0 * cs2 * cs2));
  }
}

/* ------------------------------------------------------------ geometry */

#define WD(o, a, i) ((o)->wd[a][(i) + 1])
#define CC(o, a, i) ((o)->cc[a][(i) + 1])

static void build_axis(int n, const double* f, int bc, double* w, double* c) {
  int i;
  for (i = 0; i < n; ++i) {
    w[i + 1] = f[i + 1] - f[i];
    c[i + 1] = 0.5 * (f[i] + f[i + 1]);
  }
  w[0] = bc == O3_PERIODIC ? w[n] : w[1];
  w[n + 1] = bc == O3_PERIODIC ? w[1] : w[n];
  c[0] = f[0] - 0.5 * w[0];
  c[n + 1] = f[n] + 0.5 * w[n + 1];
}

/* ------------------------------------------------------------ public API */

Oracle3* or3_create(int nx, int ny, int nz, const double* xf, const double* yf, const double* zf,
                    int q, double c, double cfl, double alpha, int bcx, int bcy, int bcz) {
  Oracle3* o;
  int a, i;
  const double* fs[3] = {xf, yf, zf};
  int bcs[3] = {bcx, bcy, bcz};
  double dmin;
  if (nx < 1 || ny < 1 || nz < 1 || (q != 15 && q != 19 && q != 7) || !(c > 0) || !(cfl > 0) ||
      !(alpha > 0))
    return NULL;
  for (a = 0; a < 3; ++a)
    if (bcs[a] != O3_PERIODIC && bcs[a] != O3_MIRROR && bcs[a] != O3_DIRICHLET) return NULL;
  o = (Oracle3*)calloc(1, sizeof(Oracle3));
  o->n[0] = nx; o->n[1] = ny; o->n[2] = nz;
  o->q = q; o->c = c; o->cfl = cfl; o->alpha = alpha;
  set_lattice(o);
  dmin = 1e300;
  for (a = 0; a < 3; ++a) {
    int n = o->n[a];
    o->bc[a] = bcs[a];
    o->fc[a] = (double*)malloc(sizeof(double) * (n + 1));
    memcpy(o->fc[a], fs[a], sizeof(double) * (n + 1));
    o->wd[a] = (double*)malloc(sizeof(double) * (n + 2));
    o->cc[a] = (double*)malloc(sizeof(double) * (n + 2));
    build_axis(n, o->fc[a], bcs[a], o->wd[a], o->cc[a]);
    for (i = 0; i < n; ++i) if (WD(o, a, i) < dmin) dmin = WD(o, a, i);
  }
  o->f = (double*)calloc((size_t)q * nx * ny * nz, sizeof(double));
  o->lambda = alpha / o->cs2;
  o->dt = cfl * dmin / c;
  o->h = 0.5 * o->dt;
  {
    double L = o->lambda, dt = o->dt, h = o->h;
    o->a1 = (2.0 * L - h) / (2.0 * L + dt); /* eq. 2.21 */
    o->b1 = 3.0 * h / (2.0 * L + dt);
    o->a2 = (2.0 * L - dt) / (2.0 * L + dt); /* eq. 2.13 */
    o->b2 = 2.0 * dt / (2.0 * L + dt);
    o->a3 = 2.0 * L / (2.0 * L + h); /* eq. 2.22 */
    o->b3 = h / (2.0 * L + h);
  }
  return o;
}

/* Threads of the OpenMP build: n > 0 sets them; returns the number a step
 * uses (1 in the serial build). */
int or3_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

void or3_destroy(Oracle3* o) {
  int a;
  if (!o) return;
  for (a = 0; a < 3; ++a) { free(o->fc[a]); free(o->wd[a]); free(o->cc[a]); }
  free(o->f);
  free(o->src_g);
  free(o);
}

/* B_a(phi) = sum_k b[a*(deg+1) + k] phi^k, a = x, y, z */
int or3_set_B(Oracle3* o, int deg, const double* b) {
  int a, k;
  if (deg < 0 || deg > O3_MAXDEG) return -1;
  memset(o->b, 0, sizeof(o->b));
  for (a = 0; a < 3; ++a)
    for (k = 0; k <= deg; ++k) o->b[a][k] = b[a * (deg + 1) + k];
  o->bdeg = deg;
  return 0;
}

/* D(phi): six components xx, yy, zz, xy, xz, yz, each deg+1 coefficients */
int or3_set_D(Oracle3* o, int deg, const double* d) {
  static const int AB[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  int m, k;
  if (deg < 0 || deg > O3_MAXDEG) return -1;
  memset(o->d, 0, sizeof(o->d));
  for (m = 0; m < 6; ++m)
    for (k = 0; k <= deg; ++k) {
      o->d[AB[m][0]][AB[m][1]][k] = d[m * (deg + 1) + k];
      o->d[AB[m][1]][AB[m][0]][k] = d[m * (deg + 1) + k];
    }
  o->ddeg = deg;
  return 0;
}

/* lambda, dt, h, a1, b1, a2, b2, a3, b3, cs2 */
void or3_constants(const Oracle3* o, double* out) {
  out[0] = o->lambda; out[1] = o->dt; out[2] = o->h;
  out[3] = o->a1; out[4] = o->b1; out[5] = o->a2; out[6] = o->b2;
  out[7] = o->a3; out[8] = o->b3; out[9] = o->cs2;
}

void or3_feq(const Oracle3* o, double phi, double* E) { feq(o, phi, E); }

static size_t ncells(const Oracle3* o) { return (size_t)o->n[0] * o->n[1] * o->n[2]; }
static size_t cidx(const Oracle3* o, int i, int j, int k) {
  return ((size_t)k * o->n[1] + j) * o->n[0] + i;
}

/* ------------------------------------------------------------ sources */

/* n terms: G_j (g, [n][nz][ny][nx], copied), powers k_j in 0..3 and growth
 * rates gamma_j; n = 0 removes the source.  Returns -1 on a bad argument. */
int or3_set_source_terms(Oracle3* o, int n, const double* g, const int* pw, const double* gam) {
  const size_t N = ncells(o);
  int j;
  if (n < 0 || n > O3_MAXTERMS || (n > 0 && (!g || !pw || !gam))) return -1;
  for (j = 0; j < n; ++j)
    if (pw[j] < 0 || pw[j] > O3_MAXPOW) return -1;
  free(o->src_g);
  o->src_g = NULL;
  o->src_n = n;
  o->src_implicit = 0;
  if (n == 0) return 0;
  o->src_g = (double*)malloc(sizeof(double) * N * n);
  memcpy(o->src_g, g, sizeof(double) * N * n);
  for (j = 0; j < n; ++j) {
    o->src_pow[j] = pw[j];
    o->src_gam[j] = gam[j];
    if (pw[j] > 0) o->src_implicit = 1;
  }
  return 0;
}

/* S_i = F_i + R_i for a source value F at phi: F_i = w_i F (eq. 2.3),
 * R_i = w_i c_i.B'(phi) F / c_s^2 (Remark 3, C = int B'B'^T) */
static void source_dist(const Oracle3* o, double phi, double F, double* S) {
  double bp[3] = {0.0, 0.0, 0.0}, p = 1.0;
  int a, k, i;
  for (k = 1; k <= o->bdeg; ++k) {
    for (a = 0; a < 3; ++a) bp[a] += (double)k * o->b[a][k] * p;
    p *= phi;
  }
  for (i = 0; i < o->q; ++i) {
    double cb = 0.0;
    for (a = 0; a < 3; ++a) cb += o->cv[i][a] * bp[a];
    S[i] = o->w[i] * F + o->w[i] * cb * F / o->cs2;
  }
}

/* coefficients a_k of F = sum_k a_k phi^k at time t, G_j = (1 - r) G_j(cL) +
 * r G_j(cR) (r = 0: the centre of cell cL) */
static void source_coefs(const Oracle3* o, size_t cL, size_t cR, double r, double t, double* a) {
  const size_t N = ncells(o);
  int j, k;
  for (k = 0; k <= O3_MAXPOW; ++k) a[k] = 0.0;
  for (j = 0; j < o->src_n; ++j) {
    double gL = o->src_g[(size_t)j * N + cL], gR = o->src_g[(size_t)j * N + cR];
    a[o->src_pow[j]] += exp(o->src_gam[j] * t) * (gL + r * (gR - gL));
  }
}

static double poly3(const double* a, double phi) {
  return a[0] + phi * (a[1] + phi * (a[2] + phi * a[3]));
}

/* phi with phi - tau F(phi) / 2 = s (tau = dt in a cell, eq. 2.25; tau = h at
 * a face, eq. 2.27): explicit when F does not depend on phi, else Newton's
 * method from phi = s */
static double solve_conserved(const Oracle3* o, double s, double tau, const double* a) {
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

/* phi of interior cell c at the current time (Sec. 2: sum f~; with a source
 * the root of phi = sum f~ + dt F(phi) / 2) and F there (F may be NULL) */
static double cell_phi_F(const Oracle3* o, size_t c, double* F) {
  const size_t N = ncells(o);
  double s = 0.0, a[O3_MAXPOW + 1], phi;
  int m;
  for (m = 0; m < o->q; ++m) s += o->f[m * N + c];
  if (!o->src_n) {
    if (F) *F = 0.0;
    return s;
  }
  source_coefs(o, c, c, 0.0, o->t, a);
  phi = solve_conserved(o, s, o->dt, a);
  if (F) *F = poly3(a, phi);
  return phi;
}

/* Initialisation (Sec. 4): f~ = E(phi) with point values at the centres; with
 * a source f = E at t = 0 (Omega = 0), so f~ = E - dt S / 2 (eq. 2.25). */
void or3_set_phi(Oracle3* o, const double* phi) {
  size_t c, N = ncells(o);
  int k;
  double E[O3_MAXQ], S[O3_MAXQ], a[O3_MAXPOW + 1];
  for (c = 0; c < N; ++c) {
    feq(o, phi[c], E);
    for (k = 0; k < o->q; ++k) o->f[k * N + c] = E[k];
    if (o->src_n) {
      source_coefs(o, c, c, 0.0, 0.0, a);
      source_dist(o, phi[c], poly3(a, phi[c]), S);
      for (k = 0; k < o->q; ++k) o->f[k * N + c] = E[k] - 0.5 * o->dt * S[k];
    }
  }
  o->step = 0; o->t = 0.0;
}

void or3_set_f(Oracle3* o, const double* f) { memcpy(o->f, f, sizeof(double) * o->q * ncells(o)); }
void or3_get_f(const Oracle3* o, double* f) { memcpy(f, o->f, sizeof(double) * o->q * ncells(o)); }
double or3_time(const Oracle3* o) { return o->t; }

/* phi = sum_i f~_i (Sec. 2, after eq. 2.13; with a source, cell_phi_F) */
void or3_get_phi(const Oracle3* o, double* phi) {
  size_t c, N = ncells(o);
  for (c = 0; c < N; ++c) phi[c] = cell_phi_F(o, c, NULL);
}

/* ------------------------------------------------------------ step */

static int wrap_or_clamp(int i, int n, int bc) {
  if (i >= 0 && i < n) return i;
  if (bc == O3_PERIODIC) return (i + n) % n;
  return i < 0 ? 0 : n - 1;
}

/* position of ghost cell (i, j, k) in one step's boundary values */
static size_t shell_index(const Oracle3* o, int i, int j, int k) {
  const size_t nx = o->n[0], ny = o->n[1], nz = o->n[2];
  const size_t zplane = (nx + 2) * (ny + 2), yslab = (nx + 2) * nz, xcol = ny * nz;
  if (k == -1) return (size_t)(j + 1) * (nx + 2) + (size_t)(i + 1);
  if (k == (int)nz) return zplane + (size_t)(j + 1) * (nx + 2) + (size_t)(i + 1);
  if (j == -1) return 2 * zplane + (size_t)k * (nx + 2) + (size_t)(i + 1);
  if (j == (int)ny) return 2 * zplane + yslab + (size_t)k * (nx + 2) + (size_t)(i + 1);
  if (i == -1) return 2 * zplane + 2 * yslab + (size_t)k * ny + (size_t)j;
  return 2 * zplane + 2 * yslab + xcol + (size_t)k * ny + (size_t)j; /* i == nx */
}

/* fbar+ = a1 f~ + b1 E(phi) (eq. 2.21) at cell (i, j, k) of the ghost shell;
 * ring: the step's boundary values (NULL without Dirichlet walls) */
static void fbar_plus(const Oracle3* o, int i, int j, int k, const double* ring, double* out) {
  int idx[3] = {i, j, k}, s[3], a, m, dir = 0;
  size_t N = ncells(o), c;
  double ft[O3_MAXQ], E[O3_MAXQ], phi = 0.0, tmp[O3_MAXQ];
  for (a = 0; a < 3; ++a) s[a] = wrap_or_clamp(idx[a], o->n[a], o->bc[a]);
  c = cidx(o, s[0], s[1], s[2]);
  for (m = 0; m < o->q; ++m) ft[m] = o->f[m * N + c];
  if (!o->src_n) {
    for (m = 0; m < o->q; ++m) phi += ft[m];
    feq(o, phi, E);
    for (m = 0; m < o->q; ++m) out[m] = o->a1 * ft[m] + o->b1 * E[m];
  } else {
    double S[O3_MAXQ], L = o->lambda, dt = o->dt, h = o->h, F;
    phi = cell_phi_F(o, c, &F);
    feq(o, phi, E);
    source_dist(o, phi, F, S);
    for (m = 0; m < o->q; ++m) {
      /* f~ = f - dt/2 Omega - dt/2 S with Omega = -(f - E)/lambda, solved for f */
      double f = (2.0 * L * ft[m] + dt * E[m] + L * dt * S[m]) / (2.0 * L + dt);
      /* fbar = f - h/2 Omega - h/2 S (eq. 2.27, first line), then fbar+ (second line) */
      double fb = f + h / (2.0 * L) * (f - E[m]) - 0.5 * h * S[m];
      out[m] = (2.0 * L - h) / (2.0 * L + h) * fb + 2.0 * h / (2.0 * L + h) * E[m] +
               2.0 * L * h / (2.0 * L + h) * S[m];
    }
  }
  for (a = 0; a < 3; ++a)
    if ((idx[a] < 0 || idx[a] >= o->n[a]) && o->bc[a] == O3_DIRICHLET) dir = 1;
  if (dir) {
    /* non-equilibrium extrapolation from the nearest interior cell */
    double Eg[O3_MAXQ];
    feq(o, ring[shell_index(o, i, j, k)], Eg);
    for (m = 0; m < o->q; ++m) out[m] = Eg[m] + (out[m] - E[m]);
    return;
  }
  for (a = 0; a < 3; ++a) {
    int wall = (idx[a] < 0 || idx[a] >= o->n[a]) && o->bc[a] == O3_MIRROR;
    if (!wall) continue;
    memcpy(tmp, out, sizeof(double) * (size_t)o->q);
    for (m = 0; m < o->q; ++m) out[m] = tmp[o->mir[a][m]];
  }
}

/* f~+ = a2 f~ + b2 E(phi) (eq. 2.13) at interior cell c; with a source the
 * second line of eq. 2.25 adds 2 lambda dt / (2 lambda + dt) S */
static void ftilde_plus(const Oracle3* o, size_t c, double* out) {
  size_t N = ncells(o);
  double ft[O3_MAXQ], E[O3_MAXQ], S[O3_MAXQ], phi, F;
  int m;
  for (m = 0; m < o->q; ++m) ft[m] = o->f[m * N + c];
  phi = cell_phi_F(o, c, &F);
  feq(o, phi, E);
  for (m = 0; m < o->q; ++m) out[m] = o->a2 * ft[m] + o->b2 * E[m];
  if (!o->src_n) return;
  source_dist(o, phi, F, S);
  for (m = 0; m < o->q; ++m) out[m] += 2.0 * o->lambda * o->dt / (2.0 * o->lambda + o->dt) * S[m];
}

/* Access to fbar+ of the ghost shell through a callback so that the full
 * step (a precomputed array) and the sampled step (a local block) share the
 * face and update code. */
typedef const double* (*GetG)(const void* ctx, int i, int j, int k);

/* central-difference slope of fbar+ along axis b at cell (i, j, k) */
static void slope(const Oracle3* o, GetG G, const void* ctx, int i, int j, int k, int b, double* s) {
  int lo[3] = {i, j, k}, hi[3] = {i, j, k}, m;
  const double *fm, *fp;
  double dist;
  lo[b] -= 1; hi[b] += 1;
  fm = G(ctx, lo[0], lo[1], lo[2]);
  fp = G(ctx, hi[0], hi[1], hi[2]);
  dist = CC(o, b, hi[b]) - CC(o, b, lo[b]);
  for (m = 0; m < o->q; ++m) s[m] = (fp[m] - fm[m]) / dist;
}

/* Flux c_n f_b through the face of axis a between the cell below (i, j, k)
 * minus one along a and the cell (i, j, k): reconstruction (eq. 2.20),
 * characteristic shift (eq. 2.19 as eq. 2.26), phi_b = sum fbar,
 * f_b = a3 fbar + b3 E(phi_b) (eq. 2.22), flux (eq. 2.9). */
static void face_flux(const Oracle3* o, GetG G, const void* ctx, int a, int i, int j, int k,
                      double* flux) {
  int L[3] = {i, j, k}, R[3] = {i, j, k}, m, b;
  const double *fL, *fR;
  double sL[2][O3_MAXQ], sR[2][O3_MAXQ], fb[O3_MAXQ], E[O3_MAXQ], phib = 0.0, dn, wl;
  int tb[2], nt = 0;
  L[a] -= 1;
  fL = G(ctx, L[0], L[1], L[2]);
  fR = G(ctx, R[0], R[1], R[2]);
  dn = CC(o, a, R[a]) - CC(o, a, L[a]);
  wl = o->fc[a][R[a]] - CC(o, a, L[a]);
  for (b = 0; b < 3; ++b)
    if (b != a) {
      slope(o, G, ctx, L[0], L[1], L[2], b, sL[nt]);
      slope(o, G, ctx, R[0], R[1], R[2], b, sR[nt]);
      tb[nt++] = b;
    }
  for (m = 0; m < o->q; ++m) {
    double Gn = (fR[m] - fL[m]) / dn;
    double v = fL[m] + wl * Gn;
    double shift = o->cv[m][a] * Gn;
    int t;
    for (t = 0; t < 2; ++t) shift += o->cv[m][tb[t]] * 0.5 * (sL[t][m] + sR[t][m]);
    fb[m] = v - o->h * shift;
  }
  for (m = 0; m < o->q; ++m) phib += fb[m];
  if (!o->src_n) {
    feq(o, phib, E);
    for (m = 0; m < o->q; ++m) flux[m] = o->cv[m][a] * (o->a3 * fb[m] + o->b3 * E[m]);
  } else {
    /* F at the face at t_n + h (where fbar lives, eq. 2.27), each G_j
       interpolated linearly between the centres (a ghost takes its source
       cell's); phi_b = sum fbar + h F_b / 2; f from the first line of eq. 2.27 */
    double S[O3_MAXQ], Lm = o->lambda, h = o->h, ac[O3_MAXPOW + 1], Fb;
    int sl[3], sr[3], b2;
    for (b2 = 0; b2 < 3; ++b2) {
      sl[b2] = wrap_or_clamp(L[b2], o->n[b2], o->bc[b2]);
      sr[b2] = wrap_or_clamp(R[b2], o->n[b2], o->bc[b2]);
    }
    source_coefs(o, cidx(o, sl[0], sl[1], sl[2]), cidx(o, sr[0], sr[1], sr[2]), wl / dn, o->t + h, ac);
    phib = solve_conserved(o, phib, h, ac);
    Fb = poly3(ac, phib);
    feq(o, phib, E);
    source_dist(o, phib, Fb, S);
    for (m = 0; m < o->q; ++m)
      flux[m] = o->cv[m][a] * (2.0 * Lm * fb[m] + h * E[m] + Lm * h * S[m]) / (2.0 * Lm + h);
  }
}

/* eq. 2.24 on a Cartesian cell: the surface integral of eq. 2.9 with the
 * midpoint rule on each of the six faces, over |V| */
static void update_cell(const Oracle3* o, GetG G, const void* ctx, int i, int j, int k,
                        double* out) {
  double ftp[O3_MAXQ], lo[O3_MAXQ], hi[O3_MAXQ], div[O3_MAXQ];
  int a, m, idx[3] = {i, j, k};
  for (m = 0; m < o->q; ++m) div[m] = 0.0;
  for (a = 0; a < 3; ++a) {
    int up[3] = {i, j, k};
    up[a] += 1;
    face_flux(o, G, ctx, a, i, j, k, lo);
    face_flux(o, G, ctx, a, up[0], up[1], up[2], hi);
    for (m = 0; m < o->q; ++m) div[m] += (hi[m] - lo[m]) / WD(o, a, idx[a]);
  }
  ftilde_plus(o, cidx(o, i, j, k), ftp);
  for (m = 0; m < o->q; ++m) out[m] = ftp[m] - o->dt * div[m];
}

typedef struct {
  const Oracle3* o;
  double* g;  /* fbar+ on cells -1..n per axis, [(k+1)][(j+1)][(i+1)][q] */
} FullCtx;

/* number of boundary values of one step */
size_t or3_shell_len(const Oracle3* o) {
  const size_t nx = o->n[0], ny = o->n[1], nz = o->n[2];
  return 2 * (nx + 2) * (ny + 2) + 2 * (nx + 2) * nz + 2 * ny * nz;
}

static const double* full_get(const void* ctx, int i, int j, int k) {
  const FullCtx* F = (const FullCtx*)ctx;
  const Oracle3* o = F->o;
  return F->g + ((((size_t)(k + 1) * (o->n[1] + 2)) + (j + 1)) * (o->n[0] + 2) + (i + 1)) * o->q;
}

static void step_once(Oracle3* o, const double* ring) {
  const int nx = o->n[0], ny = o->n[1], nz = o->n[2], q = o->q;
  const size_t N = ncells(o);
  FullCtx F;
  double* fn = (double*)malloc(sizeof(double) * N * q);
  int i, j, k, m;
  F.o = o;
  F.g = (double*)malloc(sizeof(double) * (size_t)(nx + 2) * (ny + 2) * (nz + 2) * q);
#pragma omp parallel for private(i, j)
  for (k = -1; k <= nz; ++k)
    for (j = -1; j <= ny; ++j)
      for (i = -1; i <= nx; ++i) fbar_plus(o, i, j, k, ring, (double*)full_get(&F, i, j, k));
#pragma omp parallel for private(i, j, m)
  for (k = 0; k < nz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx; ++i) {
        double out[O3_MAXQ];
        update_cell(o, full_get, &F, i, j, k, out);
        for (m = 0; m < q; ++m) fn[m * N + cidx(o, i, j, k)] = out[m];
      }
  memcpy(o->f, fn, sizeof(double) * N * q);
  free(F.g);
  free(fn);
  o->step += 1;
  o->t += o->dt;
}

/* Advance nsteps.  rings: the boundary values of nsteps consecutive steps
 * (step s reads rings + s * or3_shell_len), NULL without Dirichlet walls. */
void or3_step(Oracle3* o, int nsteps, const double* rings) {
  int s;
  const size_t len = or3_shell_len(o);
  for (s = 0; s < nsteps; ++s) step_once(o, rings ? rings + (size_t)s * len : NULL);
}

typedef struct {
  const Oracle3* o;
  int ci, cj, ck;
  double g[3][3][3][O3_MAXQ];  /* fbar+ on the 3^3 block around the cell */
} LocalCtx;

static const double* local_get(const void* ctx, int i, int j, int k) {
  const LocalCtx* L = (const LocalCtx*)ctx;
  return L->g[k - L->ck + 1][j - L->cj + 1][i - L->ci + 1];
}

/* One step evaluated only at the listed cells (triples i, j, k), without
 * changing the state; the same face and update code as the full step.
 * out: [ncells][q]. */
void or3_step_cells(const Oracle3* o, int ncells_, const int* cells, const double* ring, double* out) {
  int n, a, b, c;
  LocalCtx* L = (LocalCtx*)malloc(sizeof(LocalCtx));
  L->o = o;
  for (n = 0; n < ncells_; ++n) {
    int i = cells[3 * n], j = cells[3 * n + 1], k = cells[3 * n + 2];
    L->ci = i; L->cj = j; L->ck = k;
    for (c = -1; c <= 1; ++c)
      for (b = -1; b <= 1; ++b)
        for (a = -1; a <= 1; ++a) fbar_plus(o, i + a, j + b, k + c, ring, L->g[c + 1][b + 1][a + 1]);
    update_cell(o, local_get, L, i, j, k, out + (size_t)n * o->q);
  }
  free(L);
}

/* GRE (eq. 4.1, unweighted) and area-weighted relative L2 against phi_a */
void or3_errors(const Oracle3* o, const double* phi_a, double* gre, double* rel_l2) {
  int i, j, k;
  double num = 0.0, den = 0.0, e2 = 0.0, r2 = 0.0;
  for (k = 0; k < o->n[2]; ++k)
    for (j = 0; j < o->n[1]; ++j)
      for (i = 0; i < o->n[0]; ++i) {
        size_t c = cidx(o, i, j, k);
        double phi = cell_phi_F(o, c, NULL), v = WD(o, 0, i) * WD(o, 1, j) * WD(o, 2, k);
        num += fabs(phi_a[c] - phi);
        den += fabs(phi_a[c]);
        e2 += v * (phi - phi_a[c]) * (phi - phi_a[c]);
        r2 += v * phi_a[c] * phi_a[c];
      }
  *gre = num / den;
  *rel_l2 = sqrt(e2 / r2);
}

double or3_mass(const Oracle3* o) {
  int i, j, k;
  double s = 0.0;
  for (k = 0; k < o->n[2]; ++k)
    for (j = 0; j < o->n[1]; ++j)
      for (i = 0; i < o->n[0]; ++i) {
        size_t c = cidx(o, i, j, k);
        s += cell_phi_F(o, c, NULL) * WD(o, 0, i) * WD(o, 1, j) * WD(o, 2, k);
      }
  return s;
}
