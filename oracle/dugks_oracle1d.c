/*
 * Plain FP64 CPU oracle for one DUGKS time step on the D1Q3 lattice (eq. 2.4)
 * of the convection-diffusion equation (eq. 2.1, F = 0) with a convection
 * term that depends on x and t as well as on phi (Shang, Chai, Wang, Shi,
 * arXiv 1906.11036, Remark 3 and Example 4.6):
 *
 *   B(phi, x, t) = b(x, t) phi,   b(x, t) = (p0 + p1 t) x + q0 exp(q1 t + q2 t^2),
 *   D(phi, t)    = d(t) phi,      d(t)    = r0 + r1 t.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  It shares no code,
 * header, table or constant generator with the HIP library, nor with the
 * two- and three-dimensional oracles.
 *
 * IEEE binary64, built with -O2 -ffp-contract=off, no fast-math, no
 * intrinsics.  Sums over the three directions run in index order 0, 1, 2.
 *
 * Because B depends on x and t, the auxiliary moment is C = 0 (Remark 3):
 *   E_i = w_i [phi + c_i B / c_s^2 + (c_s^2 D - c_s^2 phi)(c_i^2 - c_s^2) / (2 c_s^4)]
 * (eq. 2.3 in one dimension) and R_i = w_i c_i dB/dt / c_s^2.  The source
 * distribution R enters through the shifted distributions of eqs. 2.25 and
 * 2.27, applied literally: f from f~ (first line of eq. 2.25), fbar and
 * fbar+ from eq. 2.27, f~+ from the second line of eq. 2.25, f at the face
 * from the first line of eq. 2.27.  Since sum_i R_i = 0, phi = sum f~ in a
 * cell and phi_b = sum fbar at a face.
 *
 * Readings of points the paper leaves open (each one also listed in the
 * design notes):
 *   - dB/dt at a cell centre at t_n is the backward difference
 *     [b(x, t_n) phi^n - b(x, t_{n-1}) phi^{n-1}] / dt (the paper evaluates
 *     the time derivatives of its source distributions by such differences,
 *     Sec. 2 after eq. 2.13); at the first step phi^{-1} = phi^0 and
 *     t_{-1} = -dt;
 *   - dB/dt at a face is the linear interpolation (eq. 2.20) of the two
 *     cells' values at t_n; E at the face is taken at (x_b, t_n + h);
 *   - f~ is initialised as f - dt R / 2 with f = E(phi_0) (Sec. 4, Omega = 0);
 *   - dt = cfl * (smallest cell width) / c, lambda = alpha / c_s^2;
 *   - boundary ghosts: periodic (wrapped cell; only for b independent of x,
 *     p0 = p1 = 0, since the wrapped face must see one b) or Dirichlet by
 *     non-equilibrium extrapolation, fbar+_g = E(phi_g, x_g) + (fbar+_a -
 *     E(phi_a, x_a)) with phi_g the caller's value at the ghost centre at t_n
 *     (the ghost takes the width of the adjacent cell); the ghost's dB/dt
 *     comes from its own data at t_n and t_{n-1}.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { O1_PERIODIC = 0, O1_DIRICHLET = 1 };

typedef struct {
  int nx, bc;
  double c, cfl, alpha;
  double cv[3], w[3], cs2;
  double p0, p1, q0, q1, q2, r0, r1;
  double lambda, dt, h;
  double *xf, *wd, *xc;     /* faces [nx+1]; widths and centres [nx+2], ghosts at 0 and nx+1 */
  double *f;                /* f~ [3][nx] */
  double *phi_prev;         /* phi^{n-1} [nx] */
  double gprev[2];          /* Dirichlet ghost values at t_{n-1} */
  int have_gprev;
  long step;
  double t;
} Oracle1;

static double coef_b(const Oracle1* o, double x, double t) {
  return (o->p0 + o->p1 * t) * x + o->q0 * exp(o->q1 * t + o->q2 * t * t);
}
static double coef_d(const Oracle1* o, double t) { return o->r0 + o->r1 * t; }

/* eq. 2.3 with C = 0 in one dimension (I = 1, tensors are scalars) */
static void feq(const Oracle1* o, double phi, double x, double t, double* E) {
  const double cs2 = o->cs2, B = coef_b(o, x, t) * phi, D = coef_d(o, t) * phi;
  int i;
  for (i = 0; i < 3; ++i) {
    const double ci = o->cv[i];
    E[i] = o->w[i] * (phi + ci * B / cs2 + (cs2 * D - cs2 * phi) * (ci * ci - cs2) / (2.0 * cs2 * cs2));
  }
}

/* R_i = w_i c_i dB/dt / c_s^2 (Remark 3, C = 0) */
static void rdist(const Oracle1* o, double dB, double* R) {
  int i;
  for (i = 0; i < 3; ++i) R[i] = o->w[i] * o->cv[i] * dB / o->cs2;
}

Oracle1* or1_create(int nx, const double* xf, double c, double cfl, double alpha, int bc,
                    const double* coef) {
  Oracle1* o;
  int i;
  double wmin;
  if (nx < 1 || !(c > 0) || !(cfl > 0 && cfl < 1) || !(alpha > 0)) return NULL;
  if (bc != O1_PERIODIC && bc != O1_DIRICHLET) return NULL;
  /* periodic walls need b periodic in x: no x-dependence */
  if (bc == O1_PERIODIC && (coef[0] != 0.0 || coef[1] != 0.0)) return NULL;
  for (i = 0; i < nx; ++i)
    if (!(xf[i + 1] > xf[i])) return NULL;
  o = (Oracle1*)calloc(1, sizeof(Oracle1));
  o->nx = nx;
  o->bc = bc;
  o->c = c;
  o->cfl = cfl;
  o->alpha = alpha;
  /* D1Q3, eq. 2.4 */
  o->cv[0] = 0.0;
  o->cv[1] = c;
  o->cv[2] = -c;
  o->w[0] = 2.0 / 3.0;
  o->w[1] = 1.0 / 6.0;
  o->w[2] = 1.0 / 6.0;
  o->cs2 = c * c / 3.0;
  o->p0 = coef[0];
  o->p1 = coef[1];
  o->q0 = coef[2];
  o->q1 = coef[3];
  o->q2 = coef[4];
  o->r0 = coef[5];
  o->r1 = coef[6];
  o->xf = (double*)malloc(sizeof(double) * (nx + 1));
  o->wd = (double*)malloc(sizeof(double) * (nx + 2));
  o->xc = (double*)malloc(sizeof(double) * (nx + 2));
  memcpy(o->xf, xf, sizeof(double) * (nx + 1));
  for (i = 0; i < nx; ++i) {
    o->wd[i + 1] = xf[i + 1] - xf[i];
    o->xc[i + 1] = 0.5 * (xf[i] + xf[i + 1]);
  }
  if (bc == O1_PERIODIC) {
    const double L = xf[nx] - xf[0];
    o->wd[0] = o->wd[nx];
    o->xc[0] = o->xc[nx] - L;
    o->wd[nx + 1] = o->wd[1];
    o->xc[nx + 1] = o->xc[1] + L;
  } else {
    o->wd[0] = o->wd[1];
    o->xc[0] = xf[0] - 0.5 * o->wd[1];
    o->wd[nx + 1] = o->wd[nx];
    o->xc[nx + 1] = xf[nx] + 0.5 * o->wd[nx];
  }
  wmin = o->wd[1];
  for (i = 1; i <= nx; ++i)
    if (o->wd[i] < wmin) wmin = o->wd[i];
  o->lambda = alpha / o->cs2;
  o->dt = cfl * wmin / c;
  o->h = 0.5 * o->dt;
  o->f = (double*)calloc((size_t)3 * nx, sizeof(double));
  o->phi_prev = (double*)calloc((size_t)nx, sizeof(double));
  return o;
}

void or1_destroy(Oracle1* o) {
  if (!o) return;
  free(o->xf);
  free(o->wd);
  free(o->xc);
  free(o->f);
  free(o->phi_prev);
  free(o);
}

/* out: lambda, dt, h, cs2 */
void or1_constants(const Oracle1* o, double* out) {
  out[0] = o->lambda;
  out[1] = o->dt;
  out[2] = o->h;
  out[3] = o->cs2;
}
double or1_time(const Oracle1* o) { return o->t; }
void or1_set_time(Oracle1* o, double t) { o->t = t; }
void or1_feq(const Oracle1* o, double phi, double x, double t, double* E) { feq(o, phi, x, t, E); }
void or1_rdist(const Oracle1* o, double dB, double* R) { rdist(o, dB, R); }

/* f = E(phi0) at the current time (Omega = 0), f~ = f - dt R / 2 with dB/dt
 * from phi^{-1} = phi^0 at t - dt; phi^{n-1} = phi0. */
void or1_set_phi(Oracle1* o, const double* phi0) {
  const int nx = o->nx;
  int j, i;
  for (j = 0; j < nx; ++j) {
    double E[3], R[3];
    const double x = o->xc[j + 1], t = o->t;
    const double dB = (coef_b(o, x, t) * phi0[j] - coef_b(o, x, t - o->dt) * phi0[j]) / o->dt;
    feq(o, phi0[j], x, t, E);
    rdist(o, dB, R);
    for (i = 0; i < 3; ++i) o->f[(size_t)i * nx + j] = E[i] - 0.5 * o->dt * R[i];
    o->phi_prev[j] = phi0[j];
  }
  o->have_gprev = 0;
  o->step = 0;
}

/* f~ [3][nx] and phi^{n-1} [nx] as the state */
void or1_set_state(Oracle1* o, const double* f, const double* phi_prev) {
  memcpy(o->f, f, sizeof(double) * 3 * (size_t)o->nx);
  memcpy(o->phi_prev, phi_prev, sizeof(double) * (size_t)o->nx);
  o->have_gprev = 0;
}
void or1_get_f(const Oracle1* o, double* f) { memcpy(f, o->f, sizeof(double) * 3 * (size_t)o->nx); }
void or1_get_phi_prev(const Oracle1* o, double* p) { memcpy(p, o->phi_prev, sizeof(double) * (size_t)o->nx); }

static double cell_phi(const Oracle1* o, int j) {
  double s = 0.0;
  int i;
  for (i = 0; i < 3; ++i) s += o->f[(size_t)i * o->nx + j];
  return s;
}

void or1_get_phi(const Oracle1* o, double* phi) {
  int j;
  for (j = 0; j < o->nx; ++j) phi[j] = cell_phi(o, j);
}

/* Per-cell quantities at t_n for cell j (0..nx-1): phi, dB/dt, fbar+ and f~+
 * (eqs. 2.25 and 2.27 applied literally). */
static void cell_state(const Oracle1* o, int j, double* phi_out, double* dB_out, double* fbp,
                       double* ftp) {
  const double lam = o->lambda, dt = o->dt, h = o->h, t = o->t, x = o->xc[j + 1];
  double E[3], R[3], phi;
  int i;
  phi = cell_phi(o, j);
  *phi_out = phi;
  *dB_out = (coef_b(o, x, t) * phi - coef_b(o, x, t - dt) * o->phi_prev[j]) / dt;
  feq(o, phi, x, t, E);
  rdist(o, *dB_out, R);
  for (i = 0; i < 3; ++i) {
    const double ft = o->f[(size_t)i * o->nx + j];
    /* f~ = f + dt/(2 lambda) (f - E) - dt/2 R   (first line of eq. 2.25) */
    const double f = (ft + dt / (2.0 * lam) * E[i] + 0.5 * dt * R[i]) / (1.0 + dt / (2.0 * lam));
    /* fbar = f - h/2 Omega - h/2 R              (first line of eq. 2.27) */
    const double fb = f + h / (2.0 * lam) * (f - E[i]) - 0.5 * h * R[i];
    if (fbp)
      fbp[i] = (2.0 * lam - h) / (2.0 * lam + h) * fb + 2.0 * h / (2.0 * lam + h) * E[i] +
               2.0 * lam * h / (2.0 * lam + h) * R[i];
    if (ftp)
      ftp[i] = (2.0 * lam - dt) / (2.0 * lam + dt) * ft + 2.0 * dt / (2.0 * lam + dt) * E[i] +
               2.0 * lam * dt / (2.0 * lam + dt) * R[i];
  }
}

/* fbar+ and dB/dt of cell k in 0..nx+1 (0 and nx+1 are ghosts); ghost data
 * g[0], g[1] at t_n and gp[0], gp[1] at t_{n-1} for Dirichlet walls. */
static void ext_state(const Oracle1* o, int k, const double* g, const double* gp, double* fbp,
                      double* dB) {
  const int nx = o->nx;
  double phi;
  if (k >= 1 && k <= nx) {
    cell_state(o, k - 1, &phi, dB, fbp, NULL);
    return;
  }
  if (o->bc == O1_PERIODIC) {
    cell_state(o, k == 0 ? nx - 1 : 0, &phi, dB, fbp, NULL);
    return;
  }
  {
    const int a = k == 0 ? 0 : nx - 1, side = k == 0 ? 0 : 1;
    const double xg = o->xc[k], xa = o->xc[a + 1], t = o->t;
    double fa[3], dBa, phia, Eg[3], Ea[3];
    int i;
    cell_state(o, a, &phia, &dBa, fa, NULL);
    feq(o, g[side], xg, t, Eg);
    feq(o, phia, xa, t, Ea);
    for (i = 0; i < 3; ++i) fbp[i] = Eg[i] + (fa[i] - Ea[i]);
    *dB = (coef_b(o, xg, t) * g[side] - coef_b(o, xg, t - o->dt) * gp[side]) / o->dt;
  }
}

/* f at face m (between extended cells m and m+1, m = 0..nx) at t_n + h */
static void face_f(const Oracle1* o, int m, const double* g, const double* gp, double* fface) {
  const double lam = o->lambda, h = o->h, t = o->t;
  const double xL = o->xc[m], xR = o->xc[m + 1], xb = o->xf[m];
  double fL[3], fR[3], dBL, dBR, fbar[3], E[3], R[3], phib, dBb;
  int i;
  ext_state(o, m, g, gp, fL, &dBL);
  ext_state(o, m + 1, g, gp, fR, &dBR);
  for (i = 0; i < 3; ++i) {
    /* eq. 2.20: slope and value of fbar+ at the face, then eqs. 2.19/2.26 */
    const double s = (fR[i] - fL[i]) / (xR - xL);
    const double fb = fL[i] + s * (xb - xL);
    fbar[i] = fb - h * o->cv[i] * s;
  }
  phib = fbar[0] + fbar[1] + fbar[2];
  dBb = dBL + (dBR - dBL) * (xb - xL) / (xR - xL);
  feq(o, phib, xb, t + h, E);
  rdist(o, dBb, R);
  for (i = 0; i < 3; ++i)
    /* fbar = f + h/(2 lambda)(f - E) - h/2 R  solved for f (eq. 2.27) */
    fface[i] = (fbar[i] + h / (2.0 * lam) * E[i] + 0.5 * h * R[i]) / (1.0 + h / (2.0 * lam));
}

static void update_cell(const Oracle1* o, int j, const double* g, const double* gp, double* out) {
  double ftp[3], phi, dB, fW[3], fE[3];
  int i;
  cell_state(o, j, &phi, &dB, NULL, ftp);
  face_f(o, j, g, gp, fW);
  face_f(o, j + 1, g, gp, fE);
  for (i = 0; i < 3; ++i)
    /* eq. 2.24 with the flux of eq. 2.9 */
    out[i] = ftp[i] - o->dt / o->wd[j + 1] * o->cv[i] * (fE[i] - fW[i]);
}

/* ghosts: for Dirichlet walls, 2 values (left, right ghost centre) per step
 * at t_n, t_{n+1}, ...; ignored for periodic walls. */
void or1_step(Oracle1* o, int nsteps, const double* ghosts) {
  const int nx = o->nx;
  double* nf = (double*)malloc(sizeof(double) * 3 * (size_t)nx);
  double* np = (double*)malloc(sizeof(double) * (size_t)nx);
  int s, j, i;
  for (s = 0; s < nsteps; ++s) {
    double g[2] = {0.0, 0.0}, gp[2];
    if (o->bc == O1_DIRICHLET) {
      g[0] = ghosts[2 * s];
      g[1] = ghosts[2 * s + 1];
    }
    gp[0] = o->have_gprev ? o->gprev[0] : g[0];
    gp[1] = o->have_gprev ? o->gprev[1] : g[1];
    for (j = 0; j < nx; ++j) {
      double out[3];
      update_cell(o, j, g, gp, out);
      for (i = 0; i < 3; ++i) nf[(size_t)i * nx + j] = out[i];
      np[j] = cell_phi(o, j);
    }
    memcpy(o->f, nf, sizeof(double) * 3 * (size_t)nx);
    memcpy(o->phi_prev, np, sizeof(double) * (size_t)nx);
    o->gprev[0] = g[0];
    o->gprev[1] = g[1];
    o->have_gprev = 1;
    o->step += 1;
    o->t += o->dt;
  }
  free(nf);
  free(np);
}

/* one step evaluated at the listed cells, state unchanged; ghosts as one step
 * of or1_step; the ghost values at t_{n-1} are those of the last step taken */
void or1_step_cells(const Oracle1* o, int ncells, const int* cells, const double* ghosts, double* out) {
  double g[2] = {0.0, 0.0}, gp[2];
  int n;
  if (o->bc == O1_DIRICHLET) {
    g[0] = ghosts[0];
    g[1] = ghosts[1];
  }
  gp[0] = o->have_gprev ? o->gprev[0] : g[0];
  gp[1] = o->have_gprev ? o->gprev[1] : g[1];
  for (n = 0; n < ncells; ++n) update_cell(o, cells[n], g, gp, out + 3 * (size_t)n);
}

/* GRE (eq. 4.1, unweighted) and width-weighted relative L2 against phi_a */
void or1_errors(const Oracle1* o, const double* phi_a, double* gre, double* rel_l2) {
  double num = 0.0, den = 0.0, e2 = 0.0, r2 = 0.0;
  int j;
  for (j = 0; j < o->nx; ++j) {
    const double p = cell_phi(o, j), d = p - phi_a[j], v = o->wd[j + 1];
    num += fabs(d);
    den += fabs(phi_a[j]);
    e2 += d * d * v;
    r2 += phi_a[j] * phi_a[j] * v;
  }
  *gre = num / den;
  *rel_l2 = sqrt(e2 / r2);
}

double or1_mass(const Oracle1* o) {
  double m = 0.0;
  int j;
  for (j = 0; j < o->nx; ++j) m += cell_phi(o, j) * o->wd[j + 1];
  return m;
}
