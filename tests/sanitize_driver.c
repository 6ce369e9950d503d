/* Drives the three CPU oracles (2-D, 3-D, 1-D) through every boundary kind,
 * source terms and the sampled step, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py).  Exits 0 when
 * every call returned and the results are finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void* or_create(int nx, int ny, const double* xf, const double* yf, int q, double c, double cfl,
                double alpha, int bcx, int bcy);
void or_destroy(void* o);
int or_set_B(void* o, int deg, const double* bx, const double* by);
int or_set_D(void* o, int deg, const double* dxx, const double* dxy, const double* dyy);
int or_set_source_terms(void* o, int n, const double* g, const int* pow, const double* gam);
void or_set_phi(void* o, const double* phi);
void or_get_phi(const void* o, double* phi);
void or_step(void* o, int nsteps, const double* rings);
void or_step_cells(const void* o, int ncells, const int* cells, const double* ring, double* out);
void or_fbar_plus_all(const void* o, const double* ring, double* out);
double or_mass(const void* o);

void* or3_create(int nx, int ny, int nz, const double* xf, const double* yf, const double* zf, int q,
                 double c, double cfl, double alpha, int bcx, int bcy, int bcz);
void or3_destroy(void* o);
int or3_set_B(void* o, int deg, const double* b);
int or3_set_D(void* o, int deg, const double* d);
void or3_set_phi(void* o, const double* phi);
void or3_get_phi(const void* o, double* phi);
size_t or3_shell_len(const void* o);
int or3_set_source_terms(void* o, int n, const double* g, const int* pow, const double* gam);
void or3_step(void* o, int nsteps, const double* rings);
void or3_step_cells(const void* o, int ncells, const int* cells, const double* ring, double* out);

void* or1_create(int nx, const double* xf, double c, double cfl, double alpha, int bc, const double* coef);
void or1_destroy(void* o);
void or1_set_phi(void* o, const double* phi0);
void or1_get_phi(const void* o, double* phi);
void or1_step(void* o, int nsteps, const double* ghosts);
void or1_step_cells(const void* o, int ncells, const int* cells, const double* ghosts, double* out);

static int bad = 0;
static void check(const double* v, size_t n, const char* what) {
  size_t i;
  for (i = 0; i < n; ++i)
    if (!isfinite(v[i])) { fprintf(stderr, "%s: non-finite value at %zu\n", what, i); bad = 1; return; }
}

static double* faces(int n, int stretched) {
  double* f = (double*)malloc(sizeof(double) * (n + 1));
  int i;
  for (i = 0; i <= n; ++i) {
    double s = (double)i / n;
    f[i] = stretched ? 0.5 * (1.0 + tanh(1.5 * (2.0 * s - 1.0)) / tanh(1.5)) : s;
  }
  return f;
}

static void two_d(int q, int bc, int src) {
  const int nx = 13, ny = 9, steps = 3, len = 2 * (nx + ny) + 4;
  double *xf = faces(nx, bc != 0), *yf = faces(ny, bc != 0);
  double bx[3] = {0.0, 0.2, -0.1}, by[3] = {0.0, -0.1, 0.15};
  double dxx[3] = {0.0, 1.0, 0.2}, dxy[3] = {0.0, 0.1, 0.0}, dyy[3] = {0.0, 0.9, 0.1};
  double d5xx[2] = {0.0, 1.0}, d5xy[2] = {0.0, 0.0};
  double *phi = malloc(sizeof(double) * nx * ny), *ring = malloc(sizeof(double) * len * steps);
  double *g = malloc(sizeof(double) * 2 * nx * ny), out[4 * 9], *gp = malloc(sizeof(double) * (nx + 2) * (ny + 2) * 9);
  int pw[2] = {0, 2}, cells[8] = {0, 0, nx - 1, ny - 1, 0, ny - 1, nx / 2, 0}, i;
  double gam[2] = {0.3, 0.0};
  void* o = or_create(nx, ny, xf, yf, q, 1.7, 0.5, 2e-3, bc, bc);
  if (!o) { fprintf(stderr, "or_create failed\n"); bad = 1; return; }
  or_set_B(o, 2, bx, by);
  if (q == 9) or_set_D(o, 2, dxx, dxy, dyy); else or_set_D(o, 1, d5xx, d5xy, d5xx);
  for (i = 0; i < nx * ny; ++i) phi[i] = 0.5 + 0.1 * sin(0.7 * i);
  for (i = 0; i < len * steps; ++i) ring[i] = 0.5 + 0.05 * cos(0.3 * i);
  for (i = 0; i < 2 * nx * ny; ++i) g[i] = 0.2 * sin(0.11 * i);
  if (src) or_set_source_terms(o, 2, g, pw, gam);
  or_set_phi(o, phi);
  or_step_cells(o, 4, cells, bc == 1 ? ring : NULL, out);
  check(out, 4 * q, "2-D sampled step");
  or_fbar_plus_all(o, bc == 1 ? ring : NULL, gp);
  check(gp, (size_t)(nx + 2) * (ny + 2) * q, "2-D fbar+");
  or_step(o, steps, bc == 1 ? ring : NULL);
  or_get_phi(o, phi);
  check(phi, nx * ny, "2-D phi");
  if (!isfinite(or_mass(o))) bad = 1;
  or_destroy(o);
  free(xf); free(yf); free(phi); free(ring); free(g); free(gp);
}

static void three_d(int q, int bx_, int by_, int bz_, int src) {
  const int nx = 6, ny = 5, nz = 4, steps = 2, n = nx * ny * nz;
  double *xf = faces(nx, 1), *yf = faces(ny, 0), *zf = faces(nz, 1);
  double b[9] = {0.0, 0.1, 0.05, 0.0, -0.1, 0.0, 0.0, 0.05, 0.1};
  double d[12] = {0.0, 1.0, 0.0, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double *phi = malloc(sizeof(double) * n), *ring, out[3 * 19];
  int cells[9] = {0, 0, 0, nx - 1, ny - 1, nz - 1, 2, 0, nz - 1}, i;
  size_t len;
  void* o = or3_create(nx, ny, nz, xf, yf, zf, q, 1.3, 0.5, 1e-3, bx_, by_, bz_);
  if (!o) { fprintf(stderr, "or3_create failed\n"); bad = 1; return; }
  if (q != 7) d[7] = 0.05;   /* an xy term of D (D3Q7 takes D = phi I only) */
  or3_set_B(o, 2, b);
  or3_set_D(o, 1, d);
  len = or3_shell_len(o);
  if (src) {
    double* g = malloc(sizeof(double) * 2 * n);
    int pw[2] = {1, 0};
    double gam[2] = {0.0, 0.4};
    for (i = 0; i < 2 * n; ++i) g[i] = 0.3 * cos(0.17 * i);
    if (or3_set_source_terms(o, 2, g, pw, gam) != 0) bad = 1;
    free(g);
  }
  ring = malloc(sizeof(double) * len * steps);
  for (i = 0; i < n; ++i) phi[i] = 0.5 + 0.1 * cos(0.37 * i);
  for (i = 0; i < (int)(len * steps); ++i) ring[i] = 0.5 + 0.05 * sin(0.21 * i);
  or3_set_phi(o, phi);
  or3_step_cells(o, 3, cells, ring, out);
  check(out, 3 * q, "3-D sampled step");
  or3_step(o, steps, ring);
  or3_get_phi(o, phi);
  check(phi, n, "3-D phi");
  or3_destroy(o);
  free(xf); free(yf); free(zf); free(phi); free(ring);
}

static void one_d(void) {
  const int nx = 20, steps = 3;
  double* xf = faces(nx, 1);
  double coef[7] = {0.1, 0.2, 1.0, 0.5, 0.1, 1.0, 0.3}, phi[20], ghosts[6], out[2 * 3];
  int cells[2] = {0, nx - 1}, i;
  void* o = or1_create(nx, xf, 1.0, 0.5, 1e-3, 1, coef);
  if (!o) { fprintf(stderr, "or1_create failed\n"); bad = 1; return; }
  for (i = 0; i < nx; ++i) phi[i] = 0.5 + 0.1 * sin(0.5 * i);
  for (i = 0; i < 2 * steps; ++i) ghosts[i] = 0.4 + 0.01 * i;
  or1_set_phi(o, phi);
  or1_step_cells(o, 2, cells, ghosts, out);
  check(out, 6, "1-D sampled step");
  or1_step(o, steps, ghosts);
  or1_get_phi(o, phi);
  check(phi, nx, "1-D phi");
  or1_destroy(o);
  free(xf);
}

int main(void) {
  int q, bc;
  for (q = 9; q >= 5; q -= 4)
    for (bc = 0; bc <= 2; ++bc) two_d(q, bc, q == 9 && bc != 2);
  three_d(19, 1, 2, 0, 1);
  three_d(19, 0, 0, 0, 0);
  three_d(15, 2, 1, 1, 1);
  three_d(7, 1, 1, 2, 1);
  one_d();
  if (!bad) printf("sanitized oracle runs: ok\n");
  return bad;
}
