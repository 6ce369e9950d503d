/*
 * libdugks, one-dimensional path: the DUGKS time step of Sec. 2 of Shang,
 * Chai, Wang, Shi, "Discrete unified gas kinetic scheme for nonlinear
 * convection-diffusion equations" (arXiv 1906.11036) on the D1Q3 lattice
 * (eq. 2.4) for a convection term that depends on x and t as well as on phi,
 * the case of Remark 3 with C = 0 (Example 4.6):
 *
 *   d_t phi + d_x B = d_x (alpha d_x D),     (eq. 2.1 with F = 0)
 *   B = b(x, t) phi,  b = (p0 + p1 t) x + q0 exp(q1 t + q2 t^2),
 *   D = d(t) phi,     d = r0 + r1 t,
 *   E_i = w_i [phi + c_i B / c_s^2 + (c_s^2 D - c_s^2 phi)(c_i^2 - c_s^2) / (2 c_s^4)]  (eq. 2.3, C = 0),
 *   R_i = w_i c_i dB/dt / c_s^2                                                   (Remark 3).
 *
 * Same conventions as dugks.h: C ABI, every call returns an int code of
 * dugks.h (DUGKS_OK = 0, negative on error), dugks1_last_error() names the
 * problem.  The caller owns the device workspace (dugks1_workspace_bytes,
 * 256-byte aligned) and the stream; the library owns only its host handle.
 * Stepping is asynchronous on the bound stream; read-outs synchronise.
 *
 * Readings (as in the CPU oracle): dB/dt at a cell at t_n is the backward
 * difference [b(x, t_n) phi^n - b(x, t_{n-1}) phi^{n-1}] / dt (phi^{-1} = phi^0
 * at the first step after dugks1_set_phi), so the state is f~ and phi^{n-1};
 * dB/dt at a face is the linear interpolation of eq. 2.20 of the two cells'
 * values; E at a face is taken at (x_b, t_n + h); lambda = alpha / c_s^2,
 * c_s^2 = c^2/3; dt = cfl * (smallest cell width) / c; walls are periodic
 * (only for b independent of x: p0 = p1 = 0) or Dirichlet by non-equilibrium
 * extrapolation from caller data at the ghost centres.
 */
#ifndef DUGKS1D_H
#define DUGKS1D_H

#include <stddef.h>

#include "dugks.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DUGKS1_ABI_VERSION 1

typedef struct dugks1_params {
  int abi_version; /* must be DUGKS1_ABI_VERSION */
  int storage;     /* DUGKS_F64 or DUGKS_F32 */
  int bc;          /* DUGKS_BC_PERIODIC or DUGKS_BC_DIRICHLET (both walls) */
  double c;        /* lattice speed, > 0 */
  double cfl;      /* CFL number, 0 < cfl < 1 */
  double alpha;    /* diffusion coefficient of eq. 2.1, > 0 */
  double coef[7];  /* p0, p1, q0, q1, q2, r0, r1 of b(x, t) and d(t) above */
  double t0;       /* time of the state given to dugks1_set_phi / dugks1_set_state */
} dugks1_params;

typedef struct dugks1_info {
  double dt, h, lambda, cs2;
  double time;            /* t0 + steps * dt */
  long long steps;        /* steps taken since the last set_phi / set_state */
  int nx, storage, bc;
  int dirichlet_left;     /* Dirichlet steps still available from the last dugks1_set_dirichlet */
  size_t state_bytes;     /* bytes of one state buffer (f~ and phi^{n-1}) */
} dugks1_info;

typedef struct dugks1_ctx dugks1_ctx;

/* Create an instance on nx cells with faces xf[0..nx] (host, copied, strictly
 * increasing).  No device work.  Errors: E_ARG (sizes, faces, c, cfl, alpha,
 * abi_version, periodic walls with p0 or p1 non-zero), E_UNSUPPORTED (storage,
 * boundary kind).  On an error other than a NULL out, *out still receives a
 * handle for dugks1_last_error / dugks1_destroy. */
int dugks1_create(dugks1_ctx** out, int nx, const double* xf, const dugks1_params* p);

/* Device workspace needed, in bytes. */
size_t dugks1_workspace_bytes(const dugks1_ctx* ctx);

/* Attach the caller's workspace (device, >= dugks1_workspace_bytes, 256-byte
 * aligned) and stream (hipStream_t as void*); uploads the mesh tables.
 * Errors: E_ARG, E_HIP. */
int dugks1_bind(dugks1_ctx* ctx, void* dev_workspace, size_t bytes, void* hip_stream);

/* f = E(phi) at t0 (Sec. 4, Omega = 0), f~ = f - dt R / 2 with dB/dt from
 * phi^{-1} = phi at t0 - dt; phi^{n-1} = phi.  phi [nx] binary64 (host if
 * on_device == 0).  Resets the step count and time to t0.  Errors: E_STATE
 * (not bound), E_ARG, E_HIP. */
int dugks1_set_phi(dugks1_ctx* ctx, const double* phi, int on_device);

/* f~ [3][nx] and phi^{n-1} [nx] (binary64) as the state at t0. */
int dugks1_set_state(dugks1_ctx* ctx, const double* f, const double* phi_prev, int on_device);

/* Dirichlet data: ghosts [2 * nsteps] (device, caller-owned, kept alive while
 * stepping): phi at the left and the right ghost centre (half a cell outside
 * each wall, the adjacent cell's width) at the times of the next nsteps
 * steps, t_n, t_n + dt, ...  Each step consumes one pair; the pair of the
 * previous step gives the ghosts' dB/dt (the first step after set_phi /
 * set_state uses the current pair for both).  Errors: E_ARG, E_STATE
 * (periodic walls). */
int dugks1_set_dirichlet(dugks1_ctx* ctx, const double* ghosts, int nsteps);

/* Advance nsteps >= 0 steps (asynchronous).  Errors: E_STATE (not bound, no
 * state, Dirichlet data exhausted: nothing is stepped), E_HIP. */
int dugks1_step(dugks1_ctx* ctx, int nsteps);

/* phi = sum_i f~_i [nx], f~ [3][nx], phi^{n-1} [nx], binary64 (host if
 * on_device == 0).  Synchronise. */
int dugks1_get_phi(dugks1_ctx* ctx, double* out, int on_device);
int dugks1_get_f(dugks1_ctx* ctx, double* out, int on_device);
int dugks1_get_phi_prev(dugks1_ctx* ctx, double* out, int on_device);

/* mass = sum phi |V|; with ref (device, [nx], or NULL) also the GRE of eq.
 * 4.1 (unweighted) and the width-weighted relative L2 difference.  Output
 * pointers may be NULL.  Synchronises.  A non-finite cell returns E_UNSTABLE. */
int dugks1_reduce(dugks1_ctx* ctx, const double* ref_dev, double* mass, double* gre, double* rel_l2);

/* Time nsteps steps with hipEvents on the bound stream (the state advances). */
int dugks1_time_steps(dugks1_ctx* ctx, int nsteps, float* ms_total);

int dugks1_get_info(const dugks1_ctx* ctx, dugks1_info* out);
const char* dugks1_last_error(const dugks1_ctx* ctx);
void dugks1_destroy(dugks1_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DUGKS1D_H */
