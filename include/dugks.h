/*
 * dugks.h -- C ABI of libdugks: the discrete unified gas kinetic scheme
 * (DUGKS) step for the nonlinear convection-diffusion equation
 *
 *     d_t phi + div B(phi) = div(alpha div D(phi)) + F(x, t, phi)      (eq. 2.1)
 *
 * on 2-D Cartesian meshes (uniform or stretched) with the D2Q9 lattice of
 * eq. 2.5 or the D2Q5 lattice of Remark 3, for MI355X (gfx950).
 *
 * Paper: J. Shang, Z. Chai, H. Wang, B. Shi, "Discrete unified gas kinetic
 * scheme for nonlinear convection-diffusion equations", arXiv:1906.11036.
 *
 * ---------------------------------------------------------------- conventions
 * - Every call returns int: DUGKS_OK (0) or a negative DUGKS_E_* code; the
 *   message of the last failure is dugks_last_error(handle).  No C++
 *   exception crosses this boundary.
 * - Ownership: the caller owns all device memory.  The library asks for one
 *   workspace of dugks_workspace_bytes() bytes (device, 256-byte aligned) and
 *   keeps every device array of the instance in it; the library owns only
 *   its opaque host handle.  Host arrays passed in are copied before the call
 *   returns.  The library never frees caller memory.
 * - Streams: work is enqueued on the hipStream_t given to dugks_bind (NULL =
 *   the default stream).  Stepping is asynchronous; dugks_get_phi,
 *   dugks_get_f, dugks_get_diag, dugks_error_norms and dugks_checkpoint
 *   synchronise the stream.  A failure inside device work (a non-finite
 *   value, FP16 overflow) is reported by the next synchronising call.
 * - Arrays of cell values are row-major [ny][nx] (x fastest); distributions
 *   are [q][ny][nx].  Direction i has velocity c*(cx_i, cy_i) with
 *   (cx, cy) = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
 *   (eq. 2.5); D2Q5 uses the first five.
 *
 * ------------------------------------------------------------- the method
 * Constants (Sec. 2, Sec. 3): c_s^2 = c^2/3, lambda = alpha / c_s^2,
 * dt = cfl * min(cell width in x or y) / c, h = dt/2.
 * Equilibrium (eq. 2.3):
 *   E_i = w_i [phi + c_i.B/c_s^2 + (c_s^2 D + C - c_s^2 phi I):(c_i c_i - c_s^2 I)/(2 c_s^4)]
 * with C(phi) = integral_0^phi B'(s) B'(s)^T ds (Remark 3); D2Q5 uses the
 * linear equilibrium E_i = w_i (phi + c_i.B/c_s^2) of Remark 3, which needs
 * D = phi I.  The library tracks f~ (eq. 2.11); one step is the summary at
 * the end of Sec. 2:
 *   fbar+ = (2L-h)/(2L+dt) f~ + 3h/(2L+dt) E          (eq. 2.21)
 *   f~+   = 4/3 fbar+ - 1/3 f~                         (eq. 2.23)
 *   fbar at each face centre from the two adjacent cells (eq. 2.20): normal
 *     derivative (R - L)/(x_R - x_L), value L + (x_face - x_L) * derivative;
 *     tangential derivative = mean of the two cells' central differences;
 *     fbar_b = value - h c_i.grad (eq. 2.19 in the form of eq. 2.26)
 *   phi_b = sum_i fbar_b,i ; f_b = 2L/(2L+h) fbar_b + h/(2L+h) E(phi_b)  (eq. 2.22)
 *   f~(t+dt) = f~+ - dt [c_x (f_E - f_W)/dx + c_y (f_N - f_S)/dy]   (eqs. 2.9, 2.24)
 * Boundaries use a one-cell ghost ring (corners included):
 *   PERIODIC  wrapped cell;
 *   DIRICHLET non-equilibrium extrapolation: fbar+_g = E(phi_g) + fbar+_a - E(phi_a),
 *             a = adjacent interior cell (diagonal one for corners), phi_g
 *             given by the caller at the ghost centre for each step;
 *   MIRROR    zero-flux specular wall: fbar+_g,i = fbar+_a,m(i), m reverses
 *             the wall-normal velocity component.
 * Wall ghosts have the width of the adjacent interior cell; periodic ghosts
 * the width of the wrapped cell.  Where a DIRICHLET axis meets a MIRROR axis, the
 * corner ghost takes the DIRICHLET rule.
 * Initialisation (Sec. 4): f~ = E(phi).
 */
#ifndef DUGKS_H
#define DUGKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DUGKS_ABI_VERSION 4
#define DUGKS_MAX_DEG 4        /* B and D: polynomials in phi of degree <= 4 */
#define DUGKS_MAX_SRC_TERMS 6  /* terms of a source F(x, t, phi) */
#define DUGKS_MAX_SRC_POW 3    /* highest power of phi in a source term */

/* return codes */
#define DUGKS_OK 0
#define DUGKS_E_ARG (-1)         /* invalid argument */
#define DUGKS_E_STATE (-2)       /* call not valid in the handle's state */
#define DUGKS_E_HIP (-3)         /* a HIP runtime call failed */
#define DUGKS_E_UNSTABLE (-4)    /* non-finite value or FP16 overflow seen on the device */
#define DUGKS_E_UNSUPPORTED (-5) /* valid request outside what this library implements */
#define DUGKS_E_NOMEM (-6)       /* workspace too small */
#define DUGKS_E_FORMAT (-7)      /* checkpoint rejected */

/* storage of f~ on the device */
#define DUGKS_F64 0     /* f~ in binary64, binary64 arithmetic */
#define DUGKS_F32 1     /* f~ in binary32, binary32 arithmetic, binary64 moment sums */
#define DUGKS_F16NEQ 2  /* phi in binary32 + g_i = s (f~_i - E_i(phi)) in binary16 for
                           i >= 1 (g_0 = -sum g_i); s a power of two chosen each step
                           from the previous step's max over i >= 1 of |f~_i - E_i|;
                           binary32 arithmetic */
#define DUGKS_BF16NEQ 3 /* as DUGKS_F16NEQ with bfloat16 and s = 1 (bfloat16 has the exponent
                           range of binary32) */

/* boundary kinds (per side: west, east, south, north) */
#define DUGKS_BC_PERIODIC 0
#define DUGKS_BC_DIRICHLET 1
#define DUGKS_BC_MIRROR 2

/* kernels */
#define DUGKS_KERNEL_FUSED 0 /* one fused kernel per step, column strips marched in y */
#define DUGKS_KERNEL_PLAIN 1 /* one cell per thread, neighbours read from global memory;
                                binary64 storage only */

/* launch schedules */
#define DUGKS_SCHED_GRID 0       /* one wave per work item */
#define DUGKS_SCHED_PERSISTENT 1 /* a fixed grid of waves striding over the work list */

/* diagnostic flags */
#define DUGKS_FLAG_NONFINITE 1
#define DUGKS_FLAG_OVERFLOW 2

typedef struct dugks_params {
  int abi_version; /* must be DUGKS_ABI_VERSION */
  int storage;     /* DUGKS_F64 / F32 / F16NEQ / BF16NEQ */
  int bc[4];       /* west, east, south, north; periodic sides come in pairs and
                      both walls of an axis are of one kind */
  int kernel;      /* DUGKS_KERNEL_FUSED or DUGKS_KERNEL_PLAIN */
  double c;        /* lattice speed, > 0 */
  double cfl;      /* CFL number, 0 < cfl < 1 (Sec. 2, Sec. 4) */
  double alpha;    /* diffusion coefficient of eq. 2.1, > 0 */
} dugks_params;

typedef struct dugks_info {
  double dt, h, lambda, cs2;
  double a1, b1, a2, b2, a3, b3; /* eqs. 2.21, 2.13, 2.22 */
  int nx, ny, q, storage, pitch;
  int eq_degree;          /* degree of E_i(phi) as a polynomial in phi */
  int rows_per_wave;      /* current launch configuration */
  int waves_per_block;
  int schedule;
  int xcd_remap;
  long long work_items;
  size_t state_bytes;     /* bytes of one f~ buffer (read once and written once per step) */
  long long graph_steps;  /* steps replayed from captured hipGraphs since dugks_bind */
  long long eager_steps;  /* steps launched one by one since dugks_bind */
  int xy_symmetric;       /* 1: E_i and E_j have bitwise the same coefficients for every pair
                             i, j whose velocities differ by swapping x and y (B_x = B_y,
                             D_xx = D_yy), in every instance of the context or batch; the
                             binary32 and 16-bit steps without a source then evaluate one
                             polynomial per pair (same values) */
} dugks_info;

typedef struct dugks_diag {
  long long step; /* steps taken since dugks_set_phi / dugks_set_f */
  double t;       /* step * dt */
  double dt;
  double mass;    /* sum_j phi_j |V_j| */
  double max_neq; /* max over i >= 1 of |f~_i - E_i(phi)| of the last step's output (16-bit
                     storage), else 0 */
  double scale;   /* power-of-two scale of the stored state (16-bit storage), else 1 */
  int flags;      /* DUGKS_FLAG_* */
} dugks_diag;

typedef struct dugks_ctx dugks_ctx;
typedef struct dugks_batch dugks_batch;

/* Create an instance on nx x ny cells with faces xf[0..nx], yf[0..ny]
 * (strictly increasing, host, copied) and q in {9, 5}.  No device work.
 * B = D = 0 until set.  Errors: E_ARG (sizes < 1, non-monotone faces, c,
 * cfl or alpha out of range, bad abi_version), E_UNSUPPORTED (q, storage,
 * kernel or boundary combination not built).  On an error other than a NULL
 * out, *out still receives a handle whose dugks_last_error() names the
 * problem; destroy it with dugks_destroy(). */
int dugks_create(dugks_ctx** out, int nx, int ny, const double* xf, const double* yf, int q,
                 const dugks_params* p);

/* Device workspace needed by the instance, in bytes. */
size_t dugks_workspace_bytes(const dugks_ctx* ctx);

/* Attach the caller's workspace (device pointer, >= dugks_workspace_bytes,
 * 256-byte aligned) and stream (hipStream_t as void*).  Uploads the mesh and
 * coefficient tables.  May be called again to move the instance; the state
 * is then undefined until set.  Errors: E_ARG, E_NOMEM, E_HIP. */
int dugks_bind(dugks_ctx* ctx, void* dev_workspace, size_t bytes, void* hip_stream);

/* B(phi) = sum_{k<=deg} (bx[k], by[k]) phi^k (host arrays of deg+1 values).
 * C = int_0^phi B'B'^T is formed by the library (Remark 3).  deg <= 4.
 * Call before dugks_set_phi.  Errors: E_ARG. */
int dugks_set_B(dugks_ctx* ctx, int deg, const double* bx, const double* by);

/* D(phi) = sum_{k<=deg} [[dxx[k], dxy[k]], [dxy[k], dyy[k]]] phi^k, deg <= 4.
 * With q = 5 only D = phi I is accepted (Remark 3).  Errors: E_ARG, E_UNSUPPORTED. */
int dugks_set_D(dugks_ctx* ctx, int deg, const double* dxx, const double* dxy, const double* dyy);

/* Source term F of eq. 2.1, F(x, t) = exp(gamma t) G(x), with G given at the
 * cell centres: g_dev is a device array [ny][nx] of binary64 values,
 * caller-owned, read by every later initialisation, step and read-out (keep it
 * alive and unchanged while the source is set); g_dev == NULL removes the
 * source.  Its distributions are F_i = w_i F (eq. 2.3) and, since
 * C = int B'B'^T, R_i = w_i c_i.B'(phi) F / c_s^2 (Remark 3); they enter
 * through the shifted distributions of eqs. 2.24-2.27, so that
 * phi = sum_i f~_i + dt F / 2.  F at a face is the linear interpolation of G
 * between the two cell centres (as eq. 2.20), at t_n + h (where fbar of eq.
 * 2.27 lives); a ghost cell takes the G of the cell whose distribution it
 * copies.  Set the source before dugks_set_phi: the initial f~ is
 * E(phi) - dt (F_i + R_i) / 2.  Same as dugks_set_source_terms with one term
 * of power 0.
 * Errors: E_UNSUPPORTED (16-bit storage or the plain kernel), E_ARG (gamma
 * not finite), E_HIP. */
int dugks_set_source(dugks_ctx* ctx, const double* g_dev, double gamma);

/* Source term F of eq. 2.1 depending on phi, as a sum of nterms <=
 * DUGKS_MAX_SRC_TERMS terms
 *     F(x, t, phi) = sum_j exp(gammas[j] t) phi^powers[j] G_j(x),
 * powers[j] in 0..DUGKS_MAX_SRC_POW, with the G_j given at the cell centres:
 * g_dev is a device array [nterms][ny][nx] of binary64 values, caller-owned
 * and kept alive and unchanged while the source is set; powers and gammas are
 * host arrays (copied).  nterms == 0 removes the source.  This covers Example
 * 4.2's k phi (1 - phi^delta) and Example 4.5's eq. 4.5.3.  Distributions,
 * face rule and initialisation are those of dugks_set_source with F at the
 * current phi; when some power is > 0 the conserved value is implicit (the
 * paper notes this after eq. 2.27): phi = sum f~ + dt F(phi) / 2 in a cell and
 * phi_b = sum fbar + h F_b(phi_b) / 2 at a face, each solved by Newton's method
 * from the explicit sum until the update is at most 1e-15 (1 + |phi|) in
 * binary64 (2.4e-7 in binary32), at most 8 (6) updates.  Errors: E_ARG
 * (nterms, a power out of range, a rate not finite, NULL arrays, more than
 * 4 GiB of G), E_UNSUPPORTED (16-bit storage or the plain kernel), E_HIP. */
int dugks_set_source_terms(dugks_ctx* ctx, int nterms, const double* g_dev, const int* powers,
                           const double* gammas);

/* Dirichlet data: ring_dev (device, caller-owned, must outlive the steps)
 * holds nsteps rings of 2(nx+ny)+4 binary64 values, phi at the ghost
 * centres at t_n = n dt for step n = 0..nsteps-1 counted from the last
 * dugks_set_phi / dugks_set_f.  Ring order: row j = -1 (i = -1..nx), row
 * j = ny (i = -1..nx), column i = -1 (j = 0..ny-1), column i = nx
 * (j = 0..ny-1).  Stepping past nsteps returns E_STATE.  Errors: E_ARG. */
int dugks_set_dirichlet(dugks_ctx* ctx, const double* ring_dev, int nsteps);

/* Initialise f~ = E(phi) (Sec. 4; with a source E(phi) - dt (F_i + R_i) / 2)
 * from phi [ny][nx] (binary64, host if on_device == 0, else device) and reset
 * step and time to 0.  Errors: E_STATE (not bound), E_HIP. */
int dugks_set_phi(dugks_ctx* ctx, const double* phi, int on_device);

/* Set f~ directly from [q][ny][nx] binary64 values (encoded to the storage
 * format) and reset step and time to 0. */
int dugks_set_f(dugks_ctx* ctx, const double* f, int on_device);

/* Advance nsteps >= 0 steps, asynchronously on the bound stream.  Runs of
 * four or more steps that start at a step divisible by 4 are replayed from
 * captured hipGraphs of 32 and 4 steps (captured on first use on a stream of
 * the library's own, launched on the bound stream after a one-thread kernel
 * that writes the run's first step index to the workspace, from which the
 * captured kernels take the time of their Dirichlet data and sources); the
 * rest, and every step of the plain kernel, are launched one by one.
 * dugks_info counts both kinds.  Errors: E_STATE (not initialised, Dirichlet
 * data exhausted), E_HIP. */
int dugks_step(dugks_ctx* ctx, int nsteps);

/* phi = sum_i f~_i (Sec. 2) accumulated in binary64 (with a source the root
 * of phi = sum_i f~_i + dt F(x, t, phi) / 2 at the current time), into
 * out [ny][nx] (host if on_device == 0, else device).  Synchronises. */
int dugks_get_phi(dugks_ctx* ctx, double* out, int on_device);

/* f~ decoded to binary64 [q][ny][nx].  Synchronises. */
int dugks_get_f(dugks_ctx* ctx, double* out, int on_device);

/* Step count, time, mass and flags; runs the device reductions and
 * synchronises.  Returns E_UNSTABLE (with *out filled) if a flag is set. */
int dugks_get_diag(dugks_ctx* ctx, dugks_diag* out);

/* GRE of eq. 4.1 (unweighted sums over cells) and the area-weighted relative
 * L2 error of phi against ref_dev [ny][nx] (device, binary64).  Binary64
 * reductions in a fixed order.  Synchronises.  Returns E_UNSTABLE, with both
 * norms NaN, when some cell's phi is not finite. */
int dugks_error_norms(dugks_ctx* ctx, const double* ref_dev, double* rel_l2, double* gre);

/* For callers that cannot allocate (code under hipGraph capture, tight
 * serving loops, harnesses that forbid allocation): the norms of
 * dugks_error_norms written to out_dev[0] = relative L2 and out_dev[1] = GRE
 * (device, binary64, caller-owned), asynchronously on the bound stream; no
 * synchronisation, no host copy and no allocation (no hipMalloc, hipFree or
 * allocating library routine).  The binary64 partial sums go to a static
 * array of the library, one per GPU, of 1024 x 8 doubles (64 KiB), held until
 * the process ends; its size does not depend on the grid, so no grid size is
 * refused for lack of room.  Every call on a GPU rewrites that array in full
 * before reading it: calls that overlap on one GPU (two streams, two threads)
 * race and must be ordered by the caller.  The sums are those of
 * dugks_error_norms in the same order; both norms are NaN when some cell's phi
 * is not finite.  Errors: E_ARG (NULL pointer), E_STATE
 * (no state), E_HIP (launch, or the scratch address lookup on first use on a
 * device). */
int dugks_error_norms_noalloc(dugks_ctx* ctx, const double* ref_dev, double* out_dev);

/* Serialise the state (header with ABI version, sizes, storage, step, time,
 * scale slots and a hash of mesh, parameters and coefficients, then the
 * active f~ buffer and a checksum) into host_buf.  With host_buf == NULL only
 * *len is set to the size needed.  Synchronises.  Errors: E_ARG (buffer too
 * small), E_STATE. */
int dugks_checkpoint(dugks_ctx* ctx, void* host_buf, size_t* len);

/* Restore a checkpoint taken from an instance with the same mesh,
 * parameters and coefficients.  Errors: E_FORMAT (bad magic, version, size,
 * hash or checksum), E_STATE (not bound). */
int dugks_restore(dugks_ctx* ctx, const void* host_buf, size_t len);

/* Launch configuration: rows_per_wave (rows each wave marches, 1..4096),
 * waves_per_block (1, 2 or 4; also 8 for binary32 and 16-bit storage without
 * a source, whose step kernel runs two waves per SIMD; setting a source later
 * turns an 8 into 4), schedule (DUGKS_SCHED_*), xcd_remap (0/1: map
 * consecutive work to one XCD's L2).  Results do not depend on it.
 * Errors: E_ARG. */
int dugks_set_launch(dugks_ctx* ctx, int rows_per_wave, int waves_per_block, int schedule,
                     int xcd_remap);

/* Time trial_steps steps for each candidate launch configuration and keep the
 * fastest.  Writes only the inactive buffer: the state is unchanged.  Every
 * trial step reads the Dirichlet data of the current step.  Synchronises.
 * Errors: E_STATE (no state, or Dirichlet data not covering the current
 * step), E_HIP. */
int dugks_autotune(dugks_ctx* ctx, int trial_steps);

/* Constants and the launch configuration in use. */
int dugks_get_info(const dugks_ctx* ctx, dugks_info* out);

/* ------------------------------------------------------------ batches
 * Many independent instances advanced by one launch per step (one work list
 * over all instances' column strips).  Every instance uses the batch's
 * storage and the fused kernel; Dirichlet walls are not built for batches. */
typedef struct dugks_instance_desc {
  int nx, ny, q;
  const double* xf; /* host, nx+1 faces, copied */
  const double* yf; /* host, ny+1 faces, copied */
  dugks_params p;   /* storage and kernel fields are ignored */
  int b_deg;
  double bx[DUGKS_MAX_DEG + 1], by[DUGKS_MAX_DEG + 1];
  int d_deg;
  double dxx[DUGKS_MAX_DEG + 1], dxy[DUGKS_MAX_DEG + 1], dyy[DUGKS_MAX_DEG + 1];
} dugks_instance_desc;

/* Create a batch of n >= 1 instances (desc host array, copied).  Errors as
 * dugks_create, per instance. */
int dugks_batch_create(dugks_batch** out, int n, const dugks_instance_desc* desc, int storage);
size_t dugks_batch_workspace_bytes(const dugks_batch* b);
int dugks_batch_bind(dugks_batch* b, void* dev_workspace, size_t bytes, void* hip_stream);
/* f~ = E(phi) for instance i (phi [ny_i][nx_i]).  The batch has one clock
 * (one step count, buffer parity and 16-bit scale phase for all instances):
 * instance i starts at step 0.  If the batch has stepped since its instances
 * were last set, every other instance then holds a state of another step and
 * is marked stale: stepping, autotuning and reading a stale instance return
 * E_STATE until each instance has been set again. */
int dugks_batch_set_phi(dugks_batch* b, int i, const double* phi, int on_device);
/* Source of instance i, as dugks_set_source (g_dev [ny_i][nx_i]).  A launch
 * over a batch in which some instance has a source evaluates the source path
 * for every instance; those without one read G = 0 and give the same result
 * as without it.  Errors: E_ARG (bad index), as dugks_set_source. */
int dugks_batch_set_source(dugks_batch* b, int i, const double* g_dev, double gamma);
/* Source terms of instance i, as dugks_set_source_terms (g_dev [nterms][ny_i][nx_i]). */
int dugks_batch_set_source_terms(dugks_batch* b, int i, int nterms, const double* g_dev,
                                 const int* powers, const double* gammas);
int dugks_batch_autotune(dugks_batch* b, int trial_steps);
int dugks_batch_set_launch(dugks_batch* b, int rows_per_wave, int waves_per_block, int schedule,
                           int xcd_remap);
/* Advance every instance nsteps steps (each with its own dt), replayed from
 * captured hipGraphs as dugks_step describes.  Errors: E_STATE (an instance
 * without a state at the batch clock), E_HIP. */
int dugks_batch_step(dugks_batch* b, int nsteps);
int dugks_batch_get_phi(dugks_batch* b, int i, double* out, int on_device);
int dugks_batch_get_info(const dugks_batch* b, int i, dugks_info* out);
/* Total cells of all instances and bytes of one f~ buffer over all instances. */
int dugks_batch_totals(const dugks_batch* b, long long* cells, size_t* state_bytes);
/* Advance every instance nsteps steps like dugks_batch_step, with hipEvents
 * recorded on the bound stream before the first and after the last launch;
 * synchronises and returns the elapsed time in *ms_total. */
int dugks_batch_time_steps(dugks_batch* b, int nsteps, float* ms_total);

/* Single-instance counterpart of dugks_batch_time_steps. */
int dugks_time_steps(dugks_ctx* ctx, int nsteps, float* ms_total);

/* Message of the last failure on this handle (dugks_ctx* or dugks_batch*),
 * owned by the handle; "" if none. */
const char* dugks_last_error(const void* handle);

/* Free a dugks_ctx* or dugks_batch* (not the caller's workspace). */
void dugks_destroy(void* handle);

#ifdef __cplusplus
}
#endif

#endif /* DUGKS_H */
