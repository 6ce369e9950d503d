/*
 * libdugks, three-dimensional path: the DUGKS time step of Sec. 2 of
 * Shang, Chai, Wang, Shi, "Discrete unified gas kinetic scheme for nonlinear
 * convection-diffusion equations" (arXiv 1906.11036) on the D3Q15 (eq. 2.28),
 * D3Q19 (eq. 2.6) and D3Q7 (Remark 3) lattices, on a Cartesian mesh of
 * nx x ny x nz cells with strictly increasing face coordinates per axis.
 *
 * Same conventions as dugks.h: C ABI, every call returns an int code of
 * dugks.h (DUGKS_OK = 0, negative on error), dugks3_last_error() names the
 * problem.  The caller owns the device workspace (dugks3_workspace_bytes,
 * 256-byte aligned) and the stream; the library owns only its host handle.
 * Stepping is asynchronous on the bound stream; read-outs synchronise.
 *
 * Readings (as in the CPU oracle): lambda = alpha / c_s^2, c_s^2 = c^2/3;
 * dt = cfl * (smallest cell width along any axis) / c; C = int_0^phi B'B'^T
 * (Remark 3); each tangential derivative at a face is the mean of the two
 * cells' central differences along that axis; walls per axis are periodic,
 * zero-flux mirrors (fbar+ of the adjacent cell with the wall-normal velocity
 * reversed) or Dirichlet by non-equilibrium extrapolation, the treatment of
 * Sec. 4 (a ghost with a Dirichlet wall on any of its out-of-range axes takes
 * fbar+_g = E(phi_g) + fbar+_a - E(phi_a), a the nearest interior cell);
 * D3Q7 uses weights 0 and 1/6 and the linear equilibrium of Remark 3
 * (D = phi I only).  Sources F(x, t, phi) as in two dimensions
 * (dugks3_set_source_terms) run in the fused step.
 */
#ifndef DUGKS3D_H
#define DUGKS3D_H

#include <stddef.h>

#include "dugks.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DUGKS3_ABI_VERSION 1

typedef struct dugks3_params {
  int abi_version; /* must be DUGKS3_ABI_VERSION */
  int storage;     /* DUGKS_F64 or DUGKS_F32 */
  int bc[3];       /* per axis x, y, z: DUGKS_BC_PERIODIC, DUGKS_BC_MIRROR or
                      DUGKS_BC_DIRICHLET (data from dugks3_set_dirichlet) */
  double c;        /* lattice speed, > 0 */
  double cfl;      /* CFL number, 0 < cfl < 1 */
  double alpha;    /* diffusion coefficient of eq. 2.1, > 0 */
} dugks3_params;

typedef struct dugks3_info {
  double dt, h, lambda, cs2;
  double a1, b1, a2, b2, a3, b3;
  int nx, ny, nz, q, storage, pitch;
  int eq_degree;          /* degree of E_i(phi) as a polynomial in phi */
  int rows_per_block;     /* launch: rows of a block (see dugks3_set_launch) */
  int planes_per_block;   /* launch: planes swept by a block */
  long long blocks;       /* blocks per step */
  size_t state_bytes;     /* bytes of one f~ buffer */
} dugks3_info;

typedef struct dugks3_ctx dugks3_ctx;

/* Create an instance on nx x ny x nz cells with faces xf[0..nx], yf[0..ny],
 * zf[0..nz] (host, copied) and q in {15, 19, 7}.  No device work; B = D = 0
 * until set.  Errors: E_ARG (sizes, faces, c, cfl, alpha, abi_version),
 * E_UNSUPPORTED (q, storage, boundary kind).  On an error other than a NULL
 * out, *out still receives a handle for dugks3_last_error / dugks3_destroy. */
int dugks3_create(dugks3_ctx** out, int nx, int ny, int nz, const double* xf, const double* yf,
                  const double* zf, int q, const dugks3_params* p);

/* Device workspace needed, in bytes. */
size_t dugks3_workspace_bytes(const dugks3_ctx* ctx);

/* Attach the caller's workspace (device, >= dugks3_workspace_bytes, 256-byte
 * aligned) and stream (hipStream_t as void*); uploads the tables.  Errors:
 * E_ARG, E_NOMEM, E_HIP. */
int dugks3_bind(dugks3_ctx* ctx, void* dev_workspace, size_t bytes, void* hip_stream);

/* B(phi) = sum_{k<=deg} (b[k], b[deg+1+k], b[2(deg+1)+k]) phi^k (host, 3(deg+1)
 * values: the x, then y, then z coefficients), deg <= 4.  Errors: E_ARG. */
int dugks3_set_B(dugks3_ctx* ctx, int deg, const double* b);

/* D(phi) = sum_{k<=deg} D_k phi^k, symmetric, given as six runs of deg+1
 * coefficients: xx, yy, zz, xy, xz, yz (host), deg <= 4.  q = 7 accepts only
 * D = phi I.  Errors: E_ARG, E_UNSUPPORTED. */
int dugks3_set_D(dugks3_ctx* ctx, int deg, const double* d);

/* f~ = E(phi) (Sec. 4) from phi [nz][ny][nx] (binary64; host if on_device == 0);
 * resets the step count.  Errors: E_STATE (not bound), E_ARG, E_HIP. */
int dugks3_set_phi(dugks3_ctx* ctx, const double* phi, int on_device);

/* f~ [q][nz][ny][nx] (binary64) as the state; resets the step count. */
int dugks3_set_f(dugks3_ctx* ctx, const double* f, int on_device);

/* Bytes of scratch the source path needs: 0 (every lattice takes the source
 * in the fused step; kept for callers that size a scratch array). */
size_t dugks3_source_scratch_bytes(const dugks3_ctx* ctx);

/* Source F(x, t, phi) = sum_{j < nterms} exp(gammas[j] t) phi^powers[j] G_j(x)
 * of eq. 2.1, with F_i = w_i F and R_i = w_i c_i.B'(phi) F / c_s^2 (eq. 2.3,
 * Remark 3) in eqs. 2.25 and 2.27, as dugks_set_source_terms: g_dev (device,
 * binary64, caller-owned, must outlive the steps) holds nterms shapes of
 * [nz][ny][nx]; powers in 0..DUGKS_MAX_SRC_POW; nterms <= DUGKS_MAX_SRC_TERMS
 * (0 removes the source).  The conserved value solves phi = sum f~ +
 * dt F(phi) / 2 in a cell at t_n and phi_b = sum fbar + h F(phi_b) / 2 at a
 * face at t_n + h (each G_j interpolated between the two centres; a ghost
 * takes the G_j of the cell it copies), by Newton's method when F depends on
 * phi (binary64: update <= 1e-15 (1 + |phi|), at most 8; binary32: 2.4e-7,
 * at most 6).  Set before dugks3_set_phi (f~ = E(phi) - dt S / 2 at t = 0).
 * The step takes the source in the fused kernel; scratch_dev and
 * scratch_bytes are not used (may be NULL and 0).  Errors: E_ARG (nterms, a
 * power out of range, a rate not finite, NULL arrays). */
int dugks3_set_source_terms(dugks3_ctx* ctx, int nterms, const double* g_dev, const int* powers,
                            const double* gammas, void* scratch_dev, size_t scratch_bytes);

/* Dirichlet data: ring_dev (device, caller-owned, must outlive the steps)
 * holds nsteps blocks of shell-length binary64 values, phi at the ghost-cell
 * centres at t_n = n dt for step n = 0..nsteps-1 counted from the last
 * dugks3_set_phi / dugks3_set_f.  Shell length 2(nx+2)(ny+2) + 2(nx+2)nz +
 * 2 ny nz, in the order: the z = -1 and z = nz planes (each [ny+2][nx+2], j
 * and i from -1), the y = -1 and y = ny slabs (each [nz][nx+2], i from -1),
 * the x = -1 and x = nx columns (each [nz][ny]).  A ghost centre lies half
 * the adjacent interior cell's width outside the wall (half the wrapped
 * cell's width along a periodic axis); values read: the ghosts with a
 * Dirichlet wall on one of their out-of-range axes.  Stepping with a
 * Dirichlet axis past nsteps (or without data) returns E_STATE.  Errors:
 * E_ARG (nsteps < 0, NULL data with nsteps > 0). */
int dugks3_set_dirichlet(dugks3_ctx* ctx, const double* ring_dev, int nsteps);

/* Advance nsteps >= 0 steps (asynchronous).  Errors: E_STATE, E_HIP. */
int dugks3_step(dugks3_ctx* ctx, int nsteps);

/* phi = sum_i f~_i [nz][ny][nx] and f~ [q][nz][ny][nx], binary64 (host if
 * on_device == 0).  Synchronise. */
int dugks3_get_phi(dugks3_ctx* ctx, double* out, int on_device);
int dugks3_get_f(dugks3_ctx* ctx, double* out, int on_device);

/* mass = sum phi |V|; with ref (device, [nz][ny][nx], or NULL) also the GRE of
 * eq. 4.1 (unweighted) and the volume-weighted relative L2 difference.  Any
 * output pointer may be NULL.  Synchronises.  A non-finite cell returns
 * E_UNSTABLE. */
int dugks3_reduce(dugks3_ctx* ctx, const double* ref_dev, double* mass, double* gre,
                  double* rel_l2);

/* Launch configuration: rows per block and planes swept per block (>= 1).
 * binary32: 2 to 4 rows; binary64: 1 or 2 rows.  D3Q15 and D3Q19 give each
 * row two or four waves, each holding a part of the directions: four for
 * D3Q19 in binary32 at 3 or 4 rows and in binary64 at 2 rows, and for D3Q15
 * the same on periodic meshes; two otherwise.  LDS per block: g of 3 planes
 * of the rows and the two halo rows, raw f~ of 1 or 2 staged planes (of the
 * rows and the halo rows with two waves a row; of the rows only with four,
 * whose halo rows go through registers), 4 face sums per row and wave, and
 * with the halo rows in registers their four quarter sums of phi (2 x 4 x 64
 * binary64).  Binary32 takes one staging slot where that alone brings a
 * block within 80 KiB (two blocks a CU), else two; binary64 one.  D3Q7
 * gives each row one wave (binary32: 5 x (rows + 2) x q x 64 x 4
 * bytes of LDS; binary64: one more wave per halo row, 3 x (rows + 2) x q x
 * 64 x 8 bytes).  A launch needing more LDS than the device allows per block
 * is refused.  With a source the step takes the split-direction kernel's
 * instantiation with mirror code for every mesh and lattice (D3Q7 then with
 * two waves a row).  Defaults, with a source or without: 2 rows (binary64),
 * 4 rows (binary32; D3Q15 with walls: 2); planes: D3Q15 and D3Q19 the power
 * of two in 4..128 that
 * minimises (rounds of blocks over 256 CUs) x (planes + 3), D3Q7 32 halved
 * down to 4 while the grid would have fewer than 512 blocks.  Every launch
 * gives bitwise the same result.
 * Errors: E_ARG. */
int dugks3_set_launch(dugks3_ctx* ctx, int rows_per_block, int planes_per_block);

/* Time nsteps steps with hipEvents on the bound stream (the state advances). */
int dugks3_time_steps(dugks3_ctx* ctx, int nsteps, float* ms_total);

/* Time trial_steps steps (at least 1, after one untimed step) for every
 * valid launch shape (rows per block in the storage's range, planes per
 * block 4, 8, ..., 128, within the LDS limit) and keep the fastest.  Trial
 * steps read the current state and the current step's Dirichlet data and
 * write only the inactive buffer: the state and the step count are
 * unchanged, and since every launch gives bitwise the same result, so is
 * every later step.  Synchronises.  Errors: E_STATE (not bound, no
 * state, Dirichlet data not covering the current step), E_HIP. */
int dugks3_autotune(dugks3_ctx* ctx, int trial_steps);

int dugks3_get_info(const dugks3_ctx* ctx, dugks3_info* out);

/* ------------------------------------------------------------------ batches
 * Many D3Q15 or D3Q19 instances (one lattice, one storage; sizes, meshes,
 * walls and coefficients their own) advanced by one launch per step, as the
 * two-dimensional batch: each instance keeps its context (created, set up,
 * bound and given its state as usual; caller-owned, kept bound to the same
 * workspace while in the batch), and the batch's launch covers the blocks of
 * all of them (rows and planes per block shared; the instantiation for the
 * largest coefficient count, with mirror code if any instance has a wall).
 * D3Q19 instances get bitwise what they get alone; D3Q15 ones the same up to
 * the order of the face sums when a walled batch holds periodic instances
 * (the walled instantiation splits the directions in two parts, the periodic
 * one in four).  Sources are not batched (E_UNSUPPORTED at the step).
 * Create: E_ARG (n < 1, an invalid context, a mix of lattices or storages),
 * E_UNSUPPORTED (D3Q7). */
typedef struct dugks3_batch dugks3_batch;
int dugks3_batch_create(dugks3_batch** out, int n, dugks3_ctx* const* ctxs);
/* Device bytes of the batch's table (instance pointers and block offsets). */
size_t dugks3_batch_workspace_bytes(const dugks3_batch* b);
/* Workspace (device, 256-byte aligned) and stream; every instance must be
 * bound.  Errors: E_ARG, E_NOMEM, E_STATE, E_HIP. */
int dugks3_batch_bind(dugks3_batch* b, void* dev_workspace, size_t bytes, void* hip_stream);
/* Rows and planes per block for the batch's launch (ranges as
 * dugks3_set_launch; defaults 2 rows binary64, 4 binary32, 32 planes). */
int dugks3_batch_set_launch(dugks3_batch* b, int rows_per_block, int planes_per_block);
/* nsteps steps of every instance, one launch each; the instances must be at
 * the same step count, with Dirichlet data covering the steps (E_STATE) and
 * no source (E_UNSUPPORTED).  Asynchronous; each context's step count
 * advances. */
int dugks3_batch_step(dugks3_batch* b, int nsteps);
/* dugks3_batch_step timed with hipEvents on the batch's stream. */
int dugks3_batch_time_steps(dugks3_batch* b, int nsteps, float* ms_total);
/* The launch shape, the grid's blocks and the cells of all instances (any
 * pointer may be NULL). */
int dugks3_batch_get_info(const dugks3_batch* b, int* rows_per_block, int* planes_per_block,
                          long long* blocks, long long* cells);
const char* dugks3_batch_last_error(const dugks3_batch* b);
void dugks3_batch_destroy(dugks3_batch* b);
const char* dugks3_last_error(const dugks3_ctx* ctx);
void dugks3_destroy(dugks3_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DUGKS3D_H */
