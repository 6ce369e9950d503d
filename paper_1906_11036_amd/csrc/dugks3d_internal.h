// Internal layout shared by the host runtime and the gfx950 kernels of the
// three-dimensional DUGKS step (D3Q15 of eq. 2.28, D3Q19 of eq. 2.6, D3Q7 of
// Remark 3).
//
// One f~ buffer is Q direction planes, each [nz][ny][pitch] with pitch = nx
// rounded up to 64 elements.  Two buffers (ping-pong): step n reads buffer
// n%2.  Storage binary64 or binary32.
#pragma once

#include <stdint.h>

#include "dugks.h"
#include "dugks3d.h"

namespace dugks3 {

constexpr int kMaxQ = 19;
constexpr int kMaxCoef = 8;     // E_i(phi) has degree <= 7
constexpr int kLanes = 64;      // one wave covers 64 columns ...
constexpr int kCols = 62;       // ... of which 62 are updated; lanes 0 and 63 are halo
constexpr int kGeo = 5;         // per face: 3 reconstruction factors, tangential factor, update factor
// rows of a block: binary32 2..4 (one wave per row, the halo rows staged by
// all waves); binary64 1..2 interior rows plus one wave per halo row
constexpr int kMinRows32 = 2, kMaxRows32 = 4;
constexpr int kMinRows64 = 1, kMaxRows64 = 2;

// Per-instance constants and pointers (kernels read them with scalar loads).
// Scaled distributions as in the two-dimensional kernels:
//   g = fbar+ / b1 = (a1/b1) f~ + E(phi)      f~+ = (4/3) b1 g - f~ / 3
//   phi_b = b1 sum gbar                       F = f_b / b3 = (a3 b1/b3) gbar + E(phi_b)
// Axis tables: for axis a, face between cells m-1 and m at [(m+1)*kGeo + 0..2]
// (factors for normal velocity -c, 0, +c), at [(m+1)*kGeo + 3] the tangential
// factor h c / (2 (x_{m+1} - x_{m-1})) of cell m and at [(m+1)*kGeo + 4] the
// update factor dt c b3 / width of cell m.
struct alignas(64) Inst3 {
  void* buf[2];
  const double* geo[3];
  const float* geof[3];
  long long plane;         // elements per direction plane: nz * ny * pitch
  unsigned buf_bytes;      // bytes of one buffer (< 4 GiB)
  int n[3];
  int pitch, q;
  int bc[3];               // DUGKS_BC_PERIODIC, DUGKS_BC_DIRICHLET or DUGKS_BC_MIRROR per axis
  int ncoef, storage;
  double ra, rb, b1, kg, inv_b1;
  float raf, rbf, b1f, kgf, inv_b1f;
  // Dirichlet data (caller-owned, binary64): step n reads ring + n * ring_len,
  // phi at the ghost-shell centres (order: see shell_index)
  const double* ring;
  long long ring_len;
  double e[kMaxQ][kMaxCoef];   // E_i(phi) = sum_k e[i][k] phi^k (eq. 2.3)
  float ef[kMaxQ][kMaxCoef];
  // sources (src_n = 0: none): F(x, t, phi) = sum_j exp(src_gam[j] t)
  // phi^src_pow[j] G_j(x), G_j as [src_n][nz][ny][nx] binary64 (caller-owned)
  const double* src_g;
  long long src_plane;     // nx * ny * nz
  int src_n, src_implicit; // implicit: some term depends on phi
  int src_pow[DUGKS_MAX_SRC_TERMS];
  double src_gam[DUGKS_MAX_SRC_TERMS];
  double dt, lambda;
  double bp[3][4];         // c B'_a(phi) / c_s^2 as polynomials in phi (B' has degree <= 3)
};

// A batch of instances stepped by one launch: instance k takes blocks
// first[k] .. first[k+1] - 1 (after the XCD remap) with its own strips, tiles
// and plane chunks; insts == nullptr: one instance (the kernel's arguments).
struct Batch3 {
  const Inst3* const* insts;
  const long long* first;
  int n;
  long long step;   // the step index (selects each instance's Dirichlet data)
};

struct Launch3 {
  int rows = 4;     // rows per block (see kMinRows32 .. kMaxRows64)
  int planes = 64;  // planes swept per block
};

// Position of ghost cell (i, j, k) (one index out of its range -1..n) in one
// step's Dirichlet data: the z = -1 and z = nz planes ([ny+2][nx+2], j and i
// from -1), the y = -1 and y = ny slabs ([nz][nx+2]), then the x = -1 and
// x = nx columns ([nz][ny]).
__host__ __device__ inline long long shell_index(int nx, int ny, int nz, int i, int j, int k) {
  const long long zplane = (long long)(nx + 2) * (ny + 2), yslab = (long long)(nx + 2) * nz;
  if (k < 0) return (long long)(j + 1) * (nx + 2) + (i + 1);
  if (k >= nz) return zplane + (long long)(j + 1) * (nx + 2) + (i + 1);
  if (j < 0) return 2 * zplane + (long long)k * (nx + 2) + (i + 1);
  if (j >= ny) return 2 * zplane + yslab + (long long)k * (nx + 2) + (i + 1);
  if (i < 0) return 2 * zplane + 2 * yslab + (long long)k * ny + j;
  return 2 * zplane + 2 * yslab + (long long)ny * nz + (long long)k * ny + j;
}
inline long long shell_len(int nx, int ny, int nz) {
  return 2LL * (nx + 2) * (ny + 2) + 2LL * (nx + 2) * nz + 2LL * ny * nz;
}

// Blocks of one step for the launch (x strips x row tiles x plane chunks).
long long step3_blocks(const Inst3& h, const Launch3& l);
// step: the step index since the state was set (selects the Dirichlet data)
int launch_step3(const Inst3* d, const Inst3& h, int parity, long long step, const Launch3& l, void* stream);
// one step of a batch (D3Q15 / D3Q19, no source): ncoef the largest of the
// instances, walls whether any has a wall (the instantiation with mirror
// code then runs them all), blocks the grid (first[n] of the table)
int launch_step3_batch(const Batch3& bt, const Inst3& h, int parity, bool walls, long long blocks,
                       const Launch3& l, void* stream);
// LDS bytes of one block of the step kernel (walls: the instantiation with
// mirror code, for a non-periodic axis or more than four coefficients)
// src: the source instantiation (D3Q7 then runs the staged kernel too)
size_t step3_lds_bytes(int storage, int q, bool walls, const Launch3& l, bool src = false);
int launch_init3(const Inst3* d, const Inst3& h, const double* phi, int parity, void* stream);
int launch_set_f3(const Inst3* d, const Inst3& h, const double* f, int parity, void* stream);
int launch_get_phi3(const Inst3* d, const Inst3& h, double* out, int parity, long long step, void* stream);
int launch_get_f3(const Inst3* d, const Inst3& h, double* out, int parity, void* stream);
// out[0] mass, [1] sum|phi-ref|, [2] sum|ref|, [3] sum (phi-ref)^2 |V|, [4] sum ref^2 |V|,
// [5] non-finite cells; widths = dx[0..nx) dy[0..ny) dz[0..nz); partial holds
// reduce3_partials() * 8 doubles.
int launch_reduce3(const Inst3* d, const Inst3& h, const double* ref, int parity, long long step,
                   const double* widths, double* partial, double* out, void* stream);
int reduce3_partials();

}  // namespace dugks3
