// Internal layout shared by the host runtime and the gfx950 kernels of libdugks.
//
// One f~ buffer of an instance is a set of planes [P][ny][pitch]; pitch is nx
// rounded up to 64 elements so every row starts on a 128-byte boundary.
//   DUGKS_F64   : P = q planes of double
//   DUGKS_F32   : P = q planes of float
//   16-bit neq  : plane 0 = phi (float, 4-byte elements), planes 1..q-1 = g_i
//                 (2-byte elements, g_0 = -sum g_i is not stored)
// Two buffers per instance (ping-pong): step n reads buffer n%2, writes the other.
#pragma once

#include <stdint.h>

#include "dugks.h"

namespace dugks {

constexpr int kMaxQ = 9;
constexpr int kMaxCoef = 8;     // E_i(phi) has degree <= 7 (C has degree 2*4-1)
constexpr int kStripLanes = 64; // one wave covers 64 columns ...
constexpr int kStripCols = 62;  // ... of which 62 are updated; lanes 0 and 63 are halo
constexpr int kGeo = 5;
constexpr int kRhoCoef = 4;     // B'(phi) has degree <= 3
constexpr int kMaxSrcTerms = DUGKS_MAX_SRC_TERMS;
constexpr int kSrcPow = 4;      // a source term carries phi^k, k <= 3

// Per-instance constants and pointers, read by the kernels with scalar loads.
//
// The step works with scaled distributions so that one set of polynomial
// coefficients (those of E_i) serves the cell and the face:
//   g = fbar+ / b1 = (a1/b1) f~ + E(phi)                       (eq. 2.21 over b1)
//   f~+ = (4/3) b1 g - f~ / 3                                  (eq. 2.23)
//   phi_b = b1 sum_i gbar_i                                    (gbar = face value of g)
//   F = f_b / b3 = (a3 b1 / b3) gbar + E(phi_b)                (eq. 2.22 over b3)
// and the update factor of each column / row carries the b3 back.
//
// With a source F(x, t, phi) = sum_j exp(gamma_j t) phi^k_j G_j(x) (eq. 2.1's F,
// k_j <= 3) its distributions are S_i = F_i + R_i = F rho_i(phi),
// rho_i = w_i (1 + c_i.B'(phi) / c_s^2) (eq. 2.3, Remark 3), evaluated as
// w_i (1 + e_xi bp_x(phi) + e_yi bp_y(phi)) with e_i the integer lattice
// directions and bp = c B' / c_s^2; eqs. 2.25 / 2.27 add lambda S to g and to F:
//   phi = sum f~ + dt F(phi) / 2,  g += lambda F rho(phi),
//   phi_b = b1 sum gbar + h F_b(phi_b) / 2,  F += lambda F_b rho(phi_b),
// with F_b built from each G_j interpolated linearly between the two centres,
// at t + h.  When some k_j > 0 both relations are implicit and are solved by
// Newton's method.
struct alignas(64) InstDev {
  void* buf[2];            // ping-pong f~ buffers
  const double* colgeo;    // (nx+2) x kGeo doubles, column c = -1..nx at [(c+1)*kGeo]
  const double* rowgeo;    // (ny+2) x kGeo doubles, row r = -1..ny
  const float* colgeo_f;   // float copies
  const float* rowgeo_f;
  const double* ring;      // Dirichlet data, ring_steps x ring_len (or null)
  float* slots;            // 16-bit storage: 4 max|f~ - E| slots (unscaled)
  unsigned* flags;         // DUGKS_FLAG_* bits, sticky
  long long plane;         // elements per plane = ny * pitch
  unsigned buf_bytes;      // bytes of one buffer (< 4 GiB, the buffer resource range)
  int nx, ny, pitch, q;
  int bcx, bcy;            // DUGKS_BC_* per axis
  int ring_len, ring_steps;
  int ncoef;               // number of used polynomial coefficients (degree + 1)
  int storage;
  double ra, rb, b1, inv_b1, kg, a2, opra;     // a1/b1, a3 b1/b3, b1, 1/b1, 4/3 b1, a2, 1 + a1/b1
  float raf, rbf, b1f, inv_b1f, kgf, a2f, oepraf, a1f;
  // 16-bit storage holds g / (1 + ra) in registers: ra/(1+ra), b1 (1+ra), rb (1+ra), 1/(b1 (1+ra))
  float ra_of, b1_of, rb_of, inv_b1_of;
  // E_i(phi) = sum_k e[i][k] phi^k  (eq. 2.3 with C = int_0^phi B'B'^T)
  double e[kMaxQ][kMaxCoef];
  float ef[kMaxQ][kMaxCoef];
  // source (src_n == 0: none); G_j as [src_n][ny][nx] binary64, caller-owned
  const double* src_g;
  unsigned src_bytes;       // src_n * nx * ny * 8
  unsigned src_plane;       // nx * ny * 8: bytes of one G_j
  int src_n;                // number of terms
  int src_implicit;         // some term depends on phi
  int src_pow[kMaxSrcTerms];
  double src_gam[kMaxSrcTerms];
  double dt, lambda, half_dt, half_h;
  float lambdaf, half_dtf, half_hf;
  double bp[2][kRhoCoef];    // c B'_x / c_s^2 and c B'_y / c_s^2 as polynomials in phi
  float bpf[2][kRhoCoef];
};

// One unit of work: instance, first interior column of the strip, row range.
struct WorkItem {
  int inst, x0, y0, y1;
};

// Launch configuration.
struct Launch {
  int rows_per_wave = 16;
  int waves_per_block = 2;
  int schedule = DUGKS_SCHED_GRID;
  int xcd_remap = 1;
};

// Kernel entry points (dugks_kernels.hip), all enqueued on `stream`; each
// returns 0 or -1 when the launch failed.
struct StepArgs {
  const InstDev* insts;     // device table
  const WorkItem* items;    // device work list
  int nitems;
  int parity;               // index of the buffer read by this step
  long long step;           // step index of the input state
  int q, storage, ncoef;    // template selectors, uniform over the launch
  int src;                  // 0: no source; 1: one phi-free term each; kSrcPow: otherwise
  int sym;                  // every instance x<->y symmetric (E_k = E_swap(k) bitwise)
  int persistent_blocks;    // blocks of the persistent schedule
  // when set, the step index is step + *step_base (captured graphs: step is the
  // offset within the graph, the base is written before each replay)
  const long long* step_base = nullptr;
};

int launch_step_fused(const StepArgs& a, const Launch& l, void* stream, int measure);
int launch_step_plain(const StepArgs& a, int nx, int ny, void* stream);
// zero slots[(step + which) & 3] of every instance
int launch_clear_slot(const InstDev* insts, int ninst, long long step, int which, void* stream);
int launch_init_eq(const InstDev* d, const InstDev& h, const double* phi, int parity, void* stream);
// pass 0: max |f~ - E| into slots[slot]; pass 1: encode f~ with that slot's scale
int launch_set_f_pass(const InstDev* d, const InstDev& h, const double* f, int parity, int pass,
                      int slot, void* stream);
// phi at step `step` (the source term, if any, is evaluated at t = step dt)
int launch_get_phi(const InstDev* d, const InstDev& h, double* out, int parity, long long step,
                   void* stream);
int launch_get_f(const InstDev* d, const InstDev& h, double* out, int parity, long long step,
                 void* stream);
// Sums over cells into out[0..7] (device): [0] mass, [1] sum|phi-ref|, [2] sum|ref|,
// [3] sum (phi-ref)^2 |V|, [4] sum ref^2 |V|, [5] non-finite cells.  partial
// holds reduce_partials() * 8 doubles; widths = dx[0..nx) then dy[0..ny).
int launch_reduce_widths(const InstDev* d, const InstDev& h, const double* ref, int parity,
                         long long step, const double* widths, double* partial, double* out,
                         void* stream);
int reduce_partials();
// Relative L2 and GRE of the instance's phi against ref into out_dev[0..1]
// (device), with the partial sums in the library's static per-GPU scratch
// (no allocation, no synchronisation).  Returns 0, -1 (launch failed) or -2
// (scratch address lookup failed).
int launch_norms_noalloc(const InstDev* d, const InstDev& h, const double* ref, int parity,
                         long long step, const double* widths, double* out_dev, void* stream);
int launch_fill_u32(unsigned* p, unsigned v, long long n, void* stream);
int launch_set_i64(long long* p, long long v, void* stream);

// Power-of-two scale of the 16-bit formats for a maximum |f~ - E| of m.
float neq_scale_host(int storage, float m);

}  // namespace dugks
