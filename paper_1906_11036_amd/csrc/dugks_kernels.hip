// gfx950 kernels of libdugks: the DUGKS step (summary at the end of Sec. 2 of
// Shang, Chai, Wang, Shi, arXiv:1906.11036) for D2Q9 / D2Q5, plus the
// initialisation, encode/decode and reduction kernels around it.
//
// Fused step design (one wave = one work item):
//   - A wave owns a strip of 64 consecutive columns (lanes), of which lanes
//     1..62 are updated and lanes 0 and 63 are halo columns; it marches down a
//     chunk of rows.  f~ is read once per row per lane (coalesced 256-byte rows
//     per plane) and the new f~ is written once: the state crosses HBM once in
//     each direction per step, halo columns and the two halo rows per chunk
//     aside.
//   - fbar+ of three rows (j-1, j, j+1) lives in registers.  Neighbouring
//     columns are reached with whole-wave DPP shifts (wave_shr:1 / wave_shl:1),
//     so no LDS and no barrier is used.
//   - Each lane computes exactly two faces per row: the face on its west side
//     and the face above its cell.  The east face comes from the lane to the
//     right; the face below was computed on the previous row.
//   - Moment sums: the cell phi of the binary64 and binary32 storages and the
//     stored phi of the new state in the 16-bit formats are accumulated in
//     binary64 and rounded once; the interface phi is a binary64 sum in
//     binary64 storage and a balanced binary32 tree sum otherwise (binary64
//     when DUGKS_FACE_SUM64 is set).  Everything else runs in the storage's
//     arithmetic type.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "dugks_internal.h"

namespace dugks {

// Rows loaded ahead of the row being consumed by the step kernel.  A row of
// the 16-bit formats is small (20 bytes a cell for D2Q9), so two rows stay in
// flight to keep enough bytes outstanding per wave; the wider formats keep one.
#ifndef DUGKS_PREFETCH
#define DUGKS_PREFETCH 1
#endif
#ifndef DUGKS_PREFETCH_NEQ
#define DUGKS_PREFETCH_NEQ 2
#endif

// ------------------------------------------------------------------ lattice
// D2Q9 of eq. 2.5 (integer components; velocities are c times these).
__host__ __device__ constexpr int lat_cx(int k) {
  return (k == 1 || k == 5 || k == 8) ? 1 : ((k == 3 || k == 6 || k == 7) ? -1 : 0);
}
__host__ __device__ constexpr int lat_cy(int k) {
  return (k == 2 || k == 5 || k == 6) ? 1 : ((k == 4 || k == 7 || k == 8) ? -1 : 0);
}
// lattice weights: D2Q9 4/9, 1/9 (x4), 1/36 (x4); D2Q5 1/3, 1/6 (x4)
template <int Q> __host__ __device__ constexpr double lat_w(int k) {
  return Q == 9 ? (k == 0 ? 4.0 / 9.0 : (k <= 4 ? 1.0 / 9.0 : 1.0 / 36.0)) : (k == 0 ? 1.0 / 3.0 : 1.0 / 6.0);
}
// reversal of the x (resp. y) component: the specular mirror of a wall
__host__ __device__ constexpr int mir_x(int k) {
  return k == 1 ? 3 : k == 3 ? 1 : k == 5 ? 6 : k == 6 ? 5 : k == 7 ? 8 : k == 8 ? 7 : k;
}
__host__ __device__ constexpr int mir_y(int k) {
  return k == 2 ? 4 : k == 4 ? 2 : k == 5 ? 8 : k == 8 ? 5 : k == 6 ? 7 : k == 7 ? 6 : k;
}

// ---------------------------------------------------------- storage traits
template <int ST> struct Stor;
template <> struct Stor<DUGKS_F64> { using T = double; static constexpr bool neq = false; };
template <> struct Stor<DUGKS_F32> { using T = float; static constexpr bool neq = false; };
template <> struct Stor<DUGKS_F16NEQ> { using T = float; static constexpr bool neq = true; };
template <> struct Stor<DUGKS_BF16NEQ> { using T = float; static constexpr bool neq = true; };

__device__ __forceinline__ float bf16_to_f32(uint16_t u) {
  return __uint_as_float(((uint32_t)u) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {  // round to nearest even
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ float h16_to_f32(uint16_t u) {
  return (float)__builtin_bit_cast(_Float16, u);
}
__device__ __forceinline__ uint16_t f32_to_h16(float x) {  // round to nearest even
  return __builtin_bit_cast(uint16_t, (_Float16)x);
}

template <int ST> __device__ __forceinline__ float g_to_f32(uint16_t u) {
  if constexpr (ST == DUGKS_F16NEQ) return h16_to_f32(u);
  else return bf16_to_f32(u);
}
template <int ST> __device__ __forceinline__ uint16_t f32_to_g(float x) {
  if constexpr (ST == DUGKS_F16NEQ) return f32_to_h16(x);
  else return f32_to_bf16(x);
}
// 16-bit layout: after the phi plane, (Q - 1) / 2 planes of 32-bit words; the
// word of pair p holds direction 2p + 1 in its low half and 2p + 2 in its high
// half, so one load or store moves two directions.
template <int ST> __device__ __forceinline__ float g_lo(unsigned u) {
  return g_to_f32<ST>((uint16_t)u);
}
template <int ST> __device__ __forceinline__ float g_hi(unsigned u) {
  if constexpr (ST == DUGKS_F16NEQ) return g_to_f32<ST>((uint16_t)(u >> 16));
  else return __uint_as_float(u & 0xffff0000u);
}
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 h16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
// x and y rounded to nearest even into one word (x low, y high)
template <int ST> __device__ __forceinline__ unsigned f32x2_to_g(float x, float y) {
  const f32x2_t v = {x, y};
  if constexpr (ST == DUGKS_F16NEQ) return __builtin_bit_cast(unsigned, __builtin_convertvector(v, h16x2_t));
  else return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
}
template <int ST> __device__ __forceinline__ float g_limit() {
  return ST == DUGKS_F16NEQ ? 65504.0f : 3.0e38f;
}

// Power-of-two scale s such that max_{i >= 1} |f~_i - E_i| * s lies in (2^13, 2^14].
__host__ __device__ inline float neq_scale(float m) {
  if (!(m > 0.0f) || !(m < 3.0e38f)) return 1.0f;
  int e;
  (void)frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  int k = 14 - e;
  k = k > 100 ? 100 : (k < -100 ? -100 : k);
  return ldexpf(1.0f, k);
}

// Scale of a 16-bit format.  bfloat16 has the exponent range of binary32, so a
// power-of-two scale changes none of its rounded values outside the subnormal
// range: it stores f~ - E unscaled (s = 1).  binary16 stores s (f~ - E).
template <int ST> __host__ __device__ inline float neq_scale_for(float m) {
  if constexpr (ST == DUGKS_BF16NEQ) return 1.0f;
  else return neq_scale(m);
}

// ------------------------------------------------------------ DPP helpers
// wave_shr:1 -> lane l receives lane l-1; wave_shl:1 -> lane l receives lane l+1.
// Lanes without a source (0 for shr, 63 for shl) read 0 (bound_ctrl); their
// results are never used.
__device__ __forceinline__ float shr1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float shl1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ double shr1(double v) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_mov_dpp(p.x, 0x138, 0xF, 0xF, true);
  p.y = __builtin_amdgcn_mov_dpp(p.y, 0x138, 0xF, 0xF, true);
  return __builtin_bit_cast(double, p);
}
__device__ __forceinline__ double shl1(double v) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_mov_dpp(p.x, 0x130, 0xF, 0xF, true);
  p.y = __builtin_amdgcn_mov_dpp(p.y, 0x130, 0xF, 0xF, true);
  return __builtin_bit_cast(double, p);
}

// ------------------------------------------------------------ coefficients
template <typename T> struct Coef;
template <> struct Coef<double> {
  __device__ static const double* e(const InstDev* I, int k) { return I->e[k]; }
  __device__ static double ra(const InstDev* I) { return I->ra; }
  __device__ static double rb(const InstDev* I) { return I->rb; }
  __device__ static double b1(const InstDev* I) { return I->b1; }
  __device__ static double inv_b1(const InstDev* I) { return I->inv_b1; }
  __device__ static double kg(const InstDev* I) { return I->kg; }
  __device__ static const double* col(const InstDev* I) { return I->colgeo; }
  __device__ static const double* row(const InstDev* I) { return I->rowgeo; }
  __device__ static const double* bp(const InstDev* I, int a) { return I->bp[a]; }
  __device__ static double lambda(const InstDev* I) { return I->lambda; }
  __device__ static double half_dt(const InstDev* I) { return I->half_dt; }
  __device__ static double half_h(const InstDev* I) { return I->half_h; }
};
template <> struct Coef<float> {
  __device__ static const float* e(const InstDev* I, int k) { return I->ef[k]; }
  __device__ static float ra(const InstDev* I) { return I->raf; }
  __device__ static float rb(const InstDev* I) { return I->rbf; }
  __device__ static float b1(const InstDev* I) { return I->b1f; }
  __device__ static float inv_b1(const InstDev* I) { return I->inv_b1f; }
  __device__ static float kg(const InstDev* I) { return I->kgf; }
  __device__ static const float* col(const InstDev* I) { return I->colgeo_f; }
  __device__ static const float* row(const InstDev* I) { return I->rowgeo_f; }
  __device__ static const float* bp(const InstDev* I, int a) { return I->bpf[a]; }
  __device__ static float lambda(const InstDev* I) { return I->lambdaf; }
  __device__ static float half_dt(const InstDev* I) { return I->half_dtf; }
  __device__ static float half_h(const InstDev* I) { return I->half_hf; }
};

// A wave-uniform value placed in a vector register.
__device__ __forceinline__ float to_vgpr(float s) {
  float v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

// The direction whose velocity is direction k's with x and y swapped, and the
// smaller index of the two.  When B_x = B_y and D_xx = D_yy, E_k = E_swap(k)
// (eq. 2.3 is symmetric under the swap), so an x<->y symmetric instance
// evaluates one polynomial for each such pair.
template <int Q> __host__ __device__ constexpr int swap_xy(int k) {
  for (int j = 0; j < Q; ++j)
    if (lat_cx(j) == lat_cy(k) && lat_cy(j) == lat_cx(k)) return j;
  return k;
}
template <int Q> __host__ __device__ constexpr int sym_rep(int k) {
  return swap_xy<Q>(k) < k ? swap_xy<Q>(k) : k;
}
static_assert(sym_rep<9>(2) == 1 && sym_rep<9>(4) == 3 && sym_rep<9>(8) == 6 && sym_rep<9>(5) == 5 &&
                  sym_rep<9>(7) == 7 && sym_rep<5>(2) == 1 && sym_rep<5>(4) == 3,
              "D2Q9 / D2Q5 direction order");

// p(x) = sum_{m < NC} c[m] x^m by Horner's rule
template <int NC, typename T> __device__ __forceinline__ T horner(const T* c, T x) {
  T r = c[NC - 1];
#pragma unroll
  for (int m = NC - 2; m >= 0; --m) r = fma(r, x, c[m]);
  return r;
}

// Coefficients of one instance for a work item.  Binary32 equilibria of
// degree <= 3 (36 values for D2Q9) are loaded once into wave-uniform
// registers and shared by the cell, the faces and the 16-bit encode; larger
// sets are read through the scalar cache where they are used.  SYM: every
// instance of the launch is x<->y symmetric (E_k and E_swap(k) have the same
// coefficients, checked bitwise on the host), and E_k evaluates the
// polynomial of sym_rep(k), which the compiler then shares within a cell or
// face: the same values with fewer instructions.
template <typename T, int Q, int NC, bool SYM = false> struct Eq {
  static constexpr bool kHeld = sizeof(T) == 4 && NC <= 4;
  T c[kHeld ? Q : 1][kHeld ? NC : 1];
  const InstDev* I;
  T ra, rb, b1, inv_b1, kg;
  __device__ __forceinline__ void load(const InstDev* __restrict__ inst) {
    using C = Coef<T>;
    I = inst;
    if constexpr (kHeld) {
#pragma unroll
      for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int m = 0; m < NC; ++m) c[k][m] = C::e(I, k)[m];
    }
    ra = C::ra(I);
    rb = C::rb(I);
    b1 = C::b1(I);
    inv_b1 = C::inv_b1(I);
    kg = C::kg(I);
  }
  // Horner's first step fma(c[NC-1], x, c[NC-2]) may read one scalar register
  // only: with the top coefficients in vector registers it needs no copy (the
  // 16-bit step, bound by its instruction count, takes 18 fewer a row; the
  // binary32 step, bound by memory, runs slower with the extra registers).
  __device__ __forceinline__ void top_to_vgpr() {
    if constexpr (kHeld && NC >= 2) {
#pragma unroll
      for (int k = 0; k < Q; ++k) c[k][NC - 1] = to_vgpr(c[k][NC - 1]);
    }
  }
  // The 16-bit formats hold g / (1 + ra) (one FMA a direction at the decode):
  // the faces and the ghost rule then take b1, rb and 1/b1 times 1 + ra.
  __device__ __forceinline__ void scale_g_16() {
    b1 = I->b1_of;
    rb = I->rb_of;
    inv_b1 = I->inv_b1_of;
  }
  __device__ __forceinline__ T E(int k, T x) const {
    const int r = SYM ? sym_rep<Q>(k) : k;
    if constexpr (kHeld) return horner<NC>(c[r], x);
    else return horner<NC>(Coef<T>::e(I, r), x);
  }
};

// Source constants of an instance (eq. 2.3's F_i and R_i through rho_i, eqs.
// 2.25 and 2.27); empty without a source.  NF: 0 without a source, 1 for
// sources independent of phi, kSrcPow when F is a polynomial in phi.
template <typename T, int Q, int NF> struct SrcEq;
template <typename T, int Q> struct SrcEq<T, Q, 0> {
  __device__ __forceinline__ void load(const InstDev*) {}
};
template <typename T, int Q, int NF> struct SrcEq {
  T bx[kRhoCoef], by[kRhoCoef];
  T lam, hdt, hh;
  bool implicit;   // some term of this instance depends on phi
  __device__ __forceinline__ void load(const InstDev* __restrict__ I) {
    implicit = NF > 1 && I->src_implicit != 0;
#pragma unroll
    for (int m = 0; m < kRhoCoef; ++m) {
      bx[m] = Coef<T>::bp(I, 0)[m];
      by[m] = Coef<T>::bp(I, 1)[m];
    }
    lam = Coef<T>::lambda(I);
    hdt = Coef<T>::half_dt(I);
    hh = Coef<T>::half_h(I);
  }
  // lambda S_i = lambda F w_i (1 + c_i.B'(x) / c_s^2) for the directions in MASK
  // (bit k set: direction k wanted)
  template <unsigned MASK>
  __device__ __forceinline__ void lam_s(T F, T x, T* out) const {
    const T lf = lam * F;
    const T px = horner<kRhoCoef>(bx, x) * lf, py = horner<kRhoCoef>(by, x) * lf;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (!((MASK >> k) & 1u)) continue;
      T v = lf;
      if (lat_cx(k) != 0) v = lat_cx(k) > 0 ? v + px : v - px;
      if (lat_cy(k) != 0) v = lat_cy(k) > 0 ? v + py : v - py;
      out[k] = (T)lat_w<Q>(k) * v;
    }
  }
};

// Interface phi in binary64 for the binary32 and 16-bit formats too.
#ifndef DUGKS_FACE_SUM64
#define DUGKS_FACE_SUM64 0
#endif

// Sum over directions of the interface values: binary64 for the binary64
// path, a balanced binary32 tree otherwise (or a binary64 sum rounded once).
template <int Q> __device__ __forceinline__ double dir_sum(const double* v) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) s += v[k];
  return s;
}
template <int Q> __device__ __forceinline__ float dir_sum(const float* v) {
  if constexpr (DUGKS_FACE_SUM64) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) s += (double)v[k];
    return (float)s;
  }
  float t[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) t[k] = v[k];
#pragma unroll
  for (int w = 1; w < Q; w *= 2)
#pragma unroll
    for (int k = 0; k + w < Q; k += 2 * w) t[k] += t[k + w];
  return t[0];
}

// Conserved value v with v - half_tau P(v) = s, P(v) = sum_{k<NF} a[k] v^k
// (half_tau = dt/2 in a cell, eq. 2.25; h/2 at a face, eq. 2.27).  Explicit
// when F does not depend on phi (NF = 1, or an instance whose terms all have
// power 0 in a launch for sources that do: the same root, rounded the same
// way as in a launch without such sources); otherwise Newton's method from
// v = s until the update is at most tol (1 + |v|) (1e-15 in binary64, 2.4e-7
// in binary32) or after 8 (6) updates.
template <int NF, typename T>
__device__ __forceinline__ T solve_conserved(T s, T half_tau, const T* a, bool implicit = true) {
  if (NF == 1 || !implicit) {
    return fma(half_tau, a[0], s);
  } else {
    constexpr bool dbl = sizeof(T) == 8;
    const T tol = dbl ? (T)1e-15 : (T)2.4e-7;
    T v = s;
#pragma unroll 1
    for (int it = 0; it < (dbl ? 8 : 6); ++it) {
      const T P = horner<NF>(a, v);
      T dP = (T)(NF - 1) * a[NF - 1];
#pragma unroll
      for (int m = NF - 2; m >= 1; --m) dP = fma(dP, v, (T)m * a[m]);
      const T d = (v - half_tau * P - s) / ((T)1 - half_tau * dP);
      v -= d;
      if (!(fabs(d) > tol * ((T)1 + fabs(v)))) break;
    }
    return v;
  }
}

// ------------------------------------------------------------ memory
// Pointer into the constant address space: uniform loads through it become
// scalar loads.  Only for data that no kernel writes while it is read.
template <typename T> using CPtr = const __attribute__((address_space(4))) T*;
template <typename T> __device__ __forceinline__ CPtr<T> as_constant(const T* p) {
  return (CPtr<T>)p;
}

// Raw stored values of one cell.
template <int Q, int ST> struct Raw;
template <int Q> struct Raw<Q, DUGKS_F64> { double v[Q]; };
template <int Q> struct Raw<Q, DUGKS_F32> { float v[Q]; };
template <int Q> struct Raw<Q, DUGKS_F16NEQ> { float phi; unsigned g2[(Q - 1) / 2]; };
template <int Q> struct Raw<Q, DUGKS_BF16NEQ> { float phi; unsigned g2[(Q - 1) / 2]; };

typedef unsigned v2u __attribute__((ext_vector_type(2)));

// Buffer resource over one f~ buffer: the per-lane byte offset goes in a VGPR,
// the plane offset in an SGPR; accesses outside [0, bytes) read 0 / are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <int Q, int ST>
__device__ __forceinline__ void load_raw_buf(Raw<Q, ST>& r, __amdgpu_buffer_rsrc_t R, unsigned plane,
                                             unsigned idx) {
  if constexpr (ST == DUGKS_F64) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const unsigned soff = (unsigned)k * plane * 8u;
      r.v[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(R, idx * 8u, soff, 0));
    }
  } else if constexpr (ST == DUGKS_F32) {
#pragma unroll
    for (int k = 0; k < Q; ++k)
      r.v[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(R, idx * 4u, (unsigned)k * plane * 4u, 0));
  } else {
    static_assert((Q - 1) % 2 == 0, "directions 1..Q-1 in pairs");
    r.phi = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(R, idx * 4u, 0u, 0));
#pragma unroll
    for (int p = 0; p < (Q - 1) / 2; ++p)
      r.g2[p] = __builtin_amdgcn_raw_buffer_load_b32(R, idx * 4u, (unsigned)(p + 1) * plane * 4u, 0);
  }
}

// Pointer-based loads (the plain kernel).
template <int Q, int ST>
__device__ __forceinline__ void load_raw(Raw<Q, ST>& r, const char* buf, long long plane,
                                         long long off) {
  if constexpr (ST == DUGKS_F64) {
    const double* b = (const double*)buf;
#pragma unroll
    for (int k = 0; k < Q; ++k) r.v[k] = b[k * plane + off];
  } else if constexpr (ST == DUGKS_F32) {
    const float* b = (const float*)buf;
#pragma unroll
    for (int k = 0; k < Q; ++k) r.v[k] = b[k * plane + off];
  } else {
    r.phi = ((const float*)buf)[off];
    const unsigned* g = (const unsigned*)buf + plane;
#pragma unroll
    for (int p = 0; p < (Q - 1) / 2; ++p) r.g2[p] = g[p * plane + off];
  }
}

// Scale factors of the 16-bit formats for this step.
struct Scales {
  float inv_in;  // 1 / s of the input buffer
  float out;     // s of the output buffer
};

// g = fbar+ / b1 (eq. 2.21) of the source cell and f~+ (eq. 2.23) when wanted.
// With a source, pc = the coefficients of F at the cell centre at t_n as a
// polynomial in phi: phi solves phi = sum f~ + dt F(phi) / 2 and g gains
// lambda F rho(phi) (eqs. 2.25, 2.27).
template <int Q, int ST, int NC, int NF = 0, bool SYM = false>
__device__ __forceinline__ void cell_g(const InstDev* __restrict__ I,
                                       const Eq<typename Stor<ST>::T, Q, NC, SYM>& eq,
                                       const Raw<Q, ST>& r, const Scales& sc,
                                       typename Stor<ST>::T* g, typename Stor<ST>::T* ftp,
                                       bool want_ftp, typename Stor<ST>::T& phi_out,
                                       const SrcEq<typename Stor<ST>::T, Q, NF>& se = {},
                                       const typename Stor<ST>::T* pc = nullptr) {
  using T = typename Stor<ST>::T;
  constexpr bool SRC = NF > 0;
  static_assert(!SRC || !Stor<ST>::neq, "sources run in binary64 / binary32 storage");
  if constexpr (!Stor<ST>::neq) {
    double phi = 0.0;  // phi = sum_i f~_i (Sec. 2), binary64
#pragma unroll
    for (int k = 0; k < Q; ++k) phi += (double)r.v[k];
    T Fc = 0;
    if constexpr (SRC) {
      double a[NF];
#pragma unroll
      for (int k = 0; k < NF; ++k) a[k] = (double)pc[k];
      phi = solve_conserved<NF, double>(phi, (double)se.hdt, a, se.implicit);
    }
    const T p = (T)phi;
    const T ra = eq.ra;
    if constexpr (SRC) {
      Fc = NF == 1 ? pc[0] : horner<NF>(pc, p);
      T ls[Q];
      se.template lam_s<(1u << Q) - 1u>(Fc, p, ls);
#pragma unroll
      for (int k = 0; k < Q; ++k) g[k] = fma(ra, r.v[k], eq.E(k, p) + ls[k]);
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) g[k] = fma(ra, r.v[k], eq.E(k, p));
    }
    if (want_ftp) {
      const T kg = eq.kg;
#pragma unroll
      for (int k = 0; k < Q; ++k) ftp[k] = fma(kg, g[k], (T)(-1.0 / 3.0) * r.v[k]);
    }
    phi_out = p;
  } else {
    const float p = r.phi;
    float gs[Q];
    float sum = 0.0f;
#pragma unroll
    for (int p = 0; p < (Q - 1) / 2; ++p) {
      gs[2 * p + 1] = g_lo<ST>(r.g2[p]);
      gs[2 * p + 2] = g_hi<ST>(r.g2[p]);
    }
#pragma unroll
    for (int k = 1; k < Q; ++k) sum += gs[k];
    gs[0] = -sum;
    // f~ = E + gs / s:  g = (1 + ra) E + ra gs / s, held as g / (1 + ra) =
    // E + (ra / (1 + ra)) gs / s;  f~+ = E + a2 gs / s
    const float ras = I->ra_of * sc.inv_in, a2s = I->a2f * sc.inv_in;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const float E = eq.E(k, p);
      g[k] = fma(ras, gs[k], E);
      if (want_ftp) ftp[k] = fma(a2s, gs[k], E);
    }
    phi_out = p;
  }
}

// Ghost rules on g of the source cell a (already in g).
template <int Q, int ST, int NC, bool SYM = false>
__device__ __forceinline__ void ghost_g(const InstDev* __restrict__ I,
                                        const Eq<typename Stor<ST>::T, Q, NC, SYM>& eq,
                                        typename Stor<ST>::T* g, typename Stor<ST>::T phi_a,
                                        bool wall_x, bool wall_y, double phi_g) {
  using T = typename Stor<ST>::T;
  const bool dir = (wall_x && I->bcx == DUGKS_BC_DIRICHLET) || (wall_y && I->bcy == DUGKS_BC_DIRICHLET);
  if (dir) {
    // non-equilibrium extrapolation: fbar+_g = E(phi_g) + (fbar+_a - E(phi_a))
    const T pg = (T)phi_g, ib = eq.inv_b1;
#pragma unroll
    for (int k = 0; k < Q; ++k) g[k] = fma(eq.E(k, pg) - eq.E(k, phi_a), ib, g[k]);
  } else {
    T t[Q];
    if (wall_x) {
#pragma unroll
      for (int k = 0; k < Q; ++k) t[k] = g[mir_x(k)];
#pragma unroll
      for (int k = 0; k < Q; ++k) g[k] = t[k];
    }
    if (wall_y) {
#pragma unroll
      for (int k = 0; k < Q; ++k) t[k] = g[mir_y(k)];
#pragma unroll
      for (int k = 0; k < Q; ++k) g[k] = t[k];
    }
  }
}

__device__ __forceinline__ int ring_index(int nx, int ny, int i, int j) {
  if (j == -1) return i + 1;
  if (j == ny) return (nx + 2) + i + 1;
  if (i == -1) return 2 * (nx + 2) + j;
  return 2 * (nx + 2) + ny + j;
}

__device__ __forceinline__ int src_index(int i, int n, int bc) {
  if (i >= 0 && i < n) return i;
  if (bc == DUGKS_BC_PERIODIC) {
    int w = i < 0 ? i + n : i - n;
    return w < 0 ? 0 : (w >= n ? n - 1 : w);
  }
  return i < 0 ? 0 : n - 1;
}

// Pairwise sum of N values.
template <int N, typename T> __device__ __forceinline__ T tree_sum(const T* v) {
  if constexpr (N == 1) return v[0];
  else return tree_sum<N / 2>(v) + tree_sum<N - N / 2>(v + N / 2);
}

// Number of directions with a velocity component normal to an x-face (NRM 0)
// or a y-face (NRM 1).
template <int Q, int NRM> constexpr int normal_count() {
  int n = 0;
  for (int k = 0; k < Q; ++k)
    if ((NRM == 0 ? lat_cx(k) : lat_cy(k)) != 0) ++n;
  return n;
}

// Sum of g over the directions without a component normal to an x-face (NRM
// 0) or a y-face (NRM 1).
template <int Q, int NRM, typename T> __device__ __forceinline__ T zero_normal_sum(const T* g) {
  T s = 0;
  bool first = true;
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if ((NRM == 0 ? lat_cx(k) : lat_cy(k)) == 0) {
      s = first ? g[k] : s + g[k];
      first = false;
    }
  return s;
}

// Directions with a velocity component normal to an x-face (NRM 0) or a
// y-face (NRM 1), as a bit mask.
template <int Q, int NRM> constexpr unsigned normal_mask() {
  unsigned m = 0;
  for (int k = 0; k < Q; ++k)
    if ((NRM == 0 ? lat_cx(k) : lat_cy(k)) != 0) m |= 1u << k;
  return m;
}

// Half-step interface distribution (eq. 2.20, eq. 2.19 in the form of eq.
// 2.26) on g, the interface phi, and F = f_b / b3 (eq. 2.22) for directions
// with a normal velocity component.  ts[k] = dL + dR, the sum of the two
// cells' central-difference numerators along the face (directions with a
// tangential component).  NRM = 0 for x-faces, 1 for y-faces.
// With a source, pb_c = the coefficients of F at the face point at t_n + h as
// a polynomial in phi: phi_b solves phi_b = sum fbar + h F(phi_b) / 2 and F
// gains lambda F(phi_b) rho(phi_b) (eq. 2.27 solved for f).
//
// ZS (the 16-bit step): directions without a normal component enter only
// phi_b, and they all take the same a0, so their sum is interpolated from the
// two cells' sums zL, zR of g over those directions (plus their tangential
// terms) instead of direction by direction.
template <int Q, int NC, int NRM, typename T, int NF = 0, bool ZS = false, bool SYM = false>
__device__ __forceinline__ void face(const Eq<T, Q, NC, SYM>& eq, const T* L, const T* R, const T* ts,
                                     T am, T a0, T ap, T tau, T* out,
                                     const SrcEq<T, Q, NF>& se = {}, const T* pb_c = nullptr,
                                     T zL = 0, T zR = 0) {
  constexpr bool SRC = NF > 0;
  static_assert(!(SRC && ZS), "interpolated sums without a source only");
  T gb[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int cn = NRM == 0 ? lat_cx(k) : lat_cy(k);
    const int ct = NRM == 0 ? lat_cy(k) : lat_cx(k);
    if (ZS && cn == 0) continue;
    const T al = cn > 0 ? ap : (cn < 0 ? am : a0);
    T v = fma(al, R[k] - L[k], L[k]);
    if (ct != 0) v = fma((T)(-ct) * tau, ts[k], v);
    gb[k] = v;
  }
  // phi(x_b, t + h) = sum_i fbar_i = b1 sum_i gbar_i  (+ h F_b / 2)
  T pb;
  if constexpr (ZS) {
    T tz = 0;   // sum of -c_t ts over the directions without a normal component
    bool first = true;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int cn = NRM == 0 ? lat_cx(k) : lat_cy(k);
      const int ct = NRM == 0 ? lat_cy(k) : lat_cx(k);
      if (cn == 0 && ct != 0) {
        const T t = ct > 0 ? -ts[k] : ts[k];
        tz = first ? t : tz + t;
        first = false;
      }
    }
    T v[Q];
    int n = 0;
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if ((NRM == 0 ? lat_cx(k) : lat_cy(k)) != 0) v[n++] = gb[k];
    v[n++] = fma(tau, tz, fma(a0, zR - zL, zL));
    pb = tree_sum<normal_count<Q, NRM>() + 1>(v) * eq.b1;
  } else {
    pb = (T)(dir_sum<Q>(gb) * eq.b1);
  }
  T Fb = 0;
  if constexpr (SRC) {
    pb = solve_conserved<NF, T>(pb, se.hh, pb_c, se.implicit);
    Fb = NF == 1 ? pb_c[0] : horner<NF>(pb_c, pb);
  }
  const T rb = eq.rb;
  T ls[Q];
  if constexpr (SRC) se.template lam_s<normal_mask<Q, NRM>()>(Fb, pb, ls);
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int cn = NRM == 0 ? lat_cx(k) : lat_cy(k);
    if (cn != 0) {
      if constexpr (SRC)
        out[k] = fma(rb, gb[k], eq.E(k, pb) + ls[k]);
      else
        out[k] = fma(rb, gb[k], eq.E(k, pb));
    }
  }
}

// Map a block index so that consecutive logical blocks land on one XCD
// (blocks are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_logical(int b, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int x = b & 7, i = b >> 3;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ---------------------------------------------------------- fused step
// GH: the item touches a wall (ghost rules needed); items that do not use a
// branch-free row computation.
// NF: 0 without a source; 1 when every source of the launch is one term
// independent of phi (one G a row); kSrcPow otherwise (up to kMaxSrcTerms
// terms, F a polynomial in phi).  An instance without a source has no terms
// and gives the result of the source-free step; one with a single phi-free
// term gives the same result in either kind of launch.
template <int Q, int ST, int NC, bool GH, int NF, bool SYM = false>
__device__ __forceinline__ void step_item(const InstDev* __restrict__ I, const WorkItem it,
                                          int parity, long long step, int lane, bool measure) {
  using T = typename Stor<ST>::T;
  using C = Coef<T>;
  constexpr bool SRC = NF > 0;
  constexpr int NFA = NF > 0 ? NF : 1;   // array extents
  constexpr int NT = NF > 1 ? kMaxSrcTerms : 1;
  constexpr int PF = Stor<ST>::neq ? DUGKS_PREFETCH_NEQ : DUGKS_PREFETCH;
  constexpr bool ZS = Stor<ST>::neq;     // faces interpolate the zero-normal sums
  static_assert(PF == 1 || PF == 2, "one or two rows ahead");
  static_assert(!SRC || PF == 1, "source rows follow the one-row prefetch");
  Eq<T, Q, NC, SYM> eq;
  eq.load(I);
  SrcEq<T, Q, NF> se;
  se.load(I);
  const int nx = I->nx, ny = I->ny, pitch = I->pitch, bcx = I->bcx, bcy = I->bcy;
  const unsigned plane = (unsigned)I->plane;
  const __amdgpu_buffer_rsrc_t Rin = rsrc(I->buf[parity], I->buf_bytes);
  const __amdgpu_buffer_rsrc_t Rout = rsrc(I->buf[parity ^ 1], I->buf_bytes);

  Scales sc{1.0f, 1.0f};
  if constexpr (Stor<ST>::neq) {
    sc.inv_in = 1.0f / neq_scale_for<ST>(I->slots[(step + 2) & 3]);
    sc.out = neq_scale_for<ST>(I->slots[(step + 3) & 3]);
    eq.scale_g_16();
    eq.top_to_vgpr();
  }

  const int c = it.x0 - 1 + lane;
  const int sc_col = src_index(c < nx + 1 ? c : nx, nx, bcx);
  const bool wall_x = (c < 0 || c >= nx) && bcx != DUGKS_BC_PERIODIC;
  const bool live = lane >= 1 && lane <= kStripCols && c < nx;
  const bool strip_touches_x_wall = bcx != DUGKS_BC_PERIODIC && (it.x0 == 0 || it.x0 + kStripCols >= nx);

  // per-column geometry: W-face coefficients, tangential factor, update factor
  const T* cg = C::col(I) + (long long)((c + 1 < nx + 1 ? c + 1 : nx + 1)) * kGeo;
  const T cam = cg[0], ca0 = cg[1], cap = cg[2], ctau = cg[3], ck = cg[4];
  // Row factors are wave-uniform: read them through the scalar cache (a
  // generic pointer would give flat loads, whose completion can only be
  // awaited together with every row load in flight).
  const CPtr<T> rg = as_constant(C::row(I));

  const double* ring = (I->ring != nullptr) ? I->ring + step * I->ring_len : nullptr;

  // Source: G_j of each row's cells (a ghost takes the G_j of the cell it
  // copies), each term scaled by exp(gamma_j t) at t_n for the cells (pc) and
  // at t_n + h for the faces (FC), and summed by power of phi.
  __amdgpu_buffer_rsrc_t Rg = rsrc(nullptr, 0u);
  int nt = 0;
  unsigned gplane = 0;
  T en[NT], eh[NT];
  int pw[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) { en[t] = 0; eh[t] = 0; pw[t] = 0; }
  if constexpr (SRC) {
    Rg = rsrc(I->src_g, I->src_bytes);
    nt = I->src_n;
    gplane = I->src_plane;
    const double tn = (double)step * I->dt;
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (t < nt) {
        en[t] = (T)exp(I->src_gam[t] * tn);
        eh[t] = (T)exp(I->src_gam[t] * (tn + I->half_dt));
        pw[t] = NF == 1 ? 0 : I->src_pow[t];
      }
  }
  auto load_gsrc = [&](int r, T* gr) {
    const unsigned off = (unsigned)(src_index(r, ny, bcy) * nx + sc_col) * 8u;
#pragma unroll
    for (int t = 0; t < NT; ++t)
      gr[t] = t < nt ? (T)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                       Rg, off, (unsigned)t * gplane, 0))
                     : (T)0;
  };
  // coefficients of F as a polynomial in phi at the cell (t_n) and for the faces (t_n + h)
  auto coefs = [&](const T* gr, T* pc, T* pf) {
#pragma unroll
    for (int k = 0; k < NFA; ++k) { pc[k] = 0; pf[k] = 0; }
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (t < nt) {
#pragma unroll
        for (int k = 0; k < NFA; ++k)
          if (pw[t] == k) {
            pc[k] = fma(en[t], gr[t], pc[k]);
            pf[k] = fma(eh[t], gr[t], pf[k]);
          }
      }
  };

  auto make_row = [&](const Raw<Q, ST>& raw, int r, T* g, T* ftp, bool want_ftp, const T* gr,
                      T* pf) {
    T phi_a;
    T pc[NFA];
    coefs(gr, pc, pf);
    cell_g<Q, ST, NC, NF>(I, eq, raw, sc, g, ftp, want_ftp, phi_a, se, pc);
    if constexpr (!GH) return;
    const bool wall_y = (r < 0 || r >= ny) && bcy != DUGKS_BC_PERIODIC;
    if (wall_y || strip_touches_x_wall) {
      if (wall_x || wall_y) {
        double pg = 0.0;
        if (ring != nullptr) pg = ring[ring_index(nx, ny, c < -1 ? -1 : (c > nx ? nx : c), r)];
        ghost_g<Q, ST, NC>(I, eq, g, phi_a, wall_x, wall_y, pg);
      }
    }
  };
  auto row_idx = [&](int r) -> unsigned {
    return (unsigned)(src_index(r, ny, bcy) * pitch + sc_col);
  };

  const int y0 = it.y0, y1 = it.y1;
  // Per-row values live in slot (row - y0) % 3: g (G), g of lane-1 (LS), f~+
  // (FT), x-slope numerators (SX), the face above the row (FY) and the raw
  // loads (RW).  The loop is unrolled three times so that rotating the window
  // is a change of register names, not a copy.
  T G[3][Q], LS[3][Q], FT[3][Q], SX[3][Q], FY[3][Q], ts[Q], dy[Q], fW[Q];
  Raw<Q, ST> RW[3];
  T ZX[3], ZY[3];  // g summed over the directions with c_x = 0 / c_y = 0 (ZS)
  T GR[3][NT];     // source G_j of the row whose raw values sit in RW[.]
  T FC[3][NFA];    // face-time coefficients of F of the row made into G[.]
  T pfb[NFA];      // the same interpolated to a face
#pragma unroll
  for (int s3 = 0; s3 < 3; ++s3) {
#pragma unroll
    for (int t = 0; t < NT; ++t) GR[s3][t] = 0;
#pragma unroll
    for (int k = 0; k < NFA; ++k) FC[s3][k] = 0;
  }

  // prologue: row y0-1 in slot 2, row y0 in slot 0, the face below row y0 in FY[2]
  load_raw_buf<Q, ST>(RW[2], Rin, plane, row_idx(y0 - 1));
  load_raw_buf<Q, ST>(RW[0], Rin, plane, row_idx(y0));
  load_raw_buf<Q, ST>(RW[1], Rin, plane, row_idx(y0 + 1));
  if constexpr (SRC) {
    load_gsrc(y0 - 1, GR[2]);
    load_gsrc(y0, GR[0]);
    load_gsrc(y0 + 1, GR[1]);
  }
  make_row(RW[2], y0 - 1, G[2], FT[2], false, GR[2], FC[2]);
  make_row(RW[0], y0, G[0], FT[0], true, GR[0], FC[0]);
  if constexpr (ZS) {
    ZX[2] = zero_normal_sum<Q, 0>(G[2]);
    ZY[2] = zero_normal_sum<Q, 1>(G[2]);
    ZX[0] = zero_normal_sum<Q, 0>(G[0]);
    ZY[0] = zero_normal_sum<Q, 1>(G[0]);
  }
  if constexpr (PF == 2)  // two rows in flight ahead of the row being consumed
    load_raw_buf<Q, ST>(RW[2], Rin, plane, row_idx(y0 + 2 <= y1 ? y0 + 2 : y1));
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    if (!ZS || lat_cx(k) != 0) LS[0][k] = shr1(G[0][k]);
    if (lat_cx(k) != 0) {
      SX[0][k] = shl1(G[0][k]) - LS[0][k];
      ts[k] = (shl1(G[2][k]) - shr1(G[2][k])) + SX[0][k];
    }
  }
  {
    const CPtr<T> g = rg + (long long)(y0 + 1) * kGeo;
#pragma unroll
    for (int k = 0; k < NFA; ++k) pfb[k] = fma(g[1], FC[0][k] - FC[2][k], FC[2][k]);
    if constexpr (ZS)
      face<Q, NC, 1, T, 0, true>(eq, G[2], G[0], ts, g[0], g[1], g[2], ctau, FY[2], {}, nullptr, ZY[2], ZY[0]);
    else
      face<Q, NC, 1, T, NF>(eq, G[2], G[0], ts, g[0], g[1], g[2], ctau, FY[2], se, pfb);
  }

  bool bad = false, ovf = false;
  float mx = 0.0f;
  auto body = [&](int j, auto slot) {
    constexpr int s0 = decltype(slot)::value, sp = (s0 + 1) % 3, sm = (s0 + 2) % 3;
    // row j+1 is in RW[sp]; the next load goes PF rows further
    if constexpr (PF == 2)
      load_raw_buf<Q, ST>(RW[s0], Rin, plane, row_idx(j + 3 <= y1 ? j + 3 : y1));
    else
      load_raw_buf<Q, ST>(RW[sm], Rin, plane, row_idx(j + 2 <= y1 ? j + 2 : y1));
    if constexpr (SRC) load_gsrc(j + 2 <= y1 ? j + 2 : y1, GR[sm]);
    make_row(RW[sp], j + 1, G[sp], FT[sp], true, GR[sp], FC[sp]);
    if constexpr (ZS) {
      ZX[sp] = zero_normal_sum<Q, 0>(G[sp]);
      ZY[sp] = zero_normal_sum<Q, 1>(G[sp]);
    }
    const CPtr<T> gj = rg + (long long)(j + 1) * kGeo;   // row j: its S face and factors
    const CPtr<T> gn = rg + (long long)(j + 2) * kGeo;   // row j+1: S face = N face of row j
    const T rtau = gj[3], rk = gj[4];
    // x-slope numerators of row j+1: g(lane+1) - g(lane-1)
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (!ZS || lat_cx(k) != 0) LS[sp][k] = shr1(G[sp][k]);
      if (lat_cx(k) != 0) {
        SX[sp][k] = shl1(G[sp][k]) - LS[sp][k];
        ts[k] = SX[s0][k] + SX[sp][k];
      }
    }
#pragma unroll
    for (int k = 0; k < NFA; ++k) pfb[k] = fma(gn[1], FC[sp][k] - FC[s0][k], FC[s0][k]);
    if constexpr (ZS)
      face<Q, NC, 1, T, 0, true>(eq, G[s0], G[sp], ts, gn[0], gn[1], gn[2], ctau, FY[s0], {}, nullptr,
                                 ZY[s0], ZY[sp]);
    else
      face<Q, NC, 1, T, NF>(eq, G[s0], G[sp], ts, gn[0], gn[1], gn[2], ctau, FY[s0], se, pfb);
    // west face of this lane's cell: left state from lane-1; y-slope numerators
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (lat_cy(k) != 0) {
        dy[k] = G[sp][k] - G[sm][k];
        ts[k] = shr1(dy[k]) + dy[k];
      }
    if constexpr (SRC) {
#pragma unroll
      for (int k = 0; k < NFA; ++k) {
        const T gl = shr1(FC[s0][k]);
        pfb[k] = fma(ca0, FC[s0][k] - gl, gl);
      }
      face<Q, NC, 0, T, NF>(eq, LS[s0], G[s0], ts, cam, ca0, cap, rtau, fW, se, pfb);
    } else if constexpr (ZS) {
      face<Q, NC, 0, T, 0, true>(eq, LS[s0], G[s0], ts, cam, ca0, cap, rtau, fW, {}, nullptr,
                                 shr1(ZX[s0]), ZX[s0]);
    } else {
      face<Q, NC, 0>(eq, LS[s0], G[s0], ts, cam, ca0, cap, rtau, fW);
    }
    // update (eq. 2.24): f~(t+dt) = f~+ - dt c_i.(flux differences)/width
    T o[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      T v = FT[s0][k];
      if (lat_cx(k) != 0) v = fma((T)(-lat_cx(k)) * ck, shl1(fW[k]) - fW[k], v);
      if (lat_cy(k) != 0) v = fma((T)(-lat_cy(k)) * rk, FY[s0][k] - FY[sm][k], v);
      o[k] = v;
    }
    if (live) {
      const unsigned idx = (unsigned)(j * pitch + c);
      if constexpr (!Stor<ST>::neq) {
        bad |= !__builtin_isfinite(o[0]);
        if (!measure) {
#pragma unroll
          for (int k = 0; k < Q; ++k) {
            if constexpr (ST == DUGKS_F64)
              __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, o[k]), Rout, idx * 8u,
                                                    (unsigned)k * plane * 8u, 0);
            else
              __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, o[k]), Rout, idx * 4u,
                                                    (unsigned)k * plane * 4u, 0);
          }
        }
      } else {
        double ps = (double)o[0];         // phi(t + dt) = sum_i f~_i in binary64,
#pragma unroll
        for (int k = 1; k < Q; ++k) ps += (double)o[k];
        const float pf = (float)ps;       // rounded once to the stored binary32
        bad |= !__builtin_isfinite(pf);
        float m1 = 0.0f;                  // max |f~_i - E_i| over the stored i >= 1
        float sq[Q];
#pragma unroll
        for (int k = 1; k < Q; ++k) {
          const float d = o[k] - eq.E(k, pf);
          m1 = fmaxf(m1, fabsf(d));
          float s = d * sc.out;
          // binary16: saturate (an overflow is flagged below); bfloat16 has
          // binary32's range
          if constexpr (ST == DUGKS_F16NEQ) s = __builtin_amdgcn_fmed3f(s, -g_limit<ST>(), g_limit<ST>());
          sq[k] = s;
        }
        ovf |= !measure && m1 * sc.out > g_limit<ST>();
        mx = fmaxf(mx, m1);
        if (!measure) {
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, pf), Rout, idx * 4u, 0u, 0);
#pragma unroll
          for (int p = 0; p < (Q - 1) / 2; ++p)
            __builtin_amdgcn_raw_buffer_store_b32(f32x2_to_g<ST>(sq[2 * p + 1], sq[2 * p + 2]), Rout,
                                                  idx * 4u, (unsigned)(p + 1) * plane * 4u, 0);
        }
      }
    }
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  int j = y0;
  for (; j + 3 <= y1; j += 3) {
    body(j, S0{});
    body(j + 1, S1{});
    body(j + 2, S2{});
  }
  if (j < y1) body(j, S0{});
  if (j + 1 < y1) body(j + 1, S1{});
  if constexpr (Stor<ST>::neq) {
    // wave maximum of |f~_i - E_i| (i >= 1) over updated cells -> the instance's slot
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0 && mx > 0.0f) {
      const int slot = measure ? (int)((step + 3) & 3) : (int)(step & 3);
      atomicMax((unsigned*)(I->slots + slot), __float_as_uint(mx));
    }
  }
  if (__any(bad) && lane == 0) atomicOr(I->flags, (unsigned)DUGKS_FLAG_NONFINITE);
  if (__any(ovf) && lane == 0) atomicOr(I->flags, (unsigned)DUGKS_FLAG_OVERFLOW);
}

// Occupancy target of the step kernel (waves per SIMD): bounds the register
// allocation so that enough waves stay resident to hide HBM latency.
#ifndef DUGKS_WAVES_PER_EU_F32
#define DUGKS_WAVES_PER_EU_F32 2
#endif
#ifndef DUGKS_WAVES_PER_EU_F64
#define DUGKS_WAVES_PER_EU_F64 1
#endif
#ifndef DUGKS_WAVES_PER_EU_NEQ
#define DUGKS_WAVES_PER_EU_NEQ 3
#endif
// The 16-bit step is bound by its instruction count: three waves per SIMD
// (168 registers, spills outside the row loop only) hide more of its latency
// than two.  The source path holds more per row (G and its window): one wave
// per SIMD, the full register file, no spills.
template <int ST, int NF> struct Occupancy {
  static constexpr int value = NF > 0 ? 1
                               : ST == DUGKS_F64 ? DUGKS_WAVES_PER_EU_F64
                               : Stor<ST>::neq   ? DUGKS_WAVES_PER_EU_NEQ
                                                 : DUGKS_WAVES_PER_EU_F32;
};
// Threads per block: at two waves per SIMD a block may hold 8 waves (fewer,
// larger blocks to dispatch); at one wave per SIMD at most 4.
template <int ST, int NF> constexpr int step_max_threads() {
  return Occupancy<ST, NF>::value >= 2 ? 512 : 256;
}

template <int Q, int ST, int NC, int NF, bool SYM>
__global__ __launch_bounds__((step_max_threads<ST, NF>())) __attribute__((amdgpu_waves_per_eu(Occupancy<ST, NF>::value)))
void k_step(const InstDev* __restrict__ insts,
                                              const WorkItem* __restrict__ items, int nitems,
                                              int parity, long long step, int xcd_remap,
                                              int persistent, int measure,
                                              const long long* __restrict__ step_base) {
  // a captured launch takes its step index as an offset from a base in device
  // memory, set before each replay
  if (step_base != nullptr) step += step_base[0];
  const int wpb = blockDim.x >> 6;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int b = xcd_remap ? xcd_logical(blockIdx.x, gridDim.x) : blockIdx.x;
  int item = b * wpb + w;
  const int stride = persistent ? gridDim.x * wpb : nitems;
  for (; item < nitems; item += stride) {
    const WorkItem it = items[item];
    const InstDev* I = insts + it.inst;
    const bool wall_x = I->bcx != DUGKS_BC_PERIODIC && (it.x0 == 0 || it.x0 + kStripCols >= I->nx);
    const bool wall_y = I->bcy != DUGKS_BC_PERIODIC && (it.y0 == 0 || it.y1 == I->ny);
    if (wall_x || wall_y)
      step_item<Q, ST, NC, true, NF, SYM>(I, it, parity, step, lane, measure != 0);
    else
      step_item<Q, ST, NC, false, NF, SYM>(I, it, parity, step, lane, measure != 0);
    if (!persistent) break;
  }
}

// Clear slot (step+which)&3 of every instance before a 16-bit step.
__global__ void k_clear_next_slot(const InstDev* __restrict__ insts, int ninst, long long step,
                                  int which) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) insts[i].slots[(step + which) & 3] = 0.0f;
}

// ------------------------------------------------------- plain FP64 step
// One thread per cell; every neighbour value is read from global memory and
// g of the 3x3 neighbourhood is recomputed per cell.
template <int Q, int NC>
__global__ __launch_bounds__(256) void k_step_plain(const InstDev* __restrict__ I, int parity,
                                                    long long step) {
  const int nx = I->nx, ny = I->ny, pitch = I->pitch;
  Eq<double, Q, NC> eq;
  eq.load(I);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nx || j >= ny) return;
  const long long plane = I->plane;
  const char* in = (const char*)I->buf[parity];
  double* out = (double*)I->buf[parity ^ 1];
  const double* ring = (I->ring != nullptr) ? I->ring + step * I->ring_len : nullptr;
  Scales sc{1.0f, 1.0f};
  double g[3][3][Q];
  for (int b = -1; b <= 1; ++b)
    for (int a = -1; a <= 1; ++a) {
      const int ci = i + a, cj = j + b;
      Raw<Q, DUGKS_F64> raw;
      load_raw<Q, DUGKS_F64>(raw, in, plane,
                             (long long)src_index(cj, ny, I->bcy) * pitch + src_index(ci, nx, I->bcx));
      double phi_a, dummy[Q];
      cell_g<Q, DUGKS_F64, NC>(I, eq, raw, sc, g[b + 1][a + 1], dummy, false, phi_a);
      const bool wx = (ci < 0 || ci >= nx) && I->bcx != DUGKS_BC_PERIODIC;
      const bool wy = (cj < 0 || cj >= ny) && I->bcy != DUGKS_BC_PERIODIC;
      if (wx || wy) {
        const double pg = ring != nullptr ? ring[ring_index(nx, ny, ci, cj)] : 0.0;
        ghost_g<Q, DUGKS_F64, NC>(I, eq, g[b + 1][a + 1], phi_a, wx, wy, pg);
      }
    }
  const double* cg = I->colgeo;
  const double* rg = I->rowgeo;
  const double* cW = cg + (long long)(i + 1) * kGeo;   // W face of column i
  const double* cE = cg + (long long)(i + 2) * kGeo;   // W face of column i+1
  const double* rS = rg + (long long)(j + 1) * kGeo;
  const double* rN = rg + (long long)(j + 2) * kGeo;
  double ts[Q], fW[Q], fE[Q], fS[Q], fN[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) ts[k] = (g[2][0][k] - g[0][0][k]) + (g[2][1][k] - g[0][1][k]);
  face<Q, NC, 0>(eq, g[1][0], g[1][1], ts, cW[0], cW[1], cW[2], rS[3], fW);
#pragma unroll
  for (int k = 0; k < Q; ++k) ts[k] = (g[2][1][k] - g[0][1][k]) + (g[2][2][k] - g[0][2][k]);
  face<Q, NC, 0>(eq, g[1][1], g[1][2], ts, cE[0], cE[1], cE[2], rS[3], fE);
#pragma unroll
  for (int k = 0; k < Q; ++k) ts[k] = (g[0][2][k] - g[0][0][k]) + (g[1][2][k] - g[1][0][k]);
  face<Q, NC, 1>(eq, g[0][1], g[1][1], ts, rS[0], rS[1], rS[2], cW[3], fS);
#pragma unroll
  for (int k = 0; k < Q; ++k) ts[k] = (g[1][2][k] - g[1][0][k]) + (g[2][2][k] - g[2][0][k]);
  face<Q, NC, 1>(eq, g[1][1], g[2][1], ts, rN[0], rN[1], rN[2], cW[3], fN);
  Raw<Q, DUGKS_F64> raw;
  load_raw<Q, DUGKS_F64>(raw, in, plane, (long long)j * pitch + i);
  double gc[Q], ftp[Q], phi;
  cell_g<Q, DUGKS_F64, NC>(I, eq, raw, sc, gc, ftp, true, phi);
  const double kx = cW[4], ky = rS[4];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double v = ftp[k];
    if (lat_cx(k) != 0) v = fma(-lat_cx(k) * kx, fE[k] - fW[k], v);
    if (lat_cy(k) != 0) v = fma(-lat_cy(k) * ky, fN[k] - fS[k], v);
    out[k * plane + (long long)j * pitch + i] = v;
  }
}

// -------------------------------------------------- init, encode, decode
// Equilibrium of phi in binary64 (eq. 2.3 through the per-direction polynomial).
template <int Q>
__device__ __forceinline__ void feq64(const InstDev* __restrict__ I, double phi, double* E) {
  const int nc = I->ncoef;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double r = I->e[k][nc - 1];
    for (int m = nc - 2; m >= 0; --m) r = fma(r, phi, I->e[k][m]);
    E[k] = r;
  }
}

// The conserved value of interior cell (i, j) at step `step` from s = sum f~:
// s without a source; with one the root of phi = s + dt F(x, t, phi) / 2 (eq.
// 2.25 summed with the moments of eq. 2.7), as the step kernel solves it.
__device__ __forceinline__ double src_cell_phi(const InstDev* __restrict__ I, int i, int j,
                                               long long step, double s) {
  if (I->src_n == 0) return s;
  const long long N = (long long)I->nx * I->ny;
  const double t = (double)step * I->dt;
  double a[kSrcPow] = {0.0, 0.0, 0.0, 0.0};
  for (int u = 0; u < I->src_n; ++u) {
    const double g = I->src_g[u * N + (long long)j * I->nx + i];
    const double e = exp(I->src_gam[u] * t);
    const int k = I->src_implicit ? I->src_pow[u] : 0;
    for (int m = 0; m < kSrcPow; ++m)
      if (m == k) a[m] = fma(e, g, a[m]);
  }
  return solve_conserved<kSrcPow, double>(s, I->half_dt, a, I->src_implicit != 0);
}

// 16-bit encode of f~ (binary64 values) at one cell.
template <int Q, int ST>
__device__ __forceinline__ void encode_neq(const InstDev* __restrict__ I, char* buf, long long off,
                                           const double* f, float s, float* maxdev) {
  double ps = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) ps += f[k];
  const float pf = (float)ps;
  const int nc = I->ncoef;
  float m = 0.0f;
  float sq[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    float E = I->ef[k][nc - 1];
    for (int mm = nc - 2; mm >= 0; --mm) E = fmaf(E, pf, I->ef[k][mm]);
    const float d = (float)(f[k] - (double)E);
    if (k > 0) m = fmaxf(m, fabsf(d));   // the stored directions
    sq[k] = d * s;
  }
  if (s > 0.0f) {
    unsigned* gb = (unsigned*)buf + I->plane;
#pragma unroll
    for (int p = 0; p < (Q - 1) / 2; ++p) gb[p * I->plane + off] = f32x2_to_g<ST>(sq[2 * p + 1], sq[2 * p + 2]);
    ((float*)buf)[off] = pf;
  }
  *maxdev = m;
}

template <int Q, int ST>
__global__ void k_init_eq(const InstDev* __restrict__ I, const double* __restrict__ phi, int parity) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= I->nx || j >= I->ny) return;
  const long long off = (long long)j * I->pitch + i;
  const double p = phi[(long long)j * I->nx + i];
  char* buf = (char*)I->buf[parity];
  if constexpr (!Stor<ST>::neq) {
    double E[Q];
    feq64<Q>(I, p, E);
    if (I->src_n > 0) {
      // f = E at t = 0 (Omega = 0): f~ = E - dt S / 2 with S_i = F(x, 0, phi)
      // rho_i(phi) (eq. 2.25), F(x, 0, phi) = sum_j phi^k_j G_j(x)
      const long long N = (long long)I->nx * I->ny;
      double F = 0.0;
      for (int t = 0; t < I->src_n; ++t) {
        double pk = 1.0;
        for (int m = 0; m < I->src_pow[t]; ++m) pk *= p;
        F += pk * I->src_g[t * N + (long long)j * I->nx + i];
      }
      const double px = horner<kRhoCoef>(I->bp[0], p), py = horner<kRhoCoef>(I->bp[1], p);
#pragma unroll
      for (int k = 0; k < Q; ++k)
        E[k] -= I->half_dt * F * lat_w<Q>(k) * (1.0 + lat_cx(k) * px + lat_cy(k) * py);
    }
    using T = typename Stor<ST>::T;
#pragma unroll
    for (int k = 0; k < Q; ++k) ((T*)buf)[k * I->plane + off] = (T)E[k];
  } else {
    // f~ = E(phi) exactly for the stored phi: g = 0
    ((float*)buf)[off] = (float)p;
    unsigned* gb = (unsigned*)buf + I->plane;
#pragma unroll
    for (int p2 = 0; p2 < (Q - 1) / 2; ++p2) gb[p2 * I->plane + off] = 0u;
  }
}

// pass 0: max_{i >= 1} |f~_i - E_i| into slots[slot]; pass 1: encode with that slot's scale
template <int Q, int ST>
__global__ void k_set_f(const InstDev* __restrict__ I, const double* __restrict__ f, int parity,
                        int pass, int slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  const bool in = i < I->nx && j < I->ny;
  const long long N = (long long)I->nx * I->ny;
  const long long off = (long long)j * I->pitch + i;
  char* buf = (char*)I->buf[parity];
  double v[Q];
  if (in) {
#pragma unroll
    for (int k = 0; k < Q; ++k) v[k] = f[k * N + (long long)j * I->nx + i];
  }
  if constexpr (!Stor<ST>::neq) {
    using T = typename Stor<ST>::T;
    if (in && pass == 1) {
#pragma unroll
      for (int k = 0; k < Q; ++k) ((T*)buf)[k * I->plane + off] = (T)v[k];
    }
  } else {
    float m = 0.0f;
    if (in) encode_neq<Q, ST>(I, buf, off, v, pass == 1 ? neq_scale_for<ST>(I->slots[slot]) : 0.0f, &m);
    if (pass == 0) {
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
      if ((threadIdx.x & 63) == 0 && m > 0.0f)
        atomicMax((unsigned*)(I->slots + slot), __float_as_uint(m));
    }
  }
}

// f~ of one cell in binary64
template <int Q, int ST>
__device__ __forceinline__ void decode(const InstDev* __restrict__ I, const char* buf, long long off,
                                       float inv_s, double* f) {
  if constexpr (!Stor<ST>::neq) {
    using T = typename Stor<ST>::T;
#pragma unroll
    for (int k = 0; k < Q; ++k) f[k] = (double)((const T*)buf)[k * I->plane + off];
  } else {
    const float p = ((const float*)buf)[off];
    const unsigned* gb = (const unsigned*)buf + I->plane;
    const int nc = I->ncoef;
    float gs = 0.0f;
    float g[Q];
#pragma unroll
    for (int p = 0; p < (Q - 1) / 2; ++p) {
      const unsigned u = gb[p * I->plane + off];
      g[2 * p + 1] = g_lo<ST>(u);
      g[2 * p + 2] = g_hi<ST>(u);
    }
#pragma unroll
    for (int k = 1; k < Q; ++k) gs += g[k];
    g[0] = -gs;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      float E = I->ef[k][nc - 1];
      for (int m = nc - 2; m >= 0; --m) E = fmaf(E, p, I->ef[k][m]);
      f[k] = (double)fmaf(g[k], inv_s, E);
    }
  }
}

template <int Q, int ST>
__global__ void k_get_phi(const InstDev* __restrict__ I, double* __restrict__ out, int parity,
                          long long step) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= I->nx || j >= I->ny) return;
  const long long off = (long long)j * I->pitch + i;
  const char* buf = (const char*)I->buf[parity];
  double phi;
  if constexpr (Stor<ST>::neq) {
    phi = (double)((const float*)buf)[off];  // the stored moment; sum g_i = 0 by construction
  } else {
    double f[Q];
    decode<Q, ST>(I, buf, off, 1.0f, f);
    phi = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) phi += f[k];
    phi = src_cell_phi(I, i, j, step, phi);
  }
  out[(long long)j * I->nx + i] = phi;
}

template <int Q, int ST>
__global__ void k_get_f(const InstDev* __restrict__ I, double* __restrict__ out, int parity,
                        long long step) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= I->nx || j >= I->ny) return;
  const long long off = (long long)j * I->pitch + i;
  const long long N = (long long)I->nx * I->ny;
  float inv_s = 1.0f;
  if constexpr (Stor<ST>::neq) inv_s = 1.0f / neq_scale_for<ST>(I->slots[(step + 2) & 3]);
  double f[Q];
  decode<Q, ST>(I, (const char*)I->buf[parity], off, inv_s, f);
#pragma unroll
  for (int k = 0; k < Q; ++k) out[k * N + (long long)j * I->nx + i] = f[k];
}

// ------------------------------------------------------------ reductions
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;
constexpr int kRedVals = 8;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int Q, int ST>
__global__ __launch_bounds__(kRedThreads) void k_reduce(const InstDev* __restrict__ I,
                                                        const double* __restrict__ ref, int parity,
                                                        long long step,
                                                        const double* __restrict__ widths,
                                                        double* __restrict__ partial) {
  const long long N = (long long)I->nx * I->ny;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const char* buf = (const char*)I->buf[parity];
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(n / I->nx), i = (int)(n - (long long)j * I->nx);
    const long long off = (long long)j * I->pitch + i;
    double phi;
    if constexpr (Stor<ST>::neq) {
      phi = (double)((const float*)buf)[off];
    } else {
      double f[Q];
      decode<Q, ST>(I, buf, off, 1.0f, f);
      phi = 0.0;
#pragma unroll
      for (int k = 0; k < Q; ++k) phi += f[k];
      phi = src_cell_phi(I, i, j, step, phi);
    }
    const double vol = widths[i] * widths[I->nx + j];
    if (!__builtin_isfinite(phi)) {
      acc[5] += 1.0;
      continue;
    }
    acc[0] += phi * vol;
    if (ref != nullptr) {
      const double r = ref[n], d = phi - r;
      acc[1] += fabs(d);
      acc[2] += fabs(r);
      acc[3] += d * d * vol;
      acc[4] += r * r * vol;
    }
  }
  __shared__ double sh[kRedThreads / 64][6];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    const double s = wave_sum(acc[v]);
    if (lane == 0) sh[w][v] = s;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double s = 0.0;
    for (int ww = 0; ww < kRedThreads / 64; ++ww) s += sh[ww][threadIdx.x];
    partial[blockIdx.x * kRedVals + threadIdx.x] = s;
  }
}

__global__ void k_reduce_final(const double* __restrict__ partial, int nblocks,
                               double* __restrict__ out) {
  // one thread per value, partials summed in block order: deterministic
  const int v = threadIdx.x;
  if (v >= kRedVals) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b * kRedVals + v];
  out[v] = s;
}

// Final pass of the allocation-free norms: the partial sums in block order (as
// k_reduce_final), then out[0] = relative L2, out[1] = GRE (eq. 4.1); NaN for
// both when some cell is not finite (those cells are left out of the sums).
__global__ void k_norms_final(const double* __restrict__ partial, int nblocks,
                              double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double r[6] = {0, 0, 0, 0, 0, 0};
  for (int v = 1; v < 6; ++v)
    for (int b = 0; b < nblocks; ++b) r[v] += partial[b * kRedVals + v];
  if (r[5] > 0) {
    out[0] = out[1] = __builtin_nan("");
    return;
  }
  out[0] = r[4] > 0 ? sqrt(r[3] / r[4]) : (r[3] > 0 ? INFINITY : 0.0);
  out[1] = r[2] > 0 ? r[1] / r[2] : (r[1] > 0 ? INFINITY : 0.0);
}

// Scratch of the allocation-free norms: kRedBlocks x kRedVals partial sums,
// fully rewritten by every call (nothing needs clearing).  One copy per GPU,
// held until the process ends; host code uses only the address returned by
// hipGetSymbolAddress, never the name.
constexpr int kScratchDoubles = kRedBlocks * kRedVals;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {nullptr};

// Address of the current device's scratch, looked up once per device.
static int scratch_ptr(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return -1;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

__global__ void k_set_i64(long long* p, long long v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void k_fill_u32(unsigned* p, unsigned v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// --------------------------------------------------------------- launch
static inline hipStream_t S(void* s) { return (hipStream_t)s; }

#define DUGKS_CHECK_LAUNCH() return hipGetLastError() == hipSuccess ? 0 : -1

template <int Q, int ST>
static int launch_step_q_st(const StepArgs& a, const Launch& l, void* stream, int measure) {
  const int wpb = l.waves_per_block;
  const int blocks_needed = (a.nitems + wpb - 1) / wpb;
  int blocks = blocks_needed;
  const int persistent = (l.schedule == DUGKS_SCHED_PERSISTENT && a.persistent_blocks > 0 &&
                          a.persistent_blocks < blocks_needed);
  if (persistent) blocks = a.persistent_blocks;
  if (blocks <= 0) return 0;
  dim3 grid(blocks), block(64 * wpb);
#define DUGKS_STEP_LAUNCH(NC_, NF_, SYM_)                                                          \
  hipLaunchKernelGGL((k_step<Q, ST, NC_, NF_, SYM_>), grid, block, 0, S(stream), a.insts, a.items, \
                     a.nitems, a.parity, a.step, l.xcd_remap, persistent, measure, a.step_base)
#define DUGKS_STEP_NC(NF_, SYM_)                          \
  switch (a.ncoef) {                                      \
    case 2: DUGKS_STEP_LAUNCH(2, NF_, SYM_); break;       \
    case 4: DUGKS_STEP_LAUNCH(4, NF_, SYM_); break;       \
    default: DUGKS_STEP_LAUNCH(8, NF_, SYM_); break;      \
  }
  if constexpr (Stor<ST>::neq) {   // bound by instructions: the symmetric variant pays most here
    if (a.src) return -1;  // sources run in binary64 / binary32 storage only
    if (a.sym) {
      DUGKS_STEP_NC(0, true);
    } else {
      DUGKS_STEP_NC(0, false);
    }
  } else if (a.src == kSrcPow) {
    DUGKS_STEP_NC(kSrcPow, false);
  } else if (a.src) {
    DUGKS_STEP_NC(1, false);
  } else if (a.sym && ST == DUGKS_F32) {   // binary32 without a source: a little faster too
    DUGKS_STEP_NC(0, true);
  } else {
    DUGKS_STEP_NC(0, false);
  }
#undef DUGKS_STEP_NC
#undef DUGKS_STEP_LAUNCH
  DUGKS_CHECK_LAUNCH();
}

template <int Q>
static int launch_plain_q(const StepArgs& a, int nx, int ny, void* stream) {
  dim3 grid((nx + 255) / 256, ny), block(256);
  switch (a.ncoef) {
    case 2:
      hipLaunchKernelGGL((k_step_plain<Q, 2>), grid, block, 0, S(stream), a.insts, a.parity, a.step);
      break;
    case 4:
      hipLaunchKernelGGL((k_step_plain<Q, 4>), grid, block, 0, S(stream), a.insts, a.parity, a.step);
      break;
    default:
      hipLaunchKernelGGL((k_step_plain<Q, 8>), grid, block, 0, S(stream), a.insts, a.parity, a.step);
      break;
  }
  DUGKS_CHECK_LAUNCH();
}

int launch_step_plain(const StepArgs& a, int nx, int ny, void* stream) {
  return a.q == 9 ? launch_plain_q<9>(a, nx, ny, stream) : launch_plain_q<5>(a, nx, ny, stream);
}

template <int Q>
static int launch_step_q(const StepArgs& a, const Launch& l, void* stream, int measure) {
  switch (a.storage) {
    case DUGKS_F64: return launch_step_q_st<Q, DUGKS_F64>(a, l, stream, measure);
    case DUGKS_F32: return launch_step_q_st<Q, DUGKS_F32>(a, l, stream, measure);
    case DUGKS_F16NEQ: return launch_step_q_st<Q, DUGKS_F16NEQ>(a, l, stream, measure);
    default: return launch_step_q_st<Q, DUGKS_BF16NEQ>(a, l, stream, measure);
  }
}

int launch_step_fused(const StepArgs& a, const Launch& l, void* stream, int measure) {
  return a.q == 9 ? launch_step_q<9>(a, l, stream, measure) : launch_step_q<5>(a, l, stream, measure);
}

int launch_clear_slot(const InstDev* insts, int ninst, long long step, int which, void* stream) {
  hipLaunchKernelGGL(k_clear_next_slot, dim3((ninst + 255) / 256), dim3(256), 0, S(stream), insts,
                     ninst, step, which);
  DUGKS_CHECK_LAUNCH();
}

template <int Q>
static int init_q(const InstDev* d, const InstDev& h, const double* phi, int parity, void* stream) {
  dim3 grid((h.nx + 255) / 256, h.ny), block(256);
  switch (h.storage) {
    case DUGKS_F64: hipLaunchKernelGGL((k_init_eq<Q, DUGKS_F64>), grid, block, 0, S(stream), d, phi, parity); break;
    case DUGKS_F32: hipLaunchKernelGGL((k_init_eq<Q, DUGKS_F32>), grid, block, 0, S(stream), d, phi, parity); break;
    case DUGKS_F16NEQ: hipLaunchKernelGGL((k_init_eq<Q, DUGKS_F16NEQ>), grid, block, 0, S(stream), d, phi, parity); break;
    default: hipLaunchKernelGGL((k_init_eq<Q, DUGKS_BF16NEQ>), grid, block, 0, S(stream), d, phi, parity); break;
  }
  DUGKS_CHECK_LAUNCH();
}
int launch_init_eq(const InstDev* d, const InstDev& h, const double* phi, int parity, void* stream) {
  return h.q == 9 ? init_q<9>(d, h, phi, parity, stream) : init_q<5>(d, h, phi, parity, stream);
}

template <int Q>
static int set_f_q(const InstDev* d, const InstDev& h, const double* f, int parity, int pass,
                   int slot, void* stream) {
  dim3 grid((h.nx + 255) / 256, h.ny), block(256);
  switch (h.storage) {
    case DUGKS_F64: hipLaunchKernelGGL((k_set_f<Q, DUGKS_F64>), grid, block, 0, S(stream), d, f, parity, pass, slot); break;
    case DUGKS_F32: hipLaunchKernelGGL((k_set_f<Q, DUGKS_F32>), grid, block, 0, S(stream), d, f, parity, pass, slot); break;
    case DUGKS_F16NEQ: hipLaunchKernelGGL((k_set_f<Q, DUGKS_F16NEQ>), grid, block, 0, S(stream), d, f, parity, pass, slot); break;
    default: hipLaunchKernelGGL((k_set_f<Q, DUGKS_BF16NEQ>), grid, block, 0, S(stream), d, f, parity, pass, slot); break;
  }
  DUGKS_CHECK_LAUNCH();
}
int launch_set_f_pass(const InstDev* d, const InstDev& h, const double* f, int parity, int pass,
                      int slot, void* stream) {
  return h.q == 9 ? set_f_q<9>(d, h, f, parity, pass, slot, stream)
                  : set_f_q<5>(d, h, f, parity, pass, slot, stream);
}

template <int Q>
static int get_phi_q(const InstDev* d, const InstDev& h, double* out, int parity, long long step,
                     void* stream) {
  dim3 grid((h.nx + 255) / 256, h.ny), block(256);
  switch (h.storage) {
    case DUGKS_F64: hipLaunchKernelGGL((k_get_phi<Q, DUGKS_F64>), grid, block, 0, S(stream), d, out, parity, step); break;
    case DUGKS_F32: hipLaunchKernelGGL((k_get_phi<Q, DUGKS_F32>), grid, block, 0, S(stream), d, out, parity, step); break;
    case DUGKS_F16NEQ: hipLaunchKernelGGL((k_get_phi<Q, DUGKS_F16NEQ>), grid, block, 0, S(stream), d, out, parity, step); break;
    default: hipLaunchKernelGGL((k_get_phi<Q, DUGKS_BF16NEQ>), grid, block, 0, S(stream), d, out, parity, step); break;
  }
  DUGKS_CHECK_LAUNCH();
}
int launch_get_phi(const InstDev* d, const InstDev& h, double* out, int parity, long long step,
                   void* stream) {
  return h.q == 9 ? get_phi_q<9>(d, h, out, parity, step, stream)
                  : get_phi_q<5>(d, h, out, parity, step, stream);
}

template <int Q>
static int get_f_q(const InstDev* d, const InstDev& h, double* out, int parity, long long step,
                   void* stream) {
  dim3 grid((h.nx + 255) / 256, h.ny), block(256);
  switch (h.storage) {
    case DUGKS_F64: hipLaunchKernelGGL((k_get_f<Q, DUGKS_F64>), grid, block, 0, S(stream), d, out, parity, step); break;
    case DUGKS_F32: hipLaunchKernelGGL((k_get_f<Q, DUGKS_F32>), grid, block, 0, S(stream), d, out, parity, step); break;
    case DUGKS_F16NEQ: hipLaunchKernelGGL((k_get_f<Q, DUGKS_F16NEQ>), grid, block, 0, S(stream), d, out, parity, step); break;
    default: hipLaunchKernelGGL((k_get_f<Q, DUGKS_BF16NEQ>), grid, block, 0, S(stream), d, out, parity, step); break;
  }
  DUGKS_CHECK_LAUNCH();
}
int launch_get_f(const InstDev* d, const InstDev& h, double* out, int parity, long long step,
                 void* stream) {
  return h.q == 9 ? get_f_q<9>(d, h, out, parity, step, stream)
                  : get_f_q<5>(d, h, out, parity, step, stream);
}

int reduce_partials() { return kRedBlocks; }

template <int Q>
static int reduce_q(const InstDev* d, const InstDev& h, const double* ref, int parity,
                    long long step, const double* widths, double* partial, void* stream) {
  dim3 grid(kRedBlocks), block(kRedThreads);
  switch (h.storage) {
    case DUGKS_F64: hipLaunchKernelGGL((k_reduce<Q, DUGKS_F64>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial); break;
    case DUGKS_F32: hipLaunchKernelGGL((k_reduce<Q, DUGKS_F32>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial); break;
    case DUGKS_F16NEQ: hipLaunchKernelGGL((k_reduce<Q, DUGKS_F16NEQ>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial); break;
    default: hipLaunchKernelGGL((k_reduce<Q, DUGKS_BF16NEQ>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial); break;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_reduce_widths(const InstDev* d, const InstDev& h, const double* ref, int parity,
                         long long step, const double* widths, double* partial, double* out,
                         void* stream) {
  int rc = h.q == 9 ? reduce_q<9>(d, h, ref, parity, step, widths, partial, stream)
                    : reduce_q<5>(d, h, ref, parity, step, widths, partial, stream);
  if (rc) return rc;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, S(stream), partial, kRedBlocks, out);
  DUGKS_CHECK_LAUNCH();
}

int launch_norms_noalloc(const InstDev* d, const InstDev& h, const double* ref, int parity,
                         long long step, const double* widths, double* out_dev, void* stream) {
  double* partial = nullptr;
  if (scratch_ptr(&partial)) return -2;
  int rc = h.q == 9 ? reduce_q<9>(d, h, ref, parity, step, widths, partial, stream)
                    : reduce_q<5>(d, h, ref, parity, step, widths, partial, stream);
  if (rc) return rc;
  hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(64), 0, S(stream), partial, kRedBlocks, out_dev);
  DUGKS_CHECK_LAUNCH();
}

int launch_set_i64(long long* p, long long v, void* stream) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, S(stream), p, v);
  DUGKS_CHECK_LAUNCH();
}

int launch_fill_u32(unsigned* p, unsigned v, long long n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, S(stream), p, v, n);
  DUGKS_CHECK_LAUNCH();
}

}  // namespace dugks

namespace dugks {
float neq_scale_host(int storage, float m) {
  return storage == DUGKS_BF16NEQ ? neq_scale_for<DUGKS_BF16NEQ>(m) : neq_scale_for<DUGKS_F16NEQ>(m);
}
}  // namespace dugks
