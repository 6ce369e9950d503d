// gfx950 kernels of the three-dimensional DUGKS step (Sec. 2) on D3Q15
// (eq. 2.28), D3Q19 (eq. 2.6) and D3Q7 (Remark 3).
//
// Fused step: a block owns a strip of 62 columns (64 lanes: one halo column
// each side), a tile of rows (one or two waves per row) and a chunk of planes, which
// it sweeps in z, with g of three planes of its rows and the two halo rows in
// LDS.  Per plane and cell it computes the west face (x; the east face is the
// next lane's west face), both y faces and the top face (z; the bottom face is
// the previous plane's top face) and the update.  x neighbours come from
// whole-wave DPP shifts, as in the 2-D kernels.  D3Q15 and D3Q19 (both
// storages) stage raw f~ through LDS with direct buffer-to-LDS loads and give
// each row two waves, one per half of the directions (k_step3p).  D3Q7, whose
// registers are no constraint, gives each row one wave: binary32 staged the
// same way (k_step3s), binary64 with its window in registers and one wave on
// each halo row (k_step3h).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dugks3d_internal.h"


namespace dugks3 {

// ------------------------------------------------------------------ lattice
// Integer directions: D3Q15 as the columns of eq. 2.28, D3Q19 as those of
// eq. 2.6; D3Q7 is the first seven of either.
__host__ __device__ constexpr int d3q15(int k, int a) {
  constexpr int t[15][3] = {{0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                            {0, 0, 1},   {0, 0, -1}, {1, 1, 1},  {1, 1, -1},  {1, -1, 1},
                            {-1, 1, 1},  {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}};
  return t[k][a];
}
__host__ __device__ constexpr int d3q19(int k, int a) {
  constexpr int t[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                            {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                            {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1},
                            {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  return t[k][a];
}
template <int Q> __host__ __device__ constexpr int ce(int k, int a) {
  return Q == 19 ? d3q19(k, a) : d3q15(k, a);
}
// the direction with component a reversed (specular mirror of a wall normal to a)
template <int Q> __host__ __device__ constexpr int mir(int k, int a) {
  for (int j = 0; j < Q; ++j) {
    bool same = true;
    for (int b = 0; b < 3; ++b)
      if (ce<Q>(j, b) != (b == a ? -ce<Q>(k, b) : ce<Q>(k, b))) same = false;
    if (same) return j;
  }
  return k;
}

// ---------------------------------------------------------------- storage
template <int ST> struct S3;
template <> struct S3<DUGKS_F64> { using T = double; };
template <> struct S3<DUGKS_F32> { using T = float; };

template <typename T> struct C3;
template <> struct C3<double> {
  __device__ static const double* e(const Inst3* I, int k) { return I->e[k]; }
  __device__ static double ra(const Inst3* I) { return I->ra; }
  __device__ static double rb(const Inst3* I) { return I->rb; }
  __device__ static double b1(const Inst3* I) { return I->b1; }
  __device__ static double kg(const Inst3* I) { return I->kg; }
  __device__ static double inv_b1(const Inst3* I) { return I->inv_b1; }
  __device__ static const double* geo(const Inst3* I, int a) { return I->geo[a]; }
};
template <> struct C3<float> {
  __device__ static const float* e(const Inst3* I, int k) { return I->ef[k]; }
  __device__ static float ra(const Inst3* I) { return I->raf; }
  __device__ static float rb(const Inst3* I) { return I->rbf; }
  __device__ static float b1(const Inst3* I) { return I->b1f; }
  __device__ static float kg(const Inst3* I) { return I->kgf; }
  __device__ static float inv_b1(const Inst3* I) { return I->inv_b1f; }
  __device__ static const float* geo(const Inst3* I, int a) { return I->geof[a]; }
};

template <int NC, typename T> __device__ __forceinline__ T horner(const T* c, T x) {
  T r = c[NC - 1];
#pragma unroll
  for (int m = NC - 2; m >= 0; --m) r = fma(r, x, c[m]);
  return r;
}

// Uniform reads through the constant address space become scalar loads.
template <typename T> using CPtr = const __attribute__((address_space(4))) T*;
template <typename T> __device__ __forceinline__ CPtr<T> as_constant(const T* p) { return (CPtr<T>)p; }
// global memory (plain vector loads and stores, not flat ones)
template <typename T> using GPtr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ GPtr<T> as_global(T* p) { return (GPtr<T>)p; }

// ------------------------------------------------------------ lane shifts
// wave_shr:1 -> lane l receives lane l-1; wave_shl:1 -> lane l receives lane l+1
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

// ------------------------------------------------------------ memory
typedef unsigned v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <int Q, typename T>
__device__ __forceinline__ void load_row(T* f, __amdgpu_buffer_rsrc_t R, unsigned plane, unsigned idx) {
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    if constexpr (sizeof(T) == 8)
      f[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(R, idx * 8u, (unsigned)k * plane * 8u, 0));
    else
      f[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(R, idx * 4u, (unsigned)k * plane * 4u, 0));
  }
}

__device__ __forceinline__ int src_index(int i, int n, int bc) {
  if (i >= 0 && i < n) return i;
  if (bc == DUGKS_BC_PERIODIC) {
    int w = i < 0 ? i + n : i - n;
    return w < 0 ? 0 : (w >= n ? n - 1 : w);
  }
  return i < 0 ? 0 : n - 1;
}

// ------------------------------------------------------------ cell and face
// E_i(phi) (eq. 2.3) evaluated from the instance's scalar table ...
template <int NC, typename T> struct EqScalar {
  const Inst3* __restrict__ I;
  __device__ __forceinline__ T operator()(int k, T x) const { return horner<NC>(C3<T>::e(I, k), x); }
};
// ... or from coefficients held in vector registers
template <int Q, int NC> struct EqVec {
  float c[Q][NC];
  __device__ __forceinline__ float operator()(int k, float x) const { return horner<NC>(c[k], x); }
};

// g = fbar+ / b1 = (a1/b1) f~ + E(phi) (eq. 2.21 over b1); phi in binary64,
// returned in the storage type.
template <int Q, typename T, typename EQ>
__device__ __forceinline__ T cell_g3(const Inst3* __restrict__ I, const EQ& E, const T* f, T* g) {
  double phi = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) phi += (double)f[k];
  const T p = (T)phi, ra = C3<T>::ra(I);
#pragma unroll
  for (int k = 0; k < Q; ++k) g[k] = fma(ra, f[k], E(k, p));
  return p;
}

// Dirichlet ghost by non-equilibrium extrapolation (the two-dimensional rule):
// fbar+_g = E(phi_g) + (fbar+_a - E(phi_a)), i.e. g_g = g_a + (E(phi_g) -
// E(phi_a)) / b1, for the directions k with sel(k); a is the interior cell
// whose g is in g (phi_a = pa), phi_g the step's data at the ghost (x, y, z).
template <int Q, typename T, typename EQ, typename SEL>
__device__ __forceinline__ void nee_ghost(const Inst3* __restrict__ I, const EQ& E, const double* ring, int x,
                                          int y, int z, T pa, T* g, SEL sel) {
  const int nx = I->n[0];
  const T pg = (T)ring[shell_index(nx, I->n[1], I->n[2], x < nx ? x : nx, y, z)];
  const T ib = C3<T>::inv_b1(I);
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (sel(k)) g[k] = fma(E(k, pg) - E(k, pa), ib, g[k]);
}
// any out-of-range axis of the cell (x wall, y wall, z index) with a Dirichlet wall
__device__ __forceinline__ bool dirichlet_ghost(const Inst3* __restrict__ I, bool wx, bool wy, int z) {
  return (wx && I->bc[0] == DUGKS_BC_DIRICHLET) || (wy && I->bc[1] == DUGKS_BC_DIRICHLET) ||
         ((z < 0 || z >= I->n[2]) && I->bc[2] == DUGKS_BC_DIRICHLET);
}

template <int Q, typename T> __device__ __forceinline__ void mirror(T* g, int a) {
  T t[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) t[k] = g[mir<Q>(k, a)];
#pragma unroll
  for (int k = 0; k < Q; ++k) g[k] = t[k];
}

template <int Q, typename T> __device__ __forceinline__ T dir_sum(const T* v) {
  if constexpr (sizeof(T) == 8) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) s += v[k];
    return s;
  } else {
    T t[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) t[k] = v[k];
#pragma unroll
    for (int w = 1; w < Q; w *= 2)
#pragma unroll
      for (int k = 0; k + w < Q; k += 2 * w) t[k] += t[k + w];
    return t[0];
  }
}

// tangential axes of a face normal to A, in increasing order
template <int A> constexpr int tan1() { return A == 0 ? 1 : 0; }
template <int A> constexpr int tan2() { return A == 2 ? 1 : 2; }

// Half-step interface distribution on a face normal to axis A (eq. 2.20,
// eq. 2.19 in the form of eq. 2.26) in the scaled form, the interface phi and
// F = f_b / b3 (eq. 2.22) for the directions with a normal component.
// t1, t2: sums of the two cells' central-difference numerators along the
// tangential axes tan1<A>, tan2<A>; tau1, tau2 their factors h c / (2 dist).
template <int Q, int A, typename T, typename EQ>
__device__ __forceinline__ void face3(const Inst3* __restrict__ I, const EQ& E, const T* L, const T* R,
                                      const T* t1, T tau1, const T* t2, T tau2, T am, T a0, T ap,
                                      T* out) {
  T gb[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int cn = ce<Q>(k, A), c1 = ce<Q>(k, tan1<A>()), c2 = ce<Q>(k, tan2<A>());
    const T al = cn > 0 ? ap : (cn < 0 ? am : a0);
    T v = fma(al, R[k] - L[k], L[k]);
    if (c1 != 0) v = fma((T)(-c1) * tau1, t1[k], v);
    if (c2 != 0) v = fma((T)(-c2) * tau2, t2[k], v);
    gb[k] = v;
  }
  const T pb = (T)(dir_sum<Q>(gb) * C3<T>::b1(I));
  const T rb = C3<T>::rb(I);
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (ce<Q>(k, A) != 0) out[k] = fma(rb, gb[k], E(k, pb));
}

// ------------------------------------------------------------- sources
// F(x, t, phi) = sum_j exp(gamma_j t) phi^k_j G_j(x) (k_j <= 3): its
// coefficients as a polynomial in phi at time t, each G_j interpolated as
// G_j(c0) + r (G_j(c1) - G_j(c0)) (r = 0: the centre of cell c0).
__device__ inline void src_coefs3(const Inst3* __restrict__ I, long long c0, long long c1, double r, double t,
                                  double* a) {
  for (int m = 0; m < 4; ++m) a[m] = 0.0;
  for (int j = 0; j < I->src_n; ++j) {
    const double g0 = I->src_g[j * I->src_plane + c0], g1 = I->src_g[j * I->src_plane + c1];
    a[I->src_pow[j]] += exp(I->src_gam[j] * t) * fma(r, g1 - g0, g0);
  }
}
template <typename T> __device__ inline T poly4(const T* a, T x) {
  return fma(fma(fma(a[3], x, a[2]), x, a[1]), x, a[0]);
}
// The conserved value v with v - tau F(v) / 2 = s (tau = dt in a cell, eq.
// 2.25; h at a face, eq. 2.27): explicit when F does not depend on phi, else
// Newton's method from v = s (binary64: update <= 1e-15 (1 + |v|), at most 8;
// binary32: 2.4e-7, at most 6).
template <typename T> __device__ inline T solve_conserved3(T s, T half_tau, const T* a, bool implicit) {
  if (!implicit) return fma(half_tau, a[0], s);
  constexpr bool dbl = sizeof(T) == 8;
  const T tol = dbl ? (T)1e-15 : (T)2.4e-7;
  T v = s;
#pragma unroll 1
  for (int it = 0; it < (dbl ? 8 : 6); ++it) {
    const T P = poly4(a, v);
    const T dP = fma(fma((T)3 * a[3], v, (T)2 * a[2]), v, a[1]);
    const T d = (v - half_tau * P - s) / ((T)1 - half_tau * dP);
    v -= d;
    if (!(fabs(d) > tol * ((T)1 + fabs(v)))) break;
  }
  return v;
}
// weights of D3Q19 (eq. 2.6), D3Q15 (eq. 2.28) and D3Q7 (Remark 3)
template <int Q> __host__ __device__ constexpr double w3(int k) {
  return Q == 19 ? (k == 0 ? 1.0 / 3.0 : (k <= 6 ? 1.0 / 18.0 : 1.0 / 36.0))
         : Q == 15 ? (k == 0 ? 2.0 / 9.0 : (k <= 6 ? 1.0 / 9.0 : 1.0 / 72.0))
                   : (k == 0 ? 0.0 : 1.0 / 6.0);
}
// S_k / F = w_k (1 + c_k.B'(phi) / c_s^2): F_k and R_k of eq. 2.3 and Remark 3
template <int Q> __device__ inline double rho3(const Inst3* __restrict__ I, int k, double phi) {
  double v = 1.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (ce<Q>(k, a) != 0) v += ce<Q>(k, a) * poly4(I->bp[a], phi);
  return w3<Q>(k) * v;
}
// The source terms' time factors exp(gamma_j t) at the cells' time t_n and at
// the faces' time t_n + h, computed on the host once a step and passed by value
struct SrcTab {
  double en[DUGKS_MAX_SRC_TERMS], ef[DUGKS_MAX_SRC_TERMS];
};
using STab = const SrcTab*;
// The source's coefficients as polynomials in phi at cell `cell` (index of
// [nz][ny][nx]): an at t_n (the cell's own phi), af at t_n + h (its faces)
// (the loads of the cell's G_j, then the sums from them)
__device__ __forceinline__ void src_load3(const Inst3* __restrict__ I, long long cell, double* g) {
  const GPtr<const double> G = as_global(I->src_g);
  const int n = I->src_n;
#pragma unroll
  for (int j = 0; j < DUGKS_MAX_SRC_TERMS; ++j)
    if (j < n) g[j] = G[j * I->src_plane + cell];
}
__device__ __forceinline__ void src_coefs_from3(const Inst3* __restrict__ I, STab tb, const double* g,
                                                double* an, double* af) {
  const int n = I->src_n;
#pragma unroll
  for (int m = 0; m < 4; ++m) an[m] = af[m] = 0.0;
  // branch-free in the power: a term adds its G_j times the time factor to
  // the coefficient of its power and zero times G_j to the others (the same
  // sums; branches on the power made the compiler copy the arrays)
#pragma unroll
  for (int j = 0; j < DUGKS_MAX_SRC_TERMS; ++j) {
    if (j < n) {
      const double gj = g[j];
      const int pw = I->src_pow[j];
      const double en = tb->en[j], ef = tb->ef[j];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        an[m] = fma(pw == m ? en : 0.0, gj, an[m]);
        af[m] = fma(pw == m ? ef : 0.0, gj, af[m]);
      }
    }
  }
}
__device__ __forceinline__ void src_cell_coefs3(const Inst3* __restrict__ I, STab tb, long long cell,
                                                double* an, double* af) {
  double g[DUGKS_MAX_SRC_TERMS];
  src_load3(I, cell, g);
  src_coefs_from3(I, tb, g, an, af);
}

// A face's coefficients in the storage type: each G_j interpolated linearly
// between the two cells' centres (afL, afR: the cells' af; r the face's factor)
template <typename T>
__device__ __forceinline__ void src_face_coefs3(const double* afL, const double* afR, T r, T* a) {
#pragma unroll
  for (int m = 0; m < 4; ++m) a[m] = (T)fma((double)r, afR[m] - afL[m], afL[m]);
}

// phi of interior cell `cell` at time t from the sum of its f~ (the root of
// phi = s + dt F(phi) / 2 with a source)
__device__ inline double src_phi3(const Inst3* __restrict__ I, long long cell, double s, double t) {
  if (I->src_n == 0) return s;
  double a[4];
  src_coefs3(I, cell, cell, 0.0, t, a);
  return solve_conserved3<double>(s, 0.5 * I->dt, a, I->src_implicit != 0);
}


extern __shared__ __align__(16) unsigned char dugks3_lds[];

// --------------------------------- fused step, binary64 storage (D3Q7)
// A block owns a strip of 62 columns (64 lanes: one halo column each side), a
// tile of `rows` rows plus one halo row each side (one wave per row) and a
// chunk of planes, which it sweeps in z.  Each wave keeps g of its row at
// planes z-1, z, z+1 in registers and publishes them to LDS (three plane
// slots); after a barrier every interior wave reads its neighbour rows from
// LDS and computes, for its cells, the west face (x), both y faces, the top
// face (z; the bottom one is the previous plane's top face) and the update,
// then a second barrier protects the slot the next plane overwrites.  At most
// 2 interior rows (4 waves): a wave may hold the whole register file of its
// SIMD.
template <int Q, int ST, int NC, bool WALLS>
__global__ __launch_bounds__(256) void k_step3h(const Inst3* __restrict__ I, int parity,
                                               const double* __restrict__ ring, int rows,
                                               int planes, int strips, int tiles) {
  using T = typename S3<ST>::T;
  T* lds = (T*)dugks3_lds;
  const int W = rows + 2;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int b = blockIdx.x;
  const int sx = b % strips;
  b /= strips;
  const int tj = b % tiles, tk = b / tiles;
  const int nx = I->n[0], ny = I->n[1], nz = I->n[2];
  const int bcx = I->bc[0], bcy = I->bc[1], bcz = I->bc[2];
  const int pitch = I->pitch;
  const unsigned plane = (unsigned)I->plane;
  const int x0 = sx * kCols, y0 = tj * rows, z0 = tk * planes;
  const int y1 = min(y0 + rows, ny), z1 = min(z0 + planes, nz);
  // this wave's row; waves past the tile's upper halo row repeat it
  const int rr = y0 - 1 + w;
  const int r = rr < y1 ? rr : y1;
  const bool inner = w >= 1 && rr < y1;
  const int c = x0 - 1 + lane;
  const int scol = src_index(c < nx + 1 ? c : nx, nx, bcx);
  const bool wall_x = (c < 0 || c >= nx) && bcx != DUGKS_BC_PERIODIC;
  const bool live = inner && lane >= 1 && lane <= kCols && c < nx;
  const int srow = src_index(r, ny, bcy);
  const bool wall_y = (r < 0 || r >= ny) && bcy != DUGKS_BC_PERIODIC;

  const __amdgpu_buffer_rsrc_t Rin = rsrc(I->buf[parity], I->buf_bytes);
  const __amdgpu_buffer_rsrc_t Rout = rsrc(I->buf[parity ^ 1], I->buf_bytes);

  // column factors (per lane), row factors (uniform), plane factors (uniform)
  const T* cg = C3<T>::geo(I, 0) + (long long)(c + 1 < nx + 1 ? c + 1 : nx + 1) * kGeo;
  const T cam = cg[0], ca0 = cg[1], cap = cg[2], ctau = cg[3], ck = cg[4];
  const CPtr<T> yg = as_constant(C3<T>::geo(I, 1));
  const CPtr<T> zg = as_constant(C3<T>::geo(I, 2));
  const int ryi = (r + 1 < ny + 1 ? r + 1 : ny + 1);   // table index of row r (clamped for idle waves)
  const T ytau = yg[ryi * kGeo + 3], ky = yg[ryi * kGeo + 4];
  const T yS0 = yg[ryi * kGeo + 0], yS1 = yg[ryi * kGeo + 1], yS2 = yg[ryi * kGeo + 2];
  const int ryn = (ryi + 1 < ny + 2 ? ryi + 1 : ny + 1);
  const T yN0 = yg[ryn * kGeo + 0], yN1 = yg[ryn * kGeo + 1], yN2 = yg[ryn * kGeo + 2];

  auto row_idx = [&](int zp) -> unsigned {
    return (unsigned)((src_index(zp, nz, bcz) * ny + srow) * pitch + scol);
  };
  auto make_g = [&](const T* f, int zp, T* g) {
    const T pa = cell_g3<Q, T>(I, EqScalar<NC, T>{I}, f, g);
    if constexpr (WALLS) {
      if (dirichlet_ghost(I, wall_x, wall_y, zp)) {
        nee_ghost<Q, T>(I, EqScalar<NC, T>{I}, ring, c, r, zp, pa, g, [](int) { return true; });
      } else {
        if (wall_x) mirror<Q, T>(g, 0);
        if (wall_y) mirror<Q, T>(g, 1);
        if ((zp < 0 || zp >= nz) && bcz != DUGKS_BC_PERIODIC) mirror<Q, T>(g, 2);
      }
    }
  };
  auto lds_at = [&](int slot, int row, int k) -> T* {
    return lds + ((long long)(slot * W + row) * Q + k) * kLanes + lane;
  };
  auto publish = [&](int slot, const T* g) {
#pragma unroll
    for (int k = 0; k < Q; ++k) *lds_at(slot, w, k) = g[k];
  };

  // Window slot of plane p: (p - z0) mod 3, for g (G), raw f~ (RW) and the top z-face (FZ).
  T G[3][Q], RW[3][Q], FZ[3][Q];

  // prologue: plane z0-1 in slot 2, plane z0 in slot 0, plane z0+1 loading into RW[1]
  load_row<Q, T>(RW[2], Rin, plane, row_idx(z0 - 1));
  load_row<Q, T>(RW[0], Rin, plane, row_idx(z0));
  load_row<Q, T>(RW[1], Rin, plane, row_idx(z0 + 1 <= z1 ? z0 + 1 : z1));
  make_g(RW[2], z0 - 1, G[2]);
  make_g(RW[0], z0, G[0]);
  publish(2, G[2]);
  publish(0, G[0]);
  __syncthreads();
  if (inner) {  // bottom face of plane z0 (between z0-1 and z0)
    T t1[Q], t2[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ce<Q>(k, 0) != 0)
        t1[k] = (shl1(G[2][k]) - shr1(G[2][k])) + (shl1(G[0][k]) - shr1(G[0][k]));
      if (ce<Q>(k, 1) != 0)
        t2[k] = (*lds_at(2, w + 1, k) - *lds_at(2, w - 1, k)) + (*lds_at(0, w + 1, k) - *lds_at(0, w - 1, k));
    }
    const int zi = z0 + 1;   // table index of the face between z0-1 and z0
    face3<Q, 2, T>(I, EqScalar<NC, T>{I}, G[2], G[0], t1, ctau, t2, ytau, zg[zi * kGeo + 0], zg[zi * kGeo + 1],
                       zg[zi * kGeo + 2], FZ[2]);
  }

  bool bad = false;
  auto body = [&](int z, auto slot) {
    constexpr int s0 = decltype(slot)::value, sp = (s0 + 1) % 3, sm = (s0 + 2) % 3;
    // plane z+1: g from the raw values in RW[sp]; plane z+2 starts loading
    load_row<Q, T>(RW[sm], Rin, plane, row_idx(z + 2 <= z1 ? z + 2 : z1));
    make_g(RW[sp], z + 1, G[sp]);
    publish(sp, G[sp]);
    __syncthreads();
    if (inner) {
      const int zi = z + 1;   // table index of plane z
      const T ztau = zg[zi * kGeo + 3], kz = zg[zi * kGeo + 4];
      // f~+ = (4/3) b1 g - f~ / 3 (eq. 2.23); the update (eq. 2.24) is
      // accumulated into o face by face
      const T kgv = C3<T>::kg(I);
      T o[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) o[k] = fma(kgv, G[s0][k], (T)(-1.0 / 3.0) * RW[s0][k]);
      T sx0[Q], dY[Q], dZ[Q], t1[Q], t2[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (ce<Q>(k, 0) != 0) sx0[k] = shl1(G[s0][k]) - shr1(G[s0][k]);
        if (ce<Q>(k, 1) != 0) dY[k] = *lds_at(s0, w + 1, k) - *lds_at(s0, w - 1, k);
        if (ce<Q>(k, 2) != 0) dZ[k] = G[sp][k] - *lds_at(sm, w, k);   // plane z-1 from LDS
      }
      {  // west face (x): left state from lane - 1; the east face is lane + 1's west face
        T lw[Q], fW[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          lw[k] = shr1(G[s0][k]);
          if (ce<Q>(k, 1) != 0) t1[k] = shr1(dY[k]) + dY[k];
          if (ce<Q>(k, 2) != 0) t2[k] = shr1(dZ[k]) + dZ[k];
        }
        face3<Q, 0, T>(I, EqScalar<NC, T>{I}, lw, G[s0], t1, ytau, t2, ztau, cam, ca0, cap, fW);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (ce<Q>(k, 0) != 0) o[k] = fma((T)(-ce<Q>(k, 0)) * ck, shl1(fW[k]) - fW[k], o[k]);
      }
      {  // north face (rows r, r+1)
        T gU[Q], fN[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          gU[k] = *lds_at(s0, w + 1, k);
          if (ce<Q>(k, 0) != 0) t1[k] = sx0[k] + (shl1(gU[k]) - shr1(gU[k]));
          if (ce<Q>(k, 2) != 0) t2[k] = dZ[k] + (*lds_at(sp, w + 1, k) - *lds_at(sm, w + 1, k));
        }
        face3<Q, 1, T>(I, EqScalar<NC, T>{I}, G[s0], gU, t1, ctau, t2, ztau, yN0, yN1, yN2, fN);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (ce<Q>(k, 1) != 0) o[k] = fma((T)(-ce<Q>(k, 1)) * ky, fN[k], o[k]);
      }
      {  // south face (rows r-1, r)
        T gD[Q], fS[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          gD[k] = *lds_at(s0, w - 1, k);
          if (ce<Q>(k, 0) != 0) t1[k] = sx0[k] + (shl1(gD[k]) - shr1(gD[k]));
          if (ce<Q>(k, 2) != 0) t2[k] = dZ[k] + (*lds_at(sp, w - 1, k) - *lds_at(sm, w - 1, k));
        }
        face3<Q, 1, T>(I, EqScalar<NC, T>{I}, gD, G[s0], t1, ctau, t2, ztau, yS0, yS1, yS2, fS);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (ce<Q>(k, 1) != 0) o[k] = fma((T)ce<Q>(k, 1) * ky, fS[k], o[k]);
      }
      {  // top face (planes z, z+1); the bottom face is the previous plane's top face
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if (ce<Q>(k, 0) != 0) t1[k] = sx0[k] + (shl1(G[sp][k]) - shr1(G[sp][k]));
          if (ce<Q>(k, 1) != 0) t2[k] = dY[k] + (*lds_at(sp, w + 1, k) - *lds_at(sp, w - 1, k));
        }
        const int zt = z + 2;   // table index of the face between z and z+1
        face3<Q, 2, T>(I, EqScalar<NC, T>{I}, G[s0], G[sp], t1, ctau, t2, ytau, zg[zt * kGeo + 0], zg[zt * kGeo + 1],
                           zg[zt * kGeo + 2], FZ[s0]);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (ce<Q>(k, 2) != 0) o[k] = fma((T)(-ce<Q>(k, 2)) * kz, FZ[s0][k] - FZ[sm][k], o[k]);
      }
      if (live) {
        bad |= !__builtin_isfinite(o[0]);
        const unsigned idx = (unsigned)(((long long)z * ny + r) * pitch + c);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, o[k]), Rout, idx * 8u,
                                                  (unsigned)k * plane * 8u, 0);
          else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, o[k]), Rout, idx * 4u,
                                                  (unsigned)k * plane * 4u, 0);
        }
      }
    }
    __syncthreads();   // the next plane overwrites slot sm
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  int z = z0;
  for (; z + 3 <= z1; z += 3) {
    body(z, S0{});
    body(z + 1, S1{});
    body(z + 2, S2{});
  }
  if (z < z1) body(z, S0{});
  if (z + 1 < z1) body(z + 1, S1{});
  (void)bad;
}

// --------------------------------- fused step, binary32 storage (D3Q7)
// A block of `ROWS` waves owns ROWS rows of a 62-column strip (one row per
// wave) and sweeps a chunk of planes in z.  Raw f~ of planes z+1 and z+2 is
// staged in LDS by direct buffer-to-LDS loads (no registers held while in
// flight): each wave loads its own row, and the two halo rows are split
// between all waves.  g of planes z-1, z, z+1 sits in three LDS slots; each
// wave keeps g of its row at z and z+1 and f~+ (eq. 2.23) of z in registers.
// Per plane: stage z+2, make g of z+1 (waves 0 and 1 also the halo rows),
// barrier, faces and update of plane z, barrier.

#define LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// Renumber them so that each XCD takes a contiguous run of (strip, tile,
// chunk) indices: neighbouring strips and tiles, which read each other's
// edge columns and halo rows, then run side by side under one L2.
__device__ __forceinline__ int xcd_contiguous(int b, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int x = b & 7, i = b >> 3;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Barrier for LDS traffic only: this wave's LDS reads and writes are complete,
// then the workgroup barrier.  Outstanding global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), vmcnt and expcnt unconstrained
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}
__device__ __forceinline__ void wait_vm_all() {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  asm volatile("" ::: "memory");
}

template <int Q, int NC, int ROWS, bool WALLS>
__global__ __launch_bounds__(64 * ROWS) void k_step3s(const Inst3* __restrict__ I, int parity,
                                                       const double* __restrict__ ring, int planes,
                                                       int strips, int tiles) {
  constexpr int W = ROWS + 2;                 // LDS rows: y0-1 .. y0+ROWS
  constexpr int HX = (2 * Q + ROWS - 1) / ROWS;   // halo-row loads per wave
  __shared__ float gsl[3][W][Q][kLanes];      // g of plane p in slot (p - z0) mod 3
  __shared__ float raw0[W][Q][kLanes];        // raw f~ of planes with (p - z0) even
  __shared__ float raw1[W][Q][kLanes];        // ... and odd
  __shared__ float ecoef[Q * NC];             // E_i coefficients, read into vector registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int b = xcd_contiguous(blockIdx.x, gridDim.x);
  const int sx = b % strips;
  b /= strips;
  const int tj = b % tiles, tk = b / tiles;
  const int nx = I->n[0], ny = I->n[1], nz = I->n[2];
  const int bcx = I->bc[0], bcy = I->bc[1], bcz = I->bc[2];
  const int pitch = I->pitch;
  const unsigned plane = (unsigned)I->plane;
  const int x0 = sx * kCols, y0 = tj * ROWS, z0 = tk * planes;
  const int y1 = min(y0 + ROWS, ny), z1 = min(z0 + planes, nz);
  // this wave's row (LDS row w + 1); in a short last tile the waves past it
  // take the upper halo row y1
  const int rr = y0 + w;
  const int r = rr < y1 ? rr : y1;
  const bool inner = rr < y1;
  const int me = w + 1;
  const int c = x0 - 1 + lane;
  const int scol = src_index(c < nx + 1 ? c : nx, nx, bcx);
  const bool wall_x = (c < 0 || c >= nx) && bcx != DUGKS_BC_PERIODIC;
  const bool live = inner && lane >= 1 && lane <= kCols && c < nx;
  const int srow = src_index(r, ny, bcy);
  const bool wall_y = (r < 0 || r >= ny) && bcy != DUGKS_BC_PERIODIC;
  // halo rows: y0-1 in LDS row 0 and y1 in LDS row W-1 (unused when the tile is short)
  const int slo = src_index(y0 - 1, ny, bcy), shi = src_index(y1, ny, bcy);
  const bool wall_lo = y0 - 1 < 0 && bcy != DUGKS_BC_PERIODIC;
  const bool wall_hi = y1 >= ny && bcy != DUGKS_BC_PERIODIC;

  const __amdgpu_buffer_rsrc_t Rin = rsrc(I->buf[parity], I->buf_bytes);
  const __amdgpu_buffer_rsrc_t Rout = rsrc(I->buf[parity ^ 1], I->buf_bytes);

  const float* cg = I->geof[0] + (long long)(c + 1 < nx + 1 ? c + 1 : nx + 1) * kGeo;
  const float cam = cg[0], ca0 = cg[1], cap = cg[2], ctau = cg[3], ck = cg[4];
  const CPtr<float> yg = as_constant(I->geof[1]);
  const CPtr<float> zg = as_constant(I->geof[2]);
  const int ryi = (r + 1 < ny + 1 ? r + 1 : ny + 1);
  const float ytau = yg[ryi * kGeo + 3], ky = yg[ryi * kGeo + 4];
  const float yS0 = yg[ryi * kGeo + 0], yS1 = yg[ryi * kGeo + 1], yS2 = yg[ryi * kGeo + 2];
  const int ryn = (ryi + 1 < ny + 2 ? ryi + 1 : ny + 1);
  const float yN0 = yg[ryn * kGeo + 0], yN1 = yg[ryn * kGeo + 1], yN2 = yg[ryn * kGeo + 2];
  const float kgv = I->kgf;
  const unsigned plane4 = plane * 4u;
  // E_i coefficients in vector registers for up to 4 per direction (filled
  // from ecoef after the first barrier), else read from the scalar table
  using EV = std::conditional_t<(NC <= 4), EqVec<Q, NC>, EqScalar<NC, float>>;
  EV ev;
  if constexpr (NC > 4) ev.I = I;
  if (w == 0)
    for (int i = lane; i < Q * NC; i += kLanes) ecoef[i] = I->ef[i / NC][i % NC];

  auto cell_index = [&](int sr, int zp) __attribute__((always_inline)) -> unsigned {
    return (unsigned)((src_index(zp, nz, bcz) * ny + sr) * pitch + scol);
  };
  // stage plane zp: this wave's row, and its share of the two halo rows
  // (per-direction offsets advance in a vector register: no scalar register per direction)
  auto stage = [&](float (*raw)[Q][kLanes], int zp) __attribute__((always_inline)) {
    unsigned o = cell_index(srow, zp) * 4u;
    const int wme = me;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      __builtin_amdgcn_raw_ptr_buffer_load_lds(Rin, LDS_PTR(&raw[wme][k][0]), 4, o, 0, 0, 0);
      o += plane4;
    }
    const unsigned ilo = cell_index(slo, zp) * 4u, ihi = cell_index(shi, zp) * 4u;
    const int j0 = w * HX;
#pragma unroll
    for (int t = 0; t < HX; ++t) {
      int j = j0 + t;
      j = j < 2 * Q ? j : j - 2 * Q;   // the few surplus loads repeat earlier ones
      const bool hi = j >= Q;
      const int k = hi ? j - Q : j;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(Rin, LDS_PTR(&raw[hi ? W - 1 : 0][k][0]), 4,
                                               (hi ? ihi : ilo) + (unsigned)k * plane4, 0, 0, 0);
    }
  };
  // yr: the row's index (-1..ny), for the Dirichlet data
  auto make_g = [&](const float (*raw)[Q][kLanes], int row, bool wy, int yr, int zp, float* g, float* f) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < Q; ++k) f[k] = raw[row][k][lane];
    const float pa = cell_g3<Q, float>(I, ev, f, g);
    if constexpr (WALLS) {
      if (dirichlet_ghost(I, wall_x, wy, zp)) {
        nee_ghost<Q, float>(I, ev, ring, c, yr, zp, pa, g, [](int) { return true; });
      } else {
        if (wall_x) mirror<Q, float>(g, 0);
        if (wy) mirror<Q, float>(g, 1);
        if ((zp < 0 || zp >= nz) && bcz != DUGKS_BC_PERIODIC) mirror<Q, float>(g, 2);
      }
    }
  };
  auto publish = [&](int slot, int row, const float* g) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < Q; ++k) gsl[slot][row][k][lane] = g[k];
  };
  // g of plane zp for this wave's row (G, and f~+ in FT) and, for waves 0 and
  // 1, the halo rows; all published to slot `slot`
  auto plane_g = [&](const float (*raw)[Q][kLanes], int zp, int slot, float* G, float* FT) __attribute__((always_inline)) {
    float f[Q];
    make_g(raw, me, wall_y, r, zp, G, f);
#pragma unroll
    for (int k = 0; k < Q; ++k) FT[k] = fmaf(kgv, G[k], (-1.0f / 3.0f) * f[k]);
    publish(slot, me, G);
    if (w <= 1) {
      float gx[Q];
      const int row = w == 0 ? 0 : W - 1;
      make_g(raw, row, w == 0 ? wall_lo : wall_hi, w == 0 ? y0 - 1 : y1, zp, gx, f);
      publish(slot, row, gx);
    }
  };

  float G0[Q], G1[Q], O[Q], FT1[Q], FZb[Q], FZt[Q];

  // prologue: planes z0-1 (raw1, slot 2) and z0 (raw0, slot 0); then z0+1 into raw1
  stage(raw1, z0 - 1);
  stage(raw0, z0);
  wait_vm_all();
  lds_barrier();
  if constexpr (NC <= 4) {
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int m = 0; m < NC; ++m) ev.c[k][m] = ecoef[k * NC + m];
  }
  plane_g(raw1, z0 - 1, 2, G1, FT1);
  plane_g(raw0, z0, 0, G0, O);
  lds_barrier();
  stage(raw1, z0 + 1);   // z1 >= z0 + 1
  if (inner) {  // bottom face of plane z0
    float t1[Q], t2[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (ce<Q>(k, 0) != 0)
        t1[k] = (shl1(G1[k]) - shr1(G1[k])) + (shl1(G0[k]) - shr1(G0[k]));
      if (ce<Q>(k, 1) != 0)
        t2[k] = (gsl[2][me + 1][k][lane] - gsl[2][me - 1][k][lane]) + (gsl[0][me + 1][k][lane] - gsl[0][me - 1][k][lane]);
    }
    const int zi = z0 + 1;
    face3<Q, 2, float>(I, ev, G1, G0, t1, ctau, t2, ytau, zg[zi * kGeo + 0], zg[zi * kGeo + 1],
                           zg[zi * kGeo + 2], FZb);
  }
  wait_vm_all();
  lds_barrier();

  auto body = [&](int z, auto rsl) __attribute__((always_inline)) {
    constexpr int RS = decltype(rsl)::value;   // raw slot of plane z+1
    float (*rawN)[Q][kLanes] = RS ? raw1 : raw0;
    float (*rawF)[Q][kLanes] = RS ? raw0 : raw1;
    const int d = z - z0;
    const int s0 = d % 3, sp = (d + 1) % 3, sm = (d + 2) % 3;
    plane_g(rawN, z + 1, sp, G1, FT1);
    if (z + 2 <= z1) stage(rawF, z + 2);
    lds_barrier();
    if (inner) {
      const int zi = z + 1;
      const float ztau = zg[zi * kGeo + 3], kz = zg[zi * kGeo + 4];
      float sx0[Q], dY[Q], dZ[Q], t1[Q], t2[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (ce<Q>(k, 0) != 0) sx0[k] = shl1(G0[k]) - shr1(G0[k]);
        if (ce<Q>(k, 1) != 0) dY[k] = gsl[s0][me + 1][k][lane] - gsl[s0][me - 1][k][lane];
        if (ce<Q>(k, 2) != 0) dZ[k] = G1[k] - gsl[sm][me][k][lane];
      }
      {  // west face (x); the east face is lane + 1's west face
        float lw[Q], fW[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          lw[k] = shr1(G0[k]);
          if (ce<Q>(k, 1) != 0) t1[k] = shr1(dY[k]) + dY[k];
          if (ce<Q>(k, 2) != 0) t2[k] = shr1(dZ[k]) + dZ[k];
        }
        face3<Q, 0, float>(I, ev, lw, G0, t1, ytau, t2, ztau, cam, ca0, cap, fW);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (ce<Q>(k, 0) != 0) O[k] = fmaf((float)(-ce<Q>(k, 0)) * ck, shl1(fW[k]) - fW[k], O[k]);
      }
      {  // north face (rows r, r+1)
        float gU[Q], fN[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          gU[k] = gsl[s0][me + 1][k][lane];
          if (ce<Q>(k, 0) != 0) t1[k] = sx0[k] + (shl1(gU[k]) - shr1(gU[k]));
          if (ce<Q>(k, 2) != 0) t2[k] = dZ[k] + (gsl[sp][me + 1][k][lane] - gsl[sm][me + 1][k][lane]);
        }
        face3<Q, 1, float>(I, ev, G0, gU, t1, ctau, t2, ztau, yN0, yN1, yN2, fN);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (ce<Q>(k, 1) != 0) O[k] = fmaf((float)(-ce<Q>(k, 1)) * ky, fN[k], O[k]);
      }
      {  // south face (rows r-1, r)
        float gD[Q], fS[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          gD[k] = gsl[s0][me - 1][k][lane];
          if (ce<Q>(k, 0) != 0) t1[k] = sx0[k] + (shl1(gD[k]) - shr1(gD[k]));
          if (ce<Q>(k, 2) != 0) t2[k] = dZ[k] + (gsl[sp][me - 1][k][lane] - gsl[sm][me - 1][k][lane]);
        }
        face3<Q, 1, float>(I, ev, gD, G0, t1, ctau, t2, ztau, yS0, yS1, yS2, fS);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (ce<Q>(k, 1) != 0) O[k] = fmaf((float)ce<Q>(k, 1) * ky, fS[k], O[k]);
      }
      {  // top face (planes z, z+1); the bottom face is the previous plane's top face
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if (ce<Q>(k, 0) != 0) t1[k] = sx0[k] + (shl1(G1[k]) - shr1(G1[k]));
          if (ce<Q>(k, 1) != 0) t2[k] = dY[k] + (gsl[sp][me + 1][k][lane] - gsl[sp][me - 1][k][lane]);
        }
        const int zt = z + 2;
        face3<Q, 2, float>(I, ev, G0, G1, t1, ctau, t2, ytau, zg[zt * kGeo + 0], zg[zt * kGeo + 1],
                               zg[zt * kGeo + 2], FZt);
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (ce<Q>(k, 2) != 0) O[k] = fmaf((float)(-ce<Q>(k, 2)) * kz, FZt[k] - FZb[k], O[k]);
      }
    }
    wait_vm_all();   // the staged plane z+2 is in LDS (and older stores are done)
    if (live) {
      unsigned o = (unsigned)(((long long)z * ny + r) * pitch + c) * 4u;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, O[k]), Rout, o, 0, 0);
        o += plane4;
      }
    }
    lds_barrier();   // the next plane overwrites slot sm and reads the staged rows
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      G0[k] = G1[k];
      O[k] = FT1[k];
      if (ce<Q>(k, 2) != 0) FZb[k] = FZt[k];
    }
  };
  using R0 = std::integral_constant<int, 0>;
  using R1 = std::integral_constant<int, 1>;
  int z = z0;
  for (; z + 2 <= z1; z += 2) {
    body(z, R1{});       // (z - z0) even: plane z+1 is in raw1
    body(z + 1, R0{});
  }
  if (z < z1) body(z, R1{});
}

// ------------------------------------ fused step, directions split in two
// The staged kernels above give one wave a whole row and need all of its
// directions in registers, so a wave fills its SIMD's register file and LDS
// limits a block to a few waves.  Here two waves share a row, each taking one
// half of the directions, closed under the wall mirrors (a wall reflection
// keeps which components of c_i are zero): the cell's phi is summed from all
// directions of the staged row in LDS, and the interface phi of each face
// (eq. 2.22) from the two halves' sums, exchanged through LDS.
template <int Q> __host__ __device__ constexpr int half_of(int k) {
  const int x = ce<Q>(k, 0), y = ce<Q>(k, 1), z = ce<Q>(k, 2);
  const int nnz = (x != 0) + (y != 0) + (z != 0);
  if (Q == 19) return (nnz == 1 || (x == 0 && nnz == 2)) ? 1 : 0;   // 9 + 10
  if (Q == 15) return nnz == 3 ? 1 : 0;                              // 7 + 8
  return (x == 0 && nnz == 1) ? 1 : 0;                               // 3 + 4
}
// Binary32 with 3 or more rows splits each row four ways.  D3Q19: {rest,
// (+-1,+-1,0)}, {(+-1,0,+-1)}, {(0,+-1,+-1)}, {axis directions}, closed
// under the wall mirrors.  D3Q15 only without walls (a z mirror moves a
// corner between the last two): {rest, +-x}, {+-y, +-z}, {corners with
// c_z = +1}, {corners with c_z = -1}.  Each half is two quarters.
// Binary64 at 2 rows does the same, with its halo rows loaded into
// registers instead of staged (the LDS holds the four-part sums instead).
template <int Q, typename T, int ROWS, bool WALLS> constexpr int parts() {
  constexpr bool quarters = Q == 19 || (Q == 15 && !WALLS);
  return (quarters && ((sizeof(T) == 4 && ROWS >= 3) || (sizeof(T) == 8 && ROWS == 2))) ? 4 : 2;
}
// rows of raw f~ staged in LDS: the tile's rows and its two halo rows, or,
// with four waves a row, only the tile's rows (each wave that makes a halo
// row loads its quarter of it into registers)
template <int Q, typename T, int ROWS, bool WALLS> constexpr int staged_rows() {
  return parts<Q, T, ROWS, WALLS>() == 4 ? ROWS : ROWS + 2;
}
template <int Q, int P> __host__ __device__ constexpr int part_of(int k) {
  if (P == 2) return half_of<Q>(k);
  const int x = ce<Q>(k, 0), y = ce<Q>(k, 1), z = ce<Q>(k, 2);
  const int nnz = (x != 0) + (y != 0) + (z != 0);
  if (Q == 15) {
    if (nnz == 3) return z > 0 ? 2 : 3;
    return (nnz == 0 || x != 0) ? 0 : 1;
  }
  if (nnz <= 1) return nnz == 0 ? 0 : 3;
  return z == 0 ? 0 : (y == 0 ? 1 : 2);
}
template <int Q, int P, int H> __host__ __device__ constexpr int part_count() {
  int n = 0;
  for (int k = 0; k < Q; ++k) n += part_of<Q, P>(k) == H;
  return n;
}

// pairwise sum over the directions d with sel(d) (short dependency chains)
template <int Q, int N, typename T, typename SEL> __device__ __forceinline__ T sel_sum(const T* v, SEL sel) {
  T t[N];
  int n = 0;
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (sel(k)) t[n++] = v[k];
#pragma unroll
  for (int w = 1; w < N; w *= 2)
#pragma unroll
    for (int j = 0; j + w < N; j += 2 * w) t[j] += t[j + w];
  return t[0];
}
// Sum over this part's directions.  D3Q19 and D3Q15 sum each of their four
// quarters pairwise, a half being quarters 0 + 1 or 2 + 3, so that the total
// over the parts, (q0 + q1) + (q2 + q3), is the same for two and for four parts.
template <int Q, int P, int H, typename T> __device__ __forceinline__ T part_sum(const T* v) {
  if constexpr (Q == 19 || Q == 15) {
    auto quarter = [&](auto jc) __attribute__((always_inline)) -> T {
      constexpr int J = decltype(jc)::value;
      return sel_sum<Q, part_count<Q, 4, J>()>(v, [](int k) { return part_of<Q, 4>(k) == J; });
    };
    using J0 = std::integral_constant<int, 0>;
    using J1 = std::integral_constant<int, 1>;
    using J2 = std::integral_constant<int, 2>;
    using J3 = std::integral_constant<int, 3>;
    if constexpr (P == 4) {
      if constexpr (H == 0) return quarter(J0{});
      else if constexpr (H == 1) return quarter(J1{});
      else if constexpr (H == 2) return quarter(J2{});
      else return quarter(J3{});
    } else if constexpr (H == 0) {
      return quarter(J0{}) + quarter(J1{});
    } else {
      return quarter(J2{}) + quarter(J3{});
    }
  } else {
    return sel_sum<Q, part_count<Q, P, H>()>(v, [](int k) { return part_of<Q, P>(k) == H; });
  }
}

template <int Q, int P, int H, typename T> __device__ __forceinline__ void mirror_part(T* g, int a) {
  T t[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (part_of<Q, P>(k) == H) t[k] = g[mir<Q>(k, a)];
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (part_of<Q, P>(k) == H) g[k] = t[k];
}

// face3 in two parts: the interface g of this part's directions and their
// sum, then F from the interface phi of the sum s over all parts
template <int Q, int P, int H, int A, typename T>
__device__ __forceinline__ T face_gb(const T* L, const T* R, const T* t1, T tau1, const T* t2, T tau2, T am,
                                     T a0, T ap, T* gb) {
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    if (part_of<Q, P>(k) != H) continue;
    const int cn = ce<Q>(k, A), c1 = ce<Q>(k, tan1<A>()), c2 = ce<Q>(k, tan2<A>());
    const T al = cn > 0 ? ap : (cn < 0 ? am : a0);
    T v = fma(al, R[k] - L[k], L[k]);
    if (c1 != 0) v = fma((T)(-c1) * tau1, t1[k], v);
    if (c2 != 0) v = fma((T)(-c2) * tau2, t2[k], v);
    gb[k] = v;
  }
  return part_sum<Q, P, H>(gb);
}
template <int Q, int P, int H, int A, typename T, typename EQ>
__device__ __forceinline__ void face_out(const Inst3* __restrict__ I, const EQ& E, const T* gb, T s, T* out) {
  const T pb = (T)(s * C3<T>::b1(I));
  const T rb = C3<T>::rb(I);
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (part_of<Q, P>(k) == H && ce<Q>(k, A) != 0) out[k] = fma(rb, gb[k], E(k, pb));
}

// The same with a source (eqs. 2.27 and 2.22 with F_b): phi_b solves phi_b =
// b1 sum gbar + h F(phi_b) / 2 with the face's coefficients sa, and F gains
// lambda F(phi_b) rho(phi_b)
// (phi_b and lambda F(phi_b) from the face's sum s, then F of part H from them)
template <typename T>
__device__ __forceinline__ void face_phi_src(const Inst3* __restrict__ I, T s, const T* sa, T& pb, T& lfb) {
  pb = (T)(s * C3<T>::b1(I));
  pb = solve_conserved3<T>(pb, (T)(0.25 * I->dt), sa, I->src_implicit != 0);
  lfb = (T)I->lambda * poly4(sa, pb);
}
template <int Q, int P, int H, int A, typename T, typename EQ>
__device__ __forceinline__ void face_out_phi(const Inst3* __restrict__ I, const EQ& E, const T* gb, T pb, T lfb,
                                             T* out) {
  const T rb = C3<T>::rb(I);
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (part_of<Q, P>(k) == H && ce<Q>(k, A) != 0)
      out[k] = fma(rb, gb[k], E(k, pb) + lfb * (T)rho3<Q>(I, k, (double)pb));
}
template <int Q, int P, int H, int A, typename T, typename EQ>
__device__ __forceinline__ void face_out_src(const Inst3* __restrict__ I, const EQ& E, const T* gb, T s, const T* sa,
                                             T* out) {
  T pb, lfb;
  face_phi_src<T>(I, s, sa, pb, lfb);
  face_out_phi<Q, P, H, A>(I, E, gb, pb, lfb, out);
}

// LDS bytes of a block with ns staging slots (E coefficients aside)
// LDS of a block with ns staging slots, the halo rows' phi sums (binary64,
// when those rows go through registers) included
template <int Q, int ROWS, typename T, bool WALLS> constexpr int lds_p_bytes(int ns) {
  return 3 * (ROWS + 2) * Q * kLanes * (int)sizeof(T) + ns * staged_rows<Q, T, ROWS, WALLS>() * Q * kLanes * (int)sizeof(T) +
         4 * ROWS * parts<Q, T, ROWS, WALLS>() * kLanes * (int)sizeof(T) +
         (staged_rows<Q, T, ROWS, WALLS>() == ROWS ? 2 * 4 * kLanes * 8 : 0);
}
template <int Q, int ROWS, typename T, bool WALLS> struct LdsP {
  static constexpr int W = ROWS + 2;             // LDS rows: y0-1 .. y0+ROWS
  static constexpr int WD = sizeof(T) / 4;       // words per element
  // staging slots: binary32 two, unless one slot lets two blocks share a
  // CU's 160 KiB where two slots would not; binary64 one
  static constexpr int NS = WD == 2 ? 1
                            : (lds_p_bytes<Q, ROWS, T, WALLS>(2) > 81920 && lds_p_bytes<Q, ROWS, T, WALLS>(1) <= 81920)
                                  ? 1
                                  : 2;
  // E coefficients in vector registers (from LDS) with two slots
  static constexpr bool kVecE = WD == 1 && NS == 2;
  static constexpr int RR = staged_rows<Q, T, ROWS, WALLS>();
  static constexpr bool kHD = RR == ROWS;        // halo rows loaded into registers
  T gsl[3][W][Q][kLanes];                        // g of plane p in slot (p - z0) mod 3
  unsigned raw[NS][RR][Q][WD][kLanes];           // staged f~, binary64 as low and high words
  T psum[4][ROWS][parts<Q, T, ROWS, WALLS>()][kLanes];   // the parts' interface-g sums of four faces
};

// One wave: row rw of the tile, directions of half H.  With two slots plane
// z+2 is staged into the second while plane z+1 is read from the first; one
// slot is refilled once every wave has read it.
template <int Q, int NC, int ROWS, typename T, int H, bool WALLS, bool SRC>
__device__ __forceinline__ void step3p_half(const Inst3* __restrict__ I, int parity,
                                            const double* __restrict__ ring, STab tb, int planes,
                                            int strips, int tiles, LdsP<Q, ROWS, T, WALLS>& L,
                                            const float* ecoef, double (*hphi)[4][kLanes], int w, int rw,
                                            int blk) {
  using LP = LdsP<Q, ROWS, T, WALLS>;
  constexpr int P = parts<Q, T, ROWS, WALLS>();
  constexpr int W = LP::W, WD = LP::WD;
  constexpr int NW = P * ROWS;                   // waves per block
  constexpr int HX = (2 * Q + NW - 1) / NW;      // halo-row loads per wave
  constexpr unsigned ES = sizeof(T);
  constexpr bool kVecE = LP::kVecE && NC <= 4;
  const int lane = threadIdx.x & 63;
  int b = blk;   // the block within its instance
  const int sx = b % strips;
  b /= strips;
  const int tj = b % tiles, tk = b / tiles;
  const int nx = I->n[0], ny = I->n[1], nz = I->n[2];
  const int bcx = I->bc[0], bcy = I->bc[1], bcz = I->bc[2];
  const int pitch = I->pitch;
  const unsigned plane = (unsigned)I->plane;
  const int x0 = sx * kCols, y0 = tj * ROWS, z0 = tk * planes;
  const int y1 = min(y0 + ROWS, ny), z1 = min(z0 + planes, nz);
  // this wave's row (LDS row rw + 1); in a short last tile the rows past it
  // take the upper halo row y1
  const int rr = y0 + rw;
  const int r = rr < y1 ? rr : y1;
  const bool inner = rr < y1;
  const int me = rw + 1;
  const int c = x0 - 1 + lane;
  const int scol = src_index(c < nx + 1 ? c : nx, nx, bcx);
  const bool wall_x = (c < 0 || c >= nx) && bcx != DUGKS_BC_PERIODIC;
  const bool live = inner && lane >= 1 && lane <= kCols && c < nx;
  const int srow = src_index(r, ny, bcy);
  const bool wall_y = (r < 0 || r >= ny) && bcy != DUGKS_BC_PERIODIC;
  // halo rows: y0-1 in LDS row 0 and y1 in LDS row W-1 (unused when the tile is short)
  const int slo = src_index(y0 - 1, ny, bcy), shi = src_index(y1, ny, bcy);
  const bool wall_lo = y0 - 1 < 0 && bcy != DUGKS_BC_PERIODIC;
  const bool wall_hi = y1 >= ny && bcy != DUGKS_BC_PERIODIC;

  const __amdgpu_buffer_rsrc_t Rin = rsrc(I->buf[parity], I->buf_bytes);
  const __amdgpu_buffer_rsrc_t Rout = rsrc(I->buf[parity ^ 1], I->buf_bytes);

  const T* cg = C3<T>::geo(I, 0) + (long long)(c + 1 < nx + 1 ? c + 1 : nx + 1) * kGeo;
  const T cam = cg[0], ca0 = cg[1], cap = cg[2], ctau = cg[3], ck = cg[4];
  const CPtr<T> yg = as_constant(C3<T>::geo(I, 1));
  const CPtr<T> zg = as_constant(C3<T>::geo(I, 2));
  const int ryi = (r + 1 < ny + 1 ? r + 1 : ny + 1);
  const T ytau = yg[ryi * kGeo + 3], ky = yg[ryi * kGeo + 4];
  const T yS0 = yg[ryi * kGeo + 0], yS1 = yg[ryi * kGeo + 1], yS2 = yg[ryi * kGeo + 2];
  const int ryn = (ryi + 1 < ny + 2 ? ryi + 1 : ny + 1);
  const T yN0 = yg[ryn * kGeo + 0], yN1 = yg[ryn * kGeo + 1], yN2 = yg[ryn * kGeo + 2];
  const T kgv = C3<T>::kg(I);
  const unsigned planeB = plane * ES;
  using EV = std::conditional_t<kVecE, EqVec<Q, NC>, EqScalar<NC, T>>;
  EV ev;
  if constexpr (!kVecE) ev.I = I;

  auto cell_index = [&](int sr, int zp) __attribute__((always_inline)) -> unsigned {
    return (unsigned)((src_index(zp, nz, bcz) * ny + sr) * pitch + scol);
  };
  // stage plane zp: this wave's directions of its row, and its share of the
  // two halo rows (offsets advance in a vector register)
  T HR[LP::kHD ? Q : 1];   // raw f~ of this wave's quarter of the halo row it makes, when not staged
  auto stage = [&](int slot, int zp) __attribute__((always_inline)) {
    unsigned o = cell_index(srow, zp) * ES;
    const int wme = LP::kHD ? me - 1 : me;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (part_of<Q, P>(k) == H) {
#pragma unroll
        for (int h = 0; h < WD; ++h)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(Rin, LDS_PTR(&L.raw[slot][wme][k][h][0]), 4, o + 4u * h, 0, 0, 0);
      }
      o += planeB;
    }
    if constexpr (LP::kHD) {
      if (rw <= 1) {   // this wave's quarter of the halo row, into registers
        unsigned oh = cell_index(rw == 0 ? slo : shi, zp) * ES;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if (part_of<Q, P>(k) == H) {
            if constexpr (WD == 2)
              HR[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(Rin, oh, 0u, 0));
            else
              HR[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(Rin, oh, 0u, 0));
          }
          oh += planeB;
        }
      }
      return;
    }
    const unsigned ilo = cell_index(slo, zp) * ES, ihi = cell_index(shi, zp) * ES;
    const int j0 = w * HX;
#pragma unroll
    for (int t = 0; t < HX; ++t) {
      int j = j0 + t;
      j = j < 2 * Q ? j : j - 2 * Q;   // the few surplus loads repeat earlier ones
      const bool hi = j >= Q;
      const int k = hi ? j - Q : j;
      const unsigned oh = (hi ? ihi : ilo) + (unsigned)k * planeB;
#pragma unroll
      for (int h = 0; h < WD; ++h)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(Rin, LDS_PTR(&L.raw[slot][hi ? W - 1 : 0][k][h][0]), 4,
                                                 oh + 4u * h, 0, 0, 0);
    }
  };
  // raw f~ of LDS row `row` (g numbering; with the halo rows in registers
  // only the tile's rows are staged)
  auto raw_at = [&](int slot, int row, int k) __attribute__((always_inline)) -> T {
    const int rr = LP::kHD ? row - 1 : row;
    if constexpr (WD == 1)
      return __builtin_bit_cast(float, L.raw[slot][rr][k][0][lane]);
    else
      return __builtin_bit_cast(double, (unsigned long long)L.raw[slot][rr][k][0][lane] |
                                            ((unsigned long long)L.raw[slot][rr][k][1][lane] << 32));
  };
  // g = fbar+ / b1 (eq. 2.21 over b1) of this half's directions; phi (binary64) from all of them
  // (fromreg: the raw values are the halo row's in HR)
  // yr: the row's index (-1..ny), for the Dirichlet data
  // With a source: phi solves phi = sum f~ + dt F(phi) / 2 (eq. 2.25) and g
  // gains lambda F(phi) rho(phi); afo receives the cell's coefficients at t_n + h
  // (from the cell's G_j in gin when given, else loaded here).
  // binary64 with a source and four parts (two waves a SIMD) issues the
  // loads of the source's G_j early (registers allow it there)
  constexpr bool kPreG = SRC && sizeof(T) == 8 && P == 4;
  auto make_g = [&](int slot, int row, bool wy, int yr, int zp, T* g, T* f, auto fromreg,
                    double* afo, const double* gin) __attribute__((always_inline)) {
    constexpr bool kReg = decltype(fromreg)::value;
    // phi in binary64 as (q0 + q1) + (q2 + q3), qj the sum over quarter j in
    // index order (four chains); a halo row in registers takes the quarters'
    // sums from LDS
    double phi;
    if constexpr (kReg) {
#pragma unroll
      for (int k = 0; k < Q; ++k)
        if (part_of<Q, P>(k) == H) f[k] = HR[k];
      const int hr = rw;   // 0: the lower halo row, 1: the upper
      phi = (hphi[hr][0][lane] + hphi[hr][1][lane]) + (hphi[hr][2][lane] + hphi[hr][3][lane]);
    } else {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const T v = raw_at(slot, row, k);
        acc[part_of<Q, 4>(k)] += (double)v;
        if (part_of<Q, P>(k) == H) f[k] = v;
      }
      phi = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
    double lf = 0.0;
    if constexpr (SRC) {
      const long long cell = ((long long)src_index(zp, nz, bcz) * ny + src_index(yr, ny, bcy)) * nx + scol;
      double an[4];
      if (gin) src_coefs_from3(I, tb, gin, an, afo);
      else src_cell_coefs3(I, tb, cell, an, afo);
      phi = solve_conserved3<double>(phi, 0.5 * I->dt, an, I->src_implicit != 0);
      lf = I->lambda * poly4(an, phi);
    }
    const T p = (T)phi, ra = C3<T>::ra(I);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (part_of<Q, P>(k) != H) continue;
      if constexpr (SRC) g[k] = fma(ra, f[k], ev(k, p) + (T)(lf * rho3<Q>(I, k, phi)));
      else g[k] = fma(ra, f[k], ev(k, p));
    }
    if constexpr (WALLS) {
      if (dirichlet_ghost(I, wall_x, wy, zp)) {
        nee_ghost<Q, T>(I, ev, ring, c, yr, zp, p, g, [](int k) { return part_of<Q, P>(k) == H; });
      } else {
        if (wall_x) mirror_part<Q, P, H, T>(g, 0);
        if (wy) mirror_part<Q, P, H, T>(g, 1);
        if ((zp < 0 || zp >= nz) && bcz != DUGKS_BC_PERIODIC) mirror_part<Q, P, H, T>(g, 2);
      }
    }
  };
  auto publish = [&](int slot, int row, const T* g) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (part_of<Q, P>(k) == H) L.gsl[slot][row][k][lane] = g[k];
  };
  // g of plane zp for this wave's row (G, and f~+ in FT) and, for the waves
  // of rows 0 and 1, the halo rows; all published to slot `slot`
  // halo rows in registers: this wave's quarter sum of the cell phi of its
  // halo row, to LDS (the loads must have completed; a barrier before use)
  auto halo_sums = [&]() __attribute__((always_inline)) {
    if constexpr (LP::kHD) {
      if (rw <= 1) {
        double q = 0.0;
#pragma unroll
        for (int k = 0; k < Q; ++k)
          if (part_of<Q, P>(k) == H) q += (double)HR[k];
        hphi[rw][H][lane] = q;
      }
    }
  };
  auto plane_g = [&](int rs, int zp, int slot, T* G, T* FT, double* AF) __attribute__((always_inline)) {
    using Staged = std::integral_constant<bool, false>;
    using Halo = std::integral_constant<bool, LP::kHD>;
    T f[Q];
    double afx[4];   // a halo row's coefficients (not kept)
    // binary64 with a source, four parts: the G_j of this wave's row and of
    // its halo row are loaded before either is used
    double gme[DUGKS_MAX_SRC_TERMS], gho[DUGKS_MAX_SRC_TERMS];
    if constexpr (kPreG) {
      const long long zr = (long long)src_index(zp, nz, bcz) * ny;
      src_load3(I, (zr + src_index(r, ny, bcy)) * nx + scol, gme);
      if (rw <= 1) src_load3(I, (zr + src_index(rw == 0 ? y0 - 1 : y1, ny, bcy)) * nx + scol, gho);
    }
    make_g(rs, me, wall_y, r, zp, G, f, Staged{}, AF, kPreG ? gme : nullptr);
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (part_of<Q, P>(k) == H) FT[k] = fma(kgv, G[k], (T)(-1.0 / 3.0) * f[k]);
    publish(slot, me, G);
    if (rw <= 1) {
      T gx[Q];
      const int row = rw == 0 ? 0 : W - 1;
      make_g(rs, row, rw == 0 ? wall_lo : wall_hi, rw == 0 ? y0 - 1 : y1, zp, gx, f, Halo{}, afx,
             kPreG ? gho : nullptr);
      publish(slot, row, gx);
      if (ROWS == 1) {  // one row: its waves make both halo rows (always staged)
        make_g(rs, W - 1, wall_hi, y1, zp, gx, f, Staged{}, afx, nullptr);
        publish(slot, W - 1, gx);
      }
    }
  };
  auto put_sum = [&](int face, T s) __attribute__((always_inline)) { L.psum[face][rw][H][lane] = s; };
  // the sum over all parts: p0 + p1, or (p0 + p1) + (p2 + p3); every part
  // forms the same value
  auto total = [&](int face, T mine) __attribute__((always_inline)) -> T {
    T v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = q == H ? mine : L.psum[face][rw][q][lane];
    if constexpr (P == 4) return (v[0] + v[1]) + (v[2] + v[3]);
    else return v[0] + v[1];
  };

  T G0[Q], G1[Q], O[Q], FT1[Q], FZb[Q], FZt[Q];
  double AF0[4], AF1[4];   // with a source: the own row's face coefficients at planes z and z+1
  // one part of the pipeline differs: binary32 stages plane z+2 before the
  // first barrier of plane z (other slot), binary64 after it (same slot)
  constexpr bool two = LP::NS == 2;

  // prologue: planes z0-1 (slot 2 of g) and z0 (slot 0), plane z0+1 staged,
  // the bottom face of plane z0
  if constexpr (two && LP::kHD) {   // one plane of halo registers: planes one at a time
    stage(1, z0 - 1);
    wait_vm_all();
    halo_sums();
    lds_barrier();
    if constexpr (kVecE) {
#pragma unroll
      for (int k = 0; k < Q; ++k)
        if (part_of<Q, P>(k) == H)
#pragma unroll
          for (int m = 0; m < NC; ++m) ev.c[k][m] = ecoef[k * NC + m];
    }
    plane_g(1, z0 - 1, 2, G1, FT1, AF1);
    lds_barrier();
    stage(0, z0);
    wait_vm_all();
    halo_sums();
    lds_barrier();
    plane_g(0, z0, 0, G0, O, AF0);
    lds_barrier();
    stage(1, z0 + 1);   // z1 >= z0 + 1
  } else if constexpr (two) {
    stage(1, z0 - 1);
    stage(0, z0);
    wait_vm_all();
    lds_barrier();
    if constexpr (kVecE) {
#pragma unroll
      for (int k = 0; k < Q; ++k)
        if (part_of<Q, P>(k) == H)
#pragma unroll
          for (int m = 0; m < NC; ++m) ev.c[k][m] = ecoef[k * NC + m];
    }
    plane_g(1, z0 - 1, 2, G1, FT1, AF1);
    plane_g(0, z0, 0, G0, O, AF0);
    lds_barrier();
    stage(1, z0 + 1);   // z1 >= z0 + 1
  } else {
    stage(0, z0 - 1);
    wait_vm_all();
    halo_sums();
    lds_barrier();
    plane_g(0, z0 - 1, 2, G1, FT1, AF1);
    lds_barrier();
    stage(0, z0);
    wait_vm_all();
    halo_sums();
    lds_barrier();
    plane_g(0, z0, 0, G0, O, AF0);
    lds_barrier();
    stage(0, z0 + 1);
  }
  T gbB[Q], sB = 0;
  const int zb = z0 + 1;
  if (inner) {  // bottom face of plane z0
    T t1[Q], t2[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (part_of<Q, P>(k) != H) continue;
      if (ce<Q>(k, 0) != 0)
        t1[k] = (shl1(G1[k]) - shr1(G1[k])) + (shl1(G0[k]) - shr1(G0[k]));
      if (ce<Q>(k, 1) != 0)
        t2[k] = (L.gsl[2][me + 1][k][lane] - L.gsl[2][me - 1][k][lane]) +
                (L.gsl[0][me + 1][k][lane] - L.gsl[0][me - 1][k][lane]);
    }
    sB = face_gb<Q, P, H, 2>(G1, G0, t1, ctau, t2, ytau, (T)zg[zb * kGeo + 0], (T)zg[zb * kGeo + 1],
                          (T)zg[zb * kGeo + 2], gbB);
    put_sum(0, sB);
  }
  lds_barrier();
  if (inner) {
    if constexpr (SRC) {
      T sa[4];
      src_face_coefs3<T>(AF1, AF0, (T)zg[zb * kGeo + 1], sa);
      face_out_src<Q, P, H, 2>(I, ev, gbB, total(0, sB), sa, FZb);
    } else {
      face_out<Q, P, H, 2>(I, ev, gbB, total(0, sB), FZb);
    }
  }
  wait_vm_all();
  halo_sums();   // plane z0+1
  lds_barrier();

  auto body = [&](int z, auto rsl) __attribute__((always_inline)) {
    constexpr int RS = decltype(rsl)::value;   // staging slot of plane z+1
    const int d = z - z0;
    const int s0 = d % 3, sp = (d + 1) % 3, sm = (d + 2) % 3;
    plane_g(RS, z + 1, sp, G1, FT1, AF1);
    if constexpr (two) {
      if (z + 2 <= z1) stage(1 - RS, z + 2);
      lds_barrier();
    } else {
      lds_barrier();   // every wave has read plane z+1 from the slot
      if (z + 2 <= z1) stage(0, z + 2);
    }
    T gbW[Q], gbN[Q], gbS[Q], gbT[Q], sW = 0, sN = 0, sS = 0, sT = 0;
    // binary64 with a source, four parts: the parts that solve the north and
    // south faces load the G_j of that neighbouring row here, so that the
    // face work below hides the loads' latency (used after the next barrier)
    double gpre[DUGKS_MAX_SRC_TERMS];
    if constexpr (kPreG && (H == 1 || H == 2)) {
      if (inner)
        src_load3(I, ((long long)src_index(z, nz, bcz) * ny + src_index(H == 1 ? r + 1 : r - 1, ny, bcy)) * nx + scol,
                  gpre);
    }
    if (inner) {
      T sx0[Q], dY[Q], dZ[Q], t1[Q], t2[Q];
      const int zi = z + 1;
      const T ztau = zg[zi * kGeo + 3];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (part_of<Q, P>(k) != H) continue;
        if (ce<Q>(k, 0) != 0) sx0[k] = shl1(G0[k]) - shr1(G0[k]);
        if (ce<Q>(k, 1) != 0) dY[k] = L.gsl[s0][me + 1][k][lane] - L.gsl[s0][me - 1][k][lane];
        if (ce<Q>(k, 2) != 0) dZ[k] = G1[k] - L.gsl[sm][me][k][lane];
      }
      {  // west face (x); the east face is lane + 1's west face
        T lw[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if (part_of<Q, P>(k) != H) continue;
          lw[k] = shr1(G0[k]);
          if (ce<Q>(k, 1) != 0) t1[k] = shr1(dY[k]) + dY[k];
          if (ce<Q>(k, 2) != 0) t2[k] = shr1(dZ[k]) + dZ[k];
        }
        sW = face_gb<Q, P, H, 0>(lw, G0, t1, ytau, t2, ztau, cam, ca0, cap, gbW);
      }
      {  // north face (rows r, r+1)
        T gU[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if (part_of<Q, P>(k) != H) continue;
          gU[k] = L.gsl[s0][me + 1][k][lane];
          if (ce<Q>(k, 0) != 0) t1[k] = sx0[k] + (shl1(gU[k]) - shr1(gU[k]));
          if (ce<Q>(k, 2) != 0) t2[k] = dZ[k] + (L.gsl[sp][me + 1][k][lane] - L.gsl[sm][me + 1][k][lane]);
        }
        sN = face_gb<Q, P, H, 1>(G0, gU, t1, ctau, t2, ztau, yN0, yN1, yN2, gbN);
      }
      {  // south face (rows r-1, r)
        T gD[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if (part_of<Q, P>(k) != H) continue;
          gD[k] = L.gsl[s0][me - 1][k][lane];
          if (ce<Q>(k, 0) != 0) t1[k] = sx0[k] + (shl1(gD[k]) - shr1(gD[k]));
          if (ce<Q>(k, 2) != 0) t2[k] = dZ[k] + (L.gsl[sp][me - 1][k][lane] - L.gsl[sm][me - 1][k][lane]);
        }
        sS = face_gb<Q, P, H, 1>(gD, G0, t1, ctau, t2, ztau, yS0, yS1, yS2, gbS);
      }
      {  // top face (planes z, z+1); the bottom face is the previous plane's top face
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          if (part_of<Q, P>(k) != H) continue;
          if (ce<Q>(k, 0) != 0) t1[k] = sx0[k] + (shl1(G1[k]) - shr1(G1[k]));
          if (ce<Q>(k, 1) != 0) t2[k] = dY[k] + (L.gsl[sp][me + 1][k][lane] - L.gsl[sp][me - 1][k][lane]);
        }
        const int zt = z + 2;
        sT = face_gb<Q, P, H, 2>(G0, G1, t1, ctau, t2, ytau, (T)zg[zt * kGeo + 0], (T)zg[zt * kGeo + 1],
                              (T)zg[zt * kGeo + 2], gbT);
      }
      put_sum(0, sW);
      put_sum(1, sN);
      put_sum(2, sS);
      put_sum(3, sT);
    }
    wait_vm_all();   // this wave's loads of plane z+2 (and its older stores) are done
    if (z + 2 <= z1) halo_sums();
    // both halves' sums and the whole staged plane z+2 are in LDS; slot sm
    // (read only above) is free for the next plane's g
    lds_barrier();
    if constexpr (SRC) {
      // Each part solves phi_b of 4 / P of the four faces (west, north,
      // south, top) and writes it with lambda F(phi_b) over the face's sums,
      // which only that part reads; after a barrier every part reads all
      // four.  The coefficients of the neighbouring rows at plane z are
      // loaded, the west cell's taken from lane - 1.
      if (inner) {
        constexpr int FP = 4 / P;
        auto put_phi = [&](int face, T pb, T lf) __attribute__((always_inline)) {
          L.psum[face][rw][0][lane] = pb;
          L.psum[face][rw][1][lane] = lf;
        };
        const long long cz = (long long)src_index(z, nz, bcz) * ny;
        T sa[4], pb, lf;
        if constexpr (0 / FP == H) {
          double AFW[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) AFW[m] = shr1(AF0[m]);
          src_face_coefs3<T>(AFW, AF0, ca0, sa);
          face_phi_src<T>(I, total(0, sW), sa, pb, lf);
          put_phi(0, pb, lf);
        }
        if constexpr (1 / FP == H) {
          double AFN[4], an[4];
          if constexpr (kPreG) src_coefs_from3(I, tb, gpre, an, AFN);
          else src_cell_coefs3(I, tb, (cz + src_index(r + 1, ny, bcy)) * nx + scol, an, AFN);
          src_face_coefs3<T>(AF0, AFN, yN1, sa);
          face_phi_src<T>(I, total(1, sN), sa, pb, lf);
          put_phi(1, pb, lf);
        }
        if constexpr (2 / FP == H) {
          double AFS[4], an[4];
          if constexpr (kPreG) src_coefs_from3(I, tb, gpre, an, AFS);
          else src_cell_coefs3(I, tb, (cz + src_index(r - 1, ny, bcy)) * nx + scol, an, AFS);
          src_face_coefs3<T>(AFS, AF0, yS1, sa);
          face_phi_src<T>(I, total(2, sS), sa, pb, lf);
          put_phi(2, pb, lf);
        }
        if constexpr (3 / FP == H) {
          src_face_coefs3<T>(AF0, AF1, (T)zg[(z + 2) * kGeo + 1], sa);
          face_phi_src<T>(I, total(3, sT), sa, pb, lf);
          put_phi(3, pb, lf);
        }
      }
      lds_barrier();
    }
    if (inner) {
      const int zi = z + 1;
      const T kz = zg[zi * kGeo + 4];
      T fW[Q], fN[Q], fS[Q];
      if constexpr (SRC) {
        auto pbv = [&](int face) __attribute__((always_inline)) { return L.psum[face][rw][0][lane]; };
        auto lfv = [&](int face) __attribute__((always_inline)) { return L.psum[face][rw][1][lane]; };
        face_out_phi<Q, P, H, 0>(I, ev, gbW, pbv(0), lfv(0), fW);
        face_out_phi<Q, P, H, 1>(I, ev, gbN, pbv(1), lfv(1), fN);
        face_out_phi<Q, P, H, 1>(I, ev, gbS, pbv(2), lfv(2), fS);
        face_out_phi<Q, P, H, 2>(I, ev, gbT, pbv(3), lfv(3), FZt);
      } else {
        face_out<Q, P, H, 0>(I, ev, gbW, total(0, sW), fW);
        face_out<Q, P, H, 1>(I, ev, gbN, total(1, sN), fN);
        face_out<Q, P, H, 1>(I, ev, gbS, total(2, sS), fS);
        face_out<Q, P, H, 2>(I, ev, gbT, total(3, sT), FZt);
      }
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (part_of<Q, P>(k) != H) continue;
        if (ce<Q>(k, 0) != 0) O[k] = fma((T)(-ce<Q>(k, 0)) * ck, shl1(fW[k]) - fW[k], O[k]);
        if (ce<Q>(k, 1) != 0) O[k] = fma((T)(-ce<Q>(k, 1)) * ky, fN[k], O[k]);
        if (ce<Q>(k, 1) != 0) O[k] = fma((T)ce<Q>(k, 1) * ky, fS[k], O[k]);
        if (ce<Q>(k, 2) != 0) O[k] = fma((T)(-ce<Q>(k, 2)) * kz, FZt[k] - FZb[k], O[k]);
      }
    }
    if (live) {
      unsigned o = (unsigned)(((long long)z * ny + r) * pitch + c) * ES;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        if (part_of<Q, P>(k) == H) {
          if constexpr (WD == 1)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, O[k]), Rout, o, 0, 0);
          else
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, O[k]), Rout, o, 0, 0);
        }
        o += planeB;
      }
    }
    // no further barrier: the next plane's first barrier separates these
    // reads of the sums (with a source, of the faces' phi_b) from its writes
    // of them
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (part_of<Q, P>(k) != H) continue;
      G0[k] = G1[k];
      O[k] = FT1[k];
      if (ce<Q>(k, 2) != 0) FZb[k] = FZt[k];
    }
    if constexpr (SRC) {
#pragma unroll
      for (int m = 0; m < 4; ++m) AF0[m] = AF1[m];
    }
  };
  using R0 = std::integral_constant<int, 0>;
  using R1 = std::integral_constant<int, 1>;
  int z = z0;
  if constexpr (two) {
    for (; z + 2 <= z1; z += 2) {
      body(z, R1{});       // (z - z0) even: plane z+1 is in slot 1
      body(z + 1, R0{});
    }
    if (z < z1) body(z, R1{});
  } else {
    for (; z < z1; ++z) body(z, R0{});
  }
}

// WALLS = false: every axis periodic, no mirror code
// BATCH: the blocks of many instances (Batch3) in one launch
template <int Q, int NC, int ROWS, typename T, bool WALLS, bool SRC, bool BATCH>
__global__ __launch_bounds__((64 * parts<Q, T, ROWS, WALLS>() * ROWS)) void k_step3p(const Inst3* __restrict__ I, int parity,
                                                                       const double* __restrict__ ring,
                                                                       const SrcTab st, int planes, int strips,
                                                                       int tiles, const Batch3 bt) {
  constexpr int P = parts<Q, T, ROWS, WALLS>();
  __shared__ LdsP<Q, ROWS, T, WALLS> L;
  int blk = xcd_contiguous(blockIdx.x, gridDim.x);
  if constexpr (BATCH) {   // this block's instance: the last k with first[k] <= blk
    int lo = 0, hi = bt.n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (bt.first[mid] <= blk) lo = mid;
      else hi = mid - 1;
    }
    I = bt.insts[lo];
    blk -= (int)bt.first[lo];
    strips = (I->n[0] + kCols - 1) / kCols;
    tiles = (I->n[1] + ROWS - 1) / ROWS;
    ring = I->ring != nullptr ? I->ring + bt.step * I->ring_len : nullptr;
  }
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rw = w / P;
  // part of wave w: with four parts rotated by the row, so that each SIMD
  // (waves w, w+4, ...) runs every part once
  const int part = P == 2 ? (w & 1) : ((w + rw) & 3);
  const float* ec = nullptr;
  if constexpr (LdsP<Q, ROWS, T, WALLS>::kVecE && NC <= 4) {
    __shared__ float ecoef[Q * NC];   // E_i coefficients, read into vector registers
    if (w == 0)
      for (int i = threadIdx.x; i < Q * NC; i += kLanes) ecoef[i] = I->ef[i / NC][i % NC];
    ec = ecoef;
  }
  const STab tb = &st;
  double (*hp)[4][kLanes] = nullptr;
  if constexpr (LdsP<Q, ROWS, T, WALLS>::kHD) {
    __shared__ double hphi[2][4][kLanes];   // quarter sums of the cell phi of the two halo rows
    hp = hphi;
  }
  switch (part) {
    case 0: step3p_half<Q, NC, ROWS, T, 0, WALLS, SRC>(I, parity, ring, tb, planes, strips, tiles, L, ec, hp, w, rw, blk); break;
    case 1: step3p_half<Q, NC, ROWS, T, 1, WALLS, SRC>(I, parity, ring, tb, planes, strips, tiles, L, ec, hp, w, rw, blk); break;
    case 2:
      if constexpr (P > 2) step3p_half<Q, NC, ROWS, T, 2, WALLS, SRC>(I, parity, ring, tb, planes, strips, tiles, L, ec, hp, w, rw, blk);
      break;
    default:
      if constexpr (P > 2) step3p_half<Q, NC, ROWS, T, 3, WALLS, SRC>(I, parity, ring, tb, planes, strips, tiles, L, ec, hp, w, rw, blk);
      break;
  }
}

// -------------------------------------------------- init, copies, read-outs
template <int Q>
__device__ __forceinline__ void feq64(const Inst3* __restrict__ I, double phi, double* E) {
  const int nc = I->ncoef;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double r = I->e[k][nc - 1];
    for (int m = nc - 2; m >= 0; --m) r = fma(r, phi, I->e[k][m]);
    E[k] = r;
  }
}

template <int Q, int ST>
__global__ void k_init3(const Inst3* __restrict__ I, const double* __restrict__ phi, int parity) {
  using T = typename S3<ST>::T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= I->n[0]) return;
  const long long cell = ((long long)k * I->n[1] + j) * I->n[0] + i;
  const long long off = ((long long)k * I->n[1] + j) * I->pitch + i;
  double E[Q];
  feq64<Q>(I, phi[cell], E);
  if (I->src_n > 0) {
    // f = E at t = 0 (Omega = 0): f~ = E - dt S / 2 (eq. 2.25)
    double a[4];
    src_coefs3(I, cell, cell, 0.0, 0.0, a);
    const double F = poly4(a, phi[cell]);
#pragma unroll
    for (int m = 0; m < Q; ++m) E[m] -= 0.5 * I->dt * F * rho3<Q>(I, m, phi[cell]);
  }
  T* buf = (T*)I->buf[parity];
#pragma unroll
  for (int m = 0; m < Q; ++m) buf[m * I->plane + off] = (T)E[m];
}

template <int Q, int ST>
__global__ void k_set_f3(const Inst3* __restrict__ I, const double* __restrict__ f, int parity) {
  using T = typename S3<ST>::T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= I->n[0]) return;
  const long long N = (long long)I->n[0] * I->n[1] * I->n[2];
  const long long cell = ((long long)k * I->n[1] + j) * I->n[0] + i;
  const long long off = ((long long)k * I->n[1] + j) * I->pitch + i;
  T* buf = (T*)I->buf[parity];
#pragma unroll
  for (int m = 0; m < Q; ++m) buf[m * I->plane + off] = (T)f[m * N + cell];
}

template <int Q, int ST>
__global__ void k_get3(const Inst3* __restrict__ I, double* __restrict__ out, int parity, int want_f,
                       long long step) {
  using T = typename S3<ST>::T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= I->n[0]) return;
  const long long N = (long long)I->n[0] * I->n[1] * I->n[2];
  const long long cell = ((long long)k * I->n[1] + j) * I->n[0] + i;
  const long long off = ((long long)k * I->n[1] + j) * I->pitch + i;
  const T* buf = (const T*)I->buf[parity];
  if (want_f) {
#pragma unroll
    for (int m = 0; m < Q; ++m) out[m * N + cell] = (double)buf[m * I->plane + off];
  } else {
    double phi = 0.0;
#pragma unroll
    for (int m = 0; m < Q; ++m) phi += (double)buf[m * I->plane + off];
    out[cell] = src_phi3(I, cell, phi, (double)step * I->dt);
  }
}

constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;
constexpr int kRedVals = 8;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int Q, int ST>
__global__ __launch_bounds__(kRedThreads) void k_reduce3(const Inst3* __restrict__ I,
                                                         const double* __restrict__ ref, int parity,
                                                         long long step, const double* __restrict__ widths,
                                                         double* __restrict__ partial) {
  using T = typename S3<ST>::T;
  const int nx = I->n[0], ny = I->n[1];
  const long long N = (long long)nx * ny * I->n[2];
  const T* buf = (const T*)I->buf[parity];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(n % nx);
    const long long jk = n / nx;
    const int j = (int)(jk % ny), k = (int)(jk / ny);
    const long long off = ((long long)k * ny + j) * I->pitch + i;
    double phi = 0.0;
#pragma unroll
    for (int m = 0; m < Q; ++m) phi += (double)buf[m * I->plane + off];
    phi = src_phi3(I, n, phi, (double)step * I->dt);
    const double vol = widths[i] * widths[nx + j] * widths[nx + ny + k];
    if (!__builtin_isfinite(phi)) {
      acc[5] += 1.0;
      continue;
    }
    acc[0] += phi * vol;
    if (ref != nullptr) {
      const double rv = ref[n], d = phi - rv;
      acc[1] += fabs(d);
      acc[2] += fabs(rv);
      acc[3] += d * d * vol;
      acc[4] += rv * rv * vol;
    }
  }
  __shared__ double sh[kRedThreads / 64][6];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    const double s = wave_sum(acc[v]);
    if (lane == 0) sh[wv][v] = s;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double s = 0.0;
    for (int ww = 0; ww < kRedThreads / 64; ++ww) s += sh[ww][threadIdx.x];
    partial[blockIdx.x * kRedVals + threadIdx.x] = s;
  }
}

__global__ void k_reduce3_final(const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
  const int v = threadIdx.x;
  if (v >= kRedVals) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b * kRedVals + v];
  out[v] = s;
}

// --------------------------------------------------------------- launch
static inline hipStream_t S(void* s) { return (hipStream_t)s; }

long long step3_blocks(const Inst3& h, const Launch3& l) {
  const long long strips = (h.n[0] + kCols - 1) / kCols;
  const long long tiles = (h.n[1] + l.rows - 1) / l.rows;
  const long long chunks = (h.n[2] + l.planes - 1) / l.planes;
  return strips * tiles * chunks;
}

static size_t step3h_lds_bytes(int q, const Launch3& l) { return (size_t)3 * (l.rows + 2) * q * kLanes * 8; }

template <int Q, int NC, bool WALLS>
static void step3s_rows(const Inst3* d, int parity, const double* ring, const Launch3& l, int strips, int tiles, dim3 grid,
                        hipStream_t st) {
  switch (l.rows) {
    case 2: hipLaunchKernelGGL((k_step3s<Q, NC, 2, WALLS>), grid, dim3(128), 0, st, d, parity, ring, l.planes, strips, tiles); break;
    case 3: hipLaunchKernelGGL((k_step3s<Q, NC, 3, WALLS>), grid, dim3(192), 0, st, d, parity, ring, l.planes, strips, tiles); break;
    default: hipLaunchKernelGGL((k_step3s<Q, NC, 4, WALLS>), grid, dim3(256), 0, st, d, parity, ring, l.planes, strips, tiles); break;
  }
}
template <int Q, int NC, bool WALLS>
static void step3h_launch(const Inst3* d, const Inst3& h, int parity, const double* ring, const Launch3& l, int strips, int tiles,
                          dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((k_step3h<Q, DUGKS_F64, NC, WALLS>), grid, dim3(64 * (l.rows + 2)), step3h_lds_bytes(Q, l),
                     st, d, parity, ring, l.rows, l.planes, strips, tiles);
}
// D3Q7, one wave a row: the wall-free instantiation when every axis is
// periodic and the equilibrium polynomials have at most 4 coefficients
template <int Q, int NC>
static void step3_row_waves(const Inst3* d, const Inst3& h, int parity, const double* ring, const Launch3& l, int strips,
                            int tiles, dim3 grid, hipStream_t st) {
  const bool walls = h.bc[0] != DUGKS_BC_PERIODIC || h.bc[1] != DUGKS_BC_PERIODIC || h.bc[2] != DUGKS_BC_PERIODIC;
  if (h.storage == DUGKS_F64) {
    if (NC == 8 || walls) step3h_launch<Q, NC, true>(d, h, parity, ring, l, strips, tiles, grid, st);
    else if constexpr (NC != 8) step3h_launch<Q, NC, false>(d, h, parity, ring, l, strips, tiles, grid, st);
  } else {
    if (NC == 8 || walls) step3s_rows<Q, NC, true>(d, parity, ring, l, strips, tiles, grid, st);
    else if constexpr (NC != 8) step3s_rows<Q, NC, false>(d, parity, ring, l, strips, tiles, grid, st);
  }
}

// The launch arguments of the staged kernel
struct Args3 {
  const Inst3* d;
  int parity;
  const double* ring;
  SrcTab ss;
  int strips, tiles;
  Batch3 bt;
};
template <int Q, int NC, int ROWS, typename T, bool WALLS, bool SRC, bool BATCH>
static void step3p_go(const Args3& a, const Launch3& l, dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((k_step3p<Q, NC, ROWS, T, WALLS, SRC, BATCH>), grid, dim3(64 * parts<Q, T, ROWS, WALLS>() * ROWS),
                     0, st, a.d, a.parity, a.ring, a.ss, l.planes, a.strips, a.tiles, a.bt);
}
template <int Q, int NC, typename T, bool WALLS, bool SRC, bool BATCH = false>
static void step3p_launch(const Args3& a, const Launch3& l, dim3 grid, hipStream_t st) {
  if constexpr (sizeof(T) == 8) {   // rows 1 and 2 fit the LDS
    if (l.rows == 1) step3p_go<Q, NC, 1, T, WALLS, SRC, BATCH>(a, l, grid, st);
    else step3p_go<Q, NC, 2, T, WALLS, SRC, BATCH>(a, l, grid, st);
  } else {
    switch (l.rows) {
      case 2: step3p_go<Q, NC, 2, T, WALLS, SRC, BATCH>(a, l, grid, st); break;
      case 3: step3p_go<Q, NC, 3, T, WALLS, SRC, BATCH>(a, l, grid, st); break;
      default: step3p_go<Q, NC, 4, T, WALLS, SRC, BATCH>(a, l, grid, st); break;
    }
  }
}
// With a source: the instantiation with mirror code (it serves periodic axes too)
template <int Q, int NC, typename T>
static void step3p_rows(const Args3& a, const Inst3& h, bool walls, const Launch3& l, dim3 grid, hipStream_t st) {
  if (a.bt.insts != nullptr) {   // a batch
    if (NC == 8 || walls) step3p_launch<Q, NC, T, true, false, true>(a, l, grid, st);
    else if constexpr (NC != 8) step3p_launch<Q, NC, T, false, false, true>(a, l, grid, st);
  } else if (h.src_n > 0) step3p_launch<Q, NC, T, true, true>(a, l, grid, st);
  else if (NC == 8 || walls) step3p_launch<Q, NC, T, true, false>(a, l, grid, st);
  else if constexpr (NC != 8) step3p_launch<Q, NC, T, false, false>(a, l, grid, st);
}

template <int Q>
static int step3_q(const Args3& a, const Inst3& h, bool walls, long long blocks, const Launch3& l, void* stream) {
  const int strips = a.strips, tiles = a.tiles;
  const Inst3* d = a.d;
  const int parity = a.parity;
  const double* ring = a.ring;
  if (blocks <= 0 || blocks > 0x7fffffffLL) return -1;
  const dim3 grid((unsigned)blocks);
  const int nc = h.ncoef <= 2 ? 2 : (h.ncoef <= 4 ? 4 : 8);
  if constexpr (Q != 7) {   // split directions
    if (h.storage == DUGKS_F64) {
      switch (nc) {
        case 2: step3p_rows<Q, 2, double>(a, h, walls, l, grid, S(stream)); break;
        case 4: step3p_rows<Q, 4, double>(a, h, walls, l, grid, S(stream)); break;
        default: step3p_rows<Q, 8, double>(a, h, walls, l, grid, S(stream)); break;
      }
    } else {
      switch (nc) {
        case 2: step3p_rows<Q, 2, float>(a, h, walls, l, grid, S(stream)); break;
        case 4: step3p_rows<Q, 4, float>(a, h, walls, l, grid, S(stream)); break;
        default: step3p_rows<Q, 8, float>(a, h, walls, l, grid, S(stream)); break;
      }
    }
  } else if (h.src_n > 0) {   // D3Q7 with a source: the staged kernel, two parts a row
    if (h.storage == DUGKS_F64) {
      switch (nc) {
        case 2: step3p_launch<Q, 2, double, true, true>(a, l, grid, S(stream)); break;
        case 4: step3p_launch<Q, 4, double, true, true>(a, l, grid, S(stream)); break;
        default: step3p_launch<Q, 8, double, true, true>(a, l, grid, S(stream)); break;
      }
    } else {
      switch (nc) {
        case 2: step3p_launch<Q, 2, float, true, true>(a, l, grid, S(stream)); break;
        case 4: step3p_launch<Q, 4, float, true, true>(a, l, grid, S(stream)); break;
        default: step3p_launch<Q, 8, float, true, true>(a, l, grid, S(stream)); break;
      }
    }
  } else {   // D3Q7: a whole row per wave
    switch (nc) {
      case 2: step3_row_waves<Q, 2>(d, h, parity, ring, l, strips, tiles, grid, S(stream)); break;
      case 4: step3_row_waves<Q, 4>(d, h, parity, ring, l, strips, tiles, grid, S(stream)); break;
      default: step3_row_waves<Q, 8>(d, h, parity, ring, l, strips, tiles, grid, S(stream)); break;
    }
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_step3(const Inst3* d, const Inst3& h, int parity, long long step, const Launch3& l, void* stream) {
  // the step's Dirichlet data (no reads without a Dirichlet axis)
  const double* ring = h.ring != nullptr ? h.ring + step * h.ring_len : nullptr;
  // the source terms' time factors at t_n (cells) and t_n + h (faces)
  SrcTab ss{};
  for (int j = 0; j < h.src_n; ++j) {
    ss.en[j] = exp(h.src_gam[j] * ((double)step * h.dt));
    ss.ef[j] = exp(h.src_gam[j] * (((double)step + 0.5) * h.dt));
  }
  Args3 a{d, parity, ring, ss, (h.n[0] + kCols - 1) / kCols, (h.n[1] + l.rows - 1) / l.rows, Batch3{nullptr, nullptr, 0, 0}};
  const bool walls = h.bc[0] != DUGKS_BC_PERIODIC || h.bc[1] != DUGKS_BC_PERIODIC || h.bc[2] != DUGKS_BC_PERIODIC;
  const long long blocks = step3_blocks(h, l);
  switch (h.q) {
    case 19: return step3_q<19>(a, h, walls, blocks, l, stream);
    case 15: return step3_q<15>(a, h, walls, blocks, l, stream);
    default: return step3_q<7>(a, h, walls, blocks, l, stream);
  }
}

int launch_step3_batch(const Batch3& bt, const Inst3& h, int parity, bool walls, long long blocks,
                       const Launch3& l, void* stream) {
  if (h.src_n > 0 || bt.insts == nullptr || bt.n < 1) return -1;
  // the instance pointer, strips, tiles and Dirichlet data come from the table
  const Args3 a{nullptr, parity, nullptr, SrcTab{}, 0, 0, bt};
  switch (h.q) {
    case 19: return step3_q<19>(a, h, walls, blocks, l, stream);
    case 15: return step3_q<15>(a, h, walls, blocks, l, stream);
    default: return -1;
  }
}

size_t step3_lds_bytes(int storage, int q, bool walls, const Launch3& l, bool src) {
  if (q == 7 && !src)   // binary64: g of 3 planes (dynamic); binary32: g of 3 planes and f~ of 2
    return storage == DUGKS_F64 ? step3h_lds_bytes(q, l) : (size_t)5 * (l.rows + 2) * q * kLanes * 4;
  // g of 3 planes and staged f~ of 1 or 2 planes (LdsP), each of rows + 2
  // rows, and the parts' sums of 4 faces per row (static; the binary32 E
  // coefficients aside)
  const size_t e = storage == DUGKS_F64 ? 8 : 4;
  // parts<Q, T, ROWS, WALLS>(), walls meaning the instantiation with mirror code
  const bool quarters = q == 19 || (q == 15 && !walls);
  const size_t np = (quarters && ((storage != DUGKS_F64 && l.rows >= 3) || (storage == DUGKS_F64 && l.rows == 2))) ? 4 : 2;
  const size_t rr = np == 4 ? l.rows : l.rows + 2;   // staged_rows<>()
  const size_t hs = rr == (size_t)l.rows ? (size_t)2 * 4 * kLanes * 8 : 0;        // halo rows' phi sums
  auto bytes = [&](size_t ns) {
    return 3 * (l.rows + 2) * q * kLanes * e + ns * rr * q * kLanes * e + (size_t)4 * l.rows * np * kLanes * e + hs;
  };
  if (storage == DUGKS_F64) return bytes(1);
  return (bytes(2) > 81920 && bytes(1) <= 81920) ? bytes(1) : bytes(2);
}

#define DUGKS3_PER_CELL(KERNEL, ...)                                                               \
  do {                                                                                             \
    dim3 grid((h.n[0] + 255) / 256, h.n[1], h.n[2]), block(256);                                   \
    const bool f64 = h.storage == DUGKS_F64;                                                       \
    switch (h.q) {                                                                                 \
      case 19:                                                                                     \
        if (f64) hipLaunchKernelGGL((KERNEL<19, DUGKS_F64>), grid, block, 0, S(stream), __VA_ARGS__); \
        else hipLaunchKernelGGL((KERNEL<19, DUGKS_F32>), grid, block, 0, S(stream), __VA_ARGS__);     \
        break;                                                                                     \
      case 15:                                                                                     \
        if (f64) hipLaunchKernelGGL((KERNEL<15, DUGKS_F64>), grid, block, 0, S(stream), __VA_ARGS__); \
        else hipLaunchKernelGGL((KERNEL<15, DUGKS_F32>), grid, block, 0, S(stream), __VA_ARGS__);     \
        break;                                                                                     \
      default:                                                                                     \
        if (f64) hipLaunchKernelGGL((KERNEL<7, DUGKS_F64>), grid, block, 0, S(stream), __VA_ARGS__);  \
        else hipLaunchKernelGGL((KERNEL<7, DUGKS_F32>), grid, block, 0, S(stream), __VA_ARGS__);      \
        break;                                                                                     \
    }                                                                                              \
  } while (0)

int launch_init3(const Inst3* d, const Inst3& h, const double* phi, int parity, void* stream) {
  DUGKS3_PER_CELL(k_init3, d, phi, parity);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_set_f3(const Inst3* d, const Inst3& h, const double* f, int parity, void* stream) {
  DUGKS3_PER_CELL(k_set_f3, d, f, parity);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_get_phi3(const Inst3* d, const Inst3& h, double* out, int parity, long long step, void* stream) {
  DUGKS3_PER_CELL(k_get3, d, out, parity, 0, step);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
int launch_get_f3(const Inst3* d, const Inst3& h, double* out, int parity, void* stream) {
  DUGKS3_PER_CELL(k_get3, d, out, parity, 1, 0LL);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int reduce3_partials() { return kRedBlocks; }

int launch_reduce3(const Inst3* d, const Inst3& h, const double* ref, int parity, long long step,
                   const double* widths, double* partial, double* out, void* stream) {
  dim3 grid(kRedBlocks), block(kRedThreads);
  const bool f64 = h.storage == DUGKS_F64;
  switch (h.q) {
    case 19:
      if (f64) hipLaunchKernelGGL((k_reduce3<19, DUGKS_F64>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial);
      else hipLaunchKernelGGL((k_reduce3<19, DUGKS_F32>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial);
      break;
    case 15:
      if (f64) hipLaunchKernelGGL((k_reduce3<15, DUGKS_F64>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial);
      else hipLaunchKernelGGL((k_reduce3<15, DUGKS_F32>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial);
      break;
    default:
      if (f64) hipLaunchKernelGGL((k_reduce3<7, DUGKS_F64>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial);
      else hipLaunchKernelGGL((k_reduce3<7, DUGKS_F32>), grid, block, 0, S(stream), d, ref, parity, step, widths, partial);
      break;
  }
  if (hipGetLastError() != hipSuccess) return -1;
  hipLaunchKernelGGL(k_reduce3_final, dim3(1), dim3(64), 0, S(stream), partial, kRedBlocks, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dugks3
