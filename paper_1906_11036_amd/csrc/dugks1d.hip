// One-dimensional DUGKS step on D1Q3 (eq. 2.4) for B = b(x, t) phi and
// D = d(t) phi with C = 0 and the source distribution R_i = w_i c_i dB/dt /
// c_s^2 of Remark 3 (Example 4.6): gfx950 kernels and the host runtime behind
// include/dugks1d.h.
//
// State (two ping-pong buffers, each [4][pitch] of binary64 or binary32):
// planes 0..2 hold f~ of the directions c = 0, +c, -c; plane 3 holds phi^{n-1}.
//
// With S_i = R_i the shifted distributions of eqs. 2.25 and 2.27 reduce to
//   fbar+ = a1 f~ + b1 (E + lambda R)        f~+ = a2 f~ + b2 (E + lambda R)
//   f(x_b, t+h) = a3 fbar + b3 (E_b + lambda R_b)
// with a1 = (2 lambda - h)/(2 lambda + dt), b1 = 3h/(2 lambda + dt),
// a2 = (2 lambda - dt)/(2 lambda + dt), b2 = 2 dt/(2 lambda + dt),
// a3 = 2 lambda/(2 lambda + h), b3 = h/(2 lambda + h)  (eqs. 2.21-2.23).
// In one dimension E_0 = phi (3 - d)/3 and E_{+-} = phi (d +- 3 b / c)/6, and
// R_0 = 0, R_{+-} = +- dB/dt / (2c).
//
// Fused step kernel: a wave owns 62 consecutive cells (64 lanes, one halo
// lane each side), loads f~ and phi^{n-1} of its 64 cells, forms fbar+, f~+
// and dB/dt per lane, computes the west face of every lane (the east face is
// the next lane's west face, by DPP) and stores f~ and phi^n.  No LDS.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <string>
#include <vector>

#include "dugks1d.h"

namespace dugks1 {

constexpr int kCols = 62;
constexpr int kWavesPerBlock = 16;   // large blocks: fewer block dispatches for a streaming kernel
constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 512;

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

// Per-instance constants and tables (passed by value to the step kernel).
template <typename T> struct Inst1 {
  const T* in;            // state buffer read this step: [4][pitch]
  T* out;                 // state buffer written
  const double* xc;       // cell centres [nx + 2]: ghosts at 0 and nx + 1
  const double* xf;       // faces [nx + 1]
  const T* face;          // per face m (0..nx): factors for c_i = -c, 0, +c ([nx + 1][3])
  const T* upd;           // per cell: dt c / width [nx]
  int nx, pitch, bc;
  T a1, b1, a2, b2, a3, b3, lambda, inv_dt, c3;   // c3 = 3 / c
  T half_inv_c;                                  // 1 / (2c)
  // uniform mesh (every width equal to w): centre of extended cell k is
  // x0 + (k - 0.5) w, face m at x0 + m w; one set of face factors and one
  // update factor, so the step reads no per-cell table
  double x0, w;
  T uam, ua0, uap, uupd;
};

// Per-step coefficients: b(x, t) = p x + q and d at t_n, t_{n-1} and t_n + h;
// Dirichlet ghost values at t_n and t_{n-1} (device, may be null).
template <typename T> struct Step1 {
  T pn, qn, dn, pm, qm, ph, qh, dh;
  const double* gcur;     // [2] at t_n
  const double* gprev;    // [2] at t_{n-1}
};

template <typename T>
__device__ __forceinline__ void feq1(T phi, T b, T d, T c3, T* E) {
  E[0] = phi * ((T)3 - d) * (T)(1.0 / 3.0);
  E[1] = phi * (d + c3 * b) * (T)(1.0 / 6.0);
  E[2] = phi * (d - c3 * b) * (T)(1.0 / 6.0);
}

template <typename T, bool UNI>
__global__ __launch_bounds__(64 * kWavesPerBlock) void k_step1(const Inst1<T> I, const Step1<T> S) {
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int nx = I.nx, pitch = I.pitch;
  const int x0 = wv * kCols;
  if (x0 >= nx) return;                  // whole wave: no cell of this strip exists
  const int c = x0 - 1 + lane;           // this lane's cell (-1 and nx are ghosts)
  const bool periodic = I.bc == DUGKS_BC_PERIODIC;
  int src = c;
  if (c < 0) src = periodic ? nx - 1 : 0;
  else if (c >= nx) src = periodic ? (c - nx < nx ? c - nx : nx - 1) : nx - 1;
  const bool ghost = !periodic && (c < 0 || c >= nx);

  T f[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) f[i] = I.in[(size_t)i * pitch + src];
  const T pp = I.in[(size_t)3 * pitch + src];
  const double phid = (double)f[0] + (double)f[1] + (double)f[2];   // phi = sum f~ (binary64)
  const T phi = (T)phid;
  const T x = UNI ? (T)(I.x0 + ((double)src + 0.5) * I.w) : (T)I.xc[src + 1];
  const T dB = ((S.pn * x + S.qn) * phi - (S.pm * x + S.qm) * pp) * I.inv_dt;
  T E[3], g[3], ft[3];
  feq1(phi, S.pn * x + S.qn, S.dn, I.c3, E);
  const T lr = I.lambda * dB * I.half_inv_c;    // lambda R_+ (R_- = -R_+, R_0 = 0)
  const T ES[3] = {E[0], E[1] + lr, E[2] - lr};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g[i] = I.a1 * f[i] + I.b1 * ES[i];          // fbar+
    ft[i] = I.a2 * f[i] + I.b2 * ES[i];         // f~+
  }
  T dBl = dB;
  if (ghost) {
    // non-equilibrium extrapolation: fbar+_g = E(phi_g, x_g) + fbar+_a - E(phi_a, x_a)
    const int side = c < 0 ? 0 : 1;
    const T phg = (T)S.gcur[side], phgp = (T)S.gprev[side];
    const T xg = UNI ? (T)(I.x0 + ((c < 0 ? -1.0 : (double)nx) + 0.5) * I.w) : (T)I.xc[c < 0 ? 0 : nx + 1];
    T Eg[3];
    feq1(phg, S.pn * xg + S.qn, S.dn, I.c3, Eg);
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = Eg[i] + (g[i] - E[i]);
    dBl = ((S.pn * xg + S.qn) * phg - (S.pm * xg + S.qm) * phgp) * I.inv_dt;
  }

  // west face of this lane's cell: between lanes - 1 and lane (face index c)
  const int m = c < 0 ? 0 : (c > nx ? nx : c);
  const T am = UNI ? I.uam : I.face[(size_t)m * 3 + 0];
  const T a0 = UNI ? I.ua0 : I.face[(size_t)m * 3 + 1];
  const T ap = UNI ? I.uap : I.face[(size_t)m * 3 + 2];
  T fb[3];
  {
    const T L0 = shr1(g[0]), L1 = shr1(g[1]), L2 = shr1(g[2]), dL = shr1(dBl);
    fb[0] = L0 + a0 * (g[0] - L0);
    fb[1] = L1 + ap * (g[1] - L1);     // c_i = +c
    fb[2] = L2 + am * (g[2] - L2);     // c_i = -c
    const T phib = (T)((double)fb[0] + (double)fb[1] + (double)fb[2]);
    const T dBb = dL + a0 * (dBl - dL);
    const T xb = UNI ? (T)(I.x0 + (double)m * I.w) : (T)I.xf[m];
    T Eb[3];
    feq1(phib, S.ph * xb + S.qh, S.dh, I.c3, Eb);
    const T lrb = I.lambda * dBb * I.half_inv_c;
    fb[1] = I.a3 * fb[1] + I.b3 * (Eb[1] + lrb);
    fb[2] = I.a3 * fb[2] + I.b3 * (Eb[2] - lrb);
  }
  // flux difference (eq. 2.9): c (f_E - f_W) for +c, -c (f_E - f_W) for -c
  const T u = c >= 0 && c < nx ? (UNI ? I.uupd : I.upd[c]) : (T)0;
  const T o1 = ft[1] - u * (shl1(fb[1]) - fb[1]);
  const T o2 = ft[2] + u * (shl1(fb[2]) - fb[2]);
  if (lane >= 1 && lane <= kCols && c < nx) {
    T* o = I.out;
    o[c] = ft[0];
    o[(size_t)pitch + c] = o1;
    o[(size_t)2 * pitch + c] = o2;
    o[(size_t)3 * pitch + c] = phi;
  }
}

template <typename T>
__global__ void k_init1(Inst1<T> I, const double* __restrict__ phi0, double p0, double q0, double pm,
                        double qm, double d0, double dt, double half_dt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= I.nx) return;
  const double x = I.xc[j + 1], phi = phi0[j];
  const double b = p0 * x + q0;
  const double dB = (b * phi - (pm * x + qm) * phi) / dt;
  const double c3 = (double)I.c3;
  const double E[3] = {phi * (3.0 - d0) / 3.0, phi * (d0 + c3 * b) / 6.0, phi * (d0 - c3 * b) / 6.0};
  const double Rp = dB * (double)I.half_inv_c;
  T* o = I.out;
  o[j] = (T)E[0];
  o[(size_t)I.pitch + j] = (T)(E[1] - half_dt * Rp);
  o[(size_t)2 * I.pitch + j] = (T)(E[2] + half_dt * Rp);
  o[(size_t)3 * I.pitch + j] = (T)phi;
}

template <typename T>
__global__ void k_set1(T* __restrict__ out, const double* __restrict__ f, const double* __restrict__ pp,
                       int nx, int pitch) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nx) return;
  for (int i = 0; i < 3; ++i) out[(size_t)i * pitch + j] = (T)f[(size_t)i * nx + j];
  out[(size_t)3 * pitch + j] = (T)pp[j];
}

// what: 0 phi, 1 f~ [3][nx], 2 phi^{n-1}
template <typename T>
__global__ void k_get1(const T* __restrict__ st, double* __restrict__ out, int nx, int pitch, int what) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nx) return;
  if (what == 0)
    out[j] = (double)st[j] + (double)st[(size_t)pitch + j] + (double)st[(size_t)2 * pitch + j];
  else if (what == 1)
    for (int i = 0; i < 3; ++i) out[(size_t)i * nx + j] = (double)st[(size_t)i * pitch + j];
  else
    out[j] = (double)st[(size_t)3 * pitch + j];
}

// partial[b * 8 + k]: 0 mass, 1 sum|phi-ref|, 2 sum|ref|, 3 sum (phi-ref)^2 w, 4 sum ref^2 w, 5 non-finite
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_reduce1(const T* __restrict__ st, const double* __restrict__ ref,
                                                         const double* __restrict__ xf, int nx, int pitch,
                                                         double* __restrict__ partial) {
  __shared__ double sh[kRedThreads / 64][6];
  double a[6] = {0, 0, 0, 0, 0, 0};
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nx; j += gridDim.x * blockDim.x) {
    const double phi = (double)st[j] + (double)st[(size_t)pitch + j] + (double)st[(size_t)2 * pitch + j];
    const double w = xf[j + 1] - xf[j];
    if (!isfinite(phi)) a[5] += 1.0;
    a[0] += phi * w;
    if (ref) {
      const double d = phi - ref[j];
      a[1] += fabs(d);
      a[2] += fabs(ref[j]);
      a[3] += d * d * w;
      a[4] += ref[j] * ref[j] * w;
    }
  }
  for (int k = 0; k < 6; ++k)
    for (int off = 32; off >= 1; off >>= 1) a[k] += __shfl_xor(a[k], off);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 6; ++k) sh[wv][k] = a[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) {
      double s = 0;
      for (int v = 0; v < kRedThreads / 64; ++v) s += sh[v][k];
      partial[(size_t)blockIdx.x * 8 + k] = s;
    }
}

__global__ void k_reduce1_final(const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int k = 0; k < 6; ++k) {
    double s = 0;
    for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * 8 + k];
    out[k] = s;
  }
}

}  // namespace dugks1

// ------------------------------------------------------------------ host
using namespace dugks1;

namespace {
constexpr uint32_t kMagic1 = 0x44554731u;  // "DUG1"
size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
}  // namespace

struct dugks1_ctx {
  uint32_t magic = kMagic1;
  std::string err;
  int nx = 0, pitch = 0;
  dugks1_params p{};
  std::vector<double> xf, xc, wd;
  double cs2 = 0, lambda = 0, dt = 0, h = 0, a1 = 0, b1 = 0, a2 = 0, b2 = 0, a3 = 0, b3 = 0;
  std::vector<double> face64, upd64;
  // device
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  size_t off_buf[2] = {0, 0}, off_xc = 0, off_xf = 0, off_face = 0, off_upd = 0, off_gslot = 0,
         off_partial = 0, off_out = 0, off_stage = 0, total = 0, buf_bytes = 0, stage_bytes = 0;
  bool uniform = false;
  double uw = 0;
  bool has_state = false;
  int parity = 0;
  long long steps = 0;
  // Dirichlet data
  const double* ghosts = nullptr;
  int ghosts_n = 0, ghosts_pos = 0;
  bool have_gprev = false;     // a previous step's ghost pair exists (in the slot or the array)

  int fail(int rc, const std::string& m) { err = m; return rc; }
  int hipfail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return DUGKS_E_HIP;
  }
  bool bound() const { return ws != nullptr; }
  size_t elem() const { return p.storage == DUGKS_F64 ? 8 : 4; }
  double bcoef_p(double t) const { return p.coef[0] + p.coef[1] * t; }
  double bcoef_q(double t) const { return p.coef[2] * exp(p.coef[3] * t + p.coef[4] * t * t); }
  double dcoef(double t) const { return p.coef[5] + p.coef[6] * t; }
  double time() const { return p.t0 + (double)steps * dt; }

  template <typename T> Inst1<T> inst(int par) const {
    Inst1<T> I{};
    I.in = (const T*)(ws + off_buf[par]);
    I.out = (T*)(ws + off_buf[par ^ 1]);
    I.xc = (const double*)(ws + off_xc);
    I.xf = (const double*)(ws + off_xf);
    I.face = (const T*)(ws + off_face);
    I.upd = (const T*)(ws + off_upd);
    I.nx = nx;
    I.pitch = pitch;
    I.bc = p.bc;
    I.a1 = (T)a1; I.b1 = (T)b1; I.a2 = (T)a2; I.b2 = (T)b2; I.a3 = (T)a3; I.b3 = (T)b3;
    I.lambda = (T)lambda;
    I.inv_dt = (T)(1.0 / dt);
    I.c3 = (T)(3.0 / p.c);
    I.half_inv_c = (T)(0.5 / p.c);
    I.x0 = xf[0];
    I.w = uw;
    if (uniform) {
      I.uam = (T)face64[0];
      I.ua0 = (T)face64[1];
      I.uap = (T)face64[2];
      I.uupd = (T)upd64[0];
    }
    return I;
  }
};

#define GUARD1(ctx)                                                        \
  do {                                                                     \
    if (!(ctx) || (ctx)->magic != kMagic1) return DUGKS_E_ARG;             \
  } while (0)

static hipStream_t S1(const dugks1_ctx* x) { return x->stream; }

template <typename T> static void launch_step(dugks1_ctx* x) {
  const double tn = x->time(), tm = tn - x->dt, th = tn + x->h;
  Step1<T> S{};
  S.pn = (T)x->bcoef_p(tn); S.qn = (T)x->bcoef_q(tn); S.dn = (T)x->dcoef(tn);
  S.pm = (T)x->bcoef_p(tm); S.qm = (T)x->bcoef_q(tm);
  S.ph = (T)x->bcoef_p(th); S.qh = (T)x->bcoef_q(th); S.dh = (T)x->dcoef(th);
  if (x->p.bc == DUGKS_BC_DIRICHLET) {
    S.gcur = x->ghosts + 2 * (size_t)x->ghosts_pos;
    if (!x->have_gprev) S.gprev = S.gcur;
    else if (x->ghosts_pos > 0) S.gprev = S.gcur - 2;
    else S.gprev = (const double*)(x->ws + x->off_gslot);
  }
  const long long waves = (x->nx + kCols - 1) / kCols;
  const dim3 grid((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock)), block(64 * kWavesPerBlock);
  if (x->uniform)
    hipLaunchKernelGGL((k_step1<T, true>), grid, block, 0, S1(x), x->inst<T>(x->parity), S);
  else
    hipLaunchKernelGGL((k_step1<T, false>), grid, block, 0, S1(x), x->inst<T>(x->parity), S);
}

extern "C" {

int dugks1_create(dugks1_ctx** out, int nx, const double* xf, const dugks1_params* p) {
  if (!out) return DUGKS_E_ARG;
  dugks1_ctx* x = new dugks1_ctx();
  *out = x;
  if (!p || !xf) return x->fail(DUGKS_E_ARG, "null argument");
  if (p->abi_version != DUGKS1_ABI_VERSION) return x->fail(DUGKS_E_ARG, "abi_version mismatch");
  if (p->storage != DUGKS_F64 && p->storage != DUGKS_F32)
    return x->fail(DUGKS_E_UNSUPPORTED, "storage must be DUGKS_F64 or DUGKS_F32");
  if (p->bc != DUGKS_BC_PERIODIC && p->bc != DUGKS_BC_DIRICHLET)
    return x->fail(DUGKS_E_UNSUPPORTED, "walls must be periodic or Dirichlet");
  if (nx < 1 || nx > (1 << 30)) return x->fail(DUGKS_E_ARG, "nx must be in [1, 2^30]");
  if (!(p->c > 0) || !std::isfinite(p->c)) return x->fail(DUGKS_E_ARG, "c must be > 0");
  if (!(p->cfl > 0 && p->cfl < 1)) return x->fail(DUGKS_E_ARG, "cfl must be in (0, 1)");
  if (!(p->alpha > 0) || !std::isfinite(p->alpha)) return x->fail(DUGKS_E_ARG, "alpha must be > 0");
  for (int k = 0; k < 7; ++k)
    if (!std::isfinite(p->coef[k])) return x->fail(DUGKS_E_ARG, "coefficients must be finite");
  if (!std::isfinite(p->t0)) return x->fail(DUGKS_E_ARG, "t0 must be finite");
  if (p->bc == DUGKS_BC_PERIODIC && (p->coef[0] != 0.0 || p->coef[1] != 0.0))
    return x->fail(DUGKS_E_ARG, "periodic walls need b independent of x (p0 = p1 = 0)");
  for (int i = 0; i < nx; ++i)
    if (!(xf[i + 1] > xf[i]) || !std::isfinite(xf[i + 1]))
      return x->fail(DUGKS_E_ARG, "faces must be finite and strictly increasing");
  x->p = *p;
  x->nx = nx;
  x->pitch = (nx + 63) & ~63;
  x->xf.assign(xf, xf + nx + 1);
  x->wd.assign(nx + 2, 0.0);
  x->xc.assign(nx + 2, 0.0);
  for (int i = 0; i < nx; ++i) {
    x->wd[i + 1] = xf[i + 1] - xf[i];
    x->xc[i + 1] = 0.5 * (xf[i] + xf[i + 1]);
  }
  if (p->bc == DUGKS_BC_PERIODIC) {
    const double L = xf[nx] - xf[0];
    x->wd[0] = x->wd[nx];
    x->xc[0] = x->xc[nx] - L;
    x->wd[nx + 1] = x->wd[1];
    x->xc[nx + 1] = x->xc[1] + L;
  } else {
    x->wd[0] = x->wd[1];
    x->xc[0] = xf[0] - 0.5 * x->wd[1];
    x->wd[nx + 1] = x->wd[nx];
    x->xc[nx + 1] = xf[nx] + 0.5 * x->wd[nx];
  }
  double wmin = x->wd[1];
  for (int i = 1; i <= nx; ++i) wmin = std::min(wmin, x->wd[i]);
  x->cs2 = p->c * p->c / 3.0;
  x->lambda = p->alpha / x->cs2;
  x->dt = p->cfl * wmin / p->c;
  x->h = 0.5 * x->dt;
  const double lam = x->lambda, dt = x->dt, h = x->h;
  x->a1 = (2 * lam - h) / (2 * lam + dt);
  x->b1 = 3 * h / (2 * lam + dt);
  x->a2 = (2 * lam - dt) / (2 * lam + dt);
  x->b2 = 2 * dt / (2 * lam + dt);
  x->a3 = 2 * lam / (2 * lam + h);
  x->b3 = h / (2 * lam + h);
  // face m between extended cells m and m+1: fbar at the face = L + a (R - L)
  // with a = (x_b - x_L - h c_i) / (x_R - x_L)  (eqs. 2.19, 2.20)
  x->face64.assign((size_t)(nx + 1) * 3, 0.0);
  for (int m = 0; m <= nx; ++m) {
    const double dn = x->xc[m + 1] - x->xc[m], wl = xf[m] - x->xc[m];
    x->face64[(size_t)m * 3 + 0] = (wl + h * p->c) / dn;   // c_i = -c
    x->face64[(size_t)m * 3 + 1] = wl / dn;                // c_i = 0
    x->face64[(size_t)m * 3 + 2] = (wl - h * p->c) / dn;   // c_i = +c
  }
  x->upd64.assign(nx, 0.0);
  for (int j = 0; j < nx; ++j) x->upd64[j] = dt * p->c / x->wd[j + 1];
  // a mesh whose widths agree to 1e-12 is stepped as uniform (geometry from the index)
  x->uw = (xf[nx] - xf[0]) / nx;
  x->uniform = true;
  for (int j = 1; j <= nx; ++j)
    if (fabs(x->wd[j] - x->uw) > 1e-12 * x->uw) x->uniform = false;
  if (x->uniform) {
    const double dn = x->uw, wl = 0.5 * x->uw;
    x->face64[0] = (wl + h * p->c) / dn;
    x->face64[1] = wl / dn;
    x->face64[2] = (wl - h * p->c) / dn;
    x->upd64[0] = dt * p->c / x->uw;
  }
  x->buf_bytes = (size_t)4 * x->pitch * x->elem();
  size_t off = 0;
  x->off_buf[0] = off; off += align256(x->buf_bytes);
  x->off_buf[1] = off; off += align256(x->buf_bytes);
  x->off_xc = off; off += align256(sizeof(double) * (nx + 2));
  x->off_xf = off; off += align256(sizeof(double) * (nx + 1));
  x->off_face = off; off += align256(x->elem() * 3 * (size_t)(nx + 1));
  x->off_upd = off; off += align256(x->elem() * (size_t)nx);
  x->off_gslot = off; off += 256;
  x->off_partial = off; off += align256(sizeof(double) * 8 * kRedBlocks);
  x->off_out = off; off += 256;
  x->stage_bytes = sizeof(double) * 4 * (size_t)nx;
  x->off_stage = off; off += align256(x->stage_bytes);
  x->total = off;
  return DUGKS_OK;
}

size_t dugks1_workspace_bytes(const dugks1_ctx* x) {
  if (!x || x->magic != kMagic1) return 0;
  return x->total;
}

int dugks1_bind(dugks1_ctx* x, void* dev, size_t bytes, void* stream) {
  GUARD1(x);
  if (!dev || ((uintptr_t)dev & 255)) return x->fail(DUGKS_E_ARG, "workspace must be non-null and 256-byte aligned");
  if (bytes < x->total) return x->fail(DUGKS_E_ARG, "workspace too small");
  x->ws = (char*)dev;
  x->ws_bytes = bytes;
  x->stream = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(x->ws + x->off_xc, x->xc.data(), sizeof(double) * x->xc.size(),
                                hipMemcpyHostToDevice, S1(x));
  if (e == hipSuccess)
    e = hipMemcpyAsync(x->ws + x->off_xf, x->xf.data(), sizeof(double) * x->xf.size(), hipMemcpyHostToDevice,
                       S1(x));
  std::vector<float> f32;
  const void* face = x->face64.data();
  const void* upd = x->upd64.data();
  std::vector<float> u32;
  if (x->p.storage == DUGKS_F32) {
    f32.assign(x->face64.begin(), x->face64.end());
    u32.assign(x->upd64.begin(), x->upd64.end());
    face = f32.data();
    upd = u32.data();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(x->ws + x->off_face, face, x->elem() * x->face64.size(), hipMemcpyHostToDevice, S1(x));
  if (e == hipSuccess)
    e = hipMemcpyAsync(x->ws + x->off_upd, upd, x->elem() * x->upd64.size(), hipMemcpyHostToDevice, S1(x));
  if (e == hipSuccess) e = hipStreamSynchronize(S1(x));
  if (e != hipSuccess) {
    x->ws = nullptr;
    return x->hipfail(e, "upload mesh tables");
  }
  return DUGKS_OK;
}

static int stage_in(dugks1_ctx* x, const double* src, size_t count, int on_device, const double** dev) {
  if (on_device) {
    *dev = src;
    return DUGKS_OK;
  }
  hipError_t e = hipMemcpyAsync(x->ws + x->off_stage, src, sizeof(double) * count, hipMemcpyHostToDevice, S1(x));
  if (e != hipSuccess) return x->hipfail(e, "copy to device");
  *dev = (const double*)(x->ws + x->off_stage);
  return DUGKS_OK;
}

int dugks1_set_phi(dugks1_ctx* x, const double* phi, int on_device) {
  GUARD1(x);
  if (!x->bound()) return x->fail(DUGKS_E_STATE, "not bound");
  if (!phi) return x->fail(DUGKS_E_ARG, "null phi");
  const double* d = nullptr;
  int rc = stage_in(x, phi, x->nx, on_device, &d);
  if (rc) return rc;
  const double t0 = x->p.t0, tm = t0 - x->dt;
  const dim3 grid((x->nx + 255) / 256), block(256);
  if (x->p.storage == DUGKS_F64)
    hipLaunchKernelGGL(k_init1<double>, grid, block, 0, S1(x), x->inst<double>(1), d, x->bcoef_p(t0),
                       x->bcoef_q(t0), x->bcoef_p(tm), x->bcoef_q(tm), x->dcoef(t0), x->dt, x->h);
  else
    hipLaunchKernelGGL(k_init1<float>, grid, block, 0, S1(x), x->inst<float>(1), d, x->bcoef_p(t0),
                       x->bcoef_q(t0), x->bcoef_p(tm), x->bcoef_q(tm), x->dcoef(t0), x->dt, x->h);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(S1(x));
  if (e != hipSuccess) return x->hipfail(e, "initialise");
  x->parity = 0;   // inst(1) writes buffer 0
  x->steps = 0;
  x->has_state = true;
  x->have_gprev = false;
  return DUGKS_OK;
}

int dugks1_set_state(dugks1_ctx* x, const double* f, const double* phi_prev, int on_device) {
  GUARD1(x);
  if (!x->bound()) return x->fail(DUGKS_E_STATE, "not bound");
  if (!f || !phi_prev) return x->fail(DUGKS_E_ARG, "null argument");
  const double *df = f, *dp = phi_prev;
  if (!on_device) {
    double* st = (double*)(x->ws + x->off_stage);
    hipError_t e = hipMemcpyAsync(st, f, sizeof(double) * 3 * x->nx, hipMemcpyHostToDevice, S1(x));
    if (e == hipSuccess)
      e = hipMemcpyAsync(st + 3 * (size_t)x->nx, phi_prev, sizeof(double) * x->nx, hipMemcpyHostToDevice, S1(x));
    if (e != hipSuccess) return x->hipfail(e, "copy to device");
    df = st;
    dp = st + 3 * (size_t)x->nx;
  }
  const dim3 grid((x->nx + 255) / 256), block(256);
  if (x->p.storage == DUGKS_F64)
    hipLaunchKernelGGL(k_set1<double>, grid, block, 0, S1(x), (double*)(x->ws + x->off_buf[0]), df, dp, x->nx,
                       x->pitch);
  else
    hipLaunchKernelGGL(k_set1<float>, grid, block, 0, S1(x), (float*)(x->ws + x->off_buf[0]), df, dp, x->nx,
                       x->pitch);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(S1(x));
  if (e != hipSuccess) return x->hipfail(e, "set state");
  x->parity = 0;
  x->steps = 0;
  x->has_state = true;
  x->have_gprev = false;
  return DUGKS_OK;
}

int dugks1_set_dirichlet(dugks1_ctx* x, const double* ghosts, int nsteps) {
  GUARD1(x);
  if (x->p.bc != DUGKS_BC_DIRICHLET) return x->fail(DUGKS_E_STATE, "walls are periodic");
  if (!ghosts || nsteps < 1) return x->fail(DUGKS_E_ARG, "ghosts must be non-null with nsteps >= 1");
  if (!x->bound()) return x->fail(DUGKS_E_STATE, "not bound");
  if (x->have_gprev && x->ghosts) {
    // keep the pair of the last step taken (the ghosts' t_{n-1} values) in the slot
    const double* last = x->ghosts_pos > 0 ? x->ghosts + 2 * (size_t)(x->ghosts_pos - 1)
                                           : (const double*)(x->ws + x->off_gslot);
    if (last != (const double*)(x->ws + x->off_gslot)) {
      hipError_t e = hipMemcpyAsync(x->ws + x->off_gslot, last, 2 * sizeof(double), hipMemcpyDeviceToDevice, S1(x));
      if (e != hipSuccess) return x->hipfail(e, "keep the last ghost pair");
    }
  }
  x->ghosts = ghosts;
  x->ghosts_n = nsteps;
  x->ghosts_pos = 0;
  return DUGKS_OK;
}

int dugks1_step(dugks1_ctx* x, int nsteps) {
  GUARD1(x);
  if (!x->bound()) return x->fail(DUGKS_E_STATE, "not bound");
  if (!x->has_state) return x->fail(DUGKS_E_STATE, "no state: call dugks1_set_phi or dugks1_set_state");
  if (nsteps < 0) return x->fail(DUGKS_E_ARG, "nsteps must be >= 0");
  if (x->p.bc == DUGKS_BC_DIRICHLET && x->ghosts_n - x->ghosts_pos < nsteps)
    return x->fail(DUGKS_E_STATE, "Dirichlet data exhausted: supply more with dugks1_set_dirichlet");
  for (int s = 0; s < nsteps; ++s) {
    if (x->p.storage == DUGKS_F64) launch_step<double>(x);
    else launch_step<float>(x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return x->hipfail(e, "step launch");
    x->parity ^= 1;
    x->steps += 1;
    if (x->p.bc == DUGKS_BC_DIRICHLET) x->ghosts_pos += 1;
    x->have_gprev = true;
  }
  return DUGKS_OK;
}

static int read_out(dugks1_ctx* x, double* out, int on_device, int what) {
  GUARD1(x);
  if (!x->bound() || !x->has_state) return x->fail(DUGKS_E_STATE, "no state");
  if (!out) return x->fail(DUGKS_E_ARG, "null output");
  const size_t count = (what == 1 ? 3 : 1) * (size_t)x->nx;
  double* dst = on_device ? out : (double*)(x->ws + x->off_stage);
  const dim3 grid((x->nx + 255) / 256), block(256);
  const void* st = x->ws + x->off_buf[x->parity];
  if (x->p.storage == DUGKS_F64)
    hipLaunchKernelGGL(k_get1<double>, grid, block, 0, S1(x), (const double*)st, dst, x->nx, x->pitch, what);
  else
    hipLaunchKernelGGL(k_get1<float>, grid, block, 0, S1(x), (const float*)st, dst, x->nx, x->pitch, what);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && !on_device)
    e = hipMemcpyAsync(out, dst, sizeof(double) * count, hipMemcpyDeviceToHost, S1(x));
  if (e == hipSuccess) e = hipStreamSynchronize(S1(x));
  if (e != hipSuccess) return x->hipfail(e, "read out");
  return DUGKS_OK;
}

int dugks1_get_phi(dugks1_ctx* x, double* out, int on_device) { return read_out(x, out, on_device, 0); }
int dugks1_get_f(dugks1_ctx* x, double* out, int on_device) { return read_out(x, out, on_device, 1); }
int dugks1_get_phi_prev(dugks1_ctx* x, double* out, int on_device) { return read_out(x, out, on_device, 2); }

int dugks1_reduce(dugks1_ctx* x, const double* ref, double* mass, double* gre, double* rel_l2) {
  GUARD1(x);
  if (!x->bound() || !x->has_state) return x->fail(DUGKS_E_STATE, "no state");
  double* partial = (double*)(x->ws + x->off_partial);
  double* dout = (double*)(x->ws + x->off_out);
  const void* st = x->ws + x->off_buf[x->parity];
  const int nb = std::min(kRedBlocks, (x->nx + kRedThreads - 1) / kRedThreads);
  if (x->p.storage == DUGKS_F64)
    hipLaunchKernelGGL(k_reduce1<double>, dim3(nb), dim3(kRedThreads), 0, S1(x), (const double*)st, ref,
                       (const double*)(x->ws + x->off_xf), x->nx, x->pitch, partial);
  else
    hipLaunchKernelGGL(k_reduce1<float>, dim3(nb), dim3(kRedThreads), 0, S1(x), (const float*)st, ref,
                       (const double*)(x->ws + x->off_xf), x->nx, x->pitch, partial);
  hipLaunchKernelGGL(k_reduce1_final, dim3(1), dim3(64), 0, S1(x), partial, nb, dout);
  double h[8] = {0};
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h, dout, sizeof(double) * 6, hipMemcpyDeviceToHost, S1(x));
  if (e == hipSuccess) e = hipStreamSynchronize(S1(x));
  if (e != hipSuccess) return x->hipfail(e, "reduce");
  if (mass) *mass = h[0];
  if (ref) {
    if (gre) *gre = h[1] / h[2];
    if (rel_l2) *rel_l2 = sqrt(h[3] / h[4]);
  }
  if (h[5] > 0) return x->fail(DUGKS_E_UNSTABLE, "non-finite values in the state");
  return DUGKS_OK;
}

int dugks1_time_steps(dugks1_ctx* x, int nsteps, float* ms) {
  GUARD1(x);
  if (!ms) return x->fail(DUGKS_E_ARG, "null output");
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return x->fail(DUGKS_E_HIP, "event");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return x->fail(DUGKS_E_HIP, "event");
  }
  (void)hipEventRecord(a, S1(x));
  int rc = dugks1_step(x, nsteps);
  (void)hipEventRecord(b, S1(x));
  hipError_t e = hipEventSynchronize(b);
  float t = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  if (e != hipSuccess) return x->hipfail(e, "timing");
  *ms = t;
  return DUGKS_OK;
}

int dugks1_get_info(const dugks1_ctx* x, dugks1_info* out) {
  if (!x || x->magic != kMagic1 || !out) return DUGKS_E_ARG;
  memset(out, 0, sizeof(*out));
  out->dt = x->dt;
  out->h = x->h;
  out->lambda = x->lambda;
  out->cs2 = x->cs2;
  out->time = x->time();
  out->steps = x->steps;
  out->nx = x->nx;
  out->storage = x->p.storage;
  out->bc = x->p.bc;
  out->dirichlet_left = x->p.bc == DUGKS_BC_DIRICHLET ? x->ghosts_n - x->ghosts_pos : 0;
  out->state_bytes = x->buf_bytes;
  return DUGKS_OK;
}

const char* dugks1_last_error(const dugks1_ctx* x) {
  if (!x || x->magic != kMagic1) return "invalid handle";
  return x->err.c_str();
}

void dugks1_destroy(dugks1_ctx* x) {
  if (!x || x->magic != kMagic1) return;
  x->magic = 0;
  delete x;
}

}  // extern "C"
