// Host runtime of the three-dimensional DUGKS path (include/dugks3d.h):
// setup constants (Sec. 2, Sec. 3), per-axis mesh tables, the equilibrium as
// per-direction polynomials in phi (eq. 2.3 with C = int B'B'^T, Remark 3),
// the workspace layout, launches and read-outs.
#include <hip/hip_runtime.h>

#include <math.h>

#include <cmath>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dugks3d.h"
#include "dugks3d_internal.h"

using namespace dugks3;

namespace {

constexpr uint32_t kMagic3 = 0x44554733u;  // "DUG3"

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

const int kE15[15][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                         {0, 0, 1},  {0, 0, -1},  {1, 1, 1},  {1, 1, -1},  {1, -1, 1},
                         {-1, 1, 1}, {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}};
const int kE19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                         {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                         {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1},
                         {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

// Mesh table of one axis (layout in dugks3d_internal.h).
void axis_table(const std::vector<double>& f, int bc, double h, double c, double dt, double b3,
                std::vector<double>& geo, std::vector<double>& widths) {
  const int n = (int)f.size() - 1;
  std::vector<double> w(n + 2), xc(n + 2);
  for (int i = 0; i < n; ++i) {
    w[i + 1] = f[i + 1] - f[i];
    xc[i + 1] = 0.5 * (f[i] + f[i + 1]);
  }
  w[0] = bc == DUGKS_BC_PERIODIC ? w[n] : w[1];
  w[n + 1] = bc == DUGKS_BC_PERIODIC ? w[1] : w[n];
  xc[0] = f[0] - 0.5 * w[0];
  xc[n + 1] = f[n] + 0.5 * w[n + 1];
  geo.assign((size_t)(n + 2) * kGeo, 0.0);
  for (int m = 0; m <= n; ++m) {  // face between cells m-1 and m
    const double dn = xc[m + 1] - xc[m], wl = f[m] - xc[m];
    double* g = &geo[(size_t)(m + 1) * kGeo];
    g[0] = (wl + h * c) / dn;
    g[1] = wl / dn;
    g[2] = (wl - h * c) / dn;
  }
  for (int m = 0; m < n; ++m) {
    double* g = &geo[(size_t)(m + 1) * kGeo];
    g[3] = 0.5 * h * c / (xc[m + 2] - xc[m]);
    g[4] = dt * c / w[m + 1] * b3;
  }
  widths.assign(w.begin() + 1, w.begin() + 1 + n);
}

}  // namespace

struct dugks3_ctx {
  uint32_t magic = kMagic3;
  std::string err;
  int n[3] = {0, 0, 0};
  int q = 19;
  dugks3_params p{};
  std::vector<double> faces[3];
  int bdeg = 0, ddeg = 1;
  double b[3][DUGKS_MAX_DEG + 1] = {{0}};
  double d[6][DUGKS_MAX_DEG + 1] = {{0}};  // xx yy zz xy xz yz
  // derived
  double cs2 = 0, lambda = 0, dt = 0, h = 0, a1 = 0, b1 = 0, a2 = 0, b2 = 0, a3 = 0, b3 = 0;
  int pitch = 0, ncoef = 2;
  double e[kMaxQ][kMaxCoef] = {{0}};
  std::vector<double> geo[3], widths;
  Launch3 launch;
  // device
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  size_t off_table = 0, off_buf[2] = {0, 0}, off_geo[3] = {0, 0, 0}, off_geof[3] = {0, 0, 0},
         off_widths = 0, off_partial = 0, off_out = 0, off_stage = 0, total = 0;
  size_t buf_bytes = 0, stage_bytes = 0;
  Inst3 host{};
  bool initialised = false;
  long long step = 0;
  const double* ring = nullptr;   // Dirichlet data (device, caller-owned)
  long long ring_steps = 0;
  // sources (device, caller-owned): the shapes G_j
  const double* src_g = nullptr;
  int src_n = 0;
  int src_pow[DUGKS_MAX_SRC_TERMS] = {0};
  double src_gam[DUGKS_MAX_SRC_TERMS] = {0};

  int fail(int rc, const std::string& m) { err = m; return rc; }
  int hipfail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return DUGKS_E_HIP;
  }
  long long cells() const { return (long long)n[0] * n[1] * n[2]; }
  bool any_dirichlet() const {
    return p.bc[0] == DUGKS_BC_DIRICHLET || p.bc[1] == DUGKS_BC_DIRICHLET || p.bc[2] == DUGKS_BC_DIRICHLET;
  }
  bool bound() const { return ws != nullptr; }
  size_t elem() const { return p.storage == DUGKS_F64 ? 8 : 4; }

  void equilibrium_polys() {
    const double c = p.c;
    double w[kMaxQ];
    int e3[kMaxQ][3];
    for (int i = 0; i < q; ++i) {
      for (int a = 0; a < 3; ++a) e3[i][a] = q == 19 ? kE19[i][a] : kE15[i][a];
      w[i] = q == 15 ? (i == 0 ? 2.0 / 9 : (i <= 6 ? 1.0 / 9 : 1.0 / 72))
             : q == 19 ? (i == 0 ? 1.0 / 3 : (i <= 6 ? 1.0 / 18 : 1.0 / 36))
                       : (i == 0 ? 0.0 : 1.0 / 6);
    }
    // C_ab = int B'_a B'_b: coefficient of phi^m
    double C[3][3][kMaxCoef] = {{{0}}};
    for (int a = 0; a < 3; ++a)
      for (int bb = 0; bb < 3; ++bb)
        for (int k = 1; k <= bdeg; ++k)
          for (int l = 1; l <= bdeg; ++l) {
            const int m = k + l - 1;
            C[a][bb][m] += (double)(k * l) / m * b[a][k] * b[bb][l];
          }
    static const int AB[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    double D[3][3][kMaxCoef] = {{{0}}};
    for (int s = 0; s < 6; ++s)
      for (int m = 0; m <= DUGKS_MAX_DEG; ++m) {
        D[AB[s][0]][AB[s][1]][m] = d[s][m];
        D[AB[s][1]][AB[s][0]][m] = d[s][m];
      }
    memset(e, 0, sizeof(e));
    int deg = 1;
    for (int m = 0; m < kMaxCoef; ++m)
      for (int i = 0; i < q; ++i) {
        double v = (m == 1 ? 1.0 : 0.0);
        for (int a = 0; a < 3; ++a)
          v += c * e3[i][a] * (m <= DUGKS_MAX_DEG ? b[a][m] : 0.0) / cs2;
        if (q != 7) {
          double contr = 0.0;
          for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb) {
              const double M = cs2 * D[a][bb][m] + C[a][bb][m] - (a == bb && m == 1 ? cs2 : 0.0);
              contr += M * (c * e3[i][a] * c * e3[i][bb] - (a == bb ? cs2 : 0.0));
            }
          v += contr / (2.0 * cs2 * cs2);
        }
        e[i][m] = w[i] * v;
        if (e[i][m] != 0.0) deg = std::max(deg, m);
      }
    ncoef = deg + 1;
  }

  void fill_host() {
    Inst3& d3 = host;
    memset(&d3, 0, sizeof(d3));
    d3.buf[0] = ws + off_buf[0];
    d3.buf[1] = ws + off_buf[1];
    for (int a = 0; a < 3; ++a) {
      d3.geo[a] = (const double*)(ws + off_geo[a]);
      d3.geof[a] = (const float*)(ws + off_geof[a]);
      d3.n[a] = n[a];
      d3.bc[a] = p.bc[a];
    }
    d3.plane = (long long)n[2] * n[1] * pitch;
    d3.buf_bytes = (unsigned)buf_bytes;
    d3.pitch = pitch;
    d3.q = q;
    d3.ncoef = ncoef;
    d3.storage = p.storage;
    d3.ra = a1 / b1;
    d3.rb = a3 * b1 / b3;
    d3.b1 = b1;
    d3.kg = 4.0 / 3.0 * b1;
    d3.inv_b1 = 1.0 / b1;
    d3.raf = (float)d3.ra; d3.rbf = (float)d3.rb; d3.b1f = (float)d3.b1; d3.kgf = (float)d3.kg;
    d3.inv_b1f = (float)d3.inv_b1;
    d3.ring = ring;
    d3.ring_len = shell_len(n[0], n[1], n[2]);
    d3.src_g = src_g;
    d3.src_plane = cells();
    d3.src_n = src_n;
    d3.src_implicit = 0;
    for (int t = 0; t < src_n; ++t) {
      d3.src_pow[t] = src_pow[t];
      d3.src_gam[t] = src_gam[t];
      if (src_pow[t] > 0) d3.src_implicit = 1;
    }
    d3.dt = dt;
    d3.lambda = lambda;
    for (int a = 0; a < 3; ++a)
      for (int m = 0; m < 4; ++m) d3.bp[a][m] = p.c * (m + 1) * b[a][m + 1] / cs2;
    for (int i = 0; i < q; ++i)
      for (int m = 0; m < kMaxCoef; ++m) {
        d3.e[i][m] = e[i][m];
        d3.ef[i][m] = (float)e[i][m];
      }
  }

  int upload() {
    fill_host();
    hipError_t er = hipMemcpyAsync(ws + off_table, &host, sizeof(Inst3), hipMemcpyHostToDevice, stream);
    if (er != hipSuccess) return hipfail(er, "upload instance");
    for (int a = 0; a < 3; ++a) {
      std::vector<float> gf(geo[a].begin(), geo[a].end());
      er = hipMemcpyAsync(ws + off_geo[a], geo[a].data(), sizeof(double) * geo[a].size(),
                          hipMemcpyHostToDevice, stream);
      if (er == hipSuccess)
        er = hipMemcpyAsync(ws + off_geof[a], gf.data(), sizeof(float) * gf.size(),
                            hipMemcpyHostToDevice, stream);
      if (er != hipSuccess) return hipfail(er, "upload mesh tables");
      er = hipStreamSynchronize(stream);  // gf is a local
      if (er != hipSuccess) return hipfail(er, "synchronise");
    }
    er = hipMemcpyAsync(ws + off_widths, widths.data(), sizeof(double) * widths.size(),
                        hipMemcpyHostToDevice, stream);
    if (er != hipSuccess) return hipfail(er, "upload widths");
    er = hipStreamSynchronize(stream);
    return er == hipSuccess ? DUGKS_OK : hipfail(er, "synchronise");
  }

  const Inst3* dev() const { return (const Inst3*)(ws + off_table); }

  // LDS bytes of a block for the launch and the device limit per block
  size_t lds_bytes(const Launch3& l) const {
    // the instantiation with mirror code runs with walls, with more than four
    // equilibrium coefficients or with a source
    const bool walls = p.bc[0] != DUGKS_BC_PERIODIC || p.bc[1] != DUGKS_BC_PERIODIC ||
                       p.bc[2] != DUGKS_BC_PERIODIC || ncoef > 4 || src_n > 0;
    return step3_lds_bytes(p.storage, q, walls, l, src_n > 0);
  }
  size_t lds_limit() const {
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    return (size_t)v;
  }

  // Stage a host array into the workspace staging area (or use a device pointer).
  int stage_in(const double* src, size_t count, int on_device, const double** out) {
    if (on_device) { *out = src; return DUGKS_OK; }
    if (count * sizeof(double) > stage_bytes) return fail(DUGKS_E_ARG, "array larger than the staging area");
    hipError_t er = hipMemcpyAsync(ws + off_stage, src, count * sizeof(double), hipMemcpyHostToDevice, stream);
    if (er != hipSuccess) return hipfail(er, "copy to device");
    *out = (const double*)(ws + off_stage);
    return DUGKS_OK;
  }
  int read_out(double* out, size_t count, int on_device, int want_f) {
    if (!bound()) return fail(DUGKS_E_STATE, "not bound");
    if (!initialised) return fail(DUGKS_E_STATE, "state not initialised");
    if (!out) return fail(DUGKS_E_ARG, "out is NULL");
    double* dst = on_device ? out : (double*)(ws + off_stage);
    if (!on_device && count * sizeof(double) > stage_bytes) return fail(DUGKS_E_ARG, "too large");
    const int rc = want_f ? launch_get_f3(dev(), host, dst, (int)(step & 1), stream)
                          : launch_get_phi3(dev(), host, dst, (int)(step & 1), step, stream);
    if (rc) return fail(DUGKS_E_HIP, "read-out launch failed");
    hipError_t er = on_device ? hipSuccess
                              : hipMemcpyAsync(out, dst, count * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (er == hipSuccess) er = hipStreamSynchronize(stream);
    return er == hipSuccess ? DUGKS_OK : hipfail(er, "read-out");
  }
};

#define GUARD3(ctx)                                                      \
  do {                                                                   \
    if (!(ctx) || (ctx)->magic != kMagic3) return DUGKS_E_ARG;           \
  } while (0)

extern "C" {

int dugks3_create(dugks3_ctx** out, int nx, int ny, int nz, const double* xf, const double* yf,
                  const double* zf, int q, const dugks3_params* p) {
  if (!out) return DUGKS_E_ARG;
  dugks3_ctx* x = new dugks3_ctx();
  *out = x;
  if (!p) return x->fail(DUGKS_E_ARG, "params is NULL");
  if (p->abi_version != DUGKS3_ABI_VERSION) return x->fail(DUGKS_E_ARG, "abi_version mismatch");
  if (nx < 1 || ny < 1 || nz < 1) return x->fail(DUGKS_E_ARG, "sizes must be >= 1");
  if (ny > 65535 || nz > 65535) return x->fail(DUGKS_E_ARG, "ny and nz must be <= 65535");
  if (!xf || !yf || !zf) return x->fail(DUGKS_E_ARG, "faces are NULL");
  if (!(p->c > 0) || !(p->cfl > 0 && p->cfl < 1) || !(p->alpha > 0))
    return x->fail(DUGKS_E_ARG, "c, cfl or alpha out of range");
  if (q != 15 && q != 19 && q != 7) return x->fail(DUGKS_E_UNSUPPORTED, "q must be 15, 19 or 7");
  if (p->storage != DUGKS_F64 && p->storage != DUGKS_F32)
    return x->fail(DUGKS_E_UNSUPPORTED, "three-dimensional storage is binary64 or binary32");
  for (int a = 0; a < 3; ++a)
    if (p->bc[a] != DUGKS_BC_PERIODIC && p->bc[a] != DUGKS_BC_MIRROR && p->bc[a] != DUGKS_BC_DIRICHLET)
      return x->fail(DUGKS_E_ARG, "unknown boundary kind");
  const int ns[3] = {nx, ny, nz};
  const double* fs[3] = {xf, yf, zf};
  x->q = q;
  x->p = *p;
  double dmin = 1e300;
  for (int a = 0; a < 3; ++a) {
    x->n[a] = ns[a];
    x->faces[a].assign(fs[a], fs[a] + ns[a] + 1);
    for (int i = 0; i < ns[a]; ++i) {
      const double wdt = fs[a][i + 1] - fs[a][i];
      if (!(wdt > 0)) return x->fail(DUGKS_E_ARG, "faces must increase strictly");
      dmin = std::min(dmin, wdt);
    }
  }
  x->pitch = (nx + 63) / 64 * 64;
  x->cs2 = p->c * p->c / 3.0;
  x->lambda = p->alpha / x->cs2;
  x->dt = p->cfl * dmin / p->c;
  x->h = 0.5 * x->dt;
  const double L = x->lambda, dt = x->dt, h = x->h;
  x->a1 = (2 * L - h) / (2 * L + dt); x->b1 = 3 * h / (2 * L + dt);
  x->a2 = (2 * L - dt) / (2 * L + dt); x->b2 = 2 * dt / (2 * L + dt);
  x->a3 = 2 * L / (2 * L + h); x->b3 = h / (2 * L + h);
  x->d[0][1] = x->d[1][1] = x->d[2][1] = 1.0;   // D = phi I until set
  x->equilibrium_polys();
  x->widths.clear();
  for (int a = 0; a < 3; ++a) {
    std::vector<double> w;
    axis_table(x->faces[a], p->bc[a], h, p->c, dt, x->b3, x->geo[a], w);
    x->widths.insert(x->widths.end(), w.begin(), w.end());
  }
  const size_t plane = (size_t)nz * ny * x->pitch;
  x->buf_bytes = plane * q * x->elem();
  if (x->buf_bytes >= 4294967296ull) return x->fail(DUGKS_E_ARG, "one state buffer exceeds 4 GiB");
  // The state buffers start 2 KiB into the workspace, the instance table
  // after them, so that the table's size does not move them: the step's
  // speed depends on where they sit (HBM channel and L2 mapping).  Over
  // offsets from 0 to 2 MiB on a 256^3 D3Q19 mesh, 2 KiB is among the
  // fastest in both storages, while 2304 B costs binary64 9%.
  size_t off = 2048;
  x->off_buf[0] = off; off += align256(x->buf_bytes);
  x->off_buf[1] = off; off += align256(x->buf_bytes);
  x->off_table = off; off += align256(sizeof(Inst3));
  for (int a = 0; a < 3; ++a) {
    x->off_geo[a] = off; off += align256(sizeof(double) * x->geo[a].size());
    x->off_geof[a] = off; off += align256(sizeof(float) * x->geo[a].size());
  }
  x->off_widths = off; off += align256(sizeof(double) * x->widths.size());
  x->off_partial = off; off += align256(sizeof(double) * 8 * reduce3_partials());
  x->off_out = off; off += align256(sizeof(double) * 8);
  x->stage_bytes = sizeof(double) * (size_t)q * x->cells();
  x->off_stage = off; off += align256(x->stage_bytes);
  x->total = off;
  // default launch: binary64 two rows; binary32 four rows (D3Q15 with
  // walls: two, which lets two blocks share a CU) -- the fastest at 256^3
  const bool walls = p->bc[0] != DUGKS_BC_PERIODIC || p->bc[1] != DUGKS_BC_PERIODIC || p->bc[2] != DUGKS_BC_PERIODIC;
  x->launch.rows = p->storage == DUGKS_F64 ? 2 : ((q == 15 && walls) ? 2 : 4);
  // Planes a chunk.  D3Q15 and D3Q19: the blocks run in rounds of (CUs x
  // blocks a CU, from the LDS: 160 KiB a CU) and a block takes about
  // (planes + 3) plane times (its prologue stages and makes two planes), so
  // take the length in 4..128 that minimises rounds x (planes + 3), the
  // longer on a tie; 256 CUs.  This picks the fastest measured length on
  // D3Q19 binary32 from 48^3 to 256^3 (64^3: 8 planes, 30 us a step; 192^3:
  // 16, 428 us; 256^3: 64) and on binary64 and D3Q15 at 256^3.  D3Q7, whose
  // smaller blocks share a CU: 32 planes, halved down to 4 while the grid has
  // fewer than 512 blocks.
  {
    const long long strips = (nx + kCols - 1) / kCols, tiles = (ny + x->launch.rows - 1) / x->launch.rows;
    int best = 4;
    if (q == 7) {
      best = 32;
      while (best > 4 && strips * tiles * ((nz + best - 1) / best) < 512) best /= 2;
    } else {
      const size_t lds = x->lds_bytes(x->launch);
      const long long per_cu = std::max<long long>(1, (long long)(163840 / std::max<size_t>(lds, 1)));
      const long long slots = 256 * per_cu;
      long long best_cost = -1;
      for (int planes = 128; planes >= 4; planes /= 2) {
        const long long blocks = strips * tiles * ((nz + planes - 1) / planes);
        const long long cost = ((blocks + slots - 1) / slots) * (planes + 3);
        if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = planes; }
      }
    }
    x->launch.planes = best;
  }
  return DUGKS_OK;
}

size_t dugks3_workspace_bytes(const dugks3_ctx* ctx) {
  return (ctx && ctx->magic == kMagic3) ? ctx->total : 0;
}

int dugks3_bind(dugks3_ctx* ctx, void* ws, size_t bytes, void* stream) {
  GUARD3(ctx);
  if (!ws) return ctx->fail(DUGKS_E_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return ctx->fail(DUGKS_E_ARG, "workspace must be 256-byte aligned");
  if (bytes < ctx->total) return ctx->fail(DUGKS_E_NOMEM, "workspace too small");
  ctx->ws = (char*)ws;
  ctx->ws_bytes = bytes;
  ctx->stream = (hipStream_t)stream;
  ctx->initialised = false;
  return ctx->upload();
}

int dugks3_set_B(dugks3_ctx* ctx, int deg, const double* b) {
  GUARD3(ctx);
  if (deg < 0 || deg > DUGKS_MAX_DEG || !b) return ctx->fail(DUGKS_E_ARG, "bad B");
  memset(ctx->b, 0, sizeof(ctx->b));
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k <= deg; ++k) ctx->b[a][k] = b[a * (deg + 1) + k];
  ctx->bdeg = deg;
  ctx->equilibrium_polys();
  return ctx->bound() ? ctx->upload() : DUGKS_OK;
}

int dugks3_set_D(dugks3_ctx* ctx, int deg, const double* d) {
  GUARD3(ctx);
  if (deg < 0 || deg > DUGKS_MAX_DEG || !d) return ctx->fail(DUGKS_E_ARG, "bad D");
  if (ctx->q == 7) {
    for (int s = 0; s < 6; ++s)
      for (int k = 0; k <= deg; ++k) {
        const double want = (s < 3 && k == 1) ? 1.0 : 0.0;
        if (d[s * (deg + 1) + k] != want)
          return ctx->fail(DUGKS_E_UNSUPPORTED, "D3Q7 takes D = phi I only (Remark 3)");
      }
  }
  memset(ctx->d, 0, sizeof(ctx->d));
  for (int s = 0; s < 6; ++s)
    for (int k = 0; k <= deg; ++k) ctx->d[s][k] = d[s * (deg + 1) + k];
  ctx->ddeg = deg;
  ctx->equilibrium_polys();
  return ctx->bound() ? ctx->upload() : DUGKS_OK;
}

int dugks3_set_phi(dugks3_ctx* ctx, const double* phi, int on_device) {
  GUARD3(ctx);
  if (!ctx->bound()) return ctx->fail(DUGKS_E_STATE, "not bound");
  if (!phi) return ctx->fail(DUGKS_E_ARG, "phi is NULL");
  const double* src;
  int rc = ctx->stage_in(phi, (size_t)ctx->cells(), on_device, &src);
  if (rc) return rc;
  if (launch_init3(ctx->dev(), ctx->host, src, 0, ctx->stream)) return ctx->fail(DUGKS_E_HIP, "init launch failed");
  hipError_t er = hipStreamSynchronize(ctx->stream);
  if (er != hipSuccess) return ctx->hipfail(er, "initialise");
  ctx->step = 0;
  ctx->initialised = true;
  return DUGKS_OK;
}

int dugks3_set_f(dugks3_ctx* ctx, const double* f, int on_device) {
  GUARD3(ctx);
  if (!ctx->bound()) return ctx->fail(DUGKS_E_STATE, "not bound");
  if (!f) return ctx->fail(DUGKS_E_ARG, "f is NULL");
  const double* src;
  int rc = ctx->stage_in(f, (size_t)ctx->q * ctx->cells(), on_device, &src);
  if (rc) return rc;
  if (launch_set_f3(ctx->dev(), ctx->host, src, 0, ctx->stream)) return ctx->fail(DUGKS_E_HIP, "set_f launch failed");
  hipError_t er = hipStreamSynchronize(ctx->stream);
  if (er != hipSuccess) return ctx->hipfail(er, "set_f");
  ctx->step = 0;
  ctx->initialised = true;
  return DUGKS_OK;
}

size_t dugks3_source_scratch_bytes(const dugks3_ctx*) {
  return 0;   // every lattice takes the source in the fused step
}

int dugks3_set_source_terms(dugks3_ctx* ctx, int nterms, const double* g_dev, const int* powers,
                            const double* gammas, void* /*scratch_dev*/, size_t /*scratch_bytes*/) {
  GUARD3(ctx);
  if (nterms < 0 || nterms > DUGKS_MAX_SRC_TERMS) return ctx->fail(DUGKS_E_ARG, "nterms out of range");
  if (nterms > 0) {
    if (!g_dev || !powers || !gammas) return ctx->fail(DUGKS_E_ARG, "source arrays are NULL");
    for (int t = 0; t < nterms; ++t) {
      if (powers[t] < 0 || powers[t] > DUGKS_MAX_SRC_POW) return ctx->fail(DUGKS_E_ARG, "power out of range");
      if (!std::isfinite(gammas[t])) return ctx->fail(DUGKS_E_ARG, "growth rate not finite");
    }
  }
  ctx->src_n = nterms;
  ctx->src_g = nterms > 0 ? g_dev : nullptr;
  for (int t = 0; t < DUGKS_MAX_SRC_TERMS; ++t) {
    ctx->src_pow[t] = t < nterms ? powers[t] : 0;
    ctx->src_gam[t] = t < nterms ? gammas[t] : 0.0;
  }
  return ctx->bound() ? ctx->upload() : DUGKS_OK;
}

int dugks3_set_dirichlet(dugks3_ctx* ctx, const double* ring_dev, int nsteps) {
  GUARD3(ctx);
  if (nsteps < 0 || (nsteps > 0 && !ring_dev)) return ctx->fail(DUGKS_E_ARG, "bad Dirichlet data");
  ctx->ring = nsteps > 0 ? ring_dev : nullptr;
  ctx->ring_steps = nsteps;
  return ctx->bound() ? ctx->upload() : DUGKS_OK;
}

int dugks3_step(dugks3_ctx* ctx, int nsteps) {
  GUARD3(ctx);
  if (nsteps < 0) return ctx->fail(DUGKS_E_ARG, "nsteps < 0");
  if (!ctx->bound()) return ctx->fail(DUGKS_E_STATE, "not bound");
  if (!ctx->initialised) return ctx->fail(DUGKS_E_STATE, "state not initialised");
  if (ctx->lds_bytes(ctx->launch) > ctx->lds_limit())
    return ctx->fail(DUGKS_E_ARG, "launch needs more LDS than a block may hold");
  if (ctx->any_dirichlet() && (ctx->ring == nullptr || ctx->step + nsteps > ctx->ring_steps))
    return ctx->fail(DUGKS_E_STATE, "Dirichlet walls need data for every step (dugks3_set_dirichlet)");
  for (int s = 0; s < nsteps; ++s) {
    const int rc = launch_step3(ctx->dev(), ctx->host, (int)(ctx->step & 1), ctx->step, ctx->launch, ctx->stream);
    if (rc)
      return ctx->fail(DUGKS_E_HIP, std::string("step launch failed: ") + hipGetErrorString(hipGetLastError()));
    ctx->step += 1;
  }
  return DUGKS_OK;
}

int dugks3_get_phi(dugks3_ctx* ctx, double* out, int on_device) {
  GUARD3(ctx);
  return ctx->read_out(out, (size_t)ctx->cells(), on_device, 0);
}

int dugks3_get_f(dugks3_ctx* ctx, double* out, int on_device) {
  GUARD3(ctx);
  return ctx->read_out(out, (size_t)ctx->q * ctx->cells(), on_device, 1);
}

int dugks3_reduce(dugks3_ctx* ctx, const double* ref_dev, double* mass, double* gre, double* rel_l2) {
  GUARD3(ctx);
  if (!ctx->bound()) return ctx->fail(DUGKS_E_STATE, "not bound");
  if (!ctx->initialised) return ctx->fail(DUGKS_E_STATE, "state not initialised");
  double* o = (double*)(ctx->ws + ctx->off_out);
  if (launch_reduce3(ctx->dev(), ctx->host, ref_dev, (int)(ctx->step & 1), ctx->step,
                     (const double*)(ctx->ws + ctx->off_widths), (double*)(ctx->ws + ctx->off_partial), o,
                     ctx->stream))
    return ctx->fail(DUGKS_E_HIP, "reduction launch failed");
  double v[8];
  hipError_t er = hipMemcpyAsync(v, o, sizeof(v), hipMemcpyDeviceToHost, ctx->stream);
  if (er == hipSuccess) er = hipStreamSynchronize(ctx->stream);
  if (er != hipSuccess) return ctx->hipfail(er, "reduce");
  if (mass) *mass = v[0];
  if (gre) *gre = ref_dev ? v[1] / v[2] : 0.0;
  if (rel_l2) *rel_l2 = ref_dev ? sqrt(v[3] / v[4]) : 0.0;
  return v[5] > 0 ? ctx->fail(DUGKS_E_UNSTABLE, "non-finite cells") : DUGKS_OK;
}

int dugks3_set_launch(dugks3_ctx* ctx, int rows, int planes) {
  GUARD3(ctx);
  if (ctx->p.storage == DUGKS_F64 ? (rows < kMinRows64 || rows > kMaxRows64)
                                   : (rows < kMinRows32 || rows > kMaxRows32))
    return ctx->fail(DUGKS_E_ARG, ctx->p.storage == DUGKS_F64 ? "rows_per_block must be 1 or 2 (binary64)"
                                                            : "rows_per_block must be 2, 3 or 4 (binary32)");
  if (planes < 1) return ctx->fail(DUGKS_E_ARG, "planes_per_block must be >= 1");
  Launch3 l;
  l.rows = rows;
  l.planes = planes;
  if (ctx->bound() && ctx->lds_bytes(l) > ctx->lds_limit())
    return ctx->fail(DUGKS_E_ARG, "launch needs more LDS than a block may hold");
  ctx->launch = l;
  return DUGKS_OK;
}

int dugks3_time_steps(dugks3_ctx* ctx, int nsteps, float* ms) {
  GUARD3(ctx);
  if (!ms) return ctx->fail(DUGKS_E_ARG, "ms is NULL");
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return ctx->fail(DUGKS_E_HIP, "event create");
  hipError_t er = hipEventRecord(a, ctx->stream);
  int rc = er == hipSuccess ? dugks3_step(ctx, nsteps) : DUGKS_E_HIP;
  if (rc == DUGKS_OK) er = hipEventRecord(b, ctx->stream);
  if (rc == DUGKS_OK && er == hipSuccess) er = hipEventSynchronize(b);
  if (rc == DUGKS_OK && er == hipSuccess) er = hipEventElapsedTime(ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  return er == hipSuccess ? DUGKS_OK : ctx->hipfail(er, "timing");
}

int dugks3_autotune(dugks3_ctx* ctx, int trial_steps) {
  GUARD3(ctx);
  if (!ctx->bound()) return ctx->fail(DUGKS_E_STATE, "not bound");
  if (!ctx->initialised) return ctx->fail(DUGKS_E_STATE, "state not initialised");
  if (ctx->any_dirichlet() && (ctx->ring == nullptr || ctx->step + 1 > ctx->ring_steps))
    return ctx->fail(DUGKS_E_STATE, "Dirichlet data does not cover the current step");
  if (trial_steps < 1) trial_steps = 1;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return ctx->fail(DUGKS_E_HIP, "event create");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return ctx->fail(DUGKS_E_HIP, "event create");
  }
  // every trial reads the current buffer and writes only the other one, with
  // the current step's Dirichlet data: the state does not change
  const int parity = (int)(ctx->step & 1);
  const bool f64 = ctx->p.storage == DUGKS_F64;
  const int rmin = f64 ? kMinRows64 : kMinRows32, rmax = f64 ? kMaxRows64 : kMaxRows32;
  const int planes_c[] = {4, 8, 16, 32, 64, 128};
  Launch3 best = ctx->launch;
  float best_ms = 1e30f;
  int rc = DUGKS_OK;
  hipError_t er = hipSuccess;
  for (int rows = rmin; rows <= rmax && rc == DUGKS_OK && er == hipSuccess; ++rows)
    for (int planes : planes_c) {
      Launch3 l;
      l.rows = rows;
      l.planes = planes;
      if (ctx->lds_bytes(l) > ctx->lds_limit()) continue;
      if (launch_step3(ctx->dev(), ctx->host, parity, ctx->step, l, ctx->stream)) { rc = DUGKS_E_HIP; break; }
      er = hipEventRecord(a, ctx->stream);
      for (int t = 0; t < trial_steps && er == hipSuccess && rc == DUGKS_OK; ++t)
        if (launch_step3(ctx->dev(), ctx->host, parity, ctx->step, l, ctx->stream)) rc = DUGKS_E_HIP;
      if (rc != DUGKS_OK) break;
      if (er == hipSuccess) er = hipEventRecord(b, ctx->stream);
      if (er == hipSuccess) er = hipEventSynchronize(b);
      float ms = 0.0f;
      if (er == hipSuccess) er = hipEventElapsedTime(&ms, a, b);
      if (er != hipSuccess) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = l;
      }
    }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != DUGKS_OK) return ctx->fail(rc, "autotune launch failed");
  if (er != hipSuccess) return ctx->hipfail(er, "autotune timing");
  ctx->launch = best;
  return DUGKS_OK;
}

int dugks3_get_info(const dugks3_ctx* ctx, dugks3_info* out) {
  if (!ctx || ctx->magic != kMagic3 || !out) return DUGKS_E_ARG;
  memset(out, 0, sizeof(*out));
  out->dt = ctx->dt; out->h = ctx->h; out->lambda = ctx->lambda; out->cs2 = ctx->cs2;
  out->a1 = ctx->a1; out->b1 = ctx->b1; out->a2 = ctx->a2; out->b2 = ctx->b2;
  out->a3 = ctx->a3; out->b3 = ctx->b3;
  out->nx = ctx->n[0]; out->ny = ctx->n[1]; out->nz = ctx->n[2];
  out->q = ctx->q; out->storage = ctx->p.storage; out->pitch = ctx->pitch;
  out->eq_degree = ctx->ncoef - 1;
  out->rows_per_block = ctx->launch.rows;
  out->planes_per_block = ctx->launch.planes;
  Inst3 t{};
  for (int a = 0; a < 3; ++a) t.n[a] = ctx->n[a];
  out->blocks = step3_blocks(t, ctx->launch);
  out->state_bytes = ctx->buf_bytes;
  return DUGKS_OK;
}

const char* dugks3_last_error(const dugks3_ctx* ctx) {
  if (!ctx || ctx->magic != kMagic3) return "invalid handle";
  return ctx->err.c_str();
}

void dugks3_destroy(dugks3_ctx* ctx) {
  if (!ctx || ctx->magic != kMagic3) return;
  ctx->magic = 0;
  delete ctx;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
namespace {
constexpr uint32_t kMagicB3 = 0x44554242u;  // "DUBB"
}

struct dugks3_batch {
  uint32_t magic = kMagicB3;
  std::string err;
  std::vector<dugks3_ctx*> inst;   // caller-owned, bound, kept bound while in the batch
  int q = 19, storage = 0;
  Launch3 launch;
  std::vector<long long> first;    // blocks before instance k (n + 1 entries)
  char* ws = nullptr;              // device: the instance pointers, then `first`
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  size_t off_first = 0, total = 0;

  int fail(int rc, const std::string& m) { err = m; return rc; }
  int ncoef() const {
    int m = 2;
    for (auto* c : inst) m = std::max(m, c->ncoef);
    return m;
  }
  // the instantiation with mirror code runs if any instance has a wall or
  // more than four equilibrium coefficients
  bool walls() const {
    for (auto* c : inst)
      if (c->p.bc[0] != DUGKS_BC_PERIODIC || c->p.bc[1] != DUGKS_BC_PERIODIC || c->p.bc[2] != DUGKS_BC_PERIODIC ||
          c->ncoef > 4)
        return true;
    return false;
  }
  size_t lds_bytes(const Launch3& l) const { return step3_lds_bytes(storage, q, walls(), l); }
  void layout() {
    off_first = align256(sizeof(const Inst3*) * inst.size());
    total = off_first + align256(sizeof(long long) * (inst.size() + 1));
  }
  // the blocks of each instance for the launch, and the device table
  int upload() {
    first.assign(inst.size() + 1, 0);
    for (size_t k = 0; k < inst.size(); ++k) {
      Inst3 t{};
      for (int a = 0; a < 3; ++a) t.n[a] = inst[k]->n[a];
      first[k + 1] = first[k] + step3_blocks(t, launch);
    }
    if (first.back() > 0x7fffffffLL) return fail(DUGKS_E_ARG, "the batch needs more than 2^31 blocks");
    if (!ws) return DUGKS_OK;
    std::vector<const Inst3*> ptr(inst.size());
    for (size_t k = 0; k < inst.size(); ++k) ptr[k] = inst[k]->dev();
    hipError_t e = hipMemcpyAsync(ws, ptr.data(), sizeof(const Inst3*) * ptr.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ws + off_first, first.data(), sizeof(long long) * first.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      err = std::string("batch table upload: ") + hipGetErrorString(e);
      return DUGKS_E_HIP;
    }
    return DUGKS_OK;
  }
};

#define GUARDB3(b)                                                       \
  do {                                                                   \
    if (!(b) || (b)->magic != kMagicB3) return DUGKS_E_ARG;              \
  } while (0)

extern "C" {

int dugks3_batch_create(dugks3_batch** out, int n, dugks3_ctx* const* ctxs) {
  if (!out) return DUGKS_E_ARG;
  *out = nullptr;
  auto* b = new dugks3_batch();
  *out = b;
  if (n < 1 || !ctxs) return b->fail(DUGKS_E_ARG, "a batch needs n >= 1 contexts");
  for (int k = 0; k < n; ++k) {
    dugks3_ctx* c = ctxs[k];
    if (!c || c->magic != kMagic3) return b->fail(DUGKS_E_ARG, "invalid context in the batch");
    if (c->q == 7) return b->fail(DUGKS_E_UNSUPPORTED, "D3Q7 is not batched");
    if (k > 0 && (c->q != b->q || c->p.storage != b->storage))
      return b->fail(DUGKS_E_ARG, "the instances of a batch share the lattice and the storage");
    if (k == 0) {
      b->q = c->q;
      b->storage = c->p.storage;
    }
    b->inst.push_back(c);
  }
  b->launch.rows = b->storage == DUGKS_F64 ? 2 : 4;
  b->launch.planes = 32;
  b->layout();
  return b->upload();
}

size_t dugks3_batch_workspace_bytes(const dugks3_batch* b) {
  return (b && b->magic == kMagicB3) ? b->total : 0;
}

int dugks3_batch_bind(dugks3_batch* b, void* ws, size_t bytes, void* stream) {
  GUARDB3(b);
  if (!ws) return b->fail(DUGKS_E_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return b->fail(DUGKS_E_ARG, "workspace must be 256-byte aligned");
  if (bytes < b->total) return b->fail(DUGKS_E_NOMEM, "workspace too small");
  for (auto* c : b->inst)
    if (!c->bound()) return b->fail(DUGKS_E_STATE, "every instance must be bound first");
  b->ws = (char*)ws;
  b->ws_bytes = bytes;
  b->stream = (hipStream_t)stream;
  return b->upload();
}

int dugks3_batch_set_launch(dugks3_batch* b, int rows, int planes) {
  GUARDB3(b);
  if (b->storage == DUGKS_F64 ? (rows < kMinRows64 || rows > kMaxRows64) : (rows < kMinRows32 || rows > kMaxRows32))
    return b->fail(DUGKS_E_ARG, "rows_per_block out of range for the storage");
  if (planes < 1) return b->fail(DUGKS_E_ARG, "planes_per_block must be >= 1");
  Launch3 l;
  l.rows = rows;
  l.planes = planes;
  if (b->ws && b->lds_bytes(l) > b->inst[0]->lds_limit())
    return b->fail(DUGKS_E_ARG, "launch needs more LDS than a block may hold");
  const Launch3 keep = b->launch;
  b->launch = l;
  const int rc = b->upload();
  if (rc) b->launch = keep;
  return rc;
}

int dugks3_batch_step(dugks3_batch* b, int nsteps) {
  GUARDB3(b);
  if (nsteps < 0) return b->fail(DUGKS_E_ARG, "nsteps < 0");
  if (!b->ws) return b->fail(DUGKS_E_STATE, "not bound");
  const long long step = b->inst[0]->step;
  for (auto* c : b->inst) {
    if (!c->bound() || !c->initialised) return b->fail(DUGKS_E_STATE, "an instance has no state");
    if (c->step != step) return b->fail(DUGKS_E_STATE, "the instances of a batch must be at the same step");
    if (c->src_n > 0) return b->fail(DUGKS_E_UNSUPPORTED, "sources are not batched");
    if (c->any_dirichlet() && (c->ring == nullptr || c->step + nsteps > c->ring_steps))
      return b->fail(DUGKS_E_STATE, "Dirichlet data does not cover the requested steps");
  }
  if (b->lds_bytes(b->launch) > b->inst[0]->lds_limit())
    return b->fail(DUGKS_E_ARG, "launch needs more LDS than a block may hold");
  Inst3 h = b->inst[0]->host;   // template selectors: the largest coefficient count of the batch
  h.ncoef = b->ncoef();
  const Batch3 base{(const Inst3* const*)b->ws, (const long long*)(b->ws + b->off_first), (int)b->inst.size(), 0};
  for (int s = 0; s < nsteps; ++s) {
    Batch3 bt = base;
    bt.step = step + s;
    if (launch_step3_batch(bt, h, (int)(bt.step & 1), b->walls(), b->first.back(), b->launch, b->stream))
      return b->fail(DUGKS_E_HIP, std::string("batch step launch failed: ") + hipGetErrorString(hipGetLastError()));
    for (auto* c : b->inst) c->step += 1;
  }
  return DUGKS_OK;
}

int dugks3_batch_time_steps(dugks3_batch* b, int nsteps, float* ms) {
  GUARDB3(b);
  if (!ms) return b->fail(DUGKS_E_ARG, "ms is NULL");
  if (!b->ws) return b->fail(DUGKS_E_STATE, "not bound");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return b->fail(DUGKS_E_HIP, "event create");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return b->fail(DUGKS_E_HIP, "event create");
  }
  hipError_t er = hipEventRecord(e0, b->stream);
  int rc = er == hipSuccess ? dugks3_batch_step(b, nsteps) : DUGKS_E_HIP;
  if (rc == DUGKS_OK) er = hipEventRecord(e1, b->stream);
  if (rc == DUGKS_OK && er == hipSuccess) er = hipEventSynchronize(e1);
  if (rc == DUGKS_OK && er == hipSuccess) er = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  return er == hipSuccess ? DUGKS_OK : b->fail(DUGKS_E_HIP, "timing");
}

int dugks3_batch_get_info(const dugks3_batch* b, int* rows, int* planes, long long* blocks, long long* cells) {
  if (!b || b->magic != kMagicB3) return DUGKS_E_ARG;
  if (rows) *rows = b->launch.rows;
  if (planes) *planes = b->launch.planes;
  if (blocks) *blocks = b->first.empty() ? 0 : b->first.back();
  if (cells) {
    long long c = 0;
    for (auto* x : b->inst) c += x->cells();
    *cells = c;
  }
  return DUGKS_OK;
}

const char* dugks3_batch_last_error(const dugks3_batch* b) {
  if (!b || b->magic != kMagicB3) return "invalid handle";
  return b->err.c_str();
}

void dugks3_batch_destroy(dugks3_batch* b) {
  if (!b || b->magic != kMagicB3) return;
  b->magic = 0;
  delete b;
}

}  // extern "C"
