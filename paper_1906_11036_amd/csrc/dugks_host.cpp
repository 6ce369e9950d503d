// Host runtime of libdugks: validation, mesh and coefficient tables, the
// workspace layout, the work list, launches, graphs, diagnostics and
// checkpoints behind the C ABI of include/dugks.h.
#include <hip/hip_runtime.h>

#include <math.h>

#include <cmath>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dugks.h"
#include "dugks_internal.h"

namespace dugks {

static constexpr uint32_t kMagicCtx = 0x44554731u;    // "DUG1"
static constexpr uint32_t kMagicBatch = 0x44554742u;  // "DUGB"
// Steps per captured graph: a long graph for long runs and a short one so that
// any run of four or more steps from a phase-0 step replays a graph.  Both are
// multiples of 4, the period of the buffer parity and the 16-bit scale slots.
static constexpr int kGraphSteps[2] = {32, 4};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------------ instance
struct Instance {
  int nx = 0, ny = 0, q = 9;
  dugks_params p{};
  int bcx = 0, bcy = 0;
  std::vector<double> xf, yf;
  int bdeg = 0, ddeg = 1;
  double bx[DUGKS_MAX_DEG + 1] = {0}, by[DUGKS_MAX_DEG + 1] = {0};
  double dxx[DUGKS_MAX_DEG + 1] = {0}, dxy[DUGKS_MAX_DEG + 1] = {0}, dyy[DUGKS_MAX_DEG + 1] = {0};
  // derived
  double cs2 = 0, lambda = 0, dt = 0, h = 0, a1 = 0, b1 = 0, a2 = 0, b2 = 0, a3 = 0, b3 = 0;
  int pitch = 0, ncoef = 2;
  std::vector<double> colgeo, rowgeo, widths;
  std::vector<float> colgeo_f, rowgeo_f;
  double e[kMaxQ][kMaxCoef] = {{0}};
  // E_k = E_swap(k) bitwise for the pairs of directions that swapping x and y
  // exchanges (1-2, 3-4, and 6-8 of D2Q9): the kernels then evaluate one of each
  bool xy_sym = false;
  double bp[2][kRhoCoef] = {{0}};         // c B'(phi) / cs2 per axis, see InstDev
  // source terms exp(src_gam[j] t) phi^src_pow[j] G_j(x); G_j as [src_n][ny][nx]
  // (device, caller-owned)
  const double* src_g = nullptr;
  int src_n = 0;
  int src_pow[kMaxSrcTerms] = {0};
  double src_gam[kMaxSrcTerms] = {0};
  bool src_implicit() const {
    for (int j = 0; j < src_n; ++j)
      if (src_pow[j] > 0) return true;
    return false;
  }
  // workspace offsets
  size_t off_buf[2] = {0, 0}, off_colgeo = 0, off_rowgeo = 0, off_colgeo_f = 0, off_rowgeo_f = 0,
         off_widths = 0, off_slots = 0, off_flags = 0;
  size_t buf_bytes = 0;
  const double* ring = nullptr;
  int ring_steps = 0;

  long long cells() const { return (long long)nx * ny; }
  int planes_elem_bytes(int storage) const {
    return storage == DUGKS_F64 ? 8 : (storage == DUGKS_F32 ? 4 : 2);
  }
  size_t buffer_bytes(int storage) const {
    const size_t plane = (size_t)ny * pitch;
    if (storage == DUGKS_F64) return plane * q * 8;
    if (storage == DUGKS_F32) return plane * q * 4;
    return plane * 4 + plane * (q - 1) * 2;
  }
};

// Axis tables: ghost-aware widths and centres, then the per-column (or row)
// coefficients of the face on the low side, the tangential factor and the
// update factor.  See the header for the ghost geometry.
static void axis_tables(const std::vector<double>& f, int bc, double h, double c, double dt,
                        double b3, std::vector<double>& geo, std::vector<double>& widths) {
  const int n = (int)f.size() - 1;
  std::vector<double> w(n + 2), xc(n + 2);  // index i+1 for cell i in -1..n
  for (int i = 0; i < n; ++i) {
    w[i + 1] = f[i + 1] - f[i];
    xc[i + 1] = 0.5 * (f[i] + f[i + 1]);
  }
  w[0] = bc == DUGKS_BC_PERIODIC ? w[n] : w[1];
  w[n + 1] = bc == DUGKS_BC_PERIODIC ? w[1] : w[n];
  xc[0] = f[0] - 0.5 * w[0];
  xc[n + 1] = f[n] + 0.5 * w[n + 1];
  geo.assign((size_t)(n + 2) * kGeo, 0.0);
  for (int cc = 0; cc <= n; ++cc) {  // face between cells cc-1 and cc
    const double dn = xc[cc + 1] - xc[cc];
    const double wl = f[cc] - xc[cc];
    double* g = &geo[(size_t)(cc + 1) * kGeo];
    g[0] = (wl + h * c) / dn;  // normal velocity -c
    g[1] = wl / dn;            // normal velocity 0
    g[2] = (wl - h * c) / dn;  // normal velocity +c
  }
  for (int cc = 0; cc < n; ++cc) {
    double* g = &geo[(size_t)(cc + 1) * kGeo];
    g[3] = 0.5 * h * c / (xc[cc + 2] - xc[cc]);
    g[4] = dt * c / w[cc + 1] * b3;  // the kernels' fluxes are f_b / b3
  }
  widths.assign(w.begin() + 1, w.begin() + 1 + n);
}

static int validate_params(const dugks_params* p, std::string& err) {
  if (!p) { err = "params is NULL"; return DUGKS_E_ARG; }
  if (p->abi_version != DUGKS_ABI_VERSION) { err = "abi_version mismatch"; return DUGKS_E_ARG; }
  if (!(p->c > 0) || !std::isfinite(p->c)) { err = "c must be > 0"; return DUGKS_E_ARG; }
  if (!(p->cfl > 0) || !(p->cfl < 1)) { err = "cfl must lie in (0, 1)"; return DUGKS_E_ARG; }
  if (!(p->alpha > 0) || !std::isfinite(p->alpha)) { err = "alpha must be > 0"; return DUGKS_E_ARG; }
  for (int s = 0; s < 4; ++s)
    if (p->bc[s] < 0 || p->bc[s] > 2) { err = "unknown boundary kind"; return DUGKS_E_ARG; }
  if (p->bc[0] != p->bc[1] || p->bc[2] != p->bc[3]) {
    err = "both sides of an axis must have the same boundary kind";
    return DUGKS_E_UNSUPPORTED;
  }
  if (p->storage < DUGKS_F64 || p->storage > DUGKS_BF16NEQ) {
    err = "unknown storage";
    return DUGKS_E_UNSUPPORTED;
  }
  if (p->kernel != DUGKS_KERNEL_FUSED && p->kernel != DUGKS_KERNEL_PLAIN) {
    err = "unknown kernel";
    return DUGKS_E_UNSUPPORTED;
  }
  if (p->kernel == DUGKS_KERNEL_PLAIN && p->storage != DUGKS_F64) {
    err = "the plain kernel stores binary64 only";
    return DUGKS_E_UNSUPPORTED;
  }
  return DUGKS_OK;
}

static int init_instance(Instance& in, int nx, int ny, const double* xf, const double* yf, int q,
                         const dugks_params* p, std::string& err) {
  int rc = validate_params(p, err);
  if (rc) return rc;
  if (nx < 1 || ny < 1 || nx > (1 << 20) || ny > (1 << 20) || (long long)nx * ny > (1LL << 31)) {
    err = "grid size out of range";
    return DUGKS_E_ARG;
  }
  if (!xf || !yf) { err = "face arrays are NULL"; return DUGKS_E_ARG; }
  if (q != 9 && q != 5) { err = "q must be 9 or 5"; return DUGKS_E_UNSUPPORTED; }
  for (int i = 0; i < nx; ++i)
    if (!(xf[i + 1] > xf[i]) || !std::isfinite(xf[i])) { err = "xf must increase"; return DUGKS_E_ARG; }
  for (int j = 0; j < ny; ++j)
    if (!(yf[j + 1] > yf[j]) || !std::isfinite(yf[j])) { err = "yf must increase"; return DUGKS_E_ARG; }
  in.nx = nx; in.ny = ny; in.q = q; in.p = *p;
  in.bcx = p->bc[0]; in.bcy = p->bc[2];
  in.xf.assign(xf, xf + nx + 1);
  in.yf.assign(yf, yf + ny + 1);
  in.pitch = ((nx + 63) / 64) * 64;
  if ((size_t)ny * in.pitch * q * (p->storage == DUGKS_F64 ? 8 : 4) >= (size_t)1 << 32) {
    err = "one instance's state must stay below 4 GiB";
    return DUGKS_E_UNSUPPORTED;
  }
  // constants (Sec. 2, Sec. 3)
  in.cs2 = p->c * p->c / 3.0;
  in.lambda = p->alpha / in.cs2;
  double dmin = in.xf[1] - in.xf[0];
  for (int i = 0; i < nx; ++i) dmin = std::min(dmin, in.xf[i + 1] - in.xf[i]);
  for (int j = 0; j < ny; ++j) dmin = std::min(dmin, in.yf[j + 1] - in.yf[j]);
  in.dt = p->cfl * dmin / p->c;
  in.h = 0.5 * in.dt;
  const double L = in.lambda, dt = in.dt, h = in.h;
  in.a1 = (2 * L - h) / (2 * L + dt);
  in.b1 = 3 * h / (2 * L + dt);
  in.a2 = (2 * L - dt) / (2 * L + dt);
  in.b2 = 2 * dt / (2 * L + dt);
  in.a3 = 2 * L / (2 * L + h);
  in.b3 = h / (2 * L + h);
  // default coefficients: B = 0, D = 0
  in.bdeg = 0; in.ddeg = 0;
  memset(in.bx, 0, sizeof(in.bx)); memset(in.by, 0, sizeof(in.by));
  memset(in.dxx, 0, sizeof(in.dxx)); memset(in.dxy, 0, sizeof(in.dxy)); memset(in.dyy, 0, sizeof(in.dyy));
  std::vector<double> wx, wy;
  axis_tables(in.xf, in.bcx, in.h, p->c, in.dt, in.b3, in.colgeo, wx);
  axis_tables(in.yf, in.bcy, in.h, p->c, in.dt, in.b3, in.rowgeo, wy);
  in.widths = wx;
  in.widths.insert(in.widths.end(), wy.begin(), wy.end());
  in.colgeo_f.assign(in.colgeo.begin(), in.colgeo.end());
  in.rowgeo_f.assign(in.rowgeo.begin(), in.rowgeo.end());
  return DUGKS_OK;
}

// E_i(phi) as a polynomial in phi (eq. 2.3 with C = int_0^phi B'B'^T).
static void equilibrium_polys(Instance& in) {
  const int cxs[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int cys[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  double w[9];
  for (int i = 0; i < in.q; ++i)
    w[i] = in.q == 9 ? (i == 0 ? 4.0 / 9 : (i <= 4 ? 1.0 / 9 : 1.0 / 36)) : (i == 0 ? 1.0 / 3 : 1.0 / 6);
  double Cxx[kMaxCoef] = {0}, Cxy[kMaxCoef] = {0}, Cyy[kMaxCoef] = {0};
  for (int k = 1; k <= in.bdeg; ++k)
    for (int l = 1; l <= in.bdeg; ++l) {
      const int m = k + l - 1;
      const double f = (double)(k * l) / m;
      Cxx[m] += f * in.bx[k] * in.bx[l];
      Cxy[m] += f * in.bx[k] * in.by[l];
      Cyy[m] += f * in.by[k] * in.by[l];
    }
  const double cs2 = in.cs2, c = in.p.c;
  int deg = 1;
  memset(in.e, 0, sizeof(in.e));
  for (int m = 0; m < kMaxCoef; ++m) {
    const double Bx = m <= DUGKS_MAX_DEG ? in.bx[m] : 0.0, By = m <= DUGKS_MAX_DEG ? in.by[m] : 0.0;
    const double Dxx = m <= DUGKS_MAX_DEG ? in.dxx[m] : 0.0, Dxy = m <= DUGKS_MAX_DEG ? in.dxy[m] : 0.0,
                 Dyy = m <= DUGKS_MAX_DEG ? in.dyy[m] : 0.0;
    const double Mxx = cs2 * Dxx + Cxx[m] - (m == 1 ? cs2 : 0.0);
    const double Mxy = cs2 * Dxy + Cxy[m];
    const double Myy = cs2 * Dyy + Cyy[m] - (m == 1 ? cs2 : 0.0);
    for (int i = 0; i < in.q; ++i) {
      const double cx = c * cxs[i], cy = c * cys[i];
      double v = (m == 1 ? 1.0 : 0.0) + (cx * Bx + cy * By) / cs2;
      if (in.q == 9)
        v += (Mxx * (cx * cx - cs2) + 2.0 * Mxy * cx * cy + Myy * (cy * cy - cs2)) / (2.0 * cs2 * cs2);
      in.e[i][m] = w[i] * v;
      if (in.e[i][m] != 0.0) deg = std::max(deg, m);
    }
  }
  in.ncoef = deg + 1;
  auto same = [&](int i, int j) { return memcmp(in.e[i], in.e[j], sizeof(in.e[i])) == 0; };
  in.xy_sym = same(1, 2) && same(3, 4) && (in.q == 5 || same(6, 8));
  // F_i + R_i = F w_i (1 + c_i.B'(phi) / cs2) (eq. 2.3, Remark 3) with
  // B'(phi) = sum_{k>=1} k b_k phi^(k-1); the kernels take c B' / cs2 per axis
  memset(in.bp, 0, sizeof(in.bp));
  for (int m = 0; m < kRhoCoef && m + 1 <= in.bdeg; ++m) {
    in.bp[0][m] = c * (m + 1) * in.bx[m + 1] / cs2;
    in.bp[1][m] = c * (m + 1) * in.by[m + 1] / cs2;
  }
}

static int template_ncoef(int ncoef) { return ncoef <= 2 ? 2 : (ncoef <= 4 ? 4 : 8); }

// ---------------------------------------------------------------- engine
struct Engine {
  uint32_t magic = 0;
  std::string err;
  int storage = DUGKS_F32;
  bool plain = false;
  std::vector<Instance> inst;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  size_t off_table = 0, off_items = 0, off_partial = 0, off_redout = 0, off_stepbase = 0;
  size_t total_bytes = 0;
  std::vector<InstDev> host_table;
  std::vector<WorkItem> items;
  Launch launch;
  int persistent_blocks = 0;
  // clock: every instance whose ready flag is set holds its state at `step`
  std::vector<char> ready;
  long long step = 0;
  bool need_measure = false;
  // graphs (kGraphSteps[0] and kGraphSteps[1] steps from a phase-0 step)
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
  bool use_graph = true;
  long long graph_steps = 0, eager_steps = 0;   // steps replayed / launched one by one
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  int ncoef_launch() const {
    int m = 2;
    for (auto& in : inst) m = std::max(m, template_ncoef(in.ncoef));
    return m;
  }
  bool any_source() const {
    for (auto& in : inst)
      if (in.src_n > 0) return true;
    return false;
  }
  // source kind of a launch: 0 none, 1 every source one term of power 0 (the
  // kernel holds one G a row), kSrcPow otherwise (several terms or powers of phi)
  int source_kind() const {
    int kind = 0;
    for (auto& in : inst) {
      if (in.src_n == 0) continue;
      kind = std::max(kind, (in.src_n == 1 && in.src_pow[0] == 0) ? 1 : kSrcPow);
    }
    return kind;
  }
  // Source terms of instance k (n == 0 removes the source).  Sources run in
  // binary64 / binary32 storage with the fused kernel.
  int set_source_terms(int k, int n, const double* g, const int* pw, const double* gam) {
    if (n < 0 || n > kMaxSrcTerms) return fail(DUGKS_E_ARG, "number of source terms out of range");
    if (n > 0) {
      if (!g || !pw || !gam) return fail(DUGKS_E_ARG, "source arrays are NULL");
      if (neq()) return fail(DUGKS_E_UNSUPPORTED, "sources need binary64 or binary32 storage");
      if (plain) return fail(DUGKS_E_UNSUPPORTED, "the plain kernel takes no source");
      for (int j = 0; j < n; ++j) {
        if (pw[j] < 0 || pw[j] > DUGKS_MAX_SRC_POW) return fail(DUGKS_E_ARG, "source power out of range");
        if (!std::isfinite(gam[j])) return fail(DUGKS_E_ARG, "source rate is not finite");
      }
      if (sizeof(double) * (double)inst[k].cells() * n >= 4294967296.0)
        return fail(DUGKS_E_ARG, "source arrays exceed 4 GiB");
    }
    Instance& in = inst[k];
    in.src_n = n > 0 ? n : 0;
    in.src_g = n > 0 ? g : nullptr;
    for (int j = 0; j < kMaxSrcTerms; ++j) {
      in.src_pow[j] = j < n ? pw[j] : 0;
      in.src_gam[j] = j < n ? gam[j] : 0.0;
    }
    drop_graph();
    if (launch.waves_per_block > 4 && !wide_blocks_ok()) {   // the source path runs 4-wave blocks
      const int rc = set_launch(launch.rows_per_wave, 4, launch.schedule, launch.xcd_remap);
      if (rc) return rc;
    }
    return bound() ? upload_tables() : DUGKS_OK;
  }
  // 8-wave blocks need the step kernels compiled for two waves per SIMD
  bool wide_blocks_ok() const { return storage != DUGKS_F64 && !any_source(); }
  int fail(int rc, const std::string& m) { err = m; return rc; }
  int hipfail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return DUGKS_E_HIP;
  }

  void layout() {
    size_t off = 0;
    off_table = off; off += align256(sizeof(InstDev) * inst.size());
    build_items();
    off_items = off; off += align256(sizeof(WorkItem) * std::max<size_t>(items.size(), 1) * 1);
    // room for a work list with the smallest rows-per-wave the tuner may pick
    off += align256(sizeof(WorkItem) * max_items_bound());
    off_partial = off; off += align256(sizeof(double) * 8 * reduce_partials());
    off_redout = off; off += align256(sizeof(double) * 8);
    off_stepbase = off; off += align256(sizeof(long long));
    for (auto& in : inst) {
      in.buf_bytes = in.buffer_bytes(storage);
      in.off_buf[0] = off; off += align256(in.buf_bytes);
      in.off_buf[1] = off; off += align256(in.buf_bytes);
      in.off_colgeo = off; off += align256(sizeof(double) * in.colgeo.size());
      in.off_rowgeo = off; off += align256(sizeof(double) * in.rowgeo.size());
      in.off_colgeo_f = off; off += align256(sizeof(float) * in.colgeo_f.size());
      in.off_rowgeo_f = off; off += align256(sizeof(float) * in.rowgeo_f.size());
      in.off_widths = off; off += align256(sizeof(double) * in.widths.size());
      in.off_slots = off; off += align256(sizeof(float) * 4);
      in.off_flags = off; off += align256(sizeof(unsigned));
    }
    total_bytes = off;
  }
  size_t max_items_bound() const {
    size_t n = 0;
    for (auto& in : inst) n += (size_t)((in.nx + kStripCols - 1) / kStripCols) * (size_t)in.ny;
    return n;
  }
  void build_items() {
    items.clear();
    const int H = launch.rows_per_wave;
    for (int k = 0; k < (int)inst.size(); ++k) {
      const Instance& in = inst[k];
      for (int y0 = 0; y0 < in.ny; y0 += H)
        for (int x0 = 0; x0 < in.nx; x0 += kStripCols)
          items.push_back(WorkItem{k, x0, y0, std::min(y0 + H, in.ny)});
    }
  }

  void fill_table() {
    host_table.assign(inst.size(), InstDev{});
    for (size_t k = 0; k < inst.size(); ++k) {
      Instance& in = inst[k];
      InstDev& d = host_table[k];
      memset(&d, 0, sizeof(d));
      d.buf[0] = ws + in.off_buf[0];
      d.buf[1] = ws + in.off_buf[1];
      d.colgeo = (const double*)(ws + in.off_colgeo);
      d.rowgeo = (const double*)(ws + in.off_rowgeo);
      d.colgeo_f = (const float*)(ws + in.off_colgeo_f);
      d.rowgeo_f = (const float*)(ws + in.off_rowgeo_f);
      d.ring = in.ring;
      d.slots = (float*)(ws + in.off_slots);
      d.flags = (unsigned*)(ws + in.off_flags);
      d.plane = (long long)in.ny * in.pitch;
      d.buf_bytes = (unsigned)in.buffer_bytes(storage);
      d.nx = in.nx; d.ny = in.ny; d.pitch = in.pitch; d.q = in.q;
      d.bcx = in.bcx; d.bcy = in.bcy;
      d.ring_len = 2 * (in.nx + in.ny) + 4;
      d.ring_steps = in.ring_steps;
      d.ncoef = in.ncoef;
      d.storage = storage;
      d.ra = in.a1 / in.b1;
      d.rb = in.a3 * in.b1 / in.b3;
      d.b1 = in.b1;
      d.inv_b1 = 1.0 / in.b1;
      d.kg = 4.0 / 3.0 * in.b1;
      d.a2 = in.a2;
      d.opra = 1.0 + d.ra;
      d.raf = (float)d.ra; d.rbf = (float)d.rb; d.b1f = (float)d.b1; d.inv_b1f = (float)d.inv_b1;
      d.kgf = (float)d.kg; d.a2f = (float)d.a2; d.oepraf = (float)d.opra; d.a1f = (float)in.a1;
      d.ra_of = (float)(d.ra / d.opra); d.b1_of = (float)(d.b1 * d.opra);
      d.rb_of = (float)(d.rb * d.opra); d.inv_b1_of = (float)(1.0 / (d.b1 * d.opra));
      for (int i = 0; i < in.q; ++i)
        for (int m = 0; m < kMaxCoef; ++m) {
          d.e[i][m] = in.e[i][m];
          d.ef[i][m] = (float)d.e[i][m];
        }
      d.src_g = in.src_g;
      d.src_n = in.src_n;
      d.src_implicit = in.src_implicit() ? 1 : 0;
      d.src_plane = (unsigned)(sizeof(double) * in.cells());
      d.src_bytes = (unsigned)(sizeof(double) * in.cells() * in.src_n);
      for (int j = 0; j < kMaxSrcTerms; ++j) {
        d.src_pow[j] = in.src_pow[j];
        d.src_gam[j] = in.src_gam[j];
      }
      d.dt = in.dt;
      d.lambda = in.lambda;
      d.half_dt = 0.5 * in.dt;
      d.half_h = 0.5 * in.h;
      d.lambdaf = (float)d.lambda; d.half_dtf = (float)d.half_dt; d.half_hf = (float)d.half_h;
      for (int a = 0; a < 2; ++a)
        for (int m = 0; m < kRhoCoef; ++m) {
          d.bp[a][m] = in.bp[a][m];
          d.bpf[a][m] = (float)in.bp[a][m];
        }
    }
  }

  int upload_tables() {
    fill_table();
    hipError_t e = hipMemcpyAsync(ws + off_table, host_table.data(), sizeof(InstDev) * inst.size(),
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hipfail(e, "upload instance table");
    e = hipMemcpyAsync(ws + off_items, items.data(), sizeof(WorkItem) * items.size(),
                       hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hipfail(e, "upload work list");
    for (auto& in : inst) {
      struct { size_t off; const void* src; size_t n; } cp[] = {
          {in.off_colgeo, in.colgeo.data(), sizeof(double) * in.colgeo.size()},
          {in.off_rowgeo, in.rowgeo.data(), sizeof(double) * in.rowgeo.size()},
          {in.off_colgeo_f, in.colgeo_f.data(), sizeof(float) * in.colgeo_f.size()},
          {in.off_rowgeo_f, in.rowgeo_f.data(), sizeof(float) * in.rowgeo_f.size()},
          {in.off_widths, in.widths.data(), sizeof(double) * in.widths.size()}};
      for (auto& c : cp) {
        e = hipMemcpyAsync(ws + c.off, c.src, c.n, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hipfail(e, "upload mesh tables");
      }
    }
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "synchronise after upload");
    drop_graph();
    return DUGKS_OK;
  }

  int bind(void* w, size_t bytes, void* s) {
    if (!w) return fail(DUGKS_E_ARG, "workspace is NULL");
    if (((uintptr_t)w) & 255) return fail(DUGKS_E_ARG, "workspace must be 256-byte aligned");
    layout();
    if (bytes < total_bytes) return fail(DUGKS_E_NOMEM, "workspace too small");
    ws = (char*)w;
    ws_bytes = bytes;
    stream = (hipStream_t)s;
    if (!cap_stream) {
      hipError_t e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hipfail(e, "create capture stream");
    }
    if (!ev0) {
      hipError_t e = hipEventCreate(&ev0);
      if (e == hipSuccess) e = hipEventCreate(&ev1);
      if (e != hipSuccess) return hipfail(e, "create events");
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      persistent_blocks = cus * (16 / launch.waves_per_block);
    else
      persistent_blocks = 256 * 4;
    ready.assign(inst.size(), 0);
    step = 0;
    int rc = upload_tables();
    if (rc) return rc;
    for (auto& in : inst) {
      rc = launch_fill_u32((unsigned*)(ws + in.off_flags), 0u, 1, stream);
      if (rc == 0) rc = launch_fill_u32((unsigned*)(ws + in.off_slots), 0u, 4, stream);
      if (rc) return fail(DUGKS_E_HIP, "clear flags");
    }
    return DUGKS_OK;
  }

  bool bound() const { return ws != nullptr; }
  int state_error_for(int k) {
    if (!bound()) return fail(DUGKS_E_STATE, "not bound");
    if (inst.size() == 1) return fail(DUGKS_E_STATE, "no state (set_phi / set_f)");
    return fail(DUGKS_E_STATE, "instance " + std::to_string(k) + " holds no state at the batch clock");
  }

  const InstDev* dev_table() const { return (const InstDev*)(ws + off_table); }
  const InstDev* dev_inst(int k) const { return dev_table() + k; }

  StepArgs step_args(long long n) const {
    StepArgs a{};
    a.insts = dev_table();
    a.items = (const WorkItem*)(ws + off_items);
    a.nitems = (int)items.size();
    a.parity = (int)(n & 1);
    a.step = n;
    a.q = inst[0].q;
    a.storage = storage;
    a.ncoef = ncoef_launch();
    a.persistent_blocks = persistent_blocks;
    a.src = source_kind();
    a.sym = 1;
    for (auto& in : inst) a.sym &= in.xy_sym ? 1 : 0;
    return a;
  }

  bool neq() const { return storage == DUGKS_F16NEQ || storage == DUGKS_BF16NEQ; }

  bool all_ready() const {
    if (ready.size() != inst.size()) return false;
    for (char r : ready)
      if (!r) return false;
    return true;
  }
  bool is_ready(int k) const { return k >= 0 && k < (int)ready.size() && ready[k]; }
  int first_unready() const {
    for (size_t k = 0; k < inst.size(); ++k)
      if (k >= ready.size() || !ready[k]) return (int)k;
    return -1;
  }
  int state_error() {
    const int k = first_unready();
    if (inst.size() == 1) return fail(DUGKS_E_STATE, "state not initialised (set_phi / set_f)");
    return fail(DUGKS_E_STATE, "instance " + std::to_string(k) +
                                   " holds no state at the batch clock: after a per-instance "
                                   "set_phi / set_f on a stepped batch, every instance must be set again");
  }
  // A per-instance initialisation puts instance k at step 0.  If the engine has
  // stepped, the others hold states of another step (and the other buffer
  // parity and 16-bit slot phase): they are marked stale until set again.
  void restart_clock_for(int k) {
    if (step != 0 || ready.size() != inst.size()) ready.assign(inst.size(), 0);
    step = 0;
    ready[k] = 1;
  }
  // Dirichlet data covers steps [step, step + n)
  bool rings_cover(long long n) const {
    for (auto& in : inst)
      if ((in.bcx == DUGKS_BC_DIRICHLET || in.bcy == DUGKS_BC_DIRICHLET) &&
          (in.ring == nullptr || step + n > in.ring_steps))
        return false;
    return true;
  }

  // Enqueue one step with input index n on stream s (captured: index n after
  // the base written before each replay).
  int enqueue_step(long long n, hipStream_t s, bool measure, bool captured = false) {
    StepArgs a = step_args(n);
    if (captured) a.step_base = (const long long*)(ws + off_stepbase);
    int rc;
    if (plain) {
      rc = launch_step_plain(a, inst[0].nx, inst[0].ny, s);
    } else {
      if (neq()) {
        rc = launch_clear_slot(dev_table(), (int)inst.size(), n, measure ? 3 : 0, s);
        if (rc) return fail(DUGKS_E_HIP, "clear slot launch failed");
      }
      rc = launch_step_fused(a, launch, s, measure ? 1 : 0);
    }
    if (rc) return fail(DUGKS_E_HIP, std::string("step launch failed: ") + hipGetErrorString(hipGetLastError()));
    return DUGKS_OK;
  }

  void drop_graph() {
    for (int w = 0; w < 2; ++w) {
      if (graph_exec[w]) { (void)hipGraphExecDestroy(graph_exec[w]); graph_exec[w] = nullptr; }
      if (graph[w]) { (void)hipGraphDestroy(graph[w]); graph[w] = nullptr; }
    }
  }

  // Capture kGraphSteps[w] steps starting at step index 0; replayed at any step
  // divisible by 4 (same buffer parity and 16-bit slot phase).
  int build_graph(int w) {
    hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hipfail(e, "begin capture");
    int rc = DUGKS_OK;
    for (int k = 0; k < kGraphSteps[w] && rc == DUGKS_OK; ++k) rc = enqueue_step(k, cap_stream, false, true);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap_stream, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return hipfail(e, "end capture");
    graph[w] = g;
    e = hipGraphInstantiate(&graph_exec[w], graph[w], nullptr, nullptr, 0);
    if (e != hipSuccess) { drop_graph(); return hipfail(e, "instantiate graph"); }
    return DUGKS_OK;
  }

  int do_steps(int nsteps) {
    if (nsteps < 0) return fail(DUGKS_E_ARG, "nsteps < 0");
    if (!bound()) return fail(DUGKS_E_STATE, "not bound");
    if (!all_ready()) return state_error();
    if (!rings_cover(nsteps)) return fail(DUGKS_E_STATE, "Dirichlet data does not cover the requested steps");
    int remaining = nsteps;
    // captured launches read their step index (the time of Dirichlet data and
    // sources) as an offset from a base written before each replay
    const bool graphable = use_graph && !plain;
    while (remaining > 0) {
      if (need_measure) {
        int rc = enqueue_step(step, stream, true);
        if (rc) return rc;
        need_measure = false;
      }
      const int w = remaining >= kGraphSteps[0] ? 0 : 1;
      if (graphable && remaining >= kGraphSteps[1] && (step & 3) == 0) {
        if (!graph_exec[w]) {
          int rc = build_graph(w);
          if (rc) return rc;
        }
        if (launch_set_i64((long long*)(ws + off_stepbase), step, stream))
          return fail(DUGKS_E_HIP, "step base launch failed");
        hipError_t e = hipGraphLaunch(graph_exec[w], stream);
        if (e != hipSuccess) return hipfail(e, "graph launch");
        step += kGraphSteps[w];
        remaining -= kGraphSteps[w];
        graph_steps += kGraphSteps[w];
      } else {
        int rc = enqueue_step(step, stream, false);
        if (rc) return rc;
        step += 1;
        remaining -= 1;
        eager_steps += 1;
      }
    }
    return DUGKS_OK;
  }

  int set_launch(int rows, int wpb, int sched, int xcd) {
    if (rows < 1 || rows > 4096) return fail(DUGKS_E_ARG, "rows_per_wave out of range");
    if (wpb != 1 && wpb != 2 && wpb != 4 && !(wpb == 8 && wide_blocks_ok()))
      return fail(DUGKS_E_ARG, "waves_per_block must be 1, 2 or 4 (8: binary32 or 16-bit storage without a source)");
    if (sched != DUGKS_SCHED_GRID && sched != DUGKS_SCHED_PERSISTENT) return fail(DUGKS_E_ARG, "bad schedule");
    launch.rows_per_wave = rows;
    launch.waves_per_block = wpb;
    launch.schedule = sched;
    launch.xcd_remap = xcd ? 1 : 0;
    if (bound()) {
      int dev = 0, cus = 256;
      if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      persistent_blocks = cus * (16 / wpb);
      build_items();
      if (items.size() > max_items_bound() + 1) return fail(DUGKS_E_ARG, "work list too long");
      hipError_t e = hipMemcpyAsync(ws + off_items, items.data(), sizeof(WorkItem) * items.size(),
                                    hipMemcpyHostToDevice, stream);
      if (e != hipSuccess) return hipfail(e, "upload work list");
      e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return hipfail(e, "synchronise");
    }
    drop_graph();
    return DUGKS_OK;
  }

  int set_phi(int k, const double* phi, int on_device) {
    if (!bound()) return fail(DUGKS_E_STATE, "not bound");
    if (!phi) return fail(DUGKS_E_ARG, "phi is NULL");
    Instance& in = inst[k];
    const size_t n = (size_t)in.cells() * sizeof(double);
    double* src = (double*)phi;
    double* tmp = nullptr;
    hipError_t e;
    if (!on_device) {
      e = hipMalloc(&tmp, n);
      if (e != hipSuccess) return hipfail(e, "temporary for host phi");
      e = hipMemcpyAsync(tmp, phi, n, hipMemcpyHostToDevice, stream);
      if (e != hipSuccess) { (void)hipFree(tmp); return hipfail(e, "copy phi"); }
      src = tmp;
    }
    // the clock of the whole engine restarts at step 0 (parity 0)
    int rc = launch_init_eq(dev_inst(k), host_table[k], src, 0, stream);
    if (rc == 0 && neq()) {
      // slot 2 scales the initial state (g = 0, any scale), slot 3 is measured
      const float one = 1.0f;
      unsigned one_bits;
      memcpy(&one_bits, &one, sizeof(one_bits));
      rc = launch_fill_u32((unsigned*)(ws + in.off_slots), 0u, 4, stream);
      if (rc == 0) rc = launch_fill_u32((unsigned*)(ws + in.off_slots) + 2, one_bits, 1, stream);
    }
    if (rc == 0) rc = launch_fill_u32((unsigned*)(ws + in.off_flags), 0u, 1, stream);
    e = hipStreamSynchronize(stream);
    if (tmp) (void)hipFree(tmp);
    if (rc) return fail(DUGKS_E_HIP, "init launch failed");
    if (e != hipSuccess) return hipfail(e, "set_phi");
    restart_clock_for(k);
    need_measure = neq();
    return DUGKS_OK;
  }

  int set_f(int k, const double* f, int on_device) {
    if (!bound()) return fail(DUGKS_E_STATE, "not bound");
    if (!f) return fail(DUGKS_E_ARG, "f is NULL");
    Instance& in = inst[k];
    const size_t n = (size_t)in.cells() * in.q * sizeof(double);
    double* src = (double*)f;
    double* tmp = nullptr;
    hipError_t e;
    if (!on_device) {
      e = hipMalloc(&tmp, n);
      if (e != hipSuccess) return hipfail(e, "temporary for host f");
      e = hipMemcpyAsync(tmp, f, n, hipMemcpyHostToDevice, stream);
      if (e != hipSuccess) { (void)hipFree(tmp); return hipfail(e, "copy f"); }
      src = tmp;
    }
    int rc = launch_fill_u32((unsigned*)(ws + in.off_slots), 0u, 4, stream);
    if (rc == 0 && neq()) rc = launch_set_f_pass(dev_inst(k), host_table[k], src, 0, 0, 2, stream);
    if (rc == 0) rc = launch_set_f_pass(dev_inst(k), host_table[k], src, 0, 1, 2, stream);
    if (rc == 0) rc = launch_fill_u32((unsigned*)(ws + in.off_flags), 0u, 1, stream);
    e = hipStreamSynchronize(stream);
    if (tmp) (void)hipFree(tmp);
    if (rc) return fail(DUGKS_E_HIP, "encode launch failed");
    if (e != hipSuccess) return hipfail(e, "set_f");
    restart_clock_for(k);
    need_measure = neq();
    return DUGKS_OK;
  }

  template <class F>
  int read_out(size_t n, double* out, int on_device, F launchf) {
    double* dst = out;
    double* tmp = nullptr;
    hipError_t e;
    if (!on_device) {
      e = hipMalloc(&tmp, n);
      if (e != hipSuccess) return hipfail(e, "temporary for host output");
      dst = tmp;
    }
    int rc = launchf(dst);
    if (rc) { if (tmp) (void)hipFree(tmp); return fail(DUGKS_E_HIP, "read launch failed"); }
    if (!on_device) {
      e = hipMemcpyAsync(out, tmp, n, hipMemcpyDeviceToHost, stream);
      if (e != hipSuccess) { (void)hipFree(tmp); return hipfail(e, "copy out"); }
    }
    e = hipStreamSynchronize(stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return hipfail(e, "read");
    return DUGKS_OK;
  }

  int get_phi(int k, double* out, int on_device) {
    if (!bound() || !is_ready(k)) return state_error_for(k);
    if (!out) return fail(DUGKS_E_ARG, "out is NULL");
    const Instance& in = inst[k];
    return read_out((size_t)in.cells() * sizeof(double), out, on_device, [&](double* dst) {
      return launch_get_phi(dev_inst(k), host_table[k], dst, (int)(step & 1), step, stream);
    });
  }

  int get_f(int k, double* out, int on_device) {
    if (!bound() || !is_ready(k)) return state_error_for(k);
    if (!out) return fail(DUGKS_E_ARG, "out is NULL");
    const Instance& in = inst[k];
    return read_out((size_t)in.cells() * in.q * sizeof(double), out, on_device, [&](double* dst) {
      return launch_get_f(dev_inst(k), host_table[k], dst, (int)(step & 1), step, stream);
    });
  }

  int reduce(int k, const double* ref, double out[8], unsigned* flags, float slots[4]) {
    if (!bound() || !is_ready(k)) return state_error_for(k);
    Instance& in = inst[k];
    int rc = launch_reduce_widths(dev_inst(k), host_table[k], ref, (int)(step & 1), step,
                                  (const double*)(ws + in.off_widths), (double*)(ws + off_partial),
                                  (double*)(ws + off_redout), stream);
    if (rc) return fail(DUGKS_E_HIP, "reduce launch failed");
    hipError_t e = hipMemcpyAsync(out, ws + off_redout, 8 * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess && flags)
      e = hipMemcpyAsync(flags, ws + in.off_flags, sizeof(unsigned), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess && slots)
      e = hipMemcpyAsync(slots, ws + in.off_slots, 4 * sizeof(float), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "reduce");
    return DUGKS_OK;
  }

  int time_steps(int nsteps, float* ms) {
    if (!ms) return fail(DUGKS_E_ARG, "ms is NULL");
    hipError_t e = hipEventRecord(ev0, stream);
    if (e != hipSuccess) return hipfail(e, "event record");
    int rc = do_steps(nsteps);
    if (rc) return rc;
    e = hipEventRecord(ev1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, ev0, ev1);
    if (e != hipSuccess) return hipfail(e, "event timing");
    return DUGKS_OK;
  }

  // Time candidate launch configurations on the inactive buffer only: the
  // step writes buffer (step+1)&1 and never swaps, so the state is kept.
  int autotune(int trials) {
    if (!bound()) return fail(DUGKS_E_STATE, "not bound");
    if (!all_ready()) return state_error();
    if (trials < 1) trials = 1;
    if (plain) return DUGKS_OK;
    // every trial step reads the Dirichlet data of the current step
    if (!rings_cover(1)) return fail(DUGKS_E_STATE, "Dirichlet data does not cover the current step");
    // keep the 16-bit slots: the trial steps accumulate into them
    std::vector<std::vector<float>> saved(inst.size(), std::vector<float>(4));
    for (size_t k = 0; k < inst.size(); ++k) {
      hipError_t e = hipMemcpyAsync(saved[k].data(), ws + inst[k].off_slots, 4 * sizeof(float),
                                    hipMemcpyDeviceToHost, stream);
      if (e != hipSuccess) return hipfail(e, "save slots");
    }
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "synchronise");
    const Launch keep = launch;
    Launch best = keep;
    float best_ms = 1e30f;
    const int rows_c[] = {2, 4, 8, 16, 32, 64, 128};   // short items: more waves on small grids
    const int wpb_c[] = {1, 2, 4, 8};
    for (int sched = 0; sched < 2; ++sched)
      for (int rows : rows_c)
        for (int wpb : wpb_c) {
          if (wpb == 8 && !wide_blocks_ok()) continue;
          if (set_launch(rows, wpb, sched, 1)) return DUGKS_E_ARG;
          // warm-up
          for (int t = 0; t < 2; ++t)
            if (enqueue_step(step, stream, false)) return DUGKS_E_HIP;
          e = hipEventRecord(ev0, stream);
          for (int t = 0; t < trials && e == hipSuccess; ++t)
            if (enqueue_step(step, stream, false)) return DUGKS_E_HIP;
          if (e == hipSuccess) e = hipEventRecord(ev1, stream);
          if (e == hipSuccess) e = hipEventSynchronize(ev1);
          float ms = 0;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
          if (e != hipSuccess) return hipfail(e, "autotune timing");
          if (ms < best_ms) { best_ms = ms; best = launch; }
        }
    int rc = set_launch(best.rows_per_wave, best.waves_per_block, best.schedule, best.xcd_remap);
    if (rc) return rc;
    for (size_t k = 0; k < inst.size(); ++k) {
      e = hipMemcpyAsync(ws + inst[k].off_slots, saved[k].data(), 4 * sizeof(float),
                         hipMemcpyHostToDevice, stream);
      if (e != hipSuccess) return hipfail(e, "restore slots");
      rc = launch_fill_u32((unsigned*)(ws + inst[k].off_flags), 0u, 1, stream);
      if (rc) return fail(DUGKS_E_HIP, "clear flags");
    }
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "synchronise");
    return DUGKS_OK;
  }

  void info(int k, dugks_info* o) const {
    const Instance& in = inst[k];
    memset(o, 0, sizeof(*o));
    o->dt = in.dt; o->h = in.h; o->lambda = in.lambda; o->cs2 = in.cs2;
    o->a1 = in.a1; o->b1 = in.b1; o->a2 = in.a2; o->b2 = in.b2; o->a3 = in.a3; o->b3 = in.b3;
    o->nx = in.nx; o->ny = in.ny; o->q = in.q; o->storage = storage; o->pitch = in.pitch;
    o->eq_degree = in.ncoef - 1;
    o->rows_per_wave = launch.rows_per_wave;
    o->waves_per_block = launch.waves_per_block;
    o->schedule = launch.schedule;
    o->xcd_remap = launch.xcd_remap;
    o->work_items = (long long)items.size();
    o->state_bytes = in.buffer_bytes(storage);
    o->graph_steps = graph_steps;
    o->eager_steps = eager_steps;
    o->xy_symmetric = step_args(0).sym;
  }

  ~Engine() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

static int set_B_impl(Instance& in, int deg, const double* bx, const double* by, std::string& err) {
  if (deg < 0 || deg > DUGKS_MAX_DEG || !bx || !by) { err = "B: degree out of range or NULL"; return DUGKS_E_ARG; }
  for (int k = 0; k <= deg; ++k)
    if (!std::isfinite(bx[k]) || !std::isfinite(by[k])) { err = "B: non-finite coefficient"; return DUGKS_E_ARG; }
  memset(in.bx, 0, sizeof(in.bx)); memset(in.by, 0, sizeof(in.by));
  for (int k = 0; k <= deg; ++k) { in.bx[k] = bx[k]; in.by[k] = by[k]; }
  in.bdeg = deg;
  equilibrium_polys(in);
  return DUGKS_OK;
}

static int set_D_impl(Instance& in, int deg, const double* dxx, const double* dxy, const double* dyy,
                      std::string& err) {
  if (deg < 0 || deg > DUGKS_MAX_DEG || !dxx || !dxy || !dyy) { err = "D: degree out of range or NULL"; return DUGKS_E_ARG; }
  for (int k = 0; k <= deg; ++k)
    if (!std::isfinite(dxx[k]) || !std::isfinite(dxy[k]) || !std::isfinite(dyy[k])) {
      err = "D: non-finite coefficient";
      return DUGKS_E_ARG;
    }
  if (in.q == 5) {
    for (int k = 0; k <= deg; ++k) {
      const double want = k == 1 ? 1.0 : 0.0;
      if (dxx[k] != want || dyy[k] != want || dxy[k] != 0.0) {
        err = "D2Q5 supports only D = phi I (linear equilibrium of Remark 3)";
        return DUGKS_E_UNSUPPORTED;
      }
    }
  }
  memset(in.dxx, 0, sizeof(in.dxx)); memset(in.dxy, 0, sizeof(in.dxy)); memset(in.dyy, 0, sizeof(in.dyy));
  for (int k = 0; k <= deg; ++k) { in.dxx[k] = dxx[k]; in.dxy[k] = dxy[k]; in.dyy[k] = dyy[k]; }
  in.ddeg = deg;
  equilibrium_polys(in);
  return DUGKS_OK;
}

// ------------------------------------------------------------ checkpoint
struct CkptHeader {
  char magic[8];
  uint32_t abi, header_bytes;
  int32_t nx, ny, q, storage;
  int64_t step;
  double t, dt;
  float slots[4];
  uint64_t params_hash;
  uint64_t payload_bytes;
  uint64_t payload_checksum;
};

static uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
  return h;
}

static uint64_t params_hash(const Instance& in, int storage) {
  uint64_t h = fnv1a(&in.nx, sizeof(int));
  h = fnv1a(&in.ny, sizeof(int), h);
  h = fnv1a(&in.q, sizeof(int), h);
  h = fnv1a(&storage, sizeof(int), h);
  h = fnv1a(in.p.bc, sizeof(in.p.bc), h);
  h = fnv1a(&in.p.c, sizeof(double), h);
  h = fnv1a(&in.p.cfl, sizeof(double), h);
  h = fnv1a(&in.p.alpha, sizeof(double), h);
  h = fnv1a(in.xf.data(), sizeof(double) * in.xf.size(), h);
  h = fnv1a(in.yf.data(), sizeof(double) * in.yf.size(), h);
  h = fnv1a(in.e, sizeof(in.e), h);
  return h;
}

}  // namespace dugks

using dugks::Engine;

struct dugks_ctx : Engine {};
struct dugks_batch : Engine {};

static Engine* as_engine(const void* h) {
  if (!h) return nullptr;
  const Engine* e = (const Engine*)h;
  if (e->magic != dugks::kMagicCtx && e->magic != dugks::kMagicBatch) return nullptr;
  return (Engine*)e;
}

#define GUARD_CTX(ctx)                                                         \
  if (!(ctx) || ((Engine*)(ctx))->magic != dugks::kMagicCtx) return DUGKS_E_ARG
#define GUARD_BATCH(b)                                                         \
  if (!(b) || ((Engine*)(b))->magic != dugks::kMagicBatch) return DUGKS_E_ARG

extern "C" {

int dugks_create(dugks_ctx** out, int nx, int ny, const double* xf, const double* yf, int q,
                 const dugks_params* p) {
  if (!out) return DUGKS_E_ARG;
  *out = nullptr;
  dugks_ctx* c = new (std::nothrow) dugks_ctx();
  if (!c) return DUGKS_E_NOMEM;
  c->magic = dugks::kMagicCtx;
  c->inst.resize(1);
  int rc = dugks::init_instance(c->inst[0], nx, ny, xf, yf, q, p, c->err);
  if (rc) {
    // keep the handle so that the caller can read the message
    *out = c;
    return rc;
  }
  dugks::equilibrium_polys(c->inst[0]);
  c->storage = p->storage;
  c->plain = p->kernel == DUGKS_KERNEL_PLAIN;
  if (c->storage == DUGKS_F64) { c->launch.rows_per_wave = 32; c->launch.waves_per_block = 1; }
  *out = c;
  return DUGKS_OK;
}

size_t dugks_workspace_bytes(const dugks_ctx* ctx) {
  if (!ctx || ctx->magic != dugks::kMagicCtx || ctx->inst.empty() || ctx->inst[0].nx == 0) return 0;
  Engine tmp_view;  // layout without touching the handle
  tmp_view.storage = ctx->storage;
  tmp_view.inst = ctx->inst;
  tmp_view.launch = ctx->launch;
  tmp_view.layout();
  return tmp_view.total_bytes;
}

int dugks_bind(dugks_ctx* ctx, void* ws, size_t bytes, void* stream) {
  GUARD_CTX(ctx);
  if (ctx->inst[0].nx == 0) return ctx->fail(DUGKS_E_STATE, "instance was not created");
  return ctx->bind(ws, bytes, stream);
}

int dugks_set_B(dugks_ctx* ctx, int deg, const double* bx, const double* by) {
  GUARD_CTX(ctx);
  int rc = dugks::set_B_impl(ctx->inst[0], deg, bx, by, ctx->err);
  if (rc == 0 && ctx->bound()) rc = ctx->upload_tables();
  return rc;
}

int dugks_set_D(dugks_ctx* ctx, int deg, const double* dxx, const double* dxy, const double* dyy) {
  GUARD_CTX(ctx);
  int rc = dugks::set_D_impl(ctx->inst[0], deg, dxx, dxy, dyy, ctx->err);
  if (rc == 0 && ctx->bound()) rc = ctx->upload_tables();
  return rc;
}

int dugks_set_source(dugks_ctx* ctx, const double* g_dev, double gamma) {
  GUARD_CTX(ctx);
  const int zero = 0;
  return ctx->set_source_terms(0, g_dev ? 1 : 0, g_dev, &zero, &gamma);
}

int dugks_set_source_terms(dugks_ctx* ctx, int nterms, const double* g_dev, const int* powers,
                           const double* gammas) {
  GUARD_CTX(ctx);
  return ctx->set_source_terms(0, nterms, g_dev, powers, gammas);
}

int dugks_set_dirichlet(dugks_ctx* ctx, const double* ring_dev, int nsteps) {
  GUARD_CTX(ctx);
  if (nsteps < 0 || (nsteps > 0 && !ring_dev)) return ctx->fail(DUGKS_E_ARG, "bad Dirichlet data");
  ctx->inst[0].ring = nsteps > 0 ? ring_dev : nullptr;
  ctx->inst[0].ring_steps = nsteps;
  if (ctx->bound()) return ctx->upload_tables();
  return DUGKS_OK;
}

int dugks_set_phi(dugks_ctx* ctx, const double* phi, int on_device) {
  GUARD_CTX(ctx);
  return ctx->set_phi(0, phi, on_device);
}

int dugks_set_f(dugks_ctx* ctx, const double* f, int on_device) {
  GUARD_CTX(ctx);
  return ctx->set_f(0, f, on_device);
}

int dugks_step(dugks_ctx* ctx, int nsteps) {
  GUARD_CTX(ctx);
  return ctx->do_steps(nsteps);
}

int dugks_get_phi(dugks_ctx* ctx, double* out, int on_device) {
  GUARD_CTX(ctx);
  return ctx->get_phi(0, out, on_device);
}

int dugks_get_f(dugks_ctx* ctx, double* out, int on_device) {
  GUARD_CTX(ctx);
  return ctx->get_f(0, out, on_device);
}

int dugks_get_diag(dugks_ctx* ctx, dugks_diag* out) {
  GUARD_CTX(ctx);
  if (!out) return ctx->fail(DUGKS_E_ARG, "out is NULL");
  double r[8];
  unsigned flags = 0;
  float slots[4] = {0, 0, 0, 0};
  int rc = ctx->reduce(0, nullptr, r, &flags, slots);
  if (rc) return rc;
  memset(out, 0, sizeof(*out));
  out->step = ctx->step;
  out->dt = ctx->inst[0].dt;
  out->t = ctx->step * ctx->inst[0].dt;
  out->mass = r[0];
  out->flags = (int)flags;
  if (r[5] > 0) out->flags |= DUGKS_FLAG_NONFINITE;
  if (ctx->neq()) {
    out->max_neq = slots[(ctx->step + 2) & 3];
    out->scale = dugks::neq_scale_host(ctx->storage, slots[(ctx->step + 2) & 3]);
  } else {
    out->scale = 1.0;
  }
  if (out->flags) return ctx->fail(DUGKS_E_UNSTABLE, "non-finite value or 16-bit overflow on the device");
  return DUGKS_OK;
}

int dugks_error_norms(dugks_ctx* ctx, const double* ref_dev, double* rel_l2, double* gre) {
  GUARD_CTX(ctx);
  if (!ref_dev || !rel_l2 || !gre) return ctx->fail(DUGKS_E_ARG, "NULL argument");
  double r[8];
  int rc = ctx->reduce(0, ref_dev, r, nullptr, nullptr);
  if (rc) return rc;
  if (r[5] > 0) {   // non-finite cells are left out of the sums: no error to report
    *gre = *rel_l2 = NAN;
    return ctx->fail(DUGKS_E_UNSTABLE, "non-finite phi on the device");
  }
  *gre = r[2] > 0 ? r[1] / r[2] : (r[1] > 0 ? INFINITY : 0.0);
  *rel_l2 = r[4] > 0 ? sqrt(r[3] / r[4]) : (r[3] > 0 ? INFINITY : 0.0);
  return DUGKS_OK;
}

int dugks_error_norms_noalloc(dugks_ctx* ctx, const double* ref_dev, double* out_dev) {
  GUARD_CTX(ctx);
  if (!ref_dev || !out_dev) return ctx->fail(DUGKS_E_ARG, "NULL argument");
  if (!ctx->bound() || !ctx->all_ready()) return ctx->fail(DUGKS_E_STATE, "no state");
  const dugks::Instance& in = ctx->inst[0];
  const int rc = dugks::launch_norms_noalloc(ctx->dev_inst(0), ctx->host_table[0], ref_dev,
                                             (int)(ctx->step & 1), ctx->step,
                                             (const double*)(ctx->ws + in.off_widths), out_dev,
                                             ctx->stream);
  if (rc == -2) return ctx->fail(DUGKS_E_HIP, "hipGetSymbolAddress of the reduction scratch failed");
  if (rc) return ctx->fail(DUGKS_E_HIP, "norm launch failed");
  return DUGKS_OK;
}

int dugks_checkpoint(dugks_ctx* ctx, void* host_buf, size_t* len) {
  GUARD_CTX(ctx);
  if (!len) return ctx->fail(DUGKS_E_ARG, "len is NULL");
  const dugks::Instance& in = ctx->inst[0];
  const size_t payload = in.buffer_bytes(ctx->storage);
  const size_t need = sizeof(dugks::CkptHeader) + payload;
  if (!host_buf) { *len = need; return DUGKS_OK; }
  if (*len < need) return ctx->fail(DUGKS_E_ARG, "checkpoint buffer too small");
  if (!ctx->bound() || !ctx->all_ready()) return ctx->fail(DUGKS_E_STATE, "no state");
  dugks::CkptHeader hd;
  memset(&hd, 0, sizeof(hd));
  memcpy(hd.magic, "DUGKSCK2", 8);
  hd.abi = DUGKS_ABI_VERSION;
  hd.header_bytes = sizeof(hd);
  hd.nx = in.nx; hd.ny = in.ny; hd.q = in.q; hd.storage = ctx->storage;
  hd.step = ctx->step;
  hd.dt = in.dt;
  hd.t = ctx->step * in.dt;
  hd.params_hash = dugks::params_hash(in, ctx->storage);
  hd.payload_bytes = payload;
  char* dst = (char*)host_buf + sizeof(hd);
  hipError_t e = hipMemcpyAsync(dst, ctx->ws + in.off_buf[ctx->step & 1], payload,
                                hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hd.slots, ctx->ws + in.off_slots, sizeof(hd.slots), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return ctx->hipfail(e, "checkpoint copy");
  hd.payload_checksum = dugks::fnv1a(dst, payload);
  memcpy(host_buf, &hd, sizeof(hd));
  *len = need;
  return DUGKS_OK;
}

int dugks_restore(dugks_ctx* ctx, const void* host_buf, size_t len) {
  GUARD_CTX(ctx);
  if (!host_buf || len < sizeof(dugks::CkptHeader)) return ctx->fail(DUGKS_E_FORMAT, "checkpoint too short");
  if (!ctx->bound()) return ctx->fail(DUGKS_E_STATE, "not bound");
  dugks::CkptHeader hd;
  memcpy(&hd, host_buf, sizeof(hd));
  const dugks::Instance& in = ctx->inst[0];
  if (memcmp(hd.magic, "DUGKSCK2", 8) != 0) return ctx->fail(DUGKS_E_FORMAT, "bad magic");
  if (hd.abi != DUGKS_ABI_VERSION || hd.header_bytes != sizeof(hd))
    return ctx->fail(DUGKS_E_FORMAT, "ABI version or header size mismatch");
  if (hd.nx != in.nx || hd.ny != in.ny || hd.q != in.q || hd.storage != ctx->storage)
    return ctx->fail(DUGKS_E_FORMAT, "size or storage mismatch");
  if (hd.params_hash != dugks::params_hash(in, ctx->storage))
    return ctx->fail(DUGKS_E_FORMAT, "mesh, parameters or coefficients differ");
  const size_t payload = in.buffer_bytes(ctx->storage);
  if (hd.payload_bytes != payload || len < sizeof(hd) + payload)
    return ctx->fail(DUGKS_E_FORMAT, "payload size mismatch");
  const char* src = (const char*)host_buf + sizeof(hd);
  if (dugks::fnv1a(src, payload) != hd.payload_checksum) return ctx->fail(DUGKS_E_FORMAT, "checksum mismatch");
  if (hd.step < 0) return ctx->fail(DUGKS_E_FORMAT, "negative step");
  hipError_t e = hipMemcpyAsync(ctx->ws + in.off_buf[hd.step & 1], src, payload, hipMemcpyHostToDevice,
                                ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->ws + in.off_slots, hd.slots, sizeof(hd.slots), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    if (dugks::launch_fill_u32((unsigned*)(ctx->ws + in.off_flags), 0u, 1, ctx->stream)) e = hipErrorUnknown;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return ctx->hipfail(e, "restore copy");
  ctx->step = hd.step;
  ctx->ready.assign(1, 1);
  ctx->need_measure = false;
  return DUGKS_OK;
}

int dugks_set_launch(dugks_ctx* ctx, int rows, int wpb, int sched, int xcd) {
  GUARD_CTX(ctx);
  return ctx->set_launch(rows, wpb, sched, xcd);
}

int dugks_autotune(dugks_ctx* ctx, int trial_steps) {
  GUARD_CTX(ctx);
  return ctx->autotune(trial_steps);
}

int dugks_get_info(const dugks_ctx* ctx, dugks_info* out) {
  GUARD_CTX(ctx);
  if (!out) return DUGKS_E_ARG;
  ctx->info(0, out);
  return DUGKS_OK;
}

int dugks_time_steps(dugks_ctx* ctx, int nsteps, float* ms_total) {
  GUARD_CTX(ctx);
  return ctx->time_steps(nsteps, ms_total);
}

// ------------------------------------------------------------- batches
int dugks_batch_create(dugks_batch** out, int n, const dugks_instance_desc* d, int storage) {
  if (!out) return DUGKS_E_ARG;
  *out = nullptr;
  dugks_batch* b = new (std::nothrow) dugks_batch();
  if (!b) return DUGKS_E_NOMEM;
  b->magic = dugks::kMagicBatch;
  *out = b;
  if (n < 1 || !d) return b->fail(DUGKS_E_ARG, "empty batch");
  if (storage < DUGKS_F64 || storage > DUGKS_BF16NEQ) return b->fail(DUGKS_E_UNSUPPORTED, "unknown storage");
  b->storage = storage;
  if (storage == DUGKS_F64) { b->launch.rows_per_wave = 32; b->launch.waves_per_block = 1; }
  b->inst.resize(n);
  for (int k = 0; k < n; ++k) {
    dugks_params p = d[k].p;
    p.storage = storage;
    p.kernel = DUGKS_KERNEL_FUSED;
    int rc = dugks::init_instance(b->inst[k], d[k].nx, d[k].ny, d[k].xf, d[k].yf, d[k].q, &p, b->err);
    if (rc) { b->err = "instance " + std::to_string(k) + ": " + b->err; return rc; }
    if (b->inst[k].bcx == DUGKS_BC_DIRICHLET || b->inst[k].bcy == DUGKS_BC_DIRICHLET)
      return b->fail(DUGKS_E_UNSUPPORTED, "Dirichlet walls are not built for batches");
    if (d[k].q != d[0].q) return b->fail(DUGKS_E_UNSUPPORTED, "all instances of a batch share q");
    rc = dugks::set_B_impl(b->inst[k], d[k].b_deg, d[k].bx, d[k].by, b->err);
    if (rc == 0) rc = dugks::set_D_impl(b->inst[k], d[k].d_deg, d[k].dxx, d[k].dxy, d[k].dyy, b->err);
    if (rc) { b->err = "instance " + std::to_string(k) + ": " + b->err; return rc; }
  }
  return DUGKS_OK;
}

size_t dugks_batch_workspace_bytes(const dugks_batch* b) {
  if (!b || b->magic != dugks::kMagicBatch || b->inst.empty() || b->inst[0].nx == 0) return 0;
  Engine tmp_view;
  tmp_view.storage = b->storage;
  tmp_view.inst = b->inst;
  tmp_view.launch = b->launch;
  tmp_view.layout();
  return tmp_view.total_bytes;
}

int dugks_batch_bind(dugks_batch* b, void* ws, size_t bytes, void* stream) {
  GUARD_BATCH(b);
  if (b->inst.empty() || b->inst[0].nx == 0) return b->fail(DUGKS_E_STATE, "batch was not created");
  return b->bind(ws, bytes, stream);
}

int dugks_batch_set_phi(dugks_batch* b, int i, const double* phi, int on_device) {
  GUARD_BATCH(b);
  if (i < 0 || i >= (int)b->inst.size()) return b->fail(DUGKS_E_ARG, "instance index");
  return b->set_phi(i, phi, on_device);
}

int dugks_batch_set_source(dugks_batch* b, int i, const double* g_dev, double gamma) {
  GUARD_BATCH(b);
  if (i < 0 || i >= (int)b->inst.size()) return b->fail(DUGKS_E_ARG, "instance index");
  const int zero = 0;
  return b->set_source_terms(i, g_dev ? 1 : 0, g_dev, &zero, &gamma);
}

int dugks_batch_set_source_terms(dugks_batch* b, int i, int nterms, const double* g_dev,
                                 const int* powers, const double* gammas) {
  GUARD_BATCH(b);
  if (i < 0 || i >= (int)b->inst.size()) return b->fail(DUGKS_E_ARG, "instance index");
  return b->set_source_terms(i, nterms, g_dev, powers, gammas);
}
int dugks_batch_autotune(dugks_batch* b, int trial_steps) {
  GUARD_BATCH(b);
  return b->autotune(trial_steps);
}

int dugks_batch_set_launch(dugks_batch* b, int rows, int wpb, int sched, int xcd) {
  GUARD_BATCH(b);
  return b->set_launch(rows, wpb, sched, xcd);
}

int dugks_batch_step(dugks_batch* b, int nsteps) {
  GUARD_BATCH(b);
  return b->do_steps(nsteps);
}

int dugks_batch_get_phi(dugks_batch* b, int i, double* out, int on_device) {
  GUARD_BATCH(b);
  if (i < 0 || i >= (int)b->inst.size()) return b->fail(DUGKS_E_ARG, "instance index");
  return b->get_phi(i, out, on_device);
}

int dugks_batch_get_info(const dugks_batch* b, int i, dugks_info* out) {
  GUARD_BATCH(b);
  if (!out || i < 0 || i >= (int)b->inst.size()) return DUGKS_E_ARG;
  b->info(i, out);
  return DUGKS_OK;
}

int dugks_batch_totals(const dugks_batch* b, long long* cells, size_t* state_bytes) {
  GUARD_BATCH(b);
  long long c = 0;
  size_t s = 0;
  for (auto& in : b->inst) { c += in.cells(); s += in.buffer_bytes(b->storage); }
  if (cells) *cells = c;
  if (state_bytes) *state_bytes = s;
  return DUGKS_OK;
}

int dugks_batch_time_steps(dugks_batch* b, int nsteps, float* ms_total) {
  GUARD_BATCH(b);
  return b->time_steps(nsteps, ms_total);
}

const char* dugks_last_error(const void* h) {
  Engine* e = as_engine(h);
  return e ? e->err.c_str() : "invalid handle";
}

void dugks_destroy(void* h) {
  Engine* e = as_engine(h);
  if (!e) return;
  const uint32_t m = e->magic;
  e->magic = 0;
  if (m == dugks::kMagicCtx) delete (dugks_ctx*)e;
  else delete (dugks_batch*)e;
}

}  // extern "C"
