// Drives the host side of libdugks (create, coefficient setters, source and
// Dirichlet arguments, launch settings, checkpoint format checks, batches, the
// 3-D family with its sources, autotuner and batches, and the 1-D family)
// without a GPU, for a build of the host code with
// AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_host_sanitize.py).  Every call must return its documented code.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "dugks.h"
#include "dugks1d.h"
#include "dugks3d.h"

static int fails = 0;
#define EXPECT(call, code)                                                               \
  do {                                                                                   \
    const int rc_ = (call);                                                              \
    if (rc_ != (code)) {                                                                 \
      fprintf(stderr, "line %d: %s returned %d, expected %d\n", __LINE__, #call, rc_, code); \
      ++fails;                                                                           \
    }                                                                                    \
  } while (0)

static std::vector<double> faces(int n, double stretch) {
  std::vector<double> f(n + 1);
  for (int i = 0; i <= n; ++i) {
    const double s = (double)i / n;
    f[i] = stretch > 0 ? 0.5 * (1.0 + tanh(stretch * (2.0 * s - 1.0)) / tanh(stretch)) : s;
  }
  return f;
}

static dugks_params params2(int storage, int bcx, int bcy) {
  dugks_params p;
  memset(&p, 0, sizeof(p));
  p.abi_version = DUGKS_ABI_VERSION;
  p.storage = storage;
  p.bc[0] = p.bc[1] = bcx;
  p.bc[2] = p.bc[3] = bcy;
  p.kernel = DUGKS_KERNEL_FUSED;
  p.c = 1.3;
  p.cfl = 0.5;
  p.alpha = 1e-3;
  return p;
}

static void two_d() {
  for (int q : {9, 5})
    for (int storage = DUGKS_F64; storage <= DUGKS_BF16NEQ; ++storage)
      for (int bc = 0; bc <= 2; ++bc) {
        const int nx = 37, ny = 21;
        std::vector<double> xf = faces(nx, bc ? 1.4 : 0), yf = faces(ny, bc ? 1.1 : 0);
        dugks_params p = params2(storage, bc, bc);
        dugks_ctx* h = nullptr;
        EXPECT(dugks_create(&h, nx, ny, xf.data(), yf.data(), q, &p), DUGKS_OK);
        const double bx[3] = {0.0, 0.2, 0.1}, by[3] = {0.0, -0.1, 0.2};
        const double dxx[3] = {0.0, 1.0, 0.2}, dxy[3] = {0.0, 0.1, 0.0}, dyy[3] = {0.0, 0.9, 0.0};
        const double d5[2] = {0.0, 1.0}, z[2] = {0.0, 0.0};
        EXPECT(dugks_set_B(h, 2, bx, by), DUGKS_OK);
        EXPECT(q == 9 ? dugks_set_D(h, 2, dxx, dxy, dyy) : dugks_set_D(h, 1, d5, z, d5), DUGKS_OK);
        EXPECT(dugks_set_B(h, DUGKS_MAX_DEG + 1, bx, by), DUGKS_E_ARG);
        const int pw[2] = {0, 3}, bad_pw[1] = {DUGKS_MAX_SRC_POW + 1};
        const double gam[2] = {0.1, 0.0};
        const double* g = (const double*)(uintptr_t)256;   // never dereferenced on the host
        const int want = storage >= DUGKS_F16NEQ ? DUGKS_E_UNSUPPORTED : DUGKS_OK;
        EXPECT(dugks_set_source_terms(h, 2, g, pw, gam), want);
        EXPECT(dugks_set_source_terms(h, DUGKS_MAX_SRC_TERMS + 1, g, pw, gam), DUGKS_E_ARG);
        EXPECT(dugks_set_source_terms(h, 1, g, bad_pw, gam),
               storage >= DUGKS_F16NEQ ? DUGKS_E_UNSUPPORTED : DUGKS_E_ARG);
        EXPECT(dugks_set_source(h, nullptr, 0.0), DUGKS_OK);
        EXPECT(dugks_set_dirichlet(h, nullptr, 3), DUGKS_E_ARG);
        EXPECT(dugks_set_dirichlet(h, nullptr, 0), DUGKS_OK);
        EXPECT(dugks_set_launch(h, 16, 4, DUGKS_SCHED_GRID, 1), DUGKS_OK);
        EXPECT(dugks_set_launch(h, 16, 3, DUGKS_SCHED_GRID, 1), DUGKS_E_ARG);
        EXPECT(dugks_step(h, 1), DUGKS_E_STATE);          // not bound
        dugks_info info;
        EXPECT(dugks_get_info(h, &info), DUGKS_OK);
        if (dugks_workspace_bytes(h) < 2 * info.state_bytes) { fprintf(stderr, "workspace too small\n"); ++fails; }
        size_t len = 0;
        EXPECT(dugks_checkpoint(h, nullptr, &len), DUGKS_OK);   // size query
        if (len < info.state_bytes) { fprintf(stderr, "checkpoint size %zu\n", len); ++fails; }
        std::vector<unsigned char> junk(4096, 0xab);
        const int r = dugks_restore(h, junk.data(), junk.size());
        if (r != DUGKS_E_FORMAT && r != DUGKS_E_STATE) { fprintf(stderr, "restore of junk: %d\n", r); ++fails; }
        if (!dugks_last_error(h)) ++fails;
        dugks_destroy(h);
      }
  // rejected arguments: each leaves a handle naming the problem
  std::vector<double> xf = faces(8, 0), yf = faces(6, 0), bad = xf;
  bad[3] = bad[2];
  struct Case { int nx, ny, q; const double* x; dugks_params p; int code; };
  dugks_params ok = params2(DUGKS_F64, 0, 0), cfl = ok, abi = ok, bcmix = ok, plain = ok;
  cfl.cfl = 1.0;
  abi.abi_version = 999;
  bcmix.bc[0] = DUGKS_BC_DIRICHLET; bcmix.bc[1] = DUGKS_BC_MIRROR;
  plain.kernel = DUGKS_KERNEL_PLAIN; plain.storage = DUGKS_F32;
  const Case cases[] = {{0, 6, 9, xf.data(), ok, DUGKS_E_ARG},  {8, 6, 7, xf.data(), ok, DUGKS_E_UNSUPPORTED},
                        {8, 6, 9, bad.data(), ok, DUGKS_E_ARG}, {8, 6, 9, xf.data(), cfl, DUGKS_E_ARG},
                        {8, 6, 9, xf.data(), abi, DUGKS_E_ARG}, {8, 6, 9, xf.data(), bcmix, DUGKS_E_UNSUPPORTED},
                        {8, 6, 9, xf.data(), plain, DUGKS_E_UNSUPPORTED}};
  for (const Case& c : cases) {
    dugks_ctx* h = nullptr;
    EXPECT(dugks_create(&h, c.nx, c.ny, c.x, yf.data(), c.q, &c.p), c.code);
    if (h) {
      if (!dugks_last_error(h)[0]) ++fails;
      dugks_destroy(h);
    }
  }
}

static void batch() {
  const int n = 5;
  std::vector<std::vector<double>> fx(n), fy(n);
  std::vector<dugks_instance_desc> d(n);
  for (int i = 0; i < n; ++i) {
    fx[i] = faces(20 + 13 * i, 0);
    fy[i] = faces(17 + 7 * i, 0);
    memset(&d[i], 0, sizeof(d[i]));
    d[i].nx = 20 + 13 * i;
    d[i].ny = 17 + 7 * i;
    d[i].q = 9;
    d[i].xf = fx[i].data();
    d[i].yf = fy[i].data();
    d[i].p = params2(DUGKS_F32, 0, 0);
    d[i].b_deg = 2;
    d[i].bx[2] = d[i].by[2] = 0.1 * i;
    d[i].d_deg = 1;
    d[i].dxx[1] = d[i].dyy[1] = 1.0;
  }
  for (int storage = DUGKS_F64; storage <= DUGKS_BF16NEQ; ++storage) {
    dugks_batch* b = nullptr;
    EXPECT(dugks_batch_create(&b, n, d.data(), storage), DUGKS_OK);
    long long cells = 0;
    size_t bytes = 0;
    EXPECT(dugks_batch_totals(b, &cells, &bytes), DUGKS_OK);
    EXPECT(dugks_batch_set_launch(b, 8, 8, DUGKS_SCHED_GRID, 1), storage == DUGKS_F64 ? DUGKS_E_ARG : DUGKS_OK);
    EXPECT(dugks_batch_step(b, 1), DUGKS_E_STATE);
    dugks_info info;
    EXPECT(dugks_batch_get_info(b, n - 1, &info), DUGKS_OK);
    EXPECT(dugks_batch_get_info(b, n, &info), DUGKS_E_ARG);
    dugks_destroy(b);
  }
  d[2].nx = 0;
  dugks_batch* b = nullptr;
  EXPECT(dugks_batch_create(&b, n, d.data(), DUGKS_F32), DUGKS_E_ARG);
  if (b) dugks_destroy(b);
}

static void three_d() {
  for (int q : {19, 15, 7})
    for (int storage : {DUGKS_F64, DUGKS_F32})
      for (int bc = 0; bc <= 2; ++bc) {
        std::vector<double> xf = faces(70, 1.2), yf = faces(9, 0), zf = faces(7, 1.5);
        dugks3_params p;
        memset(&p, 0, sizeof(p));
        p.abi_version = DUGKS3_ABI_VERSION;
        p.storage = storage;
        p.bc[0] = bc; p.bc[1] = (bc + 1) % 3; p.bc[2] = (bc + 2) % 3;
        p.c = 1.1; p.cfl = 0.5; p.alpha = 1e-3;
        dugks3_ctx* h = nullptr;
        EXPECT(dugks3_create(&h, 70, 9, 7, xf.data(), yf.data(), zf.data(), q, &p), DUGKS_OK);
        const double b[9] = {0, 0.1, 0.2, 0, -0.1, 0.1, 0, 0.05, 0};
        EXPECT(dugks3_set_B(h, 2, b), DUGKS_OK);
        std::vector<double> dd(12, 0.0);
        dd[1] = dd[3] = dd[5] = 1.0;
        EXPECT(dugks3_set_D(h, 1, dd.data()), DUGKS_OK);
        EXPECT(dugks3_set_dirichlet(h, nullptr, 2), DUGKS_E_ARG);
        EXPECT(dugks3_set_launch(h, storage == DUGKS_F64 ? 2 : 4, 16), DUGKS_OK);
        EXPECT(dugks3_step(h, 1), DUGKS_E_STATE);
        dugks3_info info;
        EXPECT(dugks3_get_info(h, &info), DUGKS_OK);
        dugks3_destroy(h);
      }
}

static dugks3_ctx* make3(int q, int storage, int nx, int bcx) {
  std::vector<double> xf = faces(nx, 1.2), yf = faces(9, 0), zf = faces(7, 1.5);
  dugks3_params p;
  memset(&p, 0, sizeof(p));
  p.abi_version = DUGKS3_ABI_VERSION;
  p.storage = storage;
  p.bc[0] = bcx; p.bc[1] = DUGKS_BC_PERIODIC; p.bc[2] = DUGKS_BC_MIRROR;
  p.c = 1.1; p.cfl = 0.5; p.alpha = 1e-3;
  dugks3_ctx* h = nullptr;
  EXPECT(dugks3_create(&h, nx, 9, 7, xf.data(), yf.data(), zf.data(), q, &p), DUGKS_OK);
  return h;
}

// 3-D source arguments (no scratch), autotune and batch arguments
static void three_d_sources_and_batches() {
  const int pw[2] = {1, 0};
  const double gm[2] = {0.2, -0.4};
  void* g = (void*)(uintptr_t)256;
  for (int q : {19, 15, 7}) {
    dugks3_ctx* h = make3(q, DUGKS_F64, 40, DUGKS_BC_PERIODIC);
    EXPECT((int)dugks3_source_scratch_bytes(h), 0);
    const int bad[2] = {1, 4};
    EXPECT(dugks3_set_source_terms(h, 2, (const double*)g, bad, gm, nullptr, 0), DUGKS_E_ARG);
    EXPECT(dugks3_set_source_terms(h, 2, nullptr, pw, gm, nullptr, 0), DUGKS_E_ARG);
    EXPECT(dugks3_set_source_terms(h, 2, (const double*)g, pw, gm, nullptr, 0), DUGKS_OK);
    EXPECT(dugks3_autotune(h, 2), DUGKS_E_STATE);
    EXPECT(dugks3_set_source_terms(h, 0, nullptr, nullptr, nullptr, nullptr, 0), DUGKS_OK);
    dugks3_destroy(h);
  }
  for (int storage : {DUGKS_F64, DUGKS_F32}) {
    dugks3_ctx* hs[3] = {make3(19, storage, 40, DUGKS_BC_PERIODIC), make3(19, storage, 130, DUGKS_BC_MIRROR),
                         make3(19, storage, 9, DUGKS_BC_DIRICHLET)};
    dugks3_ctx* h15 = make3(15, storage, 40, DUGKS_BC_PERIODIC);
    dugks3_ctx* h7 = make3(7, storage, 40, DUGKS_BC_PERIODIC);
    dugks3_batch* b = nullptr;
    EXPECT(dugks3_batch_create(&b, 0, hs), DUGKS_E_ARG);
    dugks3_batch_destroy(b);
    dugks3_ctx* mixed[2] = {hs[0], h15};
    EXPECT(dugks3_batch_create(&b, 2, mixed), DUGKS_E_ARG);
    dugks3_batch_destroy(b);
    EXPECT(dugks3_batch_create(&b, 1, &h7), DUGKS_E_UNSUPPORTED);
    dugks3_batch_destroy(b);
    EXPECT(dugks3_batch_create(&b, 3, hs), DUGKS_OK);
    const size_t nb = dugks3_batch_workspace_bytes(b);
    EXPECT(nb >= 3 * sizeof(void*) + 4 * sizeof(long long), 1);
    EXPECT(dugks3_batch_step(b, 1), DUGKS_E_STATE);
    EXPECT(dugks3_batch_bind(b, (void*)(uintptr_t)4096, nb, nullptr), DUGKS_E_STATE);
    EXPECT(dugks3_batch_bind(b, nullptr, nb, nullptr), DUGKS_E_ARG);
    EXPECT(dugks3_batch_set_launch(b, storage == DUGKS_F64 ? 3 : 5, 8), DUGKS_E_ARG);
    EXPECT(dugks3_batch_set_launch(b, 2, 0), DUGKS_E_ARG);
    EXPECT(dugks3_batch_set_launch(b, 2, 5), DUGKS_OK);
    int rows = 0, planes = 0;
    long long blocks = 0, cells = 0;
    EXPECT(dugks3_batch_get_info(b, &rows, &planes, &blocks, &cells), DUGKS_OK);
    EXPECT(rows == 2 && planes == 5 && cells == (40LL + 130 + 9) * 9 * 7, 1);
    float ms = 0;
    EXPECT(dugks3_batch_time_steps(b, 1, &ms), DUGKS_E_STATE);
    EXPECT(dugks3_batch_last_error(b)[0] != 0, 1);
    dugks3_batch_destroy(b);
    for (dugks3_ctx* h : hs) dugks3_destroy(h);
    dugks3_destroy(h15);
    dugks3_destroy(h7);
  }
  EXPECT(dugks3_batch_step(nullptr, 1), DUGKS_E_ARG);
  dugks3_batch_destroy(nullptr);
}

static void one_d() {
  for (int storage : {DUGKS_F64, DUGKS_F32}) {
    std::vector<double> xf = faces(50, 1.3);
    dugks1_params p;
    memset(&p, 0, sizeof(p));
    p.abi_version = DUGKS1_ABI_VERSION;
    p.storage = storage;
    p.bc = DUGKS_BC_DIRICHLET;
    p.c = 2.0; p.cfl = 0.5; p.alpha = 1e-3;
    const double coef[7] = {0.1, 0.2, 1.0, 0.5, 0.1, 1.0, 0.3};
    memcpy(p.coef, coef, sizeof(coef));
    dugks1_ctx* h = nullptr;
    EXPECT(dugks1_create(&h, 50, xf.data(), &p), DUGKS_OK);
    EXPECT(dugks1_set_dirichlet(h, nullptr, 4), DUGKS_E_ARG);
    EXPECT(dugks1_step(h, 1), DUGKS_E_STATE);
    dugks1_info info;
    EXPECT(dugks1_get_info(h, &info), DUGKS_OK);
    dugks1_destroy(h);
  }
}

int main() {
  two_d();
  batch();
  three_d();
  three_d_sources_and_batches();
  one_d();
  if (fails == 0) printf("sanitized host runs: ok\n");
  return fails != 0;
}
