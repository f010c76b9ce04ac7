// Host-side checks of the library's argument validation and workspace
// arithmetic, built with AddressSanitizer and UndefinedBehaviorSanitizer on
// the host code and run without a GPU.  Every call here either needs no
// device (the workspace query) or carries an argument the library must
// refuse before it touches the context or any device memory, so the context
// handed in is a zeroed stand-in that the library never dereferences for
// these cases (a validation gap would reach hipSetDevice and fail there with
// COMM_EHIP instead of the expected code, which the harness reports).
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "comm.h"

static int failures = 0;

static void expect(bool ok, const char* what, int line) {
  if (!ok) {
    std::fprintf(stderr, "FAILED line %d: %s (last error: %s)\n", line, what, comm_last_error());
    ++failures;
  }
}
#define EXPECT(c) expect((c), #c, __LINE__)

static comm_dense dense(std::vector<int64_t> dims, const float* X) {
  comm_dense d;
  std::memset(&d, 0, sizeof d);
  d.ndim = (int)dims.size();  // may exceed COMM_MAX_NDIM: the library must refuse it
  for (size_t n = 0; n < dims.size() && n < COMM_MAX_NDIM; ++n) d.dims[n] = dims[n];
  d.X = X;
  return d;
}

static comm_opts opts(double beta, int L = 1, int cache = 0) {
  comm_opts o;
  std::memset(&o, 0, sizeof o);
  o.beta = beta;
  o.eps = 1e-12;
  o.eps_x = 1e-12;
  o.inner_sweeps = L;
  o.precision = COMM_FP32;
  o.cache_pq = cache;
  return o;
}

int main() {
  static float fake[64];
  float* f = fake;
  // workspace query: pure host arithmetic over every layout
  const std::vector<std::vector<int64_t>> shapes = {
      {1, 1, 1}, {2, 3, 5}, {16, 32, 64}, {17, 33, 65}, {256, 256, 256}, {1000, 3, 1}, {1 << 12, 1 << 12, 1 << 8},
      {5, 6, 7, 8}, {80, 70, 60, 50}, {4096, 4096, 1, 1}, {3, 4, 5, 6, 7}, {27, 24, 7, 100, 100}, {64, 64, 64, 64, 64}};
  for (const auto& s : shapes) {
    comm_dense x = dense(s, f);
    for (int R : {1, 5, 16, 31, 32}) {
      comm_model m;
      std::memset(&m, 0, sizeof m);
      m.kind = COMM_CP;
      m.rank = R;
      for (double beta : {0.0, 0.5, 1.0, 1.5})
        for (int cache : {0, 1, COMM_CACHE_AUTO})
          for (int op = 0; op < 3; ++op) {
            comm_opts o = opts(beta, 2, cache);
            const size_t b = comm_workspace_bytes(&x, &m, &o, op);
            EXPECT(b > 0);
          }
    }
    for (int J : {1, 4, 10, 16, 32}) {
      comm_model m;
      std::memset(&m, 0, sizeof m);
      m.kind = COMM_TUCKER;
      for (int n = 0; n < x.ndim; ++n) m.core_dims[n] = J;
      m.core = f;
      for (double beta : {0.0, 1.0, 1.5})
        for (int cache : {0, 1})
          for (int op = 0; op < 3; ++op) {
            comm_opts o = opts(beta, 1, cache);
            (void)comm_workspace_bytes(&x, &m, &o, op);  // 0 is allowed (order-N row limits)
          }
    }
  }
  // invalid shapes and models: the query answers 0
  {
    comm_model m;
    std::memset(&m, 0, sizeof m);
    m.kind = COMM_CP;
    m.rank = 8;
    comm_opts o = opts(1.0);
    for (const auto& s : std::vector<std::vector<int64_t>>{{}, {5}, {0, 3, 4}, {-1, 3, 4}, {3, 4, 5, 6, 7, 8},
                                                            {int64_t(1) << 40, 2, 2}}) {
      comm_dense x = dense(s, f);
      EXPECT(comm_workspace_bytes(&x, &m, &o, 1) == 0);
    }
    comm_dense x = dense({4, 5, 6}, f);
    EXPECT(comm_workspace_bytes(&x, nullptr, &o, 1) == 0);
    EXPECT(comm_workspace_bytes(&x, &m, nullptr, 1) == 0);
    EXPECT(comm_workspace_bytes(nullptr, &m, &o, 1) == 0);
    m.kind = COMM_TUCKER;
    m.core_dims[0] = 33;
    m.core_dims[1] = m.core_dims[2] = 4;
    EXPECT(comm_workspace_bytes(&x, &m, &o, 1) == 0);
  }

  // entry points: a NULL context, then arguments refused before any device work
  std::vector<char> stand_in(1 << 16, 0);
  comm_ctx* ctx = reinterpret_cast<comm_ctx*>(stand_in.data());
  comm_dense x = dense({8, 9, 10}, f);
  comm_model cp;
  std::memset(&cp, 0, sizeof cp);
  cp.kind = COMM_CP;
  cp.rank = 4;
  for (int n = 0; n < 3; ++n) cp.factors[n] = f;
  comm_opts good = opts(0.5, 2);
  EXPECT(comm_jcomm_outer(nullptr, &x, &cp, &good, nullptr, nullptr) == COMM_EINVAL);
  EXPECT(comm_jcomm_outer_noalloc(nullptr, &x, &cp, &good, nullptr, nullptr) == COMM_EINVAL);
  EXPECT(comm_cp_update(nullptr, &x, &cp, 0, &good, nullptr) == COMM_EINVAL);
  EXPECT(comm_beta_objective(nullptr, &x, &cp, &good, nullptr, nullptr) == COMM_EINVAL);
  for (double beta : {-0.5, 2.0, 3.0, std::numeric_limits<double>::quiet_NaN()}) {
    comm_opts o = opts(beta, 2);
    EXPECT(comm_jcomm_outer(ctx, &x, &cp, &o, nullptr, nullptr) == COMM_EINVAL);
    EXPECT(comm_jcomm_outer_noalloc(ctx, &x, &cp, &o, nullptr, nullptr) == COMM_EINVAL);
    EXPECT(comm_cp_update(ctx, &x, &cp, -1, &o, nullptr) == COMM_EINVAL);
  }
  {
    comm_opts o = opts(0.5, 0);
    EXPECT(comm_jcomm_outer(ctx, &x, &cp, &o, nullptr, nullptr) == COMM_EINVAL);
    o = opts(0.5, 1);
    o.eps = 0.0;
    EXPECT(comm_jcomm_outer(ctx, &x, &cp, &o, nullptr, nullptr) == COMM_EINVAL);
    o = opts(0.5, 1);
    o.check_inputs = 1;
    EXPECT(comm_jcomm_outer_noalloc(ctx, &x, &cp, &o, nullptr, nullptr) == COMM_EINVAL);
  }
  {
    comm_model bad = cp;
    bad.rank = 0;
    EXPECT(comm_jcomm_outer(ctx, &x, &bad, &good, nullptr, nullptr) == COMM_EINVAL);
    bad.rank = 33;
    EXPECT(comm_jcomm_outer(ctx, &x, &bad, &good, nullptr, nullptr) == COMM_EUNSUPPORTED);
    bad = cp;
    bad.factors[1] = nullptr;
    EXPECT(comm_jcomm_outer(ctx, &x, &bad, &good, nullptr, nullptr) == COMM_EINVAL);
    EXPECT(comm_cp_update(ctx, &x, &cp, 3, &good, nullptr) == COMM_EINVAL);
    EXPECT(comm_cp_update(ctx, &x, &cp, -2, &good, nullptr) == COMM_EINVAL);
    comm_dense nox = x;
    nox.X = nullptr;
    EXPECT(comm_jcomm_outer(ctx, &nox, &cp, &good, nullptr, nullptr) == COMM_EINVAL);
    comm_dense two = dense({8, 9}, f);
    EXPECT(comm_jcomm_outer(ctx, &two, &cp, &good, nullptr, nullptr) != COMM_OK);
    comm_model tk;
    std::memset(&tk, 0, sizeof tk);
    tk.kind = COMM_TUCKER;
    for (int n = 0; n < 3; ++n) {
      tk.factors[n] = f;
      tk.core_dims[n] = 4;
    }
    EXPECT(comm_jcomm_outer(ctx, &x, &tk, &good, nullptr, nullptr) == COMM_EINVAL);  // no core
    tk.core = f;
    tk.core_dims[2] = 40;
    EXPECT(comm_jcomm_outer(ctx, &x, &tk, &good, nullptr, nullptr) == COMM_EUNSUPPORTED);
    tk.kind = 7;
    EXPECT(comm_jcomm_outer(ctx, &x, &tk, &good, nullptr, nullptr) == COMM_EINVAL);
  }
  // sparse arguments
  {
    int32_t idx[3] = {0, 1, 2};
    comm_coo c;
    std::memset(&c, 0, sizeof c);
    c.ndim = 3;
    c.dims[0] = c.dims[1] = c.dims[2] = 4;
    c.nnz = 3;
    for (int n = 0; n < 3; ++n) c.idx[n] = idx;
    c.val = f;
    comm_opts kl = opts(1.0);
    comm_opts is = opts(0.0);
    EXPECT(comm_cp_jcomm_outer_coo(ctx, &c, &cp, &is, nullptr, nullptr) == COMM_EUNSUPPORTED);
    c.nnz = -1;
    EXPECT(comm_cp_jcomm_outer_coo(ctx, &c, &cp, &kl, nullptr, nullptr) == COMM_EINVAL);
    c.nnz = 3;
    c.val = nullptr;
    EXPECT(comm_cp_jcomm_outer_coo(ctx, &c, &cp, &kl, nullptr, nullptr) == COMM_EINVAL);
    c.val = f;
    c.dims[1] = 0;
    EXPECT(comm_beta_objective_coo(ctx, &c, &cp, &kl, reinterpret_cast<double*>(fake), nullptr) == COMM_EINVAL);
    c.dims[1] = 4;
    EXPECT(comm_beta_objective_coo(ctx, &c, &cp, &kl, nullptr, nullptr) == COMM_EINVAL);
    comm_opts half = opts(0.5);
    c.dims[0] = c.dims[1] = c.dims[2] = 1 << 24;
    EXPECT(comm_cp_update_coo(ctx, &c, &cp, 0, &half, nullptr) == COMM_ENOMEM);
    comm_coo_plan* plan = nullptr;
    EXPECT(comm_coo_plan_create(ctx, &c, nullptr, nullptr) == COMM_EINVAL);
    EXPECT(comm_coo_plan_destroy(plan) == COMM_OK);
  }
  // batches: refused before any problem runs
  {
    comm_problem pr[2];
    std::memset(pr, 0, sizeof pr);
    pr[0].x = &x;
    pr[0].model = &cp;
    pr[0].opts = &good;
    EXPECT(comm_jcomm_outer_batched(ctx, pr, 2, 0, nullptr) == COMM_EINVAL);  // problem 1 has NULLs
    EXPECT(comm_jcomm_outer_batched(ctx, pr, -1, 0, nullptr) == COMM_EINVAL);
    EXPECT(comm_jcomm_outer_batched(ctx, nullptr, 1, 0, nullptr) == COMM_EINVAL);
  }
  // contexts: no device here, so creation fails cleanly; destroying NULL is fine
  comm_ctx* real = nullptr;
  EXPECT(comm_create(-1, 0, &real) != COMM_OK && real == nullptr);
  EXPECT(comm_create(0, 0, nullptr) == COMM_EINVAL);
  EXPECT(comm_destroy(nullptr) == COMM_OK);
  EXPECT(comm_last_error() != nullptr);
  if (failures) {
    std::fprintf(stderr, "%d host checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
