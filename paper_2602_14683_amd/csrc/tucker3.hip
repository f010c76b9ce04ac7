// Dense 3-way Tucker: B-CoMM and J-CoMM orchestration, the small contraction
// GEMMs that turn the pass's V into the mode-1, mode-2 and core numerators,
// and the closed-form beta = 1 denominators.
//
// With V[i][j][c] = sum_k W[i][j][k] C'[k][c] (W = P or Q, from the fused pass):
//   U[i][b][c]   = sum_j B'[j][b] V[i][j][c]
//   Num1[i][a]   = sum_{b,c} G'[a][b][c] U[i][b][c]                 (factor A, App. C)
//   Ncore[a][b][c] = sum_i A'[i][a] U[i][b][c]                       (core, App. C)
//   H[i][b][c]   = sum_a A'[i][a] G'[a][b][c]
//   Num2[j][b]   = sum_{i,c} V[i][j][c] H[i][b][c]                   (factor B)
// and the mode-3 numerator comes from the pass directly.  These are the
// direct-form contractions of App. C / App. E: the partial tensor B^(n) is
// never formed; only V (J3/K of the size of X) and the I x J2 x J3 U / H.

#include "host_util.h"
#include "tucker3.h"
#include "tucker3_impl.h"

namespace comm {

TkGrid tk_grid(int I, int J) {
  TkGrid g;
  g.gi = (I + kTkTI - 1) / kTkTI;
  g.gj = (J + kTkTJ - 1) / kTkTJ;
  return g;
}

// ---------------------------------------------------------------------------------------- GEMM

constexpr int kGT = 32;   // output tile
constexpr int kGK = 32;   // k chunk

__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
  __shared__ float As[kGK][kGT + 1];
  __shared__ float Bs[kGK][kGT + 1];
  const int tiles_m = (g.M + kGT - 1) / kGT, tiles_n = (g.N + kGT - 1) / kGT;
  int id = blockIdx.x;
  const int tn = id % tiles_n;
  id /= tiles_n;
  const int tm = id % tiles_m;
  id /= tiles_m;
  const int bat = id % g.batch;
  const int split = id / g.batch;
  const int kc = (g.K + g.splits - 1) / g.splits;
  const int k0 = split * kc, k1 = min(g.K, k0 + kc);
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  float acc[2][2] = {};
  for (int kb = k0; kb < k1; kb += kGK) {
    for (int e = t; e < kGK * kGT; e += 256) {
      const int kk = e / kGT, mm = e % kGT;
      const int m = tm * kGT + mm, k = kb + kk;
      float va = 0.0f;
      if (m < g.M && k < k1)
        va = g.A[(int64_t)bat * g.sab + (int64_t)m * g.sam + (int64_t)(k / g.akin) * g.sako +
                 (int64_t)(k % g.akin) * g.saki];
      As[kk][mm] = va;
      const int n = tn * kGT + mm;
      float vb = 0.0f;
      if (n < g.N && k < k1)
        vb = g.B[(int64_t)bat * g.sbb + (int64_t)(k / g.bkin) * g.sbko + (int64_t)(k % g.bkin) * g.sbki +
                 (int64_t)n * g.sbn];
      Bs[kk][mm] = vb;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kGK; ++kk) {
      const float a0 = As[kk][2 * ty], a1 = As[kk][2 * ty + 1];
      const float b0 = Bs[kk][2 * tx], b1 = Bs[kk][2 * tx + 1];
      acc[0][0] = fmaf(a0, b0, acc[0][0]);
      acc[0][1] = fmaf(a0, b1, acc[0][1]);
      acc[1][0] = fmaf(a1, b0, acc[1][0]);
      acc[1][1] = fmaf(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int m = tm * kGT + 2 * ty + u, n = tn * kGT + 2 * tx + v;
      if (m < g.M && n < g.N) g.out[(int64_t)split * g.sos + (int64_t)bat * g.sob + (int64_t)m * g.ldo + n] = acc[u][v];
    }
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  const int tiles = ((g.M + kGT - 1) / kGT) * ((g.N + kGT - 1) / kGT) * g.batch * g.splits;
  hipLaunchKernelGGL(gemm_kernel, dim3(tiles), dim3(256), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------- closed-form den

__global__ void __launch_bounds__(1024) tk_den_closed_kernel(TkModel m, int I, int J, int K, float* den,
                                                             float* dcore) {
  __shared__ float red[32][33];
  __shared__ float S[3][32];
  __shared__ float T1[32][33], T2[32][33];
  const int t = threadIdx.x;
  const int c = t & 31, g = t >> 5;
  const FView* F[3] = {&m.A, &m.B, &m.C};
  const int rows[3] = {I, J, K};
  for (int f = 0; f < 3; ++f) {
    float s = 0.0f;
    for (int r = g; r < rows[f]; r += 32) s += F[f]->at(r, c, rows[f]);
    red[g][c] = s;
    __syncthreads();
    if (t < 32) {
      float acc = 0.0f;
      for (int q = 0; q < 32; ++q) acc += red[q][t];
      S[f][t] = acc;
    }
    __syncthreads();
  }
  // T1[a][c] = sum_b G[a][b][c] S_B[b];  T2[a][b] = sum_c G[a][b][c] S_C[c]
  {
    const int a = g, x = c;
    float s1 = 0.0f, s2 = 0.0f;
    if (a < m.J1) {
      if (x < m.J3)
        for (int b = 0; b < m.J2; ++b) s1 = fmaf(m.G[((int64_t)a * m.J2 + b) * m.ldG + x], S[1][b], s1);
      if (x < m.J2)
        for (int cc = 0; cc < m.J3; ++cc) s2 = fmaf(m.G[((int64_t)a * m.J2 + x) * m.ldG + cc], S[2][cc], s2);
    }
    T1[a][x] = s1;
    T2[a][x] = s2;
  }
  __syncthreads();
  if (t < 32) {
    float d0 = 0.0f, d1 = 0.0f, d2 = 0.0f;
    for (int q = 0; q < 32; ++q) {
      d0 = fmaf(T1[t][q], S[2][q], d0);   // a = t: sum_c T1[a][c] S_C[c]
      d1 = fmaf(S[0][q], T2[q][t], d1);   // b = t: sum_a S_A[a] T2[a][b]
      d2 = fmaf(S[0][q], T1[q][t], d2);   // c = t: sum_a S_A[a] T1[a][c]
    }
    den[t] = t < m.J1 ? d0 : 0.0f;
    den[32 + t] = t < m.J2 ? d1 : 0.0f;
    den[64 + t] = t < m.J3 ? d2 : 0.0f;
  }
  for (int e = t; e < m.J1 * m.J2 * 32; e += 1024) {
    const int ab = e >> 5, cc = e & 31;
    const int a = ab / m.J2, b = ab % m.J2;
    dcore[e] = cc < m.J3 ? S[0][a] * S[1][b] * S[2][cc] : 0.0f;
  }
}

hipError_t launch_tk_den_closed(const TkModel& m, int I, int J, int K, float* den, float* dcore, hipStream_t s) {
  hipLaunchKernelGGL(tk_den_closed_kernel, dim3(1), dim3(1024), 0, s, m, I, J, K, den, dcore);
  return hipGetLastError();
}

}  // namespace comm

// ---------------------------------------------------------------------------------------- orchestration

using namespace comm;

namespace {

// Padded copies of a Tucker model: core [J1 J2][32], factors [I_n][32].
struct TkCopy {
  float* core;
  float* fac[3];
};

struct TkWs {
  int dims[3], J[3];
  TkGrid g;
  int Kp;
  float* V;
  float* m3[2];      // mode-3 partial slots of the numerator / denominator pass
  double* obj_part;
  float* U;
  float* H;
  float* slots[2];   // numerator / denominator split-K outputs
  size_t slot_floats;
  float* den_vec;    // [3][32]
  float* dcore;      // [J1 J2][32]
  TkCopy ref, cur, num, den, user_pad;
  float *Pc, *Qc;
  size_t bytes;
};

constexpr int kSplitCore = 8, kSplit1 = 4, kSplit2 = 16;

TkWs tk_layout(const comm_dense* x, const comm_model* m, char* base, bool cache) {
  TkWs w = {};
  for (int n = 0; n < 3; ++n) {
    w.dims[n] = (int)x->dims[n];
    w.J[n] = (int)m->core_dims[n];
  }
  const int I = w.dims[0], J = w.dims[1], K = w.dims[2];
  const int J1 = w.J[0], J2 = w.J[1];
  w.g = tk_grid(I, J);
  w.Kp = (K + 31) / 32 * 32;
  Carve cv;
  cv.base = base;
  w.V = cv.take<float>((size_t)I * J * kRP);
  w.m3[0] = cv.take<float>((size_t)w.g.wgs() * w.Kp * kRP);
  w.m3[1] = cv.take<float>((size_t)w.g.wgs() * w.Kp * kRP);
  w.obj_part = cv.take<double>((size_t)w.g.wgs());
  w.U = cv.take<float>((size_t)I * J2 * kRP);
  w.H = cv.take<float>((size_t)I * J2 * kRP);
  size_t s = (size_t)kSplitCore * J1 * J2 * kRP;
  s = std::max(s, (size_t)kSplit1 * I * kRP);
  s = std::max(s, (size_t)kSplit2 * J * kRP);
  w.slot_floats = s;
  w.slots[0] = cv.take<float>(s);
  w.slots[1] = cv.take<float>(s);
  w.den_vec = cv.take<float>(3 * kRP);
  w.dcore = cv.take<float>((size_t)J1 * J2 * kRP);
  for (TkCopy* c : {&w.ref, &w.cur, &w.num, &w.den, &w.user_pad}) {
    c->core = cv.take<float>((size_t)J1 * J2 * kRP);
    for (int n = 0; n < 3; ++n) c->fac[n] = cv.take<float>((size_t)w.dims[n] * kRP);
  }
  if (cache) {
    const size_t total = (size_t)I * J * K;
    w.Pc = cv.take<float>(total);
    w.Qc = cv.take<float>(total);
  }
  w.bytes = cv.off + 256;
  return w;
}

TkModel model_of(const TkWs& w, const TkCopy& c) {
  TkModel t;
  t.G = c.core;
  t.ldG = kRP;
  t.A = FView{c.fac[0], kRP, w.J[0]};
  t.B = FView{c.fac[1], kRP, w.J[1]};
  t.C = FView{c.fac[2], kRP, w.J[2]};
  t.J1 = w.J[0];
  t.J2 = w.J[1];
  t.J3 = w.J[2];
  return t;
}

// Copy the caller's model into padded buffers (and optionally a second copy).
int tk_pad(const comm_model* m, const TkWs& w, const TkCopy& dst, const TkCopy* dst2, hipStream_t st) {
  PadArgs p = {};
  p.nf = 1;
  p.cols = w.J[2];
  p.ld = w.J[2];
  p.src[0] = m->core;
  p.rows[0] = w.J[0] * w.J[1];
  p.rows_p[0] = p.rows[0];
  p.dst[0] = dst.core;
  p.dst2[0] = dst2 ? dst2->core : nullptr;
  HIP_TRY(launch_pad_factors(p, st));
  for (int n = 0; n < 3; ++n) {
    PadArgs q = {};
    q.nf = 1;
    q.cols = w.J[n];
    q.ld = w.J[n];
    q.src[0] = m->factors[n];
    q.rows[0] = w.dims[n];
    q.rows_p[0] = w.dims[n];
    q.dst[0] = dst.fac[n];
    q.dst2[0] = dst2 ? dst2->fac[n] : nullptr;
    HIP_TRY(launch_pad_factors(q, st));
  }
  return COMM_OK;
}

struct Slots {
  const float* part;
  int n;
  int rows_total;
};

// Numerator (use_q = 0) or denominator (use_q = 1) of block `blk` (-1 core,
// 0..2 factor) contracted against the set `cs`, from X rebuilt with `rb` or
// from the cached weight.  Returns the partial slots.
int tk_contract(comm_ctx* ctx, const comm_dense* x, const comm_opts* o, const TkWs& w, int blk, bool use_q,
                const TkModel& rb, const TkModel& cs, const float* cached, bool want_obj, float* slot_buf,
                Slots* out, hipStream_t st) {
  const int I = w.dims[0], J = w.dims[1], K = w.dims[2];
  const int J1 = w.J[0], J2 = w.J[1];
  TkPassArgs a = {};
  a.X = x->X;
  a.Wc = cached;
  a.I = I;
  a.J = J;
  a.K = K;
  a.Kp = w.Kp;
  a.r = rb;
  a.n = cs;
  a.eps = (float)o->eps;
  a.eps_x = (float)o->eps_x;
  a.use_q = use_q;
  a.want_v = blk != 2;
  a.want_m3 = blk == 2;
  a.bc = make_beta_const(o->beta);
  a.V = w.V;
  a.m3 = w.m3[use_q ? 1 : 0];
  a.obj_part = w.obj_part;
  const int mode = cached ? 1 : 0;
  const int bc = beta_class_of(o->beta);
  TkModel rb2 = rb;
  (void)rb2;
  int rc = profiled(ctx, st, [&] {
    TkPassArgs b = a;
    if (want_obj) b.obj_part = w.obj_part;
    return launch_tk_pass(b, w.g, bc, mode | (want_obj ? 4 : 0), st);
  });
  if (rc) return rc;
  if (blk == 2) {
    *out = Slots{a.m3, w.g.wgs(), w.Kp};
    return COMM_OK;
  }
  if (blk == -1 || blk == 0) {
    // U[i][b][c] = sum_j B'[j][b] V[i][j][c]
    GemmArgs g = {};
    g.A = cs.B.p;
    g.sab = 0; g.sam = 1; g.akin = 1 << 30; g.sako = 0; g.saki = cs.B.ld;
    g.B = w.V;
    g.sbb = (int64_t)J * kRP; g.bkin = 1 << 30; g.sbko = 0; g.sbki = kRP; g.sbn = 1;
    g.out = w.U;
    g.sob = (int64_t)J2 * kRP; g.sos = 0; g.ldo = kRP;
    g.M = J2; g.N = kRP; g.K = J; g.batch = I; g.splits = 1;
    HIP_TRY(launch_gemm(g, st));
  }
  if (blk == 0) {
    // Num1[i][a] = sum_{(b,c)} U[i][(b,c)] G'[a][(b,c)]
    GemmArgs g = {};
    g.A = w.U;
    g.sab = 0; g.sam = (int64_t)J2 * kRP; g.akin = 1 << 30; g.sako = 0; g.saki = 1;
    g.B = cs.G;
    g.sbb = 0; g.bkin = 1 << 30; g.sbko = 0; g.sbki = 1; g.sbn = (int64_t)J2 * kRP;
    g.out = slot_buf;
    g.sob = 0; g.sos = (int64_t)I * kRP; g.ldo = kRP;
    g.M = I; g.N = J1; g.K = J2 * kRP; g.batch = 1; g.splits = kSplit1;
    HIP_TRY(launch_gemm(g, st));
    *out = Slots{slot_buf, kSplit1, I};
  } else if (blk == -1) {
    // Ncore[a][(b,c)] = sum_i A'[i][a] U[i][(b,c)]
    GemmArgs g = {};
    g.A = cs.A.p;
    g.sab = 0; g.sam = 1; g.akin = 1 << 30; g.sako = 0; g.saki = cs.A.ld;
    g.B = w.U;
    g.sbb = 0; g.bkin = 1 << 30; g.sbko = 0; g.sbki = (int64_t)J2 * kRP; g.sbn = 1;
    g.out = slot_buf;
    g.sob = 0; g.sos = (int64_t)J1 * J2 * kRP; g.ldo = (int64_t)J2 * kRP;
    g.M = J1; g.N = J2 * kRP; g.K = I; g.batch = 1; g.splits = kSplitCore;
    HIP_TRY(launch_gemm(g, st));
    *out = Slots{slot_buf, kSplitCore, J1 * J2};
  } else {
    // H[i][(b,c)] = sum_a A'[i][a] G'[a][(b,c)];  Num2[j][b] = sum_{(i,c)} V[i][j][c] H[i][b][c]
    GemmArgs g = {};
    g.A = cs.A.p;
    g.sab = 0; g.sam = cs.A.ld; g.akin = 1 << 30; g.sako = 0; g.saki = 1;
    g.B = cs.G;
    g.sbb = 0; g.bkin = 1 << 30; g.sbko = 0; g.sbki = (int64_t)J2 * kRP; g.sbn = 1;
    g.out = w.H;
    g.sob = 0; g.sos = 0; g.ldo = (int64_t)J2 * kRP;
    g.M = I; g.N = J2 * kRP; g.K = J1; g.batch = 1; g.splits = 1;
    HIP_TRY(launch_gemm(g, st));
    GemmArgs h = {};
    h.A = w.V;
    h.sab = 0; h.sam = kRP; h.akin = kRP; h.sako = (int64_t)J * kRP; h.saki = 1;
    h.B = w.H;
    h.sbb = 0; h.bkin = kRP; h.sbko = (int64_t)J2 * kRP; h.sbki = 1; h.sbn = kRP;
    h.out = slot_buf;
    h.sob = 0; h.sos = (int64_t)J * kRP; h.ldo = kRP;
    h.M = J; h.N = J2; h.K = I * kRP; h.batch = 1; h.splits = kSplit2;
    HIP_TRY(launch_gemm(h, st));
    *out = Slots{slot_buf, kSplit2, J};
  }
  return COMM_OK;
}

// One block update: max(anchor * (Num/Den)^gamma, eps) into the caller's
// block (and a padded copy).  blk -1 = core.
int tk_apply(const comm_model* m, const TkWs& w, int blk, const Slots& num, const Slots* den,
             const float* den_closed_vec, FView anchor, float* out_pad, float gamma, float eps, hipStream_t st) {
  SlotUpdateArgs u = {};
  u.njobs = 1;
  SlotJob& Jb = u.job[0];
  Jb.mode = kSlotUpdate;
  Jb.num_part = num.part;
  Jb.num_slots = num.n;
  Jb.rows_total = num.rows_total;
  if (den) {
    Jb.den_part = den->part;
    Jb.den_slots = den->n;
  } else {
    Jb.den_closed = den_closed_vec;
  }
  if (blk == -1) {
    Jb.rows = w.J[0] * w.J[1];
    Jb.cols = w.J[2];
    Jb.out_user = m->core;
    Jb.ld_user = w.J[2];
  } else {
    Jb.rows = w.dims[blk];
    Jb.cols = w.J[blk];
    Jb.out_user = m->factors[blk];
    Jb.ld_user = w.J[blk];
  }
  Jb.rows_p = Jb.rows;
  Jb.anchor = anchor;
  Jb.gamma = gamma;
  Jb.eps = eps;
  Jb.out_pad = out_pad;
  HIP_TRY(launch_slot_update(u, st));
  return COMM_OK;
}

FView block_view(const TkModel& t, int blk) {
  if (blk == -1) return FView{t.G, t.ldG, t.J3};
  return blk == 0 ? t.A : blk == 1 ? t.B : t.C;
}

float* copy_block(const TkCopy& c, int blk) { return blk == -1 ? c.core : c.fac[blk]; }

// Denominator of block `blk` at beta = 1 from the denominator set: a
// per-column vector for factors, the full dcore for the core (as one slot).
int tk_closed_den(const TkWs& w, int blk, const TkModel& ds, Slots* core_den, const float** vec, hipStream_t st) {
  HIP_TRY(launch_tk_den_closed(ds, w.dims[0], w.dims[1], w.dims[2], w.den_vec, w.dcore, st));
  if (blk == -1) {
    *core_den = Slots{w.dcore, 1, w.J[0] * w.J[1]};
    *vec = nullptr;
  } else {
    *vec = w.den_vec + blk * kRP;
  }
  return COMM_OK;
}

int tk_block(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, const TkWs& w, int blk,
             const TkModel& rb, const TkModel& ns, const TkModel& ds, const float* cacheP, const float* cacheQ,
             bool want_obj, FView anchor, float* out_pad, double* obj, hipStream_t st) {
  const bool kl = o->beta == 1.0;
  Slots num, den;
  int rc = tk_contract(ctx, x, o, w, blk, false, rb, ns, cacheP, want_obj, w.slots[0], &num, st);
  if (rc) return rc;
  if (want_obj && obj) HIP_TRY(launch_sum_f64(w.obj_part, w.g.wgs(), nullptr, obj, st));
  const float* vec = nullptr;
  Slots* denp = &den;
  if (kl) {
    if ((rc = tk_closed_den(w, blk, ds, &den, &vec, st))) return rc;
    if (blk != -1) denp = nullptr;
  } else {
    if ((rc = tk_contract(ctx, x, o, w, blk, true, rb, ds, cacheQ, false, w.slots[1], &den, st))) return rc;
  }
  return tk_apply(m, w, blk, num, denp, vec, anchor, out_pad, gamma_of(o->beta), (float)o->eps, st);
}

}  // namespace

int tucker_check_model(const comm_model* m, const comm_dense* x) {
  if (!m) return fail(COMM_EINVAL, "model is NULL");
  if (m->kind != COMM_TUCKER) return fail(COMM_EINVAL, "model kind is not Tucker");
  if (!m->core) return fail(COMM_EINVAL, "core is NULL");
  for (int n = 0; n < x->ndim; ++n) {
    if (!m->factors[n]) return fail(COMM_EINVAL, "factors[%d] is NULL", n);
    if (m->core_dims[n] < 1) return fail(COMM_EINVAL, "core_dims[%d] = %lld", n, (long long)m->core_dims[n]);
    if (m->core_dims[n] > kRP) return fail(COMM_EUNSUPPORTED, "core_dims[%d] > %d not supported", n, kRP);
  }
  return COMM_OK;
}

size_t tucker_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op) {
  const bool cache = op == 1 && o->cache_pq;
  return tk_layout(x, m, nullptr, cache).bytes;
}

int tucker_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st) {
  TkWs w = tk_layout(x, m, nullptr, false);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tk_layout(x, m, ctx->ws, false);
  // The current model lives in the caller's buffers; kernels read a padded
  // copy that is refreshed after each block update.
  if ((rc = tk_pad(m, w, w.cur, nullptr, st))) return rc;
  const TkModel cur = model_of(w, w.cur);
  std::vector<int> blocks;
  if (block == -2) blocks = {-1, 0, 1, 2};
  else blocks = {block};
  for (int blk : blocks) {
    rc = tk_block(ctx, x, m, o, w, blk, cur, cur, cur, nullptr, nullptr, false, block_view(cur, blk),
                  copy_block(w.cur, blk), nullptr, st);
    if (rc) return rc;
  }
  return COMM_OK;
}

int tucker_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st) {
  const bool cache = o->cache_pq && o->beta != 1.0;
  TkWs w = tk_layout(x, m, nullptr, cache);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tk_layout(x, m, ctx->ws, cache);
  if ((rc = tk_pad(m, w, w.ref, &w.cur, st))) return rc;
  const TkModel ref = model_of(w, w.ref);
  const TkModel cur = model_of(w, w.cur);
  bool obj_pending = obj != nullptr;
  if (cache) {
    TkPassArgs a = {};
    a.X = x->X;
    a.Pw = w.Pc;
    a.Qw = w.Qc;
    a.I = w.dims[0];
    a.J = w.dims[1];
    a.K = w.dims[2];
    a.Kp = w.Kp;
    a.r = ref;
    a.n = ref;
    a.eps = (float)o->eps;
    a.eps_x = (float)o->eps_x;
    a.bc = make_beta_const(o->beta);
    a.obj_part = w.obj_part;
    rc = profiled(ctx, st, [&] { return launch_tk_pass(a, w.g, beta_class_of(o->beta), 2 | (obj_pending ? 4 : 0), st); });
    if (rc) return rc;
    if (obj_pending) HIP_TRY(launch_sum_f64(w.obj_part, w.g.wgs(), nullptr, obj, st));
    obj_pending = false;
  }
  const float beta = (float)o->beta;
  for (int l = 0; l < o->inner_sweeps; ++l) {
    for (int blk : {-1, 0, 1, 2}) {
      // transformed blocks from the current inner iterate (Sec. 5.3, App. C.3)
      ChiArgs ca = {};
      ca.beta = beta;
      auto add = [&](const float* curp, const float* refp, int rows, float* x1, float* x2) {
        const int f = ca.nf++;
        ca.cur[f] = curp;
        ca.ref[f] = refp;
        ca.rows_p[f] = rows;
        ca.x1[f] = x1;
        ca.x2[f] = x2;
      };
      if (blk != -1) add(w.cur.core, w.ref.core, w.J[0] * w.J[1], w.num.core, w.den.core);
      for (int q = 0; q < 3; ++q)
        if (q != blk) add(w.cur.fac[q], w.ref.fac[q], w.dims[q], w.num.fac[q], w.den.fac[q]);
      HIP_TRY(launch_chi(ca, st));
      TkModel ns = model_of(w, w.num), ds = model_of(w, w.den);
      // the active block does not enter its own contraction
      if (blk == -1) { ns.G = ref.G; ds.G = ref.G; }
      else if (blk == 0) { ns.A = ref.A; ds.A = ref.A; }
      else if (blk == 1) { ns.B = ref.B; ds.B = ref.B; }
      else { ns.C = ref.C; ds.C = ref.C; }
      rc = tk_block(ctx, x, m, o, w, blk, ref, ns, ds, cache ? w.Pc : nullptr, cache ? w.Qc : nullptr, obj_pending,
                    block_view(ref, blk), copy_block(w.cur, blk), obj, st);
      if (rc) return rc;
      obj_pending = false;
    }
  }
  (void)cur;
  return COMM_OK;
}

int tucker_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                     hipStream_t st) {
  TkWs w = tk_layout(x, m, nullptr, false);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tk_layout(x, m, ctx->ws, false);
  if ((rc = tk_pad(m, w, w.cur, nullptr, st))) return rc;
  const TkModel cur = model_of(w, w.cur);
  TkPassArgs a = {};
  a.X = x->X;
  a.I = w.dims[0];
  a.J = w.dims[1];
  a.K = w.dims[2];
  a.Kp = w.Kp;
  a.r = cur;
  a.n = cur;
  a.eps = (float)o->eps;
  a.eps_x = (float)o->eps_x;
  a.bc = make_beta_const(o->beta);
  a.V = w.V;
  a.m3 = w.m3[0];
  a.obj_part = w.obj_part;
  rc = profiled(ctx, st, [&] { return launch_tk_pass(a, w.g, beta_class_of(o->beta), 0 | 4, st); });
  if (rc) return rc;
  HIP_TRY(launch_sum_f64(w.obj_part, w.g.wgs(), nullptr, out, st));
  return COMM_OK;
}
