// Dense order-4 Tucker (Sec. 4.3, App. C and Sec. 5.3 for N = 4): B-CoMM,
// J-CoMM and the objective.
//
// The two fused Tucker passes of the order-3 path run unchanged on the
// (I1 I2 I3) x I4 matrix view of X: a row is the mode-4 fibre of a triple
// (i1, i2, i3), rebuilt from
//   T3[(i1,i2,i3)][d] = sum_{a,b,c} A1[i1][a] A2[i2][b] A3[i3][c] G[a][b][c][d]
// (three mode products of the core) and the mode-4 factor.  With
// V[(i1,i2,i3)][d] = sum_{i4} W[(i1,i2,i3)][i4] A4'[i4][d] from the V pass
// (W = P or Q), the other numerators are mode products of V followed by one
// contraction with the core G' of the contraction set:
//   core   : Ncore = V x3 A3'^T x2 A2'^T x1 A1'^T
//   mode 1 : Num1[i1][a] = sum_{b,c,d} (V x3 A3'^T x2 A2'^T)[i1][b][c][d] G'[a][b][c][d]
//   mode 2 : Num2[i2][b] = sum_a sum_{c,d} (V x1 A1'^T x3 A3'^T)[a][i2][c][d] G'[a][b][c][d]
//   mode 3 : Num3[i3][c] = sum_{a,b,d} (V x1 A1'^T x2 A2'^T)[a][b][i3][d] G'[a][b][c][d]
// and the mode-4 numerator is the mode-3 pass of the order-3 path on the same
// view, against T3 of the contraction set.  Mode products are strided batched
// matrix-core GEMMs (launch_gemm); the partial tensor of each mode is never
// formed, only V and the small products of it.

#include <algorithm>

#include "host_util.h"
#include "kernels.h"
#include "tucker3.h"

namespace comm {

// [rows][32] -> [32][rows_p], zero for rows >= rows.
__global__ void __launch_bounds__(256) rows32_transpose_kernel(const float* __restrict__ in, int64_t rows,
                                                               int64_t rows_p, float* __restrict__ out) {
  __shared__ float tile[64][33];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int t = threadIdx.x;
  for (int e = t; e < 64 * 32; e += 256) {
    const int r = e >> 5, c = e & 31;
    tile[r][c] = r0 + r < rows ? in[(r0 + r) * kRP + c] : 0.0f;
  }
  __syncthreads();
  for (int e = t; e < 64 * 32; e += 256) {
    const int c = e >> 6, r = e & 63;
    if (r0 + r < rows_p) out[(int64_t)c * rows_p + r0 + r] = tile[r][c];
  }
}

// An order-4 Tucker model as the kernels see it: core entry (a, b, c, d) at
// G[((a J2 + b) J3 + c) * 32 + d]; factor views with cols = J_n.
struct Tk4Model {
  const float* G;
  FView F[4];
  int J[4];
  int rows[4];
};

// Closed-form beta = 1 denominators (Q = 1) from the column sums S_m of the
// denominator set's factors: den[n][j] = sum over the core entries with
// j_n = j of G * prod_{m != n} S_m[j_m], and dcore[(a,b,c)][d] =
// S_1[a] S_2[b] S_3[c] S_4[d].  One workgroup, fixed order.
__global__ void __launch_bounds__(1024) tk4_den_closed_kernel(Tk4Model m, float* den, float* dcore) {
  __shared__ float red[32][33];
  __shared__ float S[4][32];
  const int t = threadIdx.x;
  const int c = t & 31, g = t >> 5;
  for (int f = 0; f < 4; ++f) {
    float s = 0.0f;
    for (int r = g; r < m.rows[f]; r += 32) s += m.F[f].at(r, c, m.rows[f]);
    red[g][c] = s;
    __syncthreads();
    if (t < 32) {
      float acc = 0.0f;
      for (int q = 0; q < 32; ++q) acc += red[q][t];
      S[f][t] = acc;
    }
    __syncthreads();
  }
  if (t < 128) {
    const int n = t >> 5, j = t & 31;
    float acc = 0.0f;
    if (j < m.J[n]) {
      // the three other modes, in increasing order
      int o[3], k = 0;
      for (int q = 0; q < 4; ++q)
        if (q != n) o[k++] = q;
      int idx[4];
      idx[n] = j;
      for (int x0 = 0; x0 < m.J[o[0]]; ++x0) {
        idx[o[0]] = x0;
        for (int x1 = 0; x1 < m.J[o[1]]; ++x1) {
          idx[o[1]] = x1;
          for (int x2 = 0; x2 < m.J[o[2]]; ++x2) {
            idx[o[2]] = x2;
            const int64_t e = (((int64_t)idx[0] * m.J[1] + idx[1]) * m.J[2] + idx[2]) * kRP + idx[3];
            acc += m.G[e] * (S[o[0]][x0] * S[o[1]][x1] * S[o[2]][x2]);
          }
        }
      }
    }
    den[n * kRP + j] = acc;
  }
  const int64_t total = (int64_t)m.J[0] * m.J[1] * m.J[2] * kRP;
  for (int64_t e = t; e < total; e += 1024) {
    const int d = (int)(e & 31);
    const int64_t abc = e >> 5;
    const int cc = (int)(abc % m.J[2]);
    const int b = (int)((abc / m.J[2]) % m.J[1]);
    const int a = (int)(abc / ((int64_t)m.J[2] * m.J[1]));
    dcore[e] = d < m.J[3] ? S[0][a] * S[1][b] * S[2][cc] * S[3][d] : 0.0f;
  }
}

namespace {

struct Tk4Copy {
  float* core;     // [J1 J2 J3][32]
  float* fac[4];   // [I_n][32]; mode 4 [Kp][32]
  float* facT4;    // mode 4 transposed [32][Kp]
};

constexpr int kSplitCore4 = 8, kSplit14 = 8, kSplit34 = 32;

struct Tk4Ws {
  int dims[4], J[4];
  int np;                  // triples I1 I2 I3
  int64_t Pp;              // np rounded up to 32
  int Kp, tpw, npg;
  int64_t vwgs;
  float* T3r;              // rebuild table [np][32]
  float* T3T[2];           // the contraction sets' tables, transposed [32][Pp]
  float* V[2];             // V pass outputs [np][32]; scratch for the sets' tables
  float* m3[2];            // mode-4 partial slots [npg][Kp][32]
  double* obj_part;
  float* Y1[2];            // T3 chain: [J1 J2][I3][32], [J1][I2][I3][32]
  float* Y2[2];
  float* W3[2];            // [I1 I2][J3][32]
  float* W23[2];           // [I1][J2][J3][32]
  float* Z1[2];            // [J1][I2][I3][32]
  float* Z2[2];            // [J1][I2][J3][32]
  float* Z3[2];            // [J1][J2][I3][32]
  float* slots[2];
  float* den_vec;          // [4][32]
  float* dcore;            // [J1 J2 J3][32]
  Tk4Copy ref, cur, num, den;
  float *Pc, *Qc;
  size_t bytes;
};

Tk4Ws tk4_layout(const comm_dense* x, const comm_model* m, char* base, bool cache) {
  Tk4Ws w = {};
  for (int n = 0; n < 4; ++n) {
    w.dims[n] = (int)x->dims[n];
    w.J[n] = (int)m->core_dims[n];
  }
  const int I1 = w.dims[0], I2 = w.dims[1], I3 = w.dims[2], I4 = w.dims[3];
  const int J1 = w.J[0], J2 = w.J[1], J3 = w.J[2];
  w.np = I1 * I2 * I3;
  w.Pp = ((int64_t)w.np + 31) / 32 * 32;
  w.Kp = (I4 + 31) / 32 * 32;
  tk_m3_tiling(w.np, 1, &w.tpw, &w.npg);
  w.vwgs = tk_v_workgroups(w.np, 1);
  const size_t core = (size_t)J1 * J2 * J3 * kRP;
  Carve cv;
  cv.base = base;
  w.T3r = cv.take<float>((size_t)w.np * kRP);
  for (int k = 0; k < 2; ++k) {
    w.T3T[k] = cv.take<float>((size_t)w.Pp * kRP);
    w.V[k] = cv.take<float>((size_t)w.np * kRP);
    w.m3[k] = cv.take<float>((size_t)w.npg * w.Kp * kRP);
    w.Y1[k] = cv.take<float>((size_t)J1 * J2 * I3 * kRP);
    w.Y2[k] = cv.take<float>((size_t)J1 * I2 * I3 * kRP);
    w.W3[k] = cv.take<float>((size_t)I1 * I2 * J3 * kRP);
    w.W23[k] = cv.take<float>((size_t)I1 * J2 * J3 * kRP);
    w.Z1[k] = cv.take<float>((size_t)J1 * I2 * I3 * kRP);
    w.Z2[k] = cv.take<float>((size_t)J1 * I2 * J3 * kRP);
    w.Z3[k] = cv.take<float>((size_t)J1 * J2 * I3 * kRP);
  }
  w.obj_part = cv.take<double>((size_t)w.vwgs);
  size_t s = (size_t)kSplitCore4 * core;
  s = std::max(s, (size_t)kSplit14 * I1 * kRP);
  s = std::max(s, (size_t)J1 * I2 * kRP);
  s = std::max(s, (size_t)kSplit34 * I3 * kRP);
  w.slots[0] = cv.take<float>(s);
  w.slots[1] = cv.take<float>(s);
  w.den_vec = cv.take<float>(4 * kRP);
  w.dcore = cv.take<float>(core);
  for (Tk4Copy* c : {&w.ref, &w.cur, &w.num, &w.den}) {
    c->core = cv.take<float>(core);
    for (int n = 0; n < 3; ++n) c->fac[n] = cv.take<float>((size_t)w.dims[n] * kRP);
    c->fac[3] = cv.take<float>((size_t)w.Kp * kRP);
    c->facT4 = cv.take<float>((size_t)w.Kp * kRP);
  }
  if (cache) {
    const size_t total = (size_t)w.np * I4;
    w.Pc = cv.take<float>(total);
    w.Qc = cv.take<float>(total);
  }
  w.bytes = cv.off + 256;
  return w;
}

Tk4Model model4(const Tk4Ws& w, const Tk4Copy& c) {
  Tk4Model t;
  t.G = c.core;
  for (int n = 0; n < 4; ++n) {
    t.F[n] = FView{c.fac[n], kRP, w.J[n]};
    t.J[n] = w.J[n];
    t.rows[n] = w.dims[n];
  }
  return t;
}

// Caller's model into padded copies (and a second one), one launch.
int tk4_pad(const comm_model* m, const Tk4Ws& w, const Tk4Copy& dst, const Tk4Copy* dst2, hipStream_t st) {
  PadArgs p = {};
  p.nf = 5;
  p.cols[0] = w.J[3];
  p.ld[0] = w.J[3];
  p.src[0] = m->core;
  p.rows[0] = w.J[0] * w.J[1] * w.J[2];
  p.rows_p[0] = p.rows[0];
  p.dst[0] = dst.core;
  p.dst2[0] = dst2 ? dst2->core : nullptr;
  for (int n = 0; n < 4; ++n) {
    const int f = n + 1;
    p.cols[f] = w.J[n];
    p.ld[f] = w.J[n];
    p.src[f] = m->factors[n];
    p.rows[f] = w.dims[n];
    p.rows_p[f] = n == 3 ? w.Kp : w.dims[n];
    p.dst[f] = dst.fac[n];
    p.dst2[f] = dst2 ? dst2->fac[n] : nullptr;
    if (n == 3) {
      p.dstT[f] = dst.facT4;
      p.dst2T[f] = dst2 ? dst2->facT4 : nullptr;
    }
  }
  HIP_TRY(launch_pad_factors(p, st));
  return COMM_OK;
}

// Mode product of T viewed as L x I x R, for `sets` operand pairs at once:
// Y[l][j][r] = sum_{i < I} M(i, j) T[l][i][r].  contract: M(i, j) = F[i][j]
// (F a padded [I][32] factor, the sum runs over data rows: T x_n F^T);
// expand: M(i, j) = F[j][i] (F a padded [J][32] factor, the sum runs over a
// core index: T x_n F).
int mode_product(const float* const* F, const float* const* T, float* const* Y, int sets, int64_t L, int I, int J,
                 int64_t R, bool contract, hipStream_t st) {
  GemmArgs g = {};
  g.sab = 0;
  g.sam = contract ? 1 : kRP;
  g.sako = 0;
  g.saki = contract ? kRP : 1;
  g.akin_log2 = 30;
  g.sbb = (int64_t)I * R;
  g.sbko = 0;
  g.sbki = R;
  g.sbn = 1;
  g.bkin_log2 = 30;
  g.sob = (int64_t)J * R;
  g.sos = 0;
  g.ldo = R;
  g.M = J;
  g.N = (int)R;
  g.K = I;
  g.batch = (int)L;
  g.splits = 1;
  g.sets = sets;
  for (int k = 0; k < sets; ++k) {
    g.A[k] = F[k];
    g.B[k] = T[k];
    g.out[k] = Y[k];
  }
  HIP_TRY(launch_gemm(g, st));
  return COMM_OK;
}

// T3 of `sets` models into out[k] ([np][32]).
int tk4_t3(const Tk4Ws& w, const Tk4Model* md, int sets, float* const* out, hipStream_t st) {
  const int I1 = w.dims[0], I2 = w.dims[1], I3 = w.dims[2];
  const int J1 = w.J[0], J2 = w.J[1], J3 = w.J[2];
  const float *F[2], *T[2];
  int rc;
  // Y1[(a,b)][i3][d] = sum_c A3[i3][c] G[(a,b)][c][d]
  for (int k = 0; k < sets; ++k) {
    F[k] = md[k].F[2].p;
    T[k] = md[k].G;
  }
  if ((rc = mode_product(F, T, w.Y1, sets, (int64_t)J1 * J2, J3, I3, kRP, false, st))) return rc;
  // Y2[a][i2][(i3,d)] = sum_b A2[i2][b] Y1[a][b][(i3,d)]
  for (int k = 0; k < sets; ++k) {
    F[k] = md[k].F[1].p;
    T[k] = w.Y1[k];
  }
  if ((rc = mode_product(F, T, w.Y2, sets, J1, J2, I2, (int64_t)I3 * kRP, false, st))) return rc;
  // T3[i1][(i2,i3,d)] = sum_a A1[i1][a] Y2[a][(i2,i3,d)]
  for (int k = 0; k < sets; ++k) {
    F[k] = md[k].F[0].p;
    T[k] = w.Y2[k];
  }
  return mode_product(F, T, out, sets, 1, J1, I1, (int64_t)I2 * I3 * kRP, false, st);
}

int tk4_transpose(const Tk4Ws& w, const float* in, float* out, hipStream_t st) {
  hipLaunchKernelGGL(rows32_transpose_kernel, dim3((unsigned)((w.Pp + 63) / 64)), dim3(256), 0, st, in,
                     (int64_t)w.np, w.Pp, out);
  HIP_TRY(hipGetLastError());
  return COMM_OK;
}

struct Slots4 {
  const float* part;
  int n;
  int rows_total;
};

// Numerator slots of block blk (-1 core, 0..2) from V[k] of the contraction
// sets cs[k] (k < sets; set 1 is the denominator's).
int tk4_gemms(const Tk4Ws& w, int blk, const Tk4Model* cs, int sets, Slots4* out, hipStream_t st) {
  const int I1 = w.dims[0], I2 = w.dims[1], I3 = w.dims[2];
  const int J1 = w.J[0], J2 = w.J[1], J3 = w.J[2];
  const int64_t core_row = (int64_t)J2 * J3 * kRP;  // one a-slice of the padded core
  const float *F[2], *T[2];
  int rc;
  auto fac = [&](int n) {
    for (int k = 0; k < sets; ++k) F[k] = cs[k].F[n].p;
  };
  auto src = [&](float* const* from) {
    for (int k = 0; k < sets; ++k) T[k] = from[k];
  };
  auto gemm = [&](GemmArgs g, const float* const* A, const float* const* B, int splits, int rows) -> int {
    g.sets = sets;
    for (int k = 0; k < sets; ++k) {
      g.A[k] = A[k];
      g.B[k] = B[k];
      g.out[k] = w.slots[k];
      out[k] = Slots4{w.slots[k], splits, rows};
    }
    HIP_TRY(launch_gemm(g, st));
    return COMM_OK;
  };
  const float* Gs[2] = {cs[0].G, sets > 1 ? cs[1].G : nullptr};
  if (blk == -1 || blk == 0) {
    // W3 = V x3 A3'^T, W23 = W3 x2 A2'^T
    fac(2);
    src(w.V);
    if ((rc = mode_product(F, T, w.W3, sets, (int64_t)I1 * I2, I3, J3, kRP, true, st))) return rc;
    fac(1);
    src(w.W3);
    if ((rc = mode_product(F, T, w.W23, sets, I1, I2, J2, (int64_t)J3 * kRP, true, st))) return rc;
    GemmArgs g = {};
    g.akin_log2 = 30;
    g.bkin_log2 = 30;
    g.batch = 1;
    if (blk == -1) {
      // Ncore[a][(b,c,d)] = sum_i1 A1'[i1][a] W23[i1][(b,c,d)]
      g.sam = 1; g.saki = kRP;
      g.sbki = core_row; g.sbn = 1;
      g.sos = (int64_t)J1 * core_row; g.ldo = core_row;
      g.M = J1; g.N = (int)core_row; g.K = I1; g.splits = kSplitCore4;
      const float* A[2] = {cs[0].F[0].p, sets > 1 ? cs[1].F[0].p : nullptr};
      const float* B[2] = {w.W23[0], w.W23[1]};
      return gemm(g, A, B, kSplitCore4, J1 * J2 * J3);
    }
    // Num1[i1][a] = sum_{(b,c,d)} W23[i1][(b,c,d)] G'[a][(b,c,d)]
    g.sam = core_row; g.saki = 1;
    g.sbki = 1; g.sbn = core_row;
    g.sos = (int64_t)I1 * kRP; g.ldo = kRP;
    g.M = I1; g.N = J1; g.K = (int)core_row; g.splits = kSplit14;
    const float* A[2] = {w.W23[0], w.W23[1]};
    return gemm(g, A, Gs, kSplit14, I1);
  }
  // Z1 = V x1 A1'^T
  fac(0);
  src(w.V);
  if ((rc = mode_product(F, T, w.Z1, sets, 1, I1, J1, (int64_t)I2 * I3 * kRP, true, st))) return rc;
  GemmArgs g = {};
  g.akin_log2 = 30;
  g.bkin_log2 = 30;
  if (blk == 1) {
    // Z2 = Z1 x3 A3'^T; slot a of Num2: sum_{(c,d)} Z2[a][i2][(c,d)] G'[a][b][(c,d)]
    fac(2);
    src(w.Z1);
    if ((rc = mode_product(F, T, w.Z2, sets, (int64_t)J1 * I2, I3, J3, kRP, true, st))) return rc;
    g.sab = (int64_t)I2 * J3 * kRP; g.sam = (int64_t)J3 * kRP; g.saki = 1;
    g.sbb = core_row; g.sbki = 1; g.sbn = (int64_t)J3 * kRP;
    g.sob = (int64_t)I2 * kRP; g.ldo = kRP;
    g.M = I2; g.N = J2; g.K = J3 * kRP; g.batch = J1; g.splits = 1;
    const float* A[2] = {w.Z2[0], w.Z2[1]};
    return gemm(g, A, Gs, J1, I2);
  }
  // Z3 = Z1 x2 A2'^T; Num3[i3][c] = sum_{(a,b)} sum_d Z3[(a,b)][i3][d] G'[(a,b)][c][d]
  fac(1);
  src(w.Z1);
  if ((rc = mode_product(F, T, w.Z3, sets, J1, I2, J2, (int64_t)I3 * kRP, true, st))) return rc;
  g.sam = kRP; g.sako = (int64_t)I3 * kRP; g.saki = 1; g.akin_log2 = 5;
  g.sbko = (int64_t)J3 * kRP; g.sbki = 1; g.sbn = kRP; g.bkin_log2 = 5;
  g.sos = (int64_t)I3 * kRP; g.ldo = kRP;
  g.M = I3; g.N = J3; g.K = J1 * J2 * kRP; g.batch = 1; g.splits = kSplit34;
  const float* A[2] = {w.Z3[0], w.Z3[1]};
  return gemm(g, A, Gs, kSplit34, I3);
}

TkPassArgs pass4_args(const comm_dense* x, const comm_opts* o, const Tk4Ws& w) {
  TkPassArgs a = {};
  a.X = x->X;
  a.I = w.np;
  a.J = 1;
  a.K = w.dims[3];
  a.Kp = w.Kp;
  a.eps = (float)o->eps;
  a.eps_x = (float)o->eps_x;
  a.bc = make_beta_const(o->beta);
  a.Vn = w.V[0];
  a.Vd = w.V[1];
  a.m3n = w.m3[0];
  a.m3d = w.m3[1];
  a.obj_part = w.obj_part;
  a.tpw = w.tpw;
  a.npg = w.npg;
  a.Pp = w.Pp;
  a.xvec = (w.dims[3] % 4 == 0) && (reinterpret_cast<uintptr_t>(x->X) % 16 == 0);
  a.bf16 = o->precision == COMM_BF16;
  return a;
}

FView block_view4(const Tk4Model& t, int blk) {
  if (blk == -1) return FView{t.G, kRP, t.J[3]};
  return t.F[blk];
}

float* copy_block4(const Tk4Copy& c, int blk) { return blk == -1 ? c.core : c.fac[blk]; }

// One block update: max(anchor * (Num/Den)^gamma, eps) into the caller's block
// and the padded copy `pad` (mode 4 also its transposed copy).
int tk4_apply(const comm_model* m, const Tk4Ws& w, int blk, const Slots4& num, const Slots4* den,
              const float* den_closed_vec, FView anchor, const Tk4Copy& pad, float gamma, float eps,
              hipStream_t st) {
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
    Jb.rows = w.J[0] * w.J[1] * w.J[2];
    Jb.cols = w.J[3];
    Jb.out_user = m->core;
    Jb.ld_user = w.J[3];
  } else {
    Jb.rows = w.dims[blk];
    Jb.cols = w.J[blk];
    Jb.out_user = m->factors[blk];
    Jb.ld_user = w.J[blk];
  }
  Jb.rows_p = blk == 3 ? w.Kp : Jb.rows;
  Jb.anchor = anchor;
  Jb.gamma = gamma;
  Jb.eps = eps;
  Jb.out_pad = copy_block4(pad, blk);
  Jb.out_padT = blk == 3 ? pad.facT4 : nullptr;
  HIP_TRY(launch_slot_update(u, st));
  return COMM_OK;
}

// Update of block blk with X rebuilt from T3r and the mode-4 factor c4 (or
// read from the cached P~ / Q~), contraction sets ns / ds (their mode-4
// factors transposed in cnT / cdT; for blk = 3 their tables in w.T3T).
int tk4_block(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, const Tk4Ws& w, int blk,
              FView c4, const Tk4Model& ns, const Tk4Model& ds, const float* cnT, const float* cdT, bool cached,
              bool want_obj, FView anchor, const Tk4Copy& pad, double* obj, hipStream_t st) {
  const bool kl = o->beta == 1.0;
  const int sets = kl ? 1 : 2;
  const int bc = beta_class_of(o->beta);
  const int mode = cached ? kTkCacheRead : kTkFromX;
  TkPassArgs a = pass4_args(x, o, w);
  a.T2r = w.T3r;
  a.C = c4;
  if (cached) {
    a.Pc = w.Pc;
    a.Qc = w.Qc;
  }
  Slots4 num, den;
  int rc;
  if (blk == 3) {
    a.T2nT = w.T3T[0];
    a.T2dT = w.T3T[1];
    rc = profiled(ctx, st, [&] { return launch_tk_m3(a, bc, mode, sets, st); });
    if (rc) return rc;
    num = Slots4{w.m3[0], w.npg, w.Kp};
    den = Slots4{w.m3[1], w.npg, w.Kp};
  } else {
    a.CnT = cnT;
    a.CdT = cdT;
    rc = profiled(ctx, st, [&] { return launch_tk_v(a, bc, mode, want_obj, sets, st); });
    if (rc) return rc;
    if (want_obj && obj) HIP_TRY(launch_sum_f64(w.obj_part, w.vwgs, nullptr, obj, st));
    const Tk4Model cs[2] = {ns, ds};
    Slots4 nd[2];
    if ((rc = tk4_gemms(w, blk, cs, sets, nd, st))) return rc;
    num = nd[0];
    den = nd[1];
  }
  const float* vec = nullptr;
  const Slots4* denp = &den;
  Slots4 dcore;
  if (kl) {
    hipLaunchKernelGGL(tk4_den_closed_kernel, dim3(1), dim3(1024), 0, st, ds, w.den_vec, w.dcore);
    HIP_TRY(hipGetLastError());
    if (blk == -1) {
      dcore = Slots4{w.dcore, 1, w.J[0] * w.J[1] * w.J[2]};
      denp = &dcore;
    } else {
      vec = w.den_vec + blk * kRP;
      denp = nullptr;
    }
  }
  return tk4_apply(m, w, blk, num, denp, vec, anchor, pad, gamma_of(o->beta), (float)o->eps, st);
}

}  // namespace
}  // namespace comm

using namespace comm;

size_t tucker4_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op) {
  const bool cache = op == 1 && o->cache_pq && o->beta != 1.0;
  return tk4_layout(x, m, nullptr, cache).bytes;
}

int tucker4_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o,
                  hipStream_t st) {
  Tk4Ws w = tk4_layout(x, m, nullptr, false);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tk4_layout(x, m, ctx->ws, false);
  if ((rc = tk4_pad(m, w, w.cur, nullptr, st))) return rc;
  const Tk4Model cur = model4(w, w.cur);
  const int all[5] = {-1, 0, 1, 2, 3};
  const int nb = block == -2 ? 5 : 1;
  for (int q = 0; q < nb; ++q) {
    const int blk = block == -2 ? all[q] : block;
    // block-MM rebuilds from the current model before every block; the
    // contraction sets are the current model too
    if ((rc = tk4_t3(w, &cur, 1, &w.T3r, st))) return rc;
    if (blk == 3) {
      if ((rc = tk4_transpose(w, w.T3r, w.T3T[0], st))) return rc;
      Tk4Ws w2 = w;
      w2.T3T[1] = w.T3T[0];
      rc = tk4_block(ctx, x, m, o, w2, blk, cur.F[3], cur, cur, nullptr, nullptr, false, false,
                     block_view4(cur, blk), w.cur, nullptr, st);
    } else {
      rc = tk4_block(ctx, x, m, o, w, blk, cur.F[3], cur, cur, w.cur.facT4, w.cur.facT4, false, false,
                     block_view4(cur, blk), w.cur, nullptr, st);
    }
    if (rc) return rc;
  }
  return COMM_OK;
}

int tucker4_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj,
                  hipStream_t st) {
  const bool kl = o->beta == 1.0;
  const bool cache = o->cache_pq && !kl;
  Tk4Ws w = tk4_layout(x, m, nullptr, cache);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tk4_layout(x, m, ctx->ws, cache);
  if ((rc = tk4_pad(m, w, w.ref, &w.cur, st))) return rc;
  const Tk4Model ref = model4(w, w.ref);
  // the reference, and so its table, is fixed for the whole outer iteration
  if ((rc = tk4_t3(w, &ref, 1, &w.T3r, st))) return rc;
  bool obj_pending = obj != nullptr;
  if (cache) {
    TkPassArgs a = pass4_args(x, o, w);
    a.T2r = w.T3r;
    a.C = ref.F[3];
    a.Pw = w.Pc;
    a.Qw = w.Qc;
    rc = profiled(ctx, st, [&] { return launch_tk_v(a, beta_class_of(o->beta), kTkCacheWrite, obj_pending, 0, st); });
    if (rc) return rc;
    if (obj_pending) HIP_TRY(launch_sum_f64(w.obj_part, w.vwgs, nullptr, obj, st));
    obj_pending = false;
  }
  const float beta = (float)o->beta;
  const int core_rows = w.J[0] * w.J[1] * w.J[2];
  for (int l = 0; l < o->inner_sweeps; ++l) {
    for (int blk : {-1, 0, 1, 2, 3}) {
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
      if (blk != -1) add(w.cur.core, w.ref.core, core_rows, w.num.core, w.den.core);
      for (int q = 0; q < 4; ++q)
        if (q != blk) {
          add(w.cur.fac[q], w.ref.fac[q], q == 3 ? w.Kp : w.dims[q], w.num.fac[q], w.den.fac[q]);
          if (q == 3) {
            ca.x1T[ca.nf - 1] = w.num.facT4;
            ca.x2T[ca.nf - 1] = w.den.facT4;
          }
        }
      HIP_TRY(launch_chi(ca, st));
      Tk4Model ns = model4(w, w.num), ds = model4(w, w.den);
      // the active block does not enter its own contraction
      if (blk == -1) {
        ns.G = ref.G;
        ds.G = ref.G;
      } else {
        ns.F[blk] = ref.F[blk];
        ds.F[blk] = ref.F[blk];
      }
      if (blk == 3) {
        const Tk4Model sets[2] = {ns, ds};
        if ((rc = tk4_t3(w, sets, kl ? 1 : 2, w.V, st))) return rc;
        for (int k = 0; k < (kl ? 1 : 2); ++k)
          if ((rc = tk4_transpose(w, w.V[k], w.T3T[k], st))) return rc;
      }
      rc = tk4_block(ctx, x, m, o, w, blk, ref.F[3], ns, ds, w.num.facT4, w.den.facT4, cache, obj_pending,
                     block_view4(ref, blk), w.cur, obj, st);
      if (rc) return rc;
      obj_pending = false;
    }
  }
  return COMM_OK;
}

int tucker4_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                      hipStream_t st) {
  Tk4Ws w = tk4_layout(x, m, nullptr, false);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tk4_layout(x, m, ctx->ws, false);
  if ((rc = tk4_pad(m, w, w.cur, nullptr, st))) return rc;
  const Tk4Model cur = model4(w, w.cur);
  if ((rc = tk4_t3(w, &cur, 1, &w.T3r, st))) return rc;
  TkPassArgs a = pass4_args(x, o, w);
  a.T2r = w.T3r;
  a.C = cur.F[3];
  rc = profiled(ctx, st, [&] { return launch_tk_v(a, beta_class_of(o->beta), kTkFromX, true, 0, st); });
  if (rc) return rc;
  HIP_TRY(launch_sum_f64(w.obj_part, w.vwgs, nullptr, out, st));
  return COMM_OK;
}
