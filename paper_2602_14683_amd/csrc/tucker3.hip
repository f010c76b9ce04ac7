// Dense 3-way Tucker: B-CoMM and J-CoMM orchestration, the T2 kernel that the
// passes rebuild from, the small contraction GEMMs that turn the V pass's
// output into the mode-1, mode-2 and core numerators, and the closed-form
// beta = 1 denominators.
//
// With V[i][j][c] = sum_k W[i][j][k] C'[k][c] (W = P or Q, from the V pass):
//   U[i][b][c]   = sum_j B'[j][b] V[i][j][c]
//   Num1[i][a]   = sum_{b,c} G'[a][b][c] U[i][b][c]                 (factor A, App. C)
//   Ncore[a][b][c] = sum_i A'[i][a] U[i][b][c]                       (core, App. C)
//   H[i][b][c]   = sum_a A'[i][a] G'[a][b][c]
//   Num2[j][b]   = sum_{i,c} V[i][j][c] H[i][b][c]                   (factor B)
// and the mode-3 numerator comes from the mode-3 pass directly.  These are the
// direct-form contractions of App. C / App. E: the partial tensor B^(n) is
// never formed; only V (J3/K of the size of X) and the I x J2 x J3 U / H.

#include "host_util.h"
#include "tucker3.h"
#include "tucker3_impl.h"

namespace comm {

int64_t tk_v_workgroups(int I, int J) { return ((int64_t)I * J + kTkPairsPerWg - 1) / kTkPairsPerWg; }

// Mode-3 pass tiling: at most `groups` pair groups (partial slots; 0 takes
// kTkGroupsDefault), each of 4 waves x tpw pair tiles of 32.  More groups fill more of the
// chip per k tile; fewer keep fewer partial slots to reduce.
void tk_m3_tiling(int I, int J, int* tpw, int* npg, int groups) {
  const int64_t cap = groups > 0 ? groups : kTkGroupsDefault;
  const int64_t tiles = ((int64_t)I * J + 31) / 32;
  const int64_t t = std::max<int64_t>(1, (tiles + 4 * cap - 1) / (4 * cap));
  *tpw = (int)t;
  *npg = (int)((tiles + 4 * t - 1) / (4 * t));
}

// ---------------------------------------------------------------------------------------- T2

struct T2Args {
  TkModel m[2];
  float* out[2];
  float* outT[2];
  int I, J;
  int64_t Pp;
};

// Workgroup (i, j slab, set): T1[b][c] = sum_a A[i][a] G[a][b][c] in LDS, then
// T2[(i,j)][c] = sum_b B[j][b] T1[b][c] on the matrix cores for the slab's
// (up to) 128 j, one 32-wide j tile per wave, computed transposed (lane = j)
// so that both the row layout and the transposed copy are written with
// coalesced stores (zero for c >= J3).  Each slab recomputes T1 (J1 J2 J3
// products): cheaper than the latency of a workgroup that walks all of J.
constexpr int kT2Slab = 32 * kWaves;
__device__ __forceinline__ void tk_t2_body(const T2Args& t, uint3 bid, uint3) {
  __shared__ float t1[32][33];
  __shared__ float sa[32];
  const int nslab = (t.J + kT2Slab - 1) / kT2Slab;
  const int i = bid.x % t.I, slab = (bid.x / t.I) % nslab, set = bid.x / (t.I * nslab);
  const TkModel& m = t.m[set];
  const int I = t.I, J = t.J;
  if (threadIdx.x < 32) sa[threadIdx.x] = (int)threadIdx.x < m.J1 ? m.A.at(i, threadIdx.x, I) : 0.0f;
  __syncthreads();
  // unpredicated loads over a in batches (a predicated load per a would be
  // one dependent round trip each)
  const int64_t ga = (int64_t)m.J2 * m.ldG;
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int b = e >> 5, c = e & 31;
    float s = 0.0f;
    if (b < m.J2 && c < m.J3) {
      const float* gp = m.G + (int64_t)b * m.ldG + c;
#pragma unroll 8
      for (int a = 0; a < m.J1; ++a) s = fmaf(sa[a], gp[a * ga], s);
    }
    t1[b][c] = s;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5, w = threadIdx.x >> 6;
  float* out = t.out[set] + (int64_t)i * J * kRP;
  float* outT = t.outT[set];
  const int j0 = slab * kT2Slab + 32 * w;
  if (j0 < J) {
    // T2^T[c][j] = sum_b T1[b][c] B[j][b]: A operand T1 (lane: c), B operand B rows (lane: j)
    float brow[16];
    row16(m.B.p + (int64_t)(j0 + col) * kRP + 16 * h, j0 + col < J, brow);
    f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = mfma32(t1[16 * h + s][col], brow[s], acc);
    // acc[v] = T2[j = j0 + col][c = out_row(v, h)]
    const int j = j0 + col;
    if (j < J) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        f32x4 q = {acc[4 * g], acc[4 * g + 1], acc[4 * g + 2], acc[4 * g + 3]};
        *reinterpret_cast<f32x4*>(out + (int64_t)j * kRP + 8 * g + 4 * h) = q;
      }
      if (outT) {
#pragma unroll
        for (int v = 0; v < 16; ++v) outT[(int64_t)out_row(v, h) * t.Pp + (int64_t)i * J + j] = acc[v];
      }
    }
  }
  // the transposed copy's padding past the last pair reads as zero
  if (outT && i == I - 1 && slab == 0) {
    const int64_t np = (int64_t)I * J;
    const int pad = (int)(t.Pp - np);
    for (int e = threadIdx.x; e < 32 * pad; e += 256) outT[(int64_t)(e / pad) * t.Pp + np + e % pad] = 0.0f;
  }
}
COMM_GROUPED_KERNELS(tk_t2, T2Args, 256)

hipError_t launch_tk_t2(const TkModel* m, float* const* T2, float* const* T2T, int sets, int I, int J, int64_t Pp,
                        hipStream_t s) {
  T2Args t = {};
  for (int k = 0; k < sets; ++k) {
    t.m[k] = m[k];
    t.out[k] = T2[k];
    t.outT[k] = T2T ? T2T[k] : nullptr;
  }
  t.I = I;
  t.J = J;
  t.Pp = Pp;
  const int nslab = (J + kT2Slab - 1) / kT2Slab;
  return launch_or_record(tk_t2_kernel, tk_t2_grouped, dim3((unsigned)(I * nslab * sets)), dim3(256), 0, s, t);
}

// ---------------------------------------------------------------------------------------- GEMM

// One workgroup per 32 x 32 output tile (per set, split and batch); its four
// waves split the tile's k range and their partial tiles are summed in a
// fixed order.  Each matrix-core step consumes two k (lane half h supplies
// k = 2 s + h); operands of 16 steps are loaded before they are used.
constexpr int kGemmBatch = 16;

__device__ __forceinline__ void gemm_body(const GemmArgs& g, uint3 bid, uint3) {
  __shared__ float red[kWaves][32 * 33];
  const int tiles_m = (g.M + 31) / 32, tiles_n = (g.N + 31) / 32;
  int64_t id = bid.x;
  const int tn = (int)(id % tiles_n);
  id /= tiles_n;
  const int tm = (int)(id % tiles_m);
  id /= tiles_m;
  const int bat = (int)(id % g.batch);
  id /= g.batch;
  const int split = (int)(id % g.splits);
  const int set = (int)(id / g.splits);
  const int kc = (g.K + g.splits - 1) / g.splits;
  const int ks = split * kc, ke = min(g.K, ks + kc);
  const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5, w = threadIdx.x >> 6;
  // wave w: k in [k0, k1), a quarter of the split, rounded to whole steps
  const int steps_all = max(0, (ke - ks + 1) / 2);
  const int per = (steps_all + kWaves - 1) / kWaves;
  const int s_begin = min(steps_all, w * per), s_end = min(steps_all, s_begin + per);
  const int m = tm * 32 + col, n = tn * 32 + col;
  const float* A = g.A[set] + (int64_t)bat * g.sab + (int64_t)m * g.sam;
  const float* B = g.B[set] + (int64_t)bat * g.sbb + (int64_t)n * g.sbn;
  const int amask = (1 << g.akin_log2) - 1, bmask = (1 << g.bkin_log2) - 1;
  const bool mok = m < g.M, nok = n < g.N;
  f32x16 acc = {};
  for (int s0 = s_begin; s0 < s_end; s0 += kGemmBatch) {
    float av[kGemmBatch], bv[kGemmBatch];
#pragma unroll
    for (int u = 0; u < kGemmBatch; ++u) {
      const int k = ks + 2 * (s0 + u) + h;
      const bool kok = s0 + u < s_end && k < ke;
      av[u] = (mok && kok) ? A[(int64_t)(k >> g.akin_log2) * g.sako + (int64_t)(k & amask) * g.saki] : 0.0f;
      bv[u] = (nok && kok) ? B[(int64_t)(k >> g.bkin_log2) * g.sbko + (int64_t)(k & bmask) * g.sbki] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kGemmBatch; ++u) acc = mfma32(av[u], bv[u], acc);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) red[w][out_row(v, h) * 33 + col] = acc[v];
  __syncthreads();
  float* out = g.out[set] + (int64_t)split * g.sos + (int64_t)bat * g.sob;
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int r = e >> 5, c = e & 31;
    const int row = tm * 32 + r, cn = tn * 32 + c;
    if (row < g.M && cn < g.N) {
      float sum = red[0][r * 33 + c];
      for (int q = 1; q < kWaves; ++q) sum += red[q][r * 33 + c];
      out[(int64_t)row * g.ldo + cn] = sum;
    }
  }
}

COMM_GROUPED_KERNELS(gemm, GemmArgs, 256)

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  const int64_t tiles = (int64_t)((g.M + 31) / 32) * ((g.N + 31) / 32) * g.batch * g.splits * g.sets;
  return launch_or_record(gemm_kernel, gemm_grouped, dim3((unsigned)tiles), dim3(256), 0, s, g);
}

// ---------------------------------------------------------------------------------------- closed-form den

struct TkDenArgs {
  TkModel m;
  int I, J, K;
  float* den;
  float* dcore;
};

__device__ __forceinline__ void tk_den_closed_body(const TkDenArgs& args, uint3, uint3) {
  const TkModel& m = args.m;
  const int I = args.I, J = args.J, K = args.K;
  float* den = args.den;
  float* dcore = args.dcore;
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

COMM_GROUPED_KERNELS(tk_den_closed, TkDenArgs, 1024)

hipError_t launch_tk_den_closed(const TkModel& m, int I, int J, int K, float* den, float* dcore, hipStream_t s) {
  return launch_or_record(tk_den_closed_kernel, tk_den_closed_grouped, dim3(1), dim3(1024), 0, s,
                          TkDenArgs{m, I, J, K, den, dcore});
}

}  // namespace comm

// ---------------------------------------------------------------------------------------- orchestration

using namespace comm;

namespace {

// Padded copies of a Tucker model: core [J1 J2][32], factors [I_n][32].
// The mode-3 factor copy has Kp rows (zero past K); cur, num and den also keep
// it transposed, [32][Kp], for the V pass.
struct TkCopy {
  float* core;
  float* fac[3];
  float* facT2;
};

struct TkWs {
  int dims[3], J[3];
  int Kp, tpw, npg;
  int64_t vwgs;
  float* T2r;        // T2 of the rebuild model
  float* T2n;        // T2 of the numerator / denominator sets (mode-3 block)
  float* T2d;
  float* T2nT;       // the same, transposed [32][Pp]
  float* T2dT;
  int64_t Pp;
  float* Vn;         // V of the numerator / denominator set
  float* Vd;
  float* m3[2];      // mode-3 partial slots of the numerator / denominator
  double* obj_part;
  float* U[2];       // per set: numerator, denominator
  float* H[2];
  float* slots[2];   // numerator / denominator split-K outputs
  size_t slot_floats;
  float* kslots[3];  // beta = 1: the core, mode-1 and mode-2 numerators, kept for the outer iteration
  float* den_vec;    // [3][32]
  float* dcore;      // [J1 J2][32]
  TkCopy ref, cur, num, den, user_pad;
  float *Pc, *Qc;
  size_t bytes;
};

constexpr int kSplitCore = 8, kSplit1 = 8, kSplit2 = 32;

TkWs tk_layout(const comm_dense* x, const comm_model* m, char* base, bool cache, int groups = 0) {
  TkWs w = {};
  for (int n = 0; n < 3; ++n) {
    w.dims[n] = (int)x->dims[n];
    w.J[n] = (int)m->core_dims[n];
  }
  const int I = w.dims[0], J = w.dims[1], K = w.dims[2];
  const int J1 = w.J[0], J2 = w.J[1];
  const size_t pairs = (size_t)I * J;
  w.Kp = (K + 31) / 32 * 32;
  w.Pp = ((int64_t)pairs + 31) / 32 * 32;
  tk_m3_tiling(I, J, &w.tpw, &w.npg, groups);
  w.vwgs = tk_v_workgroups(I, J);
  Carve cv;
  cv.base = base;
  w.T2r = cv.take<float>(pairs * kRP);
  w.T2n = cv.take<float>(pairs * kRP);
  w.T2d = cv.take<float>(pairs * kRP);
  w.T2nT = cv.take<float>((size_t)w.Pp * kRP);
  w.T2dT = cv.take<float>((size_t)w.Pp * kRP);
  w.Vn = cv.take<float>(pairs * kRP);
  w.Vd = cv.take<float>(pairs * kRP);
  w.m3[0] = cv.take<float>((size_t)w.npg * w.Kp * kRP);
  w.m3[1] = cv.take<float>((size_t)w.npg * w.Kp * kRP);
  w.obj_part = cv.take<double>((size_t)w.vwgs);
  for (int k = 0; k < 2; ++k) {
    w.U[k] = cv.take<float>((size_t)I * J2 * kRP);
    w.H[k] = cv.take<float>((size_t)I * J2 * kRP);
  }
  size_t s = (size_t)kSplitCore * J1 * J2 * kRP;
  s = std::max(s, (size_t)kSplit1 * I * kRP);
  s = std::max(s, (size_t)kSplit2 * J * kRP);
  w.slot_floats = s;
  w.slots[0] = cv.take<float>(s);
  w.slots[1] = cv.take<float>(s);
  w.kslots[0] = cv.take<float>((size_t)kSplitCore * J1 * J2 * kRP);
  w.kslots[1] = cv.take<float>((size_t)kSplit1 * I * kRP);
  w.kslots[2] = cv.take<float>((size_t)kSplit2 * J * kRP);
  w.den_vec = cv.take<float>(3 * kRP);
  w.dcore = cv.take<float>((size_t)J1 * J2 * kRP);
  for (TkCopy* c : {&w.ref, &w.cur, &w.num, &w.den, &w.user_pad}) {
    c->core = cv.take<float>((size_t)J1 * J2 * kRP);
    for (int n = 0; n < 2; ++n) c->fac[n] = cv.take<float>((size_t)w.dims[n] * kRP);
    c->fac[2] = cv.take<float>((size_t)w.Kp * kRP);
    c->facT2 = nullptr;
  }
  for (TkCopy* c : {&w.cur, &w.num, &w.den}) c->facT2 = cv.take<float>((size_t)w.Kp * kRP);
  if (cache) {
    const size_t total = pairs * K;
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

// Copy the caller's model into padded buffers (and optionally a second copy),
// core and three factors in one launch.
int tk_pad(const comm_model* m, const TkWs& w, const TkCopy& dst, const TkCopy* dst2, hipStream_t st) {
  PadArgs p = {};
  p.nf = 4;
  p.cols[0] = w.J[2];
  p.ld[0] = w.J[2];
  p.src[0] = m->core;
  p.rows[0] = w.J[0] * w.J[1];
  p.rows_p[0] = p.rows[0];
  p.dst[0] = dst.core;
  p.dst2[0] = dst2 ? dst2->core : nullptr;
  for (int n = 0; n < 3; ++n) {
    const int f = n + 1;
    p.cols[f] = w.J[n];
    p.ld[f] = w.J[n];
    p.src[f] = m->factors[n];
    p.rows[f] = w.dims[n];
    p.rows_p[f] = n == 2 ? w.Kp : w.dims[n];
    p.dst[f] = dst.fac[n];
    p.dst2[f] = dst2 ? dst2->fac[n] : nullptr;
    if (n == 2) {
      p.dstT[f] = dst.facT2;
      p.dst2T[f] = dst2 ? dst2->facT2 : nullptr;
    }
  }
  HIP_TRY(launch_pad_factors(p, st));
  return COMM_OK;
}

struct Slots {
  const float* part;
  int n;
  int rows_total;
};

TkPassArgs pass_args(const comm_dense* x, const comm_opts* o, const TkWs& w) {
  TkPassArgs a = {};
  a.X = x->X;
  a.I = w.dims[0];
  a.J = w.dims[1];
  a.K = w.dims[2];
  a.Kp = w.Kp;
  a.eps = (float)o->eps;
  a.eps_x = (float)o->eps_x;
  a.bc = make_beta_const(o->beta);
  a.Vn = w.Vn;
  a.Vd = w.Vd;
  a.m3n = w.m3[0];
  a.m3d = w.m3[1];
  a.obj_part = w.obj_part;
  a.tpw = w.tpw;
  a.npg = w.npg;
  a.Pp = w.Pp;
  a.xvec = (w.dims[2] % 4 == 0) && (reinterpret_cast<uintptr_t>(x->X) % 16 == 0);
  a.bf16 = o->precision == COMM_BF16;
  return a;
}

// Numerator slots of block blk (-1 core, 0, 1) from V of the contraction set
// cs[0] (into out[0]) and, when sets = 2, the denominator from V of cs[1].
// reuse_u: U from the core block's GEMMs of the same sweep is still valid
// (same V, same B'), so mode 1 starts from it.  slot_out: where the split-K
// outputs go (default w.slots).
int tk_gemms(const TkWs& w, int blk, const TkModel* cs, int sets, Slots* out, hipStream_t st, bool reuse_u = false,
             float* const* slot_out = nullptr) {
  float* const* so = slot_out ? slot_out : w.slots;
  const int I = w.dims[0], J = w.dims[1];
  const int J1 = w.J[0], J2 = w.J[1];
  constexpr int kNoWrap = 30, kWrap32 = 5;
  const float* V[2] = {w.Vn, w.Vd};
  auto set_ptrs = [&](GemmArgs& g, auto fa, auto fb, auto fo) {
    g.sets = sets;
    for (int k = 0; k < sets; ++k) {
      g.A[k] = fa(k);
      g.B[k] = fb(k);
      g.out[k] = fo(k);
    }
  };
  if (blk == -1 || (blk == 0 && !reuse_u)) {
    // U[i][b][c] = sum_j B'[j][b] V[i][j][c]
    GemmArgs g = {};
    g.sab = 0; g.sam = 1; g.akin_log2 = kNoWrap; g.sako = 0; g.saki = kRP;
    g.sbb = (int64_t)J * kRP; g.bkin_log2 = kNoWrap; g.sbko = 0; g.sbki = kRP; g.sbn = 1;
    g.sob = (int64_t)J2 * kRP; g.sos = 0; g.ldo = kRP;
    g.M = J2; g.N = kRP; g.K = J; g.batch = I; g.splits = 1;
    set_ptrs(g, [&](int k) { return cs[k].B.p; }, [&](int k) { return V[k]; }, [&](int k) { return w.U[k]; });
    HIP_TRY(launch_gemm(g, st));
  }
  if (blk == 0) {
    // Num1[i][a] = sum_{(b,c)} U[i][(b,c)] G'[a][(b,c)]
    GemmArgs g = {};
    g.sab = 0; g.sam = (int64_t)J2 * kRP; g.akin_log2 = kNoWrap; g.sako = 0; g.saki = 1;
    g.sbb = 0; g.bkin_log2 = kNoWrap; g.sbko = 0; g.sbki = 1; g.sbn = (int64_t)J2 * kRP;
    g.sob = 0; g.sos = (int64_t)I * kRP; g.ldo = kRP;
    g.M = I; g.N = J1; g.K = J2 * kRP; g.batch = 1; g.splits = kSplit1;
    set_ptrs(g, [&](int k) { return (const float*)w.U[k]; }, [&](int k) { return cs[k].G; },
             [&](int k) { return so[k]; });
    HIP_TRY(launch_gemm(g, st));
    for (int k = 0; k < sets; ++k) out[k] = Slots{so[k], kSplit1, I};
  } else if (blk == -1) {
    // Ncore[a][(b,c)] = sum_i A'[i][a] U[i][(b,c)]
    GemmArgs g = {};
    g.sab = 0; g.sam = 1; g.akin_log2 = kNoWrap; g.sako = 0; g.saki = kRP;
    g.sbb = 0; g.bkin_log2 = kNoWrap; g.sbko = 0; g.sbki = (int64_t)J2 * kRP; g.sbn = 1;
    g.sob = 0; g.sos = (int64_t)J1 * J2 * kRP; g.ldo = (int64_t)J2 * kRP;
    g.M = J1; g.N = J2 * kRP; g.K = I; g.batch = 1; g.splits = kSplitCore;
    set_ptrs(g, [&](int k) { return cs[k].A.p; }, [&](int k) { return (const float*)w.U[k]; },
             [&](int k) { return so[k]; });
    HIP_TRY(launch_gemm(g, st));
    for (int k = 0; k < sets; ++k) out[k] = Slots{so[k], kSplitCore, J1 * J2};
  } else {
    // H[i][(b,c)] = sum_a A'[i][a] G'[a][(b,c)];  Num2[j][b] = sum_{(i,c)} V[i][j][c] H[i][b][c]
    GemmArgs g = {};
    g.sab = 0; g.sam = kRP; g.akin_log2 = kNoWrap; g.sako = 0; g.saki = 1;
    g.sbb = 0; g.bkin_log2 = kNoWrap; g.sbko = 0; g.sbki = (int64_t)J2 * kRP; g.sbn = 1;
    g.sob = 0; g.sos = 0; g.ldo = (int64_t)J2 * kRP;
    g.M = I; g.N = J2 * kRP; g.K = J1; g.batch = 1; g.splits = 1;
    set_ptrs(g, [&](int k) { return cs[k].A.p; }, [&](int k) { return cs[k].G; }, [&](int k) { return w.H[k]; });
    HIP_TRY(launch_gemm(g, st));
    GemmArgs h = {};
    h.sab = 0; h.sam = kRP; h.akin_log2 = kWrap32; h.sako = (int64_t)J * kRP; h.saki = 1;
    h.sbb = 0; h.bkin_log2 = kWrap32; h.sbko = (int64_t)J2 * kRP; h.sbki = 1; h.sbn = kRP;
    h.sob = 0; h.sos = (int64_t)J * kRP; h.ldo = kRP;
    h.M = J; h.N = J2; h.K = I * kRP; h.batch = 1; h.splits = kSplit2;
    set_ptrs(h, [&](int k) { return V[k]; }, [&](int k) { return (const float*)w.H[k]; },
             [&](int k) { return so[k]; });
    HIP_TRY(launch_gemm(h, st));
    for (int k = 0; k < sets; ++k) out[k] = Slots{so[k], kSplit2, J};
  }
  return COMM_OK;
}

// One block update: max(anchor * (Num/Den)^gamma, eps) into the caller's
// block (and a padded copy).  blk -1 = core.
float* copy_block(const TkCopy& c, int blk);

// (chi_beta >= 0: also the block's J-CoMM transforms into the num / den sets,
// as chi_kernel would compute them from the padded copy)
int tk_apply(const comm_model* m, const TkWs& w, int blk, const Slots& num, const Slots* den,
             const float* den_closed_vec, FView anchor, float* out_pad, float* out_padT, float gamma, float eps,
             hipStream_t st, float chi_beta = -1.0f) {
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
  Jb.rows_p = blk == 2 ? w.Kp : Jb.rows;
  Jb.anchor = anchor;
  Jb.gamma = gamma;
  Jb.eps = eps;
  Jb.out_pad = out_pad;
  Jb.out_padT = blk == 2 ? out_padT : nullptr;
  if (chi_beta >= 0.0f) {
    Jb.chi_ref = copy_block(w.ref, blk);
    Jb.chi_x1 = copy_block(w.num, blk);
    Jb.chi_x2 = copy_block(w.den, blk);
    Jb.chi_x1T = blk == 2 ? w.num.facT2 : nullptr;
    Jb.chi_x2T = blk == 2 ? w.den.facT2 : nullptr;
    Jb.chi_beta = chi_beta;
  }
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

// Numerator (and, unless beta = 1, denominator) slots of block blk against the
// sets ns / ds from the V of the last V pass (blk -1, 0, 1; reuse_u: the core
// block's U of this sweep serves mode 1), then the block update.
int tk_from_v(comm_model* m, const comm_opts* o, const TkWs& w, int blk, const TkModel& ns, const TkModel& ds,
              bool reuse_u, FView anchor, float* out_pad, hipStream_t st, bool with_chi = false) {
  const bool kl = o->beta == 1.0;
  const int sets = kl ? 1 : 2;
  const TkModel cs[2] = {ns, ds};
  Slots nd[2];
  int rc = tk_gemms(w, blk, cs, sets, nd, st, reuse_u);
  if (rc) return rc;
  Slots den = nd[1];
  const float* vec = nullptr;
  Slots* denp = &den;
  if (kl) {
    if ((rc = tk_closed_den(w, blk, ds, &den, &vec, st))) return rc;
    if (blk != -1) denp = nullptr;
  }
  return tk_apply(m, w, blk, nd[0], denp, vec, anchor, out_pad, w.cur.facT2, gamma_of(o->beta), (float)o->eps, st,
                  with_chi ? (float)o->beta : -1.0f);
}

// The V pass (blocks -1, 0, 1) or the mode-3 pass (block 2) over X rebuilt
// from rb (its T2 in w.T2r) or over the cached P~ / Q~, with the sets whose
// mode-3 factors (transposed) are cnT / cdT and whose T2 are in w.T2nT / T2dT.
int tk_pass(comm_ctx* ctx, const comm_dense* x, const comm_opts* o, const TkWs& w, int blk, const TkModel& rb,
            const float* cnT, const float* cdT, bool cached, bool want_obj, double* obj, hipStream_t st) {
  const int sets = o->beta == 1.0 ? 1 : 2;
  const int bc = beta_class_of(o->beta);
  const int mode = cached ? kTkCacheRead : kTkFromX;
  TkPassArgs a = pass_args(x, o, w);
  a.T2r = w.T2r;
  a.C = rb.C;
  if (cached) {
    a.Pc = w.Pc;
    a.Qc = w.Qc;
  }
  if (blk == 2) {
    a.T2nT = w.T2nT;
    a.T2dT = w.T2dT;
    return profiled(ctx, st, [&] { return launch_tk_m3(a, bc, mode, sets, st); });
  }
  a.CnT = cnT;
  a.CdT = cdT;
  int rc = profiled(ctx, st, [&] { return launch_tk_v(a, bc, mode, want_obj, sets, st); });
  if (rc) return rc;
  if (want_obj && obj) HIP_TRY(launch_sum_f64(w.obj_part, w.vwgs, nullptr, obj, st));
  return COMM_OK;
}

// Update of block blk: its pass, then its numerator / denominator and the update.
int tk_block(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, const TkWs& w, int blk,
             const TkModel& rb, const TkModel& ns, const TkModel& ds, const float* cnT, const float* cdT,
             bool cached, bool want_obj, FView anchor, float* out_pad, double* obj, hipStream_t st,
             bool with_chi = false) {
  int rc = tk_pass(ctx, x, o, w, blk, rb, cnT, cdT, cached, want_obj, obj, st);
  if (rc) return rc;
  if (blk != 2) return tk_from_v(m, o, w, blk, ns, ds, false, anchor, out_pad, st, with_chi);
  const bool kl = o->beta == 1.0;
  const Slots num{w.m3[0], w.npg, w.Kp};
  Slots den{w.m3[1], w.npg, w.Kp};
  const float* vec = nullptr;
  Slots* denp = &den;
  if (kl) {
    if ((rc = tk_closed_den(w, blk, ds, &den, &vec, st))) return rc;
    denp = nullptr;
  }
  return tk_apply(m, w, blk, num, denp, vec, anchor, out_pad, w.cur.facT2, gamma_of(o->beta), (float)o->eps, st,
                  with_chi ? (float)o->beta : -1.0f);
}

// T2 of one model into T2 (and its transposed copy into T2T unless NULL).
int tk_t2(const TkWs& w, const TkModel& md, float* T2, float* T2T, hipStream_t st) {
  float* out[1] = {T2};
  float* outT[1] = {T2T};
  HIP_TRY(launch_tk_t2(&md, out, outT, 1, w.dims[0], w.dims[1], w.Pp, st));
  return COMM_OK;
}

// T2 of the numerator and denominator sets for the mode-3 block.
int tk_t2_pair(const TkWs& w, const TkModel& m0, const TkModel& m1, hipStream_t st) {
  const TkModel m[2] = {m0, m1};
  float* out[2] = {w.T2n, w.T2d};
  float* outT[2] = {w.T2nT, w.T2dT};
  HIP_TRY(launch_tk_t2(m, out, outT, 2, w.dims[0], w.dims[1], w.Pp, st));
  return COMM_OK;
}

}  // namespace

int tucker_check_model(const comm_model* m, const comm_dense* x) {
  if (!m) return fail(COMM_EINVAL, "model is NULL");
  if (m->kind != COMM_TUCKER) return fail(COMM_EINVAL, "model kind is not Tucker");
  if (!m->core) return fail(COMM_EINVAL, "core is NULL");
  if (x->ndim < 3 || x->ndim > 5)
    return fail(COMM_EUNSUPPORTED, "dense Tucker of order %d is not supported (3 to 5)", x->ndim);
  if (x->ndim > 3) {
    int64_t rows = 1;
    for (int n = 0; n < x->ndim - 1; ++n) rows *= x->dims[n];
    if (rows > (1 << 24))
      return fail(COMM_EUNSUPPORTED, "I_1 ... I_%d = %lld exceeds 2^24", x->ndim - 1, (long long)rows);
  }
  for (int n = 0; n < x->ndim; ++n) {
    if (!m->factors[n]) return fail(COMM_EINVAL, "factors[%d] is NULL", n);
    if (m->core_dims[n] < 1) return fail(COMM_EINVAL, "core_dims[%d] = %lld", n, (long long)m->core_dims[n]);
    if (m->core_dims[n] > kRP) return fail(COMM_EUNSUPPORTED, "core_dims[%d] > %d not supported", n, kRP);
  }
  return COMM_OK;
}

size_t tucker_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op, int groups) {
  if (x->ndim > 3) return tuckern_workspace_bytes(x, m, o, op);
  const bool cache = op == 1 && o->cache_pq && o->beta != 1.0;
  return tk_layout(x, m, nullptr, cache, op == 1 ? groups : 0).bytes;
}

int tucker_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st) {
  if (x->ndim > 3) return tuckern_bcomm(ctx, x, m, block, o, st);
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
    // block-MM rebuilds from the current model before every block; the
    // contraction sets are the current model too
    if ((rc = tk_t2(w, cur, w.T2r, blk == 2 ? w.T2nT : nullptr, st))) return rc;
    if (blk == 2) {
      TkWs w2 = w;
      w2.T2dT = w.T2nT;
      rc = tk_block(ctx, x, m, o, w2, blk, cur, cur, cur, nullptr, nullptr, false, false, block_view(cur, blk),
                    copy_block(w.cur, blk), nullptr, st);
    } else {
      rc = tk_block(ctx, x, m, o, w, blk, cur, cur, cur, w.cur.facT2, w.cur.facT2, false, false,
                    block_view(cur, blk), copy_block(w.cur, blk), nullptr, st);
    }
    if (rc) return rc;
  }
  return COMM_OK;
}

int tucker_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st) {
  if (x->ndim > 3) return tuckern_jcomm(ctx, x, m, o, obj, st);
  const bool kl = o->beta == 1.0;
  const bool cache = o->cache_pq && !kl;
  const int groups = ctx->pick.tk_groups;
  TkWs w = tk_layout(x, m, nullptr, cache, groups);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tk_layout(x, m, ctx->ws, cache, groups);
  if ((rc = tk_pad(m, w, w.ref, &w.cur, st))) return rc;
  const TkModel ref = model_of(w, w.ref);
  // the reference model, and so its T2, is fixed for the whole outer iteration
  // (at beta = 1 it is also the mode-3 block's contraction set, transposed)
  if ((rc = tk_t2(w, ref, w.T2r, kl ? w.T2nT : nullptr, st))) return rc;
  bool obj_pending = obj != nullptr;
  if (cache) {
    TkPassArgs a = pass_args(x, o, w);
    a.T2r = w.T2r;
    a.C = ref.C;
    a.Pw = w.Pc;
    a.Qw = w.Qc;
    rc = profiled(ctx, st, [&] { return launch_tk_v(a, beta_class_of(o->beta), kTkCacheWrite, obj_pending, 0, st); });
    if (rc) return rc;
    if (obj_pending) HIP_TRY(launch_sum_f64(w.obj_part, w.vwgs, nullptr, obj, st));
    obj_pending = false;
  }
  const float beta = (float)o->beta;
  // transformed blocks of the current inner iterate (Sec. 5.3, App. C.3) for
  // the listed blocks (-1 core, 0..2 factors) into the num / den sets
  auto chi = [&](std::initializer_list<int> blocks) -> int {
    ChiArgs ca = {};
    ca.beta = beta;
    for (int q : blocks) {
      const int f = ca.nf++;
      ca.cur[f] = copy_block(w.cur, q);
      ca.ref[f] = copy_block(w.ref, q);
      ca.rows_p[f] = q == -1 ? w.J[0] * w.J[1] : q == 2 ? w.Kp : w.dims[q];
      ca.x1[f] = copy_block(w.num, q);
      ca.x2[f] = copy_block(w.den, q);
      if (q == 2) {
        ca.x1T[f] = w.num.facT2;
        ca.x2T[f] = w.den.facT2;
      }
    }
    HIP_TRY(launch_chi(ca, st));
    return COMM_OK;
  };

  if (kl) {
    // beta = 1: chi_1 is the reference block, so every numerator depends on
    // the reference alone and serves all L sweeps: one V pass (core, modes 1
    // and 2, and the objective) and one mode-3 pass against the reference's
    // own T2.  The sweeps then need only the closed-form denominators of the
    // current blocks and the updates.
    if ((rc = chi({2}))) return rc;  // the reference mode-3 factor, transposed, for the V pass
    if ((rc = tk_pass(ctx, x, o, w, -1, ref, w.num.facT2, nullptr, false, obj_pending, obj, st))) return rc;
    Slots num[4], unused[2];
    if ((rc = tk_gemms(w, -1, &ref, 1, unused, st, false, &w.kslots[0]))) return rc;
    num[0] = unused[0];
    if ((rc = tk_gemms(w, 0, &ref, 1, unused, st, true, &w.kslots[1]))) return rc;
    num[1] = unused[0];
    if ((rc = tk_gemms(w, 1, &ref, 1, unused, st, false, &w.kslots[2]))) return rc;
    num[2] = unused[0];
    if ((rc = tk_pass(ctx, x, o, w, 2, ref, nullptr, nullptr, false, false, nullptr, st))) return rc;
    num[3] = Slots{w.m3[0], w.npg, w.Kp};
    const TkModel cur = model_of(w, w.cur);
    for (int l = 0; l < o->inner_sweeps; ++l) {
      for (int blk : {-1, 0, 1, 2}) {
        Slots den;
        const float* vec = nullptr;
        if ((rc = tk_closed_den(w, blk, cur, &den, &vec, st))) return rc;
        rc = tk_apply(m, w, blk, num[blk + 1], blk == -1 ? &den : nullptr, vec, block_view(ref, blk),
                      copy_block(w.cur, blk), w.cur.facT2, 1.0f, (float)o->eps, st);
        if (rc) return rc;
      }
    }
    return COMM_OK;
  }

  // beta != 1, per sweep: one V pass serves the core and modes 1 and 2 (the
  // mode-3 sets do not change until the mode-3 block), then the mode-3 pass.
  // every block update writes the block's transforms with it (tk_apply), so
  // after the first sweep's start the sets are always current
  if ((rc = chi({0, 1, 2}))) return rc;
  for (int l = 0; l < o->inner_sweeps; ++l) {
    // core block: sets of the three factors, the V pass, U and the core numerators
    TkModel ns = model_of(w, w.num), ds = model_of(w, w.den);
    ns.G = ref.G;  // the active block does not enter its own contraction
    ds.G = ref.G;
    const bool want_obj = obj_pending && !cache;
    if ((rc = tk_pass(ctx, x, o, w, -1, ref, w.num.facT2, w.den.facT2, cache, want_obj, obj, st))) return rc;
    obj_pending = false;
    if ((rc = tk_from_v(m, o, w, -1, ns, ds, false, block_view(ref, -1), copy_block(w.cur, -1), st, true)))
      return rc;
    // mode 1 from the same V and U: only the core's sets changed
    ns = model_of(w, w.num);
    ds = model_of(w, w.den);
    ns.A = ref.A;
    ds.A = ref.A;
    if ((rc = tk_from_v(m, o, w, 0, ns, ds, true, block_view(ref, 0), copy_block(w.cur, 0), st, true))) return rc;
    // mode 2 from the same V: only mode 1's sets changed
    ns = model_of(w, w.num);
    ds = model_of(w, w.den);
    ns.B = ref.B;
    ds.B = ref.B;
    if ((rc = tk_from_v(m, o, w, 1, ns, ds, false, block_view(ref, 1), copy_block(w.cur, 1), st, true)))
      return rc;
    // mode 3: mode 2's sets, both sets' T2, the mode-3 pass
    ns = model_of(w, w.num);
    ds = model_of(w, w.den);
    ns.C = ref.C;
    ds.C = ref.C;
    if ((rc = tk_t2_pair(w, ns, ds, st))) return rc;
    rc = tk_block(ctx, x, m, o, w, 2, ref, ns, ds, nullptr, nullptr, cache, false, block_view(ref, 2),
                  copy_block(w.cur, 2), nullptr, st, true);
    if (rc) return rc;
  }
  return COMM_OK;
}

int tucker_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                     hipStream_t st) {
  if (x->ndim > 3) return tuckern_objective(ctx, x, m, o, out, st);
  TkWs w = tk_layout(x, m, nullptr, false);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tk_layout(x, m, ctx->ws, false);
  if ((rc = tk_pad(m, w, w.cur, nullptr, st))) return rc;
  const TkModel cur = model_of(w, w.cur);
  if ((rc = tk_t2(w, cur, w.T2r, nullptr, st))) return rc;
  TkPassArgs a = pass_args(x, o, w);
  a.T2r = w.T2r;
  a.C = cur.C;
  rc = profiled(ctx, st, [&] { return launch_tk_v(a, beta_class_of(o->beta), kTkFromX, true, 0, st); });
  if (rc) return rc;
  HIP_TRY(launch_sum_f64(w.obj_part, w.vwgs, nullptr, out, st));
  return COMM_OK;
}
