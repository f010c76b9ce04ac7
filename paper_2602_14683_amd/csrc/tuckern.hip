// Dense Tucker of order N = 4, 5 (Sec. 4.3, App. C and Sec. 5.3 for general
// N): B-CoMM, J-CoMM and the objective.
//
// The two fused Tucker passes of the order-3 path run unchanged on the
// (I_1 ... I_{N-1}) x I_N matrix view of X: a row is the mode-N fibre of the
// index tuple (i_1, ..., i_{N-1}), rebuilt from the table
//   T[(i_1..i_{N-1})][d] = (G x_1 A_1 ... x_{N-1} A_{N-1})[i_1..i_{N-1}][d]
// (N - 1 mode products of the core) and the mode-N factor.  With
// V[(i_1..i_{N-1})][d] = sum_{i_N} W[..][i_N] A'_N[i_N][d] from the V pass
// (W = P or Q), the other numerators are mode products of V:
//   core   : Ncore = V x_{N-1} A'_{N-1}^T ... x_1 A'_1^T
//   mode n : Z_n = V contracted with A'_m^T on every grouped mode m != n, then
//            Num_n[i][j] = sum over the other indices of Z_n[..i..] G'[..j..]
//            (one GEMM per leading core index, summed as partial slots),
// and the mode-N numerator is the fibre-mode pass of the order-3 path on the
// same view, against the table of the contraction set.  Mode products are a
// streaming kernel (one side of each is at most 32 wide); the last
// contraction of a grouped mode is a batched matrix-core GEMM (launch_gemm).
// The partial tensor of a mode is never formed, only V and the small products
// of it.

#include <algorithm>

#include "host_util.h"
#include "kernels.h"
#include "tucker3.h"

namespace comm {

constexpr int kTkMaxN = kMaxModes;
constexpr int kTkMaxG = kTkMaxN - 1;  // grouped modes (all but the fibre mode)

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

// An order-N Tucker model as the kernels see it: core entry (j_1..j_N) at
// G[(((j_1 J_2 + j_2) J_3 + ...) J_{N-1} + j_{N-1}) * 32 + j_N]; factor views
// with cols = J_n.
struct TkNModel {
  int N;
  const float* G;
  FView F[kTkMaxN];
  int J[kTkMaxN];
  int rows[kTkMaxN];
};

// Closed-form beta = 1 denominators (Q = 1) from the column sums S_m of the
// denominator set's factors: den[n][j] = sum over the core entries with
// j_n = j of G * prod_{m != n} S_m[j_m], and dcore[(j_1..j_{N-1})][j_N] =
// prod_m S_m[j_m].  Workgroup (j, n) for n < N forms den[n][j] (its threads
// stride over the other core entries, combined in a fixed order); the
// workgroups of row N write dcore.  Every workgroup first forms the column
// sums itself (the factors are small), in the same order.
constexpr int kDenThreads = 1024;
constexpr int kDenBatch = 4;   // independent loads in flight per thread

__global__ void __launch_bounds__(kDenThreads) tkn_den_closed_kernel(TkNModel m, float* den, float* dcore) {
  __shared__ float red[kTkMaxN][32][33];
  __shared__ float S[kTkMaxN][32];
  __shared__ float part[kDenThreads];
  const int t = threadIdx.x;
  const int c = t & 31, g = t >> 5;   // 32 row groups of 32 lanes
  const int N = m.N;
  // column sums of all factors at once: row group g of each factor (loads of
  // all factors issued together), then the 32 groups in order
  {
    float s[kTkMaxN];
#pragma unroll
    for (int f = 0; f < kTkMaxN; ++f) s[f] = 0.0f;
    int rmax = 0;
    for (int f = 0; f < N; ++f) rmax = max(rmax, m.rows[f]);
    for (int r = g; r < rmax; r += 32) {
      float v[kTkMaxN];
#pragma unroll
      for (int f = 0; f < kTkMaxN; ++f) v[f] = f < N ? m.F[f].at(r, c, m.rows[f]) : 0.0f;
#pragma unroll
      for (int f = 0; f < kTkMaxN; ++f) s[f] += v[f];
    }
#pragma unroll
    for (int f = 0; f < kTkMaxN; ++f) red[f][g][c] = s[f];
    __syncthreads();
    if (t < N * 32) {
      const int f = t >> 5;
      float acc = 0.0f;
      for (int q = 0; q < 32; ++q) acc += red[f][q][c];
      S[f][c] = acc;
    }
    __syncthreads();
  }
  // the column sums go out too (after the denominators), for the model's mass
  if (blockIdx.x == 0 && blockIdx.y == 0 && t < N * 32) den[kTkMaxN * kRP + t] = S[t >> 5][t & 31];
  const int n = blockIdx.y, j = blockIdx.x;
  if (n == N) {
    int rows = 1;
    for (int q = 0; q < N - 1; ++q) rows *= m.J[q];
    for (int e = j * kDenThreads + t; e < rows * kRP; e += gridDim.x * kDenThreads) {
      const int d = e & 31;
      float v = 0.0f;
      if (d < m.J[N - 1]) {
        v = S[N - 1][d];
        int rem = e >> 5;
        for (int q = N - 2; q >= 0; --q) {
          v *= S[q][rem % m.J[q]];
          rem /= m.J[q];
        }
      }
      dcore[e] = v;
    }
    return;
  }
  if (j >= kRP) return;
  float acc = 0.0f;
  if (j < m.J[n]) {
    int others = 1;
    for (int q = 0; q < N; ++q)
      if (q != n) others *= m.J[q];
    for (int o0 = t; o0 < others; o0 += kDenBatch * kDenThreads) {
      // kDenBatch entries per thread, their loads issued together
      int offs[kDenBatch];
      float ws[kDenBatch];
#pragma unroll
      for (int u = 0; u < kDenBatch; ++u) {
        const int o = o0 + u * kDenThreads;
        int off = 0;
        float w = 0.0f;
        if (o < others) {
          // indices of the other modes from o (last mode fastest), j at mode n
          int rem = o, mul = 1;
          w = 1.0f;
          for (int q = N - 1; q >= 0; --q) {
            int iq = j;
            if (q != n) {
              iq = rem % m.J[q];
              rem /= m.J[q];
              w *= S[q][iq];
            }
            if (q == N - 1) {
              off = iq;
              mul = kRP;
            } else {
              off += iq * mul;
              mul *= m.J[q];
            }
          }
        }
        offs[u] = off;
        ws[u] = w;
      }
      float gv[kDenBatch];
#pragma unroll
      for (int u = 0; u < kDenBatch; ++u) gv[u] = m.G[offs[u]];
#pragma unroll
      for (int u = 0; u < kDenBatch; ++u) acc += gv[u] * ws[u];
    }
  }
  part[t] = acc;
  __syncthreads();
  for (int h = kDenThreads / 2; h > 0; h >>= 1) {
    if (t < h) part[t] += part[t + h];
    __syncthreads();
  }
  if (t == 0) den[n * kRP + j] = j < m.J[n] ? part[0] : 0.0f;
}

// Total mass of the model, sum over the cells of Xhat = sum_j G[j] prod_m
// S_m[j_m] = sum_a den[0][a] S_1[a], from the closed-form denominators and
// the column sums that tkn_den_closed_kernel leaves behind them; float64,
// fixed order (one wavefront).
__global__ void __launch_bounds__(64) tkn_mass_kernel(const float* den, double* out) {
  const int t = threadIdx.x;
  double s = t < 32 ? (double)den[t] * (double)den[kTkMaxN * kRP + t] : 0.0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if (t == 0) out[0] = s;
}

namespace {

struct TkNCopy {
  float* core;            // [CR][32]
  float* fac[kTkMaxN];    // [I_n][32]; the fibre mode [Kp][32]
  float* facTL;           // fibre mode transposed [32][Kp]
};

struct TkNWs {
  int N, G;
  int dims[kTkMaxN], J[kTkMaxN];
  int64_t np;             // rows of the view: I_1 ... I_{N-1}
  int64_t Pp;             // np rounded up to 32
  int64_t CR;             // core rows: J_1 ... J_{N-1}
  int Kp, tpw, npg;
  int64_t vwgs;
  float* Tr;              // rebuild table [np][32]
  float* TT[2];           // the contraction sets' tables, transposed [32][Pp]
  float* V[2];            // V pass outputs [np][32]; scratch for the sets' tables
  float* m3[2];           // fibre-mode partial slots [npg][Kp][32]
  double* obj_part;
  float* PA[2];           // ping-pong buffers of the mode-product chains
  float* PB[2];
  float* slots[2];
  float* den_vec;         // [N][32] denominators, then [N][32] column sums
  float* dcore;           // [CR][32]
  TkNCopy ref, cur, num, den;
  float *Pc, *Qc;
  size_t bytes;
};

// Leading-core-index batches and K splits of the grouped-mode GEMM.
void mode_gemm_shape(const TkNWs& w, int n, int64_t* P, int64_t* K, int* splits) {
  int64_t pre = 1, post = 1;
  for (int q = 0; q < n; ++q) pre *= w.J[q];
  for (int q = n + 1; q < w.G; ++q) post *= w.J[q];
  *P = pre;
  *K = post * kRP;
  *splits = (int)std::max<int64_t>(1, std::min<int64_t>(8, 32 / pre));
}

// Extents of the tensor after each step of a chain over `order` (count steps),
// starting from ext; returns the largest intermediate in floats, the last
// step's output counted only when count_last.
size_t chain_peak(const TkNWs& w, int* ext, const int* order, int count, bool contract, bool count_last) {
  size_t peak = 0;
  for (int s = 0; s < count; ++s) {
    ext[order[s]] = contract ? w.J[order[s]] : w.dims[order[s]];
    if (s == count - 1 && !count_last) break;
    size_t sz = kRP;
    for (int q = 0; q < w.G; ++q) sz *= (size_t)ext[q];
    peak = std::max(peak, sz);
  }
  return peak;
}

// Contract order for block b (-1 = core): grouped modes G-1 .. 0, skipping b.
int contract_order(const TkNWs& w, int b, int* order) {
  int k = 0;
  for (int m = w.G - 1; m >= 0; --m)
    if (m != b) order[k++] = m;
  return k;
}

TkNWs tkn_layout(const comm_dense* x, const comm_model* md, char* base, bool cache) {
  TkNWs w = {};
  w.N = x->ndim;
  w.G = w.N - 1;
  for (int n = 0; n < w.N; ++n) {
    w.dims[n] = (int)x->dims[n];
    w.J[n] = (int)md->core_dims[n];
  }
  w.np = 1;
  w.CR = 1;
  for (int q = 0; q < w.G; ++q) {
    w.np *= w.dims[q];
    w.CR *= w.J[q];
  }
  w.Pp = (w.np + 31) / 32 * 32;
  const int IL = w.dims[w.N - 1];
  w.Kp = (IL + 31) / 32 * 32;
  tk_m3_tiling((int)w.np, 1, &w.tpw, &w.npg);
  w.vwgs = tk_v_workgroups((int)w.np, 1);
  // chains: the table (expand G-1 .. 0, the last step into the table) and,
  // per block, the contraction of V
  size_t pp = 0;
  {
    int ext[kTkMaxG], order[kTkMaxG];
    for (int q = 0; q < w.G; ++q) ext[q] = w.J[q];
    const int k = contract_order(w, -1, order);
    pp = std::max(pp, chain_peak(w, ext, order, k, false, false));
    for (int b = -1; b < w.G; ++b) {
      for (int q = 0; q < w.G; ++q) ext[q] = w.dims[q];
      const int kb = contract_order(w, b, order);
      pp = std::max(pp, chain_peak(w, ext, order, kb, true, true));
    }
  }
  size_t sl = 0;
  for (int n = 0; n < w.G; ++n) {
    int64_t P, K;
    int splits;
    mode_gemm_shape(w, n, &P, &K, &splits);
    sl = std::max(sl, (size_t)P * splits * w.dims[n] * kRP);
  }
  const size_t core = (size_t)w.CR * kRP;
  Carve cv;
  cv.base = base;
  w.Tr = cv.take<float>((size_t)w.np * kRP);
  for (int k = 0; k < 2; ++k) {
    w.TT[k] = cv.take<float>((size_t)w.Pp * kRP);
    w.V[k] = cv.take<float>((size_t)w.np * kRP);
    w.m3[k] = cv.take<float>((size_t)w.npg * w.Kp * kRP);
    w.PA[k] = cv.take<float>(pp);
    w.PB[k] = cv.take<float>(pp);
    w.slots[k] = cv.take<float>(sl);
  }
  w.obj_part = cv.take<double>((size_t)w.vwgs);
  w.den_vec = cv.take<float>((size_t)2 * kTkMaxN * kRP);  // denominators, then the column sums
  w.dcore = cv.take<float>(core);
  for (TkNCopy* c : {&w.ref, &w.cur, &w.num, &w.den}) {
    c->core = cv.take<float>(core);
    for (int n = 0; n < w.G; ++n) c->fac[n] = cv.take<float>((size_t)w.dims[n] * kRP);
    c->fac[w.G] = cv.take<float>((size_t)w.Kp * kRP);
    c->facTL = cv.take<float>((size_t)w.Kp * kRP);
  }
  if (cache) {
    const size_t total = (size_t)w.np * IL;
    w.Pc = cv.take<float>(total);
    w.Qc = cv.take<float>(total);
  }
  w.bytes = cv.off + 256;
  return w;
}

TkNModel modeln(const TkNWs& w, const TkNCopy& c) {
  TkNModel t = {};
  t.N = w.N;
  t.G = c.core;
  for (int n = 0; n < w.N; ++n) {
    t.F[n] = FView{c.fac[n], kRP, w.J[n]};
    t.J[n] = w.J[n];
    t.rows[n] = w.dims[n];
  }
  return t;
}

// Caller's model into padded copies (and a second one): the core and the
// factors, at most kMaxModes sources per launch.
int tkn_pad(const comm_model* m, const TkNWs& w, const TkNCopy& dst, const TkNCopy* dst2, hipStream_t st) {
  PadArgs p = {};
  auto add = [&](const float* src, int rows, int rows_p, int cols, float* d1, float* d2, float* d1T, float* d2T) {
    const int f = p.nf++;
    p.src[f] = src;
    p.rows[f] = rows;
    p.rows_p[f] = rows_p;
    p.cols[f] = cols;
    p.ld[f] = cols;
    p.dst[f] = d1;
    p.dst2[f] = d2;
    p.dstT[f] = d1T;
    p.dst2T[f] = d2T;
  };
  add(m->core, (int)w.CR, (int)w.CR, w.J[w.N - 1], dst.core, dst2 ? dst2->core : nullptr, nullptr, nullptr);
  for (int n = 0; n < w.N; ++n) {
    if (p.nf == kMaxModes) {
      HIP_TRY(launch_pad_factors(p, st));
      p = PadArgs{};
    }
    const bool last = n == w.N - 1;
    add(m->factors[n], w.dims[n], last ? w.Kp : w.dims[n], w.J[n], dst.fac[n], dst2 ? dst2->fac[n] : nullptr,
        last ? dst.facTL : nullptr, last && dst2 ? dst2->facTL : nullptr);
  }
  HIP_TRY(launch_pad_factors(p, st));
  return COMM_OK;
}

// Mode product of T viewed as L x I x R, for `sets` operand pairs at once:
// Y[l][j][r] = sum_{i < I} M(i, j) T[l][i][r].  contract: M(i, j) = F[i][j]
// (F a padded [I][32] factor, the sum runs over data rows: T x_n F^T; J <= 32);
// expand: M(i, j) = F[j][i] (F a padded [J][32] factor, the sum runs over a
// core index, I <= 32: T x_n F).  R is a multiple of 32.
//
// A streaming kernel rather than a matrix-core GEMM: one of I, J is at most
// 32 and R is long, so each thread owns one (l, r), walks i with loads that
// are contiguous in r across the wavefront, keeps up to 32 outputs in
// registers and writes them contiguous in r; the factor entries are the same
// for the whole wavefront.  Every input is read once (expand: once per 32
// outputs), every output written once, in a fixed order.
constexpr int kMpChunk = 32;

struct ModeProductArgs {
  const float* F[2];
  const float* T[2];
  float* Y[2];
  int64_t L, R;
  int I, J;
};

template <bool kContract>
__global__ void __launch_bounds__(256) mode_product_kernel(ModeProductArgs a) {
  const int set = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.L * a.R) return;
  const int64_t l = e / a.R, r = e - l * a.R;
  const float* __restrict__ F = a.F[set];
  const float* __restrict__ t = a.T[set] + l * a.I * a.R + r;
  float* __restrict__ y = a.Y[set] + l * a.J * a.R + r;
  for (int j0 = 0; j0 < a.J; j0 += kMpChunk) {
    float acc[kMpChunk];
#pragma unroll
    for (int jj = 0; jj < kMpChunk; ++jj) acc[jj] = 0.0f;
    for (int i = 0; i < a.I; ++i) {
      const float v = t[(int64_t)i * a.R];
#pragma unroll
      for (int jj = 0; jj < kMpChunk; ++jj) {
        // contract: columns of a padded [I][32] row (zero past J); expand:
        // rows j0 + jj < J of a padded [J][32] factor
        float mf = 0.0f;
        if (kContract) mf = F[(int64_t)i * kRP + jj];
        else if (j0 + jj < a.J) mf = F[(int64_t)(j0 + jj) * kRP + i];
        acc[jj] = fmaf(mf, v, acc[jj]);
      }
    }
#pragma unroll
    for (int jj = 0; jj < kMpChunk; ++jj)
      if (j0 + jj < a.J) y[(int64_t)(j0 + jj) * a.R] = acc[jj];
  }
}

// Contract with a long summed index (data rows): the workgroup's four waves
// own the same 64 positions and a quarter of i each; wave 0 adds the other
// waves' partial sums in order 1, 2, 3.
template <int kJC>
__global__ void __launch_bounds__(256) mode_contract_split_kernel(ModeProductArgs a) {
  __shared__ float red[3][kJC][64];
  const int set = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  const bool live = e < a.L * a.R;
  const int64_t l = live ? e / a.R : 0, r = live ? e - l * a.R : 0;
  const float* __restrict__ F = a.F[set];
  const float* __restrict__ t = a.T[set] + l * a.I * a.R + r;
  const int per = (a.I + 3) / 4;
  const int i0 = min(a.I, wv * per), i1 = min(a.I, i0 + per);
  float acc[kJC];
#pragma unroll
  for (int jj = 0; jj < kJC; ++jj) acc[jj] = 0.0f;
  if (live) {
#pragma unroll 4
    for (int i = i0; i < i1; ++i) {
      const float v = t[(int64_t)i * a.R];
#pragma unroll
      for (int jj = 0; jj < kJC; ++jj) acc[jj] = fmaf(F[(int64_t)i * kRP + jj], v, acc[jj]);
    }
  }
  if (wv > 0) {
#pragma unroll
    for (int jj = 0; jj < kJC; ++jj) red[wv - 1][jj][lane] = acc[jj];
  }
  __syncthreads();
  if (wv == 0 && live) {
    float* __restrict__ y = a.Y[set] + l * a.J * a.R + r;
#pragma unroll
    for (int jj = 0; jj < kJC; ++jj) {
      const float s = ((acc[jj] + red[0][jj][lane]) + red[1][jj][lane]) + red[2][jj][lane];
      if (jj < a.J) y[(int64_t)jj * a.R] = s;
    }
  }
}

int mode_product(const float* const* F, const float* const* T, float* const* Y, int sets, int64_t L, int I, int J,
                 int64_t R, bool contract, hipStream_t st) {
  if (contract ? J > kRP : I > kRP) return fail(COMM_EHIP, "mode product with %d x %d outside the 32-wide tile", I, J);
  ModeProductArgs a = {};
  for (int k = 0; k < sets; ++k) {
    a.F[k] = F[k];
    a.T[k] = T[k];
    a.Y[k] = Y[k];
  }
  a.L = L;
  a.R = R;
  a.I = I;
  a.J = J;
  if (contract && I >= 16) {
    // accumulators for the J <= 32 outputs in buckets of 8, 16 or 32
    const dim3 grid((unsigned)((L * R + 63) / 64), (unsigned)sets);
    if (J <= 8) hipLaunchKernelGGL(mode_contract_split_kernel<8>, grid, dim3(256), 0, st, a);
    else if (J <= 16) hipLaunchKernelGGL(mode_contract_split_kernel<16>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(mode_contract_split_kernel<32>, grid, dim3(256), 0, st, a);
  } else {
    const dim3 grid((unsigned)((L * R + 255) / 256), (unsigned)sets);
    if (contract) hipLaunchKernelGGL(mode_product_kernel<true>, grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL(mode_product_kernel<false>, grid, dim3(256), 0, st, a);
  }
  HIP_TRY(hipGetLastError());
  return COMM_OK;
}

// Mode products over `order`, one mode at a time, for `sets` tensors of
// extents ext[0..G-1] x 32 (updated): contract (I_m -> J_m) or expand
// (J_m -> I_m) with factor m of each model.  Intermediates alternate between
// the ping-pong buffers; the last result goes to dst when given.  out[k]
// receives the buffer holding set k's result.
int chain(const TkNWs& w, const float* const* src, int sets, int* ext, const int* order, int count, bool contract,
          const TkNModel* ms, float* const* dst, const float** out, hipStream_t st) {
  const float* cur[2] = {src[0], sets > 1 ? src[1] : nullptr};
  for (int s = 0; s < count; ++s) {
    const int m = order[s];
    int64_t L = 1, R = kRP;
    for (int q = 0; q < m; ++q) L *= ext[q];
    for (int q = m + 1; q < w.G; ++q) R *= ext[q];
    const int I = ext[m], J = contract ? w.J[m] : w.dims[m];
    float* nxt[2] = {nullptr, nullptr};
    const bool last = s == count - 1;
    for (int k = 0; k < sets; ++k) nxt[k] = (last && dst) ? dst[k] : (s % 2 == 0 ? w.PA[k] : w.PB[k]);
    const float* F[2] = {ms[0].F[m].p, sets > 1 ? ms[1].F[m].p : nullptr};
    int rc = mode_product(F, cur, nxt, sets, L, I, J, R, contract, st);
    if (rc) return rc;
    ext[m] = J;
    for (int k = 0; k < sets; ++k) cur[k] = nxt[k];
  }
  for (int k = 0; k < sets; ++k) out[k] = cur[k];
  return COMM_OK;
}

// Tables of `sets` models into dst[k] ([np][32]).
int tkn_table(const TkNWs& w, const TkNModel* md, int sets, float* const* dst, hipStream_t st) {
  int ext[kTkMaxG], order[kTkMaxG];
  for (int q = 0; q < w.G; ++q) ext[q] = w.J[q];
  const int k = contract_order(w, -1, order);
  const float* src[2] = {md[0].G, sets > 1 ? md[1].G : nullptr};
  const float* out[2];
  return chain(w, src, sets, ext, order, k, false, md, dst, out, st);
}

int tkn_transpose(const TkNWs& w, const float* in, float* out, hipStream_t st) {
  hipLaunchKernelGGL(rows32_transpose_kernel, dim3((unsigned)((w.Pp + 63) / 64)), dim3(256), 0, st, in, w.np, w.Pp,
                     out);
  HIP_TRY(hipGetLastError());
  return COMM_OK;
}

struct SlotsN {
  const float* part;
  int n;
  int rows_total;
};

// Numerator slots of block blk (-1 core, 0 .. G-1) from V[k] of the
// contraction sets cs[k] (k < sets; set 1 is the denominator's).
int tkn_numerators(const TkNWs& w, int blk, const TkNModel* cs, int sets, SlotsN* out, hipStream_t st) {
  int ext[kTkMaxG], order[kTkMaxG];
  for (int q = 0; q < w.G; ++q) ext[q] = w.dims[q];
  const int k = contract_order(w, blk, order);
  const float* src[2] = {w.V[0], w.V[1]};
  const float* Z[2];
  int rc = chain(w, src, sets, ext, order, k, true, cs, nullptr, Z, st);
  if (rc) return rc;
  if (blk == -1) {
    for (int q = 0; q < sets; ++q) out[q] = SlotsN{Z[q], 1, (int)w.CR};
    return COMM_OK;
  }
  // Num[i][j] = sum_{p < P} sum_{k < K} Z[p][i][k] G'[p][j][k], one slot per
  // (split, p)
  int64_t P, K;
  int splits;
  mode_gemm_shape(w, blk, &P, &K, &splits);
  const int In = w.dims[blk], Jn = w.J[blk];
  GemmArgs g = {};
  g.sab = (int64_t)In * K;
  g.sam = K;
  g.saki = 1;
  g.akin_log2 = 30;
  g.sbb = (int64_t)Jn * K;
  g.sbki = 1;
  g.sbn = K;
  g.bkin_log2 = 30;
  g.sob = (int64_t)In * kRP;
  g.sos = P * In * kRP;
  g.ldo = kRP;
  g.M = In;
  g.N = Jn;
  g.K = (int)K;
  g.batch = (int)P;
  g.splits = splits;
  g.sets = sets;
  for (int q = 0; q < sets; ++q) {
    g.A[q] = Z[q];
    g.B[q] = cs[q].G;
    g.out[q] = w.slots[q];
    out[q] = SlotsN{w.slots[q], (int)(P * splits), In};
  }
  HIP_TRY(launch_gemm(g, st));
  return COMM_OK;
}

TkPassArgs passn_args(const comm_dense* x, const comm_opts* o, const TkNWs& w) {
  TkPassArgs a = {};
  a.X = x->X;
  a.I = (int)w.np;
  a.J = 1;
  a.K = w.dims[w.N - 1];
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
  a.xvec = (a.K % 4 == 0) && (reinterpret_cast<uintptr_t>(x->X) % 16 == 0);
  a.bf16 = o->precision == COMM_BF16;
  return a;
}

FView block_viewn(const TkNModel& t, int blk) {
  if (blk == -1) return FView{t.G, kRP, t.J[t.N - 1]};
  return t.F[blk];
}

float* copy_blockn(const TkNCopy& c, int blk) { return blk == -1 ? c.core : c.fac[blk]; }

// One block update: max(anchor * (Num/Den)^gamma, eps) into the caller's block
// and the padded copy `pad` (the fibre mode also its transposed copy).
int tkn_apply(const comm_model* m, const TkNWs& w, int blk, const SlotsN& num, const SlotsN* den,
              const float* den_closed_vec, FView anchor, const TkNCopy& pad, float gamma, float eps,
              hipStream_t st) {
  const int last = w.N - 1;
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
    Jb.rows = (int)w.CR;
    Jb.cols = w.J[last];
    Jb.out_user = m->core;
    Jb.ld_user = w.J[last];
  } else {
    Jb.rows = w.dims[blk];
    Jb.cols = w.J[blk];
    Jb.out_user = m->factors[blk];
    Jb.ld_user = w.J[blk];
  }
  Jb.rows_p = blk == last ? w.Kp : Jb.rows;
  Jb.anchor = anchor;
  Jb.gamma = gamma;
  Jb.eps = eps;
  Jb.out_pad = copy_blockn(pad, blk);
  Jb.out_padT = blk == last ? pad.facTL : nullptr;
  HIP_TRY(launch_slot_update(u, st));
  return COMM_OK;
}

CooTkArgs coo_tk_args(const TkSparse* sp, const TkNWs& w, const comm_opts* o, const float* Tr, FView Cr) {
  CooTkArgs a = {};
  const comm_coo* x = sp->coo;
  a.N = x->ndim;
  a.nnz = x->nnz;
  for (int n = 0; n < x->ndim; ++n) {
    a.dims[n] = (int)x->dims[n];
    a.idx[n] = x->idx[n];
  }
  a.val = x->val;
  a.Tr = Tr;
  a.Cr = Cr;
  a.bc = make_beta_const(o->beta);
  a.eps = (float)o->eps;
  (void)w;
  return a;
}

// Update of block blk with X rebuilt from w.Tr and the fibre-mode factor cl
// (or read from the cached P~ / Q~), contraction sets ns / ds (their fibre-mode
// factors transposed in cnT / cdT; for the fibre block their tables in w.TT).
// With sp (sparse data) the numerator comes from the nonzeros: weights
// rebuilt from (w.Tr, cl) or, when stored, taken from sp->w; tnum is the
// contraction set's table in row layout (fibre block).
int tkn_block(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, const TkNWs& w, int blk,
              FView cl, const TkNModel& ns, const TkNModel& ds, const float* cnT, const float* cdT, bool cached,
              bool want_obj, FView anchor, const TkNCopy& pad, double* obj, hipStream_t st,
              const TkSparse* sp = nullptr, const float* tnum = nullptr, bool stored = false,
              bool reuse_v = false) {
  const bool kl = o->beta == 1.0;
  const int sets = kl ? 1 : 2;
  const int bc = beta_class_of(o->beta);
  const int mode = cached ? kTkCacheRead : kTkFromX;
  TkPassArgs a = passn_args(x, o, w);
  a.T2r = w.Tr;
  a.C = cl;
  if (cached) {
    a.Pc = w.Pc;
    a.Qc = w.Qc;
  }
  SlotsN num, den;
  int rc;
  // sparse data at beta = 1: the dense passes would only give numerators
  const bool dense_pass = !(sp && kl);
  CooTkArgs sa = {};
  if (sp) {
    sa = coo_tk_args(sp, w, o, w.Tr, cl);
    if (stored) sa.w_in = sp->w;
  }
  if (blk == w.N - 1) {
    a.T2nT = w.TT[0];
    a.T2dT = w.TT[1];
    if (dense_pass) {
      rc = profiled(ctx, st, [&] { return launch_tk_m3(a, bc, mode, sets, st); });
      if (rc) return rc;
    }
    num = SlotsN{w.m3[0], w.npg, w.Kp};
    den = SlotsN{w.m3[1], w.npg, w.Kp};
    if (sp) {
      HIP_TRY(launch_fill_zero(sp->buf, (int64_t)w.Kp * kRP, st));
      sa.op = 2;
      sa.Tc = tnum;
      sa.out = sp->buf;
      HIP_TRY(launch_coo_tucker(sa, bc, st));
      num = SlotsN{sp->buf, 1, w.Kp};
    }
  } else {
    a.CnT = cnT;
    a.CdT = cdT;
    // reuse_v: V of this sweep's core block still holds (its last-mode sets
    // have not changed since)
    if (dense_pass && !reuse_v) {
      rc = profiled(ctx, st, [&] { return launch_tk_v(a, bc, mode, want_obj, sets, st); });
      if (rc) return rc;
      if (want_obj && obj) HIP_TRY(launch_sum_f64(w.obj_part, w.vwgs, nullptr, obj, st));
    }
    if (sp && !reuse_v) {
      // V of the numerator from the nonzeros (the dense pass left it zero)
      HIP_TRY(launch_fill_zero(w.V[0], w.np * kRP, st));
      sa.op = 1;
      sa.Cc = ns.F[w.N - 1];
      sa.out = w.V[0];
      HIP_TRY(launch_coo_tucker(sa, bc, st));
    }
    const TkNModel cs[2] = {ns, ds};
    SlotsN nd[2];
    if ((rc = tkn_numerators(w, blk, cs, sets, nd, st))) return rc;
    num = nd[0];
    den = nd[1];
  }
  const float* vec = nullptr;
  const SlotsN* denp = &den;
  SlotsN dcore;
  if (kl) {
    hipLaunchKernelGGL(tkn_den_closed_kernel, dim3(kRP, w.N + 1), dim3(kDenThreads), 0, st, ds, w.den_vec, w.dcore);
    HIP_TRY(hipGetLastError());
    if (blk == -1) {
      dcore = SlotsN{w.dcore, 1, (int)w.CR};
      denp = &dcore;
    } else {
      vec = w.den_vec + blk * kRP;
      denp = nullptr;
    }
  }
  return tkn_apply(m, w, blk, num, denp, vec, anchor, pad, gamma_of(o->beta), (float)o->eps, st);
}

}  // namespace
}  // namespace comm

using namespace comm;

size_t tuckern_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op) {
  const bool cache = op == 1 && o->cache_pq && o->beta != 1.0;
  return tkn_layout(x, m, nullptr, cache).bytes;
}

int tuckern_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st,
                  const TkSparse* sp) {
  TkNWs w = tkn_layout(x, m, nullptr, false);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tkn_layout(x, m, ctx->ws, false);
  if ((rc = tkn_pad(m, w, w.cur, nullptr, st))) return rc;
  const TkNModel cur = modeln(w, w.cur);
  const int last = w.N - 1;
  const int nb = block == -2 ? w.N + 1 : 1;
  for (int q = 0; q < nb; ++q) {
    const int blk = block == -2 ? q - 1 : block;
    // block-MM rebuilds from the current model before every block; the
    // contraction sets are the current model too
    if ((rc = tkn_table(w, &cur, 1, &w.Tr, st))) return rc;
    if (blk == last) {
      if ((rc = tkn_transpose(w, w.Tr, w.TT[0], st))) return rc;
      TkNWs w2 = w;
      w2.TT[1] = w.TT[0];
      rc = tkn_block(ctx, x, m, o, w2, blk, cur.F[last], cur, cur, nullptr, nullptr, false, false,
                     block_viewn(cur, blk), w.cur, nullptr, st, sp, w.Tr);
    } else {
      rc = tkn_block(ctx, x, m, o, w, blk, cur.F[last], cur, cur, w.cur.facTL, w.cur.facTL, false, false,
                     block_viewn(cur, blk), w.cur, nullptr, st, sp, w.Tr);
    }
    if (rc) return rc;
  }
  return COMM_OK;
}

int tuckern_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st,
                  const TkSparse* sp) {
  const bool kl = o->beta == 1.0;
  const bool cache = o->cache_pq && !kl && !sp;
  TkNWs w = tkn_layout(x, m, nullptr, cache);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tkn_layout(x, m, ctx->ws, cache);
  if ((rc = tkn_pad(m, w, w.ref, &w.cur, st))) return rc;
  const TkNModel ref = modeln(w, w.ref);
  const int last = w.N - 1;
  // the reference, and so its table, is fixed for the whole outer iteration
  if ((rc = tkn_table(w, &ref, 1, &w.Tr, st))) return rc;
  bool obj_pending = obj != nullptr;
  if (sp) {
    // the nonzeros' weights at the reference, kept for the inner sweeps, and
    // their objective corrections (added once the zero cells' part is written)
    CooTkArgs sa = coo_tk_args(sp, w, o, w.Tr, ref.F[last]);
    sa.w_out = sp->w;
    sa.obj_part = obj ? sp->obj : nullptr;
    HIP_TRY(launch_coo_tucker(sa, beta_class_of(o->beta), st));
    if (kl && obj) {
      // no dense pass at beta = 1: the zero cells contribute sum Xhat, the
      // model's total mass, from the closed-form denominators' column sums
      hipLaunchKernelGGL(tkn_den_closed_kernel, dim3(kRP, w.N + 1), dim3(kDenThreads), 0, st, ref, w.den_vec, w.dcore);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(tkn_mass_kernel, dim3(1), dim3(64), 0, st, w.den_vec, obj);
      HIP_TRY(hipGetLastError());
      obj_pending = false;
    }
  }
  if (cache) {
    TkPassArgs a = passn_args(x, o, w);
    a.T2r = w.Tr;
    a.C = ref.F[last];
    a.Pw = w.Pc;
    a.Qw = w.Qc;
    rc = profiled(ctx, st, [&] { return launch_tk_v(a, beta_class_of(o->beta), kTkCacheWrite, obj_pending, 0, st); });
    if (rc) return rc;
    if (obj_pending) HIP_TRY(launch_sum_f64(w.obj_part, w.vwgs, nullptr, obj, st));
    obj_pending = false;
  }
  const float beta = (float)o->beta;
  for (int l = 0; l < o->inner_sweeps; ++l) {
    for (int blk = -1; blk < w.N; ++blk) {
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
      if (blk != -1) add(w.cur.core, w.ref.core, (int)w.CR, w.num.core, w.den.core);
      for (int q = 0; q < w.N; ++q)
        if (q != blk) {
          add(w.cur.fac[q], w.ref.fac[q], q == last ? w.Kp : w.dims[q], w.num.fac[q], w.den.fac[q]);
          if (q == last) {
            ca.x1T[ca.nf - 1] = w.num.facTL;
            ca.x2T[ca.nf - 1] = w.den.facTL;
          }
        }
      HIP_TRY(launch_chi(ca, st));
      TkNModel ns = modeln(w, w.num), ds = modeln(w, w.den);
      // the active block does not enter its own contraction
      if (blk == -1) {
        ns.G = ref.G;
        ds.G = ref.G;
      } else {
        ns.F[blk] = ref.F[blk];
        ds.F[blk] = ref.F[blk];
      }
      if (blk == last) {
        const TkNModel sets[2] = {ns, ds};
        if ((rc = tkn_table(w, sets, kl ? 1 : 2, w.V, st))) return rc;
        for (int k = 0; k < (kl ? 1 : 2); ++k)
          if ((rc = tkn_transpose(w, w.V[k], w.TT[k], st))) return rc;
      }
      // one V pass per sweep: the core block's V serves every block but the
      // last mode (whose sets enter V and change only at the last block)
      rc = tkn_block(ctx, x, m, o, w, blk, ref.F[last], ns, ds, w.num.facTL, w.den.facTL, cache, obj_pending,
                     block_viewn(ref, blk), w.cur, obj, st, sp, w.V[0], true, blk >= 0 && blk < last);
      if (rc) return rc;
      obj_pending = false;
    }
  }
  if (sp && obj) HIP_TRY(launch_sum_f64(sp->obj, coo_beta_blocks(sp->coo->nnz), obj, obj, st));
  return COMM_OK;
}

int tuckern_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                      hipStream_t st, const TkSparse* sp) {
  TkNWs w = tkn_layout(x, m, nullptr, false);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = tkn_layout(x, m, ctx->ws, false);
  if ((rc = tkn_pad(m, w, w.cur, nullptr, st))) return rc;
  const TkNModel cur = modeln(w, w.cur);
  if ((rc = tkn_table(w, &cur, 1, &w.Tr, st))) return rc;
  TkPassArgs a = passn_args(x, o, w);
  a.T2r = w.Tr;
  a.C = cur.F[w.N - 1];
  rc = profiled(ctx, st, [&] { return launch_tk_v(a, beta_class_of(o->beta), kTkFromX, true, 0, st); });
  if (rc) return rc;
  HIP_TRY(launch_sum_f64(w.obj_part, w.vwgs, nullptr, out, st));
  if (sp) {
    CooTkArgs sa = coo_tk_args(sp, w, o, w.Tr, cur.F[w.N - 1]);
    sa.obj_part = sp->obj;
    HIP_TRY(launch_coo_tucker(sa, beta_class_of(o->beta), st));
    HIP_TRY(launch_sum_f64(sp->obj, coo_beta_blocks(sp->coo->nnz), out, out, st));
  }
  return COMM_OK;
}
