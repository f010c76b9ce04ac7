// Factor-side kernels: padding copies, column sums, the J-CoMM transforms
// chi_1 / chi_2 (Sec. 5.3), the reduction of the pass's partial slots fused
// with the multiplicative block update and its eps floor (Theorem "CP block
// multiplicative update"; Sec. 5.3 inner update), the fixed-order float64
// reduction of objective partials, and the beta = 1 inner loop of J-CoMM for
// CP.  Every reduction has a fixed order, so results are bitwise
// deterministic.

#include "group.h"
#include "kernels.h"

namespace comm {

// ----------------------------------------------------------------------------------------
// Padding copies of up to 4 factors in one launch.

__device__ __forceinline__ void pad_factors_body(const PadArgs& a, uint3 bid, uint3) {
  int64_t e = (int64_t)bid.x * blockDim.x + threadIdx.x;
  int f = 0;
  while (f < a.nf && e >= (int64_t)a.rows_p[f] * kRP) {
    e -= (int64_t)a.rows_p[f] * kRP;
    ++f;
  }
  if (f >= a.nf) return;
  const int row = (int)(e / kRP), c = (int)(e % kRP);
  const float v = (row < a.rows[f] && c < a.cols[f]) ? a.src[f][(int64_t)row * a.ld[f] + c] : 0.0f;
  a.dst[f][e] = v;
  if (a.dstT[f]) a.dstT[f][(int64_t)c * a.rows_p[f] + row] = v;
  if (a.dst2[f]) a.dst2[f][e] = v;
  if (a.dst2T[f]) a.dst2T[f][(int64_t)c * a.rows_p[f] + row] = v;
}
COMM_GROUPED_KERNELS(pad_factors, PadArgs, 256)

hipError_t launch_pad_factors(const PadArgs& a, hipStream_t s) {
  int64_t n = 0;
  for (int f = 0; f < a.nf; ++f) n += (int64_t)a.rows_p[f] * kRP;
  return launch_or_record(pad_factors_kernel, pad_factors_grouped, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                          a);
}

// ----------------------------------------------------------------------------------------
// Column sums: one workgroup, 8 row groups x 32 columns, fixed order.

struct ColsumArgs {
  FView F[kMaxModes];
  int rows[kMaxModes];
  int nf;
  float* prod;       // prod[c] = product over the nf factors of the column sums
};

__device__ __forceinline__ void colsum_prod_body(const ColsumArgs& a, uint3, uint3) {
  __shared__ float part[8 * 32];
  __shared__ float res[kMaxModes][32];
  const int t = threadIdx.x;
  const int c = t & 31, g = t >> 5;
  for (int f = 0; f < a.nf; ++f) {
    float s = 0.0f;
    for (int r = g; r < a.rows[f]; r += 8) s += a.F[f].at(r, c, a.rows[f]);
    part[g * 32 + c] = s;
    __syncthreads();
    if (t < 32) {
      float acc = part[t];
      for (int q = 1; q < 8; ++q) acc += part[q * 32 + t];
      res[f][t] = acc;
    }
    __syncthreads();
  }
  if (t < 32) {
    float p = 1.0f;
    for (int f = 0; f < a.nf; ++f) p *= res[f][t];
    a.prod[t] = p;
  }
}
COMM_GROUPED_KERNELS(colsum_prod, ColsumArgs, 256)

hipError_t launch_colsum_prod(const FView* F, const int* rows, int nf, float* prod, hipStream_t s) {
  ColsumArgs a = {};
  for (int f = 0; f < nf; ++f) {
    a.F[f] = F[f];
    a.rows[f] = rows[f];
  }
  a.nf = nf;
  a.prod = prod;
  return launch_or_record(colsum_prod_kernel, colsum_prod_grouped, dim3(1), dim3(256), 0, s, a);
}

// ----------------------------------------------------------------------------------------
// chi transforms of up to 4 factors in one launch

// chi_1 = Z~ (Z/Z~)^(beta-1);  chi_2 = Z (beta <= 1) or Z~ (Z/Z~)^beta; zero
// where Z~ is (the padding).
__device__ __forceinline__ void chi_pair(float z, float zr, float beta, float& c1, float& c2) {
  c1 = 0.0f;
  c2 = 0.0f;
  if (zr > 0.0f) {
    const float u = z / zr;
    const float lu = __builtin_amdgcn_logf(u);
    c1 = (beta == 1.0f) ? zr : zr * __builtin_amdgcn_exp2f((beta - 1.0f) * lu);
    c2 = (beta <= 1.0f) ? z : zr * __builtin_amdgcn_exp2f(beta * lu);
  }
}

__device__ __forceinline__ void chi_body(const ChiArgs& a, uint3 bid, uint3) {
  int64_t e = (int64_t)bid.x * blockDim.x + threadIdx.x;
  int f = 0;
  while (f < a.nf && e >= (int64_t)a.rows_p[f] * kRP) {
    e -= (int64_t)a.rows_p[f] * kRP;
    ++f;
  }
  if (f >= a.nf) return;
  float c1, c2;
  chi_pair(a.cur[f][e], a.ref[f][e], a.beta, c1, c2);
  a.x1[f][e] = c1;
  a.x2[f][e] = c2;
  const int row = (int)(e / kRP), c = (int)(e % kRP);
  if (a.x1T[f]) a.x1T[f][(int64_t)c * a.rows_p[f] + row] = c1;
  if (a.x2T[f]) a.x2T[f][(int64_t)c * a.rows_p[f] + row] = c2;
}
COMM_GROUPED_KERNELS(chi, ChiArgs, 256)

hipError_t launch_chi(const ChiArgs& a, hipStream_t s) {
  int64_t n = 0;
  for (int f = 0; f < a.nf; ++f) n += (int64_t)a.rows_p[f] * kRP;
  return launch_or_record(chi_kernel, chi_grouped, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
}

// ----------------------------------------------------------------------------------------
// float64 sum of objective partials, compensated, fixed order (valid in
// thread 0): each thread's partials, then the lanes of each wavefront, then
// the 16 wavefronts

__device__ double block_sum_f64(const double* __restrict__ part, int64_t n, double (*lds)[2]) {
  const int t = threadIdx.x;
  double s = 0.0, c = 0.0;
  for (int64_t e = t; e < n; e += 1024) sum2_add(s, c, part[e]);
  sum2_wave(s, c);
  if ((t & 63) == 0) {
    lds[t >> 6][0] = s;
    lds[t >> 6][1] = c;
  }
  __syncthreads();
  double S = lds[0][0], C = lds[0][1];
  for (int q = 1; q < 16; ++q) {
    sum2_add(S, C, lds[q][0]);
    C += lds[q][1];
  }
  return S + C;
}

struct SumF64Args {
  const double* part;
  int64_t n;
  const double* add_to;
  double* out;
};

__device__ __forceinline__ void sum_f64_body(const SumF64Args& a, uint3, uint3) {
  __shared__ double lds[16][2];
  const double s = block_sum_f64(a.part, a.n, lds);
  if (threadIdx.x == 0) a.out[0] = s + (a.add_to ? a.add_to[0] : 0.0);
}
COMM_GROUPED_KERNELS(sum_f64, SumF64Args, 1024)

hipError_t launch_sum_f64(const double* part, int64_t n, const double* add_to, double* out, hipStream_t s) {
  return launch_or_record(sum_f64_kernel, sum_f64_grouped, dim3(1), dim3(1024), 0, s, SumF64Args{part, n, add_to, out});
}

// ----------------------------------------------------------------------------------------
// beta = 1 J-CoMM inner loop (CP).
//
// At beta = 1, chi_1(A, A~) = A~ and chi_2(A, A~) = A, and Q~ = 1, so
//   Num_J^(n) depends only on the reference (computed in the reference pass),
//   Den_J^(n)(i, r) = prod_{m != n} S^(m)(r) with S^(m) the column sums of the
//   current inner block m,
// and the anchored update is A^(n) = max(c^(n) / Den^(n), eps) with
// c^(n) = A~^(n) * Num_J^(n).  The column sums of the new block are therefore
// S^(n)(r) = sum_i max(c^(n)(i, r) / Den(r), eps), which equals T^(n)(r) / Den(r)
// with T^(n) = sum_i c^(n)(i, r) whenever no entry of column r is clipped
// (min_i c^(n)(i, r) >= eps Den(r)); otherwise the column is summed exactly.
// The L sweeps thus reduce to recurrences on 32-wide vectors, run by one
// wavefront, plus one final elementwise pass.

// Recurrence of the beta = 1 inner loop: reduces the column statistics of
// every block (all loads in one round), sums the objective partials, runs the L
// sweeps on 32-wide vectors, and leaves the last denominators in den_last.
// Every workgroup of kl_apply runs it on the same data in the same order, so
// all of them agree bitwise without synchronising.
__device__ __forceinline__ void kl_objective_out(const KlLoopArgs& a, float (*S)[32], double (*lds64)[2]);

__device__ __forceinline__ void kl_recurrence(const KlLoopArgs& a, float (*den_last)[32], float (*S)[32],
                                              double (*lds64)[2], unsigned bx) {
  __shared__ float red[3 * kMaxModes][32][33];
  __shared__ float T[kMaxModes][32], Cmin[kMaxModes][32];
  const int t = threadIdx.x;
  const int c = t & 31, g = t >> 5;
  int nblk_max = 0;
#pragma unroll
  for (int n = 0; n < kMaxModes; ++n)
    if (n < a.N) nblk_max = max(nblk_max, a.nblk[n]);
  float acc[kMaxModes][3];
#pragma unroll
  for (int n = 0; n < kMaxModes; ++n) {
    acc[n][0] = 0.0f;
    acc[n][1] = 3.402823e38f;
    acc[n][2] = 0.0f;
  }
  // the first two objective partials go out with the statistics' first round;
  // the partials are added compensated (each thread's, then the lanes, then
  // the 16 wavefronts)
  double objs = 0.0, objc = 0.0;
  const double ob0 = (a.obj_part && t < a.obj_n) ? a.obj_part[t] : 0.0;
  const double ob1 = (a.obj_part && t + 1024 < a.obj_n) ? a.obj_part[t + 1024] : 0.0;
  for (int b0 = g; b0 < nblk_max; b0 += 4 * 32) {
    float v[4][kMaxModes][3];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int n = 0; n < kMaxModes; ++n)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int b = b0 + 32 * u;
          v[u][n][k] = (n < a.N && b < a.nblk[n]) ? a.stats[n][(int64_t)b * 96 + 32 * k + c]
                                                 : (k == 1 ? 3.402823e38f : 0.0f);
        }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int n = 0; n < kMaxModes; ++n) {
        acc[n][0] += v[u][n][0];
        acc[n][1] = fminf(acc[n][1], v[u][n][1]);
        acc[n][2] += v[u][n][2];
      }
  }
  objs = ob0;
  sum2_add(objs, objc, ob1);
  if (a.obj_part)
    for (int64_t e = t + 2048; e < a.obj_n; e += 1024) sum2_add(objs, objc, a.obj_part[e]);
  sum2_wave(objs, objc);
  if ((t & 63) == 0) {
    lds64[t >> 6][0] = objs;
    lds64[t >> 6][1] = objc;
  }
#pragma unroll
  for (int n = 0; n < kMaxModes; ++n)
#pragma unroll
    for (int k = 0; k < 3; ++k) red[3 * n + k][g][c] = acc[n][k];
  __syncthreads();
  if (t < 3 * kMaxModes * 32) {
    const int q = t >> 5;
    const int n = q / 3, k = q % 3;
    float s = red[q][0][c];
    for (int gg = 1; gg < 32; ++gg) s = (k == 1) ? fminf(s, red[q][gg][c]) : s + red[q][gg][c];
    if (n < a.N) {
      if (k == 0) T[n][c] = s;
      else if (k == 1) Cmin[n][c] = s;
      else S[n][c] = s;
    }
  }
  __syncthreads();
  if (a.obj_out && bx == 0 && t < 64) kl_objective_out(a, S, lds64);

  // Every thread runs the recurrence of column c = t & 31 (the 32 threads of a
  // column compute the same values in the same order).  A column whose
  // clipped entries make T / Den inexact is summed exactly by all 1024
  // threads: thread (g, c) takes rows g, g + 32, ..., sixteen in flight, and
  // the 32 partial sums are added in the order of g.
  {
    const int col = c;
    const bool real = col < a.R;
    float Sr[kMaxModes], Tr[kMaxModes], Cr[kMaxModes], Dl[kMaxModes];
#pragma unroll
    for (int n = 0; n < kMaxModes; ++n) {
      Sr[n] = n < a.N ? S[n][col] : 1.0f;
      Tr[n] = n < a.N ? T[n][col] : 0.0f;
      Cr[n] = n < a.N ? Cmin[n][col] : 0.0f;
      Dl[n] = 1.0f;
    }
    float (*part)[33] = red[0];   // the statistics' buffer, free again
    for (int l = 0; l < a.L; ++l) {
#pragma unroll
      for (int n = 0; n < kMaxModes; ++n) {
        if (n >= a.N) break;
        float d = 1.0f;
#pragma unroll
        for (int m = 0; m < kMaxModes; ++m)
          if (m != n && m < a.N) d *= Sr[m];
        const bool clip = real && (Cr[n] < a.eps * d);
        float snew = real ? Tr[n] / d : 0.0f;
        // every wavefront holds all 32 columns, so its vote is the block's
        if (__any(clip)) {
          float s = 0.0f;
          if (clip) {
            // batches of 32 rows per thread (1024 rows per round: a round
            // reads c written by the previous launch, often on another XCD),
            // the last one's loads clamped to a valid row and its rows past
            // the end left out of the sum (the rows are added in the same
            // order as one at a time)
            const float* cp = a.c[n] + col;
            const int rows = a.rows[n];
            for (int r = g; r < rows; r += 32 * 32) {
              float v[32];
#pragma unroll
              for (int u = 0; u < 32; ++u) v[u] = cp[(int64_t)min(r + 32 * u, rows - 1) * kRP];
#pragma unroll
              for (int u = 0; u < 32; ++u)
                if (r + 32 * u < rows) s += fmaxf(v[u] / d, a.eps);
            }
          }
          part[g][col] = s;
          __syncthreads();
          if (clip) {
            float exact = part[0][col];
            for (int gg = 1; gg < 32; ++gg) exact += part[gg][col];
            snew = exact;
          }
          __syncthreads();
        }
        Sr[n] = snew;
        Dl[n] = d;
      }
    }
    if (t < 32) {
#pragma unroll
      for (int n = 0; n < kMaxModes; ++n)
        if (n < a.N) den_last[n][col] = Dl[n];
    }
  }
}

// The objective at the reference, written by wavefront 0 of workgroup 0
// before the recurrence, all lanes at once so that the recurrence's barriers
// wait little for it: the 16 wavefront partials added compensated across
// lanes, plus, for sparse data, the model's mass over every cell,
// sum_r prod_n colsum(A~^(n))_r (one lane per r).
__device__ __forceinline__ void kl_objective_out(const KlLoopArgs& a, float (*S)[32], double (*lds64)[2]) {
  const int t = threadIdx.x;
  double s = t < 16 ? lds64[t][0] : 0.0, sc = t < 16 ? lds64[t][1] : 0.0;
  sum2_wave(s, sc);
  double mass = 0.0;
  if (a.obj_add_model_mass && t < a.R) {
    mass = 1.0;
    for (int n = 0; n < a.N; ++n) mass *= (double)S[n][t];
  }
  for (int off = 32; off > 0; off >>= 1) mass += __shfl_down(mass, off);
  if (t == 0) a.obj_out[0] = (s + sc) + mass;
}

// A^(n) = max(c^(n) / Den_last^(n), eps) for all modes; each workgroup first
// runs the recurrence itself.
__device__ __forceinline__ void kl_apply_body(const KlLoopArgs& a, uint3 bid, uint3 gdim) {
  __shared__ float den_last[kMaxModes][32];
  __shared__ float S[kMaxModes][32];
  __shared__ double lds64[16][2];
  int64_t first[kMaxModes + 1];
  first[0] = 0;
#pragma unroll
  for (int n = 0; n < kMaxModes; ++n) first[n + 1] = first[n] + (n < a.N ? (int64_t)a.rows[n] * kRP : 0);
  const int64_t total = first[kMaxModes];
  const int64_t stride = (int64_t)gdim.x * blockDim.x;
  const int64_t e00 = (int64_t)bid.x * blockDim.x + threadIdx.x;
  // The thread's first kApplyPre entries: their c values are loaded before
  // the recurrence, so that the round trip overlaps its loads.  An entry's
  // mode comes from selects over the (uniform) arguments: indexing the
  // argument arrays with a per-lane mode would load them per lane.
  constexpr int kApplyPre = 2;
  float cv[kApplyPre];
  int nn[kApplyPre];
  int64_t ee[kApplyPre];
#pragma unroll
  for (int k = 0; k < kApplyPre; ++k) {
    const int64_t e0 = e00 + k * stride;
    nn[k] = -1;
    ee[k] = 0;
    cv[k] = 0.0f;
    if (e0 < total) {
      int n = 0;
#pragma unroll
      for (int m = 1; m < kMaxModes; ++m) n += e0 >= first[m] ? 1 : 0;
      int64_t base = first[0];
      const float* cp = a.c[0];
#pragma unroll
      for (int m = 1; m < kMaxModes; ++m) {
        base = n == m ? first[m] : base;
        cp = n == m ? a.c[m] : cp;
      }
      nn[k] = n;
      ee[k] = e0 - base;
      cv[k] = cp[ee[k]];
    }
  }
  kl_recurrence(a, den_last, S, lds64, bid.x);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kApplyPre; ++k) {
    const int n = nn[k];
    if (n < 0) continue;
    const int64_t e = ee[k];
    const int row = (int)(e / kRP), cc = (int)(e % kRP);
    if (cc >= a.R) continue;
    float* up = a.user[0];
    float* pp = a.cur_pad[0];
#pragma unroll
    for (int m = 1; m < kMaxModes; ++m) {
      up = n == m ? a.user[m] : up;
      pp = n == m ? a.cur_pad[m] : pp;
    }
    const float v = fmaxf(cv[k] / den_last[n][cc], a.eps);
    up[(int64_t)row * a.R + cc] = v;
    if (pp) pp[e] = v;
  }
  for (int64_t e0 = e00 + kApplyPre * stride; e0 < total; e0 += stride) {
    int64_t e = e0;
    int n = 0;
    while (n < a.N && e >= (int64_t)a.rows[n] * kRP) {
      e -= (int64_t)a.rows[n] * kRP;
      ++n;
    }
    const int row = (int)(e / kRP), cc = (int)(e % kRP);
    if (cc >= a.R) continue;
    const float v = fmaxf(a.c[n][e] / den_last[n][cc], a.eps);
    a.user[n][(int64_t)row * a.R + cc] = v;
    if (a.cur_pad[n]) a.cur_pad[n][e] = v;
  }
}
COMM_GROUPED_KERNELS(kl_apply, KlLoopArgs, 1024)

// ----------------------------------------------------------------------------------------
// Slot reduction + update.  A workgroup covers kSlotRows rows x 32 columns of
// one job with kSlotGroups groups of threads; group g sums slots g,
// g + kSlotGroups, ... with eight loads in flight per batch, and the groups are
// combined in order 0, 1, ... (fixed order: bitwise deterministic).

__device__ __forceinline__ float pow_gamma(float ratio, float gamma) {
  if (gamma == 1.0f) return ratio;
  if (gamma == 0.5f) return __builtin_amdgcn_sqrtf(ratio);
  return ratio > 0.0f ? __builtin_amdgcn_exp2f(gamma * __builtin_amdgcn_logf(ratio)) : 0.0f;
}

constexpr int kSlotOut = kSlotRows * 32;
constexpr int kSlotGroups = 1024 / kSlotOut;

__device__ __forceinline__ float sum_slots(const float* __restrict__ part, int slots, int64_t slot_stride, int64_t e,
                                           int g) {
  float acc = 0.0f;
  for (int s0 = g; s0 < slots; s0 += 8 * kSlotGroups) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int s = s0 + u * kSlotGroups;
      v[u] = s < slots ? part[(int64_t)s * slot_stride + e] : 0.0f;
    }
    acc += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  }
  return acc;
}

__device__ __forceinline__ float combine_groups(const float (*l)[kSlotOut], int o) {
  float s = l[0][o];
#pragma unroll
  for (int q = 1; q < kSlotGroups; ++q) s += l[q][o];
  return s;
}

__device__ __forceinline__ void slot_update_body(const SlotUpdateArgs& a, uint3 bid, uint3) {
  __shared__ float lnum[kSlotGroups][kSlotOut];
  __shared__ float lden[kSlotGroups][kSlotOut];
  __shared__ float lc[kSlotOut], la[kSlotOut];
  int b = (int)bid.x;
  int j = 0;
  while (j < a.njobs && b >= (a.job[j].rows_p + kSlotRows - 1) / kSlotRows) {
    b -= (a.job[j].rows_p + kSlotRows - 1) / kSlotRows;
    ++j;
  }
  if (j >= a.njobs) return;
  const SlotJob& J = a.job[j];
  const int t = threadIdx.x;
  const int g = t / kSlotOut, o = t % kSlotOut;
  const int row = kSlotRows * b + (o >> 5), c = o & 31;
  const bool live = row < J.rows && c < J.cols;
  const int64_t e = (int64_t)row * kRP + c;
  const int64_t stride = (int64_t)J.rows_total * kRP;
  float anc = 0.0f;
  if (g == 0 && live) anc = J.anchor.p[(int64_t)row * J.anchor.ld + c];
  lnum[g][o] = live ? sum_slots(J.num_part, J.num_slots, stride, e, g) : 0.0f;
  if (J.den_part) lden[g][o] = live ? sum_slots(J.den_part, J.den_slots, stride, e, g) : 0.0f;
  __syncthreads();
  if (g == 0) {
    float v = 0.0f;
    if (live) {
      const float num = combine_groups(lnum, o);
      if (J.mode == kSlotScale) {
        v = anc * num;
      } else if (J.mode == kSlotCopy) {
        v = num;
      } else {
        const float den = J.den_part ? combine_groups(lden, o) : J.den_closed[c];
        v = fmaxf(anc * pow_gamma(num / den, J.gamma), J.eps);
      }
      if (J.out_user) J.out_user[(int64_t)row * J.ld_user + c] = v;
    }
    if (row < J.rows_p) {
      if (J.out_pad) J.out_pad[e] = v;
      if (J.out_padT) J.out_padT[(int64_t)c * J.rows_p + row] = v;
      if (J.chi_x1) {
        float c1, c2;
        chi_pair(v, J.chi_ref[e], J.chi_beta, c1, c2);
        J.chi_x1[e] = c1;
        J.chi_x2[e] = c2;
        if (J.chi_x1T) J.chi_x1T[(int64_t)c * J.rows_p + row] = c1;
        if (J.chi_x2T) J.chi_x2T[(int64_t)c * J.rows_p + row] = c2;
      }
    }
    lc[o] = v;
    la[o] = anc;
  }
  if (J.stats) {
    __syncthreads();
    if (t < 32) {
      float st = 0.0f, sm = 3.402823e38f, sa = 0.0f;
      for (int r = 0; r < kSlotRows; ++r) {
        if (kSlotRows * b + r < J.rows) {
          st += lc[r * 32 + t];
          sm = fminf(sm, lc[r * 32 + t]);
          sa += la[r * 32 + t];
        }
      }
      float* out = J.stats + (int64_t)b * 96;
      out[t] = st;
      out[32 + t] = sm;
      out[64 + t] = sa;
    }
  }
}

COMM_GROUPED_KERNELS(slot_update, SlotUpdateArgs, 1024)

hipError_t launch_slot_update(const SlotUpdateArgs& a, hipStream_t s) {
  int blocks = 0;
  for (int j = 0; j < a.njobs; ++j) blocks += (a.job[j].rows_p + kSlotRows - 1) / kSlotRows;
  return launch_or_record(slot_update_kernel, slot_update_grouped, dim3(blocks), dim3(1024), 0, s, a);
}

// Debug check of caller inputs: sets `bit` in *flag when one of the n values
// is below lo or is not finite (NaN fails both comparisons, +inf the second).
__global__ void __launch_bounds__(256) check_range_kernel(const float* __restrict__ p, int64_t n, float lo, int bit,
                                                          int* flag) {
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const float v = p[e];
    bad |= !(v >= lo && v <= 3.402823466e38f);
  }
  if (bad) atomicOr(flag, bit);
}

hipError_t launch_check_range(const float* p, int64_t n, float lo, int bit, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(check_range_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, lo, bit, flag);
  return hipGetLastError();
}

hipError_t launch_kl_apply(const KlLoopArgs& a, hipStream_t s) {
  int64_t n = 0;
  for (int q = 0; q < a.N; ++q) n += (int64_t)a.rows[q] * kRP;
  int blocks = (int)((n + 1023) / 1024);
  if (blocks > 64) blocks = 64;
  return launch_or_record(kl_apply_kernel, kl_apply_grouped, dim3(blocks), dim3(1024), 0, s, a);
}

// ----------------------------------------------------------------------------------------
// Extrapolation (Sec. "Going beyond: Majorization-Minimization with Extrapolation")

// alpha = min(alpha_nes, c / (||[cur - prev]_+|| + delta)) over every block,
// the squared norm summed in float64 in a fixed order; one workgroup.
__global__ void __launch_bounds__(1024) extrap_alpha_kernel(ExtrapArgs a) {
  __shared__ double lds[1024];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int b = 0; b < a.nb; ++b) {
    const float* cur = a.cur[b];
    const float* prev = a.prev[b];
    for (int64_t e = t; e < a.count[b]; e += 1024) {
      const double d = (double)cur[e] - (double)prev[e];
      if (d > 0.0) s += d * d;
    }
  }
  lds[t] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) lds[t] += lds[t + w];
    __syncthreads();
  }
  if (t == 0) a.alpha[0] = (float)fmin(a.alpha_nes, a.c / (sqrt(lds[0]) + a.delta));
}

// For the selected blocks: prev <- cur, cur <- max(cur + alpha [cur - prev]_+, eps).
__global__ void extrap_apply_kernel(ExtrapArgs a) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  while (b < a.nb && e >= a.count[b]) {
    e -= a.count[b];
    ++b;
  }
  if (b >= a.nb) return;
  const float alpha = a.alpha[0];
  const float v = a.cur[b][e], p = a.prev[b][e];
  a.prev[b][e] = v;
  a.cur[b][e] = fmaxf(v + alpha * fmaxf(v - p, 0.0f), a.eps);
}

hipError_t launch_extrap_alpha(const ExtrapArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(extrap_alpha_kernel, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_extrap_apply(const ExtrapArgs& a, hipStream_t s) {
  int64_t n = 0;
  for (int b = 0; b < a.nb; ++b) n += a.count[b];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(extrap_apply_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace comm
