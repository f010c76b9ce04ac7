// Factor-side kernels: padding copies, column sums, the J-CoMM transforms
// chi_1 / chi_2 (Sec. 5.3), the multiplicative block update with the eps
// floor (Theorem "CP block multiplicative update"; Sec. 5.3 inner update), the
// fixed-order float64 reduction of objective partials, and the beta = 1 inner
// loop of J-CoMM for CP.  All reductions have a fixed order (deterministic).

#include "kernels.h"

namespace comm {

// ----------------------------------------------------------------------------------------

__global__ void pad_factor_kernel(const float* __restrict__ src, int rows, int cols, int ld, int rows_p,
                                  float* __restrict__ dst, float* __restrict__ dstT) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows_p * kRP) return;
  const int row = (int)(e / kRP), c = (int)(e % kRP);
  const float v = (row < rows && c < cols) ? src[(int64_t)row * ld + c] : 0.0f;
  dst[e] = v;
  if (dstT) dstT[(int64_t)c * rows_p + row] = v;
}

hipError_t launch_pad_factor(const float* src, int rows, int cols, int ld, int rows_p, float* dst, float* dstT,
                             hipStream_t s) {
  const int64_t n = (int64_t)rows_p * kRP;
  hipLaunchKernelGGL(pad_factor_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, rows, cols, ld,
                     rows_p, dst, dstT);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------------
// Column sums: one workgroup per factor, 8 row groups x 32 columns, fixed order.

struct ColsumArgs {
  const float* F[4];
  int rows[4];
  int nf;
  float* out;        // [nf][32] column sums (may be NULL)
  float* prod;       // if not NULL: prod[c] = product over the nf factors of the column sums
};

__device__ void colsum_block(const float* F, int rows, float* lds8x32, float* result32) {
  const int t = threadIdx.x;
  const int c = t & 31, g = t >> 5;
  float s = 0.0f;
  for (int r = g; r < rows; r += 8) s += F[(int64_t)r * kRP + c];
  lds8x32[g * 32 + c] = s;
  __syncthreads();
  if (t < 32) {
    float acc = lds8x32[t];
    for (int q = 1; q < 8; ++q) acc += lds8x32[q * 32 + t];
    result32[t] = acc;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) colsum_kernel(ColsumArgs a) {
  __shared__ float part[8 * 32];
  __shared__ float res[4][32];
  for (int f = 0; f < a.nf; ++f) colsum_block(a.F[f], a.rows[f], part, res[f]);
  const int t = threadIdx.x;
  if (t < 32) {
    float p = 1.0f;
    for (int f = 0; f < a.nf; ++f) {
      if (a.out) a.out[f * 32 + t] = res[f][t];
      p *= res[f][t];
    }
    if (a.prod) a.prod[t] = p;
  }
}

hipError_t launch_colsums(const float* const* F, const int* rows, int nf, float* out, hipStream_t s) {
  ColsumArgs a = {};
  for (int f = 0; f < nf; ++f) { a.F[f] = F[f]; a.rows[f] = rows[f]; }
  a.nf = nf; a.out = out; a.prod = nullptr;
  hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_colsum_prod(const float* const* F, const int* rows, int nf, float* prod, hipStream_t s) {
  ColsumArgs a = {};
  for (int f = 0; f < nf; ++f) { a.F[f] = F[f]; a.rows[f] = rows[f]; }
  a.nf = nf; a.out = nullptr; a.prod = prod;
  hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------------
// chi transforms

__global__ void chi_kernel(const float* __restrict__ cur, const float* __restrict__ ref, int rows_p, float beta,
                           float* __restrict__ x1, float* __restrict__ x2, float* __restrict__ x1T,
                           float* __restrict__ x2T) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows_p * kRP) return;
  const float z = cur[e], zr = ref[e];
  float c1 = 0.0f, c2 = 0.0f;
  if (zr > 0.0f) {
    // chi_1 = Z~ (Z/Z~)^(beta-1);  chi_2 = Z (beta < 1) or Z~ (Z/Z~)^beta
    const float u = z / zr;
    const float lu = __builtin_amdgcn_logf(u);
    c1 = (beta == 1.0f) ? zr : zr * __builtin_amdgcn_exp2f((beta - 1.0f) * lu);
    c2 = (beta < 1.0f) ? z : (beta == 1.0f ? z : zr * __builtin_amdgcn_exp2f(beta * lu));
  }
  x1[e] = c1;
  x2[e] = c2;
  const int row = (int)(e / kRP), c = (int)(e % kRP);
  if (x1T) x1T[(int64_t)c * rows_p + row] = c1;
  if (x2T) x2T[(int64_t)c * rows_p + row] = c2;
}

hipError_t launch_chi(const float* cur, const float* ref, int rows_p, float beta, float* x1, float* x2, float* x1T,
                      float* x2T, hipStream_t s) {
  const int64_t n = (int64_t)rows_p * kRP;
  hipLaunchKernelGGL(chi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cur, ref, rows_p, beta, x1, x2,
                     x1T, x2T);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------------
// Multiplicative block update

__device__ __forceinline__ float pow_gamma(float ratio, float gamma) {
  if (gamma == 1.0f) return ratio;
  if (gamma == 0.5f) return __builtin_amdgcn_sqrtf(ratio);
  return ratio > 0.0f ? __builtin_amdgcn_exp2f(gamma * __builtin_amdgcn_logf(ratio)) : 0.0f;
}

__global__ void update_kernel(UpdateArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)a.rows_p * kRP) return;
  const int row = (int)(e / kRP), c = (int)(e % kRP);
  float v = 0.0f;
  if (row < a.rows && c < a.cols) {
    float num = 0.0f;
    for (int s = 0; s < a.num_slots; ++s) num += a.num_part[((int64_t)s * a.rows_total + row) * kRP + c];
    float den;
    if (a.den_closed) {
      den = a.den_closed[c];
    } else {
      den = 0.0f;
      for (int s = 0; s < a.den_slots; ++s) den += a.den_part[((int64_t)s * a.rows_total + row) * kRP + c];
    }
    v = fmaxf(a.anchor[e] * pow_gamma(num / den, a.gamma), a.eps);
    if (a.out_user) a.out_user[(int64_t)row * a.ld_user + c] = v;
  }
  a.out_pad[e] = v;
  if (a.out_padT) a.out_padT[(int64_t)c * a.rows_p + row] = v;
}

hipError_t launch_update(const UpdateArgs& a, hipStream_t s) {
  const int64_t n = (int64_t)a.rows_p * kRP;
  hipLaunchKernelGGL(update_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// out[row][c] = anchor[row][c] * sum_s part[s][row][c] (rows < rows, else 0).
__global__ void scale_reduce_kernel(const float* __restrict__ part, int slots, int rows_total, int rows, int cols,
                                    const float* __restrict__ anchor, int rows_p, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows_p * kRP) return;
  const int row = (int)(e / kRP), c = (int)(e % kRP);
  float v = 0.0f;
  if (row < rows && c < cols) {
    float s = 0.0f;
    for (int t = 0; t < slots; ++t) s += part[((int64_t)t * rows_total + row) * kRP + c];
    v = anchor[e] * s;
  }
  out[e] = v;
}

hipError_t launch_scale_reduce(const float* part, int slots, int rows_total, int rows, int cols, const float* anchor,
                               int rows_p, float* out, hipStream_t s) {
  const int64_t n = (int64_t)rows_p * kRP;
  hipLaunchKernelGGL(scale_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, slots,
                     rows_total, rows, cols, anchor, rows_p, out);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------------
// float64 sum of partials, fixed order

__global__ void __launch_bounds__(1024) sum_f64_kernel(const double* __restrict__ part, int64_t n,
                                                       const double* __restrict__ add_to, double* __restrict__ out) {
  __shared__ double lds[1024];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t e = t; e < n; e += 1024) s += part[e];
  lds[t] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) lds[t] += lds[t + w];
    __syncthreads();
  }
  if (t == 0) out[0] = lds[0] + (add_to ? add_to[0] : 0.0);
}

hipError_t launch_sum_f64(const double* part, int64_t n, const double* add_to, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(1024), 0, s, part, n, add_to, out);
  return hipGetLastError();
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
// The L sweeps thus reduce to recurrences on 32-wide vectors plus one final
// elementwise pass; one workgroup runs them.

__global__ void __launch_bounds__(1024) kl_loop_kernel(KlLoopArgs a) {
  __shared__ float red[32][33];
  __shared__ float S[4][32], T[4][32], Cmin[4][32], DenLast[4][32], Den[32];
  __shared__ int flag[32];
  __shared__ int any_flag;
  const int t = threadIdx.x;
  const int c = t & 31, g = t >> 5;  // 32 row groups x 32 columns

  for (int n = 0; n < a.N; ++n) {
    // T, min of c; S = colsum(ref)
    float st = 0.0f, sm = 3.402823e38f, sr = 0.0f;
    for (int r = g; r < a.rows[n]; r += 32) {
      const float v = a.c[n][(int64_t)r * kRP + c];
      st += v;
      sm = fminf(sm, v);
      sr += a.ref[n][(int64_t)r * kRP + c];
    }
    red[g][c] = st;
    __syncthreads();
    if (t < 32) {
      float s = 0.0f;
      for (int q = 0; q < 32; ++q) s += red[q][t];
      T[n][t] = s;
    }
    __syncthreads();
    red[g][c] = sm;
    __syncthreads();
    if (t < 32) {
      float s = red[0][t];
      for (int q = 1; q < 32; ++q) s = fminf(s, red[q][t]);
      Cmin[n][t] = s;
    }
    __syncthreads();
    red[g][c] = sr;
    __syncthreads();
    if (t < 32) {
      float s = 0.0f;
      for (int q = 0; q < 32; ++q) s += red[q][t];
      S[n][t] = s;
    }
    __syncthreads();
  }

  for (int l = 0; l < a.L; ++l) {
    for (int n = 0; n < a.N; ++n) {
      if (t < 32) {
        float d = 1.0f;
        for (int m = 0; m < a.N; ++m)
          if (m != n) d *= S[m][t];
        Den[t] = d;
        DenLast[n][t] = d;
        flag[t] = (t < a.R) && (Cmin[n][t] < a.eps * d);
      }
      __syncthreads();
      if (t == 0) {
        int f = 0;
        for (int q = 0; q < 32; ++q) f |= flag[q];
        any_flag = f;
      }
      __syncthreads();
      if (any_flag) {
        // exact column sums of max(c / Den, eps) for the clipped columns
        float s = 0.0f;
        if (flag[c])
          for (int r = g; r < a.rows[n]; r += 32) s += fmaxf(a.c[n][(int64_t)r * kRP + c] / Den[c], a.eps);
        red[g][c] = s;
        __syncthreads();
        if (t < 32 && flag[t]) {
          float acc = 0.0f;
          for (int q = 0; q < 32; ++q) acc += red[q][t];
          S[n][t] = acc;
        }
      }
      if (t < 32 && !flag[t]) S[n][t] = (t < a.R) ? T[n][t] / Den[t] : 0.0f;
      __syncthreads();
    }
  }

  for (int n = 0; n < a.N; ++n) {
    const int64_t total = (int64_t)a.rows_p[n] * kRP;
    for (int64_t e = t; e < total; e += 1024) {
      const int row = (int)(e / kRP), cc = (int)(e % kRP);
      float v = 0.0f;
      if (row < a.rows[n] && cc < a.R) {
        v = fmaxf(a.c[n][e] / DenLast[n][cc], a.eps);
        if (a.user[n]) a.user[n][(int64_t)row * a.R + cc] = v;
      }
      a.cur_pad[n][e] = v;
      if (a.cur_padT[n]) a.cur_padT[n][(int64_t)cc * a.rows_p[n] + row] = v;
    }
  }
}

hipError_t launch_kl_loop(const KlLoopArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(kl_loop_kernel, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

}  // namespace comm
