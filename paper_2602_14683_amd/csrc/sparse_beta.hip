// Sparse COO numerators and objective correction at any beta in (0, 2): the
// part of a beta != 1 update that the nonzeros carry (Sec. 6.4, paragraph on
// sparse tensors).  The denominators, which involve Q = Xhat^(beta-1) on every
// cell, come from the dense pass run on an all-zero tensor of the same shape.

#include "kernels.h"

namespace comm {

constexpr int kCooBetaThreads = 256;

template <int BC>
__global__ void __launch_bounds__(kCooBetaThreads) coo_beta_kernel(CooBetaArgs a) {
  __shared__ double lobj[kCooBetaThreads / 64];
  const int lane = threadIdx.x & 63;
  const int r = lane & 31;
  const int64_t half = ((int64_t)blockIdx.x * kCooBetaThreads + threadIdx.x) >> 5;
  const int64_t nhalf = ((int64_t)gridDim.x * kCooBetaThreads) >> 5;
  const bool rlive = r < a.R;
  double obj = 0.0;
  // each half owns a contiguous chunk of the stream, so that equal target
  // rows of consecutive nonzeros are summed in a register (one atomic per run)
  const int64_t chunk = (a.nnz + nhalf - 1) / nhalf;
  const int64_t t0 = half * chunk, t1 = min(a.nnz, t0 + chunk);
  int run_row = -1;
  float run_acc = 0.0f;
  for (int64_t t = t0; t < t1; ++t) {
    // every lane of the half reads the same nonzero
    int ii[kMaxModes] = {};
    bool ok = true;
#pragma unroll
    for (int m = 0; m < kMaxModes; ++m) {
      if (m < a.N) {
        ii[m] = a.idx[m][t];
        ok = ok && ii[m] >= 0 && ii[m] < a.dims[m];
      }
    }
    if (!ok) continue;
    float w;
    if (a.w_in) {
      w = a.w_in[t];
    } else {
      const float x = a.val[t];
      float z = 0.0f;
      if (rlive) {
        z = 1.0f;
#pragma unroll
        for (int m = 0; m < kMaxModes; ++m)
          if (m < a.N) z *= a.rb[m].at(ii[m], r, a.dims[m]);
      }
      // sum over the 32 lanes of this half (partners stay inside the half)
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) z += __shfl_xor(z, off);
      const float y = fmaxf(z, a.eps);
      float p, q;
      weights<BC>(x, y, a.bc.beta, p, q);
      w = p;
      if (r == 0) {
        if (a.w_out) a.w_out[t] = p;
        if (a.obj_part) obj += (double)dbeta_term<BC>(x, y, a.bc) - (double)dbeta_term<BC>(0.0f, y, a.bc);
      }
    }
    if (a.mode >= 0 && rlive) {
      float c = w;
#pragma unroll
      for (int m = 0; m < kMaxModes; ++m)
        if (m < a.N && m != a.mode) c *= a.ct[m].at(ii[m], r, a.dims[m]);
      const int row = ii[a.mode];
      if (row != run_row) {
        if (run_row >= 0) unsafeAtomicAdd(&a.num[(int64_t)run_row * kRP + r], run_acc);
        run_row = row;
        run_acc = 0.0f;
      }
      run_acc += c;
    }
  }
  if (run_row >= 0 && rlive) unsafeAtomicAdd(&a.num[(int64_t)run_row * kRP + r], run_acc);
  if (a.obj_part) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) obj += __shfl_down(obj, off);
    if (lane == 0) lobj[threadIdx.x >> 6] = obj;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int q = 0; q < kCooBetaThreads / 64; ++q) s += lobj[q];
      a.obj_part[blockIdx.x] = s;
    }
  }
}

template <int BC>
__global__ void __launch_bounds__(kCooBetaThreads) coo_tucker_kernel(CooTkArgs a) {
  __shared__ double lobj[kCooBetaThreads / 64];
  const int lane = threadIdx.x & 63;
  const int d = lane & 31;
  const int64_t half = ((int64_t)blockIdx.x * kCooBetaThreads + threadIdx.x) >> 5;
  const int64_t nhalf = ((int64_t)gridDim.x * kCooBetaThreads) >> 5;
  const int L = a.N - 1;  // the fibre mode
  double obj = 0.0;
  // contiguous chunk per half; equal target rows of consecutive nonzeros are
  // summed in a register (one atomic per run)
  const int64_t chunk = (a.nnz + nhalf - 1) / nhalf;
  const int64_t t0 = half * chunk, t1 = min(a.nnz, t0 + chunk);
  int64_t run_row = -1;
  float run_acc = 0.0f;
  for (int64_t t = t0; t < t1; ++t) {
    int ii[kMaxModes] = {};
    bool ok = true;
#pragma unroll
    for (int m = 0; m < kMaxModes; ++m) {
      if (m < a.N) {
        ii[m] = a.idx[m][t];
        ok = ok && ii[m] >= 0 && ii[m] < a.dims[m];
      }
    }
    if (!ok) continue;
    int64_t row = 0;
#pragma unroll
    for (int m = 0; m < kMaxModes; ++m)
      if (m < L) row = row * a.dims[m] + ii[m];
    const int iL = ii[L];
    float w;
    if (a.w_in) {
      w = a.w_in[t];
    } else {
      float z = a.Tr[row * kRP + d] * a.Cr.at(iL, d, a.dims[L]);
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) z += __shfl_xor(z, off);
      const float x = a.val[t];
      const float y = fmaxf(z, a.eps);
      float p, q;
      weights<BC>(x, y, a.bc.beta, p, q);
      w = p;
      if (d == 0) {
        if (a.w_out) a.w_out[t] = p;
        if (a.obj_part) obj += (double)dbeta_term<BC>(x, y, a.bc) - (double)dbeta_term<BC>(0.0f, y, a.bc);
      }
    }
    if (a.op != 0) {
      const int64_t target = a.op == 1 ? row : (int64_t)iL;
      const float c = a.op == 1 ? w * a.Cc.at(iL, d, a.dims[L]) : w * a.Tc[row * kRP + d];
      if (target != run_row) {
        if (run_row >= 0) unsafeAtomicAdd(&a.out[run_row * kRP + d], run_acc);
        run_row = target;
        run_acc = 0.0f;
      }
      run_acc += c;
    }
  }
  if (run_row >= 0) unsafeAtomicAdd(&a.out[run_row * kRP + d], run_acc);
  if (a.obj_part) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) obj += __shfl_down(obj, off);
    if (lane == 0) lobj[threadIdx.x >> 6] = obj;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int q = 0; q < kCooBetaThreads / 64; ++q) s += lobj[q];
      a.obj_part[blockIdx.x] = s;
    }
  }
}

hipError_t launch_coo_tucker(const CooTkArgs& a, int bc, hipStream_t s) {
  const dim3 grid((unsigned)coo_beta_blocks(a.nnz)), block(kCooBetaThreads);
  switch (bc) {
    case kHalf: hipLaunchKernelGGL(coo_tucker_kernel<kHalf>, grid, block, 0, s, a); break;
    case kKL: hipLaunchKernelGGL(coo_tucker_kernel<kKL>, grid, block, 0, s, a); break;
    case kThreeHalf: hipLaunchKernelGGL(coo_tucker_kernel<kThreeHalf>, grid, block, 0, s, a); break;
    case kGeneral: hipLaunchKernelGGL(coo_tucker_kernel<kGeneral>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void clear_f32_kernel(float* p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0.0f;
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(clear_f32_kernel, dim3((unsigned)b), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

int coo_beta_blocks(int64_t nnz) {
  const int64_t per = kCooBetaThreads / 32;  // nonzeros per workgroup per step
  int64_t b = (nnz + per - 1) / per;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_coo_beta(const CooBetaArgs& a, int bc, hipStream_t s) {
  const dim3 grid((unsigned)coo_beta_blocks(a.nnz)), block(kCooBetaThreads);
  switch (bc) {
    case kHalf: hipLaunchKernelGGL(coo_beta_kernel<kHalf>, grid, block, 0, s, a); break;
    case kKL: hipLaunchKernelGGL(coo_beta_kernel<kKL>, grid, block, 0, s, a); break;
    case kThreeHalf: hipLaunchKernelGGL(coo_beta_kernel<kThreeHalf>, grid, block, 0, s, a); break;
    case kGeneral: hipLaunchKernelGGL(coo_beta_kernel<kGeneral>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;  // beta = 0 has no sparse form (d(0 | y) is infinite)
  }
  return hipGetLastError();
}

}  // namespace comm
