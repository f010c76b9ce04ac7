// Sparse COO numerators and objective correction at any beta in (0, 2): the
// part of a beta != 1 update that the nonzeros carry (Sec. 6.4, paragraph on
// sparse tensors).  The denominators, which involve Q = Xhat^(beta-1) on every
// cell, come from the dense pass run on an all-zero tensor of the same shape.

#include "kernels.h"

namespace comm {

constexpr int kCooBetaThreads = 256;

template <int BC>
__global__ void __launch_bounds__(kCooBetaThreads) coo_beta_kernel(CooBetaArgs a) {
  __shared__ double lobj[kCooBetaThreads / 64][2];
  const int lane = threadIdx.x & 63;
  const int r = lane & 31;
  const int64_t half = ((int64_t)blockIdx.x * kCooBetaThreads + threadIdx.x) >> 5;
  const int64_t nhalf = ((int64_t)gridDim.x * kCooBetaThreads) >> 5;
  const bool rlive = r < a.R;
  double obj = 0.0, objc = 0.0;   // compensated sum of the objective terms
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
        if (a.obj_part) sum2_add(obj, objc, (double)dbeta_term<BC>(x, y, a.bc) - (double)dbeta_term<BC>(0.0f, y, a.bc));
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
    sum2_wave(obj, objc);
    if (lane == 0) {
      lobj[threadIdx.x >> 6][0] = obj;
      lobj[threadIdx.x >> 6][1] = objc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = lobj[0][0], c = lobj[0][1];
      for (int q = 1; q < kCooBetaThreads / 64; ++q) {
        sum2_add(s, c, lobj[q][0]);
        c += lobj[q][1];
      }
      a.obj_part[blockIdx.x] = s + c;
    }
  }
}

template <int BC>
__global__ void __launch_bounds__(kCooBetaThreads) coo_tucker_kernel(CooTkArgs a) {
  __shared__ double lobj[kCooBetaThreads / 64][2];
  const int lane = threadIdx.x & 63;
  const int d = lane & 31;
  const int64_t half = ((int64_t)blockIdx.x * kCooBetaThreads + threadIdx.x) >> 5;
  const int64_t nhalf = ((int64_t)gridDim.x * kCooBetaThreads) >> 5;
  const int L = a.N - 1;  // the fibre mode
  double obj = 0.0, objc = 0.0;   // compensated sum of the objective terms
  // contiguous chunk per half; equal target rows of consecutive nonzeros are
  // summed in a register (one atomic per run)
  const int64_t chunk = (a.nnz + nhalf - 1) / nhalf;
  const int64_t t0 = half * chunk, t1 = min(a.nnz, t0 + chunk);
  int64_t run_row = -1;
  float run_acc = 0.0f;
  // kG nonzeros at a time, each step's loads issued together before their
  // first use: a nonzero past the chunk re-reads the chunk's last one, a row
  // or column past the edge reads a valid one, and masks apply afterwards (a
  // guarded load per nonzero would be a branch and a round trip each).  The
  // nonzeros are then accumulated in stream order, as one at a time.
  constexpr int kG = 4;
  const int cr_col = min(d, a.Cr.cols - 1), cc_col = a.op == 1 ? min(d, a.Cc.cols - 1) : 0;
  const float cr_mask = d < a.Cr.cols ? 1.0f : 0.0f;
  const float cc_mask = a.op == 1 && d < a.Cc.cols ? 1.0f : 0.0f;
  for (int64_t tb = t0; tb < t1; tb += kG) {
    int ii[kG][kMaxModes];
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      const int64_t t = min(tb + u, t1 - 1);
#pragma unroll
      for (int m = 0; m < kMaxModes; ++m) ii[u][m] = a.idx[m < a.N ? m : 0][t];
    }
    __builtin_amdgcn_sched_barrier(0);
    bool live[kG];
    int64_t row[kG];
    int iL[kG];
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      bool ok = tb + u < t1;
#pragma unroll
      for (int m = 0; m < kMaxModes; ++m)
        if (m < a.N) ok = ok && ii[u][m] >= 0 && ii[u][m] < a.dims[m];
      live[u] = ok;
      int64_t rr = 0;
      int il = 0;
#pragma unroll
      for (int m = 0; m < kMaxModes; ++m) {
        const int im = ok ? ii[u][m] : 0;
        if (m < L) rr = rr * a.dims[m] + im;
        if (m == L) il = im;
      }
      row[u] = rr;
      iL[u] = il;
    }
    float w[kG];
    if (a.w_in) {
#pragma unroll
      for (int u = 0; u < kG; ++u) w[u] = a.w_in[min(tb + u, t1 - 1)];
    } else {
      float tr[kG], cr[kG], xv[kG];
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        tr[u] = a.Tr[row[u] * kRP + d];
        cr[u] = a.Cr.p[(int64_t)iL[u] * a.Cr.ld + cr_col];
        xv[u] = a.val[min(tb + u, t1 - 1)];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        float z = tr[u] * (cr[u] * cr_mask);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) z += __shfl_xor(z, off);
        const float y = fmaxf(z, a.eps);
        float p, q;
        weights<BC>(xv[u], y, a.bc.beta, p, q);
        w[u] = p;
        if (d == 0 && live[u]) {
          if (a.w_out) a.w_out[tb + u] = p;
          if (a.obj_part)
            sum2_add(obj, objc, (double)dbeta_term<BC>(xv[u], y, a.bc) - (double)dbeta_term<BC>(0.0f, y, a.bc));
        }
      }
    }
    if (a.op != 0) {
      float cf[kG];
#pragma unroll
      for (int u = 0; u < kG; ++u)
        cf[u] = a.op == 1 ? a.Cc.p[(int64_t)iL[u] * a.Cc.ld + cc_col] * cc_mask : a.Tc[row[u] * kRP + d];
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        if (!live[u]) continue;
        const int64_t target = a.op == 1 ? row[u] : (int64_t)iL[u];
        const float c = w[u] * cf[u];
        if (target != run_row) {
          if (run_row >= 0) unsafeAtomicAdd(&a.out[run_row * kRP + d], run_acc);
          run_row = target;
          run_acc = 0.0f;
        }
        run_acc += c;
      }
    }
  }
  if (run_row >= 0) unsafeAtomicAdd(&a.out[run_row * kRP + d], run_acc);
  if (a.obj_part) {
    sum2_wave(obj, objc);
    if (lane == 0) {
      lobj[threadIdx.x >> 6][0] = obj;
      lobj[threadIdx.x >> 6][1] = objc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = lobj[0][0], c = lobj[0][1];
      for (int q = 1; q < kCooBetaThreads / 64; ++q) {
        sum2_add(s, c, lobj[q][0]);
        c += lobj[q][1];
      }
      a.obj_part[blockIdx.x] = s + c;
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
