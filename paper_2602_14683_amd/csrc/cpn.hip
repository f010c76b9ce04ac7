// Order-N CP (N = 4, 5) through a 3-way view: the Khatri-Rao super factor of
// the grouped modes, and the fold of the super mode's numerator into the
// numerators of the grouped modes.  Both are small next to the fused pass that
// runs between them (rows of the super mode x 32 floats).

#include "kernels.h"

namespace comm {

__global__ void __launch_bounds__(256) kr_kernel(KrArgs a) {
  const int o = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)a.rows_p * kRP) return;
  const int s = (int)(e / kRP), c = (int)(e % kRP);
  float v = 0.0f;
  if (s < a.rows) {
    int idx[kMaxGroup];
    int rem = s;
#pragma unroll
    for (int m = kMaxGroup - 1; m >= 0; --m) {
      idx[m] = 0;
      if (m < a.G) {
        idx[m] = rem % a.dims[m];
        rem /= a.dims[m];
      }
    }
    v = 1.0f;
#pragma unroll
    for (int m = 0; m < kMaxGroup; ++m)
      if (m < a.G) v *= a.f[o][m].at(idx[m], c, a.dims[m]);
  }
  a.out[o][e] = v;
}

hipError_t launch_kr(const KrArgs& a, hipStream_t s) {
  if (a.nout < 1) return hipSuccess;
  const int64_t n = (int64_t)a.rows_p * kRP;
  hipLaunchKernelGGL(kr_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)a.nout), dim3(256), 0, s, a);
  return hipGetLastError();
}

// One workgroup per output row of one job: 32 groups of 32 lanes (one lane
// per column) stride over the super-mode rows with s_mode = i, and the groups
// are combined in order.
constexpr int kFoldGroups = 32;

__global__ void __launch_bounds__(1024) fold_kernel(FoldArgs a) {
  __shared__ float red[kFoldGroups][32];
  const FoldJob& J = a.job[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= J.rows_p) return;  // uniform over the workgroup
  const int t = threadIdx.x, c = t & 31, g = t >> 5;
  const int di = a.dims[J.mode];
  float acc = 0.0f;
  if (i < di) {
    int64_t rows = 1;
#pragma unroll
    for (int m = 0; m < kMaxGroup; ++m)
      if (m < a.G) rows *= a.dims[m];
    const int64_t others = rows / di;
    const int64_t stride = (int64_t)J.rows_total * kRP;
    for (int64_t o = g; o < others; o += kFoldGroups) {
      int64_t rem = o, s = 0, mul = 1;
      float w = 1.0f;
#pragma unroll
      for (int m = kMaxGroup - 1; m >= 0; --m) {
        if (m >= a.G) continue;
        int im = i;
        if (m != J.mode) {
          im = (int)(rem % a.dims[m]);
          rem /= a.dims[m];
          w *= J.w[m].at(im, c, a.dims[m]);
        }
        s += (int64_t)im * mul;
        mul *= a.dims[m];
      }
      const float* p = J.part + s * kRP + c;
      float v = 0.0f;
      for (int q = 0; q < J.slots; ++q) v += p[(int64_t)q * stride];
      acc += v * w;
    }
  }
  red[g][c] = acc;
  __syncthreads();
  if (t < 32) {
    float sum = red[0][t];
#pragma unroll
    for (int q = 1; q < kFoldGroups; ++q) sum += red[q][t];
    J.out[(int64_t)i * kRP + t] = i < di ? sum : 0.0f;
  }
}

hipError_t launch_fold(const FoldArgs& a, hipStream_t s) {
  if (a.njobs < 1) return hipSuccess;
  int rows = 0;
  for (int j = 0; j < a.njobs; ++j) rows = rows > a.job[j].rows_p ? rows : a.job[j].rows_p;
  hipLaunchKernelGGL(fold_kernel, dim3((unsigned)rows, (unsigned)a.njobs), dim3(32 * kFoldGroups), 0, s, a);
  return hipGetLastError();
}

}  // namespace comm
