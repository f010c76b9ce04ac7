// Sparse COO J-CoMM for CP at beta = 1 (Sec. 6.4, paragraph on sparse
// tensors): numerators accumulate over the nonzeros only, and the beta = 1
// denominator prod_{m != n} colsum(A^(m)) is closed-form (Q~ = 1).
//
// Per nonzero (i, x): z_r = prod_m A~^(m)_{i_m r}, X~ = max(sum_r z_r, eps),
// w_r = x z_r / X~, and for every mode n, M^(n)[i_n][r] += w_r.  Since
// Num_J^(n)[i_n][r] = sum_nz (x / X~) prod_{m != n} A~^(m) = M^(n)[i_n][r] / A~^(n)[i_n][r],
// the product c^(n) = A~^(n) * Num_J^(n) that drives the beta = 1 inner loop
// (kernels_small.hip) is M^(n) itself.
//
// Mapping: one nonzero per half wavefront, lane = rank component; the four
// factor rows are gathered with coalesced 128-byte loads and X~ is a
// half-wave reduction.  The COO is sorted lexicographically, so modes 1 and 2
// come in runs: each half wave keeps a running sum per mode and adds it to
// global memory when the index changes.  Modes 3 and 4 are added per nonzero
// with hardware float atomics, so this path is reproducible only to rounding
// (not bitwise).  Nonzeros with an index outside [0, dims) are skipped.
//
// Objective at the reference: nonzero cells contribute d_1(x | X~) (stable
// form), zero cells contribute X~, which sums in closed form over all cells as
// sum_r prod_n colsum(A~^(n))_r minus the nonzero cells' X~.

#include "host_util.h"
#include "sparse.h"
#include "cp3_impl.h"

namespace comm {

struct CooPassArgs {
  int N, R;
  int64_t nnz;
  int dims[4];
  const int32_t* idx[4];
  const float* val;
  const float* A[4];     // caller's factors, row stride R
  float* M[4];           // [dims][32] accumulators, zeroed before the pass
  float eps;
  int64_t chunk;         // nonzeros per wavefront
  double* obj_part;      // per workgroup: sum d_1(x | X~) - sum X~ over its nonzeros
};

constexpr int kCooThreads = 256;

__device__ __forceinline__ float half_sum(float v) {
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ void __launch_bounds__(kCooThreads) coo_pass_kernel(CooPassArgs a) {
  __shared__ double lobj[kCooThreads / 64];
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
  const int wave = (int)((blockIdx.x * (int64_t)kCooThreads + threadIdx.x) >> 6);
  const int64_t t0 = (int64_t)wave * a.chunk;
  const int64_t t1 = min(a.nnz, t0 + a.chunk);
  const bool rlive = r < a.R;
  const int N = a.N;

  int cur0 = -1, cur1 = -1;
  float acc0 = 0.0f, acc1 = 0.0f;
  double obj = 0.0;
  // each half wave walks its own nonzeros; the shuffles stay within a half
  for (int64_t t = t0 + h; t < t1; t += 2) {
    int ii[4] = {0, 0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (m < N) {
        ii[m] = a.idx[m][t];
        ok = ok && ii[m] >= 0 && ii[m] < a.dims[m];
      }
    }
    const float x = a.val[t];
    float z = 0.0f;
    if (ok && rlive) {
      z = 1.0f;
#pragma unroll
      for (int m = 0; m < 4; ++m)
        if (m < N) z *= a.A[m][(int64_t)ii[m] * a.R + r];
    }
    const float xt = fmaxf(half_sum(z), a.eps);
    const float w = ok ? x * z / xt : 0.0f;
    if (ok && r == 0) {
      const float sum = x + xt;
      bool far;
      float d = kl_series(x, xt, fast_rcp(sum), far);
      if (far) d = kl_direct(x, xt);
      obj += (double)d - (double)xt;
    }
    if (!ok) continue;
    // modes 1 and 2: runs of equal index (sorted COO)
    if (ii[0] != cur0) {
      if (cur0 >= 0 && rlive) unsafeAtomicAdd(&a.M[0][(int64_t)cur0 * kRP + r], acc0);
      cur0 = ii[0];
      acc0 = 0.0f;
    }
    acc0 += w;
    if (N > 1) {
      if (ii[1] != cur1) {
        if (cur1 >= 0 && rlive) unsafeAtomicAdd(&a.M[1][(int64_t)cur1 * kRP + r], acc1);
        cur1 = ii[1];
        acc1 = 0.0f;
      }
      acc1 += w;
    }
    if (rlive) {
      if (N > 2) unsafeAtomicAdd(&a.M[2][(int64_t)ii[2] * kRP + r], w);
      if (N > 3) unsafeAtomicAdd(&a.M[3][(int64_t)ii[3] * kRP + r], w);
    }
  }
  if (rlive) {
    if (cur0 >= 0) unsafeAtomicAdd(&a.M[0][(int64_t)cur0 * kRP + r], acc0);
    if (N > 1 && cur1 >= 0) unsafeAtomicAdd(&a.M[1][(int64_t)cur1 * kRP + r], acc1);
  }
  // objective partial (lanes 0 and 32 hold the values)
  obj += __shfl_xor(obj, 32);
  if (lane == 0) lobj[threadIdx.x >> 6] = obj;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kCooThreads / 64; ++q) s += lobj[q];
    a.obj_part[blockIdx.x] = s;
  }
}

__global__ void fill_zero_kernel(float* p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0.0f;
}

}  // namespace comm

using namespace comm;

int coo_jcomm_kl(comm_ctx* ctx, const comm_coo* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st) {
  const int N = x->ndim, R = m->rank;
  int dims[4] = {0, 0, 0, 0};
  for (int n = 0; n < N; ++n) dims[n] = (int)x->dims[n];
  const int64_t chunk = 256;
  const int64_t waves = (x->nnz + chunk - 1) / chunk;
  const int blocks = (int)std::max<int64_t>(1, (waves + kCooThreads / 64 - 1) / (kCooThreads / 64));
  // workspace: accumulators M^(n) [dims][32], stats, objective partials
  Carve cv;
  float* M[4] = {};
  float* stats[4] = {};
  int64_t total_rows = 0;
  for (int n = 0; n < N; ++n) {
    M[n] = cv.take<float>((size_t)dims[n] * kRP);
    stats[n] = cv.take<float>((size_t)((dims[n] + kSlotRows - 1) / kSlotRows) * 96);
    total_rows += dims[n];
  }
  double* obj_part = cv.take<double>((size_t)blocks);
  const size_t need = cv.off + 256;
  int rc = ensure_ws(ctx, need, st);
  if (rc) return rc;
  Carve real;
  real.base = ctx->ws;
  for (int n = 0; n < N; ++n) {
    M[n] = real.take<float>((size_t)dims[n] * kRP);
    stats[n] = real.take<float>((size_t)((dims[n] + kSlotRows - 1) / kSlotRows) * 96);
  }
  obj_part = real.take<double>((size_t)blocks);

  // zero the accumulators (one contiguous range)
  {
    const int64_t n = (int64_t)(reinterpret_cast<char*>(stats[N - 1]) - reinterpret_cast<char*>(M[0])) / 4;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M[0], n);
    HIP_TRY(hipGetLastError());
  }
  CooPassArgs a = {};
  a.N = N;
  a.R = R;
  a.nnz = x->nnz;
  for (int n = 0; n < N; ++n) {
    a.dims[n] = dims[n];
    a.idx[n] = x->idx[n];
    a.A[n] = m->factors[n];
    a.M[n] = M[n];
  }
  a.val = x->val;
  a.eps = (float)o->eps;
  a.chunk = chunk;
  a.obj_part = obj_part;
  if (x->nnz > 0) {
    rc = profiled(ctx, st, [&] {
      hipLaunchKernelGGL(coo_pass_kernel, dim3(blocks), dim3(kCooThreads), 0, st, a);
      return hipGetLastError();
    });
    if (rc) return rc;
  }

  // c^(n) = M^(n) with column statistics, then the beta = 1 inner loop
  SlotUpdateArgs su = {};
  su.njobs = N;
  KlLoopArgs k = {};
  k.N = N;
  k.R = R;
  k.L = o->inner_sweeps;
  k.eps = (float)o->eps;
  for (int n = 0; n < N; ++n) {
    SlotJob& J = su.job[n];
    J.mode = kSlotCopy;
    J.num_part = M[n];
    J.num_slots = 1;
    J.rows_total = dims[n];
    J.rows = dims[n];
    J.cols = R;
    J.rows_p = dims[n];
    J.anchor = FView{m->factors[n], R, R};
    J.out_pad = nullptr;
    J.stats = stats[n];
    k.c[n] = M[n];
    k.stats[n] = stats[n];
    k.nblk[n] = (dims[n] + kSlotRows - 1) / kSlotRows;
    k.rows[n] = dims[n];
    k.cur_pad[n] = nullptr;
    k.user[n] = m->factors[n];
  }
  HIP_TRY(launch_slot_update(su, st));
  if (obj) {
    k.obj_part = x->nnz > 0 ? obj_part : nullptr;
    k.obj_n = x->nnz > 0 ? blocks : 0;
    k.obj_out = obj;
    k.obj_add_model_mass = 1;
  }
  HIP_TRY(launch_kl_apply(k, st));
  (void)total_rows;
  return COMM_OK;
}
