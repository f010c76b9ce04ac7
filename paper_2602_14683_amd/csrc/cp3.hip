// Dispatch of the fused dense 3-way CP pass (kernel templates in cp3_impl.h;
// one translation unit per beta class so that they compile in parallel).

#include "cp3_impl.h"

namespace comm {

CpGrid cp_grid(int I, int J, int K) { return cp_grid_impl(I, J, K); }

hipError_t launch_cp_pass(const CpPassArgs& a, const CpGrid& g, int beta_class, bool den, hipStream_t s) {
  if (a.cache_mode == 2) return launch_cache_read(a, g, s);
  switch (beta_class) {
    case kIS: return launch_bc_is(a, g, den, s);
    case kHalf: return launch_bc_half(a, g, den, s);
    case kKL: return launch_bc_kl(a, g, den, s);
    case kThreeHalf: return launch_bc_threehalf(a, g, den, s);
    default: return launch_bc_general(a, g, den, s);
  }
}

int64_t cp_vpass_wgs(int I, int J) { return vpass_wgs(I, J); }
int cp_vpass_m1_slots(int J) { return (J + kVTJ - 1) / kVTJ; }

hipError_t launch_cp_vpass(const CpPassArgs& a, int beta_class, hipStream_t s) {
  if (a.cache_mode == 2) return launch_vpass_cache(a, s);
  switch (beta_class) {
    case kIS: return launch_vpass_is(a, s);
    case kHalf: return launch_vpass_half(a, s);
    case kThreeHalf: return launch_vpass_threehalf(a, s);
    case kGeneral: return launch_vpass_general(a, s);
    default: return hipErrorInvalidValue;  // beta = 1 has no denominator pass
  }
}

// M2 chunks from the kept V (see launch_vfold): thread = (j, r) of an 8-j
// block, sum over its chunk of i in order.
__device__ __forceinline__ void vfold_body(const VFoldArgs& a, uint3 bid, uint3) {
  const int jl = threadIdx.x >> 5, r = threadIdx.x & 31;
  const int j = bid.x * 8 + jl;
  const int c = bid.y;
  const bool den = bid.z == 1;
  if (j >= a.J) return;
  const int ci = (a.I + kVFoldChunks - 1) / kVFoldChunks;
  const int ib = c * ci, ie = min(a.I, ib + ci);
  const float* V = den ? a.Vd : a.Vn;
  const FView& A = den ? a.Ad : a.An;
  float s0 = 0.0f, s1 = 0.0f;
  int i = ib;
  for (; i + 1 < ie; i += 2) {
    s0 = fmaf(V[((size_t)i * a.J + j) * kRP + r], A.at(i, r, a.I), s0);
    s1 = fmaf(V[((size_t)(i + 1) * a.J + j) * kRP + r], A.at(i + 1, r, a.I), s1);
  }
  if (i < ie) s0 = fmaf(V[((size_t)i * a.J + j) * kRP + r], A.at(i, r, a.I), s0);
  float* out = den ? a.outd : a.outn;
  out[((size_t)c * a.Jp + j) * kRP + r] = s0 + s1;
}
COMM_GROUPED_KERNELS(vfold, VFoldArgs, 256)

hipError_t launch_vfold(const VFoldArgs& a, hipStream_t s) {
  return launch_or_record(vfold_kernel, vfold_grouped, dim3((unsigned)((a.J + 7) / 8), kVFoldChunks, 2), dim3(256), 0,
                          s, a);
}

}  // namespace comm
