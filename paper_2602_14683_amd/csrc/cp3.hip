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

}  // namespace comm
