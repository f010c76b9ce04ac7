// Fused dense Tucker pass instantiated for beta = 3/2, general beta, and the
// cached-weight variant.
#include "tucker3_impl.h"

namespace comm {

hipError_t launch_tk_b(const TkPassArgs& a, const TkGrid& g, int bc, int mode, bool obj, hipStream_t s) {
  if (mode == kTkCacheRead) return launch_tk<kGeneral, kTkCacheRead, false>(a, g, s);
  if (bc == kThreeHalf) return launch_tk_bc<kThreeHalf>(a, g, mode, obj, s);
  return launch_tk_bc<kGeneral>(a, g, mode, obj, s);
}

hipError_t launch_tk_pass(const TkPassArgs& a, const TkGrid& g, int beta_class, int mode, hipStream_t s) {
  const bool obj = (mode & 4) != 0;
  const int m = mode & 3;
  if (m == kTkCacheRead || beta_class == kThreeHalf || beta_class == kGeneral) return launch_tk_b(a, g, beta_class, m, obj, s);
  return launch_tk_a(a, g, beta_class, m, obj, s);
}

}  // namespace comm
