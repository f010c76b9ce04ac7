// Tucker pass kernels instantiated for beta = 3/2, general beta and the
// cached-weight reads, and the dispatch over all of them.
#include "tucker3_impl.h"

namespace comm {

hipError_t launch_tk_v_b(const TkPassArgs& a, int bc, int mode, bool obj, int sets, hipStream_t s) {
  if (bc == kThreeHalf) return launch_tk_v_bc<kThreeHalf>(a, mode, obj, sets, s);
  return launch_tk_v_bc<kGeneral>(a, mode, obj, sets, s);
}

hipError_t launch_tk_m3_b(const TkPassArgs& a, int bc, int sets, hipStream_t s) {
  if (bc == kThreeHalf) return launch_tk_m3_bc<kThreeHalf>(a, sets, s);
  return launch_tk_m3_bc<kGeneral>(a, sets, s);
}

hipError_t launch_tk_v(const TkPassArgs& a, int bc, int mode, bool obj, int sets, hipStream_t s) {
  if (mode == kTkCacheRead) {
    // the cached weights carry beta already: one instantiation serves every class
    if (sets != 2 || obj) return hipErrorInvalidValue;
    return launch_v<kGeneral, kTkCacheRead, false, 2>(a, s);
  }
  if (bc == kThreeHalf || bc == kGeneral) return launch_tk_v_b(a, bc, mode, obj, sets, s);
  return launch_tk_v_a(a, bc, mode, obj, sets, s);
}

hipError_t launch_tk_m3(const TkPassArgs& a, int bc, int mode, int sets, hipStream_t s) {
  if (mode == kTkCacheRead) {
    if (sets != 2) return hipErrorInvalidValue;
    return launch_m3<kGeneral, kTkCacheRead, 2>(a, s);
  }
  if (mode != kTkFromX) return hipErrorInvalidValue;
  if (bc == kThreeHalf || bc == kGeneral) return launch_tk_m3_b(a, bc, sets, s);
  return launch_tk_m3_a(a, bc, sets, s);
}

}  // namespace comm
