// Fused dense Tucker pass instantiated for beta = 0, 1/2, 1.
#include "tucker3_impl.h"

namespace comm {

hipError_t launch_tk_a(const TkPassArgs& a, const TkGrid& g, int bc, int mode, bool obj, hipStream_t s) {
  switch (bc) {
    case kIS: return launch_tk_bc<kIS>(a, g, mode, obj, s);
    case kHalf: return launch_tk_bc<kHalf>(a, g, mode, obj, s);
    default: return launch_tk_bc<kKL>(a, g, mode, obj, s);
  }
}

}  // namespace comm
