// Fused dense CP pass instantiated for one beta class.
#include "cp3_impl.h"

namespace comm {

hipError_t launch_bc_threehalf(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s) {
  return launch_bc<kThreeHalf>(a, g, den, s);
}

hipError_t launch_vpass_threehalf(const CpPassArgs& a, hipStream_t s) { return launch_vpass_bc<kThreeHalf>(a, s); }

}  // namespace comm
