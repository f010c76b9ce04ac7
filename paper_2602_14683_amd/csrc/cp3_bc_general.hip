// Fused dense CP pass instantiated for one beta class.
#include "cp3_impl.h"

namespace comm {

hipError_t launch_bc_general(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s) {
  return launch_bc<kGeneral>(a, g, den, s);
}

hipError_t launch_cache_read(const CpPassArgs& a, const CpGrid& g, hipStream_t s) {
  return launch_v<kGeneral, kCacheNumDen, false>(a, g, s);
}

hipError_t launch_vpass_general(const CpPassArgs& a, hipStream_t s) { return launch_vpass_bc<kGeneral>(a, s); }

hipError_t launch_vpass_cache(const CpPassArgs& a, hipStream_t s) { return launch_vpass_t<kGeneral, true, false>(a, s); }

}  // namespace comm
