// Fused dense CP pass instantiated for one beta class.
#include "cp3_impl.h"

namespace comm {

template <>
hipError_t launch_bc<kKL>(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s) {
  if (den || a.cache_mode == 1) return hipErrorInvalidValue;
  return a.want_obj ? launch_v<kKL, kNumOnly, true>(a, g, s) : launch_v<kKL, kNumOnly, false>(a, g, s);
}

hipError_t launch_bc_kl(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s) {
  return launch_bc<kKL>(a, g, den, s);
}

}  // namespace comm
