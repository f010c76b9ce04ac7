// Tucker pass kernels instantiated for beta = 0, 1/2, 1.
#include "tucker3_impl.h"

namespace comm {

hipError_t launch_tk_v_a(const TkPassArgs& a, int bc, int mode, bool obj, int sets, hipStream_t s) {
  switch (bc) {
    case kIS: return launch_tk_v_bc<kIS>(a, mode, obj, sets, s);
    case kHalf: return launch_tk_v_bc<kHalf>(a, mode, obj, sets, s);
    default: return launch_tk_v_bc<kKL>(a, mode, obj, sets, s);
  }
}

hipError_t launch_tk_m3_a(const TkPassArgs& a, int bc, int sets, hipStream_t s) {
  switch (bc) {
    case kIS: return launch_tk_m3_bc<kIS>(a, sets, s);
    case kHalf: return launch_tk_m3_bc<kHalf>(a, sets, s);
    default: return launch_tk_m3_bc<kKL>(a, sets, s);
  }
}

}  // namespace comm
