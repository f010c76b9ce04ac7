// Sparse COO CP J-CoMM at beta = 1 (placeholder until the COO kernel lands).
#include <hip/hip_runtime.h>

#include "sparse.h"

int coo_jcomm_kl(comm_ctx*, const comm_coo*, comm_model*, const comm_opts*, double*, hipStream_t) {
  return COMM_EUNSUPPORTED;
}
