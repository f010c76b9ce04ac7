// Dense 3-way Tucker (placeholder until the fused Tucker pass lands).
#include <hip/hip_runtime.h>

#include "tucker3.h"

int tucker_check_model(const comm_model* m, const comm_dense* x) {
  (void)m; (void)x;
  return COMM_EUNSUPPORTED;
}
size_t tucker_workspace_bytes(const comm_dense*, const comm_model*, const comm_opts*, int) { return 0; }
int tucker_bcomm(comm_ctx*, const comm_dense*, comm_model*, int, const comm_opts*, hipStream_t) { return COMM_EUNSUPPORTED; }
int tucker_jcomm(comm_ctx*, const comm_dense*, comm_model*, const comm_opts*, double*, hipStream_t) { return COMM_EUNSUPPORTED; }
int tucker_objective(comm_ctx*, const comm_dense*, const comm_model*, const comm_opts*, double*, hipStream_t) {
  return COMM_EUNSUPPORTED;
}
