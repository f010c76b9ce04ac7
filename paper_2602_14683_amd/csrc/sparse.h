// Sparse COO CP J-CoMM at beta = 1 (sparse.hip).
#pragma once

#include "../../include/comm.h"

struct comm_ctx;

int coo_jcomm_kl(comm_ctx* ctx, const comm_coo* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st);
