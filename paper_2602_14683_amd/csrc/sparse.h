// Sparse COO CP J-CoMM at beta = 1 (sparse.hip).
#pragma once

#include "../../include/comm.h"

struct comm_ctx;

int coo_jcomm_kl(comm_ctx* ctx, const comm_coo* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st);
int coo_jcomm_kl_plan(comm_ctx* ctx, const comm_coo_plan* p, comm_model* m, const comm_opts* o, double* obj,
                      hipStream_t st);
int coo_objective_kl(comm_ctx* ctx, const comm_coo* x, const comm_model* m, const comm_opts* o, double* out,
                     hipStream_t st);
int coo_plan_build(comm_ctx* ctx, const comm_coo* x, comm_coo_plan** out, hipStream_t st);
int coo_plan_free(comm_coo_plan* p);
int coo_plan_ndim(const comm_coo_plan* p);
int64_t coo_plan_dim(const comm_coo_plan* p, int n);
