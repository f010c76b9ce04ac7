// Dense Tucker: B-CoMM and J-CoMM orchestration, order 3 (tucker3.hip) and
// orders 4 and 5 (tuckern.hip); the entry points below take any of them.
#pragma once

#include "../../include/comm.h"

struct comm_ctx;

int tucker_check_model(const comm_model* m, const comm_dense* x);
size_t tucker_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op);
int tucker_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st);
int tucker_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st);
int tucker_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                     hipStream_t st);

int tuckern_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st);
int tuckern_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st);
int tuckern_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                      hipStream_t st);
size_t tuckern_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op);
