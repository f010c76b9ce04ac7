// Dense Tucker: B-CoMM and J-CoMM orchestration, order 3 (tucker3.hip) and
// order 4 (tucker4.hip); the entry points below take either.
#pragma once

#include "../../include/comm.h"

struct comm_ctx;

int tucker_check_model(const comm_model* m, const comm_dense* x);
size_t tucker_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op);
int tucker_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st);
int tucker_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st);
int tucker_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                     hipStream_t st);

int tucker4_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st);
int tucker4_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st);
int tucker4_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                      hipStream_t st);
size_t tucker4_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op);
