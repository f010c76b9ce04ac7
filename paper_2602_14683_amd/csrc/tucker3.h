// Dense Tucker: B-CoMM and J-CoMM orchestration, order 3 (tucker3.hip) and
// orders 4 and 5 (tuckern.hip); the entry points below take any of them.
#pragma once

#include "../../include/comm.h"

struct comm_ctx;

int tucker_check_model(const comm_model* m, const comm_dense* x);
size_t tucker_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op, int groups = 0);
int tucker_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st);
int tucker_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st);
int tucker_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                     hipStream_t st);

// Sparse COO data on the order-N path (any N = 3..5): the numerators come
// from the nonzeros; the dense passes, run on an all-zero tensor x of the
// same shape, give only the Q~ denominators and the zero cells' objective
// (none at all at beta = 1, whose denominators are closed form; x->X may then
// be NULL).  Buffers: w one float per nonzero, buf [round32(I_N)][32], obj one
// double per workgroup of the sparse kernel.
struct TkSparse {
  const comm_coo* coo;
  float* w;
  float* buf;
  double* obj;
};

int tuckern_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st,
                  const TkSparse* sp = nullptr);
int tuckern_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st,
                  const TkSparse* sp = nullptr);
int tuckern_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                      hipStream_t st, const TkSparse* sp = nullptr);
size_t tuckern_workspace_bytes(const comm_dense* x, const comm_model* m, const comm_opts* o, int op);
