// Sparse COO J-CoMM for CP at beta = 1 (Sec. 6.4, paragraph on sparse
// tensors): numerators accumulate over the nonzeros only, and the beta = 1
// denominator prod_{m != n} colsum(A^(m)) is closed-form (Q~ = 1).
//
// Per nonzero (i, x): z_r = prod_m A~^(m)_{i_m r}, X~ = max(sum_r z_r, eps),
// w_r = x z_r / X~, and for every mode n, M^(n)[i_n][r] += w_r.  Since
// Num_J^(n)[i_n][r] = sum_nz (x / X~) prod_{m != n} A~^(m) = M^(n)[i_n][r] / A~^(n)[i_n][r],
// the product c^(n) = A~^(n) * Num_J^(n) that drives the beta = 1 inner loop
// (kernels_small.hip) is M^(n) itself.
//
// Mapping: one nonzero per half wavefront, lane = rank component.  Each half
// wave takes one contiguous half of its wave's chunk (a run of equal
// coordinates is split only at a half's ends), loads 32 nonzeros'
// coordinates and values with coalesced loads (validity checked once, kept as
// a ballot mask) and hands them out by lane permutes, four nonzeros at a time
// so that their factor-row gathers (128-byte rows that stay in L2, 32-bit
// offsets from the factors' bases) are in flight together; X~ is a half-wave
// reduction (DPP, then one permute), and the objective is evaluated once per
// nonzero by the lane that loaded it.  Modes
// whose coordinate the stream is sorted by come in runs: each half keeps a
// running sum per such mode and adds it to global memory when the
// coordinate changes.  Other modes are added per nonzero.  Both use hardware
// float atomics, so this path is reproducible to rounding, not bitwise.
// Nonzeros with a coordinate outside [0, dims) are skipped.
//
// Without a plan (comm_cp_jcomm_outer_coo) one pass over the caller's COO
// accumulates modes 1 and 2 by runs (the COO is expected sorted) and the
// others per nonzero; per-nonzero atomics on a heavily repeated coordinate
// serialise.  A plan (comm_coo_plan_create) keeps two device copies of the
// COO, sorted by (i1, i2) and by (i3, i4), and each outer iteration makes one
// pass over each, every mode accumulated by runs.
//
// Objective at the reference: nonzero cells contribute d_1(x | X~) (stable
// form), zero cells contribute X~, which sums in closed form over all cells as
// sum_r prod_n colsum(A~^(n))_r minus the nonzero cells' X~.

#include <hipcub/hipcub.hpp>

#include "host_util.h"
#include "sparse.h"
#include "cp3_impl.h"

struct comm_coo_plan {
  int device = 0;
  int ndim = 0;
  int64_t dims[4] = {0, 0, 0, 0};
  int64_t nnz = 0;
  int copies = 0;                 // 1 (order 2) or 2
  int order[2][4] = {};           // copy c holds mode order[c][q] in its slot q
  int runs[2] = {0, 0};           // leading modes of copy c it is sorted by
  int32_t* idx[2][4] = {};
  float* val[2] = {};
  char* mem = nullptr;
};

namespace comm {

struct CooPassArgs {
  int N, R;
  int64_t nnz;
  int dims[kMaxModes];            // in the stream's slot order
  const int32_t* idx[kMaxModes];
  const float* val;
  const float* A[kMaxModes];      // factors, slot order, row stride R
  float* M[kMaxModes];            // [dims][32] accumulators, slot order (no accumulation: unused)
  int run_modes;          // slots [0, run_modes) accumulated by runs
  int atom_modes;         // slots [run_modes, run_modes + atom_modes) per nonzero
  float eps;
  int64_t chunk;          // nonzeros per wavefront, a multiple of 64
  double* obj_part;       // per workgroup: sum d_1(x | X~) - sum X~ (NULL: no objective)
};

constexpr int kCooThreads = 256;
constexpr int kCooBatch = 4;   // nonzeros per half wave whose gathers are issued together

// Sum over the 32 lanes of a half wave (all receive it): xor 1 and xor 2 in
// the quad, the mirrored lane of the other quad, the mirrored lane of the
// other half row (DPP), then the other row of 16 (lane permute).
__device__ __forceinline__ float half_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));  // row_half_mirror
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));  // row_mirror
  return v + __shfl_xor(v, 16);
}

template <int N, int kRuns, int kAtoms>
__global__ void __launch_bounds__(kCooThreads) coo_pass_kernel(CooPassArgs a) {
  __shared__ double lobj[kCooThreads / 64][2];
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
  const int64_t wave = ((int64_t)blockIdx.x * kCooThreads + threadIdx.x) >> 6;
  const int R = a.R;
  const bool rlive = r < R;
  const int rcol = rlive ? r : R - 1;
  const uint32_t rcol4 = 4u * (uint32_t)rcol;
  const uint32_t R4 = 4u * (uint32_t)R;
  // the wave's chunk, each half wave one contiguous half of it, so that a run
  // of equal coordinates is split only where a half's range ends
  const int64_t w0 = min(a.nnz, wave * a.chunk);
  const int64_t w1 = min(a.nnz, w0 + a.chunk);
  const int64_t half0 = (w1 - w0 + 1) >> 1;
  const int64_t hb = w0 + (h ? half0 : 0);
  const int64_t he = h ? w1 : w0 + half0;
  const int64_t steps = (half0 + 31) >> 5;   // batches of 32 per half (half 0 is the longer)

  int cur[2] = {-1, -1};
  float acc[2] = {0.0f, 0.0f};
  double obj = 0.0, objc = 0.0;   // compensated sum of the objective terms
  for (int64_t sb = 0; sb < steps; ++sb) {
    // 32 nonzeros per half, one per lane, coalesced; validity once per
    // nonzero; a nonzero that is not valid reads row 0
    const int64_t t = hb + sb * 32 + r;
    const int cnt = (int)max((int64_t)0, min((int64_t)32, he - (hb + sb * 32)));
    int my[N];
    float myx = 0.0f;
    bool valid = r < cnt;
#pragma unroll
    for (int m = 0; m < N; ++m) my[m] = 0;
    if (valid) {
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const int i = a.idx[m][t];
        valid = valid && i >= 0 && i < a.dims[m];
        my[m] = i;
      }
      myx = a.val[t];
    }
    if (!valid) {
#pragma unroll
      for (int m = 0; m < N; ++m) my[m] = 0;
    }
    const uint64_t okmask = __ballot(valid);
    const int cmax = max(__shfl(cnt, 0), __shfl(cnt, 32));
    float myy = 1.0f;   // X~ of this lane's own nonzero, for the objective
    for (int j0 = 0; j0 < cmax; j0 += kCooBatch) {
      int ii[kCooBatch][N];
      float xs[kCooBatch], zs[kCooBatch];
      bool oks[kCooBatch];
#pragma unroll
      for (int u = 0; u < kCooBatch; ++u) {
        const int src = (h << 5) + j0 + u;
        oks[u] = (okmask >> src) & 1;
#pragma unroll
        for (int m = 0; m < N; ++m) ii[u][m] = __shfl(my[m], src);
        xs[u] = __shfl(myx, src);
      }
      // every gather of the batch is issued before the first use, each a
      // 32-bit offset from the factor's (uniform) base
      float g[kCooBatch][N];
#pragma unroll
      for (int u = 0; u < kCooBatch; ++u)
#pragma unroll
        for (int m = 0; m < N; ++m)
          g[u][m] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(a.A[m]) +
                                                     ((uint32_t)ii[u][m] * R4 + rcol4));
#pragma unroll
      for (int u = 0; u < kCooBatch; ++u) {
        float z = g[u][0];
#pragma unroll
        for (int m = 1; m < N; ++m) z *= g[u][m];
        zs[u] = (oks[u] && rlive) ? z : 0.0f;
      }
      float y[kCooBatch];
#pragma unroll
      for (int u = 0; u < kCooBatch; ++u) y[u] = fmaxf(half_sum(zs[u]), a.eps);
#pragma unroll
      for (int u = 0; u < kCooBatch; ++u)
        if (r == j0 + u) myy = y[u];
#pragma unroll
      for (int u = 0; u < kCooBatch; ++u) {
        if (!oks[u]) continue;
        const float w = zs[u] * (xs[u] * fast_rcp(y[u]));
#pragma unroll
        for (int q = 0; q < kRuns; ++q) {
          if (ii[u][q] != cur[q]) {
            if (cur[q] >= 0 && rlive) unsafeAtomicAdd(&a.M[q][(int64_t)cur[q] * kRP + r], acc[q]);
            cur[q] = ii[u][q];
            acc[q] = 0.0f;
          }
          acc[q] += w;
        }
        if (rlive) {
#pragma unroll
          for (int q = kRuns; q < kRuns + kAtoms; ++q) unsafeAtomicAdd(&a.M[q][(int64_t)ii[u][q] * kRP + r], w);
        }
      }
    }
    if (a.obj_part && valid) {
      bool far;
      float d = kl_series(myx, myy, fast_rcp(myx + myy), far);
      if (far) d = kl_direct(myx, myy);
      sum2_add(obj, objc, (double)d - (double)myy);
    }
  }
  if (rlive) {
#pragma unroll
    for (int q = 0; q < kRuns; ++q)
      if (cur[q] >= 0) unsafeAtomicAdd(&a.M[q][(int64_t)cur[q] * kRP + r], acc[q]);
  }
  if (a.obj_part) {
    sum2_wave(obj, objc);
    if (lane == 0) {
      lobj[threadIdx.x >> 6][0] = obj;
      lobj[threadIdx.x >> 6][1] = objc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = lobj[0][0], c = lobj[0][1];
      for (int q = 1; q < kCooThreads / 64; ++q) {
        sum2_add(s, c, lobj[q][0]);
        c += lobj[q][1];
      }
      a.obj_part[blockIdx.x] = s + c;
    }
  }
}

// ------------------------------------------------------------------ plan pass
//
// The pass over one sorted copy of a plan: the copy's leading slots
// accumulate by runs; its other slots are not accumulated (the other copy
// covers them).  Same mapping and arithmetic as coo_pass_kernel (one nonzero
// per half wave, lane = rank component, each half one contiguous half of the
// wave's chunk), with the per-nonzero bookkeeping moved out of the step:
//
// * Staging.  Each half's nonzeros are taken 32 at a time (a window): lane r
//   of half h loads nonzero 32 W + r of its half (coalesced), checks its
//   coordinates, and writes the byte offsets i_q R 4 of its factor rows and
//   its value to the wave's LDS buffer.  A nonzero with a coordinate outside
//   [0, dims) gets the value 0 and that coordinate 0; steps past the end of a
//   half read its last nonzero with the value 0.  Both contribute exactly
//   nothing (w = 0, objective term 0) and need no test in the step.  Window
//   W + 1 is loaded while window W is consumed; two buffers alternate.
// * Step.  A lane reads its half's offsets and value for the step with one
//   16-byte and one 4-byte LDS read at fixed offsets, adds its column, and
//   gathers; the gathers of the next four steps are issued before the
//   current four are evaluated.  A run ends where the row offset changes.
// * X~ is the half-wave sum by DPP within rows of 16 and one
//   v_permlane16_swap across the two rows (both rows add in the same order,
//   so every lane of a half holds the same value).
struct CooPlanPassArgs {
  int R;
  int64_t nnz;
  int dims[4];              // slot order
  const int32_t* idx[4];
  const float* val;
  const float* A[4];        // factors, slot order, row stride R
  float* M[4];              // accumulators, slot order: replicas of [dims][32]
  int64_t mrep[4];          // floats between replicas
  int rep_mask;             // workgroup b adds into replica b & rep_mask
  float eps;
  float inv_r4;             // 1 / (4 R): row of a byte offset (R < 32)
  int64_t chunk;            // nonzeros per wavefront
  double* obj_part;         // per workgroup, as in coo_pass_kernel (NULL: no objective)
};

constexpr int kPlanStep = 4;   // steps per batch of gathers

// Half-wave sum for the plan pass: DPP within each row of 16, then the other
// row of the half by ds_swizzle (xor 16 within 32 lanes), which costs no
// vector instruction; a + b and b + a are the same float, so both rows hold
// the same sum.
__device__ __forceinline__ float half_sum_swap(float v) {
  // (every source lane of these patterns exists: bound_ctrl changes nothing)
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));   // quad_perm 1,0,3,2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));   // quad_perm 2,3,0,1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, true));  // row_half_mirror
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, true));  // row_mirror
  // bit mode: and 0x1f, or 0, xor 0x10
  return v + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}

template <int N, int kRuns, bool kObj, bool kFullR>
__global__ void __launch_bounds__(kCooThreads) coo_plan_pass_kernel(CooPlanPassArgs a) {
  constexpr int kW = kCooThreads / 64;
  __shared__ uint4 s_off[kW][2][64];
  __shared__ float s_x[kW][2][64];
  __shared__ float s_y[kW][64];      // X~ of each step of the current window
  __shared__ double lobj[kW][2];
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kW + wv;
  const int R = a.R;
  const bool rlive = kFullR || r < R;
  const uint32_t rcol4 = 4u * (uint32_t)(kFullR ? r : min(r, R - 1));
  const uint32_t R4 = 4u * (uint32_t)R;
  const int64_t w0 = min(a.nnz, wave * a.chunk);
  const int64_t w1 = min(a.nnz, w0 + a.chunk);
  const int len = (int)(w1 - w0);
  const int len0 = (len + 1) >> 1;             // half 0 is the longer half
  const int lenh = h ? len - len0 : len0;
  const int64_t bh = w0 + (h ? len0 : 0);
  double obj = 0.0, objc = 0.0;   // compensated sum of the objective terms

  if (len > 0) {
    // ---- staging of window W into the lane's registers (lane = nonzero)
    int li[N];
    float lx;
    auto load_window = [&](int W) {
      const int t = W * 32 + r;
      const int64_t e = bh + min(t, lenh - 1);   // lenh = 0: half 0's last nonzero
#pragma unroll
      for (int q = 0; q < N; ++q) li[q] = a.idx[q][e];
      lx = t < lenh ? a.val[e] : 0.0f;
    };
    auto store_window = [&](int buf) {
      bool ok = true;
      uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int q = 0; q < N; ++q) {
        const bool in = li[q] >= 0 && li[q] < a.dims[q];
        ok = ok && in;
        o[q] = in ? (uint32_t)li[q] * R4 : 0u;
      }
      s_off[wv][buf][lane] = make_uint4(o[0], o[1], o[2], o[3]);
      s_x[wv][buf][lane] = ok ? lx : 0.0f;
    };
    auto lds_sync = [&] {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    const int windows = (len0 + 31) >> 5;
    // window 0 into both buffers (every buffer then holds valid offsets, so
    // the gathers issued one batch past the last window stay in bounds)
    load_window(0);
    store_window(0);
    store_window(1);
    if (windows > 1) load_window(1);
    lds_sync();

    // A run starts at the half's first nonzero; every flush is then real.
    // Runs are tracked by the row's byte offset; at rank 32 with the lane's
    // column added, which is also the lane's byte offset in the [dims][32]
    // accumulator (both rows are 128 bytes), so a flush needs no address
    // arithmetic.
    const uint32_t rkey = kFullR ? rcol4 : 0u;
    uint32_t cur[kRuns];
    float acc[kRuns];
    {
      const uint4 o4 = s_off[wv][0][32 * h];
      const uint32_t o[4] = {o4.x, o4.y, o4.z, o4.w};
#pragma unroll
      for (int q = 0; q < kRuns; ++q) {
        cur[q] = o[q] + rkey;
        acc[q] = 0.0f;
      }
    }

    // one batch: four steps' gathers, their run offsets and values
    struct Batch {
      float g[kPlanStep][N];
      uint32_t ro[kPlanStep][kRuns];
      float x[kPlanStep];
    };
    // steps j0 .. j0 + 3 of the window in buffer buf (jj = j0 mod 32)
    auto issue = [&](int buf, int jj, Batch& B) {
#pragma unroll
      for (int u = 0; u < kPlanStep; ++u) {
        const uint4 o4 = s_off[wv][buf][32 * h + jj + u];
        B.x[u] = s_x[wv][buf][32 * h + jj + u];
        const uint32_t o[4] = {o4.x, o4.y, o4.z, o4.w};
#pragma unroll
        for (int q = 0; q < N; ++q)
          B.g[u][q] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(a.A[q]) + (o[q] + rcol4));
#pragma unroll
        for (int q = 0; q < kRuns; ++q) B.ro[u][q] = o[q] + rkey;
      }
    };
    const int64_t rep = (int64_t)(blockIdx.x & (unsigned)a.rep_mask);
    float* Mq[kRuns];
#pragma unroll
    for (int q = 0; q < kRuns; ++q) Mq[q] = a.M[q] + rep * a.mrep[q];
    // the accumulator entry of run key o (R < 32: the row from the offset)
    auto acc_at = [&](int q, uint32_t o) -> float* {
      if constexpr (kFullR) return reinterpret_cast<float*>(reinterpret_cast<char*>(Mq[q]) + o);
      const uint32_t row = (uint32_t)fmaf((float)o, a.inv_r4, 0.5f);
      return Mq[q] + (int64_t)row * kRP + r;
    };
    auto consume = [&](int jj, const Batch& B) {
#pragma unroll
      for (int u = 0; u < kPlanStep; ++u) {
        float z = B.g[u][0];
#pragma unroll
        for (int q = 1; q < N; ++q) z *= B.g[u][q];
        if (!kFullR) z = rlive ? z : 0.0f;
        // (z is pinned: left free, the compiler folds its last product into
        // the first DPP add and computes it twice)
        asm volatile("" : "+v"(z));
        const float y = fmaxf(half_sum_swap(z), a.eps);
        const float w = z * (B.x[u] * fast_rcp(y));
        if constexpr (kRuns == 1) {
          if (B.ro[u][0] != cur[0]) {
            if (rlive) unsafeAtomicAdd(acc_at(0, cur[0]), acc[0]);
            cur[0] = B.ro[u][0];
            acc[0] = 0.0f;
          }
          acc[0] += w;
        } else {
          // slot 1's runs nest in slot 0's (the copy is sorted by both), so
          // slot 0 accumulates slot 1's finished runs instead of every w;
          // slot 1's run also ends where slot 0 changes
          const bool c0 = B.ro[u][0] != cur[0];
          if (c0 || B.ro[u][1] != cur[1]) {
            if (rlive) unsafeAtomicAdd(acc_at(1, cur[1]), acc[1]);
            acc[0] += acc[1];
            acc[1] = 0.0f;
            cur[1] = B.ro[u][1];
            if (c0) {
              if (rlive) unsafeAtomicAdd(acc_at(0, cur[0]), acc[0]);
              acc[0] = 0.0f;
              cur[0] = B.ro[u][0];
            }
          }
          acc[1] += w;
        }
        // X~ of the step for the objective (one lane per half: a lane
        // compare per step would pin 32 hoisted masks in scalar registers)
        if (kObj && r == 0) s_y[wv][32 * h + jj + u] = y;
      }
    };

    // One iteration per window of 32 steps, eight batches; the gathers of
    // the next batch are always issued before the current one is evaluated
    // (past the last step they read valid offsets and go unused).  Steps past
    // the end of a half carry the value 0.
    Batch bA, bB;
    issue(0, 0, bA);
    for (int W = 0; W < windows; ++W) {
      const int buf = W & 1;
#pragma unroll
      for (int k = 0; k < 8; k += 2) {
        issue(buf, 4 * (k + 1), bB);
        consume(4 * k, bA);
        if (k + 2 < 8) {
          issue(buf, 4 * (k + 2), bA);
        } else {
          // window W + 1 into the other buffer (loaded a window ago), the
          // loads of window W + 2, then the first batch of window W + 1
          if (W + 1 < windows) {
            store_window(buf ^ 1);
            if (W + 2 < windows) load_window(W + 2);
          }
          lds_sync();
          issue(buf ^ 1, 0, bA);
        }
        consume(4 * (k + 1), bB);
      }
      if (kObj) {
        // the lane's own nonzero of window W (value 0 past its half: term 0)
        lds_sync();
        const float x = s_x[wv][buf][lane];
        const float myy = s_y[wv][lane];
        bool far;
        float d = kl_series(x, myy, fast_rcp(x + myy), far);
        if (far) d = kl_direct(x, myy);
        sum2_add(obj, objc, (double)d - (double)myy);
      }
    }
    if (rlive) {
      if constexpr (kRuns == 2) {
        unsafeAtomicAdd(acc_at(1, cur[1]), acc[1]);
        acc[0] += acc[1];
      }
      unsafeAtomicAdd(acc_at(0, cur[0]), acc[0]);
    }
  }
  if (a.obj_part) {
    sum2_wave(obj, objc);
    if (lane == 0) {
      lobj[wv][0] = obj;
      lobj[wv][1] = objc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = lobj[0][0], c = lobj[0][1];
      for (int q = 1; q < kW; ++q) {
        sum2_add(s, c, lobj[q][0]);
        c += lobj[q][1];
      }
      a.obj_part[blockIdx.x] = s + c;
    }
  }
}

template <int N, int kRuns>
hipError_t launch_plan_pass_n(const CooPlanPassArgs& a, int blocks, hipStream_t st) {
  const dim3 grid((unsigned)blocks), block(kCooThreads);
  const bool full = a.R == 32;
  if (a.obj_part) {
    if (full) launch_timed(coo_plan_pass_kernel<N, kRuns, true, true>, grid, block, 0, st, a);
    else launch_timed(coo_plan_pass_kernel<N, kRuns, true, false>, grid, block, 0, st, a);
  } else {
    if (full) launch_timed(coo_plan_pass_kernel<N, kRuns, false, true>, grid, block, 0, st, a);
    else launch_timed(coo_plan_pass_kernel<N, kRuns, false, false>, grid, block, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_plan_pass(const CooPlanPassArgs& a, int N, int runs, int blocks, hipStream_t st) {
  if (N == 2 && runs == 2) return launch_plan_pass_n<2, 2>(a, blocks, st);
  if (N == 3 && runs == 2) return launch_plan_pass_n<3, 2>(a, blocks, st);
  if (N == 3 && runs == 1) return launch_plan_pass_n<3, 1>(a, blocks, st);
  if (N == 4 && runs == 2) return launch_plan_pass_n<4, 2>(a, blocks, st);
  return hipErrorInvalidValue;
}

template <int N>
hipError_t launch_coo_n(const CooPassArgs& a, int blocks, hipStream_t st) {
  const dim3 grid((unsigned)blocks), block(kCooThreads);
  if (a.run_modes == 0 && a.atom_modes == 0) launch_timed(coo_pass_kernel<N, 0, 0>, grid, block, 0, st, a);
  else if constexpr (N <= 4) {
    if (a.run_modes == 2 && a.atom_modes == N - 2) launch_timed(coo_pass_kernel<N, 2, N - 2>, grid, block, 0, st, a);
    else if (a.run_modes == 2 && a.atom_modes == 0) launch_timed(coo_pass_kernel<N, 2, 0>, grid, block, 0, st, a);
    else if (a.run_modes == 1 && a.atom_modes == 0) launch_timed(coo_pass_kernel<N, 1, 0>, grid, block, 0, st, a);
    else return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// (order 5 only without accumulation: the objective)
hipError_t launch_coo(const CooPassArgs& a, int blocks, hipStream_t st) {
  switch (a.N) {
    case 2: return launch_coo_n<2>(a, blocks, st);
    case 3: return launch_coo_n<3>(a, blocks, st);
    case 4: return launch_coo_n<4>(a, blocks, st);
    case 5: return launch_coo_n<5>(a, blocks, st);
    default: return hipErrorInvalidValue;
  }
}

// The model's mass over every cell, sum_r prod_n colsum(A^(n))_r, in float64
// (the column sums too), written to out[0].  One workgroup: thread t sums
// rows t / 32, t / 32 + 32, ... of column t % 32; the 32 row groups are
// combined in order.
struct MassArgs {
  int N, R;
  int rows[kMaxModes];
  const float* A[kMaxModes];   // row stride R
  double* out;
};

__global__ void __launch_bounds__(1024) model_mass_kernel(MassArgs a) {
  __shared__ double part[1024];
  __shared__ double cs[kMaxModes][32];
  const int t = threadIdx.x;
  const int c = t & 31, g = t >> 5;
  for (int n = 0; n < a.N; ++n) {
    double s = 0.0;
    if (c < a.R)
      for (int i = g; i < a.rows[n]; i += 32) s += (double)a.A[n][(int64_t)i * a.R + c];
    part[t] = s;
    __syncthreads();
    if (t < 32) {
      double v = 0.0;
      for (int gg = 0; gg < 32; ++gg) v += part[gg * 32 + t];
      cs[n][t] = v;
    }
    __syncthreads();
  }
  if (t == 0) {
    double mass = 0.0;
    for (int r = 0; r < a.R; ++r) {
      double p = 1.0;
      for (int n = 0; n < a.N; ++n) p *= cs[n][r];
      mass += p;
    }
    a.out[0] = mass;
  }
}

// The accumulators' replicas added (fixed order) into replica 0, which
// becomes c^(n), with the column statistics of kl_apply per block of 32 rows:
// sum of c, min of c over the block's rows, sum of the anchor A~^(n).  One
// workgroup per (mode, 32-row block), thread (row, column).
constexpr int kSumRows = 32;
struct CooSumArgs {
  int N, R, reps;
  int rows[kMaxModes];
  int first_block[kMaxModes + 1];   // workgroups of modes before n
  float* M[kMaxModes];              // reps replicas of [rows][32]
  const float* anchor[kMaxModes];   // row stride R
  float* stats[kMaxModes];          // [blocks][3][32]
};

__global__ void __launch_bounds__(1024) coo_sum_kernel(CooSumArgs a) {
  __shared__ float red[3][kSumRows][33];
  const int t = threadIdx.x;
  const int c = t & 31, rl = t >> 5;
  int n = 0;
  while (n + 1 < a.N && (int)blockIdx.x >= a.first_block[n + 1]) ++n;
  const int b = (int)blockIdx.x - a.first_block[n];
  const int row = b * kSumRows + rl;
  const bool in = row < a.rows[n];
  const int64_t e = (int64_t)row * kRP + c;
  const int64_t stride = (int64_t)a.rows[n] * kRP;
  float v = 0.0f, anc = 0.0f;
  if (in) {
    float part[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) part[s] = s < a.reps ? a.M[n][s * stride + e] : 0.0f;
    v = part[0];
#pragma unroll
    for (int s = 1; s < 8; ++s) v += part[s];
    for (int s = 8; s < a.reps; ++s) v += a.M[n][s * stride + e];
    if (c < a.R) anc = a.anchor[n][(int64_t)row * a.R + c];
  }
  __syncthreads();   // every replica read before replica 0 is overwritten
  if (in) a.M[n][e] = v;
  red[0][rl][c] = v;
  red[1][rl][c] = in ? v : 3.402823e38f;
  red[2][rl][c] = anc;
  __syncthreads();
  if (t < 96) {
    const int k = t >> 5;
    float r = red[k][0][c];
    for (int q = 1; q < kSumRows; ++q) r = k == 1 ? fminf(r, red[k][q][c]) : r + red[k][q][c];
    a.stats[n][(int64_t)b * 96 + 32 * k + c] = r;
  }
}

// p[0 .. n) = 0; p 16-byte aligned: four floats per thread, the tail alone
__global__ void fill_zero_kernel(float* p, int64_t n) {
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (e + 4 <= n) {
    *reinterpret_cast<float4*>(p + e) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  } else {
    for (int64_t f = e; f < n; ++f) p[f] = 0.0f;
  }
}

// Sort keys of a plan copy: the coordinates of its leading modes, mixed radix.
__global__ void coo_key_kernel(const int32_t* i0, const int32_t* i1, int64_t d1, int64_t nnz, uint64_t* key,
                               int32_t* pos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnz) return;
  const uint64_t a = (uint64_t)(uint32_t)i0[t];
  const uint64_t b = i1 ? (uint64_t)(uint32_t)i1[t] : 0;
  key[t] = a * (uint64_t)d1 + b;
  pos[t] = (int32_t)t;
}

struct GatherArgs {
  int N;
  int64_t nnz;
  const int32_t* perm;
  const int32_t* src[4];   // caller's coordinates, in the copy's slot order
  const float* val;
  int32_t* dst[4];
  float* dval;
};

__global__ void coo_gather_kernel(GatherArgs g) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.nnz) return;
  const int64_t p = g.perm[t];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (q < g.N) g.dst[q][t] = g.src[q][p];
  g.dval[t] = g.val[p];
}

}  // namespace comm

using namespace comm;

namespace {

int bits_for(uint64_t n) {
  int b = 1;
  while (b < 64 && (n >> b) != 0) ++b;
  return b;
}

struct CooWs {
  float* M[kMaxModes];   // reps replicas of [dims][32] each
  float* stats[kMaxModes];
  double* obj_part;
  int reps;
  size_t bytes;
};

// Accumulator replicas: the plan passes add workgroup b's run sums into
// replica b mod reps (b mod 8 is the workgroup's XCD), so the flushes of a
// Zipf-hot row are spread over eight addresses instead of queueing on one;
// slot_update adds the replicas as partial slots, in order.  One replica
// when eight would pass 32 MB.
constexpr int kCooReps = 8;

int coo_reps(int N, const int* dims) {
  int64_t rows = 0;
  for (int n = 0; n < N; ++n) rows += dims[n];
  return rows * kRP * 4 * kCooReps <= ((int64_t)32 << 20) ? kCooReps : 1;
}

CooWs coo_layout(int N, const int* dims, int blocks, char* base, int reps = 1) {
  CooWs w = {};
  Carve cv;
  cv.base = base;
  w.reps = reps;
  for (int n = 0; n < N; ++n) {
    w.M[n] = cv.take<float>((size_t)reps * dims[n] * kRP);
    w.stats[n] = cv.take<float>((size_t)((dims[n] + kSumRows - 1) / kSumRows) * 96);
  }
  w.obj_part = cv.take<double>((size_t)blocks);
  w.bytes = cv.off + 256;
  return w;
}

// Nonzeros per wavefront: long chunks (fewer run flushes at chunk ends, less
// per-wave setup) while about four waves per SIMD remain (1024 SIMDs); at
// least 256.  3.3M nonzeros: 832 per wave, 176 us per pass against 208 us at
// 256 (measured over chunks of 128 to 2048).
constexpr int64_t kCooMinChunk = 256;
constexpr int64_t kCooTargetWaves = 4096;

int64_t coo_chunk(int64_t nnz) {
  const int64_t c = (nnz + kCooTargetWaves - 1) / kCooTargetWaves;
  return std::max<int64_t>(kCooMinChunk, (c + 63) / 64 * 64);
}

int coo_blocks(int64_t nnz) {
  const int64_t chunk = coo_chunk(nnz);
  const int64_t waves = (nnz + chunk - 1) / chunk;
  return (int)std::max<int64_t>(1, (waves + kCooThreads / 64 - 1) / (kCooThreads / 64));
}

// One pass over a stream whose slot q holds mode order[q].
int coo_pass(comm_ctx* ctx, int N, const int* order, const int32_t* const* idx, const float* val, int64_t nnz,
             const int* dims, const comm_model* m, const CooWs& w, int run_modes, int atom_modes, bool obj, float eps,
             hipStream_t st) {
  if (nnz <= 0) return COMM_OK;
  CooPassArgs a = {};
  a.N = N;
  a.R = m->rank;
  a.nnz = nnz;
  for (int q = 0; q < N; ++q) {
    const int n = order[q];
    a.dims[q] = dims[n];
    a.idx[q] = idx[q];
    a.A[q] = m->factors[n];
    a.M[q] = w.M[n];
  }
  a.val = val;
  a.run_modes = run_modes;
  a.atom_modes = atom_modes;
  a.eps = eps;
  a.chunk = coo_chunk(nnz);
  a.obj_part = obj ? w.obj_part : nullptr;
  return profiled(ctx, st, [&] { return launch_coo(a, coo_blocks(nnz), st); });
}

// One pass over plan copy c (plan_pass kernel): its leading `runs` slots
// accumulate by runs.
int plan_pass(comm_ctx* ctx, const comm_coo_plan* p, int c, const int* dims, const comm_model* m, const CooWs& w,
              bool obj, float eps, hipStream_t st) {
  if (p->nnz <= 0) return COMM_OK;
  CooPlanPassArgs a = {};
  a.R = m->rank;
  a.nnz = p->nnz;
  for (int q = 0; q < p->ndim; ++q) {
    const int n = p->order[c][q];
    a.dims[q] = dims[n];
    a.idx[q] = p->idx[c][q];
    a.A[q] = m->factors[n];
    a.M[q] = w.M[n];
    a.mrep[q] = (int64_t)dims[n] * kRP;
  }
  a.rep_mask = w.reps - 1;
  a.val = p->val[c];
  a.eps = eps;
  a.inv_r4 = 1.0f / (4.0f * (float)m->rank);
  a.chunk = coo_chunk(p->nnz);
  a.obj_part = obj ? w.obj_part : nullptr;
  const int blocks = coo_blocks(p->nnz);
  return profiled(ctx, st, [&] { return launch_plan_pass(a, p->ndim, p->runs[c], blocks, st); });
}

// Zero the accumulators, run `passes`, then the beta = 1 inner loop.
template <class Passes>
int coo_outer(comm_ctx* ctx, int N, const int* dims, int64_t nnz, comm_model* m, const comm_opts* o, double* obj,
              hipStream_t st, Passes&& passes) {
  const int blocks = coo_blocks(nnz);
  const int reps = coo_reps(N, dims);
  CooWs w = coo_layout(N, dims, blocks, nullptr, reps);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = coo_layout(N, dims, blocks, ctx->ws, reps);
  {
    const int64_t n = (int64_t)(reinterpret_cast<char*>(w.stats[N - 1]) - reinterpret_cast<char*>(w.M[0])) / 4;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 1023) / 1024)), dim3(256), 0, st, w.M[0], n);
    HIP_TRY(hipGetLastError());
  }
  if ((rc = passes(w))) return rc;

  // c^(n) = M^(n) (the replicas added) with column statistics, then the
  // beta = 1 inner loop
  CooSumArgs sa = {};
  sa.N = N;
  sa.R = m->rank;
  sa.reps = w.reps;
  KlLoopArgs k = {};
  k.N = N;
  k.R = m->rank;
  k.L = o->inner_sweeps;
  k.eps = (float)o->eps;
  for (int n = 0; n < N; ++n) {
    const int nb = (dims[n] + kSumRows - 1) / kSumRows;
    sa.rows[n] = dims[n];
    sa.first_block[n + 1] = sa.first_block[n] + nb;
    sa.M[n] = w.M[n];
    sa.anchor[n] = m->factors[n];
    sa.stats[n] = w.stats[n];
    k.c[n] = w.M[n];
    k.stats[n] = w.stats[n];
    k.nblk[n] = nb;
    k.rows[n] = dims[n];
    k.cur_pad[n] = nullptr;
    k.user[n] = m->factors[n];
  }
  hipLaunchKernelGGL(coo_sum_kernel, dim3((unsigned)sa.first_block[N]), dim3(1024), 0, st, sa);
  HIP_TRY(hipGetLastError());
  if (obj) {
    k.obj_part = nnz > 0 ? w.obj_part : nullptr;
    k.obj_n = nnz > 0 ? blocks : 0;
    k.obj_out = obj;
    k.obj_add_model_mass = 1;
  }
  HIP_TRY(launch_kl_apply(k, st));
  return COMM_OK;
}

}  // namespace

int coo_jcomm_kl(comm_ctx* ctx, const comm_coo* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st) {
  const int N = x->ndim;
  int dims[4] = {0, 0, 0, 0};
  for (int n = 0; n < N; ++n) dims[n] = (int)x->dims[n];
  const int order[4] = {0, 1, 2, 3};
  const int runs = std::min(N, 2);
  return coo_outer(ctx, N, dims, x->nnz, m, o, obj, st, [&](const CooWs& w) {
    return coo_pass(ctx, N, order, x->idx, x->val, x->nnz, dims, m, w, runs, N - runs, obj != nullptr,
                    (float)o->eps, st);
  });
}

int coo_jcomm_kl_plan(comm_ctx* ctx, const comm_coo_plan* p, comm_model* m, const comm_opts* o, double* obj,
                      hipStream_t st) {
  const int N = p->ndim;
  int dims[4] = {0, 0, 0, 0};
  for (int n = 0; n < N; ++n) dims[n] = (int)p->dims[n];
  return coo_outer(ctx, N, dims, p->nnz, m, o, obj, st, [&](const CooWs& w) {
    int rc = COMM_OK;
    for (int c = 0; c < p->copies && !rc; ++c)
      rc = plan_pass(ctx, p, c, dims, m, w, c == 0 && obj != nullptr, (float)o->eps, st);
    return rc;
  });
}

// D_1(X, Xhat) over every cell without touching the zero cells (Sec. 3.2 at
// beta = 1, Sec. 6.4): a zero cell contributes d_1(0 | Xhat) = Xhat, so the
// sum over all cells is the model's mass sum_r prod_n colsum(A^(n))_r plus,
// over the nonzeros, d_1(x | X~) - X~ (the pass without accumulation).
int coo_objective_kl(comm_ctx* ctx, const comm_coo* x, const comm_model* m, const comm_opts* o, double* out,
                     hipStream_t st) {
  const int N = x->ndim;
  int dims[kMaxModes] = {0, 0, 0, 0, 0};
  for (int n = 0; n < N; ++n) dims[n] = (int)x->dims[n];
  const int blocks = coo_blocks(x->nnz);
  CooWs w = coo_layout(N, dims, blocks, nullptr);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = coo_layout(N, dims, blocks, ctx->ws);
  MassArgs ma = {};
  ma.N = N;
  ma.R = m->rank;
  for (int n = 0; n < N; ++n) {
    ma.rows[n] = dims[n];
    ma.A[n] = m->factors[n];
  }
  ma.out = out;
  hipLaunchKernelGGL(model_mass_kernel, dim3(1), dim3(1024), 0, st, ma);
  HIP_TRY(hipGetLastError());
  if (x->nnz <= 0) return COMM_OK;
  const int order[kMaxModes] = {0, 1, 2, 3, 4};
  if ((rc = coo_pass(ctx, N, order, x->idx, x->val, x->nnz, dims, m, w, 0, 0, true, (float)o->eps, st)))
    return rc;
  HIP_TRY(launch_sum_f64(w.obj_part, blocks, out, out, st));
  return COMM_OK;
}

// Two device copies of the COO: copy 0 sorted by (i1, i2) with the modes in
// their own order, copy 1 (order >= 3) sorted by (i3, i4) with slots
// (3, 4, 1, 2) (or (3, 1, 2) for order 3).  Stable sorts of (key, position)
// pairs, so the plan is a deterministic function of the input.
int coo_plan_build(comm_ctx* ctx, const comm_coo* x, comm_coo_plan** out, hipStream_t st) {
  (void)ctx;
  const int N = x->ndim;
  const int64_t nnz = x->nnz;
  if (nnz > INT32_MAX) return fail(COMM_EUNSUPPORTED, "plans hold at most 2^31 - 1 nonzeros");
  comm_coo_plan* p = new comm_coo_plan();
  p->ndim = N;
  p->nnz = nnz;
  for (int n = 0; n < N; ++n) p->dims[n] = x->dims[n];
  p->copies = N >= 3 ? 2 : 1;
  for (int q = 0; q < 4; ++q) p->order[0][q] = q;
  p->runs[0] = std::min(N, 2);
  if (N == 4) {
    const int o1[4] = {2, 3, 0, 1};
    for (int q = 0; q < 4; ++q) p->order[1][q] = o1[q];
    p->runs[1] = 2;
  } else if (N == 3) {
    const int o1[4] = {2, 0, 1, 3};
    for (int q = 0; q < 4; ++q) p->order[1][q] = o1[q];
    p->runs[1] = 1;
  }
  HIP_TRY(hipGetDevice(&p->device));
  // plan memory: per copy N coordinate arrays and the values
  Carve cv;
  for (int c = 0; c < p->copies; ++c) {
    for (int q = 0; q < N; ++q) cv.take<int32_t>((size_t)nnz);
    cv.take<float>((size_t)nnz);
  }
  const size_t plan_bytes = cv.off + 256;
  hipError_t e = hipMalloc(&p->mem, plan_bytes);
  if (e != hipSuccess) {
    delete p;
    return fail(COMM_ENOMEM, "hipMalloc(%zu) for the COO plan: %s", plan_bytes, hipGetErrorString(e));
  }
  Carve real;
  real.base = p->mem;
  for (int c = 0; c < p->copies; ++c) {
    for (int q = 0; q < N; ++q) p->idx[c][q] = real.take<int32_t>((size_t)nnz);
    p->val[c] = real.take<float>((size_t)nnz);
  }
  if (nnz == 0) {
    *out = p;
    return COMM_OK;
  }
  // scratch: keys and positions, in and out, plus the sort's temporary storage
  size_t temp_bytes = 0;
  e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                         (const int32_t*)nullptr, (int32_t*)nullptr, (int)nnz, 0, 64, st);
  char* scratch = nullptr;
  Carve sc;
  sc.take<uint64_t>((size_t)nnz);
  sc.take<uint64_t>((size_t)nnz);
  sc.take<int32_t>((size_t)nnz);
  sc.take<int32_t>((size_t)nnz);
  sc.take<char>(temp_bytes);
  const size_t scratch_bytes = sc.off + 256;
  if (e == hipSuccess) e = hipMalloc(&scratch, scratch_bytes);
  if (e != hipSuccess) {
    hipFree(p->mem);
    delete p;
    return fail(COMM_ENOMEM, "COO plan scratch of %zu bytes: %s", scratch_bytes, hipGetErrorString(e));
  }
  Carve s2;
  s2.base = scratch;
  uint64_t* kin = s2.take<uint64_t>((size_t)nnz);
  uint64_t* kout = s2.take<uint64_t>((size_t)nnz);
  int32_t* pin = s2.take<int32_t>((size_t)nnz);
  int32_t* pout = s2.take<int32_t>((size_t)nnz);
  char* temp = s2.take<char>(temp_bytes);
  const unsigned grid = (unsigned)((nnz + 255) / 256);
  int rc = COMM_OK;
  for (int c = 0; c < p->copies && !rc; ++c) {
    const int m0 = p->order[c][0];
    const int m1 = p->runs[c] > 1 ? p->order[c][1] : -1;
    const int64_t d1 = m1 >= 0 ? x->dims[m1] : 1;
    hipLaunchKernelGGL(coo_key_kernel, dim3(grid), dim3(256), 0, st, x->idx[m0], m1 >= 0 ? x->idx[m1] : nullptr, d1,
                       nnz, kin, pin);
    e = hipGetLastError();
    const int bits = bits_for((uint64_t)x->dims[m0] * (uint64_t)d1);
    if (e == hipSuccess)
      e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, kin, kout, pin, pout, (int)nnz, 0, bits, st);
    if (e == hipSuccess) {
      GatherArgs g = {};
      g.N = N;
      g.nnz = nnz;
      g.perm = pout;
      for (int q = 0; q < N; ++q) {
        g.src[q] = x->idx[p->order[c][q]];
        g.dst[q] = p->idx[c][q];
      }
      g.val = x->val;
      g.dval = p->val[c];
      hipLaunchKernelGGL(coo_gather_kernel, dim3(grid), dim3(256), 0, st, g);
      e = hipGetLastError();
    }
    if (e != hipSuccess) rc = fail(COMM_EHIP, "COO plan: %s", hipGetErrorString(e));
  }
  // the scratch is released once the sorts and gathers are done
  const hipError_t es = hipStreamSynchronize(st);
  hipFree(scratch);
  if (!rc && es != hipSuccess) rc = fail(COMM_EHIP, "COO plan: %s", hipGetErrorString(es));
  if (rc) {
    hipFree(p->mem);
    delete p;
    return rc;
  }
  *out = p;
  return COMM_OK;
}

int coo_plan_free(comm_coo_plan* p) {
  if (!p) return COMM_OK;
  int rc = COMM_OK;
  // passes still reading the copies must finish first
  HIP_TRY(hipSetDevice(p->device));
  HIP_TRY(hipDeviceSynchronize());
  if (p->mem) {
    hipError_t e = hipFree(p->mem);
    if (e != hipSuccess) rc = fail(COMM_EHIP, "hipFree: %s", hipGetErrorString(e));
  }
  delete p;
  return rc;
}

int coo_plan_ndim(const comm_coo_plan* p) { return p->ndim; }
int64_t coo_plan_dim(const comm_coo_plan* p, int n) { return p->dims[n]; }
