// Fused dense 3-way Tucker pass for gfx950 (MI355X).
//
// The Tucker reconstruction (App. C, eq. tucker_entry) is, for every (i, j)
// pair, a contraction over the third core index:
//   Xhat[(i,j)][k] = sum_c T2[(i,j)][c] C[k][c],
//   T2[(i,j)][c]   = sum_b B[j][b] T1[i][b][c],  T1[i][b][c] = sum_a A[i][a] G[a][b][c].
// A workgroup owns 8 i x 16 j pairs and all of K.  It first stages T2 for its
// 128 pairs in LDS (for the rebuild model and, separately, for the
// contraction set), then streams X in 32 (pairs) x 32 (k) tiles per wavefront
// with the same matrix-core chains as the CP pass:
//   rebuild  Xhat = T2 C^T                         (v_mfma_f32_32x32x2_f32)
//   weights  W = P or Q in registers (Sec. 4.1, Sec. 5.3), objective optional
//   mode 3   Num3[k][c] = sum_m W[m][k] T2'[m][c]   (factor numerator of mode 3,
//                                                     App. C eqs. block_factor_num,
//                                                     jmm_factor_num, direct form)
//   V        V[m][c]    = sum_k W[m][k] C'[k][c]     (complete per pair: the
//                                                     workgroup covers all of K)
// V is the only intermediate written (I x J x 32 floats, a fraction J3/K of
// X); the mode-1, mode-2 and core numerators follow from it in small kernels
// (tucker3.hip) without ever forming the partial tensor B^(n) or Xhat.
// Waves take k tiles w, w+4, ...; each k tile belongs to one wave, so the
// mode-3 partial of a tile is final within the workgroup, and V is combined
// across the four waves in a fixed order.  No atomics: deterministic.

#pragma once

#include "cp3_impl.h"

namespace comm {

constexpr int kTkTI = 8;    // i per workgroup
constexpr int kTkTJ = 16;   // j per workgroup
constexpr int kTkPairs = kTkTI * kTkTJ;
constexpr int kTkStride = 36;

enum TkMode : int { kTkFromX = 0, kTkCacheRead = 1, kTkCacheWrite = 2 };

struct TkShared {
  float t1[32 * 32];                  // T1 of one i (J2 x J3, padded)
  float t2r[kTkPairs * kTkStride];    // rebuild T2 rows
  float t2n[kTkPairs * 32];           // contraction T2' rows
  float t[kWaves][32 * kLdsT];        // per-wave transpose buffers
  float vred[kTkPairs * 32];          // V combined across waves
  double obj[kWaves];
};

// T2[(il, jl)][c] for the workgroup's pairs into dst (row stride ld).
__device__ __forceinline__ void stage_t2(const TkModel& m, int i0, int j0, int I, int J, float* t1, float* dst,
                                         int ld) {
  const int tid = threadIdx.x;
  for (int il = 0; il < kTkTI; ++il) {
    const int i = i0 + il;
    for (int e = tid; e < 32 * 32; e += kThreads) {
      const int b = e >> 5, c = e & 31;
      float s = 0.0f;
      if (i < I && b < m.J2 && c < m.J3)
        for (int a = 0; a < m.J1; ++a) s = fmaf(m.A.at(i, a, I), m.G[((size_t)a * m.J2 + b) * m.ldG + c], s);
      t1[e] = s;
    }
    __syncthreads();
    for (int e = tid; e < kTkTJ * 32; e += kThreads) {
      const int jl = e >> 5, c = e & 31;
      const int j = j0 + jl;
      float s = 0.0f;
      if (j < J)
        for (int b = 0; b < m.J2; ++b) s = fmaf(m.B.at(j, b, J), t1[b * 32 + c], s);
      dst[(il * kTkTJ + jl) * ld + c] = s;
    }
    __syncthreads();
  }
}

template <int BC, int kMode, bool kObj>
__global__ void __launch_bounds__(kThreads) tk_pass_kernel(TkPassArgs a, int gj) {
  __shared__ TkShared sh;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int col = lane & 31;
  const int h = lane >> 5;
  const int wg = blockIdx.x;
  const int bj = wg % gj, bi = wg / gj;
  const int i0 = bi * kTkTI, j0 = bj * kTkTJ;
  const int I = a.I, J = a.J, K = a.K;
  constexpr bool kRebuild = kMode != kTkCacheRead;
  const bool want_m3 = kMode != kTkCacheWrite && a.want_m3;
  const bool want_v = kMode != kTkCacheWrite && a.want_v;

  if (kRebuild) stage_t2(a.r, i0, j0, I, J, sh.t1, sh.t2r, kTkStride);
  if (want_m3) stage_t2(a.n, i0, j0, I, J, sh.t1, sh.t2n, 32);

  f32x16 vacc[4] = {};
  double obj = 0.0;
  const int nkt = (K + 31) / 32;
  for (int kt = w; kt < nkt; kt += kWaves) {
    const int kslice = kt * 32;
    const int kcol = kslice + col;
    const bool kvalid = kcol < K;
    float crow[16], ctn[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      if (kRebuild) crow[s] = a.r.C.at(kcol, 16 * h + s, K);
      ctn[s] = want_v ? a.n.C.at(kslice + 16 * h + s, col, K) : 0.0f;
    }
    f32x16 m3acc = {};
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      // tile rows: pair m = out_row(v, h) of block mb, i.e. il = 2 mb + (m >> 4), jl = m & 15
      float xv[16];
      bool valid[16];
      const float* src = kMode == kTkCacheRead ? a.Wc : a.X;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = out_row(v, h);
        const int i = i0 + 2 * mb + (m >> 4), j = j0 + (m & 15);
        valid[v] = kvalid && i < I && j < J;
        xv[v] = valid[v] ? src[((size_t)i * J + j) * K + kcol] : 0.0f;
      }
      float wv[16];
      if (kMode == kTkCacheRead) {
#pragma unroll
        for (int v = 0; v < 16; ++v) wv[v] = xv[v];
      } else {
        float arow[16];
        load16(sh.t2r + (32 * mb + col) * kTkStride + 16 * h, arow);
        f32x16 xh = {};
#pragma unroll
        for (int s = 0; s < 16; ++s) xh = mfma32(arow[s], crow[s], xh);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          float x = xv[v];
          if constexpr (BC == kIS) x = fmaxf(x, a.eps_x);
          const float y = fmaxf(xh[v], a.eps);
          float p, q, d = 0.0f;
          bool far;
          entry<BC, kObj>(x, y, a.bc, p, q, d, far);
          if constexpr (kObj) {
            if (BC == kKL && far) d = kl_direct(x, y);
            obj += (double)(valid[v] ? d : 0.0f);
          }
          p = valid[v] ? p : 0.0f;
          q = valid[v] ? q : 0.0f;
          if (kMode == kTkCacheWrite && valid[v]) {
            const int m = out_row(v, h);
            const size_t off = ((size_t)(i0 + 2 * mb + (m >> 4)) * J + (j0 + (m & 15))) * K + kcol;
            a.Pw[off] = p;
            a.Qw[off] = q;
          }
          wv[v] = a.use_q ? q : p;
        }
      }
      if (want_m3) {
        // A operand: lane (c = col, h) supplies T2'[32 mb + out_row(s, h)][col]
#pragma unroll
        for (int s = 0; s < 16; ++s) m3acc = mfma32(sh.t2n[(32 * mb + out_row(s, h)) * 32 + col], wv[s], m3acc);
      }
      if (want_v) {
        float* ldsT = sh.t[w];
#pragma unroll
        for (int v = 0; v < 16; ++v) ldsT[out_row(v, h) * kLdsT + col] = wv[v];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        float pr[16];
        load16(ldsT + col * kLdsT + 16 * h, pr);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int s = 0; s < 16; ++s) vacc[mb] = mfma32(pr[s], ctn[s], vacc[mb]);
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (want_m3 && kvalid) {
      // m3acc[v] = Num3[k = kcol][c = out_row(v, h)] over this workgroup's pairs
      float* dst = a.m3 + ((size_t)wg * a.Kp + kcol) * kRP;
#pragma unroll
      for (int v = 0; v < 16; ++v) dst[out_row(v, h)] = m3acc[v];
    }
  }

  // objective partial
  if (kObj) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) obj += __shfl_down(obj, off);
    if (lane == 0) sh.obj[w] = obj;
  }
  __syncthreads();
  if (kObj && tid == 0) {
    double s = sh.obj[0];
    for (int q = 1; q < kWaves; ++q) s += sh.obj[q];
    a.obj_part[wg] = s;
  }

  // V: combine the waves in order 0..3, then write the valid pairs
  if (want_v) {
    for (int q = 0; q < kWaves; ++q) {
      if (w == q) {
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            float& dst = sh.vred[(32 * mb + out_row(v, h)) * 32 + col];
            dst = (q == 0) ? vacc[mb][v] : dst + vacc[mb][v];
          }
      }
      __syncthreads();
    }
    for (int e = tid; e < kTkPairs * 32; e += kThreads) {
      const int p = e >> 5, c = e & 31;
      const int i = i0 + (p >> 4), j = j0 + (p & 15);
      if (i < I && j < J) a.V[((size_t)i * J + j) * kRP + c] = sh.vred[e];
    }
  }
}

template <int BC, int kMode, bool kObj>
hipError_t launch_tk(const TkPassArgs& a, const TkGrid& g, hipStream_t s) {
  hipLaunchKernelGGL((tk_pass_kernel<BC, kMode, kObj>), dim3((unsigned)g.wgs()), dim3(kThreads), 0, s, a, g.gj);
  return hipGetLastError();
}

template <int BC>
hipError_t launch_tk_bc(const TkPassArgs& a, const TkGrid& g, int mode, bool obj, hipStream_t s) {
  if (mode == kTkCacheWrite) {
    if constexpr (BC == kKL) return hipErrorInvalidValue;  // beta = 1 never caches
    else return obj ? launch_tk<BC, kTkCacheWrite, true>(a, g, s) : launch_tk<BC, kTkCacheWrite, false>(a, g, s);
  }
  return obj ? launch_tk<BC, kTkFromX, true>(a, g, s) : launch_tk<BC, kTkFromX, false>(a, g, s);
}

hipError_t launch_tk_a(const TkPassArgs& a, const TkGrid& g, int bc, int mode, bool obj, hipStream_t s);
hipError_t launch_tk_b(const TkPassArgs& a, const TkGrid& g, int bc, int mode, bool obj, hipStream_t s);

}  // namespace comm
