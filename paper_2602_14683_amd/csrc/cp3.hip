// Fused dense 3-way CP pass for gfx950 (MI355X).
//
// One pass streams X once and, per 32 (i,j)-pairs x 32 k tile held by one
// wavefront:
//   1. rebuilds Xhat on the matrix cores, Xhat[m][k] = sum_r W[m][r] C[k][r]
//      with W[m][r] = A[i(m)][r] B[j(m)][r] (Sec. 3.3; the Khatri-Rao row is
//      formed in registers, never stored);
//   2. forms the weights P = X * Xhat^(beta-2), Q = Xhat^(beta-1) in registers
//      (Sec. 4.1 / Sec. 5.3, with max(Xhat, eps) and the beta = 0 data floor);
//   3. optionally accumulates d_beta(X | Xhat) in float64 (Sec. 3.2);
//   4. contracts P (and Q) back onto the factors (CPContr of Sec. 6.1):
//        mode 3:   M3[k][r] = sum_m P[m][k] W'[m][r]          (matrix cores)
//        modes 1,2: V[m][r]  = sum_k P[m][k] C'[k][r]          (matrix cores)
//                   M1[i][r] = sum_j V[(i,j)][r] B'[j][r],  M2[j][r] = sum_i V[(i,j)][r] A'[i][r]
//      where the primed factors are the contraction set: the current factors
//      for block-MM, chi_1 / chi_2 of the current and reference factors for
//      J-CoMM (Sec. 5.3, CP inner update).
// Neither Xhat, P, Q nor any Khatri-Rao product is written to memory (P / Q
// only when the caller asks for the J-CoMM cache).
//
// MFMA: v_mfma_f32_32x32x2_f32.  A operand lane l supplies A[l%32][l/32], B
// operand B[l/32][l%32]; the 32x32 result sits in 16 registers per lane with
// D[8*(v/4) + 4*(l/32) + v%4][l%32] in register v.  Reductions over r or k use
// a permuted order that both operands agree on, so the Xhat tile produced by
// one chain is consumed by the mode-3 chain straight from registers; the
// modes-1/2 chain needs the tile with m in the lane index, which goes through
// a per-wave LDS transpose.
//
// Workgroup = 4 waves over a 16 (i) x 32 (j) x 64 (k) tile: wave w takes the
// 32-wide k slice (w & 1) and 8 of the 16 (4 i x 8 j) pair blocks (w >> 1).
// Results leave the workgroup as partial sums in fixed slots (no atomics), so
// every reduction has a fixed order and the pass is bitwise deterministic.

#include "kernels.h"

namespace comm {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kLdsT = 36;  // row stride of the per-wave transpose buffer (16-byte aligned rows)

CpGrid cp_grid(int I, int J, int K) {
  CpGrid g;
  g.gi = (I + kCpTI - 1) / kCpTI;
  g.gj = (J + kCpTJ - 1) / kCpTJ;
  g.gk = (K + kCpTK - 1) / kCpTK;
  g.Ip = g.gi * kCpTI;
  g.Jp = g.gj * kCpTJ;
  g.Kp = g.gk * kCpTK;
  return g;
}

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void load16(const float* p, float (&v)[16]) {
  const f32x4* q = reinterpret_cast<const f32x4*>(p);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 x = q[t];
    v[4 * t + 0] = x[0];
    v[4 * t + 1] = x[1];
    v[4 * t + 2] = x[2];
    v[4 * t + 3] = x[3];
  }
}

// Row of the 32x32 result held in register v by lane half h.
__device__ __forceinline__ int out_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// Contract one weight tile (P or Q) of pair block (ib, jb) with a contraction
// set.  wv: tile in the Xhat layout (lane = k, 16 m's); A'/B' rows for the
// block; Ct: this wave's 16 transposed C' values (k = 16h + s, column = lane).
template <bool kWantV>
__device__ __forceinline__ void contract_tile(const float (&wv)[16], const float (&ag)[4], const float (&bq)[4],
                                              const float (&ct)[16], bool want_m3, bool want_v,
                                              f32x16& m3acc, float (&m1loc)[4], float (&m2acc)[4][4], int jb,
                                              float* ldsT, int col, int h) {
  if (want_m3) {
#pragma unroll
    for (int s = 0; s < 16; ++s) m3acc = mfma32(ag[s >> 2] * bq[s & 3], wv[s], m3acc);
  }
  if (kWantV && want_v) {
    // transpose the tile through LDS: row m, column k
#pragma unroll
    for (int v = 0; v < 16; ++v) ldsT[out_row(v, h) * kLdsT + col] = wv[v];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    float pr[16];
    load16(ldsT + col * kLdsT + 16 * h, pr);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    f32x16 vacc = {};
#pragma unroll
    for (int s = 0; s < 16; ++s) vacc = mfma32(pr[s], ct[s], vacc);
    __builtin_amdgcn_wave_barrier();
    // vacc[4g+q] = V[(i = ib*4+g, j = jb*8 + 4h + q)][r = col]
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        m1loc[g] = fmaf(vacc[4 * g + q], bq[q], m1loc[g]);
        m2acc[jb][q] = fmaf(vacc[4 * g + q], ag[g], m2acc[jb][q]);
      }
    }
  }
}

template <int BC, bool kDen>
__global__ void __launch_bounds__(kThreads) cp3_pass_kernel(CpPassArgs a, int gj, int gk) {
  __shared__ float lds_t[kWaves][32 * kLdsT];
  __shared__ float lds_m1[2][2][kCpTI * 32];  // [num/den][k-slice][i][r]
  __shared__ float lds_red[kWaves][32 * 32];
  __shared__ double lds_obj[kWaves];

  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int col = lane & 31;
  const int h = lane >> 5;
  const int kt = w & 1;
  const int mg = w >> 1;

  const int wg = blockIdx.x;
  const int bk = wg % gk;
  const int bij = wg / gk;
  const int bj = bij % gj;
  const int bi = bij / gj;
  const int i0 = bi * kCpTI, j0 = bj * kCpTJ, k0 = bk * kCpTK;
  const int I = a.I, J = a.J, K = a.K;
  const int kcol = k0 + kt * 32 + col;  // this lane's k in the Xhat layout
  const int kslice = k0 + kt * 32;

  // Per-wave operands that do not depend on the pair block.
  float crow[16];
  if (a.cache_mode != 2) load16(a.Cr + (size_t)kcol * kRP + 16 * h, crow);
  float ctn[16], ctd[16];
  load16(a.Ctn + (size_t)col * a.Kp + kslice + 16 * h, ctn);
  if constexpr (kDen) load16(a.Ctd + (size_t)col * a.Kp + kslice + 16 * h, ctd);

  f32x16 m3n = {}, m3d = {};
  float m2n[4][4] = {}, m2d[4][4] = {};
  double obj = 0.0;
  const bool kvalid = kcol < K;

  for (int ibl = 0; ibl < 2; ++ibl) {
    const int ib = 2 * mg + ibl;
    float m1n[4] = {0.f, 0.f, 0.f, 0.f}, m1d[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      // ---- weights tile in the Xhat layout: lane = k, register v = pair row out_row(v, h)
      float pv[16], qv[16];
      bool valid[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = i0 + ib * 4 + (v >> 2);
        const int j = j0 + jb * 8 + 4 * h + (v & 3);
        valid[v] = kvalid && i < I && j < J;
      }
      if (a.cache_mode == 2) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int i = i0 + ib * 4 + (v >> 2);
          const int j = j0 + jb * 8 + 4 * h + (v & 3);
          const size_t off = ((size_t)i * J + j) * K + kcol;
          pv[v] = valid[v] ? a.Pc[off] : 0.f;
          qv[v] = (kDen && valid[v]) ? a.Qc[off] : 0.f;
        }
      } else {
        float xv[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int i = i0 + ib * 4 + (v >> 2);
          const int j = j0 + jb * 8 + 4 * h + (v & 3);
          xv[v] = valid[v] ? a.X[((size_t)i * J + j) * K + kcol] : 0.f;
        }
        // rebuild operand: lane = pair row m = col, r = 16h + s
        float arow[16], brow[16];
        {
          const int i = i0 + ib * 4 + (col >> 3);
          const int j = j0 + jb * 8 + (col & 7);
          load16(a.Ar + (size_t)i * kRP + 16 * h, arow);
          load16(a.Br + (size_t)j * kRP + 16 * h, brow);
        }
        f32x16 xh = {};
#pragma unroll
        for (int s = 0; s < 16; ++s) xh = mfma32(arow[s] * brow[s], crow[s], xh);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          float x = xv[v];
          if constexpr (BC == kIS) x = fmaxf(x, a.eps_x);
          const float y = fmaxf(xh[v], a.eps);
          float p, q;
          weights<BC>(x, y, a.bc.beta, p, q);
          pv[v] = valid[v] ? p : 0.f;
          qv[v] = valid[v] ? q : 0.f;
          if (a.want_obj && valid[v]) obj += (double)dbeta_term<BC>(x, y, a.bc);
        }
        if (a.cache_mode == 1) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            if (valid[v]) {
              const int i = i0 + ib * 4 + (v >> 2);
              const int j = j0 + jb * 8 + 4 * h + (v & 3);
              const size_t off = ((size_t)i * J + j) * K + kcol;
              a.Pw[off] = pv[v];
              a.Qw[off] = qv[v];
            }
          }
        }
      }
      if (a.want_m3 || a.want_v) {
        // contraction rows for this block: lane = r
        float ag[4], bq[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) ag[g] = a.An[(size_t)(i0 + ib * 4 + g) * kRP + col];
#pragma unroll
        for (int q = 0; q < 4; ++q) bq[q] = a.Bn[(size_t)(j0 + jb * 8 + 4 * h + q) * kRP + col];
        contract_tile<true>(pv, ag, bq, ctn, a.want_m3, a.want_v, m3n, m1n, m2n, jb, lds_t[w], col, h);
        if constexpr (kDen) {
#pragma unroll
          for (int g = 0; g < 4; ++g) ag[g] = a.Ad[(size_t)(i0 + ib * 4 + g) * kRP + col];
#pragma unroll
          for (int q = 0; q < 4; ++q) bq[q] = a.Bd[(size_t)(j0 + jb * 8 + 4 * h + q) * kRP + col];
          contract_tile<true>(qv, ag, bq, ctd, a.want_m3, a.want_v, m3d, m1d, m2d, jb, lds_t[w], col, h);
        }
      }
    }
    if (a.want_v) {
      // this wave's M1 rows ib*4+g: combine the two lane halves (different j)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float o = __shfl_xor(m1n[g], 32);
        if (h == 0) lds_m1[0][kt][(ib * 4 + g) * 32 + col] = m1n[g] + o;
        if constexpr (kDen) {
          float od = __shfl_xor(m1d[g], 32);
          if (h == 0) lds_m1[1][kt][(ib * 4 + g) * 32 + col] = m1d[g] + od;
        }
      }
    }
  }

  // ---------------------------------------------------------------- objective partial
  if (a.want_obj) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) obj += __shfl_down(obj, off);
    if (lane == 0) lds_obj[w] = obj;
  }
  __syncthreads();
  if (a.want_obj && tid == 0) {
    double s = lds_obj[0];
    for (int t = 1; t < kWaves; ++t) s += lds_obj[t];
    a.obj_part[wg] = s;
  }

  // ---------------------------------------------------------------- cross-wave reductions
  const int nsides = kDen ? 2 : 1;
  for (int side = 0; side < nsides; ++side) {
    if (a.want_m3) {
      const f32x16& acc = side == 0 ? m3n : m3d;
      // acc[v] = M3[k = col][r = out_row(v, h)] over this wave's pair blocks
#pragma unroll
      for (int v = 0; v < 16; ++v) lds_red[w][col * 32 + out_row(v, h)] = acc[v];
      __syncthreads();
      float* dst = side == 0 ? a.m3n : a.m3d;
      const size_t slot = (size_t)(bi * gj + bj);
      for (int e = tid; e < 2 * 32 * 32; e += kThreads) {
        const int ks = e >> 10;          // k slice
        const int kk = (e >> 5) & 31;
        const int r = e & 31;
        const int k = k0 + ks * 32 + kk;
        const float s = lds_red[ks][kk * 32 + r] + lds_red[2 + ks][kk * 32 + r];
        if (k < K) dst[(slot * a.Kp + k) * kRP + r] = s;
      }
      __syncthreads();
    }
    if (a.want_v) {
      float (&m2)[4][4] = side == 0 ? m2n : m2d;
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int q = 0; q < 4; ++q) lds_red[w][(jb * 8 + 4 * h + q) * 32 + col] = m2[jb][q];
      __syncthreads();
      float* d2 = side == 0 ? a.m2n : a.m2d;
      float* d1 = side == 0 ? a.m1n : a.m1d;
      const size_t slot2 = (size_t)(bi * gk + bk);
      const size_t slot1 = (size_t)(bj * gk + bk);
      for (int e = tid; e < 32 * 32; e += kThreads) {
        const int jl = e >> 5, r = e & 31;
        const float s = ((lds_red[0][e] + lds_red[1][e]) + lds_red[2][e]) + lds_red[3][e];
        if (j0 + jl < J) d2[(slot2 * a.Jp + j0 + jl) * kRP + r] = s;
      }
      for (int e = tid; e < kCpTI * 32; e += kThreads) {
        const int il = e >> 5, r = e & 31;
        const float s = lds_m1[side][0][e] + lds_m1[side][1][e];
        if (i0 + il < I) d1[(slot1 * a.Ip + i0 + il) * kRP + r] = s;
      }
      __syncthreads();
    }
  }
}

template <int BC>
static hipError_t launch_bc(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s) {
  dim3 grid((unsigned)g.wgs()), block(kThreads);
  if (den)
    hipLaunchKernelGGL((cp3_pass_kernel<BC, true>), grid, block, 0, s, a, g.gj, g.gk);
  else
    hipLaunchKernelGGL((cp3_pass_kernel<BC, false>), grid, block, 0, s, a, g.gj, g.gk);
  return hipGetLastError();
}

hipError_t launch_cp_pass(const CpPassArgs& a, const CpGrid& g, int beta_class, bool den, hipStream_t s) {
  switch (beta_class) {
    case kIS: return launch_bc<kIS>(a, g, den, s);
    case kHalf: return launch_bc<kHalf>(a, g, den, s);
    case kKL: return launch_bc<kKL>(a, g, den, s);
    case kThreeHalf: return launch_bc<kThreeHalf>(a, g, den, s);
    default: return launch_bc<kGeneral>(a, g, den, s);
  }
}

}  // namespace comm
