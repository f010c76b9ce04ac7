// Fused dense 3-way Tucker passes for gfx950 (MI355X).
//
// The Tucker reconstruction (App. C, eq. tucker_entry) of pair (i, j) is a
// 32-term contraction over the third core index,
//   Xhat[(i,j)][k] = sum_c T2[(i,j)][c] C[k][c],
//   T2[(i,j)][c]   = sum_{a,b} A[i][a] B[j][b] G[a][b][c],
// so X, read as an (I J) x K matrix with one mode-3 fibre per row, is streamed
// with the same matrix-core tiles as the CP pass once T2 is known.  T2 is
// built per model by tk_t2_kernel (I J x 32 floats, J3 / K of the size of X).
//
// V pass (core, mode-1 and mode-2 blocks): a workgroup owns 32 pairs and its
// four waves split K in 32-wide tiles, in the transposed orientation (lane =
// pair, registers = k), so that
//   rebuild  Xhat^T[k][m] = sum_c C[k][c] T2[m][c]            (v_mfma_f32_32x32x2_f32)
//   weights  P, Q in registers (Sec. 4.1, Sec. 5.3), objective optional
//   V^T      V^T[c][m]   += sum_k C'[k][c] W[m][k]             (W straight from registers)
// need no transpose; the waves' partial V are summed in a fixed order in LDS
// (the numerator and the denominator set are contracted in the same pass).
// The mode-1, mode-2 and core numerators follow from V with small GEMMs
// (tucker3.hip); the partial tensor B^(n) of App. C is never formed.
//
// Mode-3 pass: a workgroup owns a 32-wide k tile and a group of pairs, in the
// CP orientation (lane = k, registers = pairs):
//   Num3[k][c] = sum_m W[m][k] T2'[m][c]
// with the rebuilt weight tile consumed from registers; the four waves'
// partials are combined in a fixed order and written to the group's slot.
// Every reduction has a fixed order: the passes are bitwise deterministic.

#pragma once

#include "cp3_impl.h"

namespace comm {

constexpr int kTkPairsPerWg = 32;

// 16 consecutive floats of a 16-byte aligned row, or zeros.
__device__ __forceinline__ void row16(const float* p, bool ok, float (&v)[16]) {
  if (ok) {
    load16(p, v);
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = 0.0f;
  }
}

// X[m][k0 + out_row(v, h)] for the lane's row m (transposed orientation):
// four runs of four consecutive k.
template <bool kVec>
__device__ __forceinline__ void load_fibre(const float* __restrict__ row, int64_t k0, int64_t K, int h, bool ok,
                                           float (&x)[16]) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t kb = k0 + 8 * g + 4 * h;
    if constexpr (kVec) {
      f32x4 t = ok ? *reinterpret_cast<const f32x4*>(row + kb) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      x[4 * g + 0] = t[0];
      x[4 * g + 1] = t[1];
      x[4 * g + 2] = t[2];
      x[4 * g + 3] = t[3];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) x[4 * g + u] = (ok && kb + u < K) ? row[kb + u] : 0.0f;
    }
  }
}

template <int BC, int kMode, bool kObj, int kSets, bool kBf>
__device__ __forceinline__ void tk_v_body(const TkPassArgs& a, unsigned bx) {
  __shared__ float red[kWaves][kSets > 0 ? kSets : 1][32 * 33];
  __shared__ double sobj[kWaves][2];
  const int lane = threadIdx.x & 63;
  const int col = lane & 31, h = lane >> 5;
  const int w = threadIdx.x >> 6;
  const int64_t npairs = (int64_t)a.I * a.J;
  const int64_t p0 = (int64_t)bx * 32;
  const int64_t pm = p0 + col;  // this lane's pair
  const bool pvalid = pm < npairs;
  const int K = a.K;
  constexpr bool kRebuild = kMode != kTkCacheRead;
  // vector loads of the fibre need 16-byte aligned rows
  const bool vec = a.xvec != 0;

  float t2[16];
  if constexpr (kRebuild) row16(a.T2r + pm * kRP + 16 * h, pvalid, t2);
  bf16x8 t2h[2], t2l[2];
  if constexpr (kRebuild && kBf) {
    split_bf16(t2, t2h[0], t2l[0]);
    split_bf16(t2 + 8, t2h[1], t2l[1]);
  }
  f32x16 vn = {}, vd = {};
  double obj = 0.0, objc = 0.0;   // compensated sum of the objective tiles
  const float* xrow = a.X + pm * (int64_t)K;
  const float* prow = kMode == kTkCacheRead ? a.Pc + pm * (int64_t)K : nullptr;
  const float* qrow = kMode == kTkCacheRead && kSets == 2 ? a.Qc + pm * (int64_t)K : nullptr;

  // the four waves share the workgroup's 32 pairs and split the k tiles
  for (int k0 = 32 * w; k0 < K; k0 += 32 * kWaves) {
    const bool full = k0 + 32 <= K;
    float pv[16], qv[16];
    if constexpr (kMode == kTkCacheRead) {
      if (vec && full) {
        load_fibre<true>(prow, k0, K, h, pvalid, pv);
        if constexpr (kSets == 2) load_fibre<true>(qrow, k0, K, h, pvalid, qv);
      } else {
        load_fibre<false>(prow, k0, K, h, pvalid, pv);
        if constexpr (kSets == 2) load_fibre<false>(qrow, k0, K, h, pvalid, qv);
      }
    } else {
      float xv[16];
      if (!a.X) {
        // no tensor: the all-zero dense twin of sparse data (x = 0 everywhere)
#pragma unroll
        for (int v = 0; v < 16; ++v) xv[v] = 0.0f;
      } else if (vec && full) {
        load_fibre<true>(xrow, k0, K, h, pvalid, xv);
      } else {
        load_fibre<false>(xrow, k0, K, h, pvalid, xv);
      }
      // rebuild: A = C rows (lane: k = k0 + col), B = T2 rows (lane: pair)
      float crow[16];
      row16(a.C.p + (int64_t)(k0 + col) * kRP + 16 * h, k0 + col < K, crow);
      f32x16 xh = {};
      if constexpr (kBf) {
        xh = chain_bf16x3(crow, t2h, t2l, xh);
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) xh = mfma32(crow[s], t2[s], xh);
      }
      // the tile's 16 nonnegative terms per lane in float64, the lane's tiles
      // compensated
      double objt = 0.0;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int k = k0 + out_row(v, h);
        const bool ok = pvalid && k < K;
        float x = xv[v];
        if constexpr (BC == kIS) x = fmaxf(x, a.eps_x);
        const float y = fmaxf(xh[v], a.eps);
        float p, q, d = 0.0f;
        entry<BC, kObj>(x, y, a.bc, p, q, d);
        if constexpr (kObj) objt += (double)(ok ? d : 0.0f);
        pv[v] = ok ? p : 0.0f;
        qv[v] = ok ? q : 0.0f;
      }
      if constexpr (kObj) sum2_add(obj, objc, objt);
      if constexpr (kMode == kTkCacheWrite) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int k = k0 + out_row(v, h);
          if (pvalid && k < K) {
            a.Pw[pm * (int64_t)K + k] = pv[v];
            a.Qw[pm * (int64_t)K + k] = qv[v];
          }
        }
      }
    }
    if constexpr (kSets >= 1) {
      // V^T[c][m] += sum_k C'[k][c] W[m][k], k taken in the order out_row(s, h):
      // the lane's C' column comes from the transposed copy as four runs of four
      float cn[16], cd[16];
      load_fibre<true>(a.CnT + (int64_t)col * a.Kp, k0, a.Kp, h, true, cn);
      if constexpr (kSets == 2) load_fibre<true>(a.CdT + (int64_t)col * a.Kp, k0, a.Kp, h, true, cd);
      if constexpr (kBf) {
        const bf16x8 pb[2] = {pack_bf16(pv), pack_bf16(pv + 8)};
        vn = chain_bf16(cn, pb, vn);
        if constexpr (kSets == 2) {
          const bf16x8 qb[2] = {pack_bf16(qv), pack_bf16(qv + 8)};
          vd = chain_bf16(cd, qb, vd);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          vn = mfma32(cn[s], pv[s], vn);
          if constexpr (kSets == 2) vd = mfma32(cd[s], qv[s], vd);
        }
      }
    }
  }

  if constexpr (kSets >= 1) {
    // vn[v] = partial V[pair = col][c = out_row(v, h)]; combine the waves in order 0..3
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      red[w][0][col * 33 + out_row(v, h)] = vn[v];
      if constexpr (kSets == 2) red[w][1][col * 33 + out_row(v, h)] = vd[v];
    }
  }
  if constexpr (kObj) {
    sum2_wave(obj, objc);
    if (lane == 0) {
      sobj[w][0] = obj;
      sobj[w][1] = objc;
    }
  }
  __syncthreads();
  if constexpr (kSets >= 1) {
    for (int e = threadIdx.x; e < 32 * 32; e += kThreads) {
      const int r = e >> 5, c = e & 31;
      if (p0 + r < npairs) {
        float sn = red[0][0][r * 33 + c];
        for (int q = 1; q < kWaves; ++q) sn += red[q][0][r * 33 + c];
        a.Vn[(p0 + r) * kRP + c] = sn;
        if constexpr (kSets == 2) {
          float sd = red[0][1][r * 33 + c];
          for (int q = 1; q < kWaves; ++q) sd += red[q][1][r * 33 + c];
          a.Vd[(p0 + r) * kRP + c] = sd;
        }
      }
    }
  }
  if constexpr (kObj) {
    if (threadIdx.x == 0) {
      double s = sobj[0][0], c = sobj[0][1];
      for (int q = 1; q < kWaves; ++q) {
        sum2_add(s, c, sobj[q][0]);
        c += sobj[q][1];
      }
      a.obj_part[bx] = s + c;
    }
  }
}

template <int BC, int kMode, bool kObj, int kSets, bool kBf>
__global__ void __launch_bounds__(kThreads, 4) tk_v_kernel(TkPassArgs a) {
  tk_v_body<BC, kMode, kObj, kSets, kBf>(a, blockIdx.x);
}

template <int BC, int kMode, bool kObj, int kSets, bool kBf>
__global__ void __launch_bounds__(kThreads, 4) tk_v_grouped(GroupTable t) {
  uint3 bid, gdim;
  const TkPassArgs& a = group_item<TkPassArgs>(t, bid, gdim);
  tk_v_body<BC, kMode, kObj, kSets, kBf>(a, bid.x);
}

// Mode-3 pass.  Workgroup (kt, g): k tile kt, pair group g of 4 * tpw pair
// tiles; wave w takes tiles g * 4 * tpw + w * tpw + t, t < tpw.
template <int BC, int kMode, int kSets, bool kBf>
__device__ __forceinline__ void tk_m3_body(const TkPassArgs& a, unsigned bx) {
  __shared__ float red[kWaves][2][32 * 33];
  const int lane = threadIdx.x & 63;
  const int col = lane & 31, h = lane >> 5;
  const int w = threadIdx.x >> 6;
  const int K = a.K;
  const int nkt = (K + 31) / 32;
  const int kt = bx % nkt, g = bx / nkt;
  const int k0 = kt * 32;
  const int kcol = k0 + col;
  const bool kvalid = kcol < K;
  const int64_t npairs = (int64_t)a.I * a.J;
  constexpr bool kRebuild = kMode != kTkCacheRead;

  float crow[16];
  if constexpr (kRebuild) row16(a.C.p + (int64_t)kcol * kRP + 16 * h, kvalid, crow);
  bf16x8 crh[2], crl[2];
  if constexpr (kRebuild && kBf) {
    split_bf16(crow, crh[0], crl[0]);
    split_bf16(crow + 8, crh[1], crl[1]);
  }
  f32x16 an = {}, ad = {};
  const int64_t pbase = (int64_t)(g * kWaves + w) * a.tpw * 32;
  // the fibre entries of the next pair tile are loaded while the current one is processed
  auto fetch = [&](int64_t p0, float (&dst)[16], const float* src) {
    if (!src) {
      // no tensor: the all-zero dense twin of sparse data (x = 0 everywhere)
#pragma unroll
      for (int v = 0; v < 16; ++v) dst[v] = 0.0f;
      return;
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t m = p0 + out_row(v, h);
      dst[v] = (kvalid && m < npairs) ? src[m * K + kcol] : 0.0f;
    }
  };
  const float* src0 = kMode == kTkCacheRead ? a.Pc : a.X;
  float nx[16];
  fetch(pbase, nx, src0);
  for (int t = 0; t < a.tpw; ++t) {
    const int64_t p0 = pbase + (int64_t)t * 32;
    if (p0 >= npairs) break;
    float cur[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) cur[v] = nx[v];
    if (t + 1 < a.tpw) fetch(p0 + 32, nx, src0);
    float pv[16], qv[16];
    if constexpr (kMode == kTkCacheRead) {
#pragma unroll
      for (int v = 0; v < 16; ++v) pv[v] = cur[v];
      if constexpr (kSets == 2) fetch(p0, qv, a.Qc);
    } else {
      // rebuild: A = T2 rows (lane: pair p0 + col), B = C rows (lane: k)
      float t2[16];
      row16(a.T2r + (p0 + col) * kRP + 16 * h, p0 + col < npairs, t2);
      f32x16 xh = {};
      if constexpr (kBf) {
        xh = chain_bf16x3(t2, crh, crl, xh);
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) xh = mfma32(t2[s], crow[s], xh);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t m = p0 + out_row(v, h);
        const bool ok = kvalid && m < npairs;
        float x = cur[v];
        if constexpr (BC == kIS) x = fmaxf(x, a.eps_x);
        const float y = fmaxf(xh[v], a.eps);
        float p, q, d;
        entry<BC, false>(x, y, a.bc, p, q, d);
        pv[v] = ok ? p : 0.0f;
        qv[v] = ok ? q : 0.0f;
      }
    }
    // Num3[k][c] += sum_m W[m][k] T2'[m][c], m taken in the order out_row(s, h):
    // the lane's T2' column comes from the transposed copy as four runs of four
    float tn[16], td[16];
    load_fibre<true>(a.T2nT + (int64_t)col * a.Pp, p0, a.Pp, h, true, tn);
    if constexpr (kSets == 2) load_fibre<true>(a.T2dT + (int64_t)col * a.Pp, p0, a.Pp, h, true, td);
    if constexpr (kBf) {
      const bf16x8 tnb[2] = {pack_bf16(tn), pack_bf16(tn + 8)};
      an = chain_bf16(pv, tnb, an);
      if constexpr (kSets == 2) {
        const bf16x8 tdb[2] = {pack_bf16(td), pack_bf16(td + 8)};
        ad = chain_bf16(qv, tdb, ad);
      }
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        an = mfma32(pv[s], tn[s], an);
        if constexpr (kSets == 2) ad = mfma32(qv[s], td[s], ad);
      }
    }
  }
  // an[v] = Num3[k0 + out_row(v, h)][c = col]; combine the waves in order 0..3
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    red[w][0][out_row(v, h) * 33 + col] = an[v];
    if constexpr (kSets == 2) red[w][1][out_row(v, h) * 33 + col] = ad[v];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += kThreads) {
    const int r = e >> 5, c = e & 31;
    float sn = red[0][0][r * 33 + c];
    for (int q = 1; q < kWaves; ++q) sn += red[q][0][r * 33 + c];
    a.m3n[((int64_t)g * a.Kp + k0 + r) * kRP + c] = sn;
    if constexpr (kSets == 2) {
      float sd = red[0][1][r * 33 + c];
      for (int q = 1; q < kWaves; ++q) sd += red[q][1][r * 33 + c];
      a.m3d[((int64_t)g * a.Kp + k0 + r) * kRP + c] = sd;
    }
  }
}

template <int BC, int kMode, int kSets, bool kBf>
__global__ void __launch_bounds__(kThreads, 3) tk_m3_kernel(TkPassArgs a) {
  tk_m3_body<BC, kMode, kSets, kBf>(a, blockIdx.x);
}

template <int BC, int kMode, int kSets, bool kBf>
__global__ void __launch_bounds__(kThreads, 3) tk_m3_grouped(GroupTable t) {
  uint3 bid, gdim;
  const TkPassArgs& a = group_item<TkPassArgs>(t, bid, gdim);
  tk_m3_body<BC, kMode, kSets, kBf>(a, bid.x);
}

template <int BC, int kMode, bool kObj, int kSets>
hipError_t launch_v(const TkPassArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)tk_v_workgroups(a.I, a.J)), block(kThreads);
  if (a.bf16)
    return launch_or_record(tk_v_kernel<BC, kMode, kObj, kSets, true>, tk_v_grouped<BC, kMode, kObj, kSets, true>, grid,
                            block, 0, s, a);
  return launch_or_record(tk_v_kernel<BC, kMode, kObj, kSets, false>, tk_v_grouped<BC, kMode, kObj, kSets, false>, grid,
                          block, 0, s, a);
}

template <int BC, int kMode, int kSets>
hipError_t launch_m3(const TkPassArgs& a, hipStream_t s) {
  const int nkt = (a.K + 31) / 32;
  const dim3 grid((unsigned)(nkt * a.npg)), block(kThreads);
  if (a.bf16)
    return launch_or_record(tk_m3_kernel<BC, kMode, kSets, true>, tk_m3_grouped<BC, kMode, kSets, true>, grid, block, 0,
                            s, a);
  return launch_or_record(tk_m3_kernel<BC, kMode, kSets, false>, tk_m3_grouped<BC, kMode, kSets, false>, grid, block, 0,
                          s, a);
}

// Variants used per beta class: beta = 1 contracts P only (its denominators
// are closed-form) and never caches; the other classes contract P and Q.
template <int BC>
hipError_t launch_tk_v_bc(const TkPassArgs& a, int mode, bool obj, int sets, hipStream_t s) {
  if (sets == 0) {
    if (mode == kTkCacheWrite) {
      if constexpr (BC == kKL) return hipErrorInvalidValue;
      else return obj ? launch_v<BC, kTkCacheWrite, true, 0>(a, s) : launch_v<BC, kTkCacheWrite, false, 0>(a, s);
    }
    return launch_v<BC, kTkFromX, true, 0>(a, s);
  }
  if constexpr (BC == kKL) {
    if (sets != 1) return hipErrorInvalidValue;
    return obj ? launch_v<BC, kTkFromX, true, 1>(a, s) : launch_v<BC, kTkFromX, false, 1>(a, s);
  } else {
    if (sets != 2) return hipErrorInvalidValue;
    return obj ? launch_v<BC, kTkFromX, true, 2>(a, s) : launch_v<BC, kTkFromX, false, 2>(a, s);
  }
}

template <int BC>
hipError_t launch_tk_m3_bc(const TkPassArgs& a, int sets, hipStream_t s) {
  if constexpr (BC == kKL) {
    return sets == 1 ? launch_m3<BC, kTkFromX, 1>(a, s) : hipErrorInvalidValue;
  } else {
    return sets == 2 ? launch_m3<BC, kTkFromX, 2>(a, s) : hipErrorInvalidValue;
  }
}

hipError_t launch_tk_v_a(const TkPassArgs& a, int bc, int mode, bool obj, int sets, hipStream_t s);
hipError_t launch_tk_v_b(const TkPassArgs& a, int bc, int mode, bool obj, int sets, hipStream_t s);
hipError_t launch_tk_m3_a(const TkPassArgs& a, int bc, int sets, hipStream_t s);
hipError_t launch_tk_m3_b(const TkPassArgs& a, int bc, int sets, hipStream_t s);

}  // namespace comm
