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
//
// Rank <= 16 (float32 tiles) has a narrow variant (kR16): the reconstruction
// reduces over 16 r in 8 matrix-core steps instead of 16, and the three
// contractions run on v_mfma_f32_16x16x4f32 with 16-wide r, half the matrix
// work of the 32-wide tiles padded with zero columns.  The weight tile reaches
// the mode-3 contraction by lane swaps (v_permlane16_swap) that gather the
// k < 16 and k >= 16 halves of register pairs, and the modes-1/2 contraction
// through the same LDS transpose.

#pragma once

#include "group.h"
#include "kernels.h"

namespace comm {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kLdsT = 36;  // row stride of the per-wave transpose buffer (16-byte aligned rows)

inline CpGrid cp_grid_impl(int I, int J, int K) {
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

// bf16 matrix cores (v_mfma_f32_32x32x16_bf16): lane l supplies eight values
// of A row l%32 and of B column l%32 along the reduction; as with the fp32
// tiles, any order of the reduction index that both operands share is valid.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// v[o .. o+7] rounded to bf16 (to nearest even).
__device__ __forceinline__ bf16x8 pack_bf16(const float* v) {
  bf16x8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = (__bf16)v[j];
  return r;
}

// Split v = hi + lo with hi = bf16(v), lo = bf16(v - hi): the three products
// hi*hi + hi*lo + lo*hi carry about 16 bits of each operand.
__device__ __forceinline__ void split_bf16(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 t = (__bf16)v[j];
    hi[j] = t;
    lo[j] = (__bf16)(v[j] - (float)t);
  }
}

// sum_{s<16} a[s] b[s] over the tile's reduction index with split-bf16
// operands (b already split, two halves of eight).
__device__ __forceinline__ f32x16 chain_bf16x3(const float (&a)[16], const bf16x8 (&bh)[2], const bf16x8 (&bl)[2],
                                               f32x16 acc) {
  bf16x8 ah[2], al[2];
  split_bf16(a, ah[0], al[0]);
  split_bf16(a + 8, ah[1], al[1]);
  // small terms first
  acc = mfma_bf16(al[0], bh[0], acc);
  acc = mfma_bf16(al[1], bh[1], acc);
  acc = mfma_bf16(ah[0], bl[0], acc);
  acc = mfma_bf16(ah[1], bl[1], acc);
  acc = mfma_bf16(ah[0], bh[0], acc);
  acc = mfma_bf16(ah[1], bh[1], acc);
  return acc;
}

// The same with plain bf16 operands.
__device__ __forceinline__ f32x16 chain_bf16(const float (&a)[16], const bf16x8 (&b)[2], f32x16 acc) {
  acc = mfma_bf16(pack_bf16(a), b[0], acc);
  return mfma_bf16(pack_bf16(a + 8), b[1], acc);
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

__device__ __forceinline__ void load8(const float* p, float (&v)[8]) {
  const f32x4* q = reinterpret_cast<const f32x4*>(p);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f32x4 x = q[t];
    v[4 * t + 0] = x[0];
    v[4 * t + 1] = x[1];
    v[4 * t + 2] = x[2];
    v[4 * t + 3] = x[3];
  }
}

// v_mfma_f32_16x16x4f32: A operand lane l supplies A[l%16][l/16], B operand
// B[l/16][l%16]; the 16x16 result sits in 4 registers per lane with
// D[4*(l/16) + v][l%16] in register v.
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Exchange the odd 16-lane rows of x with the even rows of y: afterwards x
// holds rows (x0, y0, x2, y2) and y rows (x1, y1, x3, y3).  In the Xhat
// layout (lane = 32 h + k) x then carries k < 16 and y k >= 16, each for both
// registers and both lane halves.
__device__ __forceinline__ void swap_rows16(float& x, float& y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}

// Row of the 32x32 result held in register v by lane half h.
__device__ __forceinline__ int out_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// d_1(x | y) = y - x - x log(y / x) without cancellation: with
// s = (y - x) / (y + x), log(y / x) = 2 atanh(s), which gives
// d_1 = s^2 [(x + y) - 2 x s S(s^2)],  S(z) = sum_{k>=0} z^k / (2k + 3).
// For z < 1/16 (|s| < 1/4) -2 S(z) is replaced by a cubic fitted for least
// maximum relative error (Lawson's iteration on a fine grid, coefficients
// rounded to float32): 1.0e-7 relative error including the float32 Horner
// evaluation, three FMAs.  Entries with |s| >= 1/4 ("far") take the direct
// form y - x - x log(y / x); there |log(y / x)| > 0.51 and d > 0.15 x, so its
// float32 rounding costs at most about 1e-6 of the term.
constexpr float kKlFar = 0.0625f;  // z = s^2 at |s| = 1/4

__device__ __forceinline__ float kl_series_core(float x, float s, float z, float sum) {
  float T = -0.2467406839132309f;
  T = fmaf(T, z, -0.28473302721977234f);
  T = fmaf(T, z, -0.40001240372657776f);
  T = fmaf(T, z, -0.6666666269302368f);
  return z * fmaf(x * s, T, sum);
}

// Series form with its far flag; x = 0 gives y.  `rsum` is 1 / (x + y).
__device__ __forceinline__ float kl_series(float x, float y, float rsum, bool& far) {
  const float sum = x + y;
  const float s = (y - x) * rsum;
  const float z = s * s;
  far = z >= kKlFar && x > 0.0f;
  const float d = kl_series_core(x, s, z, sum);
  return x > 0.0f ? d : y;
}

__device__ __forceinline__ float kl_direct(float x, float y) {
  return (y - x) - x * (fast_log2(y * fast_rcp(x)) * 0.69314718055994531f);
}

// Weights and (optionally) the objective term of one entry.  At beta = 1 one
// reciprocal of y (x + y) serves both P = x / y and the objective's s.  Both
// forms of d_1 are evaluated and the far flag selects one: a tile of a few
// hundred entries nearly always holds a far one, so a branch would run for
// almost every tile.  The direct form takes log(y / x) = -log(P), with P
// raised to the smallest normal float so that x = 0 gives 0 * (-126) and the
// direct form returns y, the exact term; x = 0 always has s = 1 and so takes it.
template <int BC, bool kObj>
__device__ __forceinline__ void entry(float x, float y, const BetaConst& bc, float& p, float& q, float& d) {
  if constexpr (BC == kKL) {
    q = 1.0f;
    if constexpr (kObj) {
      const float sum = x + y;
      const float r = fast_rcp(y * sum);
      p = x * (sum * r);
      const float diff = y - x;
      const float s = diff * (y * r);
      const float z = s * s;
      const float ds = kl_series_core(x, s, z, sum);
      const float dd = fmaf(x * 0.69314718055994531f, fast_log2(fmaxf(p, 1.17549435e-38f)), diff);
      d = z >= kKlFar ? dd : ds;
    } else {
      p = x * fast_rcp(y);
    }
  } else {
    weights<BC>(x, y, bc.beta, p, q);
    if constexpr (kObj) d = dbeta_term<BC>(x, y, bc);
  }
}

// Contract one weight tile (P or Q) of pair block (ib, jb) with a contraction
// set.  wv: tile in the Xhat layout (lane = k, 16 m's); ag/bq: A'/B' entries
// (column = lane) of the block's 4 i's and this lane half's 4 j's; ct: this
// wave's 16 transposed C' values (k = 16h + s).
template <bool kBf>
__device__ __forceinline__ void contract_tile(const float (&wv)[16], const float (&ag)[4], const float (&bq)[4],
                                              const float (&ct)[16], const bf16x8 (&ctb)[2], bool want_m3,
                                              bool want_v, f32x16& m3acc, float (&m1loc)[4], float (&m2acc)[4],
                                              float* ldsT, int col, int h) {
  if (want_m3) {
    if constexpr (kBf) {
      float wa[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) wa[s] = ag[s >> 2] * bq[s & 3];
      bf16x8 wb[2] = {pack_bf16(wv), pack_bf16(wv + 8)};
      m3acc = chain_bf16(wa, wb, m3acc);
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) m3acc = mfma32(ag[s >> 2] * bq[s & 3], wv[s], m3acc);
    }
  }
  if (want_v) {
    // transpose the tile through LDS: row m, column k
#pragma unroll
    for (int v = 0; v < 16; ++v) ldsT[out_row(v, h) * kLdsT + col] = wv[v];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    float pr[16];
    load16(ldsT + col * kLdsT + 16 * h, pr);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    f32x16 vacc = {};
    if constexpr (kBf) {
      vacc = chain_bf16(pr, ctb, vacc);
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) vacc = mfma32(pr[s], ct[s], vacc);
    }
    __builtin_amdgcn_wave_barrier();
    // vacc[4g+q] = V[(i = ib*4+g, j = jb*8 + 4h + q)][r = col]
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        m1loc[g] = fmaf(vacc[4 * g + q], bq[q], m1loc[g]);
        m2acc[q] = fmaf(vacc[4 * g + q], ag[g], m2acc[q]);
      }
    }
  }
}

// The same for rank <= 16 with 16-wide tiles; lane l, c16 = l % 16, g = l / 16.
// ag[t]: A' of i_local = 2t + (g & 1); bq[q]: B' of j_local = 4 (g >> 1) + q;
// ct[s]: C'[kslice + 8g + s]; all at column r = c16.  m3acc[kb][v] =
// M3[k = 16 kb + c16][r = 4g + v]; m1loc[t], t < 2: M1 of i_local 2t + (g & 1) over
// this lane's j half; m2acc[q]: M2 of j_local 4 (g >> 1) + q over this lane's
// i's.
__device__ __forceinline__ void contract_tile16(const float (&wv)[16], const float (&ag)[2], const float (&bq)[4],
                                                const float (&ct)[8], bool want_m3, bool want_v, f32x4 (&m3acc)[2],
                                                float (&m1loc)[4], float (&m2acc)[4], float* ldsT, int col, int h,
                                                int c16, int g) {
  if (want_m3) {
    // pair u = registers (v, v + 4), v = (u & 3) + 8 (u >> 2): after the row
    // swap lane group g holds m = (i_local 2 (u >> 2) + (g & 1), j_local
    // 4 (g >> 1) + (u & 3)), at k = c16 in lo and k = 16 + c16 in hi
    float lo[8], hi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int v = (u & 3) + 8 * (u >> 2);
      lo[u] = wv[v];
      hi[u] = wv[v + 4];
      swap_rows16(lo[u], hi[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float wa = ag[u >> 2] * bq[u & 3];
      m3acc[0] = mfma16(wa, lo[u], m3acc[0]);
      m3acc[1] = mfma16(wa, hi[u], m3acc[1]);
    }
  }
  if (want_v) {
#pragma unroll
    for (int v = 0; v < 16; ++v) ldsT[out_row(v, h) * kLdsT + col] = wv[v];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    // A operand row c16 of row block mb is m = (i_local 2 mb + ((c16 >> 2) & 1),
    // j_local 4 (c16 >> 3) + (c16 & 3)); the reduction runs over k = 8g + s, so
    // result row 4g + v is (i_local 2 mb + (g & 1), j_local 4 (g >> 1) + v)
    float pr[2][8];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const int m = 8 * (2 * mb + ((c16 >> 2) & 1)) + 4 * (c16 >> 3) + (c16 & 3);
      load8(ldsT + m * kLdsT + 8 * g, pr[mb]);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    f32x4 vacc[2] = {};
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int t = 0; t < 8; ++t) vacc[mb] = mfma16(pr[mb][t], ct[t], vacc[mb]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        m1loc[mb] = fmaf(vacc[mb][q], bq[q], m1loc[mb]);
        m2acc[q] = fmaf(vacc[mb][q], ag[mb], m2acc[q]);
      }
    }
  }
}

// kNumOnly: contract P;  kNumDen: contract P and Q;  kCacheNumDen: P~ / Q~ read
// from the cache instead of X + rebuild, both contracted;  kCacheWrite: rebuild,
// write P~ / Q~ to the cache, no contraction.
enum PassVariant : int { kNumOnly = 0, kNumDen = 1, kCacheNumDen = 2, kCacheWrite = 3 };

constexpr int kSA = 36;  // row stride of the staged rebuild rows (bank spread for 16-byte reads)

static_assert(kCpTI * 32 % kThreads == 0 && kCpTJ * 32 % kThreads == 0, "staging loops take whole rounds");

// FView::at in two halves, for batches of loads that stay in flight
// together: the load always reads a clamped, valid address (rows and cols are
// at least 1), and the mask (scale by 0 outside rows x cols; a factor entry is
// finite) is applied after the batch.  A select on the loaded value would be
// turned back into a branch around each load.
__device__ __forceinline__ float load_clamped(const FView& f, int row, int c, int rows) {
  return f.p[(size_t)min(row, rows - 1) * f.ld + min(c, f.cols - 1)];
}
__device__ __forceinline__ float mask_of(const FView& f, int row, int c, int rows) {
  return (row < rows && c < f.cols) ? 1.0f : 0.0f;
}

struct PassShared {
  union {
    float t[kWaves][32 * kLdsT];    // per-wave transpose buffers (main loop)
    float red[kWaves][32 * 32];     // cross-wave reduction (epilogue, after a barrier)
  };
  float m1[2][2][kCpTI * 32];        // [num/den][k-slice][i][r]
  float ra[kCpTI * kSA];             // rebuild rows of A (i0 .. i0+15)
  float rb[kCpTJ * kSA];             // rebuild rows of B (j0 .. j0+31)
  float na[kCpTI * 32], nb[kCpTJ * 32];  // contraction rows for P
  float da[kCpTI * 32], db[kCpTJ * 32];  // contraction rows for Q
  double obj[kWaves][2];
};

// X (or cached P/Q) values of pair block (ib, jb) in the Xhat layout.
// Interior tiles read through a buffer resource based at the pair block: the
// row offsets are uniform (scalar offset), the lane's offset is fixed for the
// whole pass (vector offset), so a load needs no address arithmetic.  Only
// shapes whose in-tile byte offsets stay below 2^31 (xbuf) have interior
// tiles; others take the guarded path everywhere.
template <bool kInterior>
__device__ __forceinline__ void load_tile(const float* __restrict__ base, int ib, int jb, unsigned lane_off,
                                          int i0, int j0, int I, int J, int K, bool kvalid, int h,
                                          float (&x)[16]) {
  const int sK = K, sJK = J * K;
  const float* blk = base + ((size_t)(i0 + ib * 4) * J + (j0 + jb * 8)) * K;
  if constexpr (kInterior) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(blk), 0, 0x7FFFFFFF, 0x00020000);
    const int voff = (int)(lane_off * 4u);
#pragma unroll
    for (int v = 0; v < 16; ++v)
      x[v] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                           rs, voff, ((v >> 2) * sJK + (v & 3) * sK) * 4, 0));
  } else {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float* rowp = blk + (size_t)((v >> 2) * sJK + (v & 3) * sK);
      const int i = i0 + ib * 4 + (v >> 2);
      const int j = j0 + jb * 8 + 4 * h + (v & 3);
      x[v] = (kvalid && i < I && j < J) ? rowp[lane_off] : 0.0f;
    }
  }
}

template <int BC, int kVar, bool kObj, bool kInterior, bool kBf, bool kR16>
__device__ __forceinline__ void pass_body(const CpPassArgs& a, PassShared& sh, int wg, int bi, int bj, int bk,
                                          int gj, int gk) {
  static_assert(!(kBf && kR16), "the narrow tiles are float32 only");
  constexpr bool kDen = kVar == kNumDen || kVar == kCacheNumDen;
  constexpr bool kCache = kVar == kCacheNumDen;
  constexpr bool kWrite = kVar == kCacheWrite;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int col = lane & 31;
  const int h = lane >> 5;
  const int c16 = lane & 15, g16 = lane >> 4;  // the 16-wide tiles' lane split
  const int kt = w & 1;
  const int mg = w >> 1;
  const int i0 = bi * kCpTI, j0 = bj * kCpTJ, k0 = bk * kCpTK;
  const int I = a.I, J = a.J, K = a.K;
  const int kslice = k0 + kt * 32;
  const int kcol = kslice + col;
  const bool kvalid = kcol < K;
  const unsigned lane_off = (unsigned)(4 * h * K + kt * 32 + col) + (unsigned)k0;

  // Every global load of the prologue is issued before the first wait: the
  // wave's first pair block of X, its C operands, then the factor rows that
  // the workgroup stages in LDS (one round trip instead of one per loop step).
  const float* src0 = kCache ? a.Pc : a.X;
  float xb[2][16], qb[2][16];
  // X known to be all zero (the dense twin of a sparse tensor): x = 0 is not
  // loaded, and P = 0 is not contracted (its slots stay zero)
  const bool xz = BC != kKL && !kCache && a.x_zero;
  if (xz) {
#pragma unroll
    for (int v = 0; v < 16; ++v) xb[0][v] = xb[1][v] = 0.0f;
  } else {
    load_tile<kInterior>(src0, 2 * mg, 0, lane_off, i0, j0, I, J, K, kvalid, h, xb[0]);
  }
  if (kCache) load_tile<kInterior>(a.Qc, 2 * mg, 0, lane_off, i0, j0, I, J, K, kvalid, h, qb[0]);

  // ---- per-wave operands that do not depend on the pair block:
  // rebuild C rows (k = kcol, r = 16h + s) and contraction C columns
  // (r = col, k = kslice + 16h + s)
  // (16-wide: rebuild r = 8h + s, contraction columns r = c16 at k = kslice + 8 g16 + s, s < 8)
  // An interior workgroup whose factor views are all 32 wide reads every
  // operand in bounds: plain loads, without the clamps and masks of FView::at.
  const bool full = kInterior && !kR16 && (kCache || (a.r.A.cols == kRP && a.r.B.cols == kRP && a.r.C.cols == kRP)) &&
                    a.n.A.cols == kRP && a.n.B.cols == kRP && a.n.C.cols == kRP &&
                    (!kDen || (a.d.A.cols == kRP && a.d.B.cols == kRP && a.d.C.cols == kRP));
  float crow[16], ctn[16], ctd[16];
  if constexpr (kR16) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (!kCache) crow[s] = a.r.C.at(kcol, 8 * h + s, K);
      ctn[s] = a.n.C.at(kslice + 8 * g16 + s, c16, K);
      if (kDen) ctd[s] = a.d.C.at(kslice + 8 * g16 + s, c16, K);
    }
  } else if (full) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      if (!kCache) crow[s] = a.r.C.p[(size_t)kcol * a.r.C.ld + 16 * h + s];
      ctn[s] = a.n.C.p[(size_t)(kslice + 16 * h + s) * a.n.C.ld + col];
      if (kDen) ctd[s] = a.d.C.p[(size_t)(kslice + 16 * h + s) * a.d.C.ld + col];
    }
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      if (!kCache) crow[s] = a.r.C.at(kcol, 16 * h + s, K);
      ctn[s] = a.n.C.at(kslice + 16 * h + s, col, K);
      if (kDen) ctd[s] = a.d.C.at(kslice + 16 * h + s, col, K);
    }
  }

  // ---- stage the workgroup's factor rows in LDS (zero outside rows x cols):
  // all loads into registers first, then the stores (a store between two loads
  // would keep the second load waiting behind the first)
  constexpr int kQA = kCpTI * 32 / kThreads, kQB = kCpTJ * 32 / kThreads;
  float sa[kQA][3], sb[kQB][3];
  if (full) {
#pragma unroll
    for (int q = 0; q < kQA; ++q) {
      const int e = tid + q * kThreads;
      const size_t i = (size_t)(i0 + (e >> 5));
      const int c = e & 31;
      sa[q][0] = kCache ? 0.0f : a.r.A.p[i * a.r.A.ld + c];
      sa[q][1] = a.n.A.p[i * a.n.A.ld + c];
      sa[q][2] = kDen ? a.d.A.p[i * a.d.A.ld + c] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kQB; ++q) {
      const int e = tid + q * kThreads;
      const size_t j = (size_t)(j0 + (e >> 5));
      const int c = e & 31;
      sb[q][0] = kCache ? 0.0f : a.r.B.p[j * a.r.B.ld + c];
      sb[q][1] = a.n.B.p[j * a.n.B.ld + c];
      sb[q][2] = kDen ? a.d.B.p[j * a.d.B.ld + c] : 0.0f;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kQA; ++q) {
      const int e = tid + q * kThreads;
      const int i = i0 + (e >> 5), c = e & 31;
      sa[q][0] = kCache ? 0.0f : load_clamped(a.r.A, i, c, I);
      sa[q][1] = load_clamped(a.n.A, i, c, I);
      sa[q][2] = kDen ? load_clamped(a.d.A, i, c, I) : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kQB; ++q) {
      const int e = tid + q * kThreads;
      const int j = j0 + (e >> 5), c = e & 31;
      sb[q][0] = kCache ? 0.0f : load_clamped(a.r.B, j, c, J);
      sb[q][1] = load_clamped(a.n.B, j, c, J);
      sb[q][2] = kDen ? load_clamped(a.d.B, j, c, J) : 0.0f;
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  if (!full) {
    // the masks after the batch of loads (scale by 0 outside rows x cols)
#pragma unroll
    for (int q = 0; q < kQA; ++q) {
      const int e = tid + q * kThreads;
      const int i = i0 + (e >> 5), c = e & 31;
      sa[q][0] *= mask_of(a.r.A, i, c, I);
      sa[q][1] *= mask_of(a.n.A, i, c, I);
      sa[q][2] *= mask_of(a.d.A, i, c, I);
    }
#pragma unroll
    for (int q = 0; q < kQB; ++q) {
      const int e = tid + q * kThreads;
      const int j = j0 + (e >> 5), c = e & 31;
      sb[q][0] *= mask_of(a.r.B, j, c, J);
      sb[q][1] *= mask_of(a.n.B, j, c, J);
      sb[q][2] *= mask_of(a.d.B, j, c, J);
    }
  }
#pragma unroll
  for (int q = 0; q < kQA; ++q) {
    const int e = tid + q * kThreads;
    if (!kCache) sh.ra[(e >> 5) * kSA + (e & 31)] = sa[q][0];
    sh.na[e] = sa[q][1];
    if (kDen) sh.da[e] = sa[q][2];
  }
#pragma unroll
  for (int q = 0; q < kQB; ++q) {
    const int e = tid + q * kThreads;
    if (!kCache) sh.rb[(e >> 5) * kSA + (e & 31)] = sb[q][0];
    sh.nb[e] = sb[q][1];
    if (kDen) sh.db[e] = sb[q][2];
  }
  __syncthreads();
  // bf16 forms of the per-wave operands (split for the rebuild)
  bf16x8 crh[2], crl[2], ctnb[2], ctdb[2];
  if constexpr (kBf) {
    if (!kCache) {
      split_bf16(crow, crh[0], crl[0]);
      split_bf16(crow + 8, crh[1], crl[1]);
    }
    ctnb[0] = pack_bf16(ctn);
    ctnb[1] = pack_bf16(ctn + 8);
    if (kDen) {
      ctdb[0] = pack_bf16(ctd);
      ctdb[1] = pack_bf16(ctd + 8);
    }
  }

  f32x16 m3n = {}, m3d = {};
  f32x4 m3n16[2] = {}, m3d16[2] = {};
  float m2n[4][4] = {}, m2d[4][4] = {};
  float m1n[4] = {}, m1d[4] = {};
  double obj = 0.0;
  const bool want_m3 = !kWrite && a.want_m3, want_v = !kWrite && a.want_v;

  // The reconstruction of pair block t + 1 is issued on the matrix cores
  // before tile t's entries are evaluated, so that a wave's vector work
  // overlaps its own matrix-core work.
  auto rebuild = [&](int ibx, int jbx) -> f32x16 {
    // rebuild operand: lane = pair row m = col, r = 16h + s
    f32x16 acc = {};
    if constexpr (kR16) {
      // r = 8h + s: the lane halves split the 16 live columns
      float arow8[8], brow8[8];
      load8(sh.ra + (ibx * 4 + (col >> 3)) * kSA + 8 * h, arow8);
      load8(sh.rb + (jbx * 8 + (col & 7)) * kSA + 8 * h, brow8);
#pragma unroll
      for (int s = 0; s < 8; ++s) acc = mfma32(arow8[s] * brow8[s], crow[s], acc);
      return acc;
    }
    float arow[16], brow[16];
    load16(sh.ra + (ibx * 4 + (col >> 3)) * kSA + 16 * h, arow);
    load16(sh.rb + (jbx * 8 + (col & 7)) * kSA + 16 * h, brow);
    if constexpr (kBf) {
      float av[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) av[s] = arow[s] * brow[s];
      acc = chain_bf16x3(av, crh, crl, acc);
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) acc = mfma32(arow[s] * brow[s], crow[s], acc);
    }
    return acc;
  };
  // On for the KL objective pass only: it runs at two waves per SIMD, which
  // leave room for the second accumulator (at three, the KL pass without
  // the objective, it would spill); 256^3: 50.2 against 50.5-50.9 us.
  constexpr bool kPipe = BC == kKL && kObj && !kR16 && !kCache;
  f32x16 xh_cur = {};
  if constexpr (kPipe) xh_cur = rebuild(2 * mg, 0);

  for (int ibl = 0; ibl < 2; ++ibl) {
  const int ib = 2 * mg + ibl;
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) {
    const int t = ibl * 4 + jb;
    f32x16 xh_next = {};
    if constexpr (kPipe) {
      if (t + 1 < 8) xh_next = rebuild(2 * mg + ((t + 1) >> 2), (jb + 1) & 3);
    } else if constexpr (!kCache) {
      xh_cur = rebuild(ib, jb);
    }
    if (t + 1 < 8) {
      // prefetch the next pair block (the next i block after jb = 3)
      const int ibn = 2 * mg + ((t + 1) >> 2), jbn = (jb + 1) & 3;
      if (!xz) load_tile<kInterior>(src0, ibn, jbn, lane_off, i0, j0, I, J, K, kvalid, h, xb[(jb + 1) & 1]);
      if (kCache) load_tile<kInterior>(a.Qc, ibn, jbn, lane_off, i0, j0, I, J, K, kvalid, h, qb[(jb + 1) & 1]);
    }
    const float(&xv)[16] = xb[jb & 1];

    bool valid[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      if (kInterior) {
        valid[v] = true;
      } else {
        const int i = i0 + ib * 4 + (v >> 2);
        const int j = j0 + jb * 8 + 4 * h + (v & 3);
        valid[v] = kvalid && i < I && j < J;
      }
    }

    float pv[16], qv[16];
    if (kCache) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        pv[v] = xv[v];
        qv[v] = qb[jb & 1][v];
      }
    } else {
      const f32x16& xh = xh_cur;
      // the tile's 16 nonnegative terms per lane enter a float64 sum in pairs
      // (each pair added once in float32: one rounding, like the terms'
      // own); a lane adds its wave's eight tiles in float64 (error <= 7 *
      // 2^-53 of its sum); the lanes, waves and workgroups are then added
      // compensated
      double objt = 0.0;
      float objp = 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float x = xv[v];
        if constexpr (BC == kIS) x = fmaxf(x, a.eps_x);
        const float y = fmaxf(xh[v], a.eps);
        float p, q, d = 0.0f;
        entry<BC, kObj>(x, y, a.bc, p, q, d);
        pv[v] = valid[v] ? p : 0.f;
        qv[v] = valid[v] ? q : 0.f;
        if (kObj) {
          const float dv = valid[v] ? d : 0.0f;
          if (v & 1) objt += (double)(objp + dv);
          else objp = dv;
        }
        // the general objective terms are long: keep the scheduler from
        // interleaving all sixteen entries (register pressure).  The KL term
        // is short enough to leave free (two waves per SIMD, no spills).
        if constexpr (kObj && BC != kKL) {
          if ((v & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
      }
      // pin the tile's objective here: left free, the compiler sinks the
      // sixteen terms past the contraction and keeps x, y and 1 / (x + y) alive
      if constexpr (kObj && BC == kKL) asm volatile("" : "+v"(objt));
      if constexpr (kObj) obj += objt;
      if (kWrite) {
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

    if (!kWrite && (want_m3 || want_v) && kR16) {
      float ag2[2], bq4[4], ct8[8];
#pragma unroll
      for (int t = 0; t < 2; ++t) ag2[t] = sh.na[(ib * 4 + 2 * t + (g16 & 1)) * 32 + c16];
#pragma unroll
      for (int q = 0; q < 4; ++q) bq4[q] = sh.nb[(jb * 8 + 4 * (g16 >> 1) + q) * 32 + c16];
#pragma unroll
      for (int t = 0; t < 8; ++t) ct8[t] = ctn[t];
      if (!xz)
        contract_tile16(pv, ag2, bq4, ct8, want_m3, want_v, m3n16, m1n, m2n[jb], sh.t[w], col, h, c16, g16);
      if (kDen) {
#pragma unroll
        for (int t = 0; t < 2; ++t) ag2[t] = sh.da[(ib * 4 + 2 * t + (g16 & 1)) * 32 + c16];
#pragma unroll
        for (int q = 0; q < 4; ++q) bq4[q] = sh.db[(jb * 8 + 4 * (g16 >> 1) + q) * 32 + c16];
#pragma unroll
        for (int t = 0; t < 8; ++t) ct8[t] = ctd[t];
        contract_tile16(qv, ag2, bq4, ct8, want_m3, want_v, m3d16, m1d, m2d[jb], sh.t[w], col, h, c16, g16);
      }
    } else if (!kWrite && (want_m3 || want_v)) {
      float ag[4], bq[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) ag[g] = sh.na[(ib * 4 + g) * 32 + col];
#pragma unroll
      for (int q = 0; q < 4; ++q) bq[q] = sh.nb[(jb * 8 + 4 * h + q) * 32 + col];
      if (!xz) contract_tile<kBf>(pv, ag, bq, ctn, ctnb, want_m3, want_v, m3n, m1n, m2n[jb], sh.t[w], col, h);
      if (kDen) {
#pragma unroll
        for (int g = 0; g < 4; ++g) ag[g] = sh.da[(ib * 4 + g) * 32 + col];
#pragma unroll
        for (int q = 0; q < 4; ++q) bq[q] = sh.db[(jb * 8 + 4 * h + q) * 32 + col];
        contract_tile<kBf>(qv, ag, bq, ctd, ctdb, want_m3, want_v, m3d, m1d, m2d[jb], sh.t[w], col, h);
      }
    }
    if constexpr (kPipe) xh_cur = xh_next;
    if (kR16 && jb == 3 && want_v) {
      // rows ib*4 + 2t + (g16 & 1): combine the two j halves (lanes l, l ^ 32)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int row = (ib * 4 + 2 * t + (g16 & 1)) * 32 + c16;
        const float o = __shfl_xor(m1n[t], 32);
        if (h == 0) sh.m1[0][kt][row] = m1n[t] + o;
        m1n[t] = 0.0f;
        if (kDen) {
          const float od = __shfl_xor(m1d[t], 32);
          if (h == 0) sh.m1[1][kt][row] = m1d[t] + od;
          m1d[t] = 0.0f;
        }
      }
    } else if (jb == 3 && want_v) {
      // this wave's M1 rows ib*4+g: combine the two lane halves (different j)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float o = __shfl_xor(m1n[g], 32);
        if (h == 0) sh.m1[0][kt][(ib * 4 + g) * 32 + col] = m1n[g] + o;
        m1n[g] = 0.0f;
        if (kDen) {
          const float od = __shfl_xor(m1d[g], 32);
          if (h == 0) sh.m1[1][kt][(ib * 4 + g) * 32 + col] = m1d[g] + od;
          m1d[g] = 0.0f;
        }
      }
    }
  }
  }

  // ---------------------------------------------------------------- objective partial
  if (kObj) {
    double oc = 0.0;
    sum2_wave(obj, oc);
    if (lane == 0) {
      sh.obj[w][0] = obj;
      sh.obj[w][1] = oc;
    }
  }
  __syncthreads();
  if (kObj && tid == 0) {
    double s = sh.obj[0][0], c = sh.obj[0][1];
    for (int q = 1; q < kWaves; ++q) {
      sum2_add(s, c, sh.obj[q][0]);
      c += sh.obj[q][1];
    }
    a.obj_part[wg] = s + c;
  }

  // ---------------------------------------------------------------- cross-wave reductions
  constexpr int nsides = kDen ? 2 : 1;
  if constexpr (kR16) {
    // the same reductions over 16 live columns (the slots' columns >= 16 are
    // not written; every reader stops at the rank)
#pragma unroll
    for (int side = 0; side < nsides; ++side) {
      if (want_m3) {
        const f32x4(&acc)[2] = side == 0 ? m3n16 : m3d16;
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int v = 0; v < 4; ++v) sh.red[w][(16 * kb + c16) * 32 + 4 * g16 + v] = acc[kb][v];
        __syncthreads();
        float* dst = side == 0 ? a.m3n : a.m3d;
        const size_t slot = (size_t)(bi * gj + bj);
        for (int e = tid; e < 2 * 32 * 16; e += kThreads) {
          const int ks = e >> 9;
          const int kk = (e >> 4) & 31;
          const int r = e & 15;
          const int k = k0 + ks * 32 + kk;
          const float s = sh.red[ks][kk * 32 + r] + sh.red[2 + ks][kk * 32 + r];
          if (k < K) dst[(slot * a.Kp + k) * kRP + r] = s;
        }
        __syncthreads();
      }
      if (want_v) {
        float(&m2)[4][4] = side == 0 ? m2n : m2d;
        // combine the two i parities (lanes l, l ^ 16)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float sv = m2[jb][q] + __shfl_xor(m2[jb][q], 16);
            if ((g16 & 1) == 0) sh.red[w][(jb * 8 + 4 * (g16 >> 1) + q) * 32 + c16] = sv;
          }
        __syncthreads();
        float* d2 = side == 0 ? a.m2n : a.m2d;
        float* d1 = side == 0 ? a.m1n : a.m1d;
        const size_t slot2 = (size_t)(bi * gk + bk);
        const size_t slot1 = (size_t)(bj * gk + bk);
        for (int e = tid; e < 32 * 16; e += kThreads) {
          const int jl = e >> 4, r = e & 15;
          const int o = jl * 32 + r;
          const float sv = ((sh.red[0][o] + sh.red[1][o]) + sh.red[2][o]) + sh.red[3][o];
          if (j0 + jl < J) d2[(slot2 * a.Jp + j0 + jl) * kRP + r] = sv;
        }
        for (int e = tid; e < kCpTI * 16; e += kThreads) {
          const int il = e >> 4, r = e & 15;
          const int o = il * 32 + r;
          const float sv = sh.m1[side][0][o] + sh.m1[side][1][o];
          if (i0 + il < I) d1[(slot1 * a.Ip + i0 + il) * kRP + r] = sv;
        }
        __syncthreads();
      }
    }
    return;
  }
#pragma unroll
  for (int side = 0; side < nsides; ++side) {
    if (want_m3) {
      const f32x16& acc = side == 0 ? m3n : m3d;
      // acc[v] = M3[k = col][r = out_row(v, h)] over this wave's pair blocks
#pragma unroll
      for (int v = 0; v < 16; ++v) sh.red[w][col * 32 + out_row(v, h)] = acc[v];
      __syncthreads();
      float* dst = side == 0 ? a.m3n : a.m3d;
      const size_t slot = (size_t)(bi * gj + bj);
      for (int e = tid; e < 2 * 32 * 32; e += kThreads) {
        const int ks = e >> 10;  // k slice
        const int kk = (e >> 5) & 31;
        const int r = e & 31;
        const int k = k0 + ks * 32 + kk;
        const float s = sh.red[ks][kk * 32 + r] + sh.red[2 + ks][kk * 32 + r];
        if (k < K) dst[(slot * a.Kp + k) * kRP + r] = s;
      }
      __syncthreads();
    }
    if (want_v) {
      float(&m2)[4][4] = side == 0 ? m2n : m2d;
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int q = 0; q < 4; ++q) sh.red[w][(jb * 8 + 4 * h + q) * 32 + col] = m2[jb][q];
      __syncthreads();
      float* d2 = side == 0 ? a.m2n : a.m2d;
      float* d1 = side == 0 ? a.m1n : a.m1d;
      const size_t slot2 = (size_t)(bi * gk + bk);
      const size_t slot1 = (size_t)(bj * gk + bk);
      for (int e = tid; e < 32 * 32; e += kThreads) {
        const int jl = e >> 5, r = e & 31;
        const float s = ((sh.red[0][e] + sh.red[1][e]) + sh.red[2][e]) + sh.red[3][e];
        if (j0 + jl < J) d2[(slot2 * a.Jp + j0 + jl) * kRP + r] = s;
      }
      for (int e = tid; e < kCpTI * 32; e += kThreads) {
        const int il = e >> 5, r = e & 31;
        const float s = sh.m1[side][0][e] + sh.m1[side][1][e];
        if (i0 + il < I) d1[(slot1 * a.Ip + i0 + il) * kRP + r] = s;
      }
      __syncthreads();
    }
  }
}

template <int BC, int kVar, bool kObj, bool kBf, bool kR16>
__device__ __forceinline__ void cp3_pass_entry(const CpPassArgs& a, int wg, int gj, int gk) {
  __shared__ PassShared sh;
  const int bk = wg % gk;
  const int bij = wg / gk;
  const int bj = bij % gj;
  const int bi = bij / gj;
  const bool interior =
      a.xbuf && (bi + 1) * kCpTI <= a.I && (bj + 1) * kCpTJ <= a.J && (bk + 1) * kCpTK <= a.K;
  if (interior)
    pass_body<BC, kVar, kObj, true, kBf, kR16>(a, sh, wg, bi, bj, bk, gj, gk);
  else
    pass_body<BC, kVar, kObj, false, kBf, kR16>(a, sh, wg, bi, bj, bk, gj, gk);
}

// Waves per SIMD the pass is compiled for: three for KL without the
// objective (its PassShared, with the transpose and reduction buffers
// aliased, leaves room for three workgroups per CU), two for KL with it (the
// float64 objective sums would spill at three), two for the other classes
// without the objective, one with it (their objective terms are long).
template <int BC, bool kObj>
constexpr int pass_waves() {
  return BC == kKL ? (kObj ? 2 : 3) : (!kObj ? 2 : 1);
}

template <int BC, int kVar, bool kObj, bool kBf, bool kR16>
__global__ void __launch_bounds__(kThreads, (pass_waves<BC, kObj>())) cp3_pass_kernel(CpPassArgs a, int gj, int gk) {
  cp3_pass_entry<BC, kVar, kObj, kBf, kR16>(a, blockIdx.x, gj, gk);
}

// The pass launch of one problem in a grouped launch.
struct CpPassLaunch {
  CpPassArgs a;
  int gj, gk;
};

template <int BC, int kVar, bool kObj, bool kBf, bool kR16>
__global__ void __launch_bounds__(kThreads, (pass_waves<BC, kObj>())) cp3_pass_grouped(GroupTable t) {
  uint3 bid, gdim;
  const CpPassLaunch& l = group_item<CpPassLaunch>(t, bid, gdim);
  cp3_pass_entry<BC, kVar, kObj, kBf, kR16>(l.a, (int)bid.x, l.gj, l.gk);
}

// ---------------------------------------------------------------------------------------- V pass
//
// The mode-1 pass of a J-CoMM sweep at beta != 1 with the shared
// intermediate kept: V[(i,j)][r] = sum_k P~[i,j,k] C'[k][r] (and the same of
// Q~ with the denominator set) summed over all of K, written to memory, with
// the mode-1 numerators M1 = sum_j V B' folded from it.  Mode 2's numerators
// are then M2 = sum_i V A'_new with the mode-1 block's new transforms (C is
// unchanged until mode 3), a fold over V instead of a second pass over X.
//
// Workgroup = 4 i x 32 j pairs over all of K: wave w takes the pair block of
// the 4 i and j0 + 8w .. j0 + 8w + 7 and walks the 32-wide k slices,
// accumulating V in registers; rebuild rows and the B' rows of the fold are
// staged in LDS, the per-slice C operands are read from memory (they stay in
// the caches).  Slots: M1 one per j block (bj), rows i; V [I*J][32] per set.

constexpr int kVTI = 4;
constexpr int kVTJ = 32;

struct VPassShared {
  float t[kWaves][32 * kLdsT];          // per-wave transpose buffers
  float m1[2][kWaves][kVTI * 32];       // [num/den][wave][i][r]
  float ra[kVTI * kSA];                 // rebuild rows of A
  float rb[kVTJ * kSA];                 // rebuild rows of B
  float nb[kVTJ * 32], db[kVTJ * 32];   // B' rows of the numerator / denominator sets
  double obj[kWaves][2];
};

template <int BC, bool kCache, bool kObj, bool kBf, bool kInterior>
__device__ __forceinline__ void vpass_body(const CpPassArgs& a, VPassShared& sh, int bi, int bj, int wg) {
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int col = lane & 31;
  const int h = lane >> 5;
  const int I = a.I, J = a.J, K = a.K;
  const int i0 = bi * kVTI, j0 = bj * kVTJ;
  const int jb = w;  // this wave's 8 j

  // stage the rebuild rows (A: 4 i, B: 32 j) and the fold's B' rows
  for (int e = tid; e < kVTI * 32; e += kThreads) {
    const int i = i0 + (e >> 5), c = e & 31;
    if (!kCache) sh.ra[(e >> 5) * kSA + c] = load_clamped(a.r.A, i, c, I) * mask_of(a.r.A, i, c, I);
  }
  for (int e = tid; e < kVTJ * 32; e += kThreads) {
    const int j = j0 + (e >> 5), c = e & 31;
    if (!kCache) sh.rb[(e >> 5) * kSA + c] = load_clamped(a.r.B, j, c, J) * mask_of(a.r.B, j, c, J);
    sh.nb[e] = load_clamped(a.n.B, j, c, J) * mask_of(a.n.B, j, c, J);
    sh.db[e] = load_clamped(a.d.B, j, c, J) * mask_of(a.d.B, j, c, J);
  }
  __syncthreads();

  // the rebuild operand of this wave's pair block: lane = pair m = col, r = 16h + s
  float wr[16];
  if (!kCache) {
    float arow[16], brow[16];
    load16(sh.ra + (col >> 3) * kSA + 16 * h, arow);
    load16(sh.rb + (jb * 8 + (col & 7)) * kSA + 16 * h, brow);
#pragma unroll
    for (int s = 0; s < 16; ++s) wr[s] = arow[s] * brow[s];
  }
  bf16x8 wrh[2], wrl[2];
  if constexpr (kBf) {
    if (!kCache) {
      split_bf16(wr, wrh[0], wrl[0]);
      split_bf16(wr + 8, wrh[1], wrl[1]);
    }
  }

  bool pvalid[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = i0 + (v >> 2);
    const int j = j0 + jb * 8 + 4 * h + (v & 3);
    pvalid[v] = i < I && j < J;
  }

  f32x16 vn = {}, vd = {};
  double obj = 0.0, objc = 0.0;
  const float* src0 = kCache ? a.Pc : a.X;
  const bool xz = !kCache && a.x_zero;
  const int nk = (K + 31) / 32;
  for (int ks = 0; ks < nk; ++ks) {
    const int kslice = ks * 32;
    const int kcol = kslice + col;
    const bool kvalid = kcol < K;
    const unsigned lane_off = (unsigned)(4 * h * K + kslice + col);
    float xv[16], qv_in[16];
    const bool full = kInterior && kslice + 32 <= K;
    if (xz) {
      // the all-zero twin of sparse data: nothing to load
#pragma unroll
      for (int v = 0; v < 16; ++v) xv[v] = 0.0f;
    } else if (full) {
      load_tile<true>(src0, 0, jb, lane_off, i0, j0, I, J, K, true, h, xv);
      if (kCache) load_tile<true>(a.Qc, 0, jb, lane_off, i0, j0, I, J, K, true, h, qv_in);
    } else {
      load_tile<false>(src0, 0, jb, lane_off, i0, j0, I, J, K, kvalid, h, xv);
      if (kCache) load_tile<false>(a.Qc, 0, jb, lane_off, i0, j0, I, J, K, kvalid, h, qv_in);
    }
    // per-slice C operands: rebuild rows (k = kcol, r = 16h + s) and the
    // contraction columns (r = col, k = kslice + 16h + s)
    float crow[16], ctn[16], ctd[16];
    // a whole slice with 32-wide views: plain loads, without FView::at's guards
    const bool fullc = kslice + 32 <= K && (kCache || a.r.C.cols == kRP) && a.n.C.cols == kRP && a.d.C.cols == kRP;
    if (fullc) {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if (!kCache) crow[s] = a.r.C.p[(size_t)kcol * a.r.C.ld + 16 * h + s];
        ctn[s] = a.n.C.p[(size_t)(kslice + 16 * h + s) * a.n.C.ld + col];
        ctd[s] = a.d.C.p[(size_t)(kslice + 16 * h + s) * a.d.C.ld + col];
      }
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if (!kCache) crow[s] = a.r.C.at(kcol, 16 * h + s, K);
        ctn[s] = a.n.C.at(kslice + 16 * h + s, col, K);
        ctd[s] = a.d.C.at(kslice + 16 * h + s, col, K);
      }
    }
    float pv[16], qv[16];
    if (kCache) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        pv[v] = xv[v];
        qv[v] = qv_in[v];
      }
    } else {
      f32x16 xh = {};
      if constexpr (kBf) {
        bf16x8 crh[2], crl[2];
        split_bf16(crow, crh[0], crl[0]);
        split_bf16(crow + 8, crh[1], crl[1]);
        xh = mfma_bf16(wrl[0], crh[0], xh);
        xh = mfma_bf16(wrl[1], crh[1], xh);
        xh = mfma_bf16(wrh[0], crl[0], xh);
        xh = mfma_bf16(wrh[1], crl[1], xh);
        xh = mfma_bf16(wrh[0], crh[0], xh);
        xh = mfma_bf16(wrh[1], crh[1], xh);
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) xh = mfma32(wr[s], crow[s], xh);
      }
      // the tile's terms in float64, the tiles of the lane compensated
      double objt = 0.0;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float x = xv[v];
        if constexpr (BC == kIS) x = fmaxf(x, a.eps_x);
        const float y = fmaxf(xh[v], a.eps);
        float p, q, d = 0.0f;
        entry<BC, kObj>(x, y, a.bc, p, q, d);
        const bool ok = kvalid && pvalid[v];
        pv[v] = ok ? p : 0.0f;
        qv[v] = ok ? q : 0.0f;
        if (kObj) objt += (double)(ok ? d : 0.0f);
        if constexpr (kObj) {
          if ((v & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
      }
      if constexpr (kObj) sum2_add(obj, objc, objt);
    }
    // V += P C' and Vd += Q C'd through the per-wave LDS transpose
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const float(&wv)[16] = side == 0 ? pv : qv;
      const float(&ct)[16] = side == 0 ? ctn : ctd;
      float* ldsT = sh.t[w];
#pragma unroll
      for (int v = 0; v < 16; ++v) ldsT[out_row(v, h) * kLdsT + col] = wv[v];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      float pr[16];
      load16(ldsT + col * kLdsT + 16 * h, pr);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      f32x16& acc = side == 0 ? vn : vd;
      if constexpr (kBf) {
        const bf16x8 ctb[2] = {pack_bf16(ct), pack_bf16(ct + 8)};
        acc = chain_bf16(pr, ctb, acc);
      } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) acc = mfma32(pr[s], ct[s], acc);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }

  // acc[4g+q] = V[(i0 + g, j0 + 8 jb + 4h + q)][r = col]: store V, fold M1
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const f32x16& acc = side == 0 ? vn : vd;
    float* Vout = side == 0 ? a.Vn : a.Vd;
    const float* bset = side == 0 ? sh.nb : sh.db;
    float m1[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int jl = jb * 8 + 4 * h + q;
        const int i = i0 + g, j = j0 + jl;
        if (i < I && j < J) Vout[((size_t)i * J + j) * kRP + col] = acc[4 * g + q];
        m1[g] = fmaf(acc[4 * g + q], bset[jl * 32 + col], m1[g]);
      }
      const float o = __shfl_xor(m1[g], 32);
      if (h == 0) sh.m1[side][w][g * 32 + col] = m1[g] + o;
    }
  }
  if (kObj) {
    sum2_wave(obj, objc);
    if (lane == 0) {
      sh.obj[w][0] = obj;
      sh.obj[w][1] = objc;
    }
  }
  __syncthreads();
  if (kObj && tid == 0) {
    double s = sh.obj[0][0], c = sh.obj[0][1];
    for (int q = 1; q < kWaves; ++q) {
      sum2_add(s, c, sh.obj[q][0]);
      c += sh.obj[q][1];
    }
    a.obj_part[wg] = s + c;
  }
  // M1 rows i0 .. i0 + 3 of slot bj: the four waves' j blocks in order
  for (int e = tid; e < 2 * kVTI * 32; e += kThreads) {
    const int side = e / (kVTI * 32), il = (e >> 5) & (kVTI - 1), r = e & 31;
    const int idx = il * 32 + r;
    const float sum = ((sh.m1[side][0][idx] + sh.m1[side][1][idx]) + sh.m1[side][2][idx]) + sh.m1[side][3][idx];
    float* d1 = side == 0 ? a.m1n : a.m1d;
    if (i0 + il < I) d1[((size_t)bj * a.Ip + i0 + il) * kRP + r] = sum;
  }
}

template <int BC, bool kCache, bool kObj, bool kBf>
__device__ __forceinline__ void cp3_vpass_entry(const CpPassArgs& a, int wg, int gj) {
  __shared__ VPassShared sh;
  const int bi = wg / gj, bj = wg % gj;
  const bool interior = a.xbuf && (bi + 1) * kVTI <= a.I && (bj + 1) * kVTJ <= a.J;
  if (interior)
    vpass_body<BC, kCache, kObj, kBf, true>(a, sh, bi, bj, wg);
  else
    vpass_body<BC, kCache, kObj, kBf, false>(a, sh, bi, bj, wg);
}

template <int BC, bool kCache, bool kObj, bool kBf>
__global__ void __launch_bounds__(kThreads, kObj ? 1 : 2) cp3_vpass_kernel(CpPassArgs a, int gj) {
  cp3_vpass_entry<BC, kCache, kObj, kBf>(a, blockIdx.x, gj);
}

struct CpVPassLaunch {
  CpPassArgs a;
  int gj;
};

template <int BC, bool kCache, bool kObj, bool kBf>
__global__ void __launch_bounds__(kThreads, kObj ? 1 : 2) cp3_vpass_grouped(GroupTable t) {
  uint3 bid, gdim;
  const CpVPassLaunch& l = group_item<CpVPassLaunch>(t, bid, gdim);
  cp3_vpass_entry<BC, kCache, kObj, kBf>(l.a, (int)bid.x, l.gj);
}

inline int64_t vpass_wgs(int I, int J) { return (int64_t)((I + kVTI - 1) / kVTI) * ((J + kVTJ - 1) / kVTJ); }

template <int BC, bool kCache, bool kObj>
hipError_t launch_vpass_t(const CpPassArgs& a, hipStream_t s) {
  const int gj = (a.J + kVTJ - 1) / kVTJ;
  const dim3 grid((unsigned)vpass_wgs(a.I, a.J));
  const CpVPassLaunch l{a, gj};
  if (a.bf16) {
    if (record_grouped(cp3_vpass_grouped<BC, kCache, kObj, true>, grid, dim3(kThreads), 0, l)) return hipSuccess;
    launch_timed(cp3_vpass_kernel<BC, kCache, kObj, true>, grid, dim3(kThreads), 0, s, a, gj);
  } else {
    if (record_grouped(cp3_vpass_grouped<BC, kCache, kObj, false>, grid, dim3(kThreads), 0, l)) return hipSuccess;
    launch_timed(cp3_vpass_kernel<BC, kCache, kObj, false>, grid, dim3(kThreads), 0, s, a, gj);
  }
  return hipGetLastError();
}

template <int BC>
hipError_t launch_vpass_bc(const CpPassArgs& a, hipStream_t s) {
  return a.want_obj ? launch_vpass_t<BC, false, true>(a, s) : launch_vpass_t<BC, false, false>(a, s);
}

template <int BC, int kVar, bool kObj>
hipError_t launch_v(const CpPassArgs& a, const CpGrid& g, hipStream_t s) {
  const dim3 grid((unsigned)g.wgs()), block(kThreads);
  const CpPassLaunch l{a, g.gj, g.gk};
  if (a.bf16) {
    if (record_grouped(cp3_pass_grouped<BC, kVar, kObj, true, false>, grid, block, 0, l)) return hipSuccess;
    launch_timed(cp3_pass_kernel<BC, kVar, kObj, true, false>, grid, block, 0, s, a, g.gj, g.gk);
  } else if (a.r16) {
    if (record_grouped(cp3_pass_grouped<BC, kVar, kObj, false, true>, grid, block, 0, l)) return hipSuccess;
    launch_timed(cp3_pass_kernel<BC, kVar, kObj, false, true>, grid, block, 0, s, a, g.gj, g.gk);
  } else {
    if (record_grouped(cp3_pass_grouped<BC, kVar, kObj, false, false>, grid, block, 0, l)) return hipSuccess;
    launch_timed(cp3_pass_kernel<BC, kVar, kObj, false, false>, grid, block, 0, s, a, g.gj, g.gk);
  }
  return hipGetLastError();
}

// Dispatch for one beta class; instantiated once per translation unit cp3_bc*.hip.
template <int BC>
hipError_t launch_bc(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s) {
  if (a.cache_mode == 1)
    return a.want_obj ? launch_v<BC, kCacheWrite, true>(a, g, s) : launch_v<BC, kCacheWrite, false>(a, g, s);
  if (den) return a.want_obj ? launch_v<BC, kNumDen, true>(a, g, s) : launch_v<BC, kNumDen, false>(a, g, s);
  return a.want_obj ? launch_v<BC, kNumOnly, true>(a, g, s) : launch_v<BC, kNumOnly, false>(a, g, s);
}

// beta = 1 never contracts Q (its denominators are closed-form) and never
// caches: only the P-only variants exist.
template <>
hipError_t launch_bc<kKL>(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s);

hipError_t launch_bc_is(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s);
hipError_t launch_bc_half(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s);
hipError_t launch_bc_kl(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s);
hipError_t launch_bc_threehalf(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s);
hipError_t launch_bc_general(const CpPassArgs& a, const CpGrid& g, bool den, hipStream_t s);
hipError_t launch_cache_read(const CpPassArgs& a, const CpGrid& g, hipStream_t s);
hipError_t launch_vpass_is(const CpPassArgs& a, hipStream_t s);
hipError_t launch_vpass_half(const CpPassArgs& a, hipStream_t s);
hipError_t launch_vpass_threehalf(const CpPassArgs& a, hipStream_t s);
hipError_t launch_vpass_general(const CpPassArgs& a, hipStream_t s);
hipError_t launch_vpass_cache(const CpPassArgs& a, hipStream_t s);

}  // namespace comm
