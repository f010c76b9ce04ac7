// Device-side scalar math shared by the dense and sparse kernels: the power
// step that forms the weights P = X * Xhat^(beta-2), Q = Xhat^(beta-1)
// (Sec. 4.1 and the reference-powered tensors of Sec. 5.3) and a
// cancellation-free evaluation of the beta-divergence term d_beta(x | y)
// (Sec. 3.2, Definition of the beta-divergence).
#pragma once

#include <hip/hip_runtime.h>

namespace comm {

// beta classes with dedicated fast paths; everything else is kGeneral.
enum BetaClass : int { kIS = 0, kHalf = 1, kKL = 2, kThreeHalf = 3, kGeneral = 4 };

constexpr int kSeriesTerms = 16;  // h(u) series terms u^2 .. u^17

// Per-call constants of the beta-divergence term.
struct BetaConst {
  float beta;
  float inv_bb1;                 // 1 / (beta (beta - 1)) for beta not in {0, 1}
  float inv_beta;                // 1 / beta (beta > 0)
  float series[kSeriesTerms];    // c_k, k = 2..17, see dbeta_term
};

// Compensated float64 summation of the objective (Knuth's TwoSum): s holds
// the running sum, c the rounding errors of the additions into s, and s + c
// the compensated result.  Every reduction of objective partials over lanes,
// wavefronts and workgroups goes through these, so the sum carries about one
// rounding of the float64 result however many partials it adds.
__device__ __forceinline__ void sum2_add(double& s, double& c, double x) {
  const double t = s + x;
  const double bp = t - s;
  c += (s - (t - bp)) + (x - bp);
  s = t;
}

// (s, c) of every lane of the wavefront into lane 0, in a fixed order.
__device__ __forceinline__ void sum2_wave(double& s, double& c) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double s2 = __shfl_down(s, off);
    const double c2 = __shfl_down(c, off);
    sum2_add(s, c, s2);
    c += c2;
  }
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Weights for one entry: x is the data value (already floored at eps_x when
// beta = 0), y = max(Xhat, eps).  Returns P in p and Q in q.
template <int BC>
__device__ __forceinline__ void weights(float x, float y, float beta, float& p, float& q) {
  if constexpr (BC == kIS) {
    float r = fast_rcp(y);
    q = r;
    p = x * r * r;
  } else if constexpr (BC == kHalf) {
    float rs = fast_rsq(y);
    q = rs;
    p = x * rs * rs * rs;
  } else if constexpr (BC == kKL) {
    q = 1.0f;
    p = x * fast_rcp(y);
  } else if constexpr (BC == kThreeHalf) {
    q = fast_sqrt(y);
    p = x * fast_rsq(y);
  } else {
    float l = fast_log2(y);
    q = fast_exp2((beta - 1.0f) * l);
    p = x * fast_exp2((beta - 2.0f) * l);
  }
}

// x^beta for x > 0.
template <int BC>
__device__ __forceinline__ float pow_beta(float x, float beta) {
  if constexpr (BC == kIS) return 1.0f;
  else if constexpr (BC == kHalf) return fast_sqrt(x);
  else if constexpr (BC == kKL) return x;
  else if constexpr (BC == kThreeHalf) return x * fast_sqrt(x);
  else return fast_exp2(beta * fast_log2(x));
}

// d_beta(x | y) for x >= 0, y > 0, evaluated without catastrophic
// cancellation.  With q = y / x and u = log q, d_beta(x | y) = x^beta h(u) where
//   h(u) = ((beta-1) e^{beta u} - beta e^{(beta-1) u} + 1) / (beta (beta-1))
//        = sum_{k>=2} (beta^{k-1} - (beta-1)^{k-1}) u^k / k!
// (expanding both exponentials; beta = 1 gives e^u - 1 - u and beta = 0 gives
// e^{-u} - 1 + u, the KL and IS branches).  For |u| < 1 the series is summed by
// Horner (16 terms, truncation below 1e-11 relative for beta < 2); elsewhere
// the closed form loses at most a few bits.  For |q - 1| < 0.29 the logarithm
// is taken as 2 atanh(t / (2 + t)), t = q - 1, which keeps u accurate near 0.
// At x = 0: d = y (beta = 1) or y^beta / beta (beta > 0).
// Every path is evaluated and the right one selected (no divergent branches).
template <int BC>
__device__ __forceinline__ float dbeta_term(float x, float y, const BetaConst& bc) {
  if constexpr (BC == kKL) {
    // beta = 1: d = x g(t) with t = y / x - 1 and g(t) = t - log(1 + t).  Near
    // t = 0, with s = t / (2 + t): log(1 + t) = 2 atanh(s) and t = 2 s / (1 - s),
    // so g = 2 s^2 (1 / (1 - s) - s (1/3 + s^2/5 + ... + s^8/11)), free of
    // cancellation (|t| < 0.29: |s| < 0.17, truncation below 1e-9 relative);
    // elsewhere t - log(y / x) loses at most a few bits.  At x = 0: d = y.
    const bool zero = !(x > 0.0f);
    const float xs = zero ? 1.0f : x;
    const float rx = fast_rcp(xs);
    const float t = (y - xs) * rx;
    const float s = t * fast_rcp(2.0f + t);
    const float s2 = s * s;
    float a = fmaf(s2, 1.0f / 11.0f, 1.0f / 9.0f);
    a = fmaf(s2, a, 1.0f / 7.0f);
    a = fmaf(s2, a, 1.0f / 5.0f);
    a = fmaf(s2, a, 1.0f / 3.0f);
    const float g_near = 2.0f * s2 * (fast_rcp(1.0f - s) - s * a);
    const float g_far = t - fast_log2(y * rx) * 0.69314718055994531f;
    const float g = fabsf(t) < 0.29f ? g_near : g_far;
    (void)bc;
    return zero ? y : xs * g;
  }
  const bool zero = !(x > 0.0f);
  const float xs = zero ? 1.0f : x;
  const float rx = fast_rcp(xs);
  const float t = (y - xs) * rx;
  const float q = y * rx;
  // u = log q, from the atanh series near q = 1, else from log2
  const float s = t * fast_rcp(2.0f + t);
  const float s2 = s * s;
  float a = fmaf(s2, 1.0f / 9.0f, 1.0f / 7.0f);
  a = fmaf(s2, a, 1.0f / 5.0f);
  a = fmaf(s2, a, 1.0f / 3.0f);
  a = fmaf(s2, a, 1.0f);
  const float u_near = 2.0f * s * a;
  const float u_far = fast_log2(q) * 0.69314718055994531f;
  const float u = fabsf(t) < 0.29f ? u_near : u_far;
  // h(u): series for |u| < 1, closed form otherwise
  float acc = bc.series[kSeriesTerms - 1];
#pragma unroll
  for (int k = kSeriesTerms - 2; k >= 0; --k) acc = fmaf(acc, u, bc.series[k]);
  const float h_series = acc * u * u;
  float h_closed;
  if constexpr (BC == kKL) {
    h_closed = (q - 1.0f) - u;
  } else if constexpr (BC == kIS) {
    h_closed = (fast_rcp(q) - 1.0f) + u;
  } else {
    const float qb = fast_exp2(bc.beta * u * 1.4426950408889634f);
    const float qb1 = qb * fast_rcp(q);
    h_closed = ((bc.beta - 1.0f) * qb - bc.beta * qb1 + 1.0f) * bc.inv_bb1;
  }
  const float h = fabsf(u) < 1.0f ? h_series : h_closed;
  const float d = pow_beta<BC>(xs, bc.beta) * h;
  float d0;
  if constexpr (BC == kKL) d0 = y;
  else if constexpr (BC == kIS) d0 = 0.0f;  // unreachable: x is floored at eps_x > 0
  else d0 = pow_beta<BC>(y, bc.beta) * bc.inv_beta;
  return zero ? d0 : d;
}

}  // namespace comm
