// Host-visible declarations of the kernel launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dmath.h"

namespace comm {

// Padded rank / core width every dense kernel works with: factor copies in the
// workspace are [rows_padded][32] row-major with zero padding.
constexpr int kRP = 32;

// ----------------------------------------------------------------------------------------
// Dense 3-way CP pass
// ----------------------------------------------------------------------------------------
constexpr int kCpTI = 16;  // i per workgroup
constexpr int kCpTJ = 32;  // j per workgroup
constexpr int kCpTK = 64;  // k per workgroup

struct CpGrid {
  int gi, gj, gk;          // workgroups per mode
  int Ip, Jp, Kp;          // padded extents (multiples of the tile)
  int64_t wgs() const { return (int64_t)gi * gj * gk; }
  int m3_slots() const { return gi * gj; }
  int m1_slots() const { return gj * gk; }
  int m2_slots() const { return gi * gk; }
};

CpGrid cp_grid(int I, int J, int K);

struct CpPassArgs {
  const float* X;          // I x J x K, row-major (unused when reading the cache)
  const float* Pc;         // cached P~ (cache_mode 2)
  const float* Qc;         // cached Q~ (cache_mode 2)
  float* Pw;               // cache targets (cache_mode 1)
  float* Qw;
  int cache_mode;          // 0 none, 1 write P/Q, 2 read P/Q instead of X + rebuild
  int I, J, K;
  int Ip, Jp, Kp;          // padded extents: rows of one partial slot; Kp is also the
                           // row stride of the transposed operands
  const float* Ar;         // rebuild set, [Ip][32], [Jp][32], [Kp][32]
  const float* Br;
  const float* Cr;
  const float* An;         // contraction set for P: [Ip][32], [Jp][32], transposed C [32][Kp]
  const float* Bn;
  const float* Ctn;
  const float* Ad;         // contraction set for Q
  const float* Bd;
  const float* Ctd;
  float eps, eps_x;
  int want_v;              // numerators / denominators of modes 1 and 2
  int want_m3;             // numerator / denominator of mode 3
  int want_obj;
  BetaConst bc;
  float* m3n;              // partial slots: m3 [gi*gj][Kp][32], m1 [gj*gk][Ip][32], m2 [gi*gk][Jp][32]
  float* m1n;
  float* m2n;
  float* m3d;
  float* m1d;
  float* m2d;
  double* obj_part;        // one float64 partial per workgroup
};

hipError_t launch_cp_pass(const CpPassArgs& a, const CpGrid& g, int beta_class, bool den, hipStream_t s);

// ----------------------------------------------------------------------------------------
// Small factor-side kernels
// ----------------------------------------------------------------------------------------

// dst[row][c] = src[row * ld + c] for row < rows, c < cols, zero elsewhere in
// [rows_p][32]; optionally also the transposed copy dstT[c][row] ([32][rows_p]).
hipError_t launch_pad_factor(const float* src, int rows, int cols, int ld, int rows_p,
                             float* dst, float* dstT, hipStream_t s);

// Column sums of padded factors: out[f*32 + c] = sum_row F_f[row][c] for the
// nf factors (fixed summation order).
hipError_t launch_colsums(const float* const* F, const int* rows, int nf, float* out, hipStream_t s);

// J-CoMM transformed blocks (Sec. 5.3): x1 = chi_1(cur, ref), x2 = chi_2(cur, ref),
// over [rows_p][32] padded buffers; entries with ref == 0 (padding) stay zero.
// Optional transposed copies x1T / x2T ([32][rows_p]).
hipError_t launch_chi(const float* cur, const float* ref, int rows_p, float beta,
                      float* x1, float* x2, float* x1T, float* x2T, hipStream_t s);

struct UpdateArgs {
  const float* num_part;  int num_slots;  // partial slots [slots][rows_total][32]
  const float* den_part;  int den_slots;  // ignored when den_closed
  int rows_total;          // row count of one slot
  int rows;                // valid rows of this factor
  int cols;                // valid columns (rank)
  const float* anchor;     // [rows_p][32] multiplicative pre-factor (current or reference block)
  const float* den_closed; // if not NULL: den[c] = den_closed[c] for every row
  float gamma;
  float eps;
  float* out_pad;          // [rows_p][32]
  float* out_padT;         // optional transposed copy [32][rows_p]
  int rows_p;
  float* out_user;         // optional caller buffer, row stride ld_user
  int ld_user;
};
// Block update max(anchor * (Num / Den)^gamma, eps) with Num / Den summed over
// the partial slots in a fixed order.
hipError_t launch_update(const UpdateArgs& a, hipStream_t s);

// prod[c] = prod_f colsum(F_f)[c] (closed-form beta = 1 denominator: Q = 1 makes
// Den^(n) = prod_{m != n} colsum(A^(m))).  One workgroup, fixed order.
hipError_t launch_colsum_prod(const float* const* F, const int* rows, int nf, float* prod, hipStream_t s);

// out[row][c] = anchor[row][c] * sum_s part[s][row][c] over the slots (fixed order),
// zero outside rows x cols.
hipError_t launch_scale_reduce(const float* part, int slots, int rows_total, int rows, int cols,
                               const float* anchor, int rows_p, float* out, hipStream_t s);

// Sum of n float64 partials in a fixed order; writes *out (device).  If add_to
// is not NULL its value is added.
hipError_t launch_sum_f64(const double* part, int64_t n, const double* add_to, double* out, hipStream_t s);

// beta = 1 J-CoMM inner loop for CP (kernels_small.hip): given
// c^(n) = A~^(n) * Num_J^(n) for every mode, runs L sweeps and writes the new
// factors.
struct KlLoopArgs {
  int N, R, L;
  float eps;
  const float* c[4];       // [rows_p][32]
  const float* ref[4];     // padded reference factors
  int rows[4];
  int rows_p[4];
  float* cur_pad[4];       // padded outputs
  float* cur_padT[4];      // optional transposed outputs
  float* user[4];          // optional caller buffers (row stride R)
};
hipError_t launch_kl_loop(const KlLoopArgs& a, hipStream_t s);

}  // namespace comm
