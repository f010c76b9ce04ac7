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

// Read-only view of a factor matrix: `rows` x `cols` valid entries, row-major
// with row stride ld; entries outside read as zero.  Views cover both caller
// buffers (ld = R) and the padded workspace copies (ld = 32).
struct FView {
  const float* p;
  int ld;
  int cols;
  __device__ __forceinline__ float at(int row, int c, int rows) const {
    return (row < rows && c < cols) ? p[(size_t)row * ld + c] : 0.0f;
  }
};

struct FSet {
  FView A, B, C;  // modes 1, 2, 3
};

struct CpPassArgs {
  const float* X;          // I x J x K, row-major (unused when reading the cache)
  const float* Pc;         // cached P~ (cache_mode 2)
  const float* Qc;         // cached Q~ (cache_mode 2)
  float* Pw;               // cache targets (cache_mode 1)
  float* Qw;
  int cache_mode;          // 0 none, 1 write P/Q, 2 read P/Q instead of X + rebuild
  int I, J, K;
  int Ip, Jp, Kp;          // padded extents: rows of one partial slot
  FSet r;                  // rebuild set
  FSet n;                  // contraction set for P
  FSet d;                  // contraction set for Q
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
// Small factor-side kernels (kernels_small.hip)
// ----------------------------------------------------------------------------------------

// dst[f][row][c] = src[f][row * ld + c] for row < rows[f], c < cols, zero elsewhere
// in [rows_p][32]; optional transposed copy dstT[f][c][row] and second copies.
struct PadArgs {
  int nf;
  int cols, ld;
  const float* src[4];
  int rows[4];
  int rows_p[4];
  float* dst[4];
  float* dstT[4];
  float* dst2[4];
  float* dst2T[4];
};
hipError_t launch_pad_factors(const PadArgs& a, hipStream_t s);

// prod[c] = prod_f colsum(F_f)[c] (closed-form beta = 1 denominator: Q = 1 makes
// Den^(n) = prod_{m != n} colsum(A^(m))).  One workgroup, fixed order.
hipError_t launch_colsum_prod(const FView* F, const int* rows, int nf, float* prod, hipStream_t s);

// J-CoMM transformed blocks (Sec. 5.3): x1 = chi_1(cur, ref), x2 = chi_2(cur, ref)
// over [rows_p][32] padded buffers; entries with ref == 0 (padding) stay zero.
struct ChiArgs {
  int nf;
  float beta;
  const float* cur[4];
  const float* ref[4];
  int rows_p[4];
  float* x1[4];
  float* x2[4];
  float* x1T[4];   // optional transposed copies [32][rows_p]
  float* x2T[4];
};
hipError_t launch_chi(const ChiArgs& a, hipStream_t s);

// beta = 1 J-CoMM inner loop for CP.  At beta = 1, chi_1(A, A~) = A~ and
// chi_2(A, A~) = A with Q~ = 1, so Num_J^(n) depends only on the reference and
// Den_J^(n)(i, r) = prod_{m != n} S^(m)(r), S the column sums of the current
// inner blocks; the update is A^(n) = max(c^(n) / Den^(n), eps) with
// c^(n) = A~^(n) * Num_J^(n), whose column sums are T^(n) / Den when no entry of
// the column clips (min c >= eps Den) and are summed exactly otherwise.  The L
// sweeps reduce to recurrences on 32-wide vectors; kl_apply runs them (every
// workgroup redundantly, from the per-block column statistics of the slot
// reduction) and writes max(c / Den_last, eps).
struct KlLoopArgs {
  int N, R, L;
  float eps;
  const float* c[4];       // [rows_p][32]
  const float* stats[4];   // [nblk][3][32]
  int nblk[4];
  int rows[4];
  float* cur_pad[4];       // optional padded outputs [rows_p][32]
  float* user[4];          // caller buffers (row stride R)
  const double* obj_part;  // optional: objective partials to sum into *obj_out
  int64_t obj_n;
  double* obj_out;         // written if not NULL
  int obj_add_model_mass;  // also add sum_r prod_n colsum(A~^(n))_r (sparse objective)
};
hipError_t launch_kl_apply(const KlLoopArgs& a, hipStream_t s);

// Reduction of partial slots [slots][rows_total][32] (fixed order) fused with
//   kSlotScale:  out = anchor * Num, plus per-block column statistics
//                (sum of out, min of out over valid rows, sum of anchor)
//   kSlotCopy:   out = Num, with the same statistics
//   kSlotUpdate: out = max(anchor * (Num / Den)^gamma, eps), Den from its own
//                slots or den_closed[c]
// A workgroup covers kSlotRows rows x 32 columns of one job.
constexpr int kSlotRows = 2;
enum SlotMode : int { kSlotScale = 0, kSlotUpdate = 1, kSlotCopy = 2 };
struct SlotJob {
  int mode;
  const float* num_part;  int num_slots;
  const float* den_part;  int den_slots;   // NULL: use den_closed
  const float* den_closed;
  int rows_total;          // rows of one slot
  int rows, cols;          // valid extent
  int rows_p;              // rows written to out_pad (>= rows)
  FView anchor;            // multiplicative pre-factor
  float gamma, eps;
  float* out_pad;          // optional [rows_p][32]
  float* out_padT;         // optional [32][rows_p]
  float* out_user;         // optional caller buffer (valid rows x cols), row stride ld_user
  int ld_user;
  float* stats;            // scale mode: [ceil(rows_p / kSlotRows)][3][32]
};
struct SlotUpdateArgs {
  int njobs;
  SlotJob job[4];
};
hipError_t launch_slot_update(const SlotUpdateArgs& a, hipStream_t s);

// Sum of n float64 partials in a fixed order; writes *out (device).  If add_to
// is not NULL its value is added.
hipError_t launch_sum_f64(const double* part, int64_t n, const double* add_to, double* out, hipStream_t s);


// ----------------------------------------------------------------------------------------
// Dense 3-way Tucker (tucker3_impl.h, tucker3.hip)
// ----------------------------------------------------------------------------------------

// A Tucker model as seen by the kernels: core entry (a, b, c) at
// G[(a * J2 + b) * ldG + c]; factors as views with cols = J_n.
struct TkModel {
  const float* G;
  int ldG;
  FView A, B, C;
  int J1, J2, J3;
};

struct TkPassArgs {
  const float* X;          // I x J x K
  const float* Wc;         // cached weight tensor (cache read)
  float* Pw;               // cache targets (cache write)
  float* Qw;
  int I, J, K, Kp;
  TkModel r;               // rebuild model
  TkModel n;               // contraction set
  float eps, eps_x;
  int use_q;               // contract Q instead of P
  int want_v, want_m3;
  BetaConst bc;
  float* V;                // [I][J][32]
  float* m3;               // [workgroups][Kp][32] partial slots
  double* obj_part;        // one float64 partial per workgroup
};

struct TkGrid {
  int gi, gj;
  int wgs() const { return gi * gj; }
};
TkGrid tk_grid(int I, int J);
// mode (bits 0-1): 0 = from X, 1 = read the cached weight Wc, 2 = from X and
// write P~ / Q~; bit 2 set: also accumulate the objective (not with mode 1).
hipError_t launch_tk_pass(const TkPassArgs& a, const TkGrid& g, int beta_class, int mode, hipStream_t s);

// Small strided GEMM with split-K partial slots (fixed order, deterministic):
//   out[split][batch][m][n] = sum_{k in split} A(batch, m, k) B(batch, k, n)
// with A(b, m, k) = A[b * sab + m * sam + (k / akin) * sako + (k % akin) * saki]
// and  B(b, k, n) = B[b * sbb + (k / bkin) * sbko + (k % bkin) * sbki + n * sbn];
// out row stride ldo, batch stride sob, split stride sos.
struct GemmArgs {
  const float* A;
  int64_t sab, sam, sako, saki;
  int akin;
  const float* B;
  int64_t sbb, sbko, sbki, sbn;
  int bkin;
  float* out;
  int64_t sob, sos, ldo;
  int M, N, K, batch, splits;
};
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s);

// Closed-form beta = 1 Tucker denominators from the column sums S of the
// denominator set (Q = 1): den[0][a] = sum_bc G[a][b][c] S_B[b] S_C[c],
// den[1][b] = sum_ac G S_A S_C, den[2][c] = sum_ab G S_A S_B and
// dcore[(a J2 + b)][c] = S_A[a] S_B[b] S_C[c].
hipError_t launch_tk_den_closed(const TkModel& m, int I, int J, int K, float* den /*[3][32]*/,
                                float* dcore /*[J1 J2][32]*/, hipStream_t s);

}  // namespace comm
