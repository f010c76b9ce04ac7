// Host-visible declarations of the kernel launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dmath.h"

namespace comm {

// Padded rank / core width every dense kernel works with: factor copies in the
// workspace are [rows_padded][32] row-major with zero padding.
constexpr int kRP = 32;

// Largest tensor order of the dense CP path (orders 4 and 5 run through a
// 3-way view, see KrArgs below).
constexpr int kMaxModes = 5;

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
  int bf16;                // 1: rebuild in split bf16 (three products), contractions in bf16
  BetaConst bc;
  float* m3n;              // partial slots: m3 [gi*gj][Kp][32], m1 [gj*gk][Ip][32], m2 [gi*gk][Jp][32]
  float* m1n;
  float* m2n;
  float* m3d;
  float* m1d;
  float* m2d;
  double* obj_part;        // one float64 partial per workgroup
  int x_zero;              // X is all zero and not read (x = 0 everywhere); P is then
                           // zero and its contractions are skipped (beta != 1 only)
  int xbuf;                // interior tiles may read X (or the cache) through a buffer
                           // resource: 16 J K + 32 K < 2^31 (every in-tile byte offset fits)
  float* Vn;               // V pass (launch_cp_vpass): V of the numerator / denominator set, [I*J][32]
  float* Vd;
  int r16;                 // every factor column >= 16 is zero (rank <= 16): 16-wide tiles
                           // (float32 only; ignored with bf16); slot columns >= 16 are then not written
};

hipError_t launch_cp_pass(const CpPassArgs& a, const CpGrid& g, int beta_class, bool den, hipStream_t s);
// The mode-1 pass of a beta != 1 J-CoMM sweep that keeps V (numerator and
// denominator sets) for mode 2; M1 slots one per 32-wide j block (into m1n /
// m1d, rows Ip), the objective partials (want_obj, not with the cache) one
// per workgroup of cp_vpass_wgs.
hipError_t launch_cp_vpass(const CpPassArgs& a, int beta_class, hipStream_t s);
int64_t cp_vpass_wgs(int I, int J);
int cp_vpass_m1_slots(int J);
// M2 from the kept V: slots[c][j][r] = sum over i in chunk c of V[i][j][r] A'[i][r]
// (kVFoldChunks chunks, rows Jp), numerator and denominator sets.
constexpr int kVFoldChunks = 8;
struct VFoldArgs {
  int I, J, Jp;
  const float* Vn;
  const float* Vd;
  FView An, Ad;            // the mode-1 block's transforms
  float* outn;
  float* outd;
};
hipError_t launch_vfold(const VFoldArgs& a, hipStream_t s);

// ----------------------------------------------------------------------------------------
// Small factor-side kernels (kernels_small.hip)
// ----------------------------------------------------------------------------------------

// dst[f][row][c] = src[f][row * ld + c] for row < rows[f], c < cols, zero elsewhere
// in [rows_p][32]; optional transposed copy dstT[f][c][row] and second copies.
struct PadArgs {
  int nf;
  int cols[kMaxModes], ld[kMaxModes];      // valid columns and row stride of each source
  const float* src[kMaxModes];
  int rows[kMaxModes];
  int rows_p[kMaxModes];
  float* dst[kMaxModes];
  float* dstT[kMaxModes];
  float* dst2[kMaxModes];
  float* dst2T[kMaxModes];
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
  const float* cur[kMaxModes];
  const float* ref[kMaxModes];
  int rows_p[kMaxModes];
  float* x1[kMaxModes];
  float* x2[kMaxModes];
  float* x1T[kMaxModes];   // optional transposed copies [32][rows_p]
  float* x2T[kMaxModes];
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
  const float* c[kMaxModes];       // [rows_p][32]
  const float* stats[kMaxModes];   // [nblk][3][32]
  int nblk[kMaxModes];
  int rows[kMaxModes];
  float* cur_pad[kMaxModes];       // optional padded outputs [rows_p][32]
  float* user[kMaxModes];          // caller buffers (row stride R)
  const double* obj_part;  // optional: objective partials to sum into *obj_out
  int64_t obj_n;
  double* obj_out;         // written if not NULL
  int obj_add_model_mass;  // also add sum_r prod_n colsum(A~^(n))_r (sparse objective)
};
hipError_t launch_kl_apply(const KlLoopArgs& a, hipStream_t s);
// Sets `bit` in *flag if one of the n floats at p is below lo or not finite.
hipError_t launch_check_range(const float* p, int64_t n, float lo, int bit, int* flag, hipStream_t s);

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
  // optional: the J-CoMM transforms of the new block (as chi_kernel computes
  // them from out_pad), written for rows < rows_p: chi_1 to chi_x1, chi_2 to
  // chi_x2 (and transposed copies when set), against chi_ref [rows_p][32]
  const float* chi_ref;
  float* chi_x1;
  float* chi_x2;
  float* chi_x1T;
  float* chi_x2T;
  float chi_beta;
};
struct SlotUpdateArgs {
  int njobs;
  SlotJob job[kMaxModes];
};
hipError_t launch_slot_update(const SlotUpdateArgs& a, hipStream_t s);

// Order-N CP (N = 4, 5) through a 3-way view.  Modes 1..G (G = N - 2) are
// fused into one super mode s = (i_1, ..., i_G), row-major (i_1 slowest), so
// that the caller's tensor, unchanged in memory, is the 3-way tensor
// (I_1 ... I_G) x I_{N-1} x I_N, and the CP model with factors
// (KR, A^(N-1), A^(N)) rebuilds it exactly, KR the row-wise (Khatri-Rao)
// product KR[s, r] = prod_{m < G} A^(m)[i_m, r] (Sec. 3.3).
constexpr int kMaxGroup = kMaxModes - 2;

// KR of G factors into [rows_p][32] (zero rows and columns beyond the valid
// extent); up to two products per launch.
struct KrArgs {
  int G;
  int dims[kMaxGroup];
  int rows, rows_p;        // prod dims, padded rows written
  int nout;
  FView f[2][kMaxGroup];
  float* out[2];
};
hipError_t launch_kr(const KrArgs& a, hipStream_t s);

// Numerator (or denominator) of a grouped mode from the super mode's partial
// slots: out[i, r] = sum_{s : s_mode = i} (sum_slot part[slot][s][r])
// * prod_{m != mode} W^(m)[s_m, r] (CPContr^(n) of Sec. 6.1 taken in two
// steps: over modes N-1 and N in the pass, over the other grouped modes here).
// Rows dims[mode]..rows_p-1 are written as zero.  Fixed order: deterministic.
struct FoldJob {
  int mode;
  const float* part;
  int slots, rows_total;   // part is [slots][rows_total][32]
  FView w[kMaxGroup];      // entry `mode` unused
  float* out;              // [rows_p][32]
  int rows_p;
};
struct FoldArgs {
  int G;
  int dims[kMaxGroup];
  int njobs;
  FoldJob job[2 * kMaxGroup];
};
hipError_t launch_fold(const FoldArgs& a, hipStream_t s);

// Extrapolation of the parameter blocks (contiguous caller buffers, `count`
// entries each).  launch_extrap_alpha writes alpha_t to alpha[0]; launch_
// extrap_apply reads it and moves the listed blocks, saving their old values
// in prev.
constexpr int kMaxBlocks = kMaxModes + 1;  // a Tucker core and its factors
struct ExtrapArgs {
  int nb;
  float* cur[kMaxBlocks];
  float* prev[kMaxBlocks];
  int64_t count[kMaxBlocks];
  double alpha_nes, c, delta;
  float* alpha;
  float eps;
};
hipError_t launch_extrap_alpha(const ExtrapArgs& a, hipStream_t s);
hipError_t launch_extrap_apply(const ExtrapArgs& a, hipStream_t s);

// Sparse COO at any beta in (0, 2) (Sec. 6.4, paragraph on sparse tensors):
// per nonzero t (half a wavefront, lane = rank component), X~_t from the
// rebuild set rb, P_t = x_t max(X~_t, eps)^(beta-2), and for `mode` >= 0
// num[i_mode][r] += P_t prod_{m != mode} ct_m[i_m][r] (float atomics).  With
// w_in the weights come from an earlier call instead of a rebuild; w_out
// keeps them.  obj_part (one value per workgroup) receives the sum over the
// nonzeros of d(x | X~) - d(0 | X~), the correction of a dense evaluation at
// X = 0.  Nonzeros with a coordinate outside [0, dims) are skipped.
struct CooBetaArgs {
  int N, R;
  int64_t nnz;
  int dims[kMaxModes];
  const int32_t* idx[kMaxModes];
  const float* val;
  FView rb[kMaxModes];
  FView ct[kMaxModes];
  int mode;
  float* num;              // [dims[mode]][32], zeroed by the caller
  const float* w_in;
  float* w_out;
  double* obj_part;
  BetaConst bc;
  float eps;
};
int coo_beta_blocks(int64_t nnz);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);
hipError_t launch_coo_beta(const CooBetaArgs& a, int beta_class, hipStream_t s);

// Sparse COO data for an order-N Tucker model (N = 3..5) on the
// (I_1 ... I_{N-1}) x I_N view: per nonzero t (half a wavefront, lane = d)
// X~_t = sum_d T[row_t][d] C[i_N][d] from the rebuild table T and fibre-mode
// factor C, P_t = x_t max(X~_t, eps)^(beta-2) (or w_in[t]); then
//   op 1: out[row_t][d] += P_t Cc[i_N][d]   (the V rows: P contracted on mode N)
//   op 2: out[i_N][d]   += P_t Tc[row_t][d] (the fibre-mode numerator)
// with the contraction set's fibre factor Cc / table Tc (float atomics).
// w_out keeps the weights; obj_part receives per workgroup the sum over the
// nonzeros of d(x | X~) - d(0 | X~).  Out-of-range coordinates are skipped.
struct CooTkArgs {
  int N;
  int64_t nnz;
  int dims[kMaxModes];
  const int32_t* idx[kMaxModes];
  const float* val;
  const float* Tr;
  FView Cr;
  int op;
  const float* Tc;
  FView Cc;
  float* out;
  const float* w_in;
  float* w_out;
  double* obj_part;
  BetaConst bc;
  float eps;
};
hipError_t launch_coo_tucker(const CooTkArgs& a, int beta_class, hipStream_t s);

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

// T2[(i, j)][c] = sum_{a,b} A[i][a] B[j][b] G[a][b][c] for every pair, row
// stride 32 (zero past J3): the Tucker reconstruction is X^[(i,j)][k] =
// sum_c T2[(i,j)][c] C[k][c].
// sets = 1 or 2 models (m[0] -> T2[0], m[1] -> T2[1]) in one launch.  The
// factor B of each model must be a padded [J][32] copy.  T2T[set], when not
// NULL, also receives the transposed [32][Pp] layout, zero for pairs >= I J.
hipError_t launch_tk_t2(const TkModel* m, float* const* T2, float* const* T2T, int sets, int I, int J, int64_t Pp,
                        hipStream_t s);

// Arguments of the two Tucker pass kernels.  X is read as an (I J) x K matrix:
// row (i, j) is the mode-3 fibre of pair (i, j).
struct TkPassArgs {
  const float* X;
  const float* Pc;         // cached P~ / Q~ (cache read)
  const float* Qc;
  float* Pw;               // cache targets (cache write)
  float* Qw;
  int I, J, K, Kp;
  const float* T2r;        // rebuild T2 [(I J)][32]
  FView C;                 // rebuild mode-3 factor
  const float* CnT;        // V pass: mode-3 factor of the numerator / denominator set,
  const float* CdT;        //   transposed [32][Kp], zero for k >= K
  const float* T2nT;       // mode-3 pass: T2 of the numerator / denominator set,
  const float* T2dT;       //   transposed [32][Pp], zero for pairs >= I J
  int64_t Pp;              // I J rounded up to a multiple of 32
  int xvec;                // fibres may be read as 16-byte vectors (K % 4 == 0, X 16-byte aligned)
  int bf16;                // 1: rebuild in split bf16, contraction tiles in bf16
  float eps, eps_x;
  BetaConst bc;
  float* Vn;               // V pass outputs [(I J)][32]
  float* Vd;
  float* m3n;              // mode-3 pass outputs: partial slots [npg][Kp][32]
  float* m3d;
  double* obj_part;        // one float64 partial per workgroup of the V pass
  int tpw, npg;            // mode-3 pass: pair tiles per wave, pair groups
};

enum TkMode : int { kTkFromX = 0, kTkCacheRead = 1, kTkCacheWrite = 2 };

// V pass, one workgroup per 32 pairs, its four waves splitting K:
//   Vn[(i,j)][c] = sum_k P[(i,j)][k] Cn[k][c]
//   Vd[(i,j)][c] = sum_k Q[(i,j)][k] Cd[k][c]   (sets = 2)
// sets = 0 computes only the objective (obj) or only the cache (cache write).
// Workgroups: ceil(I J / 32); obj_part gets one value per workgroup.
int64_t tk_v_workgroups(int I, int J);
hipError_t launch_tk_v(const TkPassArgs& a, int beta_class, int mode, bool obj, int sets, hipStream_t s);

// Mode-3 pass: m3n[g][k][c] = sum over pair group g of P[(i,j)][k] T2n[(i,j)][c]
// (and m3d with Q and T2d when sets = 2).
void tk_m3_tiling(int I, int J, int* tpw, int* npg, int groups = 0);
hipError_t launch_tk_m3(const TkPassArgs& a, int beta_class, int mode, int sets, hipStream_t s);

// Small strided GEMMs on the matrix cores, split-K partial slots (fixed order,
// deterministic), for one or two operand sets at once:
//   out[set][split][batch][m][n] = sum_{k in split} A_set(batch, m, k) B_set(batch, k, n)
// with A(b, m, k) = A[b * sab + m * sam + (k >> akin_log2) * sako + (k & (2^akin_log2 - 1)) * saki]
// and  B(b, k, n) = B[b * sbb + (k >> bkin_log2) * sbko + (k & (2^bkin_log2 - 1)) * sbki + n * sbn];
// out row stride ldo, batch stride sob, split stride sos.
struct GemmArgs {
  const float* A[2];
  int64_t sab, sam, sako, saki;
  int akin_log2;
  const float* B[2];
  int64_t sbb, sbko, sbki, sbn;
  int bkin_log2;
  float* out[2];
  int64_t sob, sos, ldo;
  int M, N, K, batch, splits, sets;
};
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s);

// Closed-form beta = 1 Tucker denominators from the column sums S of the
// denominator set (Q = 1): den[0][a] = sum_bc G[a][b][c] S_B[b] S_C[c],
// den[1][b] = sum_ac G S_A S_C, den[2][c] = sum_ab G S_A S_B and
// dcore[(a J2 + b)][c] = S_A[a] S_B[b] S_C[c].
hipError_t launch_tk_den_closed(const TkModel& m, int I, int J, int K, float* den /*[3][32]*/,
                                float* dcore /*[J1 J2][32]*/, hipStream_t s);

}  // namespace comm
