/*
 * comm.h -- C ABI of the MI355X (gfx950) library for contraction-only
 * majorization-minimization updates of nonnegative CP and Tucker models under
 * beta-divergences (Leplat, "Joint Majorization-Minimization for Nonnegative CP
 * and Tucker Decompositions under beta-Divergences: Unfolding-Free Updates").
 *
 * Problem (Sec. 3): a nonnegative data tensor X (I_1 x ... x I_N), a CP model
 * (factors A^(n), I_n x R) or a Tucker model (core G, J_1 x ... x J_N, and
 * factors A^(n), I_n x J_n), all parameters >= eps (Assumption "positivity
 * safeguard"), and beta in [0, 2).
 *
 * Conventions shared by every entry point
 *   - Tensors, factors and cores are caller-owned DEVICE buffers of float32,
 *     contiguous row-major (last index fastest).  Factor n is I_n x R (CP) or
 *     I_n x J_n (Tucker), row stride R (or J_n).
 *   - Model parameters are updated IN PLACE.
 *   - Every call is asynchronous on the given HIP stream (NULL = default
 *     stream).  Results are visible after the caller synchronises the stream.
 *   - Arguments are validated on the host before anything is launched; on an
 *     error nothing is modified and the call returns a nonzero code, with a
 *     message available from comm_last_error() (thread-local).
 *   - Outputs are clipped to >= eps.  Inputs with entries < eps violate the
 *     precondition of the paper's updates; the library checks them only when
 *     opts.check_inputs is set (a debug mode that synchronises the stream).
 *   - Device faults surface at the caller's next synchronisation, or through
 *     comm_check().
 *   - No C++ exception crosses this interface.
 *   - Calls sharing one context must not overlap in time (the context owns
 *     the scratch workspace); use one context per concurrent stream.
 *   - Dense reductions are deterministic: the same inputs give bitwise
 *     identical outputs on the same device.
 *
 * Supported in this version: dense CP of order 3, 4 and 5 (rank R <= 32; at
 * orders 4 and 5 the product I_1 ... I_{N-2} must not exceed 2^24); dense
 * Tucker of order 3, 4 and 5 (core sizes J_n <= 32; at orders 4 and 5 the
 * product I_1 ... I_{N-1} must not exceed 2^24); sparse COO CP of order 2 to
 * 4 at beta = 1 and of order 3 to 5 at any beta in (0, 2); sparse COO Tucker
 * of order 3 to 5 at beta in (0, 2).  Other shapes return COMM_EUNSUPPORTED.  The sparse paths
 * accumulate with float atomics and are reproducible to rounding only; the
 * dense paths are deterministic.
 *
 * Dense CP of order N = 4, 5 runs through a 3-way view of the same memory:
 * modes 1..N-2 form one mode of extent I_1 ... I_{N-2} whose factor is the
 * row-wise (Khatri-Rao) product of theirs, so the view's CP model rebuilds the
 * same tensor, and the numerator of each of those modes is the view's
 * numerator contracted with the other grouped factors (the mode-n
 * contraction of Sec. 6.1 in two steps).  Per sweep this costs N passes over X
 * for B-CoMM, and for J-CoMM one pass at beta = 1 and three at beta != 1
 * (modes 1..N-2 share one).
 *
 * Dense Tucker of order N = 4, 5 runs the fused passes of order 3 on the
 * (I_1 ... I_{N-1}) x I_N matrix view: a row is rebuilt from the core
 * multiplied by the first N - 1 factors (mode products) and the last factor,
 * and the numerators of the core and of modes 1 to N - 1 are mode products of
 * the pass's output contracted with the core (App. C for general N).
 */
#ifndef COMM_H_
#define COMM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define COMM_OK 0
#define COMM_EINVAL 1        /* bad argument: NULL pointer, dims, rank, beta outside [0,2), eps <= 0, L < 1 */
#define COMM_EUNSUPPORTED 2  /* valid problem outside what this build implements */
#define COMM_ENOMEM 3        /* workspace would exceed the context's limit, or allocation failed */
#define COMM_EHIP 4          /* HIP runtime error; message carries hipGetErrorString */

/* Model kinds. */
#define COMM_CP 0
#define COMM_TUCKER 1

/* Arithmetic of the matrix-core tiles.  Power step, updates and all
 * reductions outside the tiles are float32 in both; the objective is
 * accumulated in float64 in both.
 *   COMM_FP32: float32 tiles.
 *   COMM_BF16: contraction tiles (numerators, denominators) with bf16
 *              operands and float32 accumulation; the reconstruction tile
 *              with split-bf16 operands (x = hi + lo, three products), about
 *              16 significant bits per operand, because the power step and
 *              the objective read it.  Dense CP and Tucker passes; the
 *              small Tucker GEMMs that follow the passes, and the sparse
 *              path (no matrix-core tiles), compute in float32 either way. */
#define COMM_FP32 0
#define COMM_BF16 1

/* comm_opts.cache_pq: take the choice recorded by comm_tune_jcomm. */
#define COMM_CACHE_AUTO (-1)

typedef struct comm_ctx comm_ctx;

/* Largest order of comm_dense and comm_model. */
#define COMM_MAX_NDIM 5

/* Dense data tensor X >= 0 (Sec. 3.1).  X points to prod(dims) floats. */
typedef struct {
  int ndim;
  int64_t dims[COMM_MAX_NDIM];
  const float* X;
} comm_dense;

/* Model parameters Theta (Sec. 3.3).
 *   kind == COMM_CP:     rank R, factors[n] -> I_n x R; core unused.
 *   kind == COMM_TUCKER: core_dims J_n, core -> J_1 x ... x J_N,
 *                        factors[n] -> I_n x J_n; rank unused. */
typedef struct {
  int kind;
  int rank;
  int64_t core_dims[COMM_MAX_NDIM];
  float* factors[COMM_MAX_NDIM];
  float* core;
} comm_model;

/* Options.
 *   beta          in [0, 2).
 *   eps           lower bound on every parameter (> 0); the reconstruction
 *                 also enters powers, logs and divisions as max(Xhat, eps).
 *   eps_x         at beta = 0 the data enter as max(X, eps_x) (> 0).
 *   inner_sweeps  L >= 1, inner sweeps per J-CoMM outer iteration.
 *   precision     COMM_FP32 or COMM_BF16 (see above).
 *   cache_pq      J-CoMM at beta != 1: 1 = store P~ and Q~ once per outer
 *                 iteration in the workspace and stream them in the inner
 *                 passes; 0 = recompute them from X and the reference;
 *                 COMM_CACHE_AUTO = the choice comm_tune_jcomm recorded for
 *                 this problem in the context, else 1 if the workspace the
 *                 cache needs is within the context's limit, else 0.  Both
 *                 give the same results; only time and workspace differ.
 *                 Other values are refused (COMM_EINVAL).
 *   check_inputs  debug mode: 1 = before anything is launched, verify on the
 *                 device that the data are finite and >= 0 (dense X, or the
 *                 COO values) and every parameter is finite and >= eps
 *                 (the precondition Theta >= eps of the updates); a violation
 *                 returns COMM_EINVAL with nothing modified.  The check
 *                 synchronises the stream, so it cannot run under stream
 *                 capture.  0 = no check (default). */
typedef struct {
  double beta;
  double eps;
  double eps_x;
  int inner_sweeps;
  int precision;
  int cache_pq;
  int check_inputs;
} comm_opts;

/* Sparse COO data, for the CP and Tucker entry points that take it (each
 * states its orders and its range of beta).  idx[n][t] is the mode-n
 * coordinate of nonzero t (int32, 0 <= idx < dims[n]); val[t] > 0.  Device
 * buffers, read only. */
typedef struct {
  int ndim;
  int64_t dims[COMM_MAX_NDIM];
  int64_t nnz;
  const int32_t* idx[COMM_MAX_NDIM];
  const float* val;
} comm_coo;

/* One problem of a batched call: the arguments of comm_jcomm_outer. */
typedef struct {
  const comm_dense* x;
  comm_model* model;
  const comm_opts* opts;
  double* obj_ref_dev; /* may be NULL */
} comm_problem;

/* Flags of comm_jcomm_outer_batched. */
#define COMM_BATCH_GRAPH 1 /* capture the batch into a HIP graph; replay it while the problem list is unchanged */
/* Run the problems' launches grouped: each kernel that several problems run at
 * the same point of their sequence is launched once for all of them, its
 * workgroups reading their problem's arguments from a table in device memory
 * (one stream; results bitwise those of separate calls).  Dense problems of
 * order 3 only: a batch holding another order runs ungrouped. */
#define COMM_BATCH_GROUPED 2

/* Create a context on HIP device `device`.  The context owns a scratch
 * workspace that grows on demand up to `workspace_limit_bytes` (0 = no limit).
 * Returns COMM_OK and sets *out, or an error code. */
int comm_create(int device, size_t workspace_limit_bytes, comm_ctx** out);

/* Synchronise the context's last stream and free its workspace. */
int comm_destroy(comm_ctx* ctx);

/* Synchronise the stream of the context's last call and report an
 * asynchronous HIP error raised since (a device fault in a kernel), as
 * COMM_EHIP with the runtime's message; COMM_OK otherwise. */
int comm_check(comm_ctx* ctx);

/* Autotuning of J-CoMM (not a passage of the paper: a choice between
 * equivalent evaluations of the same update).  For the problem given (shapes,
 * rank or core sizes, beta, precision and L of x, model and opts;
 * opts->cache_pq is ignored), runs one untimed and then `reps` timed outer
 * iterations of each variant, each from a device copy of the model's
 * parameters, so the caller's model is left as it was.  The variants:
 *   - beta != 1: P~ / Q~ cached (cache_pq = 1) or recomputed (0);
 *   - dense CP at rank <= 16 with float32 tiles: 16-wide (16x16x4 matrix-core
 *     shapes) or 32-wide pass tiles (rank padded to 32);
 *   - dense CP of order 3 at beta != 1: modes 1 and 2 of a sweep from one V
 *     pass (V = P~ x3 chi(C), kept for mode 2) or from a pass each;
 *   - dense Tucker of order 3: at most 128, 64 or 256 pair groups (partial
 *     slots) in the mode-3 pass.
 * The fastest is stored in the context's autotune table.  An entry fixes the
 * launch shapes (the last two choices) of every J-CoMM call on a problem with
 * the same key in this context, single, batched or allocation-free, and its
 * cache choice for calls with cache_pq = COMM_CACHE_AUTO; a call with an
 * explicit cache_pq and the entry's cache choice gives bitwise the AUTO
 * result.  Different choices change only the order of float32 sums.  Cache
 * variants that cannot run (workspace limit) are skipped.  A problem with a
 * single variant (CP at beta = 1, orders 4 and 5 at beta = 1) records the
 * defaults without timing.
 *   reps     1 to 1000.
 *   choice   if not NULL, receives the recorded cache choice (0 or 1).
 *   ms       if not NULL, receives ms[0] and ms[1], the mean time of one outer
 *            iteration in milliseconds of the fastest variant that recomputes
 *            (0) and that caches (1), NaN when none ran.
 * The call allocates a copy of the parameters, may grow the workspace to the
 * largest variant's, synchronises `stream`, and drops the cached graph of the
 * batched entry point.  Errors as for comm_jcomm_outer. */
int comm_tune_jcomm(comm_ctx* ctx, const comm_dense* x, const comm_model* model, const comm_opts* opts, int reps,
                    int* choice, double* ms, void* stream);

/* What the autotune table holds for a problem (the key as for
 * comm_tune_jcomm; buffer pointers are not read).  found = 0: no entry, and
 * the other fields give the defaults a call would run with. */
typedef struct {
  int found;      /* 1 if comm_tune_jcomm recorded this problem */
  int cache_pq;   /* the recorded cache choice (0 without an entry) */
  int wshare;     /* dense CP of order 3 at beta != 1: 1 = modes 1 and 2 from one V pass; -1 otherwise */
  int tk_groups;  /* dense Tucker of order 3: pair-group cap of the mode-3 pass; 0 otherwise */
  int cp_tile;    /* dense CP: width of the pass tiles, 16 or 32; 0 for Tucker */
  int variants;   /* variants timed for the entry (0: untimed defaults) */
  double ms;      /* mean time of one outer iteration of the recorded variant (NaN if untimed) */
} comm_tune_entry;

int comm_tune_lookup(comm_ctx* ctx, const comm_dense* x, const comm_model* model, const comm_opts* opts,
                     comm_tune_entry* out);

/* Record a table entry directly (a choice timed earlier, in another process,
 * or fixed by the caller); the same effect on later calls as an entry that
 * comm_tune_jcomm recorded.  Read from `entry`: cache_pq (0 or 1; 0 at
 * beta = 1), wshare (-1 = by precision, or 0 / 1 for dense CP of order 3 at
 * beta != 1; -1 otherwise) and tk_groups (0 = 128, or 1 to 1024 for dense
 * Tucker of order 3; 0 otherwise) and cp_tile (0 = by rank and precision,
 * 32 = 32-wide, 16 = 16-wide where the rank is <= 16 with float32 tiles; 0
 * for Tucker); the other fields are ignored.  Buffer
 * pointers are not read.  Synchronises `stream` and the batched entry
 * point's streams, and drops its cached graph.  COMM_EINVAL on a field
 * outside these ranges (the table is then unchanged). */
int comm_tune_set(comm_ctx* ctx, const comm_dense* x, const comm_model* model, const comm_opts* opts,
                  const comm_tune_entry* entry, void* stream);

/* Message of the last error raised on this thread (never NULL). */
const char* comm_last_error(void);

/* Workspace bytes a call with these arguments would need (0 on invalid
 * arguments).  `op` is 0 = cp_update / tucker_update, 1 = jcomm_outer,
 * 2 = beta_objective.  Only shapes, model kind, rank / core sizes and options
 * are read; buffer pointers may be NULL (a server sizes requests before
 * loading them).  There is no context, hence no autotune table, so the
 * largest need over its choices is returned: cache_pq = COMM_CACHE_AUTO
 * counts as 1, CP J-CoMM at beta != 1 with the V pass kept for mode 2,
 * Tucker J-CoMM with 256 mode-3 pair groups. */
size_t comm_workspace_bytes(const comm_dense* x, const comm_model* model, const comm_opts* opts, int op);

/* Measurement hooks.  comm_profile_enable(ctx, every) with every >= 1 times
 * every `every`-th launch of the fused dense pass kernel (the kernel that
 * streams X) on the call's stream, starting with the first: the dispatch
 * itself stamps a pair of HIP events with the kernel's start and end (inside a
 * stream capture the pair is recorded around the launch instead); every = 0
 * turns the measurement off; every < 0 is COMM_EINVAL.  Timing a launch costs
 * the stream a few microseconds, so a sampled measurement (every > 1)
 * disturbs a timed loop less.  comm_profile_query() waits for the recorded
 * events, returns the summed time of the timed launches in milliseconds, their
 * count in *launches and, when `seen` is not NULL, the count of all pass
 * launches in *seen, since the last enable/query, and resets the record.
 * Enabling also resets it, and creates the first 2048 event pairs up front (on
 * the context's device) so that measured launches do not pay for creating
 * them; the events live until comm_destroy(). */
int comm_profile_enable(comm_ctx* ctx, int every);
int comm_profile_query(comm_ctx* ctx, double* total_ms, int64_t* launches, int64_t* seen);

/* Block-MM (B-CoMM) update of a CP model (Theorem "CP block multiplicative
 * update"; Algorithm B-CoMM).  block in 0..N-1 updates that factor; block = -1
 * runs one full sweep over modes 1..N, rebuilding Xhat and P, Q before every
 * block.  Each block: A^(n) <- max(A^(n) * (Num^(n)/Den^(n))^gamma(beta), eps)
 * with Num/Den = CPContr^(n)(P or Q; other factors). */
int comm_cp_update(comm_ctx* ctx, const comm_dense* x, comm_model* model, int block,
                   const comm_opts* opts, void* stream);

/* Block-MM update of a Tucker model (Sec. 4.3; Theorem "Tucker block
 * multiplicative updates"; App. C.2).  block = -1 updates the core, 0..N-1 a
 * factor, -2 runs a full sweep (core, then modes 1..N). */
int comm_tucker_update(comm_ctx* ctx, const comm_dense* x, comm_model* model, int block,
                       const comm_opts* opts, void* stream);

/* One outer iteration of J-CoMM (Algorithm J-CoMM; Sec. 5.3; App. C.3) for a
 * CP or Tucker model: reference Theta~ = current parameters, reference tensors
 * P~ = X * X~^(beta-2), Q~ = X~^(beta-1), then L = opts->inner_sweeps inner
 * sweeps of anchored updates Theta_b <- max(Theta~_b * (Num_J/Den_J)^gamma, eps).
 * Block order: CP modes 1..N; Tucker core, then modes 1..N.
 * If obj_ref_dev is not NULL, the objective at the reference,
 * F(Theta~) = D_beta(X, X~) (sum over all entries, float64), is written to
 * that device address. */
int comm_jcomm_outer(comm_ctx* ctx, const comm_dense* x, comm_model* model, const comm_opts* opts,
                     double* obj_ref_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * J-CoMM outer iteration of comm_jcomm_outer (same arguments, kernels, launch
 * shapes and results, bit for bit), with its workspace taken from a fixed
 * device array of COMM_NOALLOC_SCRATCH_BYTES that the library holds on each
 * GPU it runs on until the process ends.  It calls no hipMalloc, hipFree or
 * allocating library routine.
 *   - A problem whose workspace (comm_workspace_bytes, op = 1) exceeds the
 *     array returns COMM_ENOMEM before any launch.  cache_pq = 1 counts the
 *     P~/Q~ cache; COMM_CACHE_AUTO takes the autotune table's choice, or the
 *     cache when it fits, and recomputes when the cache does not fit.
 *   - opts.check_inputs is refused (COMM_EINVAL): the debug check needs a
 *     device flag of its own.
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents (nothing in it needs to start at zero: each call writes
 *     what it reads).  Calls that overlap on one GPU (other streams, threads
 *     or contexts) race: the caller orders them. */
#define COMM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int comm_jcomm_outer_noalloc(comm_ctx* ctx, const comm_dense* x, comm_model* model, const comm_opts* opts,
                             double* obj_ref_dev, void* stream);

/* One J-CoMM outer iteration (as comm_jcomm_outer) for each of `count`
 * independent problems of any mix of shapes, ranks, core sizes, beta and L:
 * the batched step of a decomposition server (not a passage of the paper; the
 * per-problem arithmetic is that of comm_jcomm_outer).
 *   - Each problem runs the same kernels with the same launch shapes and
 *     reduction order as a single call, on its own slice of a batch workspace,
 *     so its results are bitwise identical to comm_jcomm_outer on it alone,
 *     whatever else is in the batch.
 *   - Problems are spread over internal streams forked from and joined back to
 *     `stream`, so their kernels overlap on the device.  Problems must not
 *     share parameter or objective buffers.
 *   - flags = COMM_BATCH_GRAPH: the launches are captured once into a HIP graph
 *     and the graph is replayed on `stream` by every later call with the same
 *     problem list (same buffers, shapes and options, compared field by field);
 *     a different list waits for earlier replays and is captured anew.
 *   - flags |= COMM_BATCH_GROUPED: the problems' launches run grouped on
 *     `stream` (see COMM_BATCH_GROUPED), with the same bitwise results.  The
 *     launch tables live in device memory the context owns (one for eager
 *     calls, one kept with the captured graph); an eager grouped call waits for
 *     the previous one if that ran on another stream.
 *   - The batch workspace is the sum of comm_workspace_bytes(..., op = 1) over
 *     the problems (each rounded up to 256 bytes) and grows on demand within
 *     the context limit; growing it waits for earlier batched work.
 *   - Validation covers every problem before anything is launched; the message
 *     names the first bad problem. */
int comm_jcomm_outer_batched(comm_ctx* ctx, const comm_problem* problems, int count, int flags, void* stream);

/* Extrapolation weights of one outer iteration (Sec. "Going beyond:
 * Majorization-Minimization with Extrapolation"):
 *   alpha_t = min(alpha_nes, c / (||[Theta^(t) - Theta^(t-1)]_+|| + delta)),
 * one scalar for all blocks, the norm over every entry of the model.  The
 * paper fixes none of the three: the caller chooses them (e.g. alpha_nes =
 * (t - 1) / (t + 2)). */
typedef struct {
  double alpha_nes;  /* >= 0 */
  double c;          /* > 0 */
  double delta;      /* > 0 */
} comm_extrap;

/* Extrapolated B-CoMM sweep (items (i) CP and (ii) Tucker of that section).
 * `prev` has the shapes of `model` (distinct buffers) and holds, per block,
 * the value the block had before its update in the previous sweep (Theta^(t-1)).
 * alpha_t is computed on the device from model and prev; then every block, in
 * the sweep order (Tucker: core first), is moved to
 * max(A + alpha_t [A - A_prev]_+, eps) just before its own update, and the
 * block update is taken at, and anchored at, the moved block.  On return prev
 * holds each block's value before its update in this sweep, ready for the
 * next call.  alpha_dev (device float, may be NULL) receives alpha_t. */
int comm_bcomm_sweep_extrap(comm_ctx* ctx, const comm_dense* x, comm_model* model, comm_model* prev,
                            const comm_opts* opts, const comm_extrap* extrap, float* alpha_dev, void* stream);

/* J-CoMM with outer-reference extrapolation (item (iii)): the whole model is
 * moved to max(Theta + alpha_t [Theta - Theta_prev]_+, eps), prev receives the
 * model's value before the move, and one outer iteration of comm_jcomm_outer
 * runs from the moved model as its reference.  obj_ref_dev receives the
 * objective at that (extrapolated) reference. */
int comm_jcomm_outer_extrap(comm_ctx* ctx, const comm_dense* x, comm_model* model, comm_model* prev,
                            const comm_opts* opts, const comm_extrap* extrap, double* obj_ref_dev,
                            float* alpha_dev, void* stream);

/* D_beta(X, Xhat(model)) summed over all entries (Sec. 3.2, Definition of the
 * beta-divergence), written to the device address out_dev: float32 terms
 * (cancellation-free), reduced in float64 with compensated (TwoSum) sums over
 * lanes, wavefronts and workgroups in a fixed order.  Safeguards as in
 * comm_opts. */
int comm_beta_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* model,
                        const comm_opts* opts, double* out_dev, void* stream);

/* One J-CoMM outer iteration for a CP model on sparse COO counts (Sec. 6.4,
 * paragraph on sparse tensors): numerators accumulated over the nonzeros only.
 *   beta = 1: the denominator is the product of the other factors' column
 *     sums; any order 2 to 4; the objective's zero cells contribute the model
 *     value, summed in closed form.
 *   beta in (0, 2), beta != 1: the denominators involve Q = Xhat^(beta-1) on
 *     every cell, so they come from the dense pass run over the whole index
 *     space at x = 0 (the pass reads no tensor there, so the index space
 *     needs no memory; at most 2^36 cells); orders 3 to 5 (orders 4 and 5:
 *     I_1 ... I_{N-2} <= 2^24).  The nonzeros' weights P~ are formed once per outer
 *     iteration.  Results are reproducible to float rounding (atomics).
 *   beta = 0 returns COMM_EUNSUPPORTED (d(0 | y) is infinite).
 * If obj_ref_dev is not NULL the objective at the reference is written there. */
int comm_cp_jcomm_outer_coo(comm_ctx* ctx, const comm_coo* x, comm_model* model, const comm_opts* opts,
                            double* obj_ref_dev, void* stream);

/* Block-MM (B-CoMM) update of a CP model on sparse COO data at beta in (0, 2)
 * (Theorem "CP block multiplicative update" with the numerators over the
 * nonzeros, Sec. 6.4): block in 0..N-1 or -1 for a sweep.  At beta = 1 the
 * denominator is closed form; otherwise it comes from the dense pass over the
 * index space as for comm_cp_jcomm_outer_coo at beta != 1 (orders 3 to 5). */
int comm_cp_update_coo(comm_ctx* ctx, const comm_coo* x, comm_model* model, int block, const comm_opts* opts,
                       void* stream);

/* D_beta(X, Xhat) over every cell of a sparse COO tensor, beta in (0, 2),
 * float64, for a CP or a Tucker model (Sec. 3.2 over the cells of Sec. 6.4):
 * the dense pass's sum of d(0 | Xhat) over the index space plus, over the
 * nonzeros, d(x | Xhat) - d(0 | Xhat).  Orders 3 to 5.  CP at beta = 1 needs
 * no dense pass: a zero cell contributes Xhat, so the zero cells sum in closed
 * form as the model's mass sum_r prod_n colsum(A^(n))_r minus the nonzeros'
 * Xhat (orders 2 to 5, any index space, workspace independent of it). */
int comm_beta_objective_coo(comm_ctx* ctx, const comm_coo* x, const comm_model* model, const comm_opts* opts,
                            double* out_dev, void* stream);

/* Tucker on sparse COO data, orders 3 to 5, beta in (0, 2) (Sec. 4.3 and
 * App. C with the numerators over the nonzeros, Sec. 6.4).  The numerators'
 * contraction of P along the last mode is a scatter of the nonzeros into the
 * rows of the (I_1 ... I_{N-1}) x I_N view, the last mode's numerator a gather
 * of the rebuild table; the remaining contractions are those of the dense
 * order-N path.  Denominators: closed form at beta = 1, otherwise the dense
 * pass over the index space at x = 0 (no memory, as for CP).  block as in
 * comm_tucker_update; the J-CoMM call as comm_jcomm_outer.  Results are
 * reproducible to float rounding (atomics). */
int comm_tucker_update_coo(comm_ctx* ctx, const comm_coo* x, comm_model* model, int block, const comm_opts* opts,
                           void* stream);
int comm_tucker_jcomm_outer_coo(comm_ctx* ctx, const comm_coo* x, comm_model* model, const comm_opts* opts,
                                double* obj_ref_dev, void* stream);

/* A sparse COO tensor prepared for repeated J-CoMM iterations (CP, beta = 1):
 * two device copies of the nonzeros, sorted by the coordinates of modes 1
 * and 2 and by those of modes 3 and 4 (order 3: mode 3), so that every
 * mode's numerator accumulates over runs of equal coordinates instead of one
 * scattered add per nonzero.  Memory: 2 x (4 ndim + 4) bytes per nonzero,
 * owned by the plan.  Not a passage of the paper: a data layout for the
 * sparse numerators of Sec. 6.4. */
typedef struct comm_coo_plan comm_coo_plan;

/* Build a plan from the caller's COO (any order of the nonzeros; at most
 * 2^31 - 1 of them).  Sorts on the device on `stream`, waits for it, and
 * keeps no reference to the caller's buffers.  Nonzeros with a coordinate
 * outside [0, dims) are kept and skipped by every pass, as in
 * comm_cp_jcomm_outer_coo. */
int comm_coo_plan_create(comm_ctx* ctx, const comm_coo* x, comm_coo_plan** out, void* stream);

/* Free a plan (NULL is a no-op).  Work using it must have completed. */
int comm_coo_plan_destroy(comm_coo_plan* plan);

/* comm_cp_jcomm_outer_coo on a planned tensor: same result up to float
 * rounding order (both paths add with hardware float atomics). */
int comm_cp_jcomm_outer_coo_plan(comm_ctx* ctx, const comm_coo_plan* plan, comm_model* model,
                                 const comm_opts* opts, double* obj_ref_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* COMM_H_ */
