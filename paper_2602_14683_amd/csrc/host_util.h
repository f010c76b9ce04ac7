// Host-side utilities shared by the C ABI implementation files: the context,
// error reporting, workspace management and beta helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/comm.h"
#include "group.h"
#include "kernels.h"

// A roctx range around one entry-point call (host side: the call's enqueue
// time), named after the entry point; shown by rocprofv3 --marker-trace.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// One entry of the autotune table (comm_tune_jcomm): which of the equivalent
// evaluations of a J-CoMM outer iteration runs.  A recorded entry fixes the
// launch shapes of every J-CoMM call on that problem in the context; the cache
// choice applies to calls with cache_pq = COMM_CACHE_AUTO.
constexpr int kTkGroupsDefault = 128, kTkGroupsMax = 256, kTkGroupsLimit = 1024;
struct TuneChoice {
  int cache_pq = 0;    // stream the P~/Q~ cache (1) or recompute it from X (0)
  int wshare = -1;     // dense CP at beta != 1: modes 1 and 2 from one V pass (1) or a pass each (0);
                       // -1: by the tile precision (float32 shares, bf16 does not)
  int tk_groups = 0;   // dense order-3 Tucker mode-3 pass: at most this many pair groups (0: 128)
  int cp_tile = 0;     // dense CP passes: 0 = 16-wide tiles at rank <= 16 (float32), else 32-wide; 32 = 32-wide
  int variants = 0;    // table entries: variants timed (0: the defaults, untimed)
  double ms = 0.0;     // table entries: mean time of one outer iteration of this variant
};

struct comm_ctx {
  int device = 0;
  size_t limit = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t last_stream = nullptr;
  float* aux = nullptr;     // small device scratch that outlives workspace growth (extrapolation weight)
  // autotune table: J-CoMM problem key -> the measured fastest of its
  // equivalent evaluations; `pick` is the choice of the call in progress
  std::map<std::vector<int64_t>, TuneChoice> tune;
  TuneChoice pick;
  // measurement: event pairs around every fused dense pass launch
  bool profiling = false;
  int profile_every = 1;       // time every profile_every-th pass launch
  int64_t profile_seen = 0;    // pass launches since enable / query
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used = 0;
  // batched calls: one workspace holding every problem's own slice, internal
  // streams the problems are spread over, and the cached graph of the last
  // captured problem list
  char* bws = nullptr;
  size_t bws_bytes = 0;
  std::vector<hipStream_t> bstreams;
  hipStream_t bcapture = nullptr;
  hipEvent_t bfork = nullptr;
  std::vector<hipEvent_t> bjoin;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> gkey;
  hipStream_t glast = nullptr;
  // grouped batches: the launch tables (device: one for eager calls, one
  // owned by the captured graph) and the pinned host image they are copied from
  char* gtab = nullptr;
  size_t gtab_bytes = 0;
  char* gtab_graph = nullptr;
  size_t gtab_graph_bytes = 0;
  char* gtab_host = nullptr;
  size_t gtab_host_bytes = 0;
  hipEvent_t gtab_copied = nullptr;
  // sparse data at beta != 1 and sparse Tucker: the sparse steps' own
  // buffers (per-nonzero weights, one numerator, objective partials)
  char* sws = nullptr;
  size_t sws_bytes = 0;
  // device address of the fixed workspace of the allocation-free J-CoMM call
  // on this context's device (looked up once per device)
  char* noalloc_ws = nullptr;
};

extern thread_local std::string g_last_error;

inline int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(COMM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// Bump allocator over the context workspace (256-byte aligned pieces).
struct Carve {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

inline int ensure_ws(comm_ctx* ctx, size_t bytes, hipStream_t stream) {
  if (bytes <= ctx->ws_bytes) return COMM_OK;
  if (ctx->limit && bytes > ctx->limit)
    return fail(COMM_ENOMEM, "workspace of %zu bytes exceeds the context limit of %zu", bytes, ctx->limit);
  if (ctx->ws) {
    HIP_TRY(hipStreamSynchronize(ctx->last_stream));
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  size_t want = bytes + bytes / 4;
  if (ctx->limit && want > ctx->limit) want = ctx->limit;
  hipError_t e = hipMalloc(&ctx->ws, want);
  if (e != hipSuccess) return fail(COMM_ENOMEM, "hipMalloc(%zu): %s", want, hipGetErrorString(e));
  ctx->ws_bytes = want;
  return COMM_OK;
}

inline int beta_class_of(double beta) {
  if (beta == 0.0) return comm::kIS;
  if (beta == 0.5) return comm::kHalf;
  if (beta == 1.0) return comm::kKL;
  if (beta == 1.5) return comm::kThreeHalf;
  return comm::kGeneral;
}

inline comm::BetaConst make_beta_const(double beta) {
  comm::BetaConst bc = {};
  bc.beta = (float)beta;
  bc.inv_bb1 = (beta != 0.0 && beta != 1.0) ? (float)(1.0 / (beta * (beta - 1.0))) : 0.0f;
  bc.inv_beta = beta > 0.0 ? (float)(1.0 / beta) : 0.0f;
  // c_k = (beta^(k-1) - (beta-1)^(k-1)) / k!, k = 2..17
  double fact = 1.0;
  for (int k = 1; k <= 17; ++k) {
    fact *= k;
    if (k >= 2) bc.series[k - 2] = (float)((std::pow(beta, k - 1) - std::pow(beta - 1.0, k - 1)) / fact);
  }
  return bc;
}

inline float gamma_of(double beta) { return beta < 1.0 ? (float)(1.0 / (2.0 - beta)) : 1.0f; }


// Event pairs created when profiling is enabled.
constexpr size_t kProfileEvents = 2048;

// Run `launch()` and, when profiling is on, count it and time the pass kernel
// it launches if it is a sampled one (used for every kernel that streams the
// dense tensor).  On an ordinary
// stream the kernel's own dispatch stamps a pair of events (launch_timed);
// the pair is returned to the pool when nothing consumed it (the launch was
// recorded for a grouped batch).  While the stream is being captured into a
// graph the pair is recorded around the launch instead.
template <class F>
int profiled(comm_ctx* ctx, hipStream_t st, F&& launch) {
  if (!ctx->profiling || comm::recorder() || ctx->profile_seen++ % ctx->profile_every != 0) {
    HIP_TRY(launch());
    return COMM_OK;
  }
  if (ctx->events_used == ctx->events.size()) {
    hipEvent_t a0, a1;
    HIP_TRY(hipEventCreate(&a0));
    HIP_TRY(hipEventCreate(&a1));
    ctx->events.emplace_back(a0, a1);
  }
  const hipEvent_t e0 = ctx->events[ctx->events_used].first;
  const hipEvent_t e1 = ctx->events[ctx->events_used].second;
  ++ctx->events_used;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) {
    HIP_TRY(hipEventRecord(e0, st));
    HIP_TRY(launch());
    HIP_TRY(hipEventRecord(e1, st));
    return COMM_OK;
  }
  comm::g_timed = comm::TimedLaunch{e0, e1};
  const hipError_t e = launch();
  const bool unused = comm::g_timed.start != nullptr;
  comm::g_timed = comm::TimedLaunch{};
  if (unused) --ctx->events_used;
  HIP_TRY(e);
  return COMM_OK;
}

int check_opts(const comm_opts* o, bool need_L);
int check_dense(const comm_dense* x);
