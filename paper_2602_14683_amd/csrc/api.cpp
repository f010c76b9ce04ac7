// C ABI entry points: argument validation, workspace management and the
// orchestration of B-CoMM and J-CoMM out of the kernels in cp3.hip,
// tucker3.hip, sparse.hip and kernels_small.hip.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/comm.h"
#include "group.h"
#include "host_util.h"
#include "kernels.h"
#include "tucker3.h"
#include "sparse.h"

using namespace comm;

thread_local std::string g_last_error = "no error";

// Workspace of comm_jcomm_outer_noalloc: one fixed array on every GPU the
// library runs on, held until the process ends.  In host code the symbol
// names a host-side stand-in, never the device memory: its device address is
// looked up once per device (with that device current) when the first
// context on it is created, and only that address is used.
constexpr size_t kNoallocBytes = COMM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[kMaxDevices] = {};

int scratch_address(int device, char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(COMM_EINVAL, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    int prev = 0;
    HIP_TRY(hipGetDevice(&prev));
    HIP_TRY(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    HIP_TRY(hipSetDevice(prev));
    if (e != hipSuccess || !p)
      return fail(COMM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_addr[device] = static_cast<char*>(p);
  }
  *out = g_scratch_addr[device];
  return COMM_OK;
}

int check_opts(const comm_opts* o, bool need_L) {
  if (!o) return fail(COMM_EINVAL, "opts is NULL");
  if (!(o->beta >= 0.0 && o->beta < 2.0)) return fail(COMM_EINVAL, "beta = %g outside [0, 2)", o->beta);
  if (!(o->eps > 0.0)) return fail(COMM_EINVAL, "eps must be > 0");
  if (o->beta == 0.0 && !(o->eps_x > 0.0)) return fail(COMM_EINVAL, "eps_x must be > 0 at beta = 0");
  if (need_L && o->inner_sweeps < 1) return fail(COMM_EINVAL, "inner_sweeps must be >= 1");
  if (o->precision != COMM_FP32 && o->precision != COMM_BF16)
    return fail(COMM_EINVAL, "precision %d is neither COMM_FP32 nor COMM_BF16", o->precision);
  if (o->cache_pq != 0 && o->cache_pq != 1 && o->cache_pq != COMM_CACHE_AUTO)
    return fail(COMM_EINVAL, "cache_pq %d is not 0, 1 or COMM_CACHE_AUTO", o->cache_pq);
  return COMM_OK;
}

// Shape of a dense tensor only (the size query needs no buffers).
int check_dense_shape(const comm_dense* x) {
  if (!x) return fail(COMM_EINVAL, "x is NULL");
  if (x->ndim < 1 || x->ndim > COMM_MAX_NDIM) return fail(COMM_EINVAL, "ndim = %d", x->ndim);
  for (int n = 0; n < x->ndim; ++n)
    if (x->dims[n] < 1 || x->dims[n] > (1 << 24)) return fail(COMM_EINVAL, "dims[%d] = %lld", n, (long long)x->dims[n]);
  if (x->ndim < 3) return fail(COMM_EUNSUPPORTED, "dense tensors of order %d are not supported (3 to 5)", x->ndim);
  if (x->ndim > 3) {
    // the first N - 2 modes form one mode of the 3-way view
    int64_t rows = 1;
    for (int n = 0; n < x->ndim - 2; ++n) rows *= x->dims[n];
    if (rows > (1 << 24))
      return fail(COMM_EUNSUPPORTED, "I_1 ... I_%d = %lld exceeds 2^24", x->ndim - 2, (long long)rows);
  }
  return COMM_OK;
}

int check_dense(const comm_dense* x) {
  int rc = check_dense_shape(x);
  if (rc) return rc;
  if (!x->X) return fail(COMM_EINVAL, "x->X is NULL");
  return COMM_OK;
}


namespace {

int check_cp_model(const comm_model* m, int ndim) {
  if (!m) return fail(COMM_EINVAL, "model is NULL");
  if (m->kind != COMM_CP) return fail(COMM_EINVAL, "model kind is not CP");
  if (m->rank < 1) return fail(COMM_EINVAL, "rank = %d", m->rank);
  if (m->rank > kRP) return fail(COMM_EUNSUPPORTED, "rank %d > %d not supported", m->rank, kRP);
  for (int n = 0; n < ndim; ++n)
    if (!m->factors[n]) return fail(COMM_EINVAL, "factors[%d] is NULL", n);
  return COMM_OK;
}

// ---------------------------------------------------------------------------------------- CP dense

// Padded workspace copies of three factors, [rows_p][32].
struct FactorSet {
  float* pad[3];
};

struct CpWs {
  CpGrid g;
  int dims[3], rows_p[3];
  FactorSet ref, cur, num, den;
  float *m3n, *m1n, *m2n, *m3d, *m1d, *m2d;
  double* obj_part;
  float* c[3];
  float* stats[3];
  float* dprod;
  float *Pc, *Qc;
  float *Vn, *Vd;    // J-CoMM at beta != 1: V kept by the mode-1 pass for mode 2
  float *f2n, *f2d;  // ... and mode 2's numerator / denominator chunks folded from it
  int r16;           // the passes run the 16-wide tiles (cp_narrow)
  size_t bytes;
};

// 16-wide pass tiles: rank <= 16 with float32 tiles, unless the autotune
// table chose the 32-wide ones.
bool cp_narrow(int rank, const comm_opts* o, const TuneChoice& pick) {
  return rank <= 16 && o->precision != COMM_BF16 && pick.cp_tile != 32;
}

bool cp_wshare(const comm_opts* o, const TuneChoice& pick) {
  if (o->beta == 1.0) return false;
  return pick.wshare >= 0 ? pick.wshare != 0 : o->precision != COMM_BF16;
}

CpWs cp_layout(const comm_dense* x, char* base, bool cache, bool vkeep = false) {
  CpWs w = {};
  for (int n = 0; n < 3; ++n) w.dims[n] = (int)x->dims[n];
  w.g = cp_grid(w.dims[0], w.dims[1], w.dims[2]);
  w.rows_p[0] = w.g.Ip;
  w.rows_p[1] = w.g.Jp;
  w.rows_p[2] = w.g.Kp;
  Carve cv;
  cv.base = base;
  for (FactorSet* s : {&w.ref, &w.cur, &w.num, &w.den})
    for (int n = 0; n < 3; ++n) s->pad[n] = cv.take<float>((size_t)w.rows_p[n] * kRP);
  const CpGrid& g = w.g;
  w.m3n = cv.take<float>((size_t)g.m3_slots() * g.Kp * kRP);
  w.m1n = cv.take<float>((size_t)g.m1_slots() * g.Ip * kRP);
  w.m2n = cv.take<float>((size_t)g.m2_slots() * g.Jp * kRP);
  w.m3d = cv.take<float>((size_t)g.m3_slots() * g.Kp * kRP);
  w.m1d = cv.take<float>((size_t)g.m1_slots() * g.Ip * kRP);
  w.m2d = cv.take<float>((size_t)g.m2_slots() * g.Jp * kRP);
  w.obj_part = cv.take<double>((size_t)std::max<int64_t>(g.wgs(), vkeep ? cp_vpass_wgs(w.dims[0], w.dims[1]) : 0));
  for (int n = 0; n < 3; ++n) {
    w.c[n] = cv.take<float>((size_t)w.rows_p[n] * kRP);
    w.stats[n] = cv.take<float>((size_t)((w.rows_p[n] + kSlotRows - 1) / kSlotRows) * 96);
  }
  w.dprod = cv.take<float>(kRP);
  if (cache) {
    const size_t total = (size_t)w.dims[0] * w.dims[1] * w.dims[2];
    w.Pc = cv.take<float>(total);
    w.Qc = cv.take<float>(total);
  }
  if (vkeep) {
    const size_t pairs = (size_t)w.dims[0] * w.dims[1];
    w.Vn = cv.take<float>(pairs * kRP);
    w.Vd = cv.take<float>(pairs * kRP);
    w.f2n = cv.take<float>((size_t)kVFoldChunks * g.Jp * kRP);
    w.f2d = cv.take<float>((size_t)kVFoldChunks * g.Jp * kRP);
  }
  w.bytes = cv.off + 256;
  return w;
}

int run_pass(comm_ctx* ctx, const CpPassArgs& a, const CpGrid& g, int bc, bool den, hipStream_t st) {
  // without X the pass must take x = 0 itself: every class but beta = 1
  // does, unless it reads the P~ / Q~ cache instead (which needs no X)
  if (!a.X && a.cache_mode != 2 && (!a.x_zero || bc == kKL))
    return fail(COMM_EHIP, "internal error: a pass without X at beta class %d", bc);
  return profiled(ctx, st, [&] { return launch_cp_pass(a, g, bc, den, st); });
}

FView user_view(const comm_model* m, int n) { return FView{m->factors[n], m->rank, m->rank}; }
FView pad_view(const float* p) { return FView{p, kRP, kRP}; }
FSet user_set(const comm_model* m) { return FSet{user_view(m, 0), user_view(m, 1), user_view(m, 2)}; }
FSet pad_set(const FactorSet& s) { return FSet{pad_view(s.pad[0]), pad_view(s.pad[1]), pad_view(s.pad[2])}; }

CpPassArgs base_pass(const comm_dense* x, const CpWs& w, const comm_opts* o) {
  CpPassArgs a = {};
  a.X = x->X;
  a.x_zero = x->X == nullptr;  // the dense twin of sparse data at beta != 1
  a.I = w.dims[0];
  a.J = w.dims[1];
  a.K = w.dims[2];
  a.Ip = w.g.Ip;
  a.Jp = w.g.Jp;
  a.Kp = w.g.Kp;
  a.eps = (float)o->eps;
  a.eps_x = (float)o->eps_x;
  a.bc = make_beta_const(o->beta);
  a.m3n = w.m3n; a.m1n = w.m1n; a.m2n = w.m2n;
  a.m3d = w.m3d; a.m1d = w.m1d; a.m2d = w.m2d;
  a.obj_part = w.obj_part;
  a.bf16 = o->precision == COMM_BF16;
  a.xbuf = 16.0 * a.J * a.K + 32.0 * a.K < 2147483648.0;
  a.r16 = w.r16;
  return a;
}

// Numerator of block n taken from elsewhere (the nonzeros of a sparse
// tensor): called with the contraction views of all N blocks (entry n is not
// read) at the point where the dense path would take its numerator slots;
// returns a [rows][32] buffer, one slot.
struct NumHook {
  std::function<int(int n, const FView* ct, const float** num)> run;
};

// Partial-slot view of mode n.
void slots_of(const CpWs& w, int n, bool den, const float** part, int* slots, int* rows_total) {
  const CpGrid& g = w.g;
  if (n == 0) { *part = den ? w.m1d : w.m1n; *slots = g.m1_slots(); *rows_total = g.Ip; }
  else if (n == 1) { *part = den ? w.m2d : w.m2n; *slots = g.m2_slots(); *rows_total = g.Jp; }
  else { *part = den ? w.m3d : w.m3n; *slots = g.m3_slots(); *rows_total = g.Kp; }
}

// Block update of mode n from the partial slots just written by a pass:
// max(anchor * (Num/Den)^gamma, eps), written to the caller's factor and, if
// given, to a padded copy.  Den is either its own slots or, at beta = 1, the
// product of the column sums of the other two factors (views `others`).
int cp_apply_update(const comm_model* m, const CpWs& w, int n, FView anchor, const FView* closed_others,
                    float* out_pad, float gamma, float eps, hipStream_t st, const float* num_override = nullptr) {
  SlotUpdateArgs u = {};
  u.njobs = 1;
  SlotJob& J = u.job[0];
  J.mode = kSlotUpdate;
  slots_of(w, n, false, &J.num_part, &J.num_slots, &J.rows_total);
  if (num_override) {
    J.num_part = num_override;
    J.num_slots = 1;
  }
  if (closed_others) {
    int rows[2], k = 0;
    for (int q = 0; q < 3; ++q)
      if (q != n) rows[k++] = w.dims[q];
    HIP_TRY(launch_colsum_prod(closed_others, rows, 2, w.dprod, st));
    J.den_closed = w.dprod;
  } else {
    int rt;
    slots_of(w, n, true, &J.den_part, &J.den_slots, &rt);
  }
  J.rows = w.dims[n];
  J.cols = m->rank;
  J.rows_p = w.rows_p[n];
  J.anchor = anchor;
  J.gamma = gamma;
  J.eps = eps;
  J.out_pad = out_pad;
  J.out_user = m->factors[n];
  J.ld_user = m->rank;
  HIP_TRY(launch_slot_update(u, st));
  return COMM_OK;
}

int cp3_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st,
              const NumHook* hook = nullptr) {
  CpWs w = cp_layout(x, nullptr, false);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = cp_layout(x, ctx->ws, false);
  w.r16 = cp_narrow(m->rank, o, ctx->pick);
  const bool kl = o->beta == 1.0;
  const int bc = beta_class_of(o->beta);
  const int first = block < 0 ? 0 : block, last = block < 0 ? 2 : block;
  const FSet cur = user_set(m);  // the caller's factors are the current blocks
  for (int n = first; n <= last; ++n) {
    CpPassArgs a = base_pass(x, w, o);
    a.r = cur;
    a.n = cur;
    a.d = cur;
    a.want_v = n < 2;
    a.want_m3 = n == 2;
    // with a hook at beta = 1 the pass would only give the numerator
    if (!(hook && kl) && (rc = run_pass(ctx, a, w.g, bc, !kl, st))) return rc;
    const float* nb = nullptr;
    if (hook) {
      const FView ct[3] = {cur.A, cur.B, cur.C};
      if ((rc = hook->run(n, ct, &nb))) return rc;
    }
    FView others[2];
    int k = 0;
    for (int q = 0; q < 3; ++q)
      if (q != n) others[k++] = user_view(m, q);
    rc = cp_apply_update(m, w, n, user_view(m, n), kl ? others : nullptr, nullptr, gamma_of(o->beta),
                         (float)o->eps, st, nb);
    if (rc) return rc;
  }
  return COMM_OK;
}

int cp3_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st,
              const NumHook* hook = nullptr) {
  const bool kl = o->beta == 1.0;
  const bool cache = !kl && o->cache_pq;
  // the mode-1 pass keeps V for mode 2 (by default with float32 tiles; see
  // own_pass below), unless the autotune table chose otherwise
  const bool vkeep = cp_wshare(o, ctx->pick);
  CpWs w = cp_layout(x, nullptr, cache, vkeep);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = cp_layout(x, ctx->ws, cache, vkeep);
  w.r16 = cp_narrow(m->rank, o, ctx->pick);
  const int bc = beta_class_of(o->beta);
  const float eps = (float)o->eps;

  if (kl) {
    // Reference pass straight from the caller's factors: Xhat~, P~ = X / Xhat~,
    // all three numerators against chi_1 = A~, and the objective at the
    // reference.  Then c^(n) = A~^(n) Num_J^(n) with column statistics, and the
    // inner sweeps, which overwrite the caller's factors last.
    CpPassArgs a = base_pass(x, w, o);
    a.r = user_set(m);
    a.n = a.r;
    a.want_v = 1;
    a.want_m3 = 1;
    a.want_obj = obj != nullptr;
    if ((rc = run_pass(ctx, a, w.g, bc, false, st))) return rc;
    SlotUpdateArgs su = {};
    su.njobs = 3;
    KlLoopArgs k = {};
    k.N = 3;
    k.R = m->rank;
    k.L = o->inner_sweeps;
    k.eps = eps;
    for (int n = 0; n < 3; ++n) {
      SlotJob& J = su.job[n];
      J.mode = kSlotScale;
      slots_of(w, n, false, &J.num_part, &J.num_slots, &J.rows_total);
      J.rows = w.dims[n];
      J.cols = m->rank;
      J.rows_p = w.rows_p[n];
      J.anchor = user_view(m, n);
      J.out_pad = w.c[n];
      J.stats = w.stats[n];
      k.c[n] = w.c[n];
      k.stats[n] = w.stats[n];
      k.nblk[n] = (w.rows_p[n] + kSlotRows - 1) / kSlotRows;
      k.rows[n] = w.dims[n];
      k.cur_pad[n] = nullptr;
      k.user[n] = m->factors[n];
    }
    if (obj) {
      k.obj_part = w.obj_part;
      k.obj_n = w.g.wgs();
      k.obj_out = obj;
    }
    HIP_TRY(launch_slot_update(su, st));
    HIP_TRY(launch_kl_apply(k, st));
    return COMM_OK;
  }

  // beta != 1: padded copies of the reference (kept fixed) and of the current
  // inner iterate (starts at the reference).
  {
    PadArgs p = {};
    p.nf = 3;
    for (int n = 0; n < 3; ++n) {
      p.cols[n] = m->rank;
      p.ld[n] = m->rank;
      p.src[n] = m->factors[n];
      p.rows[n] = w.dims[n];
      p.rows_p[n] = w.rows_p[n];
      p.dst[n] = w.ref.pad[n];
      p.dst2[n] = w.cur.pad[n];
    }
    HIP_TRY(launch_pad_factors(p, st));
  }
  const FSet ref = pad_set(w.ref);
  bool obj_pending = obj != nullptr;
  if (cache) {
    CpPassArgs a = base_pass(x, w, o);
    a.r = ref;
    a.n = ref;
    a.cache_mode = 1;
    a.Pw = w.Pc;
    a.Qw = w.Qc;
    a.want_obj = obj_pending;
    if ((rc = run_pass(ctx, a, w.g, bc, false, st))) return rc;
    if (obj_pending) HIP_TRY(launch_sum_f64(w.obj_part, w.g.wgs(), nullptr, obj, st));
    obj_pending = false;
  }
  // Per sweep (Sec. 5.3, CP inner updates in the order of modes 1, 2, 3):
  // mode 1 from the V pass, which keeps V = P~ x3 C' (numerator and
  // denominator sets) since C does not change before mode 3; mode 2 folds V
  // with the new mode-1 transforms; mode 3 from a pass of its own.
  auto chi_of = [&](std::initializer_list<int> modes) -> int {
    ChiArgs ca = {};
    ca.beta = (float)o->beta;
    for (int q : modes) {
      const int f = ca.nf++;
      ca.cur[f] = w.cur.pad[q];
      ca.ref[f] = w.ref.pad[q];
      ca.rows_p[f] = w.rows_p[q];
      ca.x1[f] = w.num.pad[q];
      ca.x2[f] = w.den.pad[q];
    }
    HIP_TRY(launch_chi(ca, st));
    return COMM_OK;
  };
  // block update of mode n from explicit slots (num_override: the hook's one slot)
  auto apply = [&](int n, const float* np, int ns, const float* dp, int ds, int rows_total,
                   const float* num_override) -> int {
    SlotUpdateArgs u = {};
    u.njobs = 1;
    SlotJob& J = u.job[0];
    J.mode = kSlotUpdate;
    J.num_part = num_override ? num_override : np;
    J.num_slots = num_override ? 1 : ns;
    J.den_part = dp;
    J.den_slots = ds;
    J.rows_total = rows_total;
    J.rows = w.dims[n];
    J.cols = m->rank;
    J.rows_p = w.rows_p[n];
    J.anchor = n == 0 ? ref.A : n == 1 ? ref.B : ref.C;  // anchored at the reference block
    J.gamma = gamma_of(o->beta);
    J.eps = eps;
    J.out_pad = w.cur.pad[n];
    J.out_user = m->factors[n];
    J.ld_user = m->rank;
    // the new block's transforms for the blocks after it (chi_kernel's values)
    J.chi_ref = w.ref.pad[n];
    J.chi_x1 = w.num.pad[n];
    J.chi_x2 = w.den.pad[n];
    J.chi_beta = (float)o->beta;
    HIP_TRY(launch_slot_update(u, st));
    return COMM_OK;
  };
  const FView numv[3] = {pad_view(w.num.pad[0]), pad_view(w.num.pad[1]), pad_view(w.num.pad[2])};
  // modes 1 and 2 through their own passes (the V pass with the fold measured
  // slower with bf16 tiles, where the contractions are cheap and the V pass's
  // per-slice operand loads are not)
  auto own_pass = [&](int n) -> int {
    CpPassArgs a = base_pass(x, w, o);
    a.r = ref;
    a.n = pad_set(w.num);
    a.d = pad_set(w.den);
    if (n == 0) { a.n.A = ref.A; a.d.A = ref.A; }
    if (n == 1) { a.n.B = ref.B; a.d.B = ref.B; }
    a.want_v = 1;
    if (cache) {
      a.cache_mode = 2;
      a.Pc = w.Pc;
      a.Qc = w.Qc;
    } else {
      a.want_obj = obj_pending;
    }
    int rc2 = run_pass(ctx, a, w.g, bc, true, st);
    if (rc2) return rc2;
    if (a.want_obj) {
      HIP_TRY(launch_sum_f64(w.obj_part, w.g.wgs(), nullptr, obj, st));
      obj_pending = false;
    }
    const float* nb = nullptr;
    if (hook && (rc2 = hook->run(n, numv, &nb))) return rc2;
    const float *np, *dp;
    int ns, ds, rt;
    slots_of(w, n, false, &np, &ns, &rt);
    slots_of(w, n, true, &dp, &ds, &rt);
    return apply(n, np, ns, dp, ds, rt, nb);
  };
  const bool wshare = vkeep;
  // every block update writes the block's transforms with it, so after the
  // first sweep's start they are always current
  if ((rc = chi_of({1, 2}))) return rc;
  for (int l = 0; l < o->inner_sweeps; ++l) {
    if (!wshare) {
      if ((rc = own_pass(0))) return rc;
      if ((rc = own_pass(1))) return rc;
    }
    // mode 1: the V pass against the sets of modes 2 and 3
    if (wshare) {
      CpPassArgs a = base_pass(x, w, o);
      a.r = ref;
      a.n = pad_set(w.num);
      a.d = pad_set(w.den);
      a.n.A = ref.A;  // the active block does not enter its own contraction
      a.d.A = ref.A;
      a.Vn = w.Vn;
      a.Vd = w.Vd;
      if (cache) {
        a.cache_mode = 2;
        a.Pc = w.Pc;
        a.Qc = w.Qc;
      } else {
        a.want_obj = obj_pending;
      }
      if ((rc = profiled(ctx, st, [&] { return launch_cp_vpass(a, bc, st); }))) return rc;
      if (a.want_obj) {
        HIP_TRY(launch_sum_f64(w.obj_part, cp_vpass_wgs(w.dims[0], w.dims[1]), nullptr, obj, st));
        obj_pending = false;
      }
      const float* nb = nullptr;
      if (hook && (rc = hook->run(0, numv, &nb))) return rc;
      const int slots = cp_vpass_m1_slots(w.dims[1]);
      if ((rc = apply(0, w.m1n, slots, w.m1d, slots, w.g.Ip, nb))) return rc;
    }
    // mode 2: fold the kept V with the new mode-1 transforms
    if (wshare) {
      VFoldArgs f = {};
      f.I = w.dims[0];
      f.J = w.dims[1];
      f.Jp = w.g.Jp;
      f.Vn = w.Vn;
      f.Vd = w.Vd;
      f.An = pad_view(w.num.pad[0]);
      f.Ad = pad_view(w.den.pad[0]);
      f.outn = w.f2n;
      f.outd = w.f2d;
      HIP_TRY(launch_vfold(f, st));
      const float* nb = nullptr;
      if (hook && (rc = hook->run(1, numv, &nb))) return rc;
      if ((rc = apply(1, w.f2n, kVFoldChunks, w.f2d, kVFoldChunks, w.g.Jp, nb))) return rc;
    }
    // mode 3: its own pass against the sets of modes 1 and 2
    {
      CpPassArgs a = base_pass(x, w, o);
      a.r = ref;
      a.n = pad_set(w.num);
      a.d = pad_set(w.den);
      a.n.C = ref.C;
      a.d.C = ref.C;
      a.want_m3 = 1;
      if (cache) {
        a.cache_mode = 2;
        a.Pc = w.Pc;
        a.Qc = w.Qc;
      }
      if ((rc = run_pass(ctx, a, w.g, bc, true, st))) return rc;
      const float* nb = nullptr;
      if (hook && (rc = hook->run(2, numv, &nb))) return rc;
      const float *np, *dp;
      int ns, ds, rt;
      slots_of(w, 2, false, &np, &ns, &rt);
      slots_of(w, 2, true, &dp, &ds, &rt);
      if ((rc = apply(2, np, ns, dp, ds, rt, nb))) return rc;
    }
  }
  return COMM_OK;
}

int cp3_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                 hipStream_t st) {
  CpWs w = cp_layout(x, nullptr, false);
  int rc = ensure_ws(ctx, w.bytes, st);
  if (rc) return rc;
  w = cp_layout(x, ctx->ws, false);
  w.r16 = cp_narrow(m->rank, o, ctx->pick);
  CpPassArgs a = base_pass(x, w, o);
  a.r = user_set(m);
  a.n = a.r;
  a.want_obj = 1;
  if ((rc = run_pass(ctx, a, w.g, beta_class_of(o->beta), false, st))) return rc;
  HIP_TRY(launch_sum_f64(w.obj_part, w.g.wgs(), nullptr, out, st));
  return COMM_OK;
}

// ---------------------------------------------------------------------------------------- CP dense, order 4 and 5

// The caller's order-N tensor (N = 4, 5) as the 3-way tensor
// (I_1 ... I_G) x I_{N-1} x I_N, G = N - 2, without a copy: mode 0 of the view
// is the super mode with factor KR(A^(1), ..., A^(G)) (KrArgs); view modes 1
// and 2 are caller modes N-2 and N-1 (0-based).
constexpr int kGrpPad = 16;

struct CpnWs {
  int N, G;
  int dims[kMaxModes];
  int grp_p[kMaxGroup];      // padded rows of the grouped modes
  comm_dense xv;             // the 3-way view
  CpWs w;                    // its workspace; w.ref.pad[0] etc. hold super factors
  float* gref[kMaxGroup];    // beta != 1 J-CoMM: padded reference grouped blocks,
  float* gcur[kMaxGroup];    //   the current inner iterate,
  float* gx1[kMaxGroup];     //   and chi_1 / chi_2 of it
  float* gx2[kMaxGroup];
  float* fnum[kMaxGroup];    // folded numerators / denominators [grp_p][32]
  float* fden[kMaxGroup];
  float* gc[kMaxGroup];      // beta = 1 J-CoMM: c = A~ * Num_J and its column statistics
  float* gstats[kMaxGroup];
  size_t bytes;
};

CpnWs cpn_layout(const comm_dense* x, char* base, bool cache) {
  CpnWs v = {};
  v.N = x->ndim;
  v.G = v.N - 2;
  int64_t rows = 1;
  for (int n = 0; n < v.N; ++n) v.dims[n] = (int)x->dims[n];
  for (int m = 0; m < v.G; ++m) {
    v.grp_p[m] = (v.dims[m] + kGrpPad - 1) / kGrpPad * kGrpPad;
    rows *= x->dims[m];
  }
  v.xv.ndim = 3;
  v.xv.dims[0] = rows;
  v.xv.dims[1] = x->dims[v.N - 2];
  v.xv.dims[2] = x->dims[v.N - 1];
  v.xv.X = x->X;
  v.w = cp_layout(&v.xv, base, cache);
  Carve cv;
  cv.base = base;
  cv.off = v.w.bytes;
  for (int m = 0; m < v.G; ++m) {
    const size_t n = (size_t)v.grp_p[m] * kRP;
    for (float** p : {&v.gref[m], &v.gcur[m], &v.gx1[m], &v.gx2[m], &v.fnum[m], &v.fden[m], &v.gc[m]})
      *p = cv.take<float>(n);
    v.gstats[m] = cv.take<float>((size_t)((v.grp_p[m] + kSlotRows - 1) / kSlotRows) * 96);
  }
  v.bytes = cv.off + 256;
  return v;
}

size_t cp_ws_bytes(const comm_dense* x, bool cache, bool vkeep = false) {
  return x->ndim == 3 ? cp_layout(x, nullptr, cache, vkeep).bytes : cpn_layout(x, nullptr, cache).bytes;
}

// Super factor(s) of the view from G grouped views each: out0 = KR(src0), and
// out1 = KR(src1) if src1 is given.
int cpn_kr(const CpnWs& v, const FView* src0, float* out0, const FView* src1, float* out1, hipStream_t st) {
  KrArgs k = {};
  k.G = v.G;
  for (int m = 0; m < v.G; ++m) {
    k.dims[m] = v.dims[m];
    k.f[0][m] = src0[m];
    if (src1) k.f[1][m] = src1[m];
  }
  k.rows = (int)v.xv.dims[0];
  k.rows_p = v.w.rows_p[0];
  k.nout = src1 ? 2 : 1;
  k.out[0] = out0;
  k.out[1] = out1;
  HIP_TRY(launch_kr(k, st));
  return COMM_OK;
}

// Numerators (weights wn) and, with wd, denominators (weights wd) of the
// grouped modes in `modes` from the super mode's partial slots of the last pass.
int cpn_fold(const CpnWs& v, const int* modes, int count, const FView* wn, const FView* wd, hipStream_t st) {
  FoldArgs f = {};
  f.G = v.G;
  for (int m = 0; m < v.G; ++m) f.dims[m] = v.dims[m];
  auto job = [&](int n, const float* part, const FView* wts, float* out) {
    FoldJob& J = f.job[f.njobs++];
    J.mode = n;
    J.part = part;
    J.slots = v.w.g.m1_slots();
    J.rows_total = v.w.g.Ip;
    for (int m = 0; m < v.G; ++m) J.w[m] = wts[m];
    J.out = out;
    J.rows_p = v.grp_p[n];
  };
  for (int q = 0; q < count; ++q) {
    job(modes[q], v.w.m1n, wn, v.fnum[modes[q]]);
    if (wd) job(modes[q], v.w.m1d, wd, v.fden[modes[q]]);
  }
  HIP_TRY(launch_fold(f, st));
  return COMM_OK;
}

// Numerator source of caller mode n: folded buffer (grouped) or the view's slots.
void cpn_num_src(const CpnWs& v, int n, bool den, const float** part, int* slots, int* rows_total, int* rows_p) {
  if (n < v.G) {
    *part = den ? v.fden[n] : v.fnum[n];
    *slots = 1;
    *rows_total = v.grp_p[n];
    *rows_p = v.grp_p[n];
  } else {
    const int q = n - v.G + 1;
    slots_of(v.w, q, den, part, slots, rows_total);
    *rows_p = v.w.rows_p[q];
  }
}

// Block update of caller mode n: max(anchor * (Num/Den)^gamma, eps), into the
// caller's factor and, if given, a padded copy.  With `closed` (beta = 1) Den
// is the product of the column sums of the other N - 1 blocks `cur`.
int cpn_apply(const CpnWs& v, comm_model* m, int n, const FView* closed, FView anchor, float* out_pad, float gamma,
              float eps, hipStream_t st, const float* num_override = nullptr) {
  SlotUpdateArgs u = {};
  u.njobs = 1;
  SlotJob& J = u.job[0];
  J.mode = kSlotUpdate;
  cpn_num_src(v, n, false, &J.num_part, &J.num_slots, &J.rows_total, &J.rows_p);
  if (num_override) {
    J.num_part = num_override;
    J.num_slots = 1;
  }
  if (closed) {
    FView others[kMaxModes];
    int rows[kMaxModes], k = 0;
    for (int q = 0; q < v.N; ++q)
      if (q != n) {
        others[k] = closed[q];
        rows[k++] = v.dims[q];
      }
    HIP_TRY(launch_colsum_prod(others, rows, k, v.w.dprod, st));
    J.den_closed = v.w.dprod;
  } else {
    int rt, rp;
    cpn_num_src(v, n, true, &J.den_part, &J.den_slots, &rt, &rp);
  }
  J.rows = v.dims[n];
  J.cols = m->rank;
  J.anchor = anchor;
  J.gamma = gamma;
  J.eps = eps;
  J.out_pad = out_pad;
  J.out_user = m->factors[n];
  J.ld_user = m->rank;
  HIP_TRY(launch_slot_update(u, st));
  return COMM_OK;
}

int cpn_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                  hipStream_t st) {
  CpnWs v = cpn_layout(x, nullptr, false);
  int rc = ensure_ws(ctx, v.bytes, st);
  if (rc) return rc;
  v = cpn_layout(x, ctx->ws, false);
  v.w.r16 = cp_narrow(m->rank, o, ctx->pick);
  FView user[kMaxModes];
  for (int n = 0; n < v.N; ++n) user[n] = user_view(m, n);
  if ((rc = cpn_kr(v, user, v.w.ref.pad[0], nullptr, nullptr, st))) return rc;
  CpPassArgs a = base_pass(&v.xv, v.w, o);
  a.r = FSet{pad_view(v.w.ref.pad[0]), user[v.N - 2], user[v.N - 1]};
  a.n = a.r;
  a.want_obj = 1;
  if ((rc = run_pass(ctx, a, v.w.g, beta_class_of(o->beta), false, st))) return rc;
  HIP_TRY(launch_sum_f64(v.w.obj_part, v.w.g.wgs(), nullptr, out, st));
  return COMM_OK;
}

// B-CoMM: every block sees the blocks updated before it, so each block has its
// own pass over X, from the super factor of the current grouped blocks.
int cpn_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st,
              const NumHook* hook = nullptr) {
  CpnWs v = cpn_layout(x, nullptr, false);
  int rc = ensure_ws(ctx, v.bytes, st);
  if (rc) return rc;
  v = cpn_layout(x, ctx->ws, false);
  v.w.r16 = cp_narrow(m->rank, o, ctx->pick);
  const bool kl = o->beta == 1.0;
  const int bc = beta_class_of(o->beta);
  const int first = block < 0 ? 0 : block, last = block < 0 ? v.N - 1 : block;
  FView cur[kMaxModes];
  for (int n = 0; n < v.N; ++n) cur[n] = user_view(m, n);
  bool super_valid = false;
  for (int n = first; n <= last; ++n) {
    if (!super_valid && (rc = cpn_kr(v, cur, v.w.ref.pad[0], nullptr, nullptr, st))) return rc;
    super_valid = true;
    const int q = n < v.G ? 0 : n - v.G + 1;
    CpPassArgs a = base_pass(&v.xv, v.w, o);
    a.r = FSet{pad_view(v.w.ref.pad[0]), cur[v.N - 2], cur[v.N - 1]};
    a.n = a.r;
    a.d = a.r;
    a.want_v = q < 2;
    a.want_m3 = q == 2;
    // with a hook at beta = 1 the pass would only give the numerator
    if (!(hook && kl)) {
      if ((rc = run_pass(ctx, a, v.w.g, bc, !kl, st))) return rc;
      if (n < v.G && (rc = cpn_fold(v, &n, 1, cur, kl ? nullptr : cur, st))) return rc;
    }
    const float* nb = nullptr;
    if (hook && (rc = hook->run(n, cur, &nb))) return rc;
    if ((rc = cpn_apply(v, m, n, kl ? cur : nullptr, cur[n], nullptr, gamma_of(o->beta), (float)o->eps, st, nb)))
      return rc;
    if (n < v.G) super_valid = false;  // a grouped block changed
  }
  return COMM_OK;
}

int cpn_chi(const CpnWs& v, float beta, const int* modes, int count, hipStream_t st) {
  ChiArgs ca = {};
  ca.beta = beta;
  for (int q = 0; q < count; ++q) {
    const int n = modes[q];
    const int f = ca.nf++;
    if (n < v.G) {
      ca.cur[f] = v.gcur[n];
      ca.ref[f] = v.gref[n];
      ca.rows_p[f] = v.grp_p[n];
      ca.x1[f] = v.gx1[n];
      ca.x2[f] = v.gx2[n];
    } else {
      const int p = n - v.G + 1;
      ca.cur[f] = v.w.cur.pad[p];
      ca.ref[f] = v.w.ref.pad[p];
      ca.rows_p[f] = v.w.rows_p[p];
      ca.x1[f] = v.w.num.pad[p];
      ca.x2[f] = v.w.den.pad[p];
    }
  }
  HIP_TRY(launch_chi(ca, st));
  return COMM_OK;
}

int cpn_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st,
              const NumHook* hook = nullptr) {
  const bool kl = o->beta == 1.0;
  const bool cache = !kl && o->cache_pq;
  CpnWs v = cpn_layout(x, nullptr, cache);
  int rc = ensure_ws(ctx, v.bytes, st);
  if (rc) return rc;
  v = cpn_layout(x, ctx->ws, cache);
  v.w.r16 = cp_narrow(m->rank, o, ctx->pick);
  const CpWs& w = v.w;
  const int N = v.N, G = v.G;
  const int bc = beta_class_of(o->beta);
  const float eps = (float)o->eps;

  if (kl) {
    // One reference pass gives the super mode's numerator and those of the
    // last two modes; the folds give the grouped modes'.  Then the closed-form
    // inner loop of the 3-way path, over all N blocks.
    FView ref[kMaxModes];
    for (int n = 0; n < N; ++n) ref[n] = user_view(m, n);
    if ((rc = cpn_kr(v, ref, w.ref.pad[0], nullptr, nullptr, st))) return rc;
    CpPassArgs a = base_pass(&v.xv, w, o);
    a.r = FSet{pad_view(w.ref.pad[0]), ref[N - 2], ref[N - 1]};
    a.n = a.r;
    a.want_v = 1;
    a.want_m3 = 1;
    a.want_obj = obj != nullptr;
    if ((rc = run_pass(ctx, a, w.g, bc, false, st))) return rc;
    int modes[kMaxGroup];
    for (int n = 0; n < G; ++n) modes[n] = n;
    if ((rc = cpn_fold(v, modes, G, ref, nullptr, st))) return rc;
    SlotUpdateArgs su = {};
    su.njobs = N;
    KlLoopArgs k = {};
    k.N = N;
    k.R = m->rank;
    k.L = o->inner_sweeps;
    k.eps = eps;
    for (int n = 0; n < N; ++n) {
      SlotJob& J = su.job[n];
      J.mode = kSlotScale;
      cpn_num_src(v, n, false, &J.num_part, &J.num_slots, &J.rows_total, &J.rows_p);
      J.rows = v.dims[n];
      J.cols = m->rank;
      J.anchor = ref[n];
      J.out_pad = n < G ? v.gc[n] : w.c[n - G + 1];
      J.stats = n < G ? v.gstats[n] : w.stats[n - G + 1];
      k.c[n] = J.out_pad;
      k.stats[n] = J.stats;
      k.nblk[n] = (J.rows_p + kSlotRows - 1) / kSlotRows;
      k.rows[n] = v.dims[n];
      k.user[n] = m->factors[n];
    }
    if (obj) {
      k.obj_part = w.obj_part;
      k.obj_n = w.g.wgs();
      k.obj_out = obj;
    }
    HIP_TRY(launch_slot_update(su, st));
    HIP_TRY(launch_kl_apply(k, st));
    return COMM_OK;
  }

  // beta != 1: padded reference and inner-iterate copies of every block; the
  // reference super factor from the reference grouped blocks.
  {
    PadArgs p = {};
    p.nf = N;
    for (int n = 0; n < N; ++n) {
      p.cols[n] = m->rank;
      p.ld[n] = m->rank;
      p.src[n] = m->factors[n];
      p.rows[n] = v.dims[n];
      if (n < G) {
        p.rows_p[n] = v.grp_p[n];
        p.dst[n] = v.gref[n];
        p.dst2[n] = v.gcur[n];
      } else {
        p.rows_p[n] = w.rows_p[n - G + 1];
        p.dst[n] = w.ref.pad[n - G + 1];
        p.dst2[n] = w.cur.pad[n - G + 1];
      }
    }
    HIP_TRY(launch_pad_factors(p, st));
  }
  FView gref[kMaxGroup], gx1[kMaxGroup], gx2[kMaxGroup];
  for (int n = 0; n < G; ++n) {
    gref[n] = pad_view(v.gref[n]);
    gx1[n] = pad_view(v.gx1[n]);
    gx2[n] = pad_view(v.gx2[n]);
  }
  if ((rc = cpn_kr(v, gref, w.ref.pad[0], nullptr, nullptr, st))) return rc;
  const FSet ref = pad_set(w.ref);
  bool obj_pending = obj != nullptr;
  if (cache) {
    CpPassArgs a = base_pass(&v.xv, w, o);
    a.r = ref;
    a.n = ref;
    a.cache_mode = 1;
    a.Pw = w.Pc;
    a.Qw = w.Qc;
    a.want_obj = obj_pending;
    if ((rc = run_pass(ctx, a, w.g, bc, false, st))) return rc;
    if (obj_pending) HIP_TRY(launch_sum_f64(w.obj_part, w.g.wgs(), nullptr, obj, st));
    obj_pending = false;
  }
  auto pass = [&](CpPassArgs& a) -> int {
    if (cache) {
      a.cache_mode = 2;
      a.Pc = w.Pc;
      a.Qc = w.Qc;
    } else {
      a.want_obj = obj_pending;
    }
    int r = run_pass(ctx, a, w.g, bc, true, st);
    if (r) return r;
    if (obj_pending) {
      HIP_TRY(launch_sum_f64(w.obj_part, w.g.wgs(), nullptr, obj, st));
      obj_pending = false;
    }
    return COMM_OK;
  };
  const int last2[2] = {N - 2, N - 1};
  for (int l = 0; l < o->inner_sweeps; ++l) {
    // grouped blocks: one pass contracts P~ and Q~ with chi of the last two
    // blocks (unchanged while the grouped blocks are updated), then a fold per block
    if ((rc = cpn_chi(v, (float)o->beta, last2, 2, st))) return rc;
    {
      CpPassArgs a = base_pass(&v.xv, w, o);
      a.r = ref;
      a.n = FSet{ref.A, pad_view(w.num.pad[1]), pad_view(w.num.pad[2])};
      a.d = FSet{ref.A, pad_view(w.den.pad[1]), pad_view(w.den.pad[2])};
      a.want_v = 1;
      if ((rc = pass(a))) return rc;
    }
    for (int n = 0; n < G; ++n) {
      int others[kMaxGroup], k = 0;
      for (int q = 0; q < G; ++q)
        if (q != n) others[k++] = q;
      if ((rc = cpn_chi(v, (float)o->beta, others, k, st))) return rc;
      if ((rc = cpn_fold(v, &n, 1, gx1, gx2, st))) return rc;
      const float* nb = nullptr;
      if (hook) {
        FView ct[kMaxModes];
        for (int q = 0; q < G; ++q) ct[q] = gx1[q];
        ct[N - 2] = pad_view(w.num.pad[1]);
        ct[N - 1] = pad_view(w.num.pad[2]);
        if ((rc = hook->run(n, ct, &nb))) return rc;
      }
      if ((rc = cpn_apply(v, m, n, nullptr, gref[n], v.gcur[n], gamma_of(o->beta), eps, st, nb))) return rc;
    }
    // the last two blocks: the super factors of chi_1 and chi_2 of the grouped blocks
    int all[kMaxGroup];
    for (int q = 0; q < G; ++q) all[q] = q;
    if ((rc = cpn_chi(v, (float)o->beta, all, G, st))) return rc;
    if ((rc = cpn_kr(v, gx1, w.num.pad[0], gx2, w.den.pad[0], st))) return rc;
    for (int q = 1; q <= 2; ++q) {
      if (q == 2 && (rc = cpn_chi(v, (float)o->beta, &last2[0], 1, st))) return rc;  // block N-2 just changed
      CpPassArgs a = base_pass(&v.xv, w, o);
      a.r = ref;
      a.n = pad_set(w.num);
      a.d = pad_set(w.den);
      if (q == 1) { a.n.B = ref.B; a.d.B = ref.B; }
      else { a.n.C = ref.C; a.d.C = ref.C; }
      a.want_v = q == 1;
      a.want_m3 = q == 2;
      if ((rc = pass(a))) return rc;
      const int n = G - 1 + q;
      const float* nb = nullptr;
      if (hook) {
        FView ct[kMaxModes];
        for (int g = 0; g < G; ++g) ct[g] = gx1[g];
        ct[N - 2] = pad_view(w.num.pad[1]);
        ct[N - 1] = pad_view(w.num.pad[2]);
        if ((rc = hook->run(n, ct, &nb))) return rc;
      }
      if ((rc = cpn_apply(v, m, n, nullptr, q == 1 ? ref.B : ref.C, w.cur.pad[q], gamma_of(o->beta), eps, st, nb)))
        return rc;
    }
  }
  return COMM_OK;
}

int cp_bcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, int block, const comm_opts* o, hipStream_t st,
             const NumHook* hook = nullptr) {
  return x->ndim == 3 ? cp3_bcomm(ctx, x, m, block, o, st, hook) : cpn_bcomm(ctx, x, m, block, o, st, hook);
}

int cp_jcomm(comm_ctx* ctx, const comm_dense* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st,
             const NumHook* hook = nullptr) {
  return x->ndim == 3 ? cp3_jcomm(ctx, x, m, o, obj, st, hook) : cpn_jcomm(ctx, x, m, o, obj, st, hook);
}

int cp_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o, double* out,
                 hipStream_t st) {
  return x->ndim == 3 ? cp3_objective(ctx, x, m, o, out, st) : cpn_objective(ctx, x, m, o, out, st);
}

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::exception& e) {
    return fail(COMM_EHIP, "internal error: %s", e.what());
  } catch (...) {
    return fail(COMM_EHIP, "internal error");
  }
}

int set_device(comm_ctx* ctx) {
  HIP_TRY(hipSetDevice(ctx->device));
  return COMM_OK;
}

// ---------------------------------------------------------------------------------------- extrapolation

// Blocks of a model in update order (Tucker: core first), with entry counts.
int model_blocks(const comm_dense* x, const comm_model* m, float** ptr, int64_t* count) {
  int nb = 0;
  if (m->kind == COMM_TUCKER) {
    ptr[nb] = m->core;
    int64_t entries = 1;
    for (int n = 0; n < x->ndim; ++n) entries *= m->core_dims[n];
    count[nb++] = entries;
  }
  for (int n = 0; n < x->ndim; ++n) {
    ptr[nb] = m->factors[n];
    count[nb++] = x->dims[n] * (m->kind == COMM_CP ? m->rank : m->core_dims[n]);
  }
  return nb;
}

int check_extrap(const comm_dense* x, const comm_model* m, const comm_model* prev, const comm_extrap* e) {
  if (!e) return fail(COMM_EINVAL, "extrap is NULL");
  if (!(e->alpha_nes >= 0.0 && std::isfinite(e->alpha_nes))) return fail(COMM_EINVAL, "alpha_nes = %g", e->alpha_nes);
  if (!(e->c > 0.0 && std::isfinite(e->c))) return fail(COMM_EINVAL, "c must be > 0");
  if (!(e->delta > 0.0 && std::isfinite(e->delta))) return fail(COMM_EINVAL, "delta must be > 0");
  if (!prev) return fail(COMM_EINVAL, "prev is NULL");
  if (prev->kind != m->kind) return fail(COMM_EINVAL, "prev is not the same kind of model");
  if (m->kind == COMM_CP && prev->rank != m->rank) return fail(COMM_EINVAL, "prev has rank %d, model %d", prev->rank,
                                                                m->rank);
  if (m->kind == COMM_TUCKER) {
    for (int n = 0; n < x->ndim; ++n)
      if (prev->core_dims[n] != m->core_dims[n]) return fail(COMM_EINVAL, "prev core_dims[%d] differs", n);
    if (!prev->core) return fail(COMM_EINVAL, "prev core is NULL");
    if (prev->core == m->core) return fail(COMM_EINVAL, "prev core aliases the model core");
  }
  for (int n = 0; n < x->ndim; ++n) {
    if (!prev->factors[n]) return fail(COMM_EINVAL, "prev factors[%d] is NULL", n);
    if (prev->factors[n] == m->factors[n]) return fail(COMM_EINVAL, "prev factors[%d] aliases the model", n);
  }
  return COMM_OK;
}

int ensure_aux(comm_ctx* ctx) {
  if (ctx->aux) return COMM_OK;
  HIP_TRY(hipMalloc(&ctx->aux, 256));
  return COMM_OK;
}

// opts->check_inputs: the data (nd values at data) finite and >= 0, every
// parameter of the model finite and >= eps; otherwise COMM_EINVAL before
// anything is updated.  The flag is the int 128 bytes into ctx->aux (the
// extrapolation weight uses its first float).  Synchronises the stream.
int input_check(comm_ctx* ctx, const float* data, int64_t nd, const comm_model* m, int ndim, const int64_t* dims,
                const comm_opts* o, hipStream_t st) {
  if (!o || !o->check_inputs) return COMM_OK;
  int rc = ensure_aux(ctx);
  if (rc) return rc;
  int* flag = reinterpret_cast<int*>(ctx->aux + 32);
  HIP_TRY(launch_fill_zero(reinterpret_cast<float*>(flag), 1, st));
  if (data) HIP_TRY(launch_check_range(data, nd, 0.0f, 1, flag, st));
  const float eps = (float)o->eps;
  int64_t core = 1;
  for (int n = 0; n < ndim; ++n) {
    const int64_t cols = m->kind == COMM_CP ? m->rank : m->core_dims[n];
    core *= m->core_dims[n];
    HIP_TRY(launch_check_range(m->factors[n], dims[n] * cols, eps, 2, flag, st));
  }
  if (m->kind == COMM_TUCKER) HIP_TRY(launch_check_range(m->core, core, eps, 2, flag, st));
  int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h & 1) return fail(COMM_EINVAL, "check_inputs: the data hold a negative or non-finite value");
  if (h & 2) return fail(COMM_EINVAL, "check_inputs: a parameter is below eps or not finite");
  return COMM_OK;
}

int64_t dense_numel(const comm_dense* x) {
  int64_t n = 1;
  for (int k = 0; k < x->ndim; ++k) n *= x->dims[k];
  return n;
}

int input_check_dense(comm_ctx* ctx, const comm_dense* x, const comm_model* m, const comm_opts* o,
                      hipStream_t st) {
  return input_check(ctx, x->X, dense_numel(x), m, x->ndim, x->dims, o, st);
}

int input_check_coo(comm_ctx* ctx, const comm_coo* x, const comm_model* m, const comm_opts* o, hipStream_t st) {
  return input_check(ctx, x->val, x->nnz, m, x->ndim, x->dims, o, st);
}

// alpha_t of the whole model into alpha (device).
int extrap_alpha(const comm_dense* x, comm_model* m, comm_model* prev, const comm_extrap* e, float* alpha,
                 hipStream_t st) {
  ExtrapArgs a = {};
  int64_t cnt[kMaxBlocks];
  a.nb = model_blocks(x, m, a.cur, cnt);
  float* pp[kMaxBlocks];
  int64_t pc[kMaxBlocks];
  model_blocks(x, prev, pp, pc);
  for (int b = 0; b < a.nb; ++b) {
    a.prev[b] = pp[b];
    a.count[b] = cnt[b];
  }
  a.alpha_nes = e->alpha_nes;
  a.c = e->c;
  a.delta = e->delta;
  a.alpha = alpha;
  HIP_TRY(launch_extrap_alpha(a, st));
  return COMM_OK;
}

// Move block b (index in update order; -1 = all blocks).
int extrap_apply(const comm_dense* x, comm_model* m, comm_model* prev, int b, float* alpha, float eps,
                 hipStream_t st) {
  float* cur[kMaxBlocks];
  float* pp[kMaxBlocks];
  int64_t cnt[kMaxBlocks], pc[kMaxBlocks];
  const int nb = model_blocks(x, m, cur, cnt);
  model_blocks(x, prev, pp, pc);
  ExtrapArgs a = {};
  for (int q = 0; q < nb; ++q) {
    if (b >= 0 && q != b) continue;
    a.cur[a.nb] = cur[q];
    a.prev[a.nb] = pp[q];
    a.count[a.nb] = cnt[q];
    ++a.nb;
  }
  a.alpha = alpha;
  a.eps = eps;
  HIP_TRY(launch_extrap_apply(a, st));
  return COMM_OK;
}

// ---------------------------------------------------------------------------------------- sparse checks

// max_ndim: 4 for the beta = 1 CP kernels, COMM_MAX_NDIM for the others.
int check_coo(const comm_coo* x, int max_ndim = 4) {
  if (!x) return fail(COMM_EINVAL, "x is NULL");
  if (x->ndim < 2 || x->ndim > COMM_MAX_NDIM) return fail(COMM_EINVAL, "ndim = %d", x->ndim);
  if (x->ndim > max_ndim) return fail(COMM_EUNSUPPORTED, "sparse data of order %d on this path (at most %d)",
                                      x->ndim, max_ndim);
  if (x->nnz < 0) return fail(COMM_EINVAL, "nnz < 0");
  for (int n = 0; n < x->ndim; ++n) {
    if (x->dims[n] < 1 || x->dims[n] > (1 << 24)) return fail(COMM_EINVAL, "dims[%d]", n);
    if (x->nnz > 0 && !x->idx[n]) return fail(COMM_EINVAL, "idx[%d] is NULL", n);
  }
  if (x->nnz > 0 && !x->val) return fail(COMM_EINVAL, "val is NULL");
  return COMM_OK;
}

int check_coo_job(int ndim, const int64_t* dims, const comm_model* model, const comm_opts* opts) {
  (void)dims;
  int rc = check_opts(opts, true);
  if (rc) return rc;
  if (opts->beta != 1.0) return fail(COMM_EUNSUPPORTED, "sparse COO path requires beta = 1");
  if (!model || model->kind != COMM_CP) return fail(COMM_EINVAL, "model must be CP");
  if (model->rank < 1) return fail(COMM_EINVAL, "rank = %d", model->rank);
  if (model->rank > kRP) return fail(COMM_EUNSUPPORTED, "rank %d > %d", model->rank, kRP);
  for (int n = 0; n < ndim; ++n)
    if (!model->factors[n]) return fail(COMM_EINVAL, "factors[%d] is NULL", n);
  return COMM_OK;
}

// ---------------------------------------------------------------------------------------- sparse, beta in (0, 2)

// Sparse COO data at beta != 1 (Sec. 6.4, paragraph on sparse tensors): the
// numerators, which involve P = X * Xhat^(beta-2), are accumulated over the
// nonzeros (coo_beta_kernel); the denominators involve Q = Xhat^(beta-1) on
// every cell, so the dense orchestration runs on the all-zero twin of the
// tensor (P = 0 there, Q and d(0 | Xhat) exact; the twin is a null X, which
// the passes read as x = 0 without loading anything) and takes its
// numerators from the nonzeros through a NumHook.  The objective is the dense
// pass's sum of d(0 | Xhat) plus, over the nonzeros, d(x | Xhat) - d(0 | Xhat).

int grow(comm_ctx* ctx, char** buf, size_t* have, size_t bytes, hipStream_t st, const char* what) {
  if (bytes <= *have) return COMM_OK;
  if (ctx->limit && bytes > ctx->limit)
    return fail(COMM_ENOMEM, "%s of %zu bytes exceeds the context limit of %zu", what, bytes, ctx->limit);
  if (*buf) {
    HIP_TRY(hipStreamSynchronize(ctx->last_stream));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipFree(*buf));
    *buf = nullptr;
    *have = 0;
  }
  hipError_t e = hipMalloc(buf, bytes);
  if (e != hipSuccess) return fail(COMM_ENOMEM, "hipMalloc(%zu) for the %s: %s", bytes, what, hipGetErrorString(e));
  *have = bytes;
  return COMM_OK;
}

struct CooBetaWs {
  float* num;    // [max dims][32] numerator of one block
  float* w;      // per-nonzero P~ (J-CoMM)
  double* obj;   // per-workgroup objective corrections
  size_t bytes;
};

CooBetaWs coo_beta_layout(const comm_coo* x, char* base) {
  CooBetaWs s = {};
  int64_t rows = 1;
  for (int n = 0; n < x->ndim; ++n) rows = std::max<int64_t>(rows, x->dims[n]);
  rows = (rows + 31) / 32 * 32;  // also the padded fibre mode of the Tucker path
  Carve cv;
  cv.base = base;
  s.num = cv.take<float>((size_t)rows * kRP);
  s.w = cv.take<float>((size_t)std::max<int64_t>(x->nnz, 1));
  s.obj = cv.take<double>((size_t)coo_beta_blocks(x->nnz));
  s.bytes = cv.off + 256;
  return s;
}

// The dense passes over the index space run a grid over every cell: 2^36
// cells bounds their index arithmetic (and their time).
constexpr uint64_t kMaxTwinCells = uint64_t(1) << 36;

int check_coo_beta(const comm_coo* x, const comm_model* model, const comm_opts* o, bool need_L) {
  int rc = check_coo(x, COMM_MAX_NDIM);
  if (!rc) rc = check_opts(o, need_L);
  if (rc) return rc;
  if (!(o->beta > 0.0))
    return fail(COMM_EUNSUPPORTED, "sparse data at beta = 0: d(0 | y) is infinite (floor X and use the dense path)");
  if (x->ndim < 3) return fail(COMM_EUNSUPPORTED, "sparse data of order %d on this path (3 to 5)", x->ndim);
  if (!model) return fail(COMM_EINVAL, "model is NULL");
  // the dense twin's shape limits (3-way view for CP, row view for Tucker)
  comm_dense xd = {};
  xd.ndim = x->ndim;
  for (int n = 0; n < x->ndim; ++n) xd.dims[n] = x->dims[n];
  xd.X = reinterpret_cast<const float*>(x->val);  // not read: shapes only
  if ((rc = check_dense_shape(&xd))) return rc;
  // cap the cell count of the index space before any product can wrap
  uint64_t cells = 1;
  for (int n = 0; n < x->ndim; ++n) {
    if (cells > (kMaxTwinCells / (uint64_t)x->dims[n]))
      return fail(COMM_ENOMEM, "the index space of this sparse tensor exceeds %llu cells (dense denominators)",
                  (unsigned long long)kMaxTwinCells);
    cells *= (uint64_t)x->dims[n];
  }
  if (model->kind == COMM_CP) return check_cp_model(model, x->ndim);
  if (model->kind == COMM_TUCKER) return tucker_check_model(model, &xd);
  return fail(COMM_EINVAL, "model kind %d", model->kind);
}

// The dense twin of x and the sparse buffers.  The twin has no memory: its
// null X tells the CP passes (every class but beta = 1, which never runs a
// dense pass on sparse data) and the Tucker passes that x = 0 everywhere.
int coo_beta_setup(comm_ctx* ctx, const comm_coo* x, comm_dense* xd, CooBetaWs* s, hipStream_t st) {
  *xd = comm_dense{};
  xd->ndim = x->ndim;
  for (int n = 0; n < x->ndim; ++n) xd->dims[n] = x->dims[n];
  xd->X = nullptr;
  const CooBetaWs probe = coo_beta_layout(x, nullptr);
  int rc = grow(ctx, &ctx->sws, &ctx->sws_bytes, probe.bytes, st, "sparse workspace");
  if (rc) return rc;
  *s = coo_beta_layout(x, ctx->sws);
  return COMM_OK;
}

CooBetaArgs coo_beta_base(const comm_coo* x, const comm_model* m, const comm_opts* o) {
  CooBetaArgs a = {};
  a.N = x->ndim;
  a.R = m->rank;
  a.nnz = x->nnz;
  for (int n = 0; n < x->ndim; ++n) {
    a.dims[n] = (int)x->dims[n];
    a.idx[n] = x->idx[n];
  }
  a.val = x->val;
  a.mode = -1;
  a.bc = make_beta_const(o->beta);
  a.eps = (float)o->eps;
  return a;
}

// The hook: numerator of block n over the nonzeros against the contraction
// views ct, with weights from a rebuild at ct (B-CoMM) or the stored P~ (J-CoMM).
NumHook coo_num_hook(const comm_coo* x, const comm_model* m, const comm_opts* o, const CooBetaWs& s, bool stored,
                     hipStream_t st) {
  NumHook h;
  h.run = [=](int n, const FView* ct, const float** num) -> int {
    HIP_TRY(launch_fill_zero(s.num, (int64_t)x->dims[n] * kRP, st));
    CooBetaArgs a = coo_beta_base(x, m, o);
    a.mode = n;
    a.num = s.num;
    for (int q = 0; q < x->ndim; ++q) {
      a.ct[q] = ct[q];
      a.rb[q] = ct[q];
    }
    if (stored) a.w_in = s.w;
    HIP_TRY(launch_coo_beta(a, beta_class_of(o->beta), st));
    *num = s.num;
    return COMM_OK;
  };
  return h;
}

int coo_beta_bcomm(comm_ctx* ctx, const comm_coo* x, comm_model* m, int block, const comm_opts* o, hipStream_t st) {
  comm_dense xd;
  CooBetaWs s;
  int rc = coo_beta_setup(ctx, x, &xd, &s, st);
  if (rc) return rc;
  const NumHook hook = coo_num_hook(x, m, o, s, false, st);
  return cp_bcomm(ctx, &xd, m, block, o, st, &hook);
}

// Sum of the objective corrections over the nonzeros at the model m, added
// to *out (which holds the dense pass's sum at X = 0).
int coo_beta_obj_add(const comm_coo* x, const comm_model* m, const comm_opts* o, const CooBetaWs& s, bool keep_w,
                     double* out, hipStream_t st) {
  CooBetaArgs a = coo_beta_base(x, m, o);
  for (int q = 0; q < x->ndim; ++q) a.rb[q] = user_view(m, q);
  a.obj_part = out ? s.obj : nullptr;
  if (keep_w) a.w_out = s.w;
  HIP_TRY(launch_coo_beta(a, beta_class_of(o->beta), st));
  if (out) HIP_TRY(launch_sum_f64(s.obj, coo_beta_blocks(x->nnz), out, out, st));
  return COMM_OK;
}

int coo_beta_jcomm(comm_ctx* ctx, const comm_coo* x, comm_model* m, const comm_opts* o, double* obj, hipStream_t st) {
  comm_dense xd;
  CooBetaWs s;
  int rc = coo_beta_setup(ctx, x, &xd, &s, st);
  if (rc) return rc;
  // P~ at the reference (the caller's model before the iteration), kept for
  // the inner sweeps; its objective corrections summed now into a partial
  // that is added after the dense pass has written the zero-cell part
  CooBetaArgs a = coo_beta_base(x, m, o);
  for (int q = 0; q < x->ndim; ++q) a.rb[q] = user_view(m, q);
  a.w_out = s.w;
  a.obj_part = obj ? s.obj : nullptr;
  HIP_TRY(launch_coo_beta(a, beta_class_of(o->beta), st));
  comm_opts od = *o;
  od.cache_pq = 0;  // the cache would hold P~ and Q~ of every cell
  const NumHook hook = coo_num_hook(x, m, &od, s, true, st);
  if ((rc = cp_jcomm(ctx, &xd, m, &od, obj, st, &hook))) return rc;
  if (obj) HIP_TRY(launch_sum_f64(s.obj, coo_beta_blocks(x->nnz), obj, obj, st));
  return COMM_OK;
}

int coo_beta_objective(comm_ctx* ctx, const comm_coo* x, const comm_model* m, const comm_opts* o, double* out,
                       hipStream_t st) {
  comm_dense xd;
  CooBetaWs s;
  // (CP at beta = 1 never comes here: its zero cells sum in closed form,
  // coo_objective_kl); no zero tensor is needed
  int rc = coo_beta_setup(ctx, x, &xd, &s, st);
  if (rc) return rc;
  if (m->kind == COMM_TUCKER) {
    const TkSparse sp{x, s.w, s.num, s.obj};
    return tuckern_objective(ctx, &xd, m, o, out, st, &sp);
  }
  if ((rc = cp_objective(ctx, &xd, m, o, out, st))) return rc;
  return coo_beta_obj_add(x, m, o, s, false, out, st);
}

// Sparse Tucker (orders 3 to 5) on the order-N path; at beta = 1 no dense pass.
int coo_tucker(comm_ctx* ctx, const comm_coo* x, comm_model* m, int block, const comm_opts* o, double* obj,
               bool jcomm, hipStream_t st) {
  comm_dense xd;
  CooBetaWs s;
  int rc = coo_beta_setup(ctx, x, &xd, &s, st);
  if (rc) return rc;
  const TkSparse sp{x, s.w, s.num, s.obj};
  comm_opts od = *o;
  od.cache_pq = 0;
  return jcomm ? tuckern_jcomm(ctx, &xd, m, &od, obj, st, &sp) : tuckern_bcomm(ctx, &xd, m, block, &od, st, &sp);
}

// ---------------------------------------------------------------------------------------- J-CoMM, one or many

int jcomm_check(const comm_dense* x, const comm_model* model, const comm_opts* opts) {
  int rc = check_opts(opts, true);
  if (!rc) rc = check_dense(x);
  if (rc) return rc;
  if (!model) return fail(COMM_EINVAL, "model is NULL");
  if (model->kind == COMM_CP) return check_cp_model(model, x->ndim);
  if (model->kind == COMM_TUCKER) return tucker_check_model(model, x);
  return fail(COMM_EINVAL, "model kind %d", model->kind);
}

size_t jcomm_ws_bytes(const comm_dense* x, const comm_model* model, const comm_opts* opts,
                      const TuneChoice& pick = TuneChoice()) {
  if (model->kind == COMM_CP) return cp_ws_bytes(x, opts->beta != 1.0 && opts->cache_pq, cp_wshare(opts, pick));
  return tucker_workspace_bytes(x, model, opts, 1, pick.tk_groups);
}

// Key of the autotune table: what fixes a J-CoMM outer iteration's launch
// sequence and sizes (model kind, shape, rank or core, beta, precision, L).
std::vector<int64_t> tune_key(const comm_dense* x, const comm_model* m, const comm_opts* o) {
  std::vector<int64_t> k = {m->kind, x->ndim};
  for (int n = 0; n < x->ndim; ++n) k.push_back(x->dims[n]);
  if (m->kind == COMM_CP) {
    k.push_back(m->rank);
  } else {
    for (int n = 0; n < x->ndim; ++n) k.push_back(m->core_dims[n]);
  }
  int64_t beta_bits;
  std::memcpy(&beta_bits, &o->beta, sizeof beta_bits);
  k.push_back(beta_bits);
  k.push_back(o->precision);
  k.push_back(o->inner_sweeps);
  return k;
}

// What tune_key reads, checked without the buffers (the table calls take a
// problem's key only).
int tune_key_check(const comm_dense* x, const comm_model* m, const comm_opts* o) {
  int rc = check_opts(o, true);
  if (!rc) rc = check_dense_shape(x);
  if (rc) return rc;
  if (!m) return fail(COMM_EINVAL, "model is NULL");
  if (m->kind == COMM_CP) {
    if (m->rank < 1) return fail(COMM_EINVAL, "rank = %d", m->rank);
  } else if (m->kind == COMM_TUCKER) {
    for (int n = 0; n < x->ndim; ++n)
      if (m->core_dims[n] < 1) return fail(COMM_EINVAL, "core_dims[%d] = %lld", n, (long long)m->core_dims[n]);
  } else {
    return fail(COMM_EINVAL, "model kind %d", m->kind);
  }
  return COMM_OK;
}

// The equivalent evaluations the tuner times for a problem, defaults first:
// the P~/Q~ cache or its recomputation (beta != 1); dense CP at rank <= 16
// with float32 tiles: 16-wide or 32-wide pass tiles; dense CP of order 3 at
// beta != 1: modes 1 and 2 from one V pass or a pass each; dense Tucker of
// order 3: the mode-3 pass's pair-group cap.  One entry means nothing to time.
std::vector<TuneChoice> tune_variants(const comm_dense* x, const comm_model* model, const comm_opts* o) {
  const std::vector<int> caches = o->beta != 1.0 ? std::vector<int>{1, 0} : std::vector<int>{0};
  const bool cp = model->kind == COMM_CP;
  std::vector<int> tiles = {0};
  if (cp && model->rank <= 16 && o->precision != COMM_BF16) tiles.push_back(32);
  std::vector<int> wshares = {-1};
  if (cp && x->ndim == 3 && o->beta != 1.0) {
    const int def = o->precision != COMM_BF16;
    wshares = {def, 1 - def};
  }
  std::vector<int> groups = {0};
  if (!cp && x->ndim == 3) groups = {kTkGroupsDefault, 64, kTkGroupsMax};
  std::vector<TuneChoice> out;
  for (int c : caches)
    for (int t : tiles)
      for (int ws : wshares)
        for (int gr : groups) {
          TuneChoice v;
          v.cache_pq = c;
          v.cp_tile = t;
          v.wshare = ws;
          v.tk_groups = gr;
          out.push_back(v);
        }
  return out;
}

int jcomm_variant(comm_ctx* ctx, const comm_dense* x, comm_model* model, const comm_opts* o, double* obj,
                  hipStream_t st) {
  return model->kind == COMM_CP ? cp_jcomm(ctx, x, model, o, obj, st) : tucker_jcomm(ctx, x, model, o, obj, st);
}

// The options and launch shapes a call runs with: a recorded table entry
// fixes the shapes, and the cache choice when cache_pq = COMM_CACHE_AUTO;
// without an entry, AUTO takes the cache if its workspace is within the
// context's limit (`limit`, 0 = none), and recomputation otherwise.
void resolve(const comm_ctx* ctx, const comm_dense* x, const comm_model* model, const comm_opts* opts,
             size_t limit, comm_opts* o, TuneChoice* pick) {
  *o = *opts;
  *pick = TuneChoice();
  const auto it = ctx->tune.find(tune_key(x, model, opts));
  if (it != ctx->tune.end()) *pick = it->second;
  if (o->cache_pq == COMM_CACHE_AUTO) {
    if (it != ctx->tune.end()) {
      o->cache_pq = it->second.cache_pq;
    } else {
      o->cache_pq = 1;
      o->cache_pq = !limit || jcomm_ws_bytes(x, model, o, *pick) <= limit ? 1 : 0;
    }
  }
}

int jcomm_run(comm_ctx* ctx, const comm_dense* x, comm_model* model, const comm_opts* opts, double* obj,
              hipStream_t st) {
  comm_opts o;
  resolve(ctx, x, model, opts, ctx->limit, &o, &ctx->pick);
  const int rc = jcomm_variant(ctx, x, model, &o, obj, st);
  ctx->pick = TuneChoice();
  return rc;
}

// Device copy of a model's parameters for the tuner (freed on scope exit).
struct TuneScratch {
  float* buf = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~TuneScratch() {
    if (buf) hipFree(buf);
    for (hipEvent_t e : ev)
      if (e) hipEventDestroy(e);
  }
};

// A batch runs every problem with the kernels and launch shapes of a single
// call, on a private slice of the batch workspace, so its result does not
// depend on what else is in the batch.  Problems are spread round-robin over
// kBatchStreams internal streams (default priority) forked from and joined
// back to the caller's stream, so the small problems' kernels overlap.
constexpr int kBatchStreams = 4;

struct BatchItem {
  comm_dense x;
  comm_model m;
  comm_opts o;      // resolved (no COMM_CACHE_AUTO)
  TuneChoice pick;  // resolved launch shapes
  double* obj;
  size_t off, bytes;
};

int batch_resources(comm_ctx* ctx) {
  if (!ctx->bstreams.empty()) return COMM_OK;
  for (int s = 0; s < kBatchStreams; ++s) {
    hipStream_t q;
    HIP_TRY(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    ctx->bstreams.push_back(q);
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->bjoin.push_back(e);
  }
  HIP_TRY(hipStreamCreateWithFlags(&ctx->bcapture, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&ctx->bfork, hipEventDisableTiming));
  return COMM_OK;
}

int batch_sync_all(comm_ctx* ctx, hipStream_t st) {
  HIP_TRY(hipStreamSynchronize(st));
  if (ctx->glast) HIP_TRY(hipStreamSynchronize(ctx->glast));
  for (hipStream_t q : ctx->bstreams) HIP_TRY(hipStreamSynchronize(q));
  return COMM_OK;
}

int batch_drop_graph(comm_ctx* ctx) {
  if (ctx->gexec) HIP_TRY(hipGraphExecDestroy(ctx->gexec));
  if (ctx->graph) HIP_TRY(hipGraphDestroy(ctx->graph));
  ctx->gexec = nullptr;
  ctx->graph = nullptr;
  ctx->gkey.clear();
  return COMM_OK;
}

int batch_ensure_ws(comm_ctx* ctx, size_t bytes, hipStream_t st) {
  if (bytes <= ctx->bws_bytes) return COMM_OK;
  if (ctx->limit && bytes > ctx->limit)
    return fail(COMM_ENOMEM, "batch workspace of %zu bytes exceeds the context limit of %zu", bytes, ctx->limit);
  int rc = batch_sync_all(ctx, st);
  if (rc) return rc;
  if ((rc = batch_drop_graph(ctx))) return rc;  // the cached graph points into the old workspace
  if (ctx->bws) HIP_TRY(hipFree(ctx->bws));
  ctx->bws = nullptr;
  ctx->bws_bytes = 0;
  size_t want = bytes + bytes / 4;
  if (ctx->limit && want > ctx->limit) want = ctx->limit;
  hipError_t e = hipMalloc(&ctx->bws, want);
  if (e != hipSuccess) return fail(COMM_ENOMEM, "hipMalloc(%zu): %s", want, hipGetErrorString(e));
  ctx->bws_bytes = want;
  return COMM_OK;
}

// Everything that decides the launches of a batch, word by word.
std::vector<int64_t> batch_key(const std::vector<BatchItem>& items, const char* ws) {
  std::vector<int64_t> k;
  auto word = [&](int64_t v) { k.push_back(v); };
  auto dbl = [&](double v) {
    int64_t b;
    std::memcpy(&b, &v, sizeof b);
    k.push_back(b);
  };
  word((int64_t)(intptr_t)ws);
  for (const BatchItem& it : items) {
    word(it.x.ndim);
    for (int n = 0; n < COMM_MAX_NDIM; ++n) word(it.x.dims[n]);
    word((int64_t)(intptr_t)it.x.X);
    word(it.m.kind);
    word(it.m.rank);
    for (int n = 0; n < COMM_MAX_NDIM; ++n) word(it.m.core_dims[n]);
    for (int n = 0; n < COMM_MAX_NDIM; ++n) word((int64_t)(intptr_t)it.m.factors[n]);
    word((int64_t)(intptr_t)it.m.core);
    dbl(it.o.beta);
    dbl(it.o.eps);
    dbl(it.o.eps_x);
    word(it.o.inner_sweeps);
    word(it.o.precision);
    word(it.o.cache_pq);
    word(it.pick.wshare);
    word(it.pick.tk_groups);
    word(it.pick.cp_tile);
    word((int64_t)(intptr_t)it.obj);
    word((int64_t)it.off);
  }
  return k;
}

// Fork from `origin`, issue every problem on its stream, join back to `origin`.
int batch_issue(comm_ctx* ctx, std::vector<BatchItem>& items, hipStream_t origin) {
  const int S = (int)ctx->bstreams.size();
  HIP_TRY(hipEventRecord(ctx->bfork, origin));
  for (hipStream_t q : ctx->bstreams) HIP_TRY(hipStreamWaitEvent(q, ctx->bfork, 0));
  for (size_t p = 0; p < items.size(); ++p) {
    BatchItem& it = items[p];
    comm_ctx sub;
    sub.device = ctx->device;
    sub.ws = ctx->bws + it.off;
    sub.ws_bytes = it.bytes;
    sub.limit = it.bytes;  // a slice never grows: a larger need is an error, not an allocation
    // it.o and it.pick hold the resolved choices the slice was sized for
    sub.pick = it.pick;
    int rc = jcomm_variant(&sub, &it.x, &it.m, &it.o, it.obj, ctx->bstreams[p % S]);
    if (rc) return rc;
  }
  for (int q = 0; q < S; ++q) {
    HIP_TRY(hipEventRecord(ctx->bjoin[q], ctx->bstreams[q]));
    HIP_TRY(hipStreamWaitEvent(origin, ctx->bjoin[q], 0));
  }
  return COMM_OK;
}

// ---- grouped batches
//
// Each problem's launches are recorded (nothing runs), then issued on one
// stream: at every step the kernel at the head of the most problems' sequences
// runs once for all of them, through its grouped twin and a table of their
// arguments; launches without a grouped twin run alone.  Each problem's own
// launches keep their order, and each workgroup computes what it computes in
// the problem's own launch, so results are bitwise those of single calls.
struct GroupLaunch {
  const void* kgrp;                     // null: closure `fn` of problem `p`
  dim3 block;
  size_t shmem;
  uint32_t blocks;
  size_t off_bucket, off_first, off_items;  // offsets in the table image
  int stride;
  const LaunchRec* rec;
};

struct GroupPlan {
  std::vector<Recorder> recs;                      // one per problem
  std::vector<std::vector<GroupLaunch>> shards;    // launches per internal stream
  std::vector<char> image;                         // all tables, 256-byte aligned pieces
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int group_record(comm_ctx* ctx, std::vector<BatchItem>& items, GroupPlan& plan) {
  plan.recs.assign(items.size(), Recorder());
  for (size_t p = 0; p < items.size(); ++p) {
    BatchItem& it = items[p];
    comm_ctx sub;
    sub.device = ctx->device;
    sub.ws = ctx->bws + it.off;
    sub.ws_bytes = it.bytes;
    sub.limit = it.bytes;
    sub.pick = it.pick;
    struct Install {
      explicit Install(Recorder* r) { g_recorder = r; }
      ~Install() { g_recorder = nullptr; }
    } install(&plan.recs[p]);
    const int rc = jcomm_variant(&sub, &it.x, &it.m, &it.o, it.obj, nullptr);
    if (rc) return rc;
  }
  return COMM_OK;
}

// Greedy grouping of the sequences of problems `ps`: at each step the kernel
// at the head of the most sequences runs once for all of them.
void group_shard(GroupPlan& plan, const std::vector<size_t>& ps, std::vector<GroupLaunch>& out) {
  const size_t P = ps.size();
  std::vector<size_t> head(P, 0);
  auto seq = [&](size_t i) -> const std::vector<LaunchRec>& { return plan.recs[ps[i]].recs; };
  auto take = [&](size_t bytes) {
    const size_t off = plan.image.size();
    plan.image.resize(align256(off + bytes), 0);
    return off;
  };
  auto same = [](const LaunchRec& a, const LaunchRec& b) {
    return a.kgrp == b.kgrp && a.block.x == b.block.x && a.shmem == b.shmem;
  };
  for (;;) {
    const LaunchRec* best = nullptr;
    int best_count = 0;
    size_t closure_i = P;
    for (size_t i = 0; i < P; ++i) {
      if (head[i] >= seq(i).size()) continue;
      const LaunchRec& r = seq(i)[head[i]];
      if (!r.kgrp) {
        if (closure_i == P) closure_i = i;
        continue;
      }
      int c = 0;
      for (size_t q = 0; q < P; ++q)
        if (head[q] < seq(q).size()) c += same(seq(q)[head[q]], r);
      if (c > best_count) {
        best = &r;
        best_count = c;
      }
    }
    if (!best) {
      if (closure_i == P) break;  // every sequence is done
      GroupLaunch g{};
      g.rec = &seq(closure_i)[head[closure_i]];
      out.push_back(g);
      ++head[closure_i];
      continue;
    }
    GroupLaunch g{};
    g.kgrp = best->kgrp;
    g.block = best->block;
    g.shmem = best->shmem;
    g.stride = (int)best->item.size();
    std::vector<const LaunchRec*> members;
    const LaunchRec key = *best;
    for (size_t q = 0; q < P; ++q) {
      if (head[q] < seq(q).size() && same(seq(q)[head[q]], key)) {
        members.push_back(&seq(q)[head[q]]);
        ++head[q];
      }
    }
    std::vector<uint32_t> first;
    uint32_t total = 0;
    for (const LaunchRec* m : members) {
      first.push_back(total);
      total += m->grid.x * m->grid.y * m->grid.z;
    }
    first.push_back(total);
    g.blocks = total;
    const size_t nb = (total + kGroupBucket - 1) / kGroupBucket;
    g.off_bucket = take(nb * sizeof(uint32_t));
    g.off_first = take(first.size() * sizeof(uint32_t));
    g.off_items = take(members.size() * (size_t)g.stride);
    uint32_t* bucket = reinterpret_cast<uint32_t*>(plan.image.data() + g.off_bucket);
    for (size_t b = 0, j = 0; b < nb; ++b) {
      const uint32_t w = (uint32_t)(b * kGroupBucket);
      while (first[j + 1] <= w) ++j;
      bucket[b] = (uint32_t)j;
    }
    std::memcpy(plan.image.data() + g.off_first, first.data(), first.size() * sizeof(uint32_t));
    for (size_t j = 0; j < members.size(); ++j)
      std::memcpy(plan.image.data() + g.off_items + j * g.stride, members[j]->item.data(), g.stride);
    out.push_back(g);
  }
}

// Problems with the same launch sequence (the same kernels in the same order)
// share a shard, where their launches group fully; the shards, balanced by
// their workgroup counts, run on the internal streams side by side.
void group_plan(GroupPlan& plan, int S) {
  std::map<std::vector<const void*>, std::vector<size_t>> by_seq;
  std::map<std::vector<const void*>, uint64_t> weight;
  for (size_t p = 0; p < plan.recs.size(); ++p) {
    std::vector<const void*> sig;
    uint64_t w = 0;
    for (const LaunchRec& r : plan.recs[p].recs) {
      sig.push_back(r.kgrp);
      w += (uint64_t)r.grid.x * r.grid.y * r.grid.z;
    }
    by_seq[sig].push_back(p);
    weight[sig] += w;
  }
  std::vector<std::pair<uint64_t, const std::vector<size_t>*>> order;
  for (const auto& kv : by_seq) order.push_back({weight[kv.first], &kv.second});
  std::stable_sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<std::vector<size_t>> members((size_t)S);
  std::vector<uint64_t> load((size_t)S, 0);
  for (const auto& o : order) {
    const size_t s = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
    members[s].insert(members[s].end(), o.second->begin(), o.second->end());
    load[s] += o.first;
  }
  plan.shards.assign((size_t)S, {});
  for (int s = 0; s < S; ++s) {
    std::sort(members[(size_t)s].begin(), members[(size_t)s].end());
    group_shard(plan, members[(size_t)s], plan.shards[(size_t)s]);
  }
}

// Copy the table image to `dev` (grown to fit, 256-aligned) through the
// context's pinned buffer, on stream st.
int group_upload(comm_ctx* ctx, const GroupPlan& plan, char** dev, size_t* dev_bytes, hipStream_t st) {
  const size_t n = std::max<size_t>(plan.image.size(), 256);
  if (!ctx->gtab_copied) HIP_TRY(hipEventCreateWithFlags(&ctx->gtab_copied, hipEventDisableTiming));
  HIP_TRY(hipEventSynchronize(ctx->gtab_copied));  // the pinned image of the last copy is free again
  if (ctx->gtab_host_bytes < n) {
    if (ctx->gtab_host) HIP_TRY(hipHostFree(ctx->gtab_host));
    ctx->gtab_host = nullptr;
    ctx->gtab_host_bytes = 0;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&ctx->gtab_host), n, hipHostMallocDefault));
    ctx->gtab_host_bytes = n;
  }
  if (*dev_bytes < n) {
    if (*dev) {
      // earlier grouped launches may still read the old table
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(*dev));
    }
    *dev = nullptr;
    *dev_bytes = 0;
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(dev), n));
    *dev_bytes = n;
  }
  std::memcpy(ctx->gtab_host, plan.image.data(), plan.image.size());
  HIP_TRY(hipMemcpyAsync(*dev, ctx->gtab_host, plan.image.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(ctx->gtab_copied, st));
  return COMM_OK;
}

int group_launch(const GroupLaunch& g, const char* dev, hipStream_t st) {
  if (!g.kgrp) return g.rec->fn(st) == hipSuccess ? COMM_OK : fail(COMM_EHIP, "launch failed");
  GroupTable t;
  // (C-style casts: in the device compilation pass these members are in the
  // constant address space)
  t.bucket = (decltype(t.bucket))(dev + g.off_bucket);
  t.first = (decltype(t.first))(dev + g.off_first);
  t.items = (decltype(t.items))(dev + g.off_items);
  t.stride = g.stride;
  void* args[] = {&t};
  HIP_TRY(hipLaunchKernel(g.kgrp, dim3(g.blocks), g.block, args, g.shmem, st));
  return COMM_OK;
}

// The shards on the internal streams, forked from and joined to `origin`.
int group_issue(comm_ctx* ctx, const GroupPlan& plan, const char* dev, hipStream_t origin) {
  const size_t S = ctx->bstreams.size();
  HIP_TRY(hipEventRecord(ctx->bfork, origin));
  for (hipStream_t q : ctx->bstreams) HIP_TRY(hipStreamWaitEvent(q, ctx->bfork, 0));
  for (size_t s = 0; s < plan.shards.size() && s < S; ++s)
    for (const GroupLaunch& g : plan.shards[s]) {
      const int rc = group_launch(g, dev, ctx->bstreams[s]);
      if (rc) return rc;
    }
  for (size_t q = 0; q < S; ++q) {
    HIP_TRY(hipEventRecord(ctx->bjoin[q], ctx->bstreams[q]));
    HIP_TRY(hipStreamWaitEvent(origin, ctx->bjoin[q], 0));
  }
  return COMM_OK;
}

int jcomm_batched(comm_ctx* ctx, const comm_problem* probs, int count, int flags, hipStream_t st) {
  std::vector<BatchItem> items((size_t)count);
  size_t total = 0;
  for (int p = 0; p < count; ++p) {
    const comm_problem& q = probs[p];
    if (!q.x || !q.model || !q.opts) return fail(COMM_EINVAL, "problem %d: x, model and opts must not be NULL", p);
    int rc = jcomm_check(q.x, q.model, q.opts);
    if (rc) {
      std::string msg = g_last_error;
      return fail(rc, "problem %d: %s", p, msg.c_str());
    }
    BatchItem& it = items[(size_t)p];
    it.x = *q.x;
    it.m = *q.model;
    // the choices are resolved once here: the slices are sized for them
    resolve(ctx, q.x, q.model, q.opts, ctx->limit, &it.o, &it.pick);
    it.obj = q.obj_ref_dev;
    it.bytes = (jcomm_ws_bytes(q.x, q.model, &it.o, it.pick) + 255) & ~size_t(255);
    total += it.bytes;
  }
  if (count == 0) return COMM_OK;
  // Automatic choices without a table entry took the cache whenever each
  // problem's own workspace fits the limit; if the batch together does not,
  // they fall back to recomputation, largest slice first, until it fits.
  while (ctx->limit && total > ctx->limit) {
    int pick = -1;
    for (int p = 0; p < count; ++p) {
      const BatchItem& it = items[(size_t)p];
      if (probs[p].opts->cache_pq != COMM_CACHE_AUTO || !it.o.cache_pq ||
          ctx->tune.count(tune_key(&it.x, &it.m, probs[p].opts)))
        continue;
      if (pick < 0 || it.bytes > items[(size_t)pick].bytes) pick = p;
    }
    if (pick < 0) break;
    BatchItem& it = items[(size_t)pick];
    it.o.cache_pq = 0;
    const size_t nb = (jcomm_ws_bytes(&it.x, &it.m, &it.o, it.pick) + 255) & ~size_t(255);
    total -= it.bytes - nb;
    it.bytes = nb;
  }
  total = 0;
  for (BatchItem& it : items) {
    it.off = total;
    total += it.bytes;
  }
  // debug input checks, eagerly on the caller's stream, before any problem runs
  for (int p = 0; p < count; ++p) {
    const int rc = input_check_dense(ctx, probs[p].x, probs[p].model, probs[p].opts, st);
    if (rc) {
      std::string msg = g_last_error;
      return fail(rc, "problem %d: %s", p, msg.c_str());
    }
  }
  int rc = batch_resources(ctx);
  if (rc) return rc;
  if ((rc = batch_ensure_ws(ctx, total, st))) return rc;
  // grouped launches: dense problems of order 3 (the only ones whose launchers
  // all have grouped twins); otherwise the problems run one by one
  bool grouped = (flags & COMM_BATCH_GROUPED) != 0;
  for (const BatchItem& it : items) grouped = grouped && it.x.ndim == 3;
  if (!(flags & COMM_BATCH_GRAPH)) {
    if (grouped) {
      GroupPlan plan;
      if ((rc = group_record(ctx, items, plan))) return rc;
      group_plan(plan, (int)ctx->bstreams.size());
      // the eager table is rewritten: launches of an earlier call on another
      // stream must be done with it
      if (ctx->glast && ctx->glast != st) HIP_TRY(hipStreamSynchronize(ctx->glast));
      if ((rc = group_upload(ctx, plan, &ctx->gtab, &ctx->gtab_bytes, st))) return rc;
      rc = group_issue(ctx, plan, ctx->gtab, st);
    } else {
      rc = batch_issue(ctx, items, st);
    }
    ctx->glast = st;
    return rc;
  }
  std::vector<int64_t> key = batch_key(items, ctx->bws);
  key.push_back(grouped ? 1 : 0);
  if (!ctx->gexec || key != ctx->gkey) {
    // a different problem list: wait for the old graph's replays, then capture anew
    if (ctx->gexec) {
      if ((rc = batch_sync_all(ctx, st))) return rc;
      if ((rc = batch_drop_graph(ctx))) return rc;
    }
    GroupPlan plan;
    if (grouped) {
      // the graph's table is written before the capture and kept with the graph
      if ((rc = group_record(ctx, items, plan))) return rc;
      group_plan(plan, (int)ctx->bstreams.size());
      if ((rc = group_upload(ctx, plan, &ctx->gtab_graph, &ctx->gtab_graph_bytes, st))) return rc;
      HIP_TRY(hipStreamSynchronize(st));
    }
    HIP_TRY(hipStreamBeginCapture(ctx->bcapture, hipStreamCaptureModeThreadLocal));
    rc = grouped ? group_issue(ctx, plan, ctx->gtab_graph, ctx->bcapture) : batch_issue(ctx, items, ctx->bcapture);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->bcapture, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(COMM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    ctx->graph = g;
    e = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      batch_drop_graph(ctx);
      return fail(COMM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    ctx->gkey = std::move(key);
  }
  HIP_TRY(hipGraphLaunch(ctx->gexec, st));
  ctx->glast = st;
  return COMM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------- C ABI

extern "C" {

const char* comm_last_error(void) { return g_last_error.c_str(); }

int comm_create(int device, size_t workspace_limit_bytes, comm_ctx** out) {
  return guarded([&]() -> int {
    if (!out) return fail(COMM_EINVAL, "out is NULL");
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(COMM_EINVAL, "device %d of %d", device, count);
    char* noalloc_ws = nullptr;
    const int rc = scratch_address(device, &noalloc_ws);
    if (rc) return rc;
    comm_ctx* c = new comm_ctx();
    c->device = device;
    c->limit = workspace_limit_bytes;
    c->noalloc_ws = noalloc_ws;
    *out = c;
    return COMM_OK;
  });
}

int comm_destroy(comm_ctx* ctx) {
  return guarded([&]() -> int {
    if (!ctx) return COMM_OK;
    int rc = COMM_OK;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->last_stream);
    if (ctx->ws) {
      hipError_t e = hipFree(ctx->ws);
      if (e != hipSuccess) rc = fail(COMM_EHIP, "hipFree: %s", hipGetErrorString(e));
    }
    for (auto& pr : ctx->events) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
    if (ctx->glast) hipStreamSynchronize(ctx->glast);
    for (hipStream_t q : ctx->bstreams) hipStreamSynchronize(q);
    batch_drop_graph(ctx);
    if (ctx->bws) {
      hipError_t e = hipFree(ctx->bws);
      if (e != hipSuccess) rc = fail(COMM_EHIP, "hipFree: %s", hipGetErrorString(e));
    }
    for (hipStream_t q : ctx->bstreams) hipStreamDestroy(q);
    for (hipEvent_t e : ctx->bjoin) hipEventDestroy(e);
    if (ctx->bcapture) hipStreamDestroy(ctx->bcapture);
    if (ctx->gtab) hipFree(ctx->gtab);
    if (ctx->gtab_graph) hipFree(ctx->gtab_graph);
    if (ctx->gtab_host) hipHostFree(ctx->gtab_host);
    if (ctx->gtab_copied) hipEventDestroy(ctx->gtab_copied);
    if (ctx->aux) hipFree(ctx->aux);
    if (ctx->sws) hipFree(ctx->sws);
    if (ctx->bfork) hipEventDestroy(ctx->bfork);
    delete ctx;
    return rc;
  });
}

int comm_check(comm_ctx* ctx) {
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = set_device(ctx);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(ctx->last_stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(COMM_EHIP, "asynchronous error: %s", hipGetErrorString(e));
    return COMM_OK;
  });
}

int comm_profile_enable(comm_ctx* ctx, int every) {
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    if (every < 0) return fail(COMM_EINVAL, "profile sampling interval %d < 0", every);
    ctx->profiling = every > 0;
    ctx->profile_every = every > 0 ? every : 1;
    ctx->profile_seen = 0;
    ctx->events_used = 0;
    // create the event pool now, so that the launches being measured do not
    // pay for event creation (the pool grows past this only on demand)
    if (ctx->profiling && ctx->events.size() < kProfileEvents) {
      if (int rc = set_device(ctx)) return rc;
      ctx->events.reserve(kProfileEvents);
      while (ctx->events.size() < kProfileEvents) {
        hipEvent_t a0, a1;
        HIP_TRY(hipEventCreate(&a0));
        if (hipEventCreate(&a1) != hipSuccess) {
          hipEventDestroy(a0);
          return fail(COMM_EHIP, "hipEventCreate failed");
        }
        ctx->events.emplace_back(a0, a1);
      }
    }
    return COMM_OK;
  });
}

int comm_profile_query(comm_ctx* ctx, double* total_ms, int64_t* launches, int64_t* seen) {
  return guarded([&]() -> int {
    if (!ctx || !total_ms || !launches) return fail(COMM_EINVAL, "NULL argument");
    double sum = 0.0;
    for (size_t k = 0; k < ctx->events_used; ++k) {
      HIP_TRY(hipEventSynchronize(ctx->events[k].second));
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, ctx->events[k].first, ctx->events[k].second));
      sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)ctx->events_used;
    if (seen) *seen = ctx->profile_seen;
    ctx->events_used = 0;
    ctx->profile_seen = 0;
    return COMM_OK;
  });
}

size_t comm_workspace_bytes(const comm_dense* x, const comm_model* model, const comm_opts* opts, int op) {
  if (check_dense_shape(x) || !model || !opts) return 0;
  // the largest need over the choices an autotune table can make: W-sharing
  // for CP, the most mode-3 pair groups for Tucker
  if (model->kind == COMM_CP) return cp_ws_bytes(x, op == 1 && opts->beta != 1.0 && opts->cache_pq, op == 1 && opts->beta != 1.0);
  if (x->ndim > 3) {
    int64_t rows = 1;
    for (int n = 0; n < x->ndim - 1; ++n) rows *= x->dims[n];
    if (rows > (1 << 24)) return 0;
  }
  for (int n = 0; n < x->ndim; ++n)
    if (model->core_dims[n] < 1 || model->core_dims[n] > kRP) return 0;
  return tucker_workspace_bytes(x, model, opts, op, kTkGroupsMax);
}

int comm_cp_update(comm_ctx* ctx, const comm_dense* x, comm_model* model, int block, const comm_opts* opts,
                   void* stream) {
  const TraceRange trace_range("comm_cp_update");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = check_opts(opts, false);
    if (!rc) rc = check_dense(x);
    if (!rc) rc = check_cp_model(model, x->ndim);
    if (rc) return rc;
    if (block < -1 || block >= x->ndim) return fail(COMM_EINVAL, "block = %d", block);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_dense(ctx, x, model, opts, st))) return rc;
    rc = cp_bcomm(ctx, x, model, block, opts, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_jcomm_outer(comm_ctx* ctx, const comm_dense* x, comm_model* model, const comm_opts* opts,
                     double* obj_ref_dev, void* stream) {
  const TraceRange trace_range("comm_jcomm_outer");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = jcomm_check(x, model, opts);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_dense(ctx, x, model, opts, st))) return rc;
    rc = jcomm_run(ctx, x, model, opts, obj_ref_dev, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_jcomm_outer_noalloc(comm_ctx* ctx, const comm_dense* x, comm_model* model, const comm_opts* opts,
                             double* obj_ref_dev, void* stream) {
  const TraceRange trace_range("comm_jcomm_outer_noalloc");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = jcomm_check(x, model, opts);
    if (rc) return rc;
    if (opts->check_inputs)
      return fail(COMM_EINVAL, "check_inputs needs a device flag of its own: not available without allocation");
    if (!ctx->noalloc_ws) return fail(COMM_EHIP, "no fixed workspace on device %d", ctx->device);
    comm_opts o;
    TuneChoice pick;
    resolve(ctx, x, model, opts, kNoallocBytes, &o, &pick);
    if (opts->cache_pq == COMM_CACHE_AUTO && o.cache_pq && jcomm_ws_bytes(x, model, &o, pick) > kNoallocBytes)
      o.cache_pq = 0;
    const size_t need = jcomm_ws_bytes(x, model, &o, pick);
    if (need > kNoallocBytes)
      return fail(COMM_ENOMEM, "workspace of %zu bytes exceeds the %zu-byte fixed array of the allocation-free call",
                  need, kNoallocBytes);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    // the single call's orchestration on a context whose workspace is the
    // fixed array: it never grows (a larger need is an error, checked above)
    comm_ctx sub;
    sub.device = ctx->device;
    sub.ws = ctx->noalloc_ws;
    sub.ws_bytes = kNoallocBytes;
    sub.limit = kNoallocBytes;
    sub.pick = pick;
    rc = jcomm_variant(&sub, x, model, &o, obj_ref_dev, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_tune_jcomm(comm_ctx* ctx, const comm_dense* x, const comm_model* model, const comm_opts* opts, int reps,
                    int* choice, double* ms, void* stream) {
  const TraceRange trace_range("comm_tune_jcomm");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = jcomm_check(x, model, opts);
    if (rc) return rc;
    if (reps < 1 || reps > 1000) return fail(COMM_EINVAL, "reps = %d (1 to 1000)", reps);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_dense(ctx, x, model, opts, st))) return rc;
    const std::vector<TuneChoice> vars = tune_variants(x, model, opts);
    double t[2] = {NAN, NAN};  // per outer iteration, fastest of each cache choice: [0] recompute, [1] cache
    TuneChoice best = vars[0];
    best.variants = 0;
    if (vars.size() > 1) {
      // the variants run on a copy of the parameters; the caller's are not touched
      comm_model sm = *model;
      size_t count[COMM_MAX_NDIM + 1] = {};
      size_t total = 0;
      for (int n = 0; n < x->ndim; ++n) {
        const int64_t cols = model->kind == COMM_CP ? model->rank : model->core_dims[n];
        count[n] = (size_t)x->dims[n] * (size_t)cols;
        total += count[n];
      }
      if (model->kind == COMM_TUCKER) {
        count[COMM_MAX_NDIM] = 1;
        for (int n = 0; n < x->ndim; ++n) count[COMM_MAX_NDIM] *= (size_t)model->core_dims[n];
        total += count[COMM_MAX_NDIM];
      }
      TuneScratch sc;
      HIP_TRY(hipMalloc(&sc.buf, total * sizeof(float)));
      HIP_TRY(hipEventCreate(&sc.ev[0]));
      HIP_TRY(hipEventCreate(&sc.ev[1]));
      size_t off = 0;
      for (int n = 0; n < x->ndim; ++n) {
        sm.factors[n] = sc.buf + off;
        off += count[n];
      }
      if (model->kind == COMM_TUCKER) sm.core = sc.buf + off;
      auto reset = [&]() -> int {
        for (int n = 0; n < x->ndim; ++n)
          HIP_TRY(hipMemcpyAsync(sm.factors[n], model->factors[n], count[n] * sizeof(float),
                                 hipMemcpyDeviceToDevice, st));
        if (model->kind == COMM_TUCKER)
          HIP_TRY(hipMemcpyAsync(sm.core, model->core, count[COMM_MAX_NDIM] * sizeof(float),
                                 hipMemcpyDeviceToDevice, st));
        return COMM_OK;
      };
      // the variants run with the context's pick set; it is cleared on every exit
      struct PickReset {
        comm_ctx* c;
        ~PickReset() { c->pick = TuneChoice(); }
      } pick_reset{ctx};
      best.ms = INFINITY;
      int timed = 0;
      for (const TuneChoice& v : vars) {
        comm_opts o = *opts;
        o.cache_pq = v.cache_pq;
        ctx->pick = v;
        if ((rc = reset())) return rc;
        // one untimed iteration (workspace growth, first touch), then reps timed
        rc = jcomm_variant(ctx, x, &sm, &o, nullptr, st);
        if (rc == COMM_ENOMEM && v.cache_pq) continue;  // no room for the cache
        if (rc) return rc;
        if ((rc = reset())) return rc;
        HIP_TRY(hipEventRecord(sc.ev[0], st));
        for (int r = 0; r < reps; ++r)
          if ((rc = jcomm_variant(ctx, x, &sm, &o, nullptr, st))) return rc;
        HIP_TRY(hipEventRecord(sc.ev[1], st));
        HIP_TRY(hipEventSynchronize(sc.ev[1]));
        float el = 0.0f;
        HIP_TRY(hipEventElapsedTime(&el, sc.ev[0], sc.ev[1]));
        const double per = (double)el / reps;
        ++timed;
        if (std::isnan(t[v.cache_pq]) || per < t[v.cache_pq]) t[v.cache_pq] = per;
        // ties go to the earlier variant (the list starts with the defaults)
        if (per < best.ms) {
          best = v;
          best.ms = per;
        }
      }
      HIP_TRY(hipStreamSynchronize(st));
      best.variants = timed;
    }
    ctx->tune[tune_key(x, model, opts)] = best;
    // a captured batch may have resolved its options with the old table; its
    // last replay ends before the graph goes
    if ((rc = batch_sync_all(ctx, st))) return rc;
    if ((rc = batch_drop_graph(ctx))) return rc;
    if (choice) *choice = best.cache_pq;
    if (ms) {
      ms[0] = t[0];
      ms[1] = t[1];
    }
    ctx->last_stream = st;
    return COMM_OK;
  });
}

int comm_tune_lookup(comm_ctx* ctx, const comm_dense* x, const comm_model* model, const comm_opts* opts,
                     comm_tune_entry* out) {
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    if (!out) return fail(COMM_EINVAL, "out is NULL");
    int rc = tune_key_check(x, model, opts);
    if (rc) return rc;
    const auto it = ctx->tune.find(tune_key(x, model, opts));
    *out = comm_tune_entry{};
    out->found = it != ctx->tune.end();
    const TuneChoice c = out->found ? it->second : TuneChoice();
    out->cache_pq = c.cache_pq;
    out->wshare = model->kind == COMM_CP && x->ndim == 3 && opts->beta != 1.0 ? (int)cp_wshare(opts, c) : -1;
    out->tk_groups = model->kind == COMM_TUCKER && x->ndim == 3 ? (c.tk_groups ? c.tk_groups : kTkGroupsDefault) : 0;
    out->cp_tile = model->kind == COMM_CP ? (cp_narrow(model->rank, opts, c) ? 16 : 32) : 0;
    out->variants = out->found ? c.variants : 0;
    out->ms = out->found && c.variants > 0 ? c.ms : NAN;
    return COMM_OK;
  });
}

int comm_tune_set(comm_ctx* ctx, const comm_dense* x, const comm_model* model, const comm_opts* opts,
                  const comm_tune_entry* entry, void* stream) {
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    if (!entry) return fail(COMM_EINVAL, "entry is NULL");
    int rc = tune_key_check(x, model, opts);
    if (rc) return rc;
    const bool cp3 = model->kind == COMM_CP && x->ndim == 3 && opts->beta != 1.0;
    const bool tk3 = model->kind == COMM_TUCKER && x->ndim == 3;
    if (entry->cache_pq != 0 && entry->cache_pq != 1)
      return fail(COMM_EINVAL, "cache_pq = %d (0 or 1)", entry->cache_pq);
    if (entry->cache_pq && opts->beta == 1.0) return fail(COMM_EINVAL, "cache_pq = 1 at beta = 1 (nothing to cache)");
    if (entry->wshare < -1 || entry->wshare > 1 || (entry->wshare != -1 && !cp3))
      return fail(COMM_EINVAL, "wshare = %d (-1, or 0 / 1 for dense CP of order 3 at beta != 1)", entry->wshare);
    if (entry->tk_groups < 0 || entry->tk_groups > kTkGroupsLimit || (entry->tk_groups && !tk3))
      return fail(COMM_EINVAL, "tk_groups = %d (0, or 1 to %d for dense Tucker of order 3)", entry->tk_groups,
                  kTkGroupsLimit);
    const bool narrow_ok = model->kind == COMM_CP && model->rank <= 16 && opts->precision != COMM_BF16;
    if (!(entry->cp_tile == 0 || (entry->cp_tile == 32 && model->kind == COMM_CP) ||
          (entry->cp_tile == 16 && narrow_ok)))
      return fail(COMM_EINVAL, "cp_tile = %d (0; 32 for CP; 16 for CP at rank <= 16 with float32 tiles)",
                  entry->cp_tile);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    TuneChoice c;
    c.cache_pq = entry->cache_pq;
    c.wshare = entry->wshare;
    c.tk_groups = entry->tk_groups;
    c.cp_tile = entry->cp_tile == 32 ? 32 : 0;
    c.variants = 0;
    c.ms = NAN;
    // a captured batch may have resolved its options with the old entry
    if ((rc = batch_sync_all(ctx, st))) return rc;
    if ((rc = batch_drop_graph(ctx))) return rc;
    ctx->tune[tune_key(x, model, opts)] = c;
    ctx->last_stream = st;
    return COMM_OK;
  });
}

int comm_jcomm_outer_batched(comm_ctx* ctx, const comm_problem* problems, int count, int flags, void* stream) {
  const TraceRange trace_range("comm_jcomm_outer_batched");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    if (count < 0 || (count > 0 && !problems)) return fail(COMM_EINVAL, "count = %d with problems = %p", count,
                                                           (const void*)problems);
    if (flags & ~(COMM_BATCH_GRAPH | COMM_BATCH_GROUPED)) return fail(COMM_EINVAL, "unknown flags 0x%x", flags);
    // every problem's arguments before anything touches the device
    for (int p = 0; p < count; ++p) {
      const comm_problem& q = problems[p];
      if (!q.x || !q.model || !q.opts) return fail(COMM_EINVAL, "problem %d: x, model and opts must not be NULL", p);
      const int vrc = jcomm_check(q.x, q.model, q.opts);
      if (vrc) {
        std::string msg = g_last_error;
        return fail(vrc, "problem %d: %s", p, msg.c_str());
      }
    }
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    rc = jcomm_batched(ctx, problems, count, flags, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_beta_objective(comm_ctx* ctx, const comm_dense* x, const comm_model* model, const comm_opts* opts,
                        double* out_dev, void* stream) {
  const TraceRange trace_range("comm_beta_objective");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    if (!out_dev) return fail(COMM_EINVAL, "out_dev is NULL");
    int rc = check_opts(opts, false);
    if (!rc) rc = check_dense(x);
    if (rc) return rc;
    if (!model) return fail(COMM_EINVAL, "model is NULL");
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (model->kind == COMM_CP) {
      if ((rc = check_cp_model(model, x->ndim))) return rc;
      if ((rc = input_check_dense(ctx, x, model, opts, st))) return rc;
      rc = cp_objective(ctx, x, model, opts, out_dev, st);
    } else if (model->kind == COMM_TUCKER) {
      if ((rc = tucker_check_model(model, x))) return rc;
      if ((rc = input_check_dense(ctx, x, model, opts, st))) return rc;
      rc = tucker_objective(ctx, x, model, opts, out_dev, st);
    } else {
      return fail(COMM_EINVAL, "model kind %d", model->kind);
    }
    ctx->last_stream = st;
    return rc;
  });
}

int comm_tucker_update(comm_ctx* ctx, const comm_dense* x, comm_model* model, int block, const comm_opts* opts,
                       void* stream) {
  const TraceRange trace_range("comm_tucker_update");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = check_opts(opts, false);
    if (!rc) rc = check_dense(x);
    if (!rc) rc = tucker_check_model(model, x);
    if (rc) return rc;
    if (block < -2 || block >= x->ndim) return fail(COMM_EINVAL, "block = %d", block);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_dense(ctx, x, model, opts, st))) return rc;
    rc = tucker_bcomm(ctx, x, model, block, opts, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_cp_jcomm_outer_coo(comm_ctx* ctx, const comm_coo* x, comm_model* model, const comm_opts* opts,
                            double* obj_ref_dev, void* stream) {
  const TraceRange trace_range("comm_cp_jcomm_outer_coo");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    if (opts && opts->beta != 1.0) {
      int rc = check_coo_beta(x, model, opts, true);
      if (rc) return rc;
      if (model->kind != COMM_CP) return fail(COMM_EINVAL, "model kind is not CP");
      if ((rc = set_device(ctx))) return rc;
      hipStream_t st = (hipStream_t)stream;
      if ((rc = input_check_coo(ctx, x, model, opts, st))) return rc;
      rc = coo_beta_jcomm(ctx, x, model, opts, obj_ref_dev, st);
      ctx->last_stream = st;
      return rc;
    }
    int rc = check_coo(x);
    if (!rc) rc = check_coo_job(x->ndim, x->dims, model, opts);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_coo(ctx, x, model, opts, st))) return rc;
    rc = coo_jcomm_kl(ctx, x, model, opts, obj_ref_dev, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_cp_update_coo(comm_ctx* ctx, const comm_coo* x, comm_model* model, int block, const comm_opts* opts,
                       void* stream) {
  const TraceRange trace_range("comm_cp_update_coo");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = check_coo_beta(x, model, opts, false);
    if (rc) return rc;
    if (model->kind != COMM_CP) return fail(COMM_EINVAL, "model kind is not CP");
    if (block < -1 || block >= x->ndim) return fail(COMM_EINVAL, "block = %d", block);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_coo(ctx, x, model, opts, st))) return rc;
    rc = coo_beta_bcomm(ctx, x, model, block, opts, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_tucker_update_coo(comm_ctx* ctx, const comm_coo* x, comm_model* model, int block, const comm_opts* opts,
                           void* stream) {
  const TraceRange trace_range("comm_tucker_update_coo");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = check_coo_beta(x, model, opts, false);
    if (rc) return rc;
    if (model->kind != COMM_TUCKER) return fail(COMM_EINVAL, "model kind is not Tucker");
    if (block < -2 || block >= x->ndim) return fail(COMM_EINVAL, "block = %d", block);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_coo(ctx, x, model, opts, st))) return rc;
    rc = coo_tucker(ctx, x, model, block, opts, nullptr, false, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_tucker_jcomm_outer_coo(comm_ctx* ctx, const comm_coo* x, comm_model* model, const comm_opts* opts,
                                double* obj_ref_dev, void* stream) {
  const TraceRange trace_range("comm_tucker_jcomm_outer_coo");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = check_coo_beta(x, model, opts, true);
    if (rc) return rc;
    if (model->kind != COMM_TUCKER) return fail(COMM_EINVAL, "model kind is not Tucker");
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_coo(ctx, x, model, opts, st))) return rc;
    rc = coo_tucker(ctx, x, model, -2, opts, obj_ref_dev, true, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_beta_objective_coo(comm_ctx* ctx, const comm_coo* x, const comm_model* model, const comm_opts* opts,
                            double* out_dev, void* stream) {
  const TraceRange trace_range("comm_beta_objective_coo");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    if (!out_dev) return fail(COMM_EINVAL, "out_dev is NULL");
    int rc;
    if (opts && opts->beta == 1.0 && model && model->kind == COMM_CP) {
      // closed form over the zero cells: no dense twin, orders 2 to 5
      rc = check_coo(x, COMM_MAX_NDIM);
      if (!rc) rc = check_opts(opts, false);
      if (!rc) rc = check_cp_model(model, x->ndim);
      if (rc) return rc;
      if ((rc = set_device(ctx))) return rc;
      hipStream_t st = (hipStream_t)stream;
      if ((rc = input_check_coo(ctx, x, model, opts, st))) return rc;
      rc = coo_objective_kl(ctx, x, model, opts, out_dev, st);
      ctx->last_stream = st;
      return rc;
    }
    rc = check_coo_beta(x, model, opts, false);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_coo(ctx, x, model, opts, st))) return rc;
    rc = coo_beta_objective(ctx, x, model, opts, out_dev, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_coo_plan_create(comm_ctx* ctx, const comm_coo* x, comm_coo_plan** out, void* stream) {
  const TraceRange trace_range("comm_coo_plan_create");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    if (!out) return fail(COMM_EINVAL, "out is NULL");
    int rc = check_coo(x);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    rc = coo_plan_build(ctx, x, out, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_coo_plan_destroy(comm_coo_plan* plan) {
  return guarded([&]() -> int { return coo_plan_free(plan); });
}

int comm_cp_jcomm_outer_coo_plan(comm_ctx* ctx, const comm_coo_plan* plan, comm_model* model, const comm_opts* opts,
                                 double* obj_ref_dev, void* stream) {
  const TraceRange trace_range("comm_cp_jcomm_outer_coo_plan");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    if (!plan) return fail(COMM_EINVAL, "plan is NULL");
    int64_t dims[4] = {0, 0, 0, 0};
    const int N = coo_plan_ndim(plan);
    for (int n = 0; n < N; ++n) dims[n] = coo_plan_dim(plan, n);
    int rc = check_coo_job(N, dims, model, opts);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check(ctx, nullptr, 0, model, N, dims, opts, st))) return rc;
    rc = coo_jcomm_kl_plan(ctx, plan, model, opts, obj_ref_dev, st);
    ctx->last_stream = st;
    return rc;
  });
}

int comm_bcomm_sweep_extrap(comm_ctx* ctx, const comm_dense* x, comm_model* model, comm_model* prev,
                            const comm_opts* opts, const comm_extrap* extrap, float* alpha_dev, void* stream) {
  const TraceRange trace_range("comm_bcomm_sweep_extrap");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = check_opts(opts, false);
    if (!rc) rc = check_dense(x);
    if (rc) return rc;
    if (!model) return fail(COMM_EINVAL, "model is NULL");
    if (model->kind == COMM_CP) rc = check_cp_model(model, x->ndim);
    else if (model->kind == COMM_TUCKER) rc = tucker_check_model(model, x);
    else rc = fail(COMM_EINVAL, "model kind %d", model->kind);
    if (!rc) rc = check_extrap(x, model, prev, extrap);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    if ((rc = ensure_aux(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_dense(ctx, x, model, opts, st))) return rc;
    float* alpha = alpha_dev ? alpha_dev : ctx->aux;
    if ((rc = extrap_alpha(x, model, prev, extrap, alpha, st))) return rc;
    // each block is moved just before its own update (Tucker: core, then modes)
    const bool tk = model->kind == COMM_TUCKER;
    const int nb = x->ndim + (tk ? 1 : 0);
    for (int b = 0; b < nb && !rc; ++b) {
      if ((rc = extrap_apply(x, model, prev, b, alpha, (float)opts->eps, st))) break;
      const int blk = tk ? b - 1 : b;
      rc = tk ? tucker_bcomm(ctx, x, model, blk, opts, st) : cp_bcomm(ctx, x, model, blk, opts, st);
    }
    ctx->last_stream = st;
    return rc;
  });
}

int comm_jcomm_outer_extrap(comm_ctx* ctx, const comm_dense* x, comm_model* model, comm_model* prev,
                            const comm_opts* opts, const comm_extrap* extrap, double* obj_ref_dev, float* alpha_dev,
                            void* stream) {
  const TraceRange trace_range("comm_jcomm_outer_extrap");
  return guarded([&]() -> int {
    if (!ctx) return fail(COMM_EINVAL, "ctx is NULL");
    int rc = jcomm_check(x, model, opts);
    if (!rc) rc = check_extrap(x, model, prev, extrap);
    if (rc) return rc;
    if ((rc = set_device(ctx))) return rc;
    if ((rc = ensure_aux(ctx))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = input_check_dense(ctx, x, model, opts, st))) return rc;
    float* alpha = alpha_dev ? alpha_dev : ctx->aux;
    if ((rc = extrap_alpha(x, model, prev, extrap, alpha, st))) return rc;
    // the outer reference is the extrapolated model; the inner iterate starts there
    if ((rc = extrap_apply(x, model, prev, -1, alpha, (float)opts->eps, st))) return rc;
    rc = jcomm_run(ctx, x, model, opts, obj_ref_dev, st);
    ctx->last_stream = st;
    return rc;
  });
}

}  // extern "C"
