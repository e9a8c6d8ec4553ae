// Host driver and C ABI of the flexibly enlarged CG solver (see include/ecg.h).
//
// The iteration (Section 4.3, Algorithm 3; Algorithm 1 without a switch):
//   k = 1      : candidate = [T^t(r_0)]                       (split kernel)
//   switch     : candidate = [T^{t/2}(r_{k-1})] on part >> l  (Section 4.2)
//   otherwise  : candidate = A W_{k-1}  (= Z_{k-1}, produced by the previous update)
//   CGS2       : twice  Y = A C, G = Q^T Y, C -= Q G          (A-orthonormalise vs Q)
//   Pre-CholQR : E = C^T C = R^T R, H = C R^{-1}, Y = A H, S = H^T Y = C'^T C',
//                u = H^T r                                    (self A-orthonormalisation)
//   update     : W_k = H C'^{-1} (stored), Z_k = Y C'^{-1}, alpha = C'^{-T} u,
//                x += H C'^{-1} alpha, r -= Y C'^{-1} alpha, rho = ||r||
// Split preconditioning (Section 4.5, eq. (zsre2)) only changes the candidate:
//   L^{-T}[T(L^{-1} r)] at k = 1 / at a switch, L^{-T} L^{-1} Z_{k-1} otherwise.
// One 24-byte device-to-host copy per iteration carries ||r||^2 and the kept-column counts.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ecg.h"
#include "ecg_internal.h"

using namespace ecg;

struct ecg_operator {
  DevCsr A;
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> rowptr;  // host copy (set-up of preconditioners)
  std::vector<int32_t> col;
  std::vector<double> val;
};

struct ecg_partition {
  int64_t n = 0;
  int t = 0;
  int* part = nullptr;  // device
  std::vector<int32_t> host;
};

struct ecg_precond {
  int kind = 0;  // 0: triangular factor L (block-Jacobi IC(0)); 1: G with M^{-1} = G G^T;
                 // 2: block-Jacobi exact Cholesky in band panel form
  DevTri tri;
  DevCsr G, Gt;  // kind 1
  DevBand band;  // kind 2
  std::vector<void*> owned;
};

namespace ecg {
bool g_stats_on = false;
}
static int g_progress_every = 0;

namespace {

thread_local std::string g_err;

// ------------------------------------------------------------------ kernel timing
struct PendingStat {
  int cls;
  hipEvent_t a, b;
  double bytes, flops;
};
std::vector<hipEvent_t> g_event_pool;
std::vector<PendingStat> g_pending;
hipEvent_t g_open = nullptr;
ecg_kernel_stats g_stats;

hipEvent_t take_event() {
  if (g_event_pool.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = g_event_pool.back();
  g_event_pool.pop_back();
  return e;
}

// Fold the recorded event pairs into g_stats (the stream has been synchronised).
void flush_stats() {
  for (const PendingStat& p : g_pending) {
    float ms = 0.f;
    if (p.a && p.b && hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_stats.count[p.cls] += 1;
      g_stats.ms[p.cls] += ms;
      g_stats.bytes[p.cls] += p.bytes;
      g_stats.flops[p.cls] += p.flops;
    }
    if (p.a) g_event_pool.push_back(p.a);
    if (p.b) g_event_pool.push_back(p.b);
  }
  g_pending.clear();
}

ecg_status fail(ecg_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(ECG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// ------------------------------------------------------------------ workspace plan
struct Plan {
  int n = 0, t0 = 0, t0p = 0, elt = 8;
  long long cap = 0;  // stored-block arena capacity, in columns of n values
  size_t off_status = 0, off_small_part = 0, off_small_out = 0, off_ref = 0, off_rinv = 0, off_cinv = 0, off_beta = 0,
         off_norm_part = 0, off_scalar = 0, off_gram_part = 0, off_G = 0, off_C = 0, off_Y = 0, off_H = 0,
         off_r = 0, off_r64 = 0, off_d = 0, off_v1 = 0, off_v2 = 0, off_Q = 0, total = 0;
  size_t gram_part_cap = 0;  // elements of T
  size_t slot_elems = 0;
};

ecg_status make_plan(int64_t n, int t, const ecg_options& o, Plan* p) {
  p->n = (int)n;
  p->t0 = t;
  p->t0p = pow2_at_least(t);
  p->elt = o.precision == ECG_FP32_REFINED ? 4 : 8;
  const int tp = p->t0p;
  p->slot_elems = (size_t)n * tp;
  const size_t slot_bytes = p->slot_elems * p->elt;
  const size_t col_bytes = (size_t)n * p->elt;
  long long cap;  // columns
  if (o.q_budget_bytes > 0) {
    cap = (long long)(o.q_budget_bytes / (int64_t)col_bytes);
  } else if (o.trunc > 0) {
    cap = (long long)o.trunc * tp;
  } else {
    cap = (long long)std::max(1, o.kmax - 1) * tp;
  }
  if (o.trunc > 0) cap = std::min<long long>(cap, (long long)o.trunc * tp);
  if (o.restart == ECG_RESTART_EVERY && o.q_budget_bytes == 0)  // one cycle at a time
    cap = std::min<long long>(cap, (long long)o.restart_every * tp);
  if (cap < tp) return fail(ECG_EINVAL, "q_budget_bytes is smaller than one stored block");
  p->cap = cap;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  const size_t small_len = (size_t)tp * tp + tp;
  const size_t small_chunks = std::min<size_t>(kSmallChunks, ((size_t)n + 255) / 256);
  p->off_status = take(sizeof(IterStatus));
  p->off_small_part = take((small_chunks + 32) * small_len * 8);  // chunks + stage-2 rows
  p->off_small_out = take(small_len * 8);
  p->off_ref = take(small_len * 8);  // candidate Gram before CGS2 / MSDO's V^T r
  p->off_rinv = take((size_t)tp * tp * 8);
  p->off_cinv = take((size_t)tp * tp * 8);
  p->off_beta = take((size_t)tp * 8);
  p->off_norm_part = take(((size_t)n / 4 + 64 + 128) * 8);  // partials + stage-2 slices
  p->off_scalar = take(64 * 8);
  // elements: partial Gram sums of the row chunks (at most one chunk per 256 rows) and the
  // first-stage sums of their reduction, capped at 2^26; the launcher uses fewer chunks when
  // they would not fit
  p->gram_part_cap = std::min<size_t>((size_t)1 << 26, ((size_t)n / 256 + 1 + 32) * (size_t)cap * tp);
  p->off_gram_part = take(p->gram_part_cap * p->elt);
  p->off_G = take((size_t)cap * tp * p->elt);
  p->off_C = take(slot_bytes);
  p->off_Y = take(slot_bytes);
  p->off_H = take(slot_bytes);
  p->off_r = take((size_t)n * p->elt);
  p->off_v1 = take((size_t)n * 8);
  p->off_v2 = take((size_t)n * 8);
  if (o.precision == ECG_FP32_REFINED) {
    p->off_r64 = take((size_t)n * 8);
    p->off_d = take((size_t)n * 8);
  }
  p->off_Q = take((size_t)cap * col_bytes);
  p->total = off;
  return ECG_OK;
}

ecg_status check_options(const ecg_options* o) {
  if (!o) return fail(ECG_EINVAL, "options is NULL");
  if (!(o->tol >= 0.0)) return fail(ECG_EINVAL, "tol must be >= 0");
  if (o->kmax < 1) return fail(ECG_EINVAL, "kmax must be >= 1");
  if (o->reduce < 0 || o->reduce > 3) return fail(ECG_EINVAL, "unknown reduction rule");
  if (o->t_min < 1) return fail(ECG_EINVAL, "t_min must be >= 1");
  if (o->min_gap < 1) return fail(ECG_EINVAL, "min_gap must be >= 1");
  if (o->reduce == ECG_REDUCE_SCHEDULE && o->n_schedule > 0 && !o->schedule)
    return fail(ECG_EINVAL, "schedule is NULL");
  if (o->precision != ECG_FP64 && o->precision != ECG_FP32_REFINED) return fail(ECG_EINVAL, "unknown precision");
  if (o->precision == ECG_FP32_REFINED && (o->max_outer < 1 || !(o->inner_tol > 0.0)))
    return fail(ECG_EINVAL, "FP32_REFINED needs max_outer >= 1 and inner_tol > 0");
  if (o->trunc < 0 || o->q_budget_bytes < 0 || o->replace_every < 0) return fail(ECG_EINVAL, "negative size option");
  if (o->precond != ECG_PRECOND_NONE && o->precond != ECG_PRECOND_SPLIT) return fail(ECG_EINVAL, "unknown precond");
  if (o->precond == ECG_PRECOND_SPLIT && !o->M) return fail(ECG_EINVAL, "precond SPLIT needs M");
  if (o->variant < ECG_SRE_CG2 || o->variant > ECG_MODIFIED_MSDO) return fail(ECG_EINVAL, "unknown variant");
  if (o->restart < ECG_RESTART_NONE || o->restart > ECG_RESTART_TOL) return fail(ECG_EINVAL, "unknown restart rule");
  if (o->restart == ECG_RESTART_EVERY && o->restart_every < 1) return fail(ECG_EINVAL, "restart_every must be >= 1");
  if (o->max_restarts < 0) return fail(ECG_EINVAL, "max_restarts must be >= 0");
  if (o->refine_keep_q < 0 || o->refine_keep_q > 2) return fail(ECG_EINVAL, "refine_keep_q must be 0, 1 or 2");
  return ECG_OK;
}

// A halving merges subdomains 2i and 2i+1 (Section 4), so every width that is halved must be
// even: the halvings the rule can make (down to t_min) are checked before any device work.
ecg_status check_halving(int t, const ecg_options& o) {
  const int tmin = std::max(o.t_min, 1);
  int steps = 0;
  if (o.reduce == ECG_REDUCE_SWITCHTOL_ONCE) steps = 1;
  else if (o.reduce == ECG_REDUCE_SWITCHTOL_REPEAT) steps = 64;
  else if (o.reduce == ECG_REDUCE_SCHEDULE) steps = o.n_schedule;
  for (int w = t, i = 0; i < steps && w / 2 >= tmin; ++i, w /= 2)
    if (w % 2) return fail(ECG_EINVAL, "halving requested at odd block width " + std::to_string(w));
  return ECG_OK;
}

// ------------------------------------------------------------------ stored blocks (arena)
// The stored blocks live in a circular arena of `cap` columns (n values each).  A block
// of width w occupies w consecutive columns, laid out row-major [n][w].  A new block goes
// right after the previous one (or at column 0 when it would run past the end); the
// oldest blocks are dropped until it no longer overlaps a stored block, so the arena
// always holds the most recent blocks (truncation, Section 3, when memory runs out).
struct QBlock {
  long long off;  // first column
  int width;
};
struct QStore {
  long long cap = 0;
  long long head = 0;
  std::deque<QBlock> blocks;  // creation order, oldest first
  long long dropped = 0;      // blocks evicted for lack of room
  // column offset for the next block of width w; evicts what it overlaps
  long long place(int w) {
    long long off = head;
    if (off + w > cap) off = 0;
    auto overlaps = [&](const QBlock& b) { return b.off < off + w && off < b.off + b.width; };
    while (!blocks.empty() && std::any_of(blocks.begin(), blocks.end(), overlaps)) {
      blocks.pop_front();
      ++dropped;
    }
    return off;
  }
  void push(long long off, int w) {
    blocks.push_back(QBlock{off, w});
    head = off + w;
  }
  void clear() {  // a restart: every stored block is discarded
    blocks.clear();
    head = 0;
  }
};

template <typename T>
int build_spans(const QStore& q, int trunc, T* Qbase, int n, std::vector<Span<T>>& spans) {
  spans.clear();
  const long long total = (long long)q.blocks.size();
  const long long nact = trunc > 0 ? std::min<long long>(total, trunc) : total;
  int goff = 0;
  for (long long j = total - nact; j < total; ++j) {
    const QBlock& b = q.blocks[j];
    if (!spans.empty()) {
      Span<T>& s = spans.back();
      const QBlock& prev = q.blocks[j - 1];
      if (s.width == b.width && prev.width == b.width && b.off == prev.off + prev.width) {
        s.nblk += 1;
        goff += b.width;
        continue;
      }
    }
    Span<T> s;
    s.base = Qbase + (size_t)b.off * n;
    s.stride = (long long)b.width * n;
    s.nblk = 1;
    s.width = b.width;
    s.goff = goff;
    spans.push_back(s);
    goff += b.width;
  }
  return goff;  // m
}

bool restart_now(const ecg_options& o, int k, double tol1, const std::vector<int>& restarts) {
  switch (o.restart) {
    case ECG_RESTART_EVERY:
      return (k - 1) % o.restart_every == 0;  // k mod j == 1
    case ECG_RESTART_TOL:
      return tol1 < o.restart_tol && (o.max_restarts == 0 || (int)restarts.size() < o.max_restarts);
  }
  return false;
}

bool switch_now(const ecg_options& o, int k, double tol1, int t_live, const std::vector<int>& switches) {
  if (t_live % 2 || t_live / 2 < std::max(o.t_min, 1)) return false;
  switch (o.reduce) {
    case ECG_REDUCE_NONE:
      return false;
    case ECG_REDUCE_SCHEDULE:
      for (int i = 0; i < o.n_schedule; ++i)
        if (o.schedule[i] == k) return true;
      return false;
    case ECG_REDUCE_SWITCHTOL_ONCE:
      return tol1 < o.switch_tol && switches.empty();
    case ECG_REDUCE_SWITCHTOL_REPEAT:
      return tol1 < o.switch_tol && (switches.empty() || k - switches.back() >= o.min_gap);
  }
  return false;
}

template <typename T>
const T* vals(const DevCsr& A);
template <>
const double* vals<double>(const DevCsr& A) { return A.val; }
template <>
const float* vals<float>(const DevCsr& A) { return A.valf; }

// Y = L^{-1} X (which 0) or L^{-T} X (which 1); for M^{-1} = G G^T: L^{-1} = G^T, L^{-T} = G.
template <typename T>
void precond_apply(const ecg_precond* M, int which, int tc, const T* X, T* Y, hipStream_t s) {
  if (M->kind == 0) {
    launch_trisolve<T>(M->tri, which, tc, X, Y, s);
  } else if (M->kind == 2) {
    launch_band_solve<T>(M->band, which, tc, X, Y, s);
  } else {
    launch_spmm<T>(which == 0 ? M->Gt : M->G, tc, X, Y, s);
  }
}

struct InnerResult {
  int kmax_left = 0x7fffffff;  // iteration budget left for this solve (all refinement steps)
  bool stagnated = false;
  long long dropped = 0;  // stored blocks evicted for lack of room
  int iters = 0;
  int deflated = 0;
  long long mem = 0;
  long long mem_peak = 0;  // largest sum of widths within one restart cycle
  std::vector<int> switches;
  std::vector<int> restarts;
  int t_final = 0;
  double rho0 = 0, rho = 0;
  ecg_status status = ECG_OK;
};

// One ECG solve on residual r (in place) accumulating the correction into x.
// rr0 = ||r||^2 on entry.  base_k offsets the iteration numbers of rho_hist/report.
// Adaptive rule of refine_keep_q: blocks kept from the previous refinement step stay only if
// re-projecting the new residual on them leaves at most this fraction of its norm.
constexpr double kKeepGain = 0.5;

// qkeep: stored blocks kept from an earlier inner solve (and left for the next one), or
// nullptr for an empty store of this solve's own.
template <typename T, typename TX>
ecg_status ecg_inner(const ecg_operator* Aop, const ecg_partition* P, const ecg_options& o, const Plan& pl,
                     char* ws, TX* x, T* r, double rr0, double tol, const double* b64_for_replace,
                     hipStream_t s, InnerResult* res, double* rho_hist, QStore* qkeep = nullptr) {
  const DevCsr& A = Aop->A;
  const int n = pl.n;
  const ecg_precond* M = (o.precond == ECG_PRECOND_SPLIT) ? o.M : nullptr;
  IterStatus* st = reinterpret_cast<IterStatus*>(ws + pl.off_status);
  double* small_part = reinterpret_cast<double*>(ws + pl.off_small_part);
  double* small_out = reinterpret_cast<double*>(ws + pl.off_small_out);
  double* refg = reinterpret_cast<double*>(ws + pl.off_ref);
  double* Rinv = reinterpret_cast<double*>(ws + pl.off_rinv);
  double* Cinv = reinterpret_cast<double*>(ws + pl.off_cinv);
  double* beta = reinterpret_cast<double*>(ws + pl.off_beta);
  double* norm_part = reinterpret_cast<double*>(ws + pl.off_norm_part);
  T* gram_part = reinterpret_cast<T*>(ws + pl.off_gram_part);
  T* G = reinterpret_cast<T*>(ws + pl.off_G);
  T* Cb = reinterpret_cast<T*>(ws + pl.off_C);
  T* Yb = reinterpret_cast<T*>(ws + pl.off_Y);
  T* Hb = reinterpret_cast<T*>(ws + pl.off_H);
  T* Qbase = reinterpret_cast<T*>(ws + pl.off_Q);

  QStore qown;
  qown.cap = pl.cap;
  QStore& q = qkeep ? *qkeep : qown;
  const long long dropped_before = q.dropped;
  std::vector<Span<T>> spans;
  IterStatus hst;

  // After r was recomputed from x (FP32 form with kept blocks): x += Q (Q^T r) restores the
  // Galerkin condition Q^T r = 0 on the stored blocks, then r = b - A x again in FP64.
  // Returns ||r||^2 in *rr_out (unchanged when nothing is stored).
  auto reproject = [&](double* rr_out) -> ecg_status {
    if constexpr (std::is_same<T, float>::value && std::is_same<TX, double>::value) {
      const int m = build_spans<T>(q, o.trunc, Qbase, n, spans);
      if (m == 0) return ECG_OK;
      launch_gram<T>(n, spans.data(), (int)spans.size(), m, 1, r, G, gram_part, pl.gram_part_cap, s);
      launch_zero(Hb, (size_t)n * sizeof(T), s);
      launch_update<T>(n, spans.data(), (int)spans.size(), 1, G, Hb, s);  // Hb = -Q (Q^T r)
      launch_axpy_f2d(n, Hb, x, s, -1.0);
      const int g = launch_residual_f(A, b64_for_replace, x, r, norm_part, s);
      launch_sum(norm_part, g, &st->rr, s);
      HIPCHK(hipMemcpyAsync(&hst, st, sizeof(IterStatus), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      *rr_out = std::max(hst.rr, 0.0);
    }
    return ECG_OK;
  };

  const double rho0 = std::sqrt(rr0);
  res->rho0 = rho0;
  res->rho = rho0;
  res->t_final = P->t;
  if (rho_hist) rho_hist[0] = rho0;
  if (rho0 == 0.0) return ECG_OK;
  const double tau = (sizeof(T) == 4 && o.deflate_tol >= 0.0) ? std::max(o.deflate_tol, 1e-10) : o.deflate_tol;

  double rho_prev = rho0, tol1 = 1.0;
  double rho_cyc = rho0, tol1_cyc = 1.0;  // restart statistic, relative to the cycle's first residual
  int k = 1, level = 0;
  const auto t_begin = std::chrono::steady_clock::now();
  int tl = P->t;                 // live width
  int tc = pow2_at_least(tl);    // padded width of the kernels
  int prev_kept = tl;
  long long cycle_mem = 0;
  std::vector<double> replaced;  // true residual norms at the residual replacements
  const int kmax = std::max(1, std::min(o.kmax, res->kmax_left));
  if (qkeep && b64_for_replace && !q.blocks.empty()) {
    // a refinement step starting from kept blocks: re-project; under the adaptive rule the
    // blocks are kept only if they hold a real part of the new residual
    double rr = rr0;
    ecg_status est = reproject(&rr);
    if (est != ECG_OK) return est;
    const double gain = rr0 > 0 ? std::sqrt(rr / rr0) : 0.0;
    const bool keep = o.refine_keep_q != 2 || gain <= kKeepGain;
    if (g_progress_every > 0) {
      std::fprintf(stderr, "ecg: refinement step: re-projection on %lld stored columns leaves %.3f of the residual; "
                   "blocks %s\n", (long long)build_spans<T>(q, o.trunc, Qbase, n, spans), gain,
                   keep ? "kept" : "dropped");
      std::fflush(stderr);
    }
    if (!keep) q.clear();
    rho_prev = std::sqrt(rr);
  }
  while (rho_prev > tol * rho0 && k < kmax) {
    // ---- candidate block (cand_live: its columns that are not already known zero)
    bool from_r = false;
    if (k == 1) {
      from_r = true;
    } else if (switch_now(o, k, tol1, tl, res->switches)) {
      level += 1;
      tl /= 2;
      tc = pow2_at_least(tl);
      res->switches.push_back(k);
      from_r = true;
      if (o.restart_at_switch) {
        q.clear();
        cycle_mem = 0;
        rho_cyc = rho_prev;
        res->restarts.push_back(k);
      }
    } else if (restart_now(o, k, tol1_cyc, res->restarts)) {
      q.clear();  // Q is emptied; the candidate comes from the residual (Section 3)
      cycle_mem = 0;
      rho_cyc = rho_prev;
      res->restarts.push_back(k);
      from_r = true;
    }
    if (o.variant == ECG_MODIFIED_MSDO) from_r = true;
    const bool msdo = (o.variant == ECG_MSDO_CG) && !from_r;
    if (msdo) {
      // beta_k = -V_{k-1}^T (M^{-1}) r_{k-1}; Cb holds V_{k-1} = A P_{k-1}
      const T* rr = r;
      if (M) {
        precond_apply<T>(M, 0, 1, r, Yb, s);
        precond_apply<T>(M, 1, 1, Yb, Hb, s);  // M^{-1} r (n x 1)
        rr = Hb;
      }
      launch_small_gram<T>(n, tc, Cb, Cb, rr, small_part, refg, s);  // refg[tc*tc..] = V^T rr
    }
    if (from_r || msdo) {
      T* dst = msdo ? Yb : Cb;  // MSDO: the split term goes next to P_{k-1} first
      if (M) {
        precond_apply<T>(M, 0, 1, r, Yb, s);  // L^{-1} r (n x 1)
        launch_split_t<T>(n, P->part, level, tc, Yb, Hb, s);
        precond_apply<T>(M, 1, tc, Hb, dst, s);
      } else {
        launch_split_t<T>(n, P->part, level, tc, r, dst, s);
      }
      if (msdo) {
        const QBlock& last = q.blocks.back();
        launch_msdo_combine<T>(n, tc, Yb, Qbase + (size_t)last.off * n, refg + (size_t)tc * tc, Cb, s);
      }
    } else if (M) {
      precond_apply<T>(M, 0, tc, Cb, Yb, s);  // Cb holds Z_{k-1} = A W_{k-1}
      precond_apply<T>(M, 1, tc, Yb, Cb, s);
    }
    // ---- CGS2 against the stored blocks
    const int m = build_spans<T>(q, o.trunc, Qbase, n, spans);
    if (m > 0) {
      // squared column norms before CGS2: the reference of the deflation test
      launch_small_gram<T>(n, tc, Cb, Cb, nullptr, small_part, refg, s);
      for (int pass = 0; pass < 2; ++pass) {
        launch_spmm<T>(A, tc, Cb, Yb, s);
        launch_gram<T>(n, spans.data(), (int)spans.size(), m, tc, Yb, G, gram_part, pl.gram_part_cap, s);
        launch_update<T>(n, spans.data(), (int)spans.size(), tc, G, Cb, s);
      }
    }
    // ---- Pre-CholQR: Euclidean step
    launch_zero(st, sizeof(IterStatus), s);
    const double w = sizeof(T);
    stat_begin(s);
    launch_small_gram<T>(n, tc, Cb, Cb, nullptr, small_part, small_out, s);
    stat_end(kStatSmallGram, w * n * 2 * tc, 2.0 * n * tc * tc, s);
    stat_begin(s);
    launch_factor(0, tc, tl, small_out, m > 0 ? refg : nullptr, tau, Rinv, nullptr, st, s);
    stat_end(kStatFactor, 0.0, (double)tc * tc * tc, s);
    stat_begin(s);
    launch_times_small<T>(n, tc, Cb, Rinv, Hb, s);
    stat_end(kStatTimesSmall, w * n * 2 * tc, 2.0 * n * tc * tc, s);
    // ---- A step, alpha and the fused update
    launch_spmm<T>(A, tc, Hb, Yb, s);
    stat_begin(s);
    launch_small_gram<T>(n, tc, Hb, Yb, r, small_part, small_out, s);
    stat_end(kStatSmallGram, w * n * (2 * tc + 1), 2.0 * n * tc * (tc + 1), s);
    stat_begin(s);
    launch_factor(1, tc, tl, small_out, nullptr, tau, Cinv, beta, st, s);
    stat_end(kStatFactor, 0.0, (double)tc * tc * tc, s);
    const long long woff = q.place(tc);  // may drop the oldest blocks (already used above)
    T* Wslot = Qbase + (size_t)woff * n;
    const int nwg = launch_final_update<T, TX>(n, tc, Hb, Yb, Cinv, beta, Wslot, Cb, x, r, norm_part, s);
    launch_sum(norm_part, nwg, &st->rr, s);
    HIPCHK(hipMemcpyAsync(&hst, st, sizeof(IterStatus), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    if (g_stats_on && g_pending.size() >= 4096) flush_stats();  // every recorded event has completed
    if (hst.breakdown) {
      res->status = ECG_EBREAKDOWN;
      g_err = "non-positive pivot in the t x t Cholesky with deflation disabled";
      break;
    }
    if (hst.keep_a == 0) {
      res->status = ECG_EBREAKDOWN;
      g_err = "every column of the block was deflated (search space exhausted)";
      break;
    }
    // ---- bookkeeping (block stored in its slot by the update kernel)
    q.push(woff, tc);
    res->mem += hst.keep_a;
    cycle_mem += hst.keep_a;
    res->mem_peak = std::max(res->mem_peak, cycle_mem);
    // a column dropped once stays zero in A W, so it is counted only where it is lost
    res->deflated += ((from_r || msdo) ? tl : prev_kept) - hst.keep_a;
    prev_kept = hst.keep_a;
    const double rho = std::sqrt(std::max(hst.rr, 0.0));
    tol1 = std::fabs(rho - rho_prev) / rho0;
    tol1_cyc = std::fabs(rho - rho_prev) / rho_cyc;
    rho_prev = rho;
    if (rho_hist) rho_hist[k] = rho;
    if (g_progress_every > 0 && k % g_progress_every == 0) {
      std::fprintf(stderr, "ecg: k=%d rho/rho0=%.3e t=%d m=%d elapsed=%.2fs\n", k, rho / rho0, tl, m + tc,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count());
      std::fflush(stderr);
    }
    if constexpr (std::is_same<T, float>::value) {
      // residual replacement: r = b - A x recomputed in FP64 (x accumulates in FP64)
      if (o.replace_every > 0 && b64_for_replace && k % o.replace_every == 0 &&
          rho_prev > tol * rho0) {
        const int g = launch_residual_f(A, b64_for_replace, x, r, norm_part, s);
        launch_sum(norm_part, g, &st->rr, s);
        HIPCHK(hipMemcpyAsync(&hst, st, sizeof(IterStatus), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double rr = std::max(hst.rr, 0.0);
        if (qkeep) {
          ecg_status est = reproject(&rr);
          if (est != ECG_OK) return est;
        }
        rho_prev = std::sqrt(rr);
        replaced.push_back(rho_prev);
        // stagnation: the true residual fell by less than 10% over the last four
        // replacements and at least 100 iterations; hand back to the FP64 refinement step
        const size_t nr = replaced.size();
        const size_t win = std::max<size_t>(4, (size_t)((100 + o.replace_every - 1) / o.replace_every));
        if (nr > win && replaced[nr - 1] > 0.9 * replaced[nr - 1 - win]) {
          ++k;
          res->stagnated = true;
          break;
        }
      }
    }
    ++k;
  }
  res->iters = k - 1;
  res->dropped += q.dropped - dropped_before;
  res->rho = rho_prev;
  res->t_final = tl;
  if (res->status == ECG_OK && rho_prev > tol * rho0) res->status = ECG_ENOTCONV;
  return ECG_OK;
}

ecg_status device_norm2(const DevCsr& A, const double* b, const double* x, double* tmp, double* part,
                        double* dscalar, hipStream_t s, double* out) {
  const int g = launch_residual(A, b, x, tmp, part, s);
  launch_sum(part, g, dscalar, s);
  HIPCHK(hipMemcpyAsync(out, dscalar, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

template <typename T>
ecg_status copy_in(T** dst, const T* src, size_t count, int on_device, hipStream_t s) {
  HIPCHK(hipMalloc(dst, std::max<size_t>(count, 1) * sizeof(T)));
  if (count) HIPCHK(hipMemcpyAsync(*dst, src, count * sizeof(T), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  return ECG_OK;
}

template <typename T>
ecg_status to_host(std::vector<T>& dst, const T* src, size_t count, int on_device, hipStream_t s) {
  dst.resize(count);
  if (!count) return ECG_OK;
  if (on_device) {
    HIPCHK(hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  } else {
    std::memcpy(dst.data(), src, count * sizeof(T));
  }
  return ECG_OK;
}

ecg_status check_csr(int64_t n, int64_t nnz, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci) {
  if (n <= 0 || n > 0x7fffffff) return fail(ECG_EINVAL, "n out of range");
  if (nnz < 0 || nnz >= 0x7fffffffLL) return fail(ECG_EINVAL, "nnz must be < 2^31");
  if (rp[0] != 0 || rp[n] != nnz) return fail(ECG_EINVAL, "rowptr must start at 0 and end at nnz");
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return fail(ECG_EINVAL, "rowptr not non-decreasing");
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (ci[k] < 0 || ci[k] >= n) return fail(ECG_EINVAL, "column index out of range");
      if (k > rp[i] && ci[k] <= ci[k - 1]) return fail(ECG_EINVAL, "columns of a row must be strictly increasing");
    }
  }
  return ECG_OK;
}

// Upload a host CSR (int64 rowptr) as DevCsr with an FP32 copy of the values.
// Diagonal form for the products (SpMM): kept when the matrix has at most kMaxDiag distinct
// diagonals and they are at least 70% filled, as for stencil operators on grids.
ecg_status upload_dia(int64_t n, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                      const std::vector<double>& v, hipStream_t s, DevCsr* out) {
  std::vector<int> offs;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      const long long o = (long long)ci[k] - i;
      if (std::find(offs.begin(), offs.end(), (int)o) == offs.end()) {
        offs.push_back((int)o);
        if ((int)offs.size() > kMaxDiag) return ECG_OK;  // not a few-diagonal matrix
      }
    }
  }
  if (offs.empty() || (double)v.size() < 0.7 * (double)offs.size() * (double)n) return ECG_OK;
  std::sort(offs.begin(), offs.end());
  const int nd = (int)offs.size();
  std::vector<double> dv((size_t)nd * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int d = (int)(std::lower_bound(offs.begin(), offs.end(), (int)(ci[k] - i)) - offs.begin());
      dv[(size_t)d * n + i] += v[k];  // duplicates, if any, add up as in the CSR product
    }
  ecg_status st;
  if ((st = copy_in(&out->dval, dv.data(), dv.size(), 0, s)) != ECG_OK) return st;
  HIPCHK(hipMalloc(&out->dvalf, dv.size() * sizeof(float)));
  launch_cast_val((int)dv.size(), out->dval, out->dvalf, s);
  out->ndiag = nd;
  for (int d = 0; d < kMaxDiag; ++d) out->dia.off[d] = d < nd ? offs[d] : 0;
  // grid stencil: offsets -c, -b, -a, 0, a, b, c (or -c, -a, 0, a, c) with b | c and c | n
  if ((nd == 7 || nd == 5) && offs[nd / 2] == 0) {
    bool sym = true;
    for (int d = 0; d < nd; ++d) sym = sym && offs[d] == -offs[nd - 1 - d];
    const long long c = offs[nd - 1], b = nd == 7 ? offs[nd - 2] : c, a = offs[nd / 2 + 1];
    if (sym && a > 0 && c % b == 0 && n % c == 0) {
      out->gnx = (int)b;
      out->gny = (int)(c / b);
      out->gnz = (int)(n / c);
      out->ga = (int)a;
    }
  }
  return ECG_OK;
}

ecg_status upload_csr(int64_t n, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                      const std::vector<double>& v, hipStream_t s, DevCsr* out, std::vector<void*>* owned,
                      bool with_dia = false) {
  std::vector<int> rp32(n + 1);
  for (int64_t i = 0; i <= n; ++i) rp32[i] = (int)rp[i];
  const size_t nnz = v.size();
  out->n = (int)n;
  out->nnz = (int)nnz;
  ecg_status st;
  if ((st = copy_in(&out->rowptr, rp32.data(), rp32.size(), 0, s)) != ECG_OK) return st;
  if ((st = copy_in(&out->col, ci.data(), nnz, 0, s)) != ECG_OK) return st;
  if ((st = copy_in(&out->val, v.data(), nnz, 0, s)) != ECG_OK) return st;
  HIPCHK(hipMalloc(&out->valf, std::max<size_t>(nnz, 1) * sizeof(float)));
  if (nnz) launch_cast_val((int)nnz, out->val, out->valf, s);
  if (with_dia && (size_t)n * kMaxDiag < ((size_t)1 << 31) && (st = upload_dia(n, rp, ci, v, s, out)) != ECG_OK)
    return st;
  HIPCHK(hipStreamSynchronize(s));
  if (owned) {
    owned->push_back(out->rowptr);
    owned->push_back(out->col);
    owned->push_back(out->val);
    owned->push_back(out->valf);
  }
  return ECG_OK;
}

// SELL-C-sigma form (see DevCsr) built on the host from the CSR arrays.
ecg_status upload_sell(int64_t n, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                       const std::vector<double>& v, hipStream_t s, DevCsr* out) {
  const int64_t npos = (n + kSellC - 1) / kSellC * kSellC;
  std::vector<int> order(npos, -1);
  for (int64_t w0 = 0; w0 < n; w0 += kSellSigma) {
    const int64_t w1 = std::min<int64_t>(n, w0 + kSellSigma);
    std::vector<int> win;
    for (int64_t i = w0; i < w1; ++i) win.push_back((int)i);
    std::stable_sort(win.begin(), win.end(),
                     [&](int a, int b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
    std::copy(win.begin(), win.end(), order.begin() + w0);
  }
  const int nslice = (int)(npos / kSellC);
  std::vector<int> sptr(nslice + 1, 0), slen(nslice, 0);
  for (int sl = 0; sl < nslice; ++sl) {
    int w = 0;
    for (int i = 0; i < kSellC; ++i) {
      const int r = order[(size_t)sl * kSellC + i];
      if (r >= 0) w = std::max(w, (int)(rp[r + 1] - rp[r]));
    }
    slen[sl] = w;
    if ((int64_t)sptr[sl] + (int64_t)w * kSellC > 0x7fffffff) return ECG_OK;  // too large: keep CSR only
    sptr[sl + 1] = sptr[sl] + w * kSellC;
  }
  const size_t total = (size_t)sptr[nslice];
  std::vector<int> scol(std::max<size_t>(total, 1));
  std::vector<double> sval(std::max<size_t>(total, 1));
  for (int sl = 0; sl < nslice; ++sl)
    for (int i = 0; i < kSellC; ++i) {
      const int r = order[(size_t)sl * kSellC + i];
      for (int k = 0; k < slen[sl]; ++k) {
        const size_t e = (size_t)sptr[sl] + (size_t)k * kSellC + i;
        const bool real = r >= 0 && k < rp[r + 1] - rp[r];
        scol[e] = real ? ci[rp[r] + k] : (r >= 0 ? r : 0);
        sval[e] = real ? v[rp[r] + k] : 0.0;
      }
    }
  ecg_status st;
  if ((st = copy_in(&out->sell_ptr, sptr.data(), sptr.size(), 0, s)) != ECG_OK) return st;
  if ((st = copy_in(&out->sell_len, slen.data(), slen.size(), 0, s)) != ECG_OK) return st;
  if ((st = copy_in(&out->sell_row, order.data(), order.size(), 0, s)) != ECG_OK) return st;
  if ((st = copy_in(&out->sell_col, scol.data(), scol.size(), 0, s)) != ECG_OK) return st;
  if ((st = copy_in(&out->sell_val, sval.data(), sval.size(), 0, s)) != ECG_OK) return st;
  HIPCHK(hipMalloc(&out->sell_valf, sval.size() * sizeof(float)));
  launch_cast_val((int)sval.size(), out->sell_val, out->sell_valf, s);
  HIPCHK(hipStreamSynchronize(s));
  out->nslice = nslice;
  return ECG_OK;
}

void free_csr(DevCsr& A) {
  (void)hipFree(A.sell_ptr);
  (void)hipFree(A.sell_len);
  (void)hipFree(A.sell_row);
  (void)hipFree(A.sell_col);
  (void)hipFree(A.sell_val);
  (void)hipFree(A.sell_valf);
  (void)hipFree(A.rowptr);
  (void)hipFree(A.col);
  (void)hipFree(A.val);
  (void)hipFree(A.valf);
  (void)hipFree(A.dval);
  (void)hipFree(A.dvalf);
  A = DevCsr();
}

// Transpose of a lower-triangular CSR (diag last) -> upper CSR (diag first); perm[kU] = kL.
void transpose_csr(int64_t n, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                   std::vector<int64_t>& rpt, std::vector<int32_t>& cit, std::vector<int>& perm) {
  const size_t nnz = ci.size();
  rpt.assign(n + 1, 0);
  for (size_t k = 0; k < nnz; ++k) rpt[ci[k] + 1]++;
  for (int64_t i = 0; i < n; ++i) rpt[i + 1] += rpt[i];
  std::vector<int64_t> pos(rpt.begin(), rpt.end() - 1);
  cit.resize(nnz);
  perm.resize(nnz);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int64_t d = pos[ci[k]]++;
      cit[d] = (int32_t)i;
      perm[d] = (int)k;
    }
}

// Level sets: for each group, rows ordered by level.  deps(i) lists rows that must be
// solved before row i.  forward: rows processed in increasing order; else decreasing.
void level_sets(int64_t n, const std::vector<int>& group, int ngroups, const std::vector<int64_t>& rp,
                const std::vector<int32_t>& ci, bool forward, std::vector<int>& lptr, std::vector<int>& lrows,
                int* maxlev_out, int maxlev_in = -1) {
  std::vector<int> lev(n, 0);
  int maxlev = 0;
  for (int64_t ii = 0; ii < n; ++ii) {
    const int64_t i = forward ? ii : n - 1 - ii;
    int l = 0;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int j = ci[k];
      if (j == i) continue;
      l = std::max(l, lev[j] + 1);
    }
    lev[i] = l;
    maxlev = std::max(maxlev, l + 1);
  }
  if (maxlev_in > maxlev) maxlev = maxlev_in;
  std::vector<int> cnt((size_t)ngroups * maxlev, 0);
  for (int64_t i = 0; i < n; ++i) cnt[(size_t)group[i] * maxlev + lev[i]]++;
  lptr.assign((size_t)ngroups * (maxlev + 1), 0);
  std::vector<int> start((size_t)ngroups * maxlev);
  int acc = 0;
  for (int g = 0; g < ngroups; ++g) {
    for (int l = 0; l < maxlev; ++l) {
      lptr[(size_t)g * (maxlev + 1) + l] = acc;
      start[(size_t)g * maxlev + l] = acc;
      acc += cnt[(size_t)g * maxlev + l];
    }
    lptr[(size_t)g * (maxlev + 1) + maxlev] = acc;
  }
  lrows.resize(n);
  for (int64_t i = 0; i < n; ++i) lrows[start[(size_t)group[i] * maxlev + lev[i]]++] = (int)i;
  *maxlev_out = maxlev;
}

ecg_status make_tri(int64_t n, const std::vector<int>& group, int ngroups, const std::vector<int64_t>& rpL,
                    const std::vector<int32_t>& ciL, const std::vector<double>& vL, hipStream_t s, ecg_precond* M,
                    std::vector<int>* permU_out) {
  std::vector<int64_t> rpU;
  std::vector<int32_t> ciU;
  std::vector<int> perm;
  transpose_csr(n, rpL, ciL, rpU, ciU, perm);
  std::vector<double> vU(vL.size());
  for (size_t k = 0; k < vU.size(); ++k) vU[k] = vL[perm[k]];
  ecg_status st;
  if ((st = upload_csr(n, rpL, ciL, vL, s, &M->tri.L, nullptr)) != ECG_OK) return st;
  if ((st = upload_csr(n, rpU, ciU, vU, s, &M->tri.U, nullptr)) != ECG_OK) return st;
  std::vector<int> lpL, lrL, lpU, lrU;
  int mlL = 0, mlU = 0;
  level_sets(n, group, ngroups, rpL, ciL, true, lpL, lrL, &mlL);
  level_sets(n, group, ngroups, rpU, ciU, false, lpU, lrU, &mlU);
  // both solves use the same level count so one field describes them
  const int ml = std::max(mlL, mlU);
  if (mlL != ml) level_sets(n, group, ngroups, rpL, ciL, true, lpL, lrL, &mlL, ml);
  if (mlU != ml) level_sets(n, group, ngroups, rpU, ciU, false, lpU, lrU, &mlU, ml);
  M->tri.ngroups = ngroups;
  M->tri.maxlev = ml;
  {
    std::vector<int> loc(n), fill(ngroups, 0);
    for (int64_t i = 0; i < n; ++i) loc[i] = fill[group[i]]++;
    M->tri.maxrows = *std::max_element(fill.begin(), fill.end());
    if ((st = copy_in(&M->tri.loc, loc.data(), loc.size(), 0, s)) != ECG_OK) return st;
    auto side = [&](const std::vector<int64_t>& rp, const std::vector<int32_t>& ci, const std::vector<int>& lr,
                    int** kr, int** lcol) -> ecg_status {
      std::vector<int> k2(2 * (size_t)n), lc(ci.size());
      for (int64_t p = 0; p < n; ++p) {
        k2[2 * p] = (int)rp[lr[p]];
        k2[2 * p + 1] = (int)rp[lr[p] + 1];
      }
      for (size_t k = 0; k < ci.size(); ++k) lc[k] = loc[ci[k]];
      ecg_status e;
      if ((e = copy_in(kr, k2.data(), k2.size(), 0, s)) != ECG_OK) return e;
      return copy_in(lcol, lc.data(), lc.size(), 0, s);
    };
    if ((st = side(rpL, ciL, lrL, &M->tri.kr_L, &M->tri.lcol_L)) != ECG_OK) return st;
    if ((st = side(rpU, ciU, lrU, &M->tri.kr_U, &M->tri.lcol_U)) != ECG_OK) return st;
  }
  if ((st = copy_in(&M->tri.lvl_ptr_L, lpL.data(), lpL.size(), 0, s)) != ECG_OK) return st;
  if ((st = copy_in(&M->tri.lvl_rows_L, lrL.data(), lrL.size(), 0, s)) != ECG_OK) return st;
  if ((st = copy_in(&M->tri.lvl_ptr_U, lpU.data(), lpU.size(), 0, s)) != ECG_OK) return st;
  if ((st = copy_in(&M->tri.lvl_rows_U, lrU.data(), lrU.size(), 0, s)) != ECG_OK) return st;
  HIPCHK(hipStreamSynchronize(s));
  if (permU_out) *permU_out = perm;
  return ECG_OK;
}

}  // namespace

void ecg::set_last_error(const char* msg) { g_err = msg ? msg : ""; }

void ecg::stat_begin(hipStream_t s) {
  if (!g_stats_on) return;
  g_open = take_event();
  if (g_open) (void)hipEventRecord(g_open, s);
}

void ecg::stat_end(int cls, double bytes, double flops, hipStream_t s) {
  if (!g_stats_on) return;
  hipEvent_t e = take_event();
  if (e) (void)hipEventRecord(e, s);
  g_pending.push_back(PendingStat{cls, g_open, e, bytes, flops});
  g_open = nullptr;
}

// ====================================================================== C ABI

// ------------------------------------------------------------------ static workspace
// The workspace of ecg_solve_noalloc: a device array of the library's code object, so that
// the call allocates nothing.  Each device holds its own copy (until the process ends); its
// address on a device is taken once, with that device current, and kept.
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

ecg_status scratch_of_current_device(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ECG_EINVAL, "device ordinal out of range for the static workspace");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ECG_EHIP, "hipGetSymbolAddress gave no address for the static workspace");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ECG_OK;
}
}  // namespace

extern "C" {

ecg_status ecg_progress(int32_t every) {
  g_progress_every = every > 0 ? every : 0;
  return ECG_OK;
}

ecg_status ecg_stats_enable(int on) {
  g_stats_on = on != 0;
  return ECG_OK;
}

ecg_status ecg_stats_read(ecg_kernel_stats* out, int reset) {
  if (!out) return fail(ECG_EINVAL, "NULL argument");
  flush_stats();
  *out = g_stats;
  if (reset) std::memset(&g_stats, 0, sizeof(g_stats));
  return ECG_OK;
}

const char* ecg_last_error(void) { return g_err.c_str(); }

ecg_status ecg_options_default(ecg_options* o) {
  if (!o) return fail(ECG_EINVAL, "options is NULL");
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->kmax = 20000;
  o->reduce = ECG_REDUCE_NONE;
  o->switch_tol = 1e-5;
  o->t_min = 1;
  o->min_gap = 1;
  o->precision = ECG_FP64;
  o->inner_tol = 1e-4;
  o->max_outer = 20;
  o->replace_every = 25;
  o->deflate_tol = 1e-14;
  o->precond = ECG_PRECOND_NONE;
  o->variant = ECG_SRE_CG2;
  o->restart = ECG_RESTART_NONE;
  o->restart_tol = 1e-5;
  o->refine_keep_q = 2;
  return ECG_OK;
}

ecg_status ecg_operator_create_csr(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                                   const double* vals, int on_device, void* hip_stream, ecg_operator** out) {
  if (!out || !rowptr || (nnz > 0 && (!colind || !vals))) return fail(ECG_EINVAL, "NULL argument");
  if (n <= 0 || n > 0x7fffffff) return fail(ECG_EINVAL, "n out of range");
  if (nnz < 0 || nnz >= 0x7fffffffLL) return fail(ECG_EINVAL, "nnz must be < 2^31");
  hipStream_t s = (hipStream_t)hip_stream;
  auto* op = new ecg_operator();
  ecg_status st;
  if ((st = to_host(op->rowptr, rowptr, (size_t)n + 1, on_device, s)) != ECG_OK ||
      (st = to_host(op->col, colind, (size_t)nnz, on_device, s)) != ECG_OK ||
      (st = to_host(op->val, vals, (size_t)nnz, on_device, s)) != ECG_OK ||
      (st = check_csr(n, nnz, op->rowptr, op->col)) != ECG_OK ||
      (st = upload_csr(n, op->rowptr, op->col, op->val, s, &op->A, nullptr, true)) != ECG_OK ||
      (op->A.ndiag == 0 && (st = upload_sell(n, op->rowptr, op->col, op->val, s, &op->A)) != ECG_OK)) {
    free_csr(op->A);
    delete op;
    return st;
  }
  op->n = n;
  op->nnz = nnz;
  *out = op;
  return ECG_OK;
}

void ecg_operator_destroy(ecg_operator* A) {
  if (!A) return;
  free_csr(A->A);
  delete A;
}

ecg_status ecg_operator_info(const ecg_operator* A, int64_t* n, int64_t* nnz) {
  if (!A) return fail(ECG_EINVAL, "NULL operator");
  if (n) *n = A->n;
  if (nnz) *nnz = A->nnz;
  return ECG_OK;
}

ecg_status ecg_partition_create(int64_t n, int32_t t, const int32_t* part, int on_device, void* hip_stream,
                                ecg_partition** out) {
  if (!out || !part) return fail(ECG_EINVAL, "NULL argument");
  if (n <= 0 || n > 0x7fffffff) return fail(ECG_EINVAL, "n out of range");
  if (t < 1 || t > kMaxT) return fail(ECG_EINVAL, "t must be in [1, 64]");
  hipStream_t s = (hipStream_t)hip_stream;
  auto* P = new ecg_partition();
  ecg_status st = to_host(P->host, part, (size_t)n, on_device, s);
  if (st != ECG_OK) {
    delete P;
    return st;
  }
  std::vector<int64_t> cnt(t, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int p = P->host[i];
    if (p < 0 || p >= t) {
      delete P;
      return fail(ECG_EINVAL, "part[i] outside [0, t)");
    }
    cnt[p]++;
  }
  for (int j = 0; j < t; ++j)
    if (cnt[j] == 0) {
      delete P;
      return fail(ECG_EINVAL, "empty subdomain " + std::to_string(j));
    }
  if ((st = copy_in(&P->part, P->host.data(), (size_t)n, 0, s)) != ECG_OK) {
    delete P;
    return st;
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    (void)hipFree(P->part);
    delete P;
    return fail(ECG_EHIP, "partition upload failed");
  }
  P->n = n;
  P->t = t;
  *out = P;
  return ECG_OK;
}

void ecg_partition_destroy(ecg_partition* P) {
  if (!P) return;
  (void)hipFree(P->part);
  delete P;
}

namespace {

// Block-Jacobi IC(0) on the blocks given by group[i] in [0, ngroups).
ecg_status build_bj_ic0(const ecg_operator* A, const std::vector<int>& group, int ngroups, hipStream_t s,
                        ecg_precond** out) {
  const int64_t n = A->n;
  // pattern of L: lower triangle of A restricted to each subdomain, diagonal last
  std::vector<int64_t> rp(n + 1, 0);
  std::vector<int32_t> ci;
  std::vector<int> apos;
  for (int64_t i = 0; i < n; ++i) {
    bool has_diag = false;
    for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
      const int j = A->col[k];
      if (j > i || group[j] != group[i]) continue;
      if (j == i) has_diag = true;
      ci.push_back(j);
      apos.push_back((int)k);
    }
    if (!has_diag) return fail(ECG_EINVAL, "matrix has a missing diagonal entry");
    rp[i + 1] = (int64_t)ci.size();
  }
  std::vector<double> v(ci.size(), 0.0);
  auto* M = new ecg_precond();
  M->kind = 0;
  std::vector<int> permU;
  ecg_status st = make_tri(n, group, ngroups, rp, ci, v, s, M, &permU);
  int* d_apos = nullptr;
  int* d_fail = nullptr;
  int* d_perm = nullptr;
  if (st == ECG_OK) st = copy_in(&d_apos, apos.data(), apos.size(), 0, s);
  if (st == ECG_OK) st = copy_in(&d_perm, permU.data(), permU.size(), 0, s);
  if (st == ECG_OK && hipMalloc(&d_fail, sizeof(int)) != hipSuccess) st = fail(ECG_EHIP, "hipMalloc failed");
  int hfail = 0;
  if (st == ECG_OK) {
    (void)hipMemsetAsync(d_fail, 0, sizeof(int), s);
    launch_ic0(A->A, M->tri, d_apos, d_fail, s);
    launch_gather((int)ci.size(), M->tri.L.val, d_perm, M->tri.U.val, s);
    launch_cast_val((int)ci.size(), M->tri.L.val, M->tri.L.valf, s);
    launch_cast_val((int)ci.size(), M->tri.U.val, M->tri.U.valf, s);
    if (hipMemcpyAsync(&hfail, d_fail, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = fail(ECG_EHIP, std::string("IC(0) factorisation: ") + hipGetErrorString(hipGetLastError()));
  }
  (void)hipFree(d_apos);
  (void)hipFree(d_fail);
  (void)hipFree(d_perm);
  if (st == ECG_OK && hfail) st = fail(ECG_EBREAKDOWN, "IC(0) pivot not positive");
  if (st != ECG_OK) {
    ecg_precond_destroy(M);
    return st;
  }
  *out = M;
  return ECG_OK;
}

// Block-Jacobi exact Cholesky: band storage per block, factorisation and panel
// preparation on the device.
ecg_status build_bj_chol(const ecg_operator* A, const std::vector<int>& group, int ngroups, hipStream_t s,
                         ecg_precond** out) {
  const int64_t n = A->n;
  std::vector<int> row_off(ngroups + 1, 0), local(n);
  for (int64_t i = 0; i < n; ++i) ++row_off[group[i] + 1];
  for (int g = 0; g < ngroups; ++g) row_off[g + 1] += row_off[g];
  std::vector<int> rows(n), fillp(row_off.begin(), row_off.end() - 1);
  for (int64_t i = 0; i < n; ++i) {
    const int g = group[i];
    local[i] = fillp[g] - row_off[g];
    rows[fillp[g]++] = (int)i;
  }
  int wraw = 0;
  for (int64_t i = 0; i < n; ++i) {
    bool has_diag = false;
    for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
      const int j = A->col[k];
      if (j == i) has_diag = true;
      if (j < i && group[j] == group[i]) wraw = std::max(wraw, local[i] - local[j]);
    }
    if (!has_diag) return fail(ECG_EINVAL, "matrix has a missing diagonal entry");
  }
  if (wraw > kBandMax)
    return fail(ECG_EINVAL, "block band " + std::to_string(wraw) + " exceeds " + std::to_string(kBandMax) +
                                " (blocks at most 128 cells wide in matrix order)");
  const int W = wraw <= 32 ? 32 : (wraw <= 64 ? 64 : kBandMax);  // a power of two (ring index)
  const int ld = W + 1;
  std::vector<long long> ab_off(ngroups + 1, 0), panel_off(ngroups + 1, 0);
  for (int g = 0; g < ngroups; ++g) {
    const int ng = row_off[g + 1] - row_off[g];
    ab_off[g + 1] = ab_off[g] + (long long)ng * ld;
    panel_off[g + 1] = panel_off[g] + (ng + kPanel - 1) / kPanel;
  }
  std::vector<double> ab(ab_off[ngroups], 0.0);
  for (int64_t i = 0; i < n; ++i) {
    const int g = group[i];
    for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
      const int j = A->col[k];
      if (j > i || group[j] != g) continue;
      ab[ab_off[g] + (long long)local[j] * ld + (local[i] - local[j])] = A->val[k];
    }
  }
  auto* M = new ecg_precond();
  M->kind = 2;
  DevBand& B = M->band;
  B.n = (int)n;
  B.nblocks = ngroups;
  B.W = W;
  B.npanels = panel_off[ngroups];
  ecg_status st = ECG_OK;
  long long* d_aboff = nullptr;
  double* d_ab = nullptr;
  int* d_fail = nullptr;
  int hfail = 0;
  if ((st = copy_in(&B.row_off, row_off.data(), row_off.size(), 0, s)) == ECG_OK &&
      (st = copy_in(&B.rows, rows.data(), rows.size(), 0, s)) == ECG_OK &&
      (st = copy_in(&B.panel_off, panel_off.data(), panel_off.size(), 0, s)) == ECG_OK &&
      (st = copy_in(&d_aboff, ab_off.data(), ab_off.size(), 0, s)) == ECG_OK &&
      (st = copy_in(&d_ab, ab.data(), ab.size(), 0, s)) == ECG_OK) {
    const size_t pbytes = (size_t)B.npanels * (2ull * kPanel * kPanel + 2ull * kPanel * W) * sizeof(double);
    if (hipMalloc(&B.panels, pbytes) != hipSuccess || hipMalloc(&d_fail, sizeof(int)) != hipSuccess) {
      st = fail(ECG_ENOMEM, "hipMalloc failed for the block Cholesky factors");
    } else {
      (void)hipMemsetAsync(d_fail, 0, sizeof(int), s);
      launch_band_chol(B, B.row_off, d_aboff, d_ab, d_fail, s);
      launch_band_panels(B, d_aboff, d_ab, s);
      if (hipMemcpyAsync(&hfail, d_fail, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        st = fail(ECG_EHIP, std::string("block Cholesky: ") + hipGetErrorString(hipGetLastError()));
    }
  }
  (void)hipFree(d_aboff);
  (void)hipFree(d_ab);
  (void)hipFree(d_fail);
  if (st == ECG_OK && hfail) st = fail(ECG_EBREAKDOWN, "block Cholesky pivot not positive (block not SPD)");
  if (st != ECG_OK) {
    ecg_precond_destroy(M);
    return st;
  }
  *out = M;
  return ECG_OK;
}

}  // namespace

ecg_status ecg_precond_create_bj_ic0(const ecg_operator* A, const ecg_partition* P, void* hip_stream,
                                     ecg_precond** out) {
  if (!A || !P || !out) return fail(ECG_EINVAL, "NULL argument");
  if (A->n != P->n) return fail(ECG_EINVAL, "operator and partition sizes differ");
  std::vector<int> group(P->host.begin(), P->host.end());
  return build_bj_ic0(A, group, P->t, (hipStream_t)hip_stream, out);
}

ecg_status ecg_precond_create_bj(const ecg_operator* A, int32_t nblocks, const int32_t* block, int on_device,
                                 int32_t kind, void* hip_stream, ecg_precond** out) {
  if (!A || !block || !out) return fail(ECG_EINVAL, "NULL argument");
  if (nblocks < 1 || nblocks > (1 << 20)) return fail(ECG_EINVAL, "nblocks out of range");
  if (kind != ECG_BJ_IC0 && kind != ECG_BJ_CHOL) return fail(ECG_EINVAL, "unknown block-Jacobi kind");
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<int32_t> hb;
  ecg_status st;
  if ((st = to_host(hb, block, (size_t)A->n, on_device, s)) != ECG_OK) return st;
  std::vector<int> count(nblocks, 0);
  for (int32_t b : hb) {
    if (b < 0 || b >= nblocks) return fail(ECG_EINVAL, "block id out of range");
    ++count[b];
  }
  for (int c : count)
    if (c == 0) return fail(ECG_EINVAL, "empty block");
  std::vector<int> group(hb.begin(), hb.end());
  return kind == ECG_BJ_IC0 ? build_bj_ic0(A, group, nblocks, s, out) : build_bj_chol(A, group, nblocks, s, out);
}

ecg_status ecg_precond_create_factor(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colind,
                                     const double* vals, int on_device, void* hip_stream, ecg_precond** out) {
  if (!out || !rowptr || !colind || !vals) return fail(ECG_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
  ecg_status st;
  if ((st = to_host(rp, rowptr, (size_t)n + 1, on_device, s)) != ECG_OK) return st;
  if ((st = to_host(ci, colind, (size_t)nnz, on_device, s)) != ECG_OK) return st;
  if ((st = to_host(v, vals, (size_t)nnz, on_device, s)) != ECG_OK) return st;
  if ((st = check_csr(n, nnz, rp, ci)) != ECG_OK) return st;
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] == rp[i] || ci[rp[i + 1] - 1] != i) return fail(ECG_EINVAL, "G must be lower triangular with the diagonal last");
    if (!(v[rp[i + 1] - 1] > 0.0)) return fail(ECG_EINVAL, "G has a non-positive diagonal entry");
  }
  std::vector<int64_t> rpt;
  std::vector<int32_t> cit;
  std::vector<int> perm;
  transpose_csr(n, rp, ci, rpt, cit, perm);
  std::vector<double> vt(v.size());
  for (size_t k = 0; k < vt.size(); ++k) vt[k] = v[perm[k]];
  auto* M = new ecg_precond();
  M->kind = 1;
  if ((st = upload_csr(n, rp, ci, v, s, &M->G, nullptr, true)) != ECG_OK ||
      (st = upload_csr(n, rpt, cit, vt, s, &M->Gt, nullptr, true)) != ECG_OK) {
    ecg_precond_destroy(M);
    return st;
  }
  *out = M;
  return ECG_OK;
}

void ecg_precond_destroy(ecg_precond* M) {
  if (!M) return;
  free_csr(M->tri.L);
  free_csr(M->tri.U);
  (void)hipFree(M->tri.lvl_ptr_L);
  (void)hipFree(M->tri.lvl_rows_L);
  (void)hipFree(M->tri.lvl_ptr_U);
  (void)hipFree(M->tri.lvl_rows_U);
  (void)hipFree(M->tri.loc);
  (void)hipFree(M->tri.kr_L);
  (void)hipFree(M->tri.kr_U);
  (void)hipFree(M->tri.lcol_L);
  (void)hipFree(M->tri.lcol_U);
  free_csr(M->G);
  free_csr(M->Gt);
  (void)hipFree(M->band.row_off);
  (void)hipFree(M->band.rows);
  (void)hipFree(M->band.panel_off);
  (void)hipFree(M->band.panels);
  delete M;
}

ecg_status ecg_workspace_size(const ecg_operator* A, const ecg_partition* P, const ecg_options* o, size_t* bytes) {
  if (!A || !P || !bytes) return fail(ECG_EINVAL, "NULL argument");
  ecg_status st = check_options(o);
  if (st != ECG_OK) return st;
  if (A->n != P->n) return fail(ECG_EINVAL, "operator and partition sizes differ");
  Plan pl;
  if ((st = make_plan(A->n, P->t, *o, &pl)) != ECG_OK) return st;
  *bytes = pl.total;
  return ECG_OK;
}

ecg_status ecg_spmv(const ecg_operator* A, const double* x, double* y, void* hip_stream) {
  if (!A || !x || !y) return fail(ECG_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)hip_stream;
  launch_spmv(A->A, x, y, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

static ecg_status solve_in(const ecg_operator* A, const ecg_partition* P, const double* b, double* x,
                           const ecg_options* o, void* workspace, size_t ws_bytes, void* hip_stream, ecg_report* rep,
                           double* rho_hist) {
  if (!A || !P || !b || !x || !workspace || !rep) return fail(ECG_EINVAL, "NULL argument");
  ecg_status st = check_options(o);
  if (st != ECG_OK) return st;
  if (A->n != P->n) return fail(ECG_EINVAL, "operator and partition sizes differ");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(ECG_EINVAL, "workspace must be 256-byte aligned");
  if (o->precond == ECG_PRECOND_SPLIT && o->M->kind == 1 && o->M->G.n != A->n)
    return fail(ECG_EINVAL, "preconditioner size differs from the operator");
  if (o->precond == ECG_PRECOND_SPLIT && o->M->kind == 0 && o->M->tri.L.n != A->n)
    return fail(ECG_EINVAL, "preconditioner size differs from the operator");
  if (o->precond == ECG_PRECOND_SPLIT && o->M->kind == 2 && o->M->band.n != A->n)
    return fail(ECG_EINVAL, "preconditioner size differs from the operator");
  if ((st = check_halving(P->t, *o)) != ECG_OK) return st;
  Plan pl;
  if ((st = make_plan(A->n, P->t, *o, &pl)) != ECG_OK) return st;
  if (ws_bytes < pl.total) return fail(ECG_ENOMEM, "workspace too small: need " + std::to_string(pl.total) + " bytes");
  hipStream_t s = (hipStream_t)hip_stream;
  char* ws = static_cast<char*>(workspace);
  std::memset(rep, 0, sizeof(*rep));
  const auto t_start = std::chrono::steady_clock::now();
  double* norm_part = reinterpret_cast<double*>(ws + pl.off_norm_part);
  double* dscal = reinterpret_cast<double*>(ws + pl.off_scalar);
  const int n = pl.n;
  InnerResult tot;
  double bnorm2 = 0.0;
  {
    // ||b||^2 via the residual kernel on a zero vector held in the H buffer
    double* zero = reinterpret_cast<double*>(ws + pl.off_v1);
    double* tmp = reinterpret_cast<double*>(ws + pl.off_v2);
    launch_zero(zero, (size_t)n * 8, s);
    if ((st = device_norm2(A->A, b, zero, tmp, norm_part, dscal, s, &bnorm2)) != ECG_OK) return st;
  }
  if (!std::isfinite(bnorm2)) return fail(ECG_EINVAL, "b contains NaN or Inf");
  ecg_status final = ECG_OK;
  int outer = 0;
  if (o->precision == ECG_FP64) {
    double* r = reinterpret_cast<double*>(ws + pl.off_r);
    const int g = launch_residual(A->A, b, x, r, norm_part, s);
    launch_sum(norm_part, g, dscal, s);
    double rr0 = 0;
    HIPCHK(hipMemcpyAsync(&rr0, dscal, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!std::isfinite(rr0)) return fail(ECG_EINVAL, "initial residual is not finite (NaN in x0?)");
    st = ecg_inner<double, double>(A, P, *o, pl, ws, x, r, rr0, o->tol, nullptr, s, &tot, rho_hist);
    if (st != ECG_OK) return st;
    final = tot.status;
    outer = 1;
    rep->relres_recursive = tot.rho0 > 0 ? tot.rho / tot.rho0 : 0.0;
  } else {
    double* r64 = reinterpret_cast<double*>(ws + pl.off_r64);
    double* d = reinterpret_cast<double*>(ws + pl.off_d);
    float* rf = reinterpret_cast<float*>(ws + pl.off_r);
    double rr = 0;
    int g = launch_residual(A->A, b, x, r64, norm_part, s);
    launch_sum(norm_part, g, dscal, s);
    HIPCHK(hipMemcpyAsync(&rr, dscal, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!std::isfinite(rr)) return fail(ECG_EINVAL, "initial residual is not finite (NaN in x0?)");
    const double rho0 = std::sqrt(rr);
    tot.rho0 = rho0;
    final = ECG_ENOTCONV;
    QStore kept;  // stored blocks carried from one refinement step to the next
    kept.cap = pl.cap;
    while (outer < o->max_outer) {
      if (std::sqrt(rr) <= o->tol * rho0) {
        final = ECG_OK;
        break;
      }
      launch_zero(d, (size_t)n * 8, s);
      launch_cast_d2f(n, r64, rf, s);
      InnerResult ir;
      ir.kmax_left = o->kmax - tot.iters;
      if (ir.kmax_left < 2) break;
      // the inner tolerance is relative to the inner initial residual, but never asks for
      // more than the outer target
      const double itol = std::max(o->inner_tol, o->tol * rho0 / std::sqrt(rr) * 0.5);
      const double rr_before = rr;
      st = ecg_inner<float, double>(A, P, *o, pl, ws, d, rf, rr, itol, r64, s, &ir, nullptr,
                                    o->refine_keep_q ? &kept : nullptr);
      if (st != ECG_OK) return st;
      tot.iters += ir.iters;
      tot.mem += ir.mem;
      tot.deflated += ir.deflated;
      tot.dropped += ir.dropped;
      for (int sw : ir.switches) tot.switches.push_back(sw);
      for (int rs : ir.restarts) tot.restarts.push_back(rs);
      tot.mem_peak = std::max(tot.mem_peak, ir.mem_peak);
      tot.t_final = ir.t_final;
      ++outer;
      launch_axpy_d(n, d, x, s);  // x += d in FP64, then the true FP64 residual below
      if (ir.status == ECG_EBREAKDOWN && ir.iters == 0) {
        final = ECG_EBREAKDOWN;
        break;
      }
      g = launch_residual(A->A, b, x, r64, norm_part, s);
      launch_sum(norm_part, g, dscal, s);
      HIPCHK(hipMemcpyAsync(&rr, dscal, 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      tot.rho = std::sqrt(rr);
      if (!(rr < 0.81 * rr_before)) break;  // a refinement step that gains < 10%: give up
    }
    if (final != ECG_EBREAKDOWN && std::sqrt(rr) <= o->tol * rho0) final = ECG_OK;
    rep->relres_recursive = rho0 > 0 ? std::sqrt(rr) / rho0 : 0.0;
  }
  // true residual in FP64
  {
    double* tmp = reinterpret_cast<double*>(ws + pl.off_v2);
    double rr = 0;
    if ((st = device_norm2(A->A, b, x, tmp, norm_part, dscal, s, &rr)) != ECG_OK) return st;
    rep->relres_true = bnorm2 > 0 ? std::sqrt(rr / bnorm2) : 0.0;
  }
  HIPCHK(hipGetLastError());
  const auto t_end = std::chrono::steady_clock::now();
  rep->iters = tot.iters;
  rep->n_switch = (int)tot.switches.size();
  for (int i = 0; i < (int)tot.switches.size() && i < 8; ++i) rep->switch_iters[i] = tot.switches[i];
  rep->t_final = tot.t_final;
  rep->outer_iters = outer;
  rep->deflated_cols = tot.deflated;
  rep->trunc_used = o->trunc > 0 ? o->trunc : 0;
  rep->blocks_dropped = (int32_t)std::min<long long>(tot.dropped, 0x7fffffff);
  rep->vectors_stored = tot.mem;
  rep->vectors_peak = tot.mem_peak;
  rep->n_restart = (int)tot.restarts.size();
  for (int i = 0; i < (int)tot.restarts.size() && i < 8; ++i) rep->restart_iters[i] = tot.restarts[i];
  rep->seconds = std::chrono::duration<double>(t_end - t_start).count();
  rep->status = final;
  if (final == ECG_EBREAKDOWN) return ECG_EBREAKDOWN;
  return final;
}

ecg_status ecg_solve(const ecg_operator* A, const ecg_partition* P, const double* b, double* x, const ecg_options* o,
                     void* workspace, size_t ws_bytes, void* hip_stream, ecg_report* rep, double* rho_hist) {
  return solve_in(A, P, b, x, o, workspace, ws_bytes, hip_stream, rep, rho_hist);
}

ecg_status ecg_solve_noalloc(const ecg_operator* A, const ecg_partition* P, const double* b, double* x,
                             const ecg_options* o, void* hip_stream, ecg_report* rep, double* rho_hist) {
  if (!A || !P || !b || !x || !rep) return fail(ECG_EINVAL, "NULL argument");
  ecg_status st = check_options(o);
  if (st != ECG_OK) return st;
  if (A->n != P->n) return fail(ECG_EINVAL, "operator and partition sizes differ");
  Plan pl;
  if ((st = make_plan(A->n, P->t, *o, &pl)) != ECG_OK) return st;
  if (pl.total > kScratchBytes)
    return fail(ECG_ENOMEM, "the solve needs " + std::to_string(pl.total) + " bytes of workspace; the static " +
                                "workspace of ecg_solve_noalloc holds " + std::to_string(kScratchBytes) +
                                " (lower kmax, or set q_budget_bytes or trunc)");
  void* ws = nullptr;
  if ((st = scratch_of_current_device(&ws)) != ECG_OK) return st;
  return solve_in(A, P, b, x, o, ws, kScratchBytes, hip_stream, rep, rho_hist);
}

// ---------------------------------------------------------------- debug entry points
ecg_status ecg_debug_spmm(const ecg_operator* A, int32_t t, const double* X, double* Y, void* hip_stream) {
  if (!A || !X || !Y) return fail(ECG_EINVAL, "NULL argument");
  if (t < 1 || t > 64 || (t & (t - 1))) return fail(ECG_EINVAL, "t must be a power of two in [1, 64]");
  hipStream_t s = (hipStream_t)hip_stream;
  launch_spmm<double>(A->A, t, X, Y, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

ecg_status ecg_debug_spmm_kernel(const ecg_operator* A, int32_t kernel, int32_t precision, int32_t t, const void* X,
                                 void* Y, void* hip_stream) {
  if (!A || !X || !Y) return fail(ECG_EINVAL, "NULL argument");
  if (t < 1 || t > 64 || (t & (t - 1))) return fail(ECG_EINVAL, "t must be a power of two in [1, 64]");
  if (kernel < kSpmmAuto || kernel > kSpmmSell) return fail(ECG_EINVAL, "unknown product kernel");
  if (kernel == kSpmmSell && A->A.nslice == 0)
    return fail(ECG_EINVAL, "the operator has no SELL-C-sigma form (it is kept for matrices without a diagonal form)");
  if (precision != 0 && precision != 1) return fail(ECG_EINVAL, "precision must be 0 (FP64) or 1 (FP32)");
  if (kernel == kSpmmDia && A->A.ndiag == 0) return fail(ECG_EINVAL, "the operator has no diagonal form");
  if (kernel == kSpmmGrid && A->A.gnx == 0) return fail(ECG_EINVAL, "the operator is not a grid stencil");
  if (kernel == kSpmmGridLds && !spmm_grid_lds_ok(A->A, t, precision == 0 ? 8 : 4))
    return fail(ECG_EINVAL, "the LDS-staged grid product does not apply to this operator and width");
  if (kernel == kSpmmGridDma && !spmm_grid_dma_ok(A->A, t, precision == 0 ? 8 : 4))
    return fail(ECG_EINVAL, "the LDS-staged grid product (direct loads) does not apply to this operator and width");
  hipStream_t s = (hipStream_t)hip_stream;
  if (precision == 0)
    launch_spmm<double>(A->A, t, static_cast<const double*>(X), static_cast<double*>(Y), s, kernel);
  else
    launch_spmm<float>(A->A, t, static_cast<const float*>(X), static_cast<float*>(Y), s, kernel);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

ecg_status ecg_debug_split(const ecg_partition* P, int32_t level, const double* v, double* out, void* hip_stream) {
  if (!P || !v || !out) return fail(ECG_EINVAL, "NULL argument");
  if (level < 0 || level > 6) return fail(ECG_EINVAL, "level out of range");
  const int t = (P->t + (1 << level) - 1) >> level;
  const int tc = pow2_at_least(t);
  hipStream_t s = (hipStream_t)hip_stream;
  launch_split<double>((int)P->n, P->part, level, tc, v, out, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

static bool pow2_le64(int v) { return v >= 1 && v <= 64 && !(v & (v - 1)); }

}  // extern "C"

namespace {
template <typename T>
ecg_status debug_gram_t(int64_t n, int32_t nb, int32_t wq, const T* Q, int32_t t, const T* Y, T* G, void* hip_stream) {
  if (!Q || !Y || !G || n <= 0 || nb < 1 || !pow2_le64(wq) || !pow2_le64(t)) return fail(ECG_EINVAL, "bad argument");
  hipStream_t s = (hipStream_t)hip_stream;
  Span<T> sp{Q, (long long)n * wq, nb, wq, 0};
  const int m = nb * wq;
  const size_t cap = (size_t)1 << 26;
  T* part = nullptr;
  HIPCHK(hipMalloc(&part, cap * sizeof(T)));
  launch_gram<T>((int)n, &sp, 1, m, t, Y, G, part, cap, s);
  hipError_t e = hipStreamSynchronize(s);
  (void)hipFree(part);
  if (e != hipSuccess) return fail(ECG_EHIP, hipGetErrorString(e));
  return ECG_OK;
}

template <typename T>
ecg_status debug_update_t(int64_t n, int32_t nb, int32_t wq, const T* Q, int32_t t, const T* G, T* W, void* hip_stream) {
  if (!Q || !W || !G || n <= 0 || nb < 1 || !pow2_le64(wq) || !pow2_le64(t)) return fail(ECG_EINVAL, "bad argument");
  hipStream_t s = (hipStream_t)hip_stream;
  Span<T> sp{Q, (long long)n * wq, nb, wq, 0};
  launch_update<T>((int)n, &sp, 1, t, G, W, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ECG_OK;
}
}  // namespace

extern "C" {

ecg_status ecg_debug_gram(int64_t n, int32_t nb, int32_t wq, const double* Q, int32_t t, const double* Y, double* G,
                          void* hip_stream) {
  return debug_gram_t<double>(n, nb, wq, Q, t, Y, G, hip_stream);
}

ecg_status ecg_debug_update(int64_t n, int32_t nb, int32_t wq, const double* Q, int32_t t, const double* G, double* W,
                            void* hip_stream) {
  return debug_update_t<double>(n, nb, wq, Q, t, G, W, hip_stream);
}

ecg_status ecg_debug_gram_f32(int64_t n, int32_t nb, int32_t wq, const float* Q, int32_t t, const float* Y, float* G,
                              void* hip_stream) {
  return debug_gram_t<float>(n, nb, wq, Q, t, Y, G, hip_stream);
}

ecg_status ecg_debug_update_f32(int64_t n, int32_t nb, int32_t wq, const float* Q, int32_t t, const float* G, float* W,
                                void* hip_stream) {
  return debug_update_t<float>(n, nb, wq, Q, t, G, W, hip_stream);
}

ecg_status ecg_debug_precond_apply(const ecg_precond* M, int32_t which, int32_t t, const double* X, double* Y,
                                   void* hip_stream) {
  if (!M || !X || !Y || (which != 0 && which != 1) || !pow2_le64(t)) return fail(ECG_EINVAL, "bad argument");
  hipStream_t s = (hipStream_t)hip_stream;
  precond_apply<double>(M, which, t, X, Y, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

}  // extern "C"
