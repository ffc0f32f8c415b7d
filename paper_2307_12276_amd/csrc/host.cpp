// Host runtime of libadl: Leja points, divided differences, sweep driver,
// exponential integrators and the C ABI (include/adl.h).
//
// Method (Deka, Kissmann, Einkemmer, ICRC 2023, Sec. 2): phi_l(A dt) v is
// approximated by Newton interpolation of phi_l((c + gamma xi) dt) at Leja
// points xi in [-2, 2], c = alpha/2, gamma = -alpha/4, applied term by term:
//   y_{k+1} = ((A - c I)/gamma - xi_k I) y_k,   p_{k+1} = p_k + d_{k+1} y_{k+1}.
// Two terms per GPU launch after the first (fused stencils + axpys + norms);
// one block of each launch takes the stopping decision of the previous
// launch's terms and sets a device stop flag, so that launches enqueued after
// convergence do no work, and the host learns the outcome once per chunk of
// launches (by spinning on a pinned host mirror that the chunk's decision
// launch writes, or by copying the control block back).
#include "op.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <system_error>
#include <thread>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

namespace adl {

// --------------------------------------------------------------------------
// error reporting
// --------------------------------------------------------------------------
static thread_local std::string g_err = "";

constexpr double kLearnedSafety = 1.2;  // learned rho is widened by this factor (capped by Gershgorin)

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ADL_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                  __FILE__, __LINE__);                                                \
  } while (0)

#define RETCHK(expr)        \
  do {                      \
    int r_ = (expr);        \
    if (r_ != ADL_OK) return r_; \
  } while (0)

// --------------------------------------------------------------------------
// Leja points on [-2, 2]: xi_0 = 2, then xi_k maximises prod_{j<k} |x - xi_j|.
// On each gap between consecutive sorted points log|prod| is strictly concave,
// so its maximiser is the zero of f'(x) = sum 1/(x - xi_j); it is tracked per
// gap by safeguarded Newton iteration.  Ties (equal products within 1e-12
// relative) go to the smaller point.
// --------------------------------------------------------------------------

static double gap_root(const std::vector<double>& pts, double a, double b, double x0) {
  double lo = a, hi = b;
  double x = (x0 > a && x0 < b) ? x0 : 0.5 * (a + b);
  for (int it = 0; it < 200; ++it) {
    double f1 = 0.0, f2 = 0.0;
    for (double p : pts) {
      const double r = 1.0 / (x - p);
      f1 += r;
      f2 -= r * r;
    }
    if (f1 > 0.0) lo = x; else hi = x;
    double xn = x - f1 / f2;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (std::fabs(xn - x) <= 2e-16 * std::fabs(x) + 1e-300 || hi - lo <= 4e-16 * std::fabs(x) + 1e-300) {
      x = xn;
      break;
    }
    x = xn;
  }
  return x;
}

static const std::vector<double>& leja_table() {
  static std::vector<double> pts;
  static std::once_flag once;
  std::call_once(once, [] {
    const int M = kMaxDegreeDefault + 1;
    pts = {2.0, -2.0, 0.0};
    std::vector<double> sorted = {-2.0, 0.0, 2.0};
    std::vector<double> guess = {-1.0, 1.0};  // maximiser guess per gap
    while ((int)pts.size() < M) {
      const int ng = (int)sorted.size() - 1;
      double best_f = -INFINITY, best_x = 0.0;
      std::vector<double> xs(ng), fs(ng);
      for (int g = 0; g < ng; ++g) {
        const double x = gap_root(pts, sorted[g], sorted[g + 1], guess[g]);
        double f = 0.0;
        for (double p : pts) f += std::log(std::fabs(x - p));
        xs[g] = x;
        fs[g] = f;
        if (f > best_f) best_f = f;
      }
      const double thr = best_f - 1e-12 * std::max(1.0, std::fabs(best_f));
      int pick = -1;
      for (int g = 0; g < ng; ++g)
        if (fs[g] >= thr && (pick < 0 || xs[g] < xs[pick])) pick = g;
      best_x = xs[pick];
      pts.push_back(best_x);
      // split the chosen gap
      std::vector<double> ns, ng2;
      ns.reserve(sorted.size() + 1);
      ng2.reserve(guess.size() + 1);
      for (int g = 0; g < ng; ++g) {
        ns.push_back(sorted[g]);
        if (g == pick) {
          ns.push_back(best_x);
          ng2.push_back(0.5 * (sorted[g] + best_x));
          ng2.push_back(0.5 * (best_x + sorted[g + 1]));
        } else {
          ng2.push_back(xs[g]);
        }
      }
      ns.push_back(sorted.back());
      sorted.swap(ns);
      guess.swap(ng2);
    }
  });
  return pts;
}

// --------------------------------------------------------------------------
// phi_l scalars: phi_0 = exp, phi_1 = (e^z - 1)/z, phi_2 = (e^z - 1 - z)/z^2;
// Taylor series sum_k z^k/(k+l)! for |z| < 1.
// --------------------------------------------------------------------------
static double phi_scalar(int l, double z) {
  if (l == 0) return std::exp(z);
  if (std::fabs(z) < 1.0) {
    double fact = 1.0;
    for (int i = 2; i <= l; ++i) fact *= i;  // l!
    double term = 1.0 / fact, s = 0.0;
    for (int k = 0; k < 30; ++k) {
      s += term;
      term *= z / (double)(k + l + 1);
    }
    return s;
  }
  const double e = std::expm1(z);
  if (l == 1) return e / z;
  return (e - z) / (z * z);
}

// --------------------------------------------------------------------------
// Plans: divided differences of g(xi) = phi_l((c + gamma xi) h)
// --------------------------------------------------------------------------
void build_plan(Plan& P, int l, double alpha, double h, int M) {
  const std::vector<double>& xi = leja_table();
  P.l = l;
  P.alpha = alpha;
  P.h = h;
  P.M = M;
  const double c = alpha / 2.0, gamma = -alpha / 4.0;
  P.d.resize(M);
  for (int k = 0; k < M; ++k) P.d[k] = phi_scalar(l, (c + gamma * xi[k]) * h);
  for (int j = 1; j < M; ++j)
    for (int k = M - 1; k >= j; --k) P.d[k] = (P.d[k] - P.d[k - 1]) / (xi[k] - xi[k - j]);
  P.shift.resize(M);
  P.s.resize(M);
  P.s[0] = 1.0;
  for (int k = 0; k < M; ++k) {
    P.shift[k] = c + gamma * xi[k];
    if (k + 1 < M) P.s[k + 1] = (2.0 - xi[k]) * P.s[k];
  }
  P.invg = 1.0 / gamma;
  P.last_degree = -1;
}

}  // namespace adl

using namespace adl;

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
  size_t kxx, kxy, kyy, ax, ay, y0, y1, p, p2, p3, p4, w1, w2, yacc, tmp, tmp2, partials, ctl, total;
};
// four Newton terms per launch on grids below this many points (the grid's
// vectors stay in the caches) ...
constexpr long kFourTermMaxPoints = 1L << 20;
// ... which is also the default there: measured on MI355X (FP64, steps/s of
// the two-stage quadrature, two terms per launch -> four, LDS rows accessed
// 16 bytes per lane, chunks ending on their targets): 256^2 +7 %, 384^2
// +15 %, 512^2 +14 %, 640^2 +44 %, 896^2 +31 %, 1000^2 +11 %

// rows of block partials per slot: three per term of a launch of up to four
constexpr int kSlotRows = 12;

static size_t max_partial_blocks(int nx, int ny) {
  // stencil launches: at most max(kMaxGrid, number of strips) blocks (one
  // column per lane and 62 output columns per strip in the two-term kernel:
  // the most strips); elementwise reductions <= 1024
  const size_t strips = (size_t)((nx + kWave - 3) / (kWave - 2));
  size_t nb = strips > (size_t)kMaxGrid ? strips : (size_t)kMaxGrid;
  if (nb < (size_t)kMaxGrid2) nb = kMaxGrid2;
  (void)ny;
  return nb > 4096 ? nb : 4096;
}

static WsLayout ws_layout(int nx, int ny, int storage) {
  const size_t n = (size_t)nx * ny;
  const size_t fs = storage == ADL_STORAGE_FP64 ? 8 : 4;
  const size_t ys = storage == ADL_STORAGE_FP32_FIELDS_Y ? 4 : 8;
  WsLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.kxx = take(n * fs);
  L.kxy = take(n * fs);
  L.kyy = take(n * fs);
  L.ax = take(n * fs);
  L.ay = take(n * fs);
  L.y0 = take(n * ys);
  L.y1 = take(n * ys);
  L.p = take(n * 8);
  L.w1 = take(n * 8);
  L.w2 = take(n * 8);
  L.yacc = take(n * 8);
  L.tmp = take(n * 8);
  L.tmp2 = take(n * 8);
  L.p2 = take(n * 8);
  L.p3 = take(n * 8);
  L.p4 = take(n * 8);
  L.partials = take(2 * kSlotRows * max_partial_blocks(nx, ny) * 8);
  L.ctl = take(4 * 128);
  L.total = o;
  return L;
}

static hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

static bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// tiling usable with these caller vectors (two-column loads need 16-byte alignment)
static const Tiling& tiling_for(const adl_op* op, const void* a, const void* b = nullptr,
                                const void* c = nullptr) {
  return (al16(a) && al16(b) && al16(c)) ? op->t : op->t1;
}

// --------------------------------------------------------------------------
// sweep: one Newton interpolation with a device stop flag
// --------------------------------------------------------------------------
struct SweepOut {
  int degree = 0;
  int status = 0;  // 1 converged, 2 non-finite, 3 degree cap
};

static int read_ctl(adl_op* op, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(op->host_ctl, op->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return ADL_OK;
}

// --------------------------------------------------------------------------
// sweep outcome mirrors (HostCtl): coherent pinned host memory in pages of
// kMirrorSlots cache lines per device, allocated on first use and kept until
// the process ends; ops take a slot at creation and give it back when
// destroyed.  Sequence numbers come from one process-wide counter, so a
// number never repeats in a slot, whichever op held it before.
// --------------------------------------------------------------------------
constexpr int kMirrorSlots = 64;
constexpr int kMirrorQueryUs = 50;  // stream query interval while spinning

struct MirrorPool {
  std::mutex m;
  std::unordered_map<int, std::vector<std::pair<HostCtl*, HostCtl*>>> free;  // device -> (host, device address)
};
static MirrorPool& mirror_pool() {
  static MirrorPool* p = new MirrorPool;  // never destroyed: slots may outlive static destructors
  return *p;
}
static std::atomic<int> g_hseq{0};

static int next_hseq() {
  int v = g_hseq.fetch_add(1, std::memory_order_relaxed) + 1;
  if (v <= 0) {  // wrapped: restart above zero (a slot starts at 0)
    g_hseq.store(1, std::memory_order_relaxed);
    v = 1;
  }
  return v;
}

static void mirror_take(adl_op* op) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  MirrorPool& P = mirror_pool();
  std::lock_guard<std::mutex> g(P.m);
  auto& fl = P.free[dev];
  if (fl.empty()) {
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, kMirrorSlots * sizeof(HostCtl),
                      hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable) != hipSuccess) {
      (void)hipGetLastError();
      return;  // the op copies the control block back instead
    }
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
      (void)hipGetLastError();
      hipHostFree(h);  // no kernel has seen it yet
      return;
    }
    std::memset(h, 0, kMirrorSlots * sizeof(HostCtl));
    for (int i = kMirrorSlots - 1; i >= 0; --i)
      fl.emplace_back(reinterpret_cast<HostCtl*>(h) + i, reinterpret_cast<HostCtl*>(d) + i);
  }
  op->hctl = fl.back().first;
  op->hctl_dev = fl.back().second;
  op->mirror_dev = dev;
  fl.pop_back();
}

static void mirror_give(adl_op* op) {
  if (!op->hctl) return;
  MirrorPool& P = mirror_pool();
  std::lock_guard<std::mutex> g(P.m);
  P.free[op->mirror_dev].emplace_back(op->hctl, op->hctl_dev);
  op->hctl = op->hctl_dev = nullptr;
}

// Waits until the chunk's decision launch has published sequence number
// op->hseq, then copies the outcome into op->host_ctl.  The stream is queried
// every kMirrorQueryUs while waiting, so that a failed launch ends the wait
// with its error.
static int await_outcome(adl_op* op, hipStream_t st) {
  const HostCtl* h = op->hctl;
  const int want = op->hseq;
  auto seen = [&] { return __atomic_load_n(&h->seq, __ATOMIC_ACQUIRE) == want; };
  auto next = std::chrono::steady_clock::now() + std::chrono::microseconds(kMirrorQueryUs);
  while (!seen()) {
    __builtin_ia32_pause();
    const auto now = std::chrono::steady_clock::now();
    if (now < next) continue;
    next = now + std::chrono::microseconds(kMirrorQueryUs);
    const hipError_t q = hipStreamQuery(st);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return fail(ADL_EHIP, "Leja sweep failed: %s", hipGetErrorString(q));
    if (seen()) break;
    return fail(ADL_EHIP, "Leja sweep ended without publishing its outcome");
  }
  op->host_ctl->stop = __atomic_load_n(&h->stop, __ATOMIC_RELAXED);
  op->host_ctl->status = __atomic_load_n(&h->status, __ATOMIC_RELAXED);
  op->host_ctl->degree = __atomic_load_n(&h->degree, __ATOMIC_RELAXED);
  return ADL_OK;
}

Plan& adl::get_plan(adl_op* op, int l, double alpha, double h) {
  for (Plan& P : op->plans)
    if (P.l == l && P.alpha == alpha && P.h == h && P.M == op->max_degree + 1) return P;
  if (op->plans.size() < 8) {
    op->plans.emplace_back();
    build_plan(op->plans.back(), l, alpha, h, op->max_degree + 1);
    return op->plans.back();
  }
  Plan& P = op->plans[op->plan_next];
  op->plan_next = (op->plan_next + 1) % (int)op->plans.size();
  build_plan(P, l, alpha, h, op->max_degree + 1);
  return P;
}

// Algorithmic HBM bytes of one Newton-Leja launch (any number of terms):
// read y_k, the three tensor fields (+ two advection fields), p_k (not at
// k = 0), w2 (when the augmented column enters); write y and p of the
// launch's last term.
static double leja_bytes(const adl_op* op, int k, bool with_w2) {
  const double fs = op->f.f32 ? 4.0 : 8.0;
  const double ys = op->storage == ADL_STORAGE_FP32_FIELDS_Y ? 4.0 : 8.0;
  double b = (k == 0 ? 8.0 : ys) + 3.0 * fs + (k == 0 ? 0.0 : 8.0) + (with_w2 ? 8.0 : 0.0) + ys + 8.0;
  if (op->f.ax) b += 2.0 * fs;
  return b * (double)op->n;
}

// Whether the Newton-Leja launches use non-temporal hints on the vectors
// they read or write once: by default when the sweep's working set (fields,
// v, three y and three p buffers) exceeds twice the 256 MiB Infinity Cache, so
// that each launch streams through it anyway.  Below that the hint evicts
// lines the next launch would find in cache (measured on MI355X: 10 % slower
// launches at 512^2 and at 2048^2, 335 MB; 4-10 % faster at 2896^2 and
// 4096^2).
constexpr double kStreamMinBytes = 512.0 * 1024 * 1024;
constexpr long kStagedMinPoints = 1L << 20;  // two-term launches stage their rows in LDS from here up
static int streaming_on(const adl_op* op) {
  if (op->streaming >= 0) return op->streaming;
  const double fs = op->f.f32 ? 4.0 : 8.0;
  const double ys = op->storage == ADL_STORAGE_FP32_FIELDS_Y ? 4.0 : 8.0;
  const double per_pt = (op->f.ax ? 5.0 : 3.0) * fs + 8.0 + 3.0 * ys + 3.0 * 8.0;
  return per_pt * (double)op->n > kStreamMinBytes ? 1 : 0;
}

// Whether the op can run four Newton terms per launch: a launch's 12 partial
// rows fit a partials slot, the sweep runs without non-temporal hints (the
// four-term kernel has none), and a periodic grid has enough rows for the
// kernel's one-wrap row rule.
static bool four_terms_ok(const adl_op* op) {
  const long nb = std::max(op->t4.nblocks, op->t41.nblocks);
  if (!four_term_rows_fit(op->ny, op->bc)) return false;
  return 12L * nb <= op->slot_stride && !streaming_on(op);
}

// Whether the op can run three Newton terms per launch (LDS-staged) on
// vectors whose tiling has `vec` columns per lane: the three-term tiling has
// two columns per lane (its stage 3 is then valid on the tiling's output
// lanes), the vectors allow it, and a launch's 9 partial rows fit a partials
// slot.
static bool three_terms_ok(const adl_op* op, int vec) {
  return vec == 2 && op->t3.vec == 2 && 9L * op->t3.nblocks <= op->slot_stride;
}
// the same for four terms per launch with LDS-staged rows (stage 4 valid on
// lanes 2 .. 61 of the tiling's strips with two columns per lane)
static bool four_staged_ok(const adl_op* op, int vec) {
  return vec == 2 && op->t4s.vec == 2 && 12L * op->t4s.nblocks <= op->slot_stride;
}

// p_out = g(A) v (top block of the augmented form when w2 != null; the
// augmented column enters with coefficient s_k * w2scale).
//
// Launches: the first term (y_0 = v) alone, then four terms per launch where
// the op runs the four-term kernel, else two while the op fuses terms (fewer
// when the degree cap is near; one per launch without fusion).  Each
// launch's block 0 takes the stopping decision of the previous launch's terms
// from its block partials; a one-block launch at the end of every chunk
// decides the chunk's last launch, and the host reads the outcome once per
// chunk.
//
// A launch stores y and p of its last term only (the norms of every term go
// into its partials).  Launch L reads y from buffer L mod 3 and p from p
// buffer (L - 1) mod 3 and writes buffers (L + 1) mod 3 and L mod 3: the
// launch that runs beside the decision of launch L writes neither of launch
// L's inputs, and every launch after it skips its work, so when the sweep
// stops at a term inside launch L (not its last), a replay of launch L on its
// intact inputs stores p of that term, bitwise what launch L computed.  The
// p buffers are p_out and two workspace vectors, arranged so that the
// predicted degree ends in p_out; otherwise the result is copied there.
// Whether a sweep on vectors of tiling T runs three terms per launch with
// LDS-staged rows (the default from kStagedMinPoints up, or mode 5)
static bool three_term_sweep(const adl_op* op, const Tiling& T) {
  const bool fours = op->fuse_terms == 6 && four_staged_ok(op, T.vec);
  const bool four = !fours && (op->fuse_terms == 4 || (op->fuse_terms == 1 && op->n < kFourTermMaxPoints)) &&
                    four_terms_ok(op);
  return !four && !fours && three_terms_ok(op, T.vec) &&
         (op->fuse_terms == 5 || (op->fuse_terms == 1 && (long)op->nx * op->ny >= kStagedMinPoints));
}

// Whether a midpoint step folds its stage vector w = A u + s into the
// sweep's first launch (the four-stage LDS march, terms 1 .. 3): one
// substep, a three-term sweep with FP64 Newton vectors whose first launch
// takes three terms, the four-term staged tiling available; by default from
// kStageFuseMinPoints up (measured, steps/s fused against a stage launch of
// its own: 4096^2 FP64 +2 %, FP32 fields +0.4 %; 2048^2 -1.2 %, 1024^2
// -1 %: the four-stage march is latency-bound, and on smaller grids its
// launch costs about as much as the two it replaces), always in mode 5
constexpr long kStageFuseMinPoints = 1L << 24;
static bool stage_fusable(const adl_op* op, const double* u, const double* s, double dt) {
  if (op->storage == ADL_STORAGE_FP32_FIELDS_Y || op->alpha == 0.0 || !op->has_bound) return false;
  if (op->fuse_terms != 5 && (long)op->nx * op->ny < kStageFuseMinPoints) return false;
  int K = substeps_for(op->alpha, dt, op->rho_max);
  if (op->learned) K = std::max(K, op->substeps_hint);
  int maxdeg = op->max_degree;
  if (op->learned && op->budget > 0 && op->budget < maxdeg) maxdeg = op->budget;
  const Tiling& T = tiling_for(op, u, s, op->p);
  return K == 1 && maxdeg >= 3 && three_term_sweep(op, T) && four_staged_ok(op, T.vec);
}

static int sweep(adl_op* op, Plan& P, const double* v, const double* w2, double w2scale, double* p_out,
                 double tol, int maxdeg, hipStream_t st, SweepOut& out, const double* stage_u = nullptr,
                 const double* stage_s = nullptr) {
  // stage_u (v null): the sweep of v = A stage_u + stage_s, whose first
  // launch computes that stage vector itself (stage_fusable)
  if (op->learned && op->budget > 0 && op->budget < maxdeg) maxdeg = op->budget;
  // (the control block is cleared by block 0 of the first launch)
  const bool ys32 = op->storage == ADL_STORAGE_FP32_FIELDS_Y;
  const Tiling& T = tiling_for(op, stage_u ? stage_u : v, p_out);
  const Tiling& T2 = T.vec == op->t2.vec ? op->t2 : op->t21;
  const Tiling& T4 = T.vec == op->t4.vec ? op->t4 : op->t41;
  const bool fuse = op->fuse_terms != 0;
  // four terms per launch with LDS-staged rows (mode 6)
  const bool fours = op->fuse_terms == 6 && four_staged_ok(op, T.vec);
  const bool four = !fours && (op->fuse_terms == 4 || (op->fuse_terms == 1 && op->n < kFourTermMaxPoints)) &&
                    four_terms_ok(op);
  // three terms per launch (LDS-staged) from kStagedMinPoints up by default
  // (4096^2 FP64 headline steps: 140 steps/s with two terms per launch, 185
  // with three), or forced by mode 5
  const bool three = three_term_sweep(op, T);
  const Tiling& T3 = op->t3;
  const Tiling& T4s = op->t4s;
  // first chunk: the last degree of this plan plus one (the degree moves by
  // about one from step to step; one launch too many costs its work, one too
  // few a second chunk and host round trip); the first sweep of a plan
  // guesses from rho h, below the degrees measured at tol 1e-10, since
  // launches past the stop still load a row group per wave
  int predicted = P.last_degree > 0 ? P.last_degree + 1
                                    : (int)(3.5 * std::sqrt(std::fabs(P.alpha) * P.h) + 4.0);
  if (predicted > maxdeg) predicted = maxdeg;
  if (predicted < 1) predicted = 1;
  const int mexp = P.last_degree > 0 ? P.last_degree : predicted;
  // launch plan: launch L covers terms kL+1 .. kL+nL
  std::vector<int> lk, ln;
  // terms of the launch after kcov terms in a chunk that ends at `target`:
  // four-term launches end the chunk on its target (a two- or one-term
  // launch for the remainder), so that a sweep stopping at the predicted
  // degree computes no terms past it
  auto plan_terms = [&](int kcov, int target) {
    auto aug = [&](int n) {  // the augmented column enters one of terms kcov+1 .. kcov+n
      if (!w2) return false;
      for (int i = 0; i < n; ++i)
        if (P.s[kcov + i] != 0.0) return true;
      return false;
    };
    // the first launch: terms 1 .. 3 from y_0 = v in the three-term form
    // (FP64 Newton vectors, no augmented column in them), else term 1 alone
    // (4096^2 headline steps of 72 terms: 24 launches instead of 1 + 24 and
    // a replay)
    if (kcov == 0) return (three && !ys32 && 3 <= maxdeg && !aug(3)) ? 3 : 1;
    const int lim = four ? std::min(target, maxdeg) : maxdeg;
    if (four && kcov + 4 <= lim && !aug(4)) return 4;
    if (fours && kcov + 4 <= maxdeg && !aug(4)) return 4;
    if (three && kcov + 3 <= lim && !aug(3)) return 3;
    const bool two = fuse && kcov + 2 <= lim && !aug(2);
    return two ? 2 : 1;
  };
  // three terms per launch from the first one: the first chunk covers the
  // last degree itself, rounded up to whole launches (one term more would
  // cost a whole launch whenever the last degree ends a launch: 4096^2
  // headline steps of degree 72, 24 launches instead of 25)
  if (P.last_degree > 0 && plan_terms(0, maxdeg) == 3) predicted = std::min(P.last_degree, maxdeg);
  // (a stage vector that the first launch cannot compute is formed first)
  if (stage_u && plan_terms(0, maxdeg) != 3) {
    HIPCHK(launch_apply(op->f, tiling_for(op, stage_u, stage_s), stage_u, op->w1, stage_s, 1.0, nullptr, 0.0, st));
    v = op->w1;
    stage_u = stage_s = nullptr;
  }
  // the chunk targets: the first chunk ends at the predicted degree, each
  // later one max(8, kcov / 4) terms on, capped at the degree limit
  auto next_target = [&](int kcov) {
    const int t = kcov == 0 ? predicted : kcov + std::max(8, kcov / 4);
    return t > maxdeg ? maxdeg : t;
  };
  // launch index of term j (terms kL+1 .. kL+nL in launch L)
  auto launch_of_term = [&](int j) -> int {
    int kcov = 0, L = 0, target = next_target(0);
    while (true) {
      if (kcov >= target) target = next_target(kcov);
      const int n = plan_terms(kcov, target);
      if (j <= kcov + n) return L;
      kcov += n;
      ++L;
    }
  };
  // buffers: y in ybuf[L mod 3] (the third one a workspace vector), p in
  // pbuf[L mod 3], p_out at the predicted degree's launch
  void* ybuf3[3];
  double* pbuf[3];
  {
    double* ws[4] = {op->p, op->p2, op->p3, op->p4};
    int wi = 0;
    auto take_ws = [&]() {
      if (ws[wi] == p_out) ++wi;
      return ws[wi++];
    };
    ybuf3[0] = op->ybuf[0];
    ybuf3[1] = op->ybuf[1];
    ybuf3[2] = take_ws();
    const int want = launch_of_term(std::max(mexp, 1)) % 3;
    for (int i = 0; i < 3; ++i) pbuf[i] = i == want ? p_out : take_ws();
  }
  LejaArgs a{};
  a.invg = P.invg;
  a.d0 = P.d[0];
  a.tol = tol;
  a.max_degree = maxdeg;
  a.ystore_f32 = ys32;
  a.stream = streaming_on(op);
  // two-term kernel: input rows staged in LDS from kStagedMinPoints up (each
  // input row then leaves memory once per run of bands: 4096^2 FP64 286 ->
  // 225-234 us per launch); the register-frame kernel on smaller grids,
  // where the staged kernel's prologue and extra barrier do not pay (measured
  // per launch, staged / frames: 512^2 1.14, 768^2 0.93-1.05, 1024^2
  // 0.87-0.92, 1536^2 0.78-0.86, 2048^2 0.84-0.89)
  a.staged = op->fuse_terms == 2 || op->fuse_terms == 5 || op->fuse_terms == 6 ||
             (op->fuse_terms == 1 && (long)op->nx * op->ny >= kStagedMinPoints);
  a.partials = op->partials;
  a.slot_stride = op->slot_stride;
  a.ctl = op->ctl;
  int kcov = 0, L = 0;
  int prev_nb = 0, prev_k = 0, prev_n = 0, prev_slot = 0;
  while (true) {
    const int target = next_target(kcov);
    const int L0 = L;
    while (kcov < target) {
      const int n = plan_terms(kcov, target);
      if (op->prof) {
        while ((int)op->evs.size() < 2 * (L - L0 + 1)) {
          hipEvent_t e;
          HIPCHK(hipEventCreate(&e));
          op->evs.push_back(e);
        }
        a.ev_start = op->evs[2 * (L - L0)];
        a.ev_stop = op->evs[2 * (L - L0) + 1];
      } else {
        a.ev_start = a.ev_stop = nullptr;
      }
      a.k = kcov;
      a.nterms = n;
      a.first = kcov == 0;
      a.yin = kcov == 0 ? (stage_u ? (const void*)stage_u : (const void*)v) : ybuf3[L % 3];
      a.yout = ybuf3[(L + 1) % 3];
      a.yin_f32 = (kcov > 0) && ys32;
      a.pin = kcov == 0 ? nullptr : pbuf[(L + 2) % 3];
      a.p = pbuf[L % 3];
      a.pmid = a.pmid2 = a.pmid3 = nullptr;
      a.w2 = (kcov == 0 && w2 && P.s[0] != 0.0) ? w2 : nullptr;
      a.w2c = P.s[kcov] * w2scale;
      a.shift = P.shift[kcov];
      a.shift2 = n >= 2 ? P.shift[kcov + 1] : 0.0;
      a.shift3 = n >= 3 ? P.shift[kcov + 2] : 0.0;
      a.shift4 = n == 4 ? P.shift[kcov + 3] : 0.0;
      a.dk1 = P.d[kcov + 1];
      a.dk2 = n >= 2 ? P.d[kcov + 2] : 0.0;
      a.dk3 = n >= 3 ? P.d[kcov + 3] : 0.0;
      a.dk4 = n == 4 ? P.d[kcov + 4] : 0.0;
      // four-term launch: field rows kept in LDS (faster than reading them
      // again on every grid measured, 256^2 to 1000^2, once the LDS rows were
      // accessed 16 bytes per lane, also where the blocks take two rounds)
      a.lds_fields = n == 4;
      a.slot = L & 1;
      a.nb_prev = prev_nb;
      a.k_prev = prev_k;
      a.nterms_prev = prev_n;
      a.slot_prev = prev_slot;
      a.decide_only = 0;
      const bool stage = kcov == 0 && stage_u != nullptr;
      if (stage) {
        // the four-stage march: w = A u + s, then terms 1 .. 3 (its p starts
        // at 0 and takes d_0 w as its first "term")
        a.stage = 1;
        a.src = stage_s;
        a.shift2 = P.shift[0];
        a.shift3 = P.shift[1];
        a.shift4 = P.shift[2];
        a.dk1 = P.d[0];
        a.dk2 = P.d[1];
        a.dk3 = P.d[2];
        a.dk4 = P.d[3];
        HIPCHK(launch_leja4s_step(op->f, T4s, a, st));
        a.stage = 0;
        a.src = nullptr;
      } else if (n == 4 && fours) HIPCHK(launch_leja4s_step(op->f, T4s, a, st));
      else if (n == 4) HIPCHK(launch_leja4_step(op->f, T4, a, st));
      else if (n == 3) HIPCHK(launch_leja3_step(op->f, T3, a, st));
      else if (n == 2) HIPCHK(launch_leja2_step(op->f, T2, a, st));
      else HIPCHK(launch_leja_step(op->f, T, a, st));
      lk.push_back(kcov);
      ln.push_back(n);
      prev_nb = stage     ? T4s.nblocks
                : n == 4  ? (fours ? T4s.nblocks : T4.nblocks)
                : n == 3  ? T3.nblocks
                : n == 2  ? T2.nblocks
                          : T.nblocks;
      prev_k = kcov;
      prev_n = n;
      prev_slot = L & 1;
      kcov += n;
      ++L;
    }
    // decision of the chunk's last launch
    a.ev_start = a.ev_stop = nullptr;
    a.k = kcov;
    a.nterms = 1;
    a.first = 0;
    a.w2 = nullptr;
    a.yin_f32 = ys32;
    a.nb_prev = prev_nb;
    a.k_prev = prev_k;
    a.nterms_prev = prev_n;
    a.slot_prev = prev_slot;
    a.decide_only = 1;
    // outcome: published to the host mirror and awaited by spinning, or (when
    // timing launches with events, which need the stream synchronised, or
    // without a mirror) copied back
    const bool spin = op->hctl && op->host_wait && !op->prof;
    a.hctl = spin ? op->hctl_dev : nullptr;
    a.hseq = spin ? (op->hseq = next_hseq()) : 0;
    HIPCHK(launch_leja_step(op->f, T, a, st));
    a.hctl = nullptr;
    RETCHK(spin ? await_outcome(op, st) : read_ctl(op, st));
    if (op->prof) {
      // launches after the one that ran beside the final decision skipped
      // their work: time the others
      const bool stopped = op->host_ctl->stop != 0;
      const int m = op->host_ctl->degree;
      bool past = false;
      for (int l = L0; l < L; ++l) {
        if (stopped && past) break;
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, op->evs[2 * (l - L0)], op->evs[2 * (l - L0) + 1]));
        // (a first launch with its stage vector reads u and s where others read v)
        const double b = leja_bytes(op, lk[l], lk[l] == 0 && ((w2 != nullptr && P.s[0] != 0.0) || stage_s));
        op->prof_ms += ms;
        op->prof_launches += 1;
        op->prof_bytes += b;
        const int kind = lk[l] == 0  ? ADL_LAUNCH_FIRST
                         : ln[l] == 4 ? ADL_LAUNCH_FOUR
                         : ln[l] == 3 ? ADL_LAUNCH_THREE
                         : ln[l] == 2 ? ADL_LAUNCH_TWO
                                      : ADL_LAUNCH_ONE;
        op->kind_ms[kind] += ms;
        op->kind_launches[kind] += 1;
        op->kind_bytes[kind] += b;
        op->kind_terms[kind] += ln[l];
        if (lk[l] >= m) past = true;  // this launch ran beside (or after) the final decision
      }
    }
    if (op->host_ctl->stop || kcov >= maxdeg) break;
  }
  out.degree = op->host_ctl->degree;
  out.status = op->host_ctl->stop ? op->host_ctl->status : 3;
  if (out.status == 1) {
    P.last_degree = out.degree;
    if (out.degree == 0) {
      HIPCHK(launch_fill(op->n, p_out, 0.0, st));
    } else {
      const int m = out.degree;
      const int Ls = launch_of_term(m);
      double* res = pbuf[Ls % 3];
      if (m != lk[Ls] + ln[Ls]) {
        // the sweep stopped inside launch Ls: replay it on its inputs (y in
        // ybuf3[Ls mod 3], p in pbuf[(Ls + 2) mod 3], both intact) storing p
        // of term m only, into p_out unless p_out holds its p input
        // (the first launch: y_0 = v, no p input; with its stage vector, v is
        // formed here first and the launch replayed in its three-term form)
        const int k = lk[Ls], n = ln[Ls], t = m - k;
        if (k == 0 && stage_u) {
          HIPCHK(launch_apply(op->f, tiling_for(op, stage_u, stage_s), stage_u, op->w1, stage_s, 1.0, nullptr, 0.0,
                              st));
          v = op->w1;
        }
        const double* pin = k == 0 ? nullptr : pbuf[(Ls + 2) % 3];
        double* dst = pin == p_out ? pbuf[Ls % 3] : p_out;
        a.ev_start = a.ev_stop = nullptr;
        a.k = k;
        a.nterms = n;
        a.first = k == 0;
        a.w2 = nullptr;
        a.yin = k == 0 ? (const void*)v : ybuf3[Ls % 3];
        a.yout = nullptr;
        a.yin_f32 = k > 0 && ys32;
        a.pin = pin;
        a.p = n == t ? dst : nullptr;
        a.pmid = t == 1 ? dst : nullptr;
        a.pmid2 = t == 2 ? dst : nullptr;
        a.pmid3 = t == 3 ? dst : nullptr;
        a.shift = P.shift[k];
        a.shift2 = n >= 2 ? P.shift[k + 1] : 0.0;
        a.shift3 = n >= 3 ? P.shift[k + 2] : 0.0;
        a.shift4 = n == 4 ? P.shift[k + 3] : 0.0;
        a.dk1 = P.d[k + 1];
        a.dk2 = n >= 2 ? P.d[k + 2] : 0.0;
        a.dk3 = n >= 3 ? P.d[k + 3] : 0.0;
        a.dk4 = n == 4 ? P.d[k + 4] : 0.0;
        a.lds_fields = n == 4;
        a.decide_only = 0;
        a.replay = 1;
        a.hctl = nullptr;
        if (n == 4 && fours) HIPCHK(launch_leja4s_step(op->f, T4s, a, st));
        else if (n == 4) HIPCHK(launch_leja4_step(op->f, T4, a, st));
        else if (n == 3) HIPCHK(launch_leja3_step(op->f, T3, a, st));
        else HIPCHK(launch_leja2_step(op->f, T2, a, st));
        a.replay = 0;
        res = dst;
      }
      if (res != p_out) HIPCHK(launch_axpby(op->n, p_out, 1.0, res, 0.0, nullptr, st));
    }
  }
  return ADL_OK;
}

int adl::substeps_for(double alpha, double dt, double rho_max) {
  const double r = std::fabs(alpha) * dt / rho_max;
  const double K = std::ceil(r);
  if (!(K < 1e6)) return 1 << 20;
  return std::max(1, (int)K);
}

struct Acc {
  int matvecs = 0, sweeps = 0, maxdeg = 0, lastdeg = 0, substeps = 0;
};

static void account(Acc& a, const SweepOut& o) {
  a.matvecs += o.degree;
  a.sweeps += 1;
  a.maxdeg = std::max(a.maxdeg, o.degree);
  a.lastdeg = o.degree;
}

static int status_to_code(int status) {
  if (status == 2) return fail(ADL_ENAN, "non-finite value in a Leja sweep (NaN/Inf input or overflow)");
  return fail(ADL_ENOCONV, "Leja sweep reached the degree cap without converging");
}

// y_acc = dt [phi_1(A dt) w1 + phi_2(A dt) w2] with K fixed substeps.
// Returns ADL_OK and ok = false if a sweep hit the degree cap.  With one
// substep and u_direct set, u_direct += dt p is applied instead (one update
// launch fewer) and `applied` is set.
static int combo_fixed(adl_op* op, const double* w1, const double* w2, double dt, double tol, int K, Acc& acc,
                       bool& ok, hipStream_t st, double* u_direct = nullptr, bool* applied = nullptr,
                       const double* stage_u = nullptr, const double* stage_s = nullptr) {
  const double h = dt / K;
  Plan& P = get_plan(op, 1, op->alpha, h);
  ok = true;
  for (int j = 0; j < K; ++j) {
    const double* f = w1;
    if (j > 0) {
      // f = A y + w1 + (j h/dt) w2
      HIPCHK(launch_apply(op->f, tiling_for(op, w1, w2), op->yacc, op->tmp, w1, 1.0, w2, (double)j * h / dt, st));
      acc.matvecs += 1;
      f = op->tmp;
    }
    SweepOut so;
    // (stage_u: w1 = A stage_u + stage_s is formed by the sweep's first launch; K = 1)
    RETCHK(sweep(op, P, f, w2, 1.0 / dt, op->p, tol, op->max_degree, st, so, j == 0 ? stage_u : nullptr,
                 j == 0 ? stage_s : nullptr));
    account(acc, so);
    if (so.status != 1) {
      if (so.status == 2) return status_to_code(2);
      ok = false;
      return ADL_OK;
    }
    if (K == 1 && u_direct) {
      HIPCHK(launch_axpby(op->n, u_direct, 1.0, u_direct, h, op->p, st));
      *applied = true;
    } else if (j == 0) {
      HIPCHK(launch_axpby(op->n, op->yacc, h, op->p, 0.0, nullptr, st));
    } else {
      HIPCHK(launch_axpby(op->n, op->yacc, 1.0, op->yacc, h, op->p, st));
    }
  }
  return ADL_OK;
}

// y_acc = dt [phi_1(A dt) w1 + phi_2(A dt) w2]  (w2 may be null); with
// u_direct set, a one-substep result may instead be added to u_direct
// directly (`applied` tells which happened).
static int phi_combo(adl_op* op, const double* w1, const double* w2, double dt, double tol, Acc& acc,
                     hipStream_t st, double* u_direct = nullptr, bool* applied = nullptr,
                     const double* stage_u = nullptr, const double* stage_s = nullptr) {
  bool dummy = false;
  if (!applied) applied = &dummy;
  *applied = false;
  if (op->alpha == 0.0) {
    HIPCHK(launch_axpby(op->n, op->yacc, dt, w1, w2 ? 0.5 * dt : 0.0, w2, st));
    acc.substeps = 0;
    return ADL_OK;
  }
  int K = substeps_for(op->alpha, dt, op->rho_max);
  if (op->learned) K = std::max(K, op->substeps_hint);
  for (int d = 0; d <= kMaxDoublings; ++d) {
    bool ok;
    if (stage_u && K > 1) {
      // substeps need w1 itself: form it
      HIPCHK(launch_apply(op->f, tiling_for(op, stage_u, stage_s), stage_u, op->w1, stage_s, 1.0, nullptr, 0.0, st));
      w1 = op->w1;
      stage_u = stage_s = nullptr;
    }
    RETCHK(combo_fixed(op, w1, w2, dt, tol, K, acc, ok, st, u_direct, applied, stage_u, stage_s));
    if (ok) {
      acc.substeps = K;
      return ADL_OK;
    }
    // a learned interval that needs more terms than predicted is suspect:
    // report it so that the caller falls back to power iteration
    if (op->learned) return status_to_code(3);
    K *= 2;
  }
  return status_to_code(3);
}

static void fill_stats(adl_stats* st, const Acc& a, adl_op* op, int code) {
  if (!st) return;
  st->matvecs = a.matvecs;
  st->sweeps = a.sweeps;
  st->max_degree = a.maxdeg;
  st->last_degree = a.lastdeg;
  st->substeps = a.substeps;
  st->status = code;
  st->alpha = op ? op->alpha : 0.0;
}

static int check_op(const adl_op* op) {
  if (!op) return fail(ADL_EINVAL, "null op");
  return ADL_OK;
}

static int check_bound(const adl_op* op) {
  if (!op->has_bound) return fail(ADL_EBOUND, "no spectral bound installed (adl_spectral_bound / adl_set_bound)");
  return ADL_OK;
}

static int check_tol(double tol) {
  if (!(tol > 0.0 && tol < 1.0)) return fail(ADL_EINVAL, "tol must be in (0, 1), got %g", tol);
  return ADL_OK;
}

static int check_dt(double dt) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ADL_EINVAL, "dt must be finite and > 0, got %g", dt);
  return ADL_OK;
}

static int gershgorin(adl_op* op, hipStream_t st, double& out) {
  HIPCHK(launch_ctl_reset(op->ctl, 1, st));
  HIPCHK(launch_gershgorin(op->f, op->partials, op->ctl, st));
  RETCHK(read_ctl(op, st));
  out = op->host_ctl->gmin;
  op->gersh = out;
  return ADL_OK;
}

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

const char* adl_last_error(void) { return g_err.c_str(); }

int adl_leja_points(int n, double* out) {
  if (!out || n < 1 || n > kMaxDegreeDefault + 1) return fail(ADL_EINVAL, "n must be in [1, %d]", kMaxDegreeDefault + 1);
  const std::vector<double>& xi = leja_table();
  std::copy(xi.begin(), xi.begin() + n, out);
  return ADL_OK;
}

int adl_newton_coefficients(int l, double alpha, double h, int n, double* out) {
  if (!out || n < 1 || n > kMaxDegreeDefault + 1) return fail(ADL_EINVAL, "n must be in [1, %d]", kMaxDegreeDefault + 1);
  if (l < 0 || l > 2) return fail(ADL_EINVAL, "l must be 0, 1 or 2");
  if (!(alpha < 0.0) || !std::isfinite(alpha) || !(h > 0.0)) return fail(ADL_EINVAL, "need alpha < 0, h > 0");
  Plan P;
  build_plan(P, l, alpha, h, n);
  std::copy(P.d.begin(), P.d.end(), out);
  return ADL_OK;
}

size_t adl_workspace_bytes(int nx, int ny, int storage, int max_degree) {
  (void)max_degree;
  if (nx < 3 || ny < 3 || storage < 0 || storage > 2) return 0;
  return ws_layout(nx, ny, storage).total;
}

int adl_op_create(int nx, int ny, double hx, double hy, int bc, int storage, const double* Dxx,
                  const double* Dxy, const double* Dyy, const double* ax, const double* ay, double ax_c,
                  double ay_c, void* workspace, size_t ws_bytes, void* stream, adl_op** out) {
  if (!out) return fail(ADL_EINVAL, "out is null");
  *out = nullptr;
  if (nx < 3 || ny < 3) return fail(ADL_EINVAL, "nx, ny must be >= 3 (got %d, %d)", nx, ny);
  if ((long)nx * ny > (1L << 31)) return fail(ADL_EINVAL, "grid too large");
  if (!(hx > 0.0) || !(hy > 0.0) || !std::isfinite(hx) || !std::isfinite(hy))
    return fail(ADL_EINVAL, "hx, hy must be finite and > 0");
  if (bc != ADL_BC_PERIODIC && bc != ADL_BC_DIRICHLET) return fail(ADL_EINVAL, "bad bc %d", bc);
  if (storage < 0 || storage > 2) return fail(ADL_EINVAL, "bad storage %d", storage);
  if (!Dxx || !Dxy || !Dyy) return fail(ADL_EINVAL, "null tensor field");
  if ((ax == nullptr) != (ay == nullptr)) return fail(ADL_EINVAL, "ax and ay must both be given or both NULL");
  if (!std::isfinite(ax_c) || !std::isfinite(ay_c)) return fail(ADL_EINVAL, "advection constants not finite");
  const WsLayout L = ws_layout(nx, ny, storage);
  if (!workspace) return fail(ADL_ENOWORKSPACE, "null workspace");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(ADL_ENOWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(ADL_ENOWORKSPACE, "workspace too small: %zu < %zu", ws_bytes, L.total);

  adl_op* op = new (std::nothrow) adl_op();
  if (!op) return fail(ADL_EINVAL, "out of host memory");
  char* base = reinterpret_cast<char*>(workspace);
  op->nx = nx;
  op->ny = ny;
  op->bc = bc;
  op->storage = storage;
  op->hx = hx;
  op->hy = hy;
  op->n = (long)nx * ny;
  const int f32 = storage != ADL_STORAGE_FP64;
  op->f.kxx = base + L.kxx;
  op->f.kxy = base + L.kxy;
  op->f.kyy = base + L.kyy;
  op->f.ax = ax ? base + L.ax : nullptr;
  op->f.ay = ay ? base + L.ay : nullptr;
  op->f.axc = ax_c / (2.0 * hx);
  op->f.ayc = ay_c / (2.0 * hy);
  op->f.nx = nx;
  op->f.ny = ny;
  op->f.bc = bc;
  op->f.f32 = f32;
  op->t = make_tiling(nx, ny, 0);
  op->t1 = make_tiling(nx, ny, 0, 1);
  op->t2 = make_tiling2(nx, ny, 0);
  op->t21 = make_tiling2(nx, ny, 0, 1);
  op->t3 = make_tiling2(nx, ny, 0, 0, kMaxGrid3);
  op->t4s = make_tiling2(nx, ny, 0, 0, kMaxGrid3, 2);
  op->t4 = make_tiling4(nx, ny);
  op->t41 = make_tiling4(nx, ny, 1);
  op->ybuf[0] = base + L.y0;
  op->ybuf[1] = base + L.y1;
  op->p = reinterpret_cast<double*>(base + L.p);
  op->w1 = reinterpret_cast<double*>(base + L.w1);
  op->w2 = reinterpret_cast<double*>(base + L.w2);
  op->yacc = reinterpret_cast<double*>(base + L.yacc);
  op->tmp = reinterpret_cast<double*>(base + L.tmp);
  op->tmp2 = reinterpret_cast<double*>(base + L.tmp2);
  op->p2 = reinterpret_cast<double*>(base + L.p2);
  op->p3 = reinterpret_cast<double*>(base + L.p3);
  op->p4 = reinterpret_cast<double*>(base + L.p4);
  op->slot_stride = kSlotRows * (long)max_partial_blocks(nx, ny);
  op->partials = reinterpret_cast<double*>(base + L.partials);
  op->ctl = reinterpret_cast<Ctl*>(base + L.ctl);
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&op->host_ctl), 4 * sizeof(Ctl), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete op;
    return fail(ADL_EHIP, "hipHostMalloc failed: %s", hipGetErrorString(e));
  }
  mirror_take(op);
  hipStream_t st = S(stream);
  const long n = op->n;
  int rc = ADL_OK;
  auto prep = [&](const double* src, double scale, const void* dst) -> int {
    HIPCHK(launch_prepare_field(n, src, scale, const_cast<void*>(dst), f32, st));
    return ADL_OK;
  };
  rc = prep(Dxx, 1.0 / (hx * hx), op->f.kxx);
  if (rc == ADL_OK) rc = prep(Dyy, 1.0 / (hy * hy), op->f.kyy);
  if (rc == ADL_OK) rc = prep(Dxy, 1.0 / (4.0 * hx * hy), op->f.kxy);
  if (rc == ADL_OK && ax) rc = prep(ax, 1.0 / (2.0 * hx), op->f.ax);
  if (rc == ADL_OK && ay) rc = prep(ay, 1.0 / (2.0 * hy), op->f.ay);
  if (rc == ADL_OK) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = fail(ADL_EHIP, "field preparation failed: %s", hipGetErrorString(e));
  }
  if (rc != ADL_OK) {
    hipHostFree(op->host_ctl);
    mirror_give(op);
    delete op;
    return rc;
  }
  (void)leja_table();
  *out = op;
  return ADL_OK;
}

int adl_op_destroy(adl_op* op) {
  if (!op) return ADL_OK;
  for (hipEvent_t e : op->evs) hipEventDestroy(e);
  if (op->host_ctl) hipHostFree(op->host_ctl);
  mirror_give(op);
  delete op;
  return ADL_OK;
}

int adl_op_set_limits(adl_op* op, int max_degree, double rho_max) {
  RETCHK(check_op(op));
  if (max_degree < 1 || max_degree > op->ws_max_degree)
    return fail(ADL_EINVAL, "max_degree must be in [1, %d]", op->ws_max_degree);
  if (!(rho_max > 0.0) || !std::isfinite(rho_max)) return fail(ADL_EINVAL, "rho_max must be > 0");
  op->max_degree = max_degree;
  op->rho_max = rho_max;
  return ADL_OK;
}

static void profile_reset(adl_op* op) {
  op->prof_ms = 0.0;
  op->prof_bytes = 0.0;
  op->prof_launches = 0;
  for (int k = 0; k < 5; ++k) {
    op->kind_ms[k] = op->kind_bytes[k] = 0.0;
    op->kind_launches[k] = op->kind_terms[k] = 0;
  }
}

int adl_op_profile(adl_op* op, int enable) {
  RETCHK(check_op(op));
  op->prof = enable != 0;
  profile_reset(op);
  return ADL_OK;
}

int adl_op_profile_read(adl_op* op, double* kernel_ms, long long* launches, double* bytes) {
  RETCHK(check_op(op));
  if (kernel_ms) *kernel_ms = op->prof_ms;
  if (launches) *launches = op->prof_launches;
  if (bytes) *bytes = op->prof_bytes;
  profile_reset(op);
  return ADL_OK;
}

int adl_op_profile_read_kind(const adl_op* op, int kind, double* kernel_ms, long long* launches, double* bytes,
                             long long* terms) {
  RETCHK(check_op(op));
  if (kind < ADL_LAUNCH_FIRST || kind > ADL_LAUNCH_THREE) return fail(ADL_EINVAL, "bad launch kind %d", kind);
  if (kernel_ms) *kernel_ms = op->kind_ms[kind];
  if (launches) *launches = op->kind_launches[kind];
  if (bytes) *bytes = op->kind_bytes[kind];
  if (terms) *terms = op->kind_terms[kind];
  return ADL_OK;
}

int adl_op_set_tiling(adl_op* op, int rows, int cols_per_lane) {
  RETCHK(check_op(op));
  if (rows < 0 || rows > op->ny) return fail(ADL_EINVAL, "rows must be in [0, ny]");
  if (cols_per_lane < 0 || cols_per_lane > 2) return fail(ADL_EINVAL, "cols_per_lane must be 0, 1 or 2");
  const Tiling t = make_tiling(op->nx, op->ny, rows, cols_per_lane);
  if (cols_per_lane == 2 && t.vec != 2) return fail(ADL_EINVAL, "two columns per lane need an even nx >= 128");
  op->t = t;
  op->t1 = make_tiling(op->nx, op->ny, rows, 1);
  op->t2 = make_tiling2(op->nx, op->ny, rows, cols_per_lane);
  op->t21 = make_tiling2(op->nx, op->ny, rows, 1);
  op->t3 = make_tiling2(op->nx, op->ny, rows, cols_per_lane, kMaxGrid3);
  op->t4s = make_tiling2(op->nx, op->ny, rows, cols_per_lane, kMaxGrid3, 2);
  op->t4 = make_tiling4(op->nx, op->ny, cols_per_lane);
  op->t41 = make_tiling4(op->nx, op->ny, 1);
  return ADL_OK;
}

int adl_op_set_term_fusion(adl_op* op, int mode) {
  RETCHK(check_op(op));
  if (mode < 0 || mode > 6) return fail(ADL_EINVAL, "term fusion mode must be 0 .. 6");
  if (mode == 6 && !four_staged_ok(op, 2))
    return fail(ADL_EINVAL, "four staged terms per launch need a grid whose tiling has two columns per lane");
  if (mode == 5 && !three_terms_ok(op, 2))
    return fail(ADL_EINVAL, "three terms per launch need a grid whose two-term tiling has two columns per lane");
  if (mode == 4 && !four_terms_ok(op))
    return fail(ADL_EINVAL, "four terms per launch need a sweep without non-temporal hints and, "
                            "on a periodic grid, ny >= 4 other than 5 and 9");
  op->fuse_terms = mode;
  return ADL_OK;
}

int adl_op_set_host_wait(adl_op* op, int mode) {
  RETCHK(check_op(op));
  if (mode != 0 && mode != 1) return fail(ADL_EINVAL, "host wait mode must be 0 or 1");
  op->host_wait = mode;
  return ADL_OK;
}

int adl_op_host_wait(const adl_op* op, int* mode) {
  RETCHK(check_op(op));
  if (!mode) return fail(ADL_EINVAL, "null mode");
  *mode = op->hctl && op->host_wait ? 1 : 0;
  return ADL_OK;
}

int adl_op_set_streaming(adl_op* op, int mode) {
  RETCHK(check_op(op));
  if (mode < -1 || mode > 1) return fail(ADL_EINVAL, "streaming mode must be -1, 0 or 1");
  op->streaming = mode;
  return ADL_OK;
}

int adl_op_get_tiling(const adl_op* op, int* vec, int* rows, int* nblocks) {
  RETCHK(check_op(op));
  if (vec) *vec = op->t.vec;
  if (rows) *rows = op->t.rows;
  if (nblocks) *nblocks = op->t.nblocks;
  return ADL_OK;
}

int adl_op_set_quad2_mode(adl_op* op, int mode) {
  RETCHK(check_op(op));
  if (mode != ADL_QUAD2_AUGMENTED && mode != ADL_QUAD2_TWO_SWEEP) return fail(ADL_EINVAL, "bad quad2 mode");
  op->quad2_mode = mode;
  return ADL_OK;
}

int adl_apply(adl_op* op, const double* x, double* y, void* stream) {
  RETCHK(check_op(op));
  if (!x || !y) return fail(ADL_EINVAL, "null vector");
  if (x == y) return fail(ADL_EINVAL, "x and y must not alias");
  HIPCHK(launch_apply(op->f, tiling_for(op, x, y), x, y, nullptr, 0.0, nullptr, 0.0, S(stream)));
  return ADL_OK;
}

int adl_spectral_bound(adl_op* op, int method, int max_iter, double rtol, uint64_t seed, double* alpha_out,
                       int* iters_out, void* stream) {
  RETCHK(check_op(op));
  if (method != ADL_BOUND_GERSHGORIN && method != ADL_BOUND_POWER) return fail(ADL_EINVAL, "bad method");
  hipStream_t st = S(stream);
  double ag;
  RETCHK(gershgorin(op, st, ag));
  if (!std::isfinite(ag)) return fail(ADL_ENAN, "non-finite Gershgorin bound (fields contain NaN/Inf?)");
  double alpha = ag;
  int iters = 0;
  if (method == ADL_BOUND_POWER) {
    if (max_iter < 1) return fail(ADL_EINVAL, "max_iter must be >= 1");
    if (!(rtol > 0.0)) return fail(ADL_EINVAL, "rtol must be > 0");
    HIPCHK(launch_ctl_reset(op->ctl, 1, st));
    const Tiling& T = op->t;
    HIPCHK(launch_power_init(T, op->n, seed, op->tmp, op->partials, st));
    double* bufs[2] = {op->tmp, op->tmp2};
    PowerArgs pa{};
    pa.rtol = rtol;
    pa.max_iter = max_iter;
    pa.nb = T.nblocks;
    pa.partials = op->partials;
    pa.ctl = op->ctl;
    int launched = 0;
    while (true) {
      const int chunk = std::min(max_iter - launched, launched == 0 ? 64 : 128);
      for (int i = 0; i < chunk; ++i) {
        const int k = launched + i;
        pa.x = bufs[k & 1];
        pa.w = bufs[(k + 1) & 1];
        pa.k = k;
        pa.decide_only = 0;
        HIPCHK(launch_power_step(op->f, T, pa, st));
      }
      launched += chunk;
      pa.k = launched;
      pa.decide_only = 1;
      HIPCHK(launch_power_step(op->f, T, pa, st));
      RETCHK(read_ctl(op, st));
      if (op->host_ctl->stop || launched >= max_iter) break;
    }
    const Ctl& c = *op->host_ctl;
    if (c.status == 2) return fail(ADL_ENAN, "non-finite value in power iteration");
    iters = c.iters;
    const double lam = c.lam;
    op->last_lambda = lam;
    alpha = -std::min(1.1 * lam, std::fabs(ag));
  }
  if (alpha == 0.0 && ag != 0.0) return fail(ADL_EBOUND, "power iteration gave lambda = 0");
  op->alpha = alpha;
  op->has_bound = true;
  op->learned = false;
  if (alpha_out) *alpha_out = alpha;
  if (iters_out) *iters_out = iters;
  return ADL_OK;
}

int adl_last_power_estimate(const adl_op* op, double* lambda) {
  RETCHK(check_op(op));
  if (!lambda) return fail(ADL_EINVAL, "null lambda");
  if (std::isnan(op->last_lambda)) return fail(ADL_EBOUND, "no power iteration has run on this op");
  *lambda = op->last_lambda;
  return ADL_OK;
}

int adl_set_bound(adl_op* op, double alpha) {
  RETCHK(check_op(op));
  if (!std::isfinite(alpha) || alpha > 0.0) return fail(ADL_EBOUND, "alpha must be finite and < 0 (got %g)", alpha);
  if (alpha == 0.0) {
    double ag = op->gersh;
    if (std::isnan(ag)) RETCHK(gershgorin(op, nullptr, ag));
    if (ag != 0.0) return fail(ADL_EBOUND, "alpha = 0 is only valid for the zero operator");
  }
  op->alpha = alpha;
  op->has_bound = true;
  op->learned = false;
  return ADL_OK;
}

int adl_get_bound(const adl_op* op, double* alpha) {
  RETCHK(check_op(op));
  if (!alpha) return fail(ADL_EINVAL, "null alpha");
  if (!op->has_bound) return fail(ADL_EBOUND, "no bound installed");
  *alpha = op->alpha;
  return ADL_OK;
}

int adl_leja_phi(adl_op* op, int l, double dt, const double* v, double* out, double tol, int max_degree,
                 adl_stats* stp, void* stream) {
  RETCHK(check_op(op));
  if (l < 0 || l > 2) return fail(ADL_EINVAL, "l must be 0, 1 or 2");
  if (!v || !out) return fail(ADL_EINVAL, "null vector");
  if (v == out) return fail(ADL_EINVAL, "out must not alias v");
  RETCHK(check_dt(dt));
  RETCHK(check_tol(tol));
  RETCHK(check_bound(op));
  const int saved = op->max_degree;
  if (max_degree > 0) {
    if (max_degree > op->ws_max_degree) return fail(ADL_EINVAL, "max_degree too large");
    op->max_degree = max_degree;
  }
  hipStream_t st = S(stream);
  Acc acc;
  int code = ADL_OK;
  auto run = [&]() -> int {
    if (op->alpha == 0.0) {
      const double f = l == 0 ? 1.0 : (l == 1 ? 1.0 : 0.5);
      HIPCHK(launch_axpby(op->n, out, f, v, 0.0, nullptr, st));
      acc.substeps = 0;
      return ADL_OK;
    }
    int K = substeps_for(op->alpha, dt, op->rho_max);
    for (int dbl = 0; dbl <= kMaxDoublings; ++dbl) {
      if (K == 1) {
        Plan& P = get_plan(op, l, op->alpha, dt);
        SweepOut so;
        RETCHK(sweep(op, P, v, nullptr, 0.0, out, tol, op->max_degree, st, so));
        account(acc, so);
        if (so.status == 1) {
          acc.substeps = 1;
          return ADL_OK;
        }
        if (so.status == 2) return status_to_code(2);
      } else if (l == 0) {
        const double h = dt / K;
        Plan& P = get_plan(op, 0, op->alpha, h);
        const double* src = v;
        double* bufs[2] = {op->tmp, op->tmp2};
        bool ok = true;
        for (int j = 0; j < K; ++j) {
          double* dst = (j == K - 1) ? out : bufs[j & 1];
          // the K chained sweeps' relative errors add up: each gets tol / K
          SweepOut so;
          RETCHK(sweep(op, P, src, nullptr, 0.0, dst, tol / K, op->max_degree, st, so));
          account(acc, so);
          if (so.status == 2) return status_to_code(2);
          if (so.status != 1) {
            ok = false;
            break;
          }
          src = dst;
        }
        if (ok) {
          acc.substeps = K;
          return ADL_OK;
        }
      } else {
        bool ok;
        if (l == 1) {
          RETCHK(combo_fixed(op, v, nullptr, dt, tol, K, acc, ok, st));
        } else {
          HIPCHK(launch_fill(op->n, op->w1, 0.0, st));
          RETCHK(combo_fixed(op, op->w1, v, dt, tol, K, acc, ok, st));
        }
        if (ok) {
          HIPCHK(launch_axpby(op->n, out, 1.0 / dt, op->yacc, 0.0, nullptr, st));
          acc.substeps = K;
          return ADL_OK;
        }
      }
      K *= 2;
    }
    return status_to_code(3);
  };
  code = run();
  op->max_degree = saved;
  fill_stats(stp, acc, op, code);
  return code;
}

static int midpoint_impl(adl_op* op, double* u, const double* S_half, double dt, double tol, adl_stats* stp,
                         void* stream) {
  RETCHK(check_op(op));
  if (!u) return fail(ADL_EINVAL, "null u");
  RETCHK(check_dt(dt));
  RETCHK(check_tol(tol));
  RETCHK(check_bound(op));
  hipStream_t st = S(stream);
  Acc acc;
  // w = A u + S(t + dt/2), or formed by the sweep's first launch itself
  // (one launch fewer over the grid: 4096^2 FP64 steps 4.99 -> 4.87 ms)
  const bool fused = stage_fusable(op, u, S_half, dt);
  if (!fused) HIPCHK(launch_apply(op->f, tiling_for(op, u, S_half), u, op->w1, S_half, 1.0, nullptr, 0.0, st));
  acc.matvecs += 1;
  bool applied = false;
  int code = phi_combo(op, fused ? nullptr : op->w1, nullptr, dt, tol, acc, st, u, &applied, fused ? u : nullptr,
                       fused ? S_half : nullptr);
  if (code == ADL_OK && !applied) {
    hipError_t e = launch_axpby(op->n, u, 1.0, u, 1.0, op->yacc, st);
    if (e != hipSuccess) code = fail(ADL_EHIP, "update failed: %s", hipGetErrorString(e));
  }
  fill_stats(stp, acc, op, code);
  return code;
}

static int quad2_impl(adl_op* op, double* u, const double* S1, const double* S2, double c1, double c2, double dt,
                      double tol, adl_stats* stp, void* stream) {
  RETCHK(check_op(op));
  if (!u) return fail(ADL_EINVAL, "null u");
  if (!std::isfinite(c1) || !std::isfinite(c2) || c1 == c2) return fail(ADL_EINVAL, "need finite c1 != c2");
  RETCHK(check_dt(dt));
  RETCHK(check_tol(tol));
  RETCHK(check_bound(op));
  hipStream_t st = S(stream);
  Acc acc;
  const double inv = 1.0 / (c2 - c1);
  // w1 = A u + (c2 S1 - c1 S2)/(c2 - c1),  w2 = (S2 - S1)/(c2 - c1) (the
  // difference taken first; with both sources, w2 is a second output of the
  // stage launch)
  const double* w2 = nullptr;
  if (S1 && S2) {
    HIPCHK(launch_apply2(op->f, tiling_for(op, u, S1, S2), u, op->w1, S1, c2 * inv, S2, -c1 * inv, op->w2, inv,
                         st));
    w2 = op->w2;
  } else {
    HIPCHK(launch_apply(op->f, tiling_for(op, u, S1, S2), u, op->w1, S1, c2 * inv, S2, -c1 * inv, st));
    if (S2) HIPCHK(launch_axpby(op->n, op->w2, inv, S2, 0.0, nullptr, st));
    else if (S1) HIPCHK(launch_axpby(op->n, op->w2, -inv, S1, 0.0, nullptr, st));
    if (S1 || S2) w2 = op->w2;
  }
  acc.matvecs += 1;
  int code = ADL_OK;
  bool applied = false;
  if (op->quad2_mode == ADL_QUAD2_AUGMENTED || op->alpha == 0.0) {
    code = phi_combo(op, op->w1, w2, dt, tol, acc, st, u, &applied);
  } else {
    // two sweeps: dt (phi_1 w1 + phi_2 w2)
    adl_stats s1{}, s2{};
    code = adl_leja_phi(op, 1, dt, op->w1, op->tmp2, tol, 0, &s1, stream);
    if (code == ADL_OK) {
      acc.matvecs += s1.matvecs;
      acc.sweeps += s1.sweeps;
      acc.maxdeg = std::max(acc.maxdeg, s1.max_degree);
      acc.lastdeg = s1.last_degree;
      acc.substeps = s1.substeps;
      if (w2) {
        // phi_2 result into w1 (w1 is no longer needed)
        code = adl_leja_phi(op, 2, dt, w2, op->w1, tol, 0, &s2, stream);
        if (code == ADL_OK) {
          acc.matvecs += s2.matvecs;
          acc.sweeps += s2.sweeps;
          acc.maxdeg = std::max(acc.maxdeg, s2.max_degree);
          acc.lastdeg = s2.last_degree;
          hipError_t e = launch_axpby(op->n, op->tmp2, 1.0, op->tmp2, 1.0, op->w1, st);
          if (e != hipSuccess) code = fail(ADL_EHIP, "combine failed");
        }
      }
      if (code == ADL_OK) {
        hipError_t e = launch_axpby(op->n, op->yacc, dt, op->tmp2, 0.0, nullptr, st);
        if (e != hipSuccess) code = fail(ADL_EHIP, "scale failed");
      }
    }
  }
  if (code == ADL_OK && !applied) {
    hipError_t e = launch_axpby(op->n, u, 1.0, u, 1.0, op->yacc, st);
    if (e != hipSuccess) code = fail(ADL_EHIP, "update failed: %s", hipGetErrorString(e));
  }
  fill_stats(stp, acc, op, code);
  return code;
}


// ---------------------------------------------------------------------------
// learned bound: statistics and MLP
// ---------------------------------------------------------------------------
int adl_field_stats(adl_op* op, double dt, float* feats, void* stream) {
  RETCHK(check_op(op));
  if (!feats) return fail(ADL_EINVAL, "null feats");
  RETCHK(check_dt(dt));
  hipStream_t st = S(stream);
  HIPCHK(launch_ctl_reset(op->ctl, 1, st));
  HIPCHK(launch_field_stats(op->f, op->hx, op->hy, dt, feats, op->partials, op->ctl, st));
  return ADL_OK;
}

int adl_mlp_forward(const float* W, const float* X, float* Y, float* act_cache, int B, void* stream) {
  if (!W || !X || !Y) return fail(ADL_EINVAL, "null pointer");
  if (B < 1) return fail(ADL_EINVAL, "B must be >= 1");
  HIPCHK(launch_mlp_forward(W, X, Y, act_cache, B, S(stream)));
  return ADL_OK;
}

int adl_mlp_backward(const float* W, const float* act_cache, const float* dY, float* dW, int B, void* stream) {
  if (!W || !act_cache || !dY || !dW) return fail(ADL_EINVAL, "null pointer");
  if (B < 1) return fail(ADL_EINVAL, "B must be >= 1");
  HIPCHK(launch_mlp_backward(W, act_cache, dY, dW, B, S(stream)));
  return ADL_OK;
}

int adl_mlp_adam_step(float* W, const float* dW, float* m1, float* m2, int t, float lr, float beta1, float beta2,
                      float eps, void* stream) {
  if (!W || !dW || !m1 || !m2) return fail(ADL_EINVAL, "null pointer");
  if (t < 1) return fail(ADL_EINVAL, "t must be >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && lr >= 0.0f))
    return fail(ADL_EINVAL, "bad Adam hyper-parameters");
  HIPCHK(launch_mlp_adam(W, dW, m1, m2, t, lr, beta1, beta2, eps, S(stream)));
  return ADL_OK;
}


// ---------------------------------------------------------------------------
// steps with the learned-bound fallback
// ---------------------------------------------------------------------------
static int fallback_to_power(adl_op* op, void* stream) {
  op->learned = false;
  double a;
  return adl_spectral_bound(op, ADL_BOUND_POWER, 2000, 1e-3, 0, &a, nullptr, stream);
}

int adl_exp_midpoint_step(adl_op* op, double* u, const double* S_half, double dt, double tol, adl_stats* stp,
                          void* stream) {
  RETCHK(check_op(op));
  const bool learned = op->learned;
  int rc = midpoint_impl(op, u, S_half, dt, tol, stp, stream);
  if (learned && (rc == ADL_ENOCONV || rc == ADL_ENAN)) {
    adl_stats first{};
    if (stp) first = *stp;
    RETCHK(fallback_to_power(op, stream));
    rc = midpoint_impl(op, u, S_half, dt, tol, stp, stream);
    if (stp) {
      stp->matvecs += first.matvecs;
      stp->sweeps += first.sweeps;
      stp->fallback = 1;
    }
  }
  return rc;
}

int adl_exp_quad2_step(adl_op* op, double* u, const double* S1, const double* S2, double c1, double c2, double dt,
                       double tol, adl_stats* stp, void* stream) {
  RETCHK(check_op(op));
  const bool learned = op->learned;
  int rc = quad2_impl(op, u, S1, S2, c1, c2, dt, tol, stp, stream);
  if (learned && (rc == ADL_ENOCONV || rc == ADL_ENAN)) {
    adl_stats first{};
    if (stp) first = *stp;
    RETCHK(fallback_to_power(op, stream));
    rc = quad2_impl(op, u, S1, S2, c1, c2, dt, tol, stp, stream);
    if (stp) {
      stp->matvecs += first.matvecs;
      stp->sweeps += first.sweeps;
      stp->fallback = 1;
    }
  }
  return rc;
}

// ---------------------------------------------------------------------------
// learned bound: dimensionless inputs and targets of the predictor
// ---------------------------------------------------------------------------
// raw statistics (adl_field_stats): log10 kpar_max, log10 kpar_mean,
// log10 kperp_max, log10 kperp_mean, a_max, a_mean, log10 hx, log10 hy, log10 dt;
// g = |alpha_G|, the Gershgorin bound, sets the scale of the spectrum and
// rho_ref = 4 kpar_max (1/hx^2 + 1/hy^2) the diffusive scale.
static double rho_ref_of(const float* f) {
  const double kmax = std::pow(10.0, (double)f[0]);
  const double hx = std::pow(10.0, (double)f[6]), hy = std::pow(10.0, (double)f[7]);
  return 4.0 * kmax * (1.0 / (hx * hx) + 1.0 / (hy * hy));
}

int adl_learned_features(const float* f, double g, float* x) {
  if (!f || !x) return fail(ADL_EINVAL, "null pointer");
  if (!(g > 0.0) || !std::isfinite(g)) return fail(ADL_EINVAL, "Gershgorin bound must be > 0");
  const double kmax = std::pow(10.0, (double)f[0]);
  const double hx = std::pow(10.0, (double)f[6]), hy = std::pow(10.0, (double)f[7]);
  const double dt = std::pow(10.0, (double)f[8]);
  const double hmin = std::min(hx, hy);
  x[0] = (float)(f[1] - f[0]);                                 // mean / max k_par
  x[1] = (float)(f[2] - f[0]);                                 // max k_perp / max k_par
  x[2] = (float)(f[3] - f[0]);                                 // mean k_perp / max k_par
  x[3] = (float)std::log10(1.0 + (double)f[4] * hmin / kmax);  // cell Peclet (max)
  x[4] = (float)std::log10(1.0 + (double)f[5] * hmin / kmax);  // cell Peclet (mean)
  x[5] = (float)(f[6] - f[7]);                                 // hx / hy
  x[6] = (float)(std::log10(g * dt) / 4.0);                    // stiffness of the step
  x[7] = (float)std::log10(1.0 + (double)f[4] * dt / hmin);    // advective Courant number
  x[8] = (float)std::log10(g / rho_ref_of(f));                 // Gershgorin / diffusive scale
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(x[i])) return fail(ADL_EINVAL, "non-finite feature");
  return ADL_OK;
}

int adl_learned_targets(const float* f, double g, double rho, int degree, int substeps, float* y) {
  if (!f || !y) return fail(ADL_EINVAL, "null pointer");
  if (!(rho > 0.0) || !(g > 0.0) || degree < 0 || substeps < 1) return fail(ADL_EINVAL, "bad label");
  const double dt = std::pow(10.0, (double)f[8]);
  y[0] = (float)(10.0 * std::log10(rho / g));
  y[1] = (float)((double)degree / std::sqrt(rho * dt / substeps + 1.0));
  y[2] = (float)std::log2((double)substeps);
  return ADL_OK;
}

int adl_learned_decode(const float* f, double g, const float* y, double* rho, int* degree, int* substeps) {
  if (!f || !y) return fail(ADL_EINVAL, "null pointer");
  if (!(g > 0.0)) return fail(ADL_EINVAL, "Gershgorin bound must be > 0");
  const double dt = std::pow(10.0, (double)f[8]);
  const double r = g * std::pow(10.0, (double)y[0] / 10.0);
  int K = (int)std::lround(std::pow(2.0, (double)y[2]));
  if (K < 1) K = 1;
  const double m = std::max(1.0, (double)y[1] * std::sqrt(r * dt / K + 1.0));
  if (rho) *rho = r;
  if (degree) *degree = (int)std::ceil(m);
  if (substeps) *substeps = K;
  return ADL_OK;
}

// Installs the learned interval of op from its field statistics f, Gershgorin
// bound ag, network input x and output y (shared by the one-op and many-op
// entry points); *m receives the predicted Leja degree.
static int install_learned(adl_op* op, const float (&f)[9], double ag, const float (&x)[9], const float (&y)[3],
                           adl_learned_info* info, int* m_out) {
  double rho;
  int m, K;
  RETCHK(adl_learned_decode(f, -ag, y, &rho, &m, &K));
  const double alpha = -std::min(kLearnedSafety * rho, std::fabs(ag));
  if (!(alpha < 0.0) || !std::isfinite(alpha)) return fail(ADL_EBOUND, "learned bound unusable");
  op->alpha = alpha;
  op->has_bound = true;
  op->learned = true;
  op->budget = std::min(op->max_degree, (int)std::ceil(1.5 * m) + 10);
  op->substeps_hint = K;
  *m_out = m;
  if (info) {
    info->rho_hat = rho;
    info->alpha = alpha;
    info->gershgorin = ag;
    info->degree_hat = m;
    info->substeps_hat = K;
    for (int i = 0; i < 9; ++i) {
      info->feats[i] = f[i];
      info->x[i] = x[i];
    }
    for (int i = 0; i < 3; ++i) info->y[i] = y[i];
  }
  return ADL_OK;
}

// Builds the plan (Newton coefficients) of op's first step of size dt on the
// installed learned interval and seeds its predicted degree m, so that the
// first chunk of the sweep is sized right.
static void seed_plan(adl_op* op, double dt, int m) {
  const int Kp = std::max(op->substeps_hint, substeps_for(op->alpha, dt, op->rho_max));
  Plan& P = get_plan(op, 1, op->alpha, dt / Kp);
  if (P.last_degree <= 0) P.last_degree = m;
}

// seed_plan for n distinct ops on up to 16 host threads (a plan is O(M^2)
// divided differences on the host, ~0.1 ms at M = 501; each thread builds the
// plans of its own ops, so the coefficients are those of the serial build)
static void seed_plans(int n, adl_op* const* ops, double dt, const int* m) {
  const long hw = std::max(1u, std::thread::hardware_concurrency());
  const int nt = (int)std::min({hw, 16L, (long)(n + 7) / 8});
  std::vector<std::thread> th;
  if (nt > 1) {
    try {
      for (int t = 0; t < nt; ++t)
        th.emplace_back([=] {
          for (int i = t; i < n; i += nt) seed_plan(ops[i], dt, m[i]);
        });
    } catch (const std::system_error&) {
      // fewer threads than asked: the serial pass below completes the rest
    }
  }
  for (std::thread& x : th) x.join();
  if ((int)th.size() < nt || nt <= 1)
    for (int i = 0; i < n; ++i) seed_plan(ops[i], dt, m[i]);  // plans already built are found, not rebuilt
}

int adl_learned_bound(adl_op* op, double dt, const float* W, float* scratch, adl_learned_info* info, void* stream) {
  RETCHK(check_op(op));
  if (!W || !scratch) return fail(ADL_EINVAL, "null W or scratch");
  RETCHK(check_dt(dt));
  hipStream_t st = S(stream);
  float* d_feat = scratch;        // 9
  float* d_x = scratch + 12;      // 9
  float* d_y = scratch + 24;      // 3
  RETCHK(adl_field_stats(op, dt, d_feat, stream));
  float f[9], x[9], y[3];
  HIPCHK(hipMemcpyAsync(f, d_feat, sizeof f, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double ag = op->gersh;
  if (std::isnan(ag)) RETCHK(gershgorin(op, st, ag));
  if (!(ag < 0.0)) return fail(ADL_EBOUND, "zero operator: no learned interval");
  RETCHK(adl_learned_features(f, -ag, x));
  HIPCHK(hipMemcpyAsync(d_x, x, sizeof x, hipMemcpyHostToDevice, st));
  HIPCHK(launch_mlp_forward(W, d_x, d_y, nullptr, 1, st));
  HIPCHK(hipMemcpyAsync(y, d_y, sizeof y, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int m = 0;
  RETCHK(install_learned(op, f, ag, x, y, info, &m));
  seed_plan(op, dt, m);
  return ADL_OK;
}

int adl_learned_bound_many(int n, adl_op* const* ops, double dt, const float* W, float* scratch,
                           adl_learned_info* infos, void* stream) {
  if (n < 1 || !ops) return fail(ADL_EINVAL, "need n >= 1 ops");
  for (int i = 0; i < n; ++i) RETCHK(check_op(ops[i]));
  {
    std::vector<adl_op*> sorted(ops, ops + n);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return fail(ADL_EINVAL, "an op appears twice");
  }
  if (!W || !scratch) return fail(ADL_EINVAL, "null W or scratch");
  if (reinterpret_cast<uintptr_t>(scratch) % 16) return fail(ADL_EINVAL, "scratch must be 16-byte aligned");
  RETCHK(check_dt(dt));
  hipStream_t st = S(stream);
  // scratch (72 n floats): statistics [0, 9n), network input [12n, 21n) and
  // output [24n, 27n) as floats; Gershgorin bounds as doubles from float 28n;
  // the jobs from byte 128n (128 B each), then their first blocks (n + 1 ints)
  unsigned char* base = reinterpret_cast<unsigned char*>(scratch);
  float* d_feat = scratch;
  float* d_x = scratch + 12L * n;
  float* d_y = scratch + 24L * n;
  double* d_gmin = reinterpret_cast<double*>(scratch + 28L * n);
  BoundJob* d_jobs = reinterpret_cast<BoundJob*>(base + 128L * n);
  int* d_blk0 = reinterpret_cast<int*>(base + 256L * n);
  // every op's statistics and missing Gershgorin bound in one launch
  std::vector<unsigned char> up(128L * n + 4L * (n + 1));
  BoundJob* jobs = reinterpret_cast<BoundJob*>(up.data());
  int* blk0 = reinterpret_cast<int*>(up.data() + 128L * n);
  long total = 0;
  for (int i = 0; i < n; ++i) {
    const adl_op* op = ops[i];
    const int nb = stats_blocks((long)op->nx * op->ny);
    BoundJob& J = jobs[i];
    J = BoundJob{};
    J.f = op->f;
    J.hx = op->hx;
    J.hy = op->hy;
    J.partials = op->partials;
    J.ctl = op->ctl;
    J.blk0 = (int)total;
    J.nb_s = nb;
    J.nb_g = std::isnan(op->gersh) ? nb : 0;
    blk0[i] = (int)total;
    total += J.nb_s + J.nb_g;
    if (total > INT_MAX) return fail(ADL_EINVAL, "too many ops for one statistics launch");
  }
  blk0[n] = (int)total;
  HIPCHK(hipMemcpyAsync(d_jobs, up.data(), up.size(), hipMemcpyHostToDevice, st));
  HIPCHK(launch_bound_stats_many(d_jobs, d_blk0, n, (int)total, dt, d_feat, d_gmin, st));
  std::vector<unsigned char> down(120L * n);
  HIPCHK(hipMemcpyAsync(down.data(), scratch, down.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const float* f = reinterpret_cast<const float*>(down.data());
  const double* gmin = reinterpret_cast<const double*>(down.data() + 112L * n);
  std::vector<float> x(9L * n), y(3L * n);
  std::vector<double> ag(n);
  for (int i = 0; i < n; ++i) {
    if (jobs[i].nb_g) ops[i]->gersh = gmin[i];
    ag[i] = ops[i]->gersh;
    if (!(ag[i] < 0.0)) return fail(ADL_EBOUND, "op %d: zero operator, no learned interval", i);
    RETCHK(adl_learned_features(&f[9L * i], -ag[i], &x[9L * i]));
  }
  // one forward pass of the network over all ops
  HIPCHK(hipMemcpyAsync(d_x, x.data(), sizeof(float) * 9 * n, hipMemcpyHostToDevice, st));
  HIPCHK(launch_mlp_forward(W, d_x, d_y, nullptr, n, st));
  HIPCHK(hipMemcpyAsync(y.data(), d_y, sizeof(float) * 3 * n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<int> m(n);
  for (int i = 0; i < n; ++i) {
    float fi[9], xi[9], yi[3];
    std::copy(&f[9L * i], &f[9L * i] + 9, fi);
    std::copy(&x[9L * i], &x[9L * i] + 9, xi);
    std::copy(&y[3L * i], &y[3L * i] + 3, yi);
    const int rc = install_learned(ops[i], fi, ag[i], xi, yi, infos ? &infos[i] : nullptr, &m[i]);
    if (rc != ADL_OK) {
      seed_plans(i, ops, dt, m.data());
      return rc;
    }
  }
  seed_plans(n, ops, dt, m.data());
  return ADL_OK;
}

int adl_mlp_mse_grad(const float* Y, const float* T, float* dY, float* loss, int B, void* stream) {
  if (!Y || !T || !dY) return fail(ADL_EINVAL, "null pointer");
  if (B < 1) return fail(ADL_EINVAL, "B must be >= 1");
  HIPCHK(launch_mlp_mse_grad(Y, T, dY, loss, B, S(stream)));
  return ADL_OK;
}

}  // extern "C"
