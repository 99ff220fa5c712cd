// liblsq C ABI and refinement drivers.
//
// LSE (Section 3.1): the generalized RQ factorization B = [0, R] Q, A = Z T Q
// is computed as two Householder QRs.  The RQ of B is the QR of the reversed
// transpose  Bt = J_n B^T J_p = Qt [Rt; 0]  so that R = J Rt^T J and
// Q = J Qt^T J (J reverses index order); then  Abar = A Q^T  is formed as the
// reversed transpose of  Qt^T (J_n A^T)  and factored as Abar = Z T.
// The correction solver (Algorithm 1) is carried out in that basis: every
// quantity that involves R or Q is kept reversed (u~ = J u, y2~ = J y2, ...).
//
// GLS (Section 3.2): W = Q [R; 0] is a plain QR; V' = Q^T V; the RQ V' = T Z
// is the QR of  Vt = J_p V'^T J_n = Zt Rv  (T = J_n Rv^T J_p, Z = J_p Zt^T J_p),
// and Algorithm 3 is carried out with the blocks of Rv.
//
// The initial guess of Algorithms 2 and 4 (null-space / Paige solution at
// u_f, then r0, v0 resp. z0) equals, in exact arithmetic, one correction
// solve started from the zero iterate with residual (b, d, 0) resp. (0, d, 0);
// the solvers here compute it that way.  Residuals and updates are FP64.
#include <algorithm>
#include <atomic>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "engine.hpp"
#include "segs.hpp"
#include "lsq.h"
#include "lsq_debug.h"

using namespace lsq;

static_assert(kSelWeights == LSQ_SELECTOR_WEIGHTS, "selector weight layout");
static_assert(kSelFeatures == LSQ_SELECTOR_FEATURES, "selector feature count");

// --------------------------------------------------------------- arena --
namespace lsq {
Arena::~Arena() { release(); }
void* Arena::alloc(size_t bytes) {
  if (frozen_) throw std::runtime_error("an allocation was requested where none is allowed");
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  while (cur_ < chunks_.size()) {
    Chunk& c = chunks_[cur_];
    if (c.used + bytes <= c.size) {
      void* p = c.base + c.used;
      c.used += bytes;
      high_ = std::max(high_, in_use());
      return p;
    }
    if (fixed_) break;
    ++cur_;
  }
  if (fixed_)
    throw std::runtime_error("the workspace needs more than the " +
                             std::to_string(chunks_.empty() ? 0 : chunks_[0].size) +
                             " bytes of the fixed scratch buffer");
  size_t sz = bytes > (size_t(256) << 20) ? bytes : (size_t(256) << 20);
  void* base = nullptr;
  LSQ_HIP(hipMalloc(&base, sz));
  chunks_.push_back(Chunk{static_cast<char*>(base), sz, bytes, true});
  cur_ = chunks_.size() - 1;
  high_ = std::max(high_, in_use());
  return base;
}
void Arena::adopt_fixed(void* base, size_t bytes) {
  release();
  chunks_.push_back(Chunk{static_cast<char*>(base), bytes, 0, false});
  cur_ = 0;
  fixed_ = true;
}
void Arena::reset() {
  for (auto& c : chunks_) c.used = 0;
  cur_ = 0;
}
Arena::Mark Arena::mark() const {
  Mark m;
  m.chunk = cur_;
  m.used = cur_ < chunks_.size() ? chunks_[cur_].used : 0;
  return m;
}
void Arena::rewind(const Mark& m) {
  for (size_t q = m.chunk + 1; q < chunks_.size(); ++q) chunks_[q].used = 0;
  if (m.chunk < chunks_.size()) chunks_[m.chunk].used = m.used;
  cur_ = m.chunk;
}
size_t Arena::capacity() const {
  size_t t = 0;
  for (const auto& c : chunks_) t += c.size;
  return t;
}
size_t Arena::in_use() const {
  size_t t = 0;
  for (const auto& c : chunks_) t += c.used;
  return t;
}
void Arena::release() {
  for (auto& c : chunks_)
    if (c.owned) (void)hipFree(c.base);
  chunks_.clear();
  cur_ = 0;
  fixed_ = false;
  high_ = 0;
}

hipEvent_t ctx_event(Ctx& ctx, int i) {
  auto& pool = *ctx.events;
  while ((int)pool.size() <= i) {
    hipEvent_t e = nullptr;
    LSQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    pool.push_back(e);
  }
  return pool[i];
}

void ktimer_begin_on(Ctx& ctx, int kind, hipStream_t s, double flops, double bytes) {
  KernelTimer* t = ctx.timer;
  if (!t || t->target != kind) return;
  if ((size_t)(2 * t->used + 2) > t->ev.size()) {
    for (int q = 0; q < 2; ++q) {
      hipEvent_t e = nullptr;
      LSQ_HIP(hipEventCreate(&e));
      t->ev.push_back(e);
    }
  }
  LSQ_HIP(hipEventRecord(t->ev[2 * t->used], s));
  t->flops += flops;
  t->bytes += bytes;
}
void ktimer_end_on(Ctx& ctx, int kind, hipStream_t s) {
  KernelTimer* t = ctx.timer;
  if (!t || t->target != kind) return;
  LSQ_HIP(hipEventRecord(t->ev[2 * t->used + 1], s));
  ++t->used;
}
void ktimer_begin(Ctx& ctx, int kind, double flops, double bytes) {
  ktimer_begin_on(ctx, kind, ctx.stream, flops, bytes);
}
void ktimer_end(Ctx& ctx, int kind) { ktimer_end_on(ctx, kind, ctx.stream); }
void ktimer_add(Ctx& ctx, int kind, double flops, double bytes) {
  KernelTimer* t = ctx.timer;
  if (!t || t->target != kind) return;
  t->flops += flops;
  t->bytes += bytes;
}
}  // namespace lsq

// Workspace of the allocation-free factored solve: one array per GPU (each
// device that loads the library holds its own copy until the process ends).
// Host code never passes the array's name to a kernel; it uses the device
// address looked up once per device by scratch_setup().
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// With `device` current: looks up the device address of that device's
// scratch array (once per device) and keeps it.
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) throw std::runtime_error("device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  LSQ_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw std::runtime_error("no device address for the scratch array");
  g_scratch_ptr[device] = ptr;
}
void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}
}  // namespace

// Everything one solve in flight needs: a stream, a workspace arena, the
// device stop-test status with its pinned host mirror, and events.  The
// handle owns one worker on the caller's stream; batched calls add workers
// with streams of their own, one host thread each.
struct Worker {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Arena arena;
  Ctx ctx;
  StopStatus* st_dev = nullptr;
  StopStatus* st_host = nullptr;   // pinned
  double* matnorms = nullptr;
  double* pin = nullptr;           // pinned host scratch (kPinDoubles)
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipStream_t side = nullptr;      // look-ahead stream (default priority)
  std::vector<hipEvent_t> events;
  std::string last_error;
  // factor applied to the Frobenius norms of the two matrices after the
  // ingest scan: 1, or 1/sqrt(2) while a complex problem runs through its
  // real embedding (whose Frobenius norms are sqrt(2) times the complex ones)
  double norm_scale = 1.0;
  // a higher rung of the escalation ladder follows the one running (set by
  // the ladder; false for solves on stored factors): a GMRES-IR rung may then
  // give up on an inner solve that cannot converge within its budget
  bool more_rungs = false;
  // classical refinement replays each step (correction, residual, stop
  // status) as one captured HIP graph; off only for inspection
  bool step_graphs = true;
  // per refinement step of the last solve on this worker: the three block
  // backward errors, and the rung (precision, solver) and inner iterations
  struct Step { double berr[3]; int prec, solver, inner; };
  std::vector<Step> history;

  void init(int dev, int num_cu, bool new_stream) {
    device = dev;
    if (new_stream) {
      LSQ_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
      own_stream = true;
    }
    LSQ_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    ctx.ws = &arena;
    ctx.stream = stream;
    ctx.side = side;
    ctx.events = &events;
    ctx.num_cu = num_cu;
    LSQ_HIP(hipMalloc(&st_dev, sizeof(StopStatus)));
    LSQ_HIP(hipHostMalloc(&st_host, sizeof(StopStatus), 0));
    LSQ_HIP(hipHostMalloc(&pin, sizeof(double) * kPinDoubles, 0));
    ctx.pin = pin;
    LSQ_HIP(hipMalloc(&matnorms, 8 * sizeof(double)));
    for (auto& e : ev) LSQ_HIP(hipEventCreate(&e));
  }
  void release() {
    if (stream) (void)hipStreamSynchronize(stream);
    arena.release();
    if (st_dev) (void)hipFree(st_dev);
    if (st_host) (void)hipHostFree(st_host);
    if (pin) (void)hipHostFree(pin);
    if (matnorms) (void)hipFree(matnorms);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : events)
      if (e) (void)hipEventDestroy(e);
    events.clear();
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
      side = nullptr;
    }
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    st_dev = nullptr; st_host = nullptr; pin = nullptr; matnorms = nullptr; stream = nullptr;
  }
};

// Diagonal ratio of an FP32 triangle in the persistent batch above which an
// instance goes to the FP64 rung without refining (see batch.hip).  The
// ratio bounds the triangle's condition number from below; on matrices
// U diag(s) V^T it runs 10 to 30 times below kappa, and FP32 classical
// refinement stops contracting fast enough near kappa = 1e6 to 1e7.  Chosen by
// a sweep of the threshold over the 2000-instance batch (1e4 .. 1e7).
constexpr double kBatchRoute = 3e5;

constexpr double kMaxBatchPre = 8.0;            // bound on the FP64-first instances per FP64 work-group

struct lsq_handle_st {
  int device = 0;
  int num_cu = 256;
  Worker w;                                     // the handle's own (caller's) stream
  std::vector<std::unique_ptr<Worker>> pool;    // batched workers
  int batch_workers = 8;
  int batch_mode = LSQ_BATCH_AUTO;
  double esc_wait_ms = 50.0;                    // bound on an FP64 consumer's wait (concurrent batch)
  double batch_route = kBatchRoute;             // diagonal-ratio route of the persistent FP32 rung
  double batch_fp64_share = 0.25;               // compute units the concurrent FP64 rung starts on
  double batch_pre = 0.0;                       // longest instances sent to FP64 at once, per FP64 work-group
  // tuned (route, FP64 share, pre) per size bucket and escalation regime: of
  // the entries whose bound is >= the batch's largest dimension and whose
  // esc_max is >= the escalation fraction the last FP32-first persistent
  // batch showed, the one with the smallest bound, then the smallest esc_max,
  // applies; none: the values above
  struct BatchTune { int max_dim; double route, share, pre, esc_max; };
  double last_escalation = 1.0;                 // nothing seen yet: the regime with the most escalations
  std::vector<BatchTune> batch_tuning;
  float* sel_w = nullptr;                       // selector weights on the device (null: none)
  KernelTimer timer;
  std::string last_error;
  bool dbg_dd = false;                          // residual inspection in double-double
  double wclk_khz = 100000.0;                   // device wall clock rate (wall_clock64)
  // last persistent batched call, per instance of its problem array: the
  // FP32 attempt's and the FP64 attempt's (start, factored, end) in ms from
  // the earliest start (NaN where an attempt did not run)
  std::vector<double> timeline;
};

namespace {

struct PrecSpec {
  int tw;      // storage bytes of the factor
  Mma mt;      // MFMA input type
  int tc;      // compute bytes of classical-IR corrections
};

bool prec_spec(int prec, PrecSpec& ps) {
  switch (prec) {
    case LSQ_PREC_FP64: ps = {8, Mma::F64, 8}; return true;
    case LSQ_PREC_FP32: ps = {4, Mma::F32, 4}; return true;
    case LSQ_PREC_BF16: ps = {4, Mma::BF16, 4}; return true;
    case LSQ_PREC_FP16: ps = {4, Mma::F16, 4}; return true;
    case LSQ_PREC_FP8E4M3: ps = {4, Mma::F8, 4}; return true;
    default: return false;
  }
}

// Panels per aggregated block for the vector application of Q and Z.  Wider
// blocks mean fewer launches per application but larger T inverses to
// prepare: classical IR applies Q and Z a few times per solve, GMRES-IR once
// per inner iteration.
constexpr int kAggPanels = 8;
constexpr int kAggPanelsGmres = 16;

int default_nb(const lsq_opts& o) { return (o.nb > 0 && o.nb <= kMaxNb) ? o.nb : kMaxNb; }

void* off(void* p, size_t bytes) { return static_cast<char*>(p) + bytes; }
const void* off(const void* p, size_t bytes) { return static_cast<const char*>(p) + bytes; }

struct LseArgs {
  int m, n, p;
  const double *A, *B, *b, *d;
  int lda, ldb;
};
struct GlsArgs {
  int n, m, p;
  const double *W, *V, *d;
  int ldw, ldv;
};

// One timing-free event owned by a solver (created on first use).
struct SolverEvent {
  hipEvent_t e = nullptr;
  SolverEvent() = default;
  SolverEvent(const SolverEvent&) = delete;
  SolverEvent& operator=(const SolverEvent&) = delete;
  ~SolverEvent() {
    if (e) (void)hipEventDestroy(e);
  }
  hipEvent_t get() {
    if (!e) LSQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return e;
  }
};

// ----------------------------------------------------------------- LSE ----
struct LseSolver {
  int m, n, p, k;
  int prec_id = 0;        // lsq_prec of the factors
  float ms_factor = 0.0f;
  // Factors kept across calls (lse_factor): prepare() goes to this context's
  // arena once per compute precision instead of once per call.
  Ctx* pctx = nullptr;
  int prepared_tc = 0;
  bool prepared_gmres = false;
  Arena::Mark pmark;      // pctx's arena right after the factorization
  bool has_pmark = false;
  // The B-side structures (R's inverse, B's aggregated blocks) depend on fb
  // only: factor() prepares them on the side stream while the main stream
  // works on Abar; b_tc is the precision they are prepared for.
  SolverEvent ev_b;
  bool b_pending = false;
  int b_tc = 0, b_panels = 0;
  PrecSpec ps;
  int tc;                 // compute precision of the correction solve
  QRFactor fb, fa;        // QR of Bt (n x p) and of Abar (m x n)
  TriBlock tR, tT11;
  void *U, *Wv, *Y2, *Y2n, *Qv, *Y1, *S, *X2, *Yt;

  void alloc_vectors(Ctx& ctx) {
    auto v = [&](int len) { return ctx.ws->alloc((size_t)tc * (len > 0 ? len : 1)); };
    U = v(n); Wv = v(m); Y2 = v(p); Y2n = v(p); Qv = v(m); Y1 = v(k); S = v(p); X2 = v(p); Yt = v(n);
  }

  void prepare_b(Ctx& ctx, int tc_, int panels) {
    trsv_prepare(ctx, tR, fb, 0, p, tc_);
    agg_prepare(ctx, fb, tc_, panels);
    b_tc = tc_;
    b_panels = panels;
  }

  // Power-of-two scales of A and B for the factorization (1 unless set
  // before factor()).
  double sA = 1.0, sB = 1.0;

  // early_tc > 0: prepare the B-side structures for that precision on the
  // side stream, overlapping the rest of the factorization.  The factors and
  // prepared structures go to ctx.ws; the factorization's temporaries to
  // scratch (ctx.ws when null).  A and B are factored scaled by sA and sB; the
  // triangular factors R and T are scaled back afterwards (exact: powers of two).
  void factor(Ctx& ctx, const double* A, int lda, const double* B, int ldb, int nb, int early_tc = 0,
              Arena* scratch = nullptr) {
    Ctx tctx = ctx;
    if (scratch) tctx.ws = scratch;
    qr_alloc(ctx, fb, n, p, ps.tw, ps.mt, nb);
    mat_convert(ctx, fb.M, ps.tw, fb.ld, B, 8, ldb, n, p, true, true, true, sB);
    qr_factor(tctx, fb);
    scale_upper(ctx, fb, 1.0 / sB);
    if (early_tc > 0 && ctx.side) {
      hipEvent_t e = ev_b.get();
      LSQ_HIP(hipEventRecord(e, ctx.stream));
      LSQ_HIP(hipStreamWaitEvent(ctx.side, e, 0));
      Ctx sctx = ctx;
      sctx.stream = ctx.side;
      prepare_b(sctx, early_tc, kAggPanels);
      LSQ_HIP(hipEventRecord(e, ctx.side));
      b_pending = true;
    }
    void* X0 = tctx.ws->alloc((size_t)ps.tw * (size_t)(n > 0 ? n : 1) * (m > 0 ? m : 1));
    mat_convert(ctx, X0, ps.tw, n > 0 ? n : 1, A, 8, lda, n, m, true, false, true, sA);
    qr_apply_left_T(tctx, fb, X0, n > 0 ? n : 1, m);
    qr_alloc(ctx, fa, m, n, ps.tw, ps.mt, nb);
    mat_convert(ctx, fa.M, ps.tw, fa.ld, X0, ps.tw, n > 0 ? n : 1, m, n, true, true, false);
    qr_factor(tctx, fa);
    scale_upper(ctx, fa, 1.0 / sA);
  }

  void prepare(Ctx& ctx, int tc_, int panels = kAggPanels) {
    tc = tc_;
    if (b_pending) {
      LSQ_HIP(hipStreamWaitEvent(ctx.stream, ev_b.get(), 0));
      b_pending = false;
    }
    if (b_tc != tc || b_panels != panels) prepare_b(ctx, tc, panels);
    trsv_prepare(ctx, tT11, fa, 0, k, tc);
    agg_prepare(ctx, fa, tc, panels);
    alloc_vectors(ctx);
  }

  // Algorithm 1 on (f1, f2, f3) (f3 may be null = 0); adds (dr, dv, dx) to (r, v, x).
  // The vector steps between the solves run as six multi-segment launches
  // (segs.hpp), each segment the same once-rounded expression as the
  // conversion or axpy it stands for.
  void correct(Ctx& ctx, const double* f1, const double* f2, const double* f3, double* x,
               double* r, double* v) {
    const size_t e = (size_t)tc;
    // u~ = J f3 (or 0), w = f1, y2 = J f2 in tc; S = 0
    vec_segs_t(ctx, {f3 ? tcopy(U, tc, f3, 8, n, true) : tzero(U, tc, n), tcopy(Wv, tc, f1, 8, m),
                     tcopy(Y2, tc, f2, 8, p, true), tzero(S, tc, p)});
    agg_apply(ctx, fb, true, U, tc);                    // u~ = Qt^T (J f3)
    agg_apply(ctx, fa, true, Wv, tc);                   // w = Z^T f1
    trsv(ctx, tR, true, Y2);                            // R y2 = f2  <=>  Rt^T (J y2) = J f2
    // J y2; u1 = J u~[p:n]
    vec_segs_t(ctx, {tcopy(Y2n, tc, Y2, tc, p, true), tcopy(Qv, tc, off(U, e * p), tc, k, true)});
    trsv(ctx, tT11, true, Qv);                          // T11^T q1 = u1
    // w1 - q1; w2 (the start of q2)
    vec_segs_t(ctx, {tadd(Y1, tc, Wv, tc, false, Qv, tc, false, k, -1.0),
                     tcopy(off(Qv, e * k), tc, off(Wv, e * k), tc, m - k)});
    gemv_upper(ctx, fa, 0, k, k, p, false, -1.0, Y2n, Y1, tc);
    trsv(ctx, tT11, false, Y1);                         // T11 y1 = w1 - q1 - T12 y2
    gemv_upper(ctx, fa, k, k, m - k, p, false, -1.0, Y2n, off(Qv, e * k), tc);   // q2 = w2 - T22 y2
    // R^T dv = T12^T q1 + T22^T q2 - u2  <=>  Rt (J dv) = J(...)
    gemv_upper(ctx, fa, 0, k, m, p, true, 1.0, Qv, S, tc);
    vec_segs_t(ctx, {tadd(X2, tc, S, tc, true, U, tc, false, p, -1.0)});
    trsv(ctx, tR, false, X2);
    // v += J dv~; J y = [y2~; J y1]
    vec_segs_t(ctx, {taxpy(v, 8, 1.0, X2, tc, p, true), tcopy(Yt, tc, Y2, tc, p),
                     tcopy(off(Yt, e * p), tc, Y1, tc, k, true)});
    agg_apply(ctx, fa, false, Qv, tc);                  // dr = Z q
    agg_apply(ctx, fb, false, Yt, tc);                  // dx = J Qt (J y)
    vec_segs_t(ctx, {taxpy(r, 8, 1.0, Qv, tc, m), taxpy(x, 8, 1.0, Yt, tc, n, true)});
  }

  // ---- GMRES-IR: block-diagonal split preconditioners of Section 5.2, FP64
  // arithmetic on the stored factors.  With u = [a; b; c] (lengths m, p, n)
  // and sa = sqrt(alpha):
  //   M_l u = [a / sa; Y R^{-1} b / (sa beta); sa U^{-T} Q c]
  //   M_r u = [a / sa; R^{-T} Y^T b / (sa beta); sa Q^T U^{-1} c]
  //   F u   = [alpha a + A c; beta B c; A^T a + beta B^T b].
  // U is n x n: T1 for m >= n (eq. lse-bdpre-mlarge); [T1 T2; 0 I] for n > m
  // (eq. lse-bdpre-nlarge), where [T1 T2] is the m x n trapezoid of the QR
  // of Abar.  Y is the trailing p x p block of U in both cases: the rows
  // k .. t-1 (t = min(m, n), k = n - p) of the trapezoid followed by n - t
  // identity rows.
  TriBlock tT1;
  double alpha = 1.0, beta = 1.0, sa = 1.0;
  double *g1 = nullptr, *g2 = nullptr, *g3 = nullptr, *g4 = nullptr, *t1 = nullptr, *t2 = nullptr;
  DualParts dpa, dpb;

  int tmn() const { return std::min(m, n); }
  void prepare_gmres(Ctx& ctx) {
    prepare(ctx, 8, kAggPanelsGmres);
    trsv_prepare(ctx, tT1, fa, 0, tmn(), 8);
    const int L = std::max(std::max(m, n), 1), N = std::max(m + p + n, 1);
    g1 = ctx.ws->get<double>(L); g2 = ctx.ws->get<double>(L); g3 = ctx.ws->get<double>(L);
    g4 = ctx.ws->get<double>(L);
    t1 = ctx.ws->get<double>(N); t2 = ctx.ws->get<double>(N);
    dual_parts_alloc(ctx, m, n, dpa);
    dual_parts_alloc(ctx, p, n, dpb);
  }
  // x (p) <- R^{-1} x or R^{-T} x, with R = J Rt^T J
  void r_solve(Ctx& ctx, double* xv, bool trans) {
    vec_convert(ctx, g3, 8, xv, 8, p, true);
    trsv(ctx, tR, !trans, g3);
    vec_convert(ctx, xv, 8, g3, 8, p, true);
  }
  // x (n) <- Q x or Q^T x, with Q = J Qt^T J
  void q_apply(Ctx& ctx, double* xv, bool trans) {
    vec_convert(ctx, g3, 8, xv, 8, n, true);
    agg_apply(ctx, fb, !trans, g3, 8);
    vec_convert(ctx, xv, 8, g3, 8, n, true);
  }
  // x (n) <- U^{-1} x: x2 stays, T1 x1 = x1 - T2 x2
  void u_solve(Ctx& ctx, double* xv) {
    const int t = tmn();
    if (n > t) gemv_upper(ctx, fa, 0, t, t, n - t, false, -1.0, xv + t, xv, 8);
    trsv(ctx, tT1, false, xv);
  }
  // x (n) <- U^{-T} x: T1^T x1 = x1, x2 -= T2^T x1
  void u_solve_t(Ctx& ctx, double* xv) {
    const int t = tmn();
    trsv(ctx, tT1, true, xv);
    if (n > t) gemv_upper(ctx, fa, 0, t, t, n - t, true, -1.0, xv, xv + t, 8);
  }
  // y (p) += s op(Y) x
  void y_apply(Ctx& ctx, bool trans, double s, const double* xv, double* yv) {
    const int t = tmn(), rows = t - k;
    gemv_upper(ctx, fa, k, k, rows, p, trans, s, xv, yv, 8);
    if (p > rows) vec_axpy(ctx, yv + rows, 8, s, xv + rows, 8, p - rows, false);
  }
  // The two preconditioner applications with their vector glue merged into
  // three segment launches each (the same arithmetic as r_solve, q_apply and
  // y_apply with their reversal, scaling and addition steps one by one).
  void m_right(Ctx& ctx, const double* u, double* out) {
    const int t = tmn(), rows = t - k;
    vec_segs(ctx, {seg_copy(out, u, m, false, 1.0 / sa), seg_zero(g1, p), seg_copy(g2, u + m + p, n)});
    gemv_upper(ctx, fa, k, k, rows, p, true, 1.0, u + m, g1, 8);                 // Y^T b
    u_solve(ctx, g2);
    vec_segs(ctx, {seg_add(g3, g1, u + m, p, true, rows), seg_copy(g4, g2, n, true)});
    trsv(ctx, tR, false, g3);                                                      // R^{-T}
    agg_apply(ctx, fb, false, g4, 8);                                              // Q^T
    vec_segs(ctx, {seg_copy(out + m, g3, p, true, 1.0 / (sa * beta)), seg_copy(out + m + p, g4, n, true, sa)});
  }
  void m_left(Ctx& ctx, const double* u, double* out) {
    const int t = tmn(), rows = t - k;
    const double s = 1.0 / (sa * beta);
    vec_segs(ctx, {seg_copy(out, u, m, false, 1.0 / sa), seg_copy(g3, u + m, p, true),
                   seg_copy(g4, u + m + p, n, true), seg_zero(out + m, p)});
    trsv(ctx, tR, true, g3);                                                       // R^{-1}
    agg_apply(ctx, fb, true, g4, 8);                                               // Q
    vec_segs(ctx, {seg_copy(g1, g3, p, true), seg_copy(g2, g4, n, true)});
    gemv_upper(ctx, fa, k, k, rows, p, false, s, g1, out + m, 8);                 // Y R^{-1} b
    u_solve_t(ctx, g2);
    vec_segs(ctx, {seg_add(out + m + rows, out + m + rows, g1 + rows, p - rows, false, 0, s),
                   seg_copy(out + m + p, g2, n, false, sa)});
  }
  void f_apply(Ctx& ctx, const LseArgs& a, const double* u, double* out);
};

// ----------------------------------------------------------------- GLS ----
struct GlsSolver {
  int n, m, p, k;         // k = n - m
  int prec_id = 0;        // lsq_prec of the factors
  float ms_factor = 0.0f;
  Ctx* pctx = nullptr;    // as for LseSolver
  int prepared_tc = 0;
  bool prepared_gmres = false;
  Arena::Mark pmark;
  bool has_pmark = false;
  SolverEvent ev_w;       // W-side structures prepared early (as LseSolver's B side)
  bool w_pending = false;
  int w_tc = 0, w_panels = 0;
  PrecSpec ps;
  int tc;
  QRFactor fw, fv;        // QR of W (n x m) and of Vt (p x n)
  TriBlock tR, tA11;
  void *U, *Wt, *H1, *H1t, *G, *H2t, *S, *X, *Hv;

  void alloc_vectors(Ctx& ctx) {
    auto v = [&](int len) { return ctx.ws->alloc((size_t)tc * (len > 0 ? len : 1)); };
    U = v(n); Wt = v(p); H1 = v(m); H1t = v(m); G = v(p); H2t = v(k); S = v(m); X = v(m); Hv = v(n);
  }

  void prepare_w(Ctx& ctx, int tc_, int panels) {
    trsv_prepare(ctx, tR, fw, 0, m, tc_);
    agg_prepare(ctx, fw, tc_, panels);
    w_tc = tc_;
    w_panels = panels;
  }

  double sW = 1.0, sV = 1.0;   // power-of-two scales of W and V (as LseSolver's sA, sB)

  void factor(Ctx& ctx, const double* W, int ldw, const double* V, int ldv, int nb, int early_tc = 0,
              Arena* scratch = nullptr) {
    Ctx tctx = ctx;
    if (scratch) tctx.ws = scratch;
    qr_alloc(ctx, fw, n, m, ps.tw, ps.mt, nb);
    mat_convert(ctx, fw.M, ps.tw, fw.ld, W, 8, ldw, n, m, false, false, false, sW);
    qr_factor(tctx, fw);
    scale_upper(ctx, fw, 1.0 / sW);
    if (early_tc > 0 && ctx.side) {
      hipEvent_t e = ev_w.get();
      LSQ_HIP(hipEventRecord(e, ctx.stream));
      LSQ_HIP(hipStreamWaitEvent(ctx.side, e, 0));
      Ctx sctx = ctx;
      sctx.stream = ctx.side;
      prepare_w(sctx, early_tc, kAggPanels);
      LSQ_HIP(hipEventRecord(e, ctx.side));
      w_pending = true;
    }
    const int ldn = n > 0 ? n : 1;
    void* Vw = tctx.ws->alloc((size_t)ps.tw * ldn * (p > 0 ? p : 1));
    mat_convert(ctx, Vw, ps.tw, ldn, V, 8, ldv, n, p, false, false, false, sV);
    qr_apply_left_T(tctx, fw, Vw, ldn, p);
    qr_alloc(ctx, fv, p, n, ps.tw, ps.mt, nb);
    mat_convert(ctx, fv.M, ps.tw, fv.ld, Vw, ps.tw, ldn, p, n, true, true, true);
    qr_factor(tctx, fv);
    scale_upper(ctx, fv, 1.0 / sV);
  }

  void prepare(Ctx& ctx, int tc_, int panels = kAggPanels) {
    tc = tc_;
    if (w_pending) {
      LSQ_HIP(hipStreamWaitEvent(ctx.stream, ev_w.get(), 0));
      w_pending = false;
    }
    if (w_tc != tc || w_panels != panels) prepare_w(ctx, tc, panels);
    trsv_prepare(ctx, tA11, fv, 0, k, tc);
    agg_prepare(ctx, fv, tc, panels);
    alloc_vectors(ctx);
  }

  // Algorithm 3 on (f1, f2, f3) (f1, f3 may be null = 0); adds (dy, dz, dx) to (y, z, x).
  // The vector steps between the solves run as six multi-segment launches,
  // as in LseSolver::correct.
  void correct(Ctx& ctx, const double* f1, const double* f2, const double* f3, double* x,
               double* y, double* z) {
    const size_t e = (size_t)tc;
    // f2, J f1 (or 0), f3 (or 0) in tc; S = 0
    vec_segs_t(ctx, {tcopy(U, tc, f2, 8, n), f1 ? tcopy(Wt, tc, f1, 8, p, true) : tzero(Wt, tc, p),
                     f3 ? tcopy(H1, tc, f3, 8, m) : tzero(H1, tc, m), tzero(S, tc, m)});
    agg_apply(ctx, fw, true, U, tc);                    // u = Q^T f2
    agg_apply(ctx, fv, true, Wt, tc);                   // J w = Zt^T (J f1)
    trsv(ctx, tR, true, H1);                            // R^T h1 = f3
    // J h1; J u2
    vec_segs_t(ctx, {tcopy(H1t, tc, H1, tc, m, true), tcopy(G, tc, off(U, e * m), tc, k, true)});
    trsv(ctx, tA11, true, G);                           // T22 g2 = u2  <=>  A11^T (J g2) = J u2
    // J w2 - J g2; J w1 (the start of J g1)
    vec_segs_t(ctx, {tadd(H2t, tc, Wt, tc, false, G, tc, false, k, -1.0),
                     tcopy(off(G, e * k), tc, off(Wt, e * k), tc, p - k)});
    // T22^T h2 = w2 - g2 - T12^T h1  <=>  A11 (J h2) = J w2 - J g2 - A12 J h1
    gemv_upper(ctx, fv, 0, k, k, m, false, -1.0, H1t, H2t, tc);
    trsv(ctx, tA11, false, H2t);
    // g1 = w1 - T11^T h1  <=>  J g1 = J w1 - A22 J h1
    gemv_upper(ctx, fv, k, k, p - k, m, false, -1.0, H1t, off(G, e * k), tc);
    // R dx = u1 - T11 g1 - T12 g2 = u1 - J (Rv[:, k:n]^T (J g))
    gemv_upper(ctx, fv, 0, k, p, m, true, 1.0, G, S, tc);
    vec_segs_t(ctx, {tadd(X, tc, U, tc, false, S, tc, true, m, -1.0)});
    trsv(ctx, tR, false, X);
    // x += dx; h = [h1; J h2~]
    vec_segs_t(ctx, {taxpy(x, 8, 1.0, X, tc, m), tcopy(Hv, tc, H1, tc, m),
                     tcopy(off(Hv, e * m), tc, H2t, tc, k, true)});
    agg_apply(ctx, fw, false, Hv, tc);                  // dz = -Q h
    agg_apply(ctx, fv, false, G, tc);                   // dy = Z^T g = J Zt (J g)
    vec_segs_t(ctx, {taxpy(z, 8, -1.0, Hv, tc, n), taxpy(y, 8, 1.0, G, tc, p, true)});
  }

  // ---- GMRES-IR: block-diagonal split preconditioners of Section 5.3, FP64
  // arithmetic on the stored factors.  With u = [a; b; c] (lengths p, n, m)
  // and sa = sqrt(alpha):
  //   M_l u = [a / sa; sa U^{-1} Q^T b; Y^T R^{-T} c / (sa beta)]
  //   M_r u = [a / sa; sa Q U^{-T} b; R^{-1} Y c / (sa beta)]
  //   F u   = [alpha a + V^T b; V a + beta W c; beta W^T b].
  // U is n x n: T2 for n <= p (eq. gls-bdpre-plarge, T = [0, T2]); [I T1; 0 T2]
  // for n > p (eq. gls-bdpre-nlarge, T = [T1; T2]).  Y is the leading m x m
  // block of U in both cases.  The QR of Vt stores Rv (t x n, t = min(n, p))
  // with T = J Rv^T J, so U = J Ut^T J for Ut = [Rv; 0 I_(n-t)], and
  // Y = J Ut[k:n, k:n]^T J (k = n - m).
  TriBlock tRv;
  double alpha = 1.0, beta = 1.0, sa = 1.0;
  double *g1 = nullptr, *g2 = nullptr, *g3 = nullptr, *g4 = nullptr, *g5 = nullptr, *g6 = nullptr;
  double *t1 = nullptr, *t2 = nullptr;
  DualParts dpv, dpw;

  int tnp() const { return std::min(n, p); }
  void prepare_gmres(Ctx& ctx) {
    prepare(ctx, 8, kAggPanelsGmres);
    trsv_prepare(ctx, tRv, fv, 0, tnp(), 8);
    const int L = std::max(std::max(n, p), 1), N = std::max(p + n + m, 1);
    g1 = ctx.ws->get<double>(L); g2 = ctx.ws->get<double>(L); g3 = ctx.ws->get<double>(L);
    g4 = ctx.ws->get<double>(L); g5 = ctx.ws->get<double>(L); g6 = ctx.ws->get<double>(L);
    t1 = ctx.ws->get<double>(N); t2 = ctx.ws->get<double>(N);
    dual_parts_alloc(ctx, n, p, dpv);
    dual_parts_alloc(ctx, n, m, dpw);
  }
  // x (n) <- U^{-1} x or U^{-T} x: U^{-1} = J Ut^{-T} J, U^{-T} = J Ut^{-1} J
  void u_solve(Ctx& ctx, double* xv, bool trans) {
    const int t = tnp();
    vec_convert(ctx, g3, 8, xv, 8, n, true);
    if (!trans) {                          // Ut^T y = g: Rv1^T y1 = g1, y2 = g2 - Rv2^T y1
      trsv(ctx, tRv, true, g3);
      if (n > t) gemv_upper(ctx, fv, 0, t, t, n - t, true, -1.0, g3, g3 + t, 8);
    } else {                               // Ut y = g: y2 = g2, Rv1 y1 = g1 - Rv2 y2
      if (n > t) gemv_upper(ctx, fv, 0, t, t, n - t, false, -1.0, g3 + t, g3, 8);
      trsv(ctx, tRv, false, g3);
    }
    vec_convert(ctx, xv, 8, g3, 8, n, true);
  }
  // out (m) = Y x or Y^T x, Y = J Ub^T J with Ub = Ut[k:n, k:n]: its first
  // t - k rows come from Rv, the rest are identity rows
  void y_apply(Ctx& ctx, const double* xv, double* out, bool trans) {
    const int rows = tnp() - k;
    vec_convert(ctx, g3, 8, xv, 8, m, true);
    vec_zero(ctx, g4, 8, m);
    gemv_upper(ctx, fv, k, k, rows, m, !trans, 1.0, g3, g4, 8);
    if (m > rows) vec_axpy(ctx, g4 + rows, 8, 1.0, g3 + rows, 8, m - rows, false);
    vec_convert(ctx, out, 8, g4, 8, m, true);
  }
  // The two preconditioner applications with their vector glue merged into
  // three segment launches each (the same arithmetic as u_solve / y_apply
  // with their reversal and scaling steps one by one; the segments' factors
  // of 1 are exact).  Buffers: g3 the U solve, g5 / g4 the Y product's
  // input / output, g1 / g2 / g6 the Q and R solves.
  void m_right(Ctx& ctx, const double* u, double* out) {
    const int t = tnp(), rows = t - k;
    vec_segs(ctx, {seg_copy(out, u, p, false, 1.0 / sa), seg_copy(g3, u + p, n, true),
                   seg_copy(g5, u + p + n, m, true), seg_zero(g4, m)});
    if (n > t) gemv_upper(ctx, fv, 0, t, t, n - t, false, -1.0, g3 + t, g3, 8);   // Ut y = J b
    trsv(ctx, tRv, false, g3);
    gemv_upper(ctx, fv, k, k, rows, m, true, 1.0, g5, g4, 8);                    // Y c
    vec_segs(ctx, {seg_copy(g1, g3, n, true), seg_add(g2, g4, g5, m, true, rows)});
    agg_apply(ctx, fw, false, g1, 8);
    trsv(ctx, tR, false, g2);
    vec_segs(ctx, {seg_copy(out + p, g1, n, false, sa), seg_copy(out + p + n, g2, m, false, 1.0 / (sa * beta))});
  }
  void m_left(Ctx& ctx, const double* u, double* out) {
    const int t = tnp(), rows = t - k;
    vec_segs(ctx, {seg_copy(out, u, p, false, 1.0 / sa), seg_copy(g1, u + p, n), seg_copy(g6, u + p + n, m),
                   seg_zero(g4, m)});
    agg_apply(ctx, fw, true, g1, 8);
    trsv(ctx, tR, true, g6);
    vec_segs(ctx, {seg_copy(g3, g1, n, true), seg_copy(g5, g6, m, true)});
    trsv(ctx, tRv, true, g3);                                                      // Ut^T y = J Q^T b
    if (n > t) gemv_upper(ctx, fv, 0, t, t, n - t, true, -1.0, g3, g3 + t, 8);
    gemv_upper(ctx, fv, k, k, rows, m, false, 1.0, g5, g4, 8);                   // Y^T R^{-T} c
    vec_segs(ctx, {seg_copy(out + p, g3, n, true, sa), seg_add(out + p + n, g4, g5, m, true, rows, 1.0,
                                                               1.0 / (sa * beta))});
  }
  void f_apply(Ctx& ctx, const GlsArgs& a, const double* u, double* out);
};

void LseSolver::f_apply(Ctx& ctx, const LseArgs& a, const double* u, double* out) {
  dual_gemv(ctx, a.A, a.lda, m, n, u + m + p, u, dpa);         // A c, A^T a
  dual_gemv(ctx, a.B, a.ldb, p, n, u + m + p, u + m, dpb);     // B c, B^T b
  combine3(ctx, CombineArgs{out, m, alpha, u, 1.0, dpa.rowp, dpa.ncb, 0.0, nullptr, 0},
           CombineArgs{out + m, p, 0.0, nullptr, beta, dpb.rowp, dpb.ncb, 0.0, nullptr, 0},
           CombineArgs{out + m + p, n, 0.0, nullptr, 1.0, dpa.colp, dpa.nrb, beta, dpb.colp, dpb.nrb});
}

void GlsSolver::f_apply(Ctx& ctx, const GlsArgs& a, const double* u, double* out) {
  dual_gemv(ctx, a.V, a.ldv, n, p, u, u + p, dpv);             // V a, V^T b
  dual_gemv(ctx, a.W, a.ldw, n, m, u + p + n, u + p, dpw);     // W c, W^T b
  combine3(ctx, CombineArgs{out, p, alpha, u, 1.0, dpv.colp, dpv.nrb, 0.0, nullptr, 0},
           CombineArgs{out + p, n, 0.0, nullptr, 1.0, dpv.rowp, dpv.ncb, beta, dpw.rowp, dpw.ncb},
           CombineArgs{out + p + n, m, 0.0, nullptr, beta, dpw.colp, dpw.nrb, 0.0, nullptr, 0});
}

// ------------------------------------------------------- rung execution --
struct RungOut {
  bool ok = false;
  // the factorization failed at this precision: 1 in the first factorization
  // (R from B, LSE; R from W, GLS), 2 in the second (T), 0 none
  int breakdown = 0;
  // FP64 rung that did not certify: 1 or 2 when the triangle R (resp. T11 /
  // T22) is numerically singular, 0 otherwise
  int singular = 0;
  int steps = 0, inner = 0;
  double berr[3] = {0, 0, 0}, berr_max = INFINITY;
  float ms_convert = 0, ms_factor = 0, ms_refine = 0;
};

// The best iterate seen by the rungs of one solve (smallest blockwise
// backward error), kept for a solve that ends without meeting tol; save()
// copies the current iterate to the caller's buffers.
struct BestIter {
  bool have = false;
  double berr[3] = {0, 0, 0}, berr_max = INFINITY;
  int steps = 0, inner = 0, prec = 0, solver = 0;
  std::function<void()> save;
  void observe(const StopStatus& st, int steps_, int inner_, int prec_, int solver_) {
    if (!save || st.converged || st.nonfinite || !(st.berr_max < berr_max)) return;
    save();
    have = true;
    for (int q = 0; q < 3; ++q) berr[q] = st.berr[q];
    berr_max = st.berr_max;
    steps = steps_;
    inner = inner_;
    prec = prec_;
    solver = solver_;
  }
};

// Pivot ratio min |t_ii| / max |t_ii| at or below which an FP64 triangle
// that did not certify is reported singular (a few units of roundoff).
constexpr double kSingularRatio = 16.0 * 1.1102230246251565e-16;

void read_status(Worker* h) {
  LSQ_HIP(hipMemcpyAsync(h->st_host, h->st_dev, sizeof(StopStatus), hipMemcpyDeviceToHost, h->stream));
  LSQ_HIP(hipStreamSynchronize(h->stream));
}

int read_int(Worker* h, const int* dptr) {
  int v = 0;
  LSQ_HIP(hipMemcpyAsync(&h->st_host->converged, dptr, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  LSQ_HIP(hipStreamSynchronize(h->stream));
  v = h->st_host->converged;
  return v;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

// Divergence / stagnation test of the refinement (the paper reports
// "diverged" without a rule): stop the rung when an iterate is not finite or
// the backward error has not halved over the last three steps.
bool stalled(const std::vector<double>& hist) {
  const size_t s = hist.size();
  if (s >= 4 && !(hist[s - 1] <= 0.5 * hist[s - 4])) return true;
  return false;
}

// After an iterate passed the stop test: whether to take one more
// correction first.  The stop test certifies berr <= tol; first-order
// perturbation theory bounds the forward error by about cond * berr, so an
// iterate certified at berr near tol = 1e-14 may sit well above the limiting
// accuracy.  With the FP64 residual one more correction (once, while berr >
// o.polish) reaches the limiting accuracy cond * u.  With the double-double
// residual the limiting accuracy no longer depends on cond, and refinement
// goes on while the corrections still change the solution blocks by more
// than 2u relative and keep at least halving (the classical stop rule on the
// size of the correction; the FP64 iterate itself bounds the accuracy at u).
void d2d(Worker* w, double* dst, const double* src, int n);

struct Continuation {
  const lsq_opts& o;
  bool dd = false;
  bool polished = false;
  double last_dx = INFINITY, prev_dx = INFINITY;   // ||dx||_inf / ||x||_inf of the last two corrections
  explicit Continuation(const lsq_opts& o_) : o(o_), dd(o_.residual == 1) {}
  void observe_dx(double r) { prev_dx = last_dx; last_dx = r; }
  bool more(const StopStatus& st, int it) {
    if (it >= o.maxit) return false;
    if (dd) return last_dx > 2.0 * 1.1102230246251565e-16 && (prev_dx == INFINITY || last_dx <= 0.5 * prev_dx);
    if (polished || !(o.polish > 0.0) || st.berr_max <= o.polish) return false;
    polished = true;
    return true;
  }
};

// One step of classical refinement (the correction, the FP64 residual and
// the copy of the stop status to the pinned host mirror) captured once as a
// HIP graph on the worker's side stream and replayed on its stream: the
// host then issues one launch per step instead of some sixty kernels.  The
// captured work must neither allocate nor synchronize; if capture fails the
// steps run kernel by kernel.
struct StepGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~StepGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
  bool capture(Worker* h, const std::function<void()>& body) {
    Ctx& ctx = h->ctx;
    if (!h->side) return false;
    KernelTimer* saved_timer = ctx.timer;          // no event records inside the graph
    hipStream_t saved = ctx.stream;
    ctx.timer = nullptr;
    ctx.stream = h->side;
    bool ok = hipStreamBeginCapture(h->side, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      try {
        body();
      } catch (const HipError&) {
        ok = false;
      }
      hipGraph_t g = nullptr;
      const bool ended = hipStreamEndCapture(h->side, &g) == hipSuccess;
      graph = g;
      ok = ok && ended && graph != nullptr;
    }
    ctx.timer = saved_timer;
    ctx.stream = saved;
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
    }
    return ok;
  }
};

// Classical refinement (Algorithms 2 and 4): init() adds the initial guess to
// the zeroed iterate, residual() evaluates the FP64 residual and the stop
// test on the device, correct() adds one correction.
RungOut run_classical(Worker* h, const std::function<void()>& zero,
                      const std::function<void()>& init, const std::function<void()>& residual,
                      const std::function<void()>& correct, const lsq_opts& o,
                      const std::function<void(const StopStatus&, int, int)>& observe,
                      Continuation& cont, bool capturable) {
  RungOut out;
  zero();
  LSQ_HIP(hipEventRecord(h->ev[2], h->stream));
  init();
  std::vector<double> hist;
  StepGraph sg;
  bool tried = false;
  for (int it = 0;; ++it) {
    if (it > 0 && sg.exec) {
      LSQ_HIP(hipGraphLaunch(sg.exec, h->stream));
      LSQ_HIP(hipStreamSynchronize(h->stream));
    } else {
      if (it > 0) correct();
      residual();
      read_status(h);
    }
    const StopStatus& st = *h->st_host;
    if (observe) observe(st, it, 0);
    hist.push_back(st.berr_max);
    for (int q = 0; q < 3; ++q) out.berr[q] = st.berr[q];
    out.berr_max = st.berr_max;
    out.steps = it;
    if (st.converged) {
      out.ok = true;
      if (!cont.more(st, it)) break;
    } else if (st.nonfinite || it >= o.maxit || stalled(hist)) {
      out.ok = false;
      break;
    }
    if (capturable && h->step_graphs && !tried) {
      tried = true;
      sg.capture(h, [&]() {
        correct();
        residual();
        LSQ_HIP(hipMemcpyAsync(h->st_host, h->st_dev, sizeof(StopStatus), hipMemcpyDeviceToHost,
                               h->ctx.stream));
      });
    }
  }
  LSQ_HIP(hipEventRecord(h->ev[3], h->stream));
  LSQ_HIP(hipEventSynchronize(h->ev[3]));
  out.ms_refine = elapsed(h->ev[2], h->ev[3]);
  return out;
}


// GMRES-IR refinement (Sections 5.2 / 5.3): the initial guess as in the
// classical case, then per outer step the scaled residual
// st = D f, GMRES on M_l F M_r w = M_l st, the correction du = M_r w, and the
// update undoing D.  ops.scale_in / ops.update hold the problem-specific scalings.
template <typename Solver, typename Args>
RungOut run_gmres(Worker* h, Solver& sv, const Args& a, int N,
                  const std::function<void()>& zero, const std::function<void()>& init,
                  const std::function<void()>& residual,
                  const std::function<double()>& alpha0,
                  const std::function<void(double*)>& scaled_residual,
                  const std::function<void(const double*)>& update, const lsq_opts& o,
                  const std::function<void(const StopStatus&, int, int)>& observe,
                  Continuation& cont) {
  Ctx& ctx = h->ctx;
  RungOut out;
  zero();
  LSQ_HIP(hipEventRecord(h->ev[2], h->stream));
  init();
  sv.alpha = o.alpha > 0 ? o.alpha : alpha0();
  sv.beta = o.beta > 0 ? o.beta : 1.0;
  sv.sa = std::sqrt(sv.alpha);
  double* st = ctx.ws->get<double>(std::max(N, 1));
  double* rhs = ctx.ws->get<double>(std::max(N, 1));
  double* w = ctx.ws->get<double>(std::max(N, 1));
  double* du = ctx.ws->get<double>(std::max(N, 1));
  auto apply = [&](const double* u, double* y) {
    sv.m_right(ctx, u, sv.t1);
    sv.f_apply(ctx, a, sv.t1, sv.t2);
    sv.m_left(ctx, sv.t2, y);
  };
  std::vector<double> hist;
  for (int it = 0;; ++it) {
    residual();
    read_status(h);
    const StopStatus& stt = *h->st_host;
    if (observe) observe(stt, it, out.inner);
    hist.push_back(stt.berr_max);
    for (int q = 0; q < 3; ++q) out.berr[q] = stt.berr[q];
    out.berr_max = stt.berr_max;
    out.steps = it;
    if (stt.converged) {
      out.ok = true;
      if (!cont.more(stt, it) || out.inner >= o.gmres_maxit) break;
    } else if (stt.nonfinite || it >= o.maxit || out.inner >= o.gmres_maxit || stalled(hist)) {
      out.ok = false;
      break;
    }
    scaled_residual(st);
    sv.m_left(ctx, st, rhs);
    // with a higher rung after this one, give up on an inner solve whose
    // rate cannot reach the inner tolerance within the rung's budget
    const GmresOut g = gmres(ctx, N, apply, rhs, w, o.gmres_restart, o.gmres_tol,
                             o.gmres_maxit - out.inner, true, h->more_rungs);
    out.inner += g.iters;
    if (g.hopeless) break;
    sv.m_right(ctx, w, du);
    update(du);
  }
  LSQ_HIP(hipEventRecord(h->ev[3], h->stream));
  LSQ_HIP(hipEventSynchronize(h->ev[3]));
  out.ms_refine = elapsed(h->ev[2], h->ev[3]);
  return out;
}

// Prepares the solver's triangular inverses, aggregated blocks and vectors for
// corrections in precision tc (with the GMRES operator's extras if gmres).
// A solver whose factors outlive the call (pctx set) keeps what it prepared
// in pctx's arena and prepares again only when tc or the solver kind changes.
// The factors' arena is rewound to the mark taken after the factorization
// before each new preparation, so alternating kinds keeps its size flat.
template <typename Solver>
void ensure_prepared(Solver& sv, Ctx& ctx, int tc, bool gmres) {
  if (sv.pctx && sv.prepared_tc == tc && (sv.prepared_gmres || !gmres)) return;
  Ctx& pc = sv.pctx ? *sv.pctx : ctx;
  if (sv.pctx && sv.has_pmark) {
    LSQ_HIP(hipStreamSynchronize(pc.stream));   // nothing in flight reads what the rewind frees
    pc.ws->rewind(sv.pmark);
  }
  if (gmres) sv.prepare_gmres(pc); else sv.prepare(pc, tc);
  sv.prepared_tc = tc;
  sv.prepared_gmres = gmres;
}

// One precision of the ladder for LSE: the factorization at prec, then the
// refinement solvers in order on the same factors (IR: Algorithm 2; GMRES:
// GMRES-IR; DIRECT: the FP64 factors with the classical loop).
// Factors an LSE at prec (the generalized RQ of Section 3.1); true if no
// panel Cholesky broke down.
// Power-of-two scale that maps a largest magnitude mx into [1/2, 1) (1 when
// mx is 0).  Every factorization works on its matrices scaled this way and
// scales the triangular factors back (exact in binary floating point): the
// FP16 and BF16 MFMA inputs rounded from them stay inside the 16-bit range
// (Section 6.1 asks for scaling on the conversion to a lower precision), and
// the Gram matrices of the Cholesky-QR panels cannot overflow or underflow.
double pow2_scale(double mx) {
  if (!(mx > 0.0) || !std::isfinite(mx)) return 1.0;
  int e = 0;
  std::frexp(mx, &e);
  return std::ldexp(1.0, -e);
}

// Factors an LSE at prec (the generalized RQ of Section 3.1); returns 0, or
// 1 / 2 when a panel Cholesky of the first / second factorization broke down.
// mx: largest magnitudes of A and B (for the scales; null: no scaling).
int lse_prefactor(Worker* h, const LseArgs& a, int prec, const lsq_opts& o, LseSolver& sv,
                  const double* mx) {
  Ctx& ctx = h->ctx;
  sv.m = a.m; sv.n = a.n; sv.p = a.p; sv.k = a.n - a.p;
  sv.prec_id = prec;
  prec_spec(prec, sv.ps);
  sv.sA = mx ? pow2_scale(mx[0]) : 1.0;
  sv.sB = mx ? pow2_scale(mx[1]) : 1.0;
  LSQ_HIP(hipEventRecord(h->ev[0], h->stream));
  sv.factor(ctx, a.A, a.lda, a.B, a.ldb, default_nb(o), prec == LSQ_PREC_FP64 ? 8 : sv.ps.tc);
  LSQ_HIP(hipEventRecord(h->ev[1], h->stream));
  const int stat_b = read_int(h, sv.fb.status);
  const int stat_a = read_int(h, sv.fa.status);
  sv.ms_factor = elapsed(h->ev[0], h->ev[1]);
  return stat_b ? 1 : (stat_a ? 2 : 0);
}

int gls_prefactor(Worker* h, const GlsArgs& a, int prec, const lsq_opts& o, GlsSolver& sv,
                  const double* mx) {
  Ctx& ctx = h->ctx;
  sv.n = a.n; sv.m = a.m; sv.p = a.p; sv.k = a.n - a.m;
  sv.prec_id = prec;
  prec_spec(prec, sv.ps);
  sv.sW = mx ? pow2_scale(mx[0]) : 1.0;
  sv.sV = mx ? pow2_scale(mx[1]) : 1.0;
  LSQ_HIP(hipEventRecord(h->ev[0], h->stream));
  sv.factor(ctx, a.W, a.ldw, a.V, a.ldv, default_nb(o), prec == LSQ_PREC_FP64 ? 8 : sv.ps.tc);
  LSQ_HIP(hipEventRecord(h->ev[1], h->stream));
  const int stat_w = read_int(h, sv.fw.status);
  const int stat_v = read_int(h, sv.fv.status);
  sv.ms_factor = elapsed(h->ev[0], h->ev[1]);
  return stat_w ? 1 : (stat_v ? 2 : 0);
}

// Singularity of an FP64 rung's triangles after it failed to certify: 1 when
// R (from B, LSE; from W, GLS) has a negligible pivot, 2 when T11 (LSE) /
// T22 (GLS) has one, else 0.
int fp64_singular(Ctx& ctx, const QRFactor& f1, int n1, const QRFactor& f2, int n2) {
  double d[2];
  diag_minmax(ctx, f1, 0, n1, d);
  if (n1 > 0 && !(d[0] > kSingularRatio * d[1])) return 1;
  diag_minmax(ctx, f2, 0, n2, d);
  if (n2 > 0 && !(d[0] > kSingularRatio * d[1])) return 2;
  return 0;
}

RungOut lse_rung(Worker* h, const LseArgs& a, int prec, const std::vector<int>& solvers,
                 const lsq_opts& o, double* x, double* r, double* v, int& attempts,
                 int& solver_used, const double* mx, BestIter* best, LseSolver* pre = nullptr,
                 int pre_code = 0) {
  Ctx& ctx = h->ctx;
  LseSolver local;
  const bool reuse = pre && pre->prec_id == prec;
  LseSolver& sv = reuse ? *pre : local;
  const int code = reuse ? pre_code : lse_prefactor(h, a, prec, o, sv, mx);
  const float ms_factor = sv.ms_factor;
  RungOut out;
  if (code != 0) {
    out.breakdown = code;
    ++attempts;
    solver_used = solvers.empty() ? LSQ_SOLVER_IR : solvers[0];
    return out;
  }
  double* f1 = ctx.ws->get<double>(a.m > 0 ? a.m : 1);
  double* f2 = ctx.ws->get<double>(a.p > 0 ? a.p : 1);
  double* f3 = ctx.ws->get<double>(a.n > 0 ? a.n : 1);
  const bool dd = o.residual == 1;
  ResidualScratch rs;
  residual_scratch_alloc(ctx, a.m, a.n, a.p, a.n, std::max(std::max(a.m, a.n), a.p), rs);
  auto residual = [&]() {
    lse_residual(ctx, a.m, a.n, a.p, a.A, a.lda, a.B, a.ldb, a.b, a.d, x, r, v, f1, f2, f3,
                 h->matnorms, o.tol, h->st_dev, dd, &rs);
  };
  auto zero = [&]() { vec_zero(ctx, x, 8, a.n); vec_zero(ctx, r, 8, a.m); vec_zero(ctx, v, 8, a.p); };
  auto init = [&]() { sv.correct(ctx, a.b, a.d, nullptr, x, r, v); };
  // double-double residual: the relative size of each correction of x
  double* xold = dd ? ctx.ws->get<double>(a.n > 0 ? a.n : 1) : nullptr;
  for (int solver : solvers) {
    ++attempts;
    solver_used = solver;
    Continuation cont(o);
    auto observe = [&](const StopStatus& st, int it, int inner) {
      (void)it;
      h->history.push_back({{st.berr[0], st.berr[1], st.berr[2]}, prec, solver, inner});
      if (best) best->observe(st, it, inner, prec, solver);
    };
    auto tracked = [&](const std::function<void()>& step) {
      if (dd) d2d(h, xold, x, a.n);
      step();
      if (dd) cont.observe_dx(rel_change(ctx, xold, x, a.n));
    };
    if (solver == LSQ_SOLVER_GMRES_IR) {
      ensure_prepared(sv, ctx, 8, true);
      const int m = a.m, p = a.p, n = a.n;
      out = run_gmres(
          h, sv, a, m + p + n, zero, init, residual,
          [&]() {
            double al = dev_norm2(ctx, r, m);
            if (!(al > 0.0)) al = std::sqrt(0.5) * min_abs_diag(ctx, sv.fa, 0, sv.tmn());
            return al > 0.0 ? al : 1.0;
          },
          [&](double* st) {
            vec_convert(ctx, st, 8, f1, 8, m, false, sv.sa);
            vec_convert(ctx, st + m, 8, f2, 8, p, false, sv.sa * sv.beta);
            vec_convert(ctx, st + m + p, 8, f3, 8, n, false, 1.0 / sv.sa);
          },
          [&](const double* du) {
            tracked([&]() {
              vec_axpy(ctx, r, 8, sv.sa, du, 8, m, false);
              vec_axpy(ctx, v, 8, -sv.sa * sv.beta, du + m, 8, p, false);
              vec_axpy(ctx, x, 8, 1.0 / sv.sa, du + m + p, 8, n, false);
            });
          },
          o, observe, cont);
    } else {
      ensure_prepared(sv, ctx, solver == LSQ_SOLVER_DIRECT ? 8 : sv.ps.tc, false);
      out = run_classical(h, zero, init, residual,
                          [&]() { tracked([&]() { sv.correct(ctx, f1, f2, f3, x, r, v); }); }, o,
                          observe, cont, !dd);
    }
    out.ms_factor = ms_factor;
    if (out.ok) break;
  }
  if (prec == LSQ_PREC_FP64 && !out.ok) out.singular = fp64_singular(ctx, sv.fb, a.p, sv.fa, sv.k);
  return out;
}

RungOut gls_rung(Worker* h, const GlsArgs& a, int prec, const std::vector<int>& solvers,
                 const lsq_opts& o, double* x, double* y, double* z, int& attempts,
                 int& solver_used, const double* mx, BestIter* best, GlsSolver* pre = nullptr,
                 int pre_code = 0) {
  Ctx& ctx = h->ctx;
  GlsSolver local;
  const bool reuse = pre && pre->prec_id == prec;
  GlsSolver& sv = reuse ? *pre : local;
  const int code = reuse ? pre_code : gls_prefactor(h, a, prec, o, sv, mx);
  const float ms_factor = sv.ms_factor;
  RungOut out;
  if (code != 0) {
    out.breakdown = code;
    ++attempts;
    solver_used = solvers.empty() ? LSQ_SOLVER_IR : solvers[0];
    return out;
  }
  double* f1 = ctx.ws->get<double>(a.p > 0 ? a.p : 1);
  double* f2 = ctx.ws->get<double>(a.n > 0 ? a.n : 1);
  double* f3 = ctx.ws->get<double>(a.m > 0 ? a.m : 1);
  const bool dd = o.residual == 1;
  ResidualScratch rs;
  residual_scratch_alloc(ctx, a.n, a.m, a.n, a.p, std::max(std::max(a.m, a.n), a.p), rs);
  auto residual = [&]() {
    gls_residual(ctx, a.n, a.m, a.p, a.W, a.ldw, a.V, a.ldv, a.d, x, y, z, f1, f2, f3,
                 h->matnorms, o.tol, h->st_dev, dd, &rs);
  };
  auto zero = [&]() { vec_zero(ctx, x, 8, a.m); vec_zero(ctx, y, 8, a.p); vec_zero(ctx, z, 8, a.n); };
  auto init = [&]() { sv.correct(ctx, nullptr, a.d, nullptr, x, y, z); };
  // double-double residual: the relative size of each correction of x and y
  double* xold = dd ? ctx.ws->get<double>(a.m > 0 ? a.m : 1) : nullptr;
  double* yold = dd ? ctx.ws->get<double>(a.p > 0 ? a.p : 1) : nullptr;
  for (int solver : solvers) {
    ++attempts;
    solver_used = solver;
    Continuation cont(o);
    auto observe = [&](const StopStatus& st, int it, int inner) {
      (void)it;
      h->history.push_back({{st.berr[0], st.berr[1], st.berr[2]}, prec, solver, inner});
      if (best) best->observe(st, it, inner, prec, solver);
    };
    auto tracked = [&](const std::function<void()>& step) {
      if (dd) { d2d(h, xold, x, a.m); d2d(h, yold, y, a.p); }
      step();
      if (dd) cont.observe_dx(std::max(rel_change(ctx, xold, x, a.m), rel_change(ctx, yold, y, a.p)));
    };
    if (solver == LSQ_SOLVER_GMRES_IR) {
      ensure_prepared(sv, ctx, 8, true);
      const int m = a.m, p = a.p, n = a.n;
      out = run_gmres(
          h, sv, a, p + n + m, zero, init, residual,
          [&]() {
            double al = dev_norm2(ctx, y, p);
            if (!(al > 0.0)) al = std::sqrt(0.5) * min_abs_diag(ctx, sv.fv, 0, sv.tnp());
            return al > 0.0 ? al : 1.0;
          },
          [&](double* st) {
            vec_convert(ctx, st, 8, f1, 8, p, false, sv.sa);
            vec_convert(ctx, st + p, 8, f2, 8, n, false, 1.0 / sv.sa);
            vec_convert(ctx, st + p + n, 8, f3, 8, m, false, sv.sa * sv.beta);
          },
          [&](const double* du) {
            tracked([&]() {
              vec_axpy(ctx, y, 8, sv.sa, du, 8, p, false);
              vec_axpy(ctx, z, 8, -1.0 / sv.sa, du + p, 8, n, false);
              vec_axpy(ctx, x, 8, sv.sa * sv.beta, du + p + n, 8, m, false);
            });
          },
          o, observe, cont);
    } else {
      ensure_prepared(sv, ctx, solver == LSQ_SOLVER_DIRECT ? 8 : sv.ps.tc, false);
      out = run_classical(h, zero, init, residual,
                          [&]() { tracked([&]() { sv.correct(ctx, f1, f2, f3, x, y, z); }); }, o,
                          observe, cont, !dd);
    }
    out.ms_factor = ms_factor;
    if (out.ok) break;
  }
  if (prec == LSQ_PREC_FP64 && !out.ok) out.singular = fp64_singular(ctx, sv.fw, a.m, sv.fv, sv.k);
  return out;
}

// Selector input and output for one instance from the factors of its first
// ladder rung (FP32, kSelFactorPrec): the triangles' diagonal statistics, the
// features and, with weights, the MLP classes.  host: 16 features, 7 logits
// (float) then 2 classes (int).
struct Selection {
  float feats[kSelFeatures];
  float logits[kSelOut];
  int cls[2] = {3, 0};
};

Selection select_run(Worker* h, int type, int m, int n, int p, const QRFactor& f1, int n1,
                     const QRFactor& f2, int k2, int n2, const float* sel_w) {
  Ctx& ctx = h->ctx;
  float* buf = ctx.ws->get<float>(64);
  int* cls = ctx.ws->get<int>(2);
  diag_stats(ctx, f1, 0, n1, buf);
  diag_stats(ctx, f2, 0, k2, buf + 3);
  diag_stats(ctx, f2, 0, n2, buf + 6);
  features(ctx, type, m, n, p, h->matnorms, buf, buf + 3, buf + 6, buf + 16);
  if (sel_w) mlp_select(ctx, sel_w, buf + 16, buf + 32, cls);
  LSQ_HIP(hipMemcpyAsync(h->pin, buf, sizeof(float) * 64, hipMemcpyDeviceToHost, h->stream));
  if (sel_w)
    LSQ_HIP(hipMemcpyAsync(h->pin + 32, cls, sizeof(int) * 2, hipMemcpyDeviceToHost, h->stream));
  LSQ_HIP(hipStreamSynchronize(h->stream));
  Selection out;
  const float* hb = reinterpret_cast<const float*>(h->pin);
  for (int i = 0; i < kSelFeatures; ++i) out.feats[i] = hb[16 + i];
  for (int i = 0; i < kSelOut; ++i) out.logits[i] = sel_w ? hb[32 + i] : 0.0f;
  if (sel_w) {
    const int* hc = reinterpret_cast<const int*>(h->pin + 32);
    out.cls[0] = hc[0];
    out.cls[1] = hc[1];
  }
  return out;
}

// Precision / solver of a selector class.
int class_prec(int c) {
  static const int map[kSelPrec] = {LSQ_PREC_FP8E4M3, LSQ_PREC_BF16, LSQ_PREC_FP16, LSQ_PREC_FP32,
                                    LSQ_PREC_FP64};
  return map[c < 0 ? 0 : (c >= kSelPrec ? kSelPrec - 1 : c)];
}
// Precision of the factorization the features are taken from: the first
// rung of the plain ladder, so that its factors are kept (no second
// factorization) whenever the selector picks an FP32 rung, and an instance it
// sends to FP64 pays the FP32 factorization but none of the failing
// refinement the ladder would run before escalating.  The diagonals of the
// FP32 triangles estimate condition numbers up to about 1/u_FP32.
constexpr int kSelFactorPrec = LSQ_PREC_FP32;
int class_solver(int c) { return c == 1 ? LSQ_SOLVER_GMRES_IR : LSQ_SOLVER_IR; }

// Escalation ladder: (precision, refinement solvers on that precision's
// factors).  Starting at the requested rung: with IR requested, each
// precision tries classical IR and then GMRES-IR on the same factors; with
// GMRES requested, GMRES-IR only; precisions rise FP8 -> BF16 -> FP16 -> FP32 and the
// ladder ends with the FP64 direct path.  The block-diagonal preconditioners
// cover every admissible shape (Sections 5.2 and 5.3), so GMRES-IR is always
// available.
std::vector<std::pair<int, std::vector<int>>> ladder(const lsq_opts& o) {
  std::vector<std::pair<int, std::vector<int>>> r;
  int prec = o.prec == LSQ_PREC_AUTO ? LSQ_PREC_FP32 : o.prec;
  int solver = o.solver == LSQ_SOLVER_AUTO ? LSQ_SOLVER_IR : o.solver;
  if (solver == LSQ_SOLVER_DIRECT || prec == LSQ_PREC_FP64) {
    r.push_back({LSQ_PREC_FP64, {LSQ_SOLVER_DIRECT}});
    return r;
  }
  if (!o.escalate) {
    r.push_back({prec, {solver}});
    return r;
  }
  std::vector<int> solvers;
  if (solver == LSQ_SOLVER_IR) solvers.push_back(LSQ_SOLVER_IR);
  solvers.push_back(LSQ_SOLVER_GMRES_IR);
  const int order[] = {LSQ_PREC_FP8E4M3, LSQ_PREC_BF16, LSQ_PREC_FP16, LSQ_PREC_FP32};
  bool on = false;
  for (int q : order) {
    if (q == prec) on = true;
    if (on) r.push_back({q, solvers});
  }
  r.push_back({LSQ_PREC_FP64, {LSQ_SOLVER_DIRECT}});
  return r;
}

int fail(lsq_handle h, int code, const std::string& msg) {
  if (h) h->last_error = msg;
  return code;
}

// Runs body on worker w: selects the device, rewinds w's arena and turns HIP
// errors into return code 4 with a message in *err.  Work left on the side
// stream (a solver's early preparation that was never consumed) finishes
// before the call returns: the next call rewinds the arena it writes into.
int guard_w(Worker* w, std::string* err, const char* fn, const std::function<int()>& body) {
  int rc = 4;
  try {
    LSQ_HIP(hipSetDevice(w->device));
    w->arena.reset();
    w->more_rungs = false;
    rc = body();
  } catch (const HipError& e) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s failed: %s", fn, e.where, hipGetErrorString(e.code));
    if (err) *err = buf;
    rc = 4;
  } catch (const std::exception& e) {
    if (err) *err = std::string(fn) + ": " + e.what();
    rc = 4;
  }
  if (w->ctx.side) (void)hipStreamSynchronize(w->ctx.side);
  return rc;
}

int guard(lsq_handle h, const char* fn, const std::function<int()>& body) {
  h->last_error.clear();
  return guard_w(&h->w, &h->last_error, fn, body);
}

}  // namespace

// A captured persistent batch (lsq_batch_plan_create): the problem set, its
// longest-first order, the launch shape taken at capture, device buffers of
// its own and the instantiated graph.
struct lsq_batch_plan_st {
  lsq_handle h = nullptr;
  std::vector<lsq_problem> probs;
  std::vector<int> order;
  lsq_opts opts{};
  double route = 0.0, fp64_share = 0.0, pre_share = 0.0;
  BatchProb* dprobs = nullptr;
  int* dorder = nullptr;
  int* dcounter = nullptr;
  int* dstarted = nullptr;
  BatchOut* dout = nullptr;
  BatchOut* dout64 = nullptr;
  EscQueue* q = nullptr;
  char* dws = nullptr;
  char* dws64 = nullptr;
  hipStream_t cap = nullptr;                    // the stream the graph was recorded on
  hipGraphExec_t exec = nullptr;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
    for (void* ptr : {(void*)dprobs, (void*)dorder, (void*)dcounter, (void*)dstarted, (void*)dout, (void*)dout64,
                      (void*)q, (void*)dws, (void*)dws64})
      if (ptr) (void)hipFree(ptr);
    dprobs = nullptr; dorder = dcounter = dstarted = nullptr; dout = dout64 = nullptr; q = nullptr;
    dws = dws64 = nullptr;
  }
};

namespace {

// Persistent batched execution of the eligible instances among todo (one
// work-group per instance): the first rung in first_prec (FP32 or FP64), the
// failures again in FP64 when escalating.  Writes res for the instances it
// certifies and returns those left for the worker ladder, longest first.
// With a plan (concurrent FP32 + FP64 mode only): on its first call the
// plan's buffers are allocated, the descriptors and the order uploaded and
// the launch sequence captured as a graph, and nothing runs; on later calls
// the graph is replayed in place of the launches.
std::vector<int> batch_persistent(lsq_handle h, const lsq_problem* probs, const std::vector<int>& todo,
                                  const lsq_opts& o, int first_prec, lsq_result* res,
                                  lsq_batch_plan_st* plan = nullptr) {
  Worker* w = &h->w;
  Ctx& ctx = w->ctx;
  const int count = (int)todo.size();
  std::vector<BatchProb> hp(count);
  std::vector<int> cur, rest;
  size_t stride = 256;
  for (int q = 0; q < count; ++q) {
    const lsq_problem& p = probs[todo[q]];
    hp[q] = BatchProb{p.type == LSQ_LSE ? 0 : 1, p.m, p.n, p.p, p.A, p.B, p.b, p.d, p.lda, p.ldb,
                      p.x, p.y};
    if (batch_eligible(hp[q])) {
      cur.push_back(q);
      stride = std::max(stride, batch_ws_bytes(hp[q]));
    } else {
      rest.push_back(todo[q]);
    }
  }
  if (cur.empty()) return rest;
  const bool capture = plan && !plan->exec;
  double route = h->batch_route, fp64_share = h->batch_fp64_share, pre_share = h->batch_pre;
  if (capture && !(first_prec == LSQ_PREC_FP32 && o.escalate && ctx.side && h->batch_mode == LSQ_BATCH_AUTO &&
                   rest.empty()))
    throw std::runtime_error("batch plan: only the concurrent FP32 + FP64 batch of eligible instances is captured");
  if (plan && plan->exec) {
    // the launch shape the graph was captured with
    route = plan->route;
    fp64_share = plan->fp64_share;
    pre_share = plan->pre_share;
  } else {
    int dim = 0;
    for (int q : cur) dim = std::max(dim, std::max(hp[q].m, std::max(hp[q].n, hp[q].p)));
    int best = -1;
    for (int e = 0; e < (int)h->batch_tuning.size(); ++e) {
      const auto& te = h->batch_tuning[e];
      if (te.max_dim < dim || te.esc_max < h->last_escalation) continue;
      if (best < 0 || te.max_dim < h->batch_tuning[best].max_dim ||
          (te.max_dim == h->batch_tuning[best].max_dim && te.esc_max < h->batch_tuning[best].esc_max))
        best = e;
    }
    if (best >= 0) {
      route = h->batch_tuning[best].route;
      fp64_share = h->batch_tuning[best].share;
      pre_share = h->batch_tuning[best].pre;
    }
  }
  const int max_grid = std::max(batch_blocks_per_cu(4), batch_blocks_per_cu(8)) * h->num_cu;
  const int grid = std::min((int)cur.size(), max_grid);
  w->arena.reset();
  BatchProb* dprobs;
  int* dorder;
  int* dcounter;
  BatchOut* dout;
  char* dws;
  if (plan) {
    if (capture) {
      plan->route = route;
      plan->fp64_share = fp64_share;
      plan->pre_share = pre_share;
      LSQ_HIP(hipMalloc(&plan->dprobs, sizeof(BatchProb) * count));
      LSQ_HIP(hipMalloc(&plan->dorder, sizeof(int) * count));
      LSQ_HIP(hipMalloc(&plan->dcounter, sizeof(int)));
      LSQ_HIP(hipMalloc(&plan->dstarted, sizeof(int)));
      LSQ_HIP(hipMalloc(&plan->dout, sizeof(BatchOut) * count));
      LSQ_HIP(hipMalloc(&plan->dws, stride * (size_t)grid));
      LSQ_HIP(hipMemcpyAsync(plan->dprobs, hp.data(), sizeof(BatchProb) * count, hipMemcpyHostToDevice,
                             ctx.stream));
    }
    dprobs = plan->dprobs;
    dorder = plan->dorder;
    dcounter = plan->dcounter;
    dout = plan->dout;
    dws = plan->dws;
  } else {
    dprobs = ctx.ws->get<BatchProb>(count);
    dorder = ctx.ws->get<int>(count);
    dcounter = ctx.ws->get<int>(1);
    dout = ctx.ws->get<BatchOut>(count);
    dws = static_cast<char*>(ctx.ws->alloc(stride * (size_t)grid));
    LSQ_HIP(hipMemcpyAsync(dprobs, hp.data(), sizeof(BatchProb) * count, hipMemcpyHostToDevice, ctx.stream));
  }
  std::vector<BatchOut> hout(count);
  std::vector<int> attempts(count, 0);
  int prec = first_prec;
  // per-instance clocks of both attempts (ticks; 0 where no attempt ran)
  std::vector<BatchOut> clk32(count), clk64(count);
  for (auto* v : {&clk32, &clk64})
    for (auto& b : *v) b.t0 = b.t1 = b.t2 = 0;
  const double tick_ms = 1.0 / h->wclk_khz;
  auto span = [&](unsigned long long a, unsigned long long b) {
    return b > a ? (float)((double)(b - a) * tick_ms) : 0.0f;
  };
  auto certified = [&](int q, int rung, const BatchOut& bo) {
    if (!res) return;
    lsq_result& r = res[todo[q]];
    r = lsq_result{};
    r.info = 0;
    r.prec_used = rung;
    r.solver_used = rung == LSQ_PREC_FP64 ? LSQ_SOLVER_DIRECT : LSQ_SOLVER_IR;
    r.attempts = attempts[q];
    r.ir_steps = bo.steps;
    for (int k = 0; k < 3; ++k) r.berr[k] = bo.berr[k];
    r.berr_max = bo.berr_max;
    // in-kernel wall clock, summed over the attempts (factorization includes
    // the instance's conversions; refinement starts with the initial solve)
    for (const BatchOut* c : {&clk32[q], &clk64[q]}) {
      r.ms_factor += span(c->t0, c->t1);
      r.ms_refine += span(c->t1, c->t2);
    }
  };
  auto record_timeline = [&]() {
    unsigned long long base = ~0ull;
    for (int q = 0; q < count; ++q)
      for (const BatchOut* c : {&clk32[q], &clk64[q]})
        if (c->t0) base = std::min(base, c->t0);
    int span_n = 0;
    for (int q = 0; q < count; ++q) span_n = std::max(span_n, todo[q] + 1);
    h->timeline.assign((size_t)6 * span_n, NAN);
    // the timeline is indexed by the caller's problem index
    for (int q = 0; q < count; ++q) {
      const BatchOut* cs[2] = {&clk32[q], &clk64[q]};
      for (int a = 0; a < 2; ++a) {
        if (!cs[a]->t0) continue;
        double* o = &h->timeline[(size_t)6 * todo[q] + 3 * a];
        o[0] = (double)(cs[a]->t0 - base) * tick_ms;
        o[1] = (double)(cs[a]->t1 - base) * tick_ms;
        o[2] = (double)(cs[a]->t2 - base) * tick_ms;
      }
    }
  };
  auto keep_clock = [&](int q, int rung, const BatchOut& bo) {
    BatchOut& c = rung == LSQ_PREC_FP64 ? clk64[q] : clk32[q];
    if (bo.info >= 0) { c.t0 = bo.t0; c.t1 = bo.t1; c.t2 = bo.t2; }
  };
  // the diagonal-ratio route scales with the factorization's unit roundoff
  // (the tuned values are for FP32, u = 2^-24; BF16 has u = 2^-8)
  const double route_bf16 = route * std::ldexp(1.0, -16);
  if ((prec == LSQ_PREC_FP32 || prec == LSQ_PREC_BF16) && o.escalate && ctx.side &&
      h->batch_mode == LSQ_BATCH_AUTO) {
    // FP32 launch with the FP64 rung running beside it: each failure is
    // queued on the device and solved in FP64 while the FP32 launch goes on;
    // what no consumer took (see batch_launch_escalating) falls through to
    // the FP64 launch below
    const int n = (int)cur.size();
    if (capture) {
      LSQ_HIP(hipMalloc(&plan->q, esc_queue_bytes(count)));
      LSQ_HIP(hipMalloc(&plan->dout64, sizeof(BatchOut) * count));
    }
    EscQueue* q = plan ? plan->q : static_cast<EscQueue*>(ctx.ws->alloc(esc_queue_bytes(count)));
    BatchOut* dout64 = plan ? plan->dout64 : ctx.ws->get<BatchOut>(count);
    // a share of the compute units (a quarter by default, about the share of
    // the FP64 work in the mixed batch) runs the FP64 rung from the start;
    // the rest join when the FP32 launch is over
    const int cu64 = std::min(h->num_cu - 1, std::max(1, (int)std::lround(h->num_cu * fp64_share)));
    const int g32 = std::min(batch_blocks_per_cu(4) * (h->num_cu - cu64), n);
    const int g64a = std::min(batch_blocks_per_cu(8) * cu64, n);
    const int g64b = std::min(batch_blocks_per_cu(8) * (h->num_cu - cu64), n);
    if (capture) LSQ_HIP(hipMalloc(&plan->dws64, stride * (size_t)(g64a + g64b)));
    char* dws64 = plan ? plan->dws64 : static_cast<char*>(ctx.ws->alloc(stride * (size_t)(g64a + g64b)));
    if (!plan || capture)
      LSQ_HIP(hipMemcpyAsync(dorder, cur.data(), sizeof(int) * n, hipMemcpyHostToDevice, ctx.stream));
    int* started = reinterpret_cast<int*>(ctx.pin + kPinDoubles - 1);   // last pinned slot
    // the longest instances (the head of the order) that the FP64 rung takes
    // at once: an FP32 attempt that escalates would put both attempts of one
    // of them on the launch's critical path
    // at most 7/8 of the batch: the FP32 rung always sees part of it, where
    // the escalation fraction that picks the next call's table entry is measured
    const int pre = std::min(n - (n + 7) / 8, (int)std::lround(pre_share * g64a));
    // the FP32 launch's work for its timer: the instances it factors
    double flops = 0.0;
    for (int i = pre; i < n; ++i) flops += batch_factor_flops(hp[cur[i]]);
    if (capture) {
      // record the launches on a stream of the plan's own (the handle's
      // stream may be the legacy default stream, which cannot be captured),
      // with no timer events inside the graph; replays go to the handle's
      // stream
      LSQ_HIP(hipStreamSynchronize(ctx.stream));
      if (!plan->cap) LSQ_HIP(hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking));
      const hipStream_t own = ctx.stream;
      KernelTimer* timer = ctx.timer;
      ctx.timer = nullptr;
      ctx.stream = plan->cap;
      hipGraph_t graph = nullptr;
      try {
        LSQ_HIP(hipStreamBeginCapture(ctx.stream, hipStreamCaptureModeThreadLocal));
        try {
          batch_capture_escalating(ctx, dprobs, dorder, n, dcounter, dws, stride, g32, dws64, g64a, g64b, q,
                                   o.tol, o.maxit, o.polish, route, dout, dout64, h->esc_wait_ms,
                                   plan->dstarted, n / 4, pre);
        } catch (...) {
          (void)hipStreamEndCapture(ctx.stream, &graph);
          throw;
        }
        LSQ_HIP(hipStreamEndCapture(ctx.stream, &graph));
      } catch (...) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();                // leave no error behind for the caller's next check
        ctx.stream = own;
        ctx.timer = timer;
        throw;
      }
      ctx.stream = own;
      ctx.timer = timer;
      const hipError_t ie = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) (void)hipGetLastError();
      LSQ_HIP(ie);
      return {};
    }
    if (plan) {
      LSQ_HIP(hipGraphLaunch(plan->exec, ctx.stream));
    } else {
      const bool lowp = prec == LSQ_PREC_BF16;
      batch_launch_escalating(ctx, dprobs, dorder, n, dcounter, dws, stride, g32, dws64, g64a, g64b, q,
                              o.tol, o.maxit, o.polish, lowp ? route_bf16 : route, dout, dout64, flops,
                              h->esc_wait_ms, started, n / 4, pre, lowp);
    }
    std::vector<BatchOut> hout64(count);
    LSQ_HIP(hipMemcpyAsync(hout.data(), dout, sizeof(BatchOut) * count, hipMemcpyDeviceToHost, ctx.stream));
    LSQ_HIP(hipMemcpyAsync(hout64.data(), dout64, sizeof(BatchOut) * count, hipMemcpyDeviceToHost, ctx.stream));
    LSQ_HIP(hipStreamSynchronize(ctx.stream));
    // the FP64 rung's work for its timer: the instances its launches solved
    // (a replayed plan records no timer events, so it adds no work either)
    if (!plan) {
      double flops64 = 0.0;
      for (int qq : cur)
        if (hout64[qq].info != -1) flops64 += batch_factor_flops(hp[qq]);
      ktimer_add(ctx, kKBatchEsc, flops64, 0.0);
    }
    // the regime for the next call's table entry: the share of the instances
    // that tried the FP32 rung and did not certify there
    if (prec == LSQ_PREC_FP32 && n > pre) {
      int failed = 0;
      for (int i = pre; i < n; ++i) failed += hout[cur[i]].info != 0;
      h->last_escalation = (double)failed / (double)(n - pre);
    }
    std::vector<int> pending;
    for (int i = 0; i < n; ++i) {
      const int qq = cur[i];
      if (i >= pre) keep_clock(qq, prec, hout[qq]);
      if (hout64[qq].info != -1) keep_clock(qq, LSQ_PREC_FP64, hout64[qq]);
    }
    for (int i = 0; i < n; ++i) {
      const int qq = cur[i];
      if (i < pre) {
        // no FP32 attempt: the FP64 rung's result, or the FP64 launch below
        if (hout64[qq].info == -1) {
          pending.push_back(qq);
        } else {
          ++attempts[qq];
          if (hout64[qq].info == 0) certified(qq, LSQ_PREC_FP64, hout64[qq]);
          else rest.push_back(todo[qq]);
        }
        continue;
      }
      ++attempts[qq];
      if (hout[qq].info == 0) {
        certified(qq, prec, hout[qq]);
      } else if (hout64[qq].info == -1) {
        pending.push_back(qq);
      } else {
        ++attempts[qq];
        if (hout64[qq].info == 0) certified(qq, LSQ_PREC_FP64, hout64[qq]);
        else rest.push_back(todo[qq]);
      }
    }
    if (pending.empty()) {
      record_timeline();
      return rest;
    }
    cur = pending;
    prec = LSQ_PREC_FP64;
  }
  if (plan) {
    // the plan's order and outputs stay as captured: this launch takes its
    // own from the arena
    dorder = ctx.ws->get<int>(count);
    dcounter = ctx.ws->get<int>(1);
    dout = ctx.ws->get<BatchOut>(count);
    dws = static_cast<char*>(ctx.ws->alloc(stride * (size_t)grid));
  }
  for (;;) {
    LSQ_HIP(hipMemcpyAsync(dorder, cur.data(), sizeof(int) * cur.size(), hipMemcpyHostToDevice, ctx.stream));
    double flops = 0.0;
    for (int q : cur) flops += batch_factor_flops(hp[q]);
    const bool last = prec == LSQ_PREC_FP64 || !o.escalate;
    const int tw = prec == LSQ_PREC_FP64 ? 8 : 4;
    const int g = std::min(batch_blocks_per_cu(tw) * h->num_cu, (int)cur.size());
    batch_launch(ctx, tw, dprobs, dorder, (int)cur.size(), dcounter, dws, stride, g, o.tol, o.maxit, o.polish,
                 !last, prec == LSQ_PREC_BF16 ? route_bf16 : route, dout, flops, prec == LSQ_PREC_BF16);
    LSQ_HIP(hipMemcpyAsync(hout.data(), dout, sizeof(BatchOut) * count, hipMemcpyDeviceToHost, ctx.stream));
    LSQ_HIP(hipStreamSynchronize(ctx.stream));
    std::vector<int> failed;
    for (int q : cur) keep_clock(q, prec, hout[q]);
    for (int q : cur) {
      ++attempts[q];
      const BatchOut& bo = hout[q];
      if (bo.info != 0) {
        failed.push_back(q);
        continue;
      }
      certified(q, prec, bo);
    }
    if (failed.empty() || prec == LSQ_PREC_FP64 || !o.escalate) {
      for (int q : failed) rest.push_back(todo[q]);
      break;
    }
    cur = failed;
    prec = LSQ_PREC_FP64;
  }
  record_timeline();
  return rest;
}
}  // namespace

// Overrides of the defaults from the environment (LSQ_PREC, LSQ_SOLVER,
// LSQ_TOL, LSQ_MAXIT, LSQ_GMRES_MAXIT, LSQ_ESCALATE, LSQ_RESIDUAL); a value
// that does not parse, or lies outside its field's range, is ignored.
static void apply_env_overrides(lsq_opts* o) {
  auto str = [](const char* k) -> const char* {
    const char* v = std::getenv(k);
    return (v && *v) ? v : nullptr;
  };
  auto num = [&](const char* k, double& out) {
    const char* v = str(k);
    if (!v) return false;
    char* end = nullptr;
    const double d = std::strtod(v, &end);
    if (end == v || *end != '\0' || !std::isfinite(d)) return false;
    out = d;
    return true;
  };
  if (const char* v = str("LSQ_PREC")) {
    static const std::pair<const char*, int> names[] = {
        {"auto", LSQ_PREC_AUTO}, {"fp8", LSQ_PREC_FP8E4M3}, {"bf16", LSQ_PREC_BF16},
        {"fp16", LSQ_PREC_FP16}, {"fp32", LSQ_PREC_FP32},    {"fp64", LSQ_PREC_FP64}};
    for (const auto& nm : names)
      if (std::strcmp(v, nm.first) == 0) o->prec = nm.second;
  }
  if (const char* v = str("LSQ_SOLVER")) {
    static const std::pair<const char*, int> names[] = {
        {"auto", LSQ_SOLVER_AUTO}, {"ir", LSQ_SOLVER_IR}, {"gmres", LSQ_SOLVER_GMRES_IR},
        {"direct", LSQ_SOLVER_DIRECT}};
    for (const auto& nm : names)
      if (std::strcmp(v, nm.first) == 0) o->solver = nm.second;
  }
  double d;
  if (num("LSQ_TOL", d) && d >= 0.0) o->tol = d;
  if (num("LSQ_MAXIT", d) && d >= 0.0 && d <= 1e6 && d == std::floor(d)) o->maxit = (int)d;
  if (num("LSQ_GMRES_MAXIT", d) && d >= 1.0 && d <= 1e6 && d == std::floor(d)) o->gmres_maxit = (int)d;
  if (num("LSQ_ESCALATE", d) && (d == 0.0 || d == 1.0)) o->escalate = (int)d;
  if (num("LSQ_RESIDUAL", d) && (d == 0.0 || d == 1.0)) o->residual = (int)d;
}

// ================================================================== C ABI ==
extern "C" {

void lsq_opts_default(lsq_opts* o) {
  if (!o) return;
  o->prec = LSQ_PREC_FP32;
  o->solver = LSQ_SOLVER_IR;
  o->tol = 1e-14;
  o->maxit = 40;
  o->gmres_restart = 30;
  o->gmres_tol = 1e-10;
  o->gmres_maxit = 300;
  o->escalate = 1;
  o->alpha = 0.0;
  o->beta = 0.0;
  o->nb = 0;
  o->polish = 8.0 * 1.1102230246251565e-16;
  o->residual = 0;
  apply_env_overrides(o);
}

int lsq_create(lsq_handle* out, int device) {
  if (!out) return -1;
  *out = nullptr;
  lsq_handle h = new (std::nothrow) lsq_handle_st();
  if (!h) return 4;
  try {
    h->device = device;
    LSQ_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    LSQ_HIP(hipGetDeviceProperties(&prop, device));
    h->num_cu = prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
      h->wclk_khz = (double)khz;
    h->w.init(device, h->num_cu, false);
    scratch_setup(device);
    LSQ_HIP(hipDeviceSynchronize());
  } catch (const HipError&) {
    lsq_destroy(h);
    return 4;
  } catch (const std::exception&) {
    lsq_destroy(h);
    return 4;
  }
  *out = h;
  return 0;
}

int lsq_destroy(lsq_handle h) {
  if (!h) return 0;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  for (auto& e : h->timer.ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& wp : h->pool) wp->release();
  h->w.release();
  if (h->sel_w) (void)hipFree(h->sel_w);
  delete h;
  return 0;
}

int lsq_set_stream(lsq_handle h, void* stream) {
  if (!h) return -1;
  h->w.stream = static_cast<hipStream_t>(stream);
  h->w.ctx.stream = h->w.stream;
  return 0;
}

int lsq_set_batch_workers(lsq_handle h, int workers) {
  if (!h) return -1;
  if (workers < 1 || workers > 64) return -2;
  h->batch_workers = workers;
  return 0;
}

int lsq_set_batch_mode(lsq_handle h, int mode) {
  if (!h) return -1;
  if (mode != LSQ_BATCH_AUTO && mode != LSQ_BATCH_WORKERS && mode != LSQ_BATCH_SEQUENTIAL)
    return fail(h, -2, "unknown batch mode");
  h->batch_mode = mode;
  return 0;
}

int lsq_dbg_lookahead(lsq_handle h, int mode) {
  if (!h) return -1;
  if (mode < 0 || mode > 1) return fail(h, -2, "look-ahead mode outside 0..1");
  h->w.ctx.lookahead = mode != 0;
  return 0;
}

int lsq_dbg_deterministic(lsq_handle h, int on) {
  if (!h) return -1;
  if (on < 0 || on > 1) return fail(h, -2, "deterministic mode outside 0..1");
  h->w.ctx.deterministic = on != 0;
  return 0;
}

int lsq_dbg_history(lsq_handle h, int max_steps, double* berr, int* rung) {
  if (!h) return -1;
  if (max_steps < 0 || (max_steps > 0 && !berr)) return -2;
  const auto& hs = h->w.history;
  const int n = (int)hs.size();
  for (int i = 0; i < n && i < max_steps; ++i) {
    for (int k = 0; k < 3; ++k) berr[3 * i + k] = hs[i].berr[k];
    if (rung) {
      rung[3 * i] = hs[i].prec;
      rung[3 * i + 1] = hs[i].solver;
      rung[3 * i + 2] = hs[i].inner;
    }
  }
  return n;
}

int lsq_batch_tuning(lsq_handle h, int n, const int* max_dim, const double* route,
                     const double* fp64_share, const double* pre, const double* esc_max) {
  if (!h) return -1;
  if (n < 0 || (n > 0 && (!max_dim || !route || !fp64_share || !pre)))
    return fail(h, -2, "lsq_batch_tuning: bad table");
  std::vector<lsq_handle_st::BatchTune> t;
  for (int i = 0; i < n; ++i) {
    const double em = esc_max ? esc_max[i] : 1.0;
    if (max_dim[i] < 1 || !(route[i] >= 0.0) || !(fp64_share[i] > 0.0 && fp64_share[i] < 1.0) ||
        !(pre[i] >= 0.0 && pre[i] <= kMaxBatchPre) || !(em >= 0.0 && em <= 1.0))
      return fail(h, -3, "lsq_batch_tuning: entry " + std::to_string(i) + " out of range");
    t.push_back({max_dim[i], route[i], fp64_share[i], pre[i], em});
  }
  h->batch_tuning = std::move(t);
  h->last_escalation = 1.0;
  return 0;
}

int lsq_dbg_batch_regime(lsq_handle h, double* last_escalation) {
  if (!h) return -1;
  if (!last_escalation) return -2;
  *last_escalation = h->last_escalation;
  return 0;
}

int lsq_dbg_batch_pre(lsq_handle h, double per_wg) {
  if (!h) return -1;
  if (!(per_wg >= 0.0 && per_wg <= kMaxBatchPre)) return fail(h, -2, "lsq_dbg_batch_pre: outside [0, 8]");
  h->batch_pre = per_wg;
  return 0;
}

int lsq_dbg_batch_split(lsq_handle h, double fp64_share) {
  if (!h) return -1;
  if (!(fp64_share > 0.0 && fp64_share < 1.0)) return fail(h, -2, "lsq_dbg_batch_split: share outside (0, 1)");
  h->batch_fp64_share = fp64_share;
  return 0;
}

int lsq_dbg_batch_route(lsq_handle h, double ratio) {
  if (!h) return -1;
  if (!(ratio >= 0.0)) return fail(h, -2, "lsq_dbg_batch_route: ratio must be >= 0");
  h->batch_route = ratio;
  return 0;
}

int lsq_dbg_batch_timeline(lsq_handle h, int count, double* out) {
  if (!h) return -1;
  if (count < 0 || (count > 0 && !out)) return -2;
  const size_t have = h->timeline.size() / 6;
  for (int i = 0; i < count; ++i)
    for (int k = 0; k < 6; ++k) out[(size_t)6 * i + k] = (size_t)i < have ? h->timeline[(size_t)6 * i + k] : NAN;
  return 0;
}

int lsq_dbg_batch_wait(lsq_handle h, double ms) {
  if (!h) return -1;
  if (!(ms >= 0.0 && ms <= 1000.0)) return fail(h, -2, "wait bound outside [0, 1000] ms");
  h->esc_wait_ms = ms;
  return 0;
}

const char* lsq_last_error(lsq_handle h) { return h ? h->last_error.c_str() : ""; }

static void fill_result(lsq_result* res, int info, int prec, int solver, int attempts,
                        const RungOut& ro) {
  if (!res) return;
  res->info = info;
  res->prec_used = prec;
  res->solver_used = solver;
  res->attempts = attempts;
  res->ir_steps = ro.steps;
  res->gmres_iters = ro.inner;
  for (int q = 0; q < 3; ++q) res->berr[q] = ro.berr[q];
  res->berr_max = ro.berr_max;
  res->ms_convert = ro.ms_convert;
  res->ms_factor = ro.ms_factor;
  res->ms_refine = ro.ms_refine;
}

}  // extern "C"

namespace {
// Ingest of one solve: FP64 norms for the stop test, the largest magnitudes
// (for the FP16 / BF16 scales) and a finiteness check, in one read of each
// input.  Returns false when an input holds a non-finite value; mx receives
// the largest magnitudes of the four inputs, ms the stream time of the scan.
bool ingest(Worker* w, const double* M1, int ld1, int r1, int c1, const double* M2, int ld2, int r2,
            int c2, const double* v1, int n1, const double* v2, int n2, double* mx, float* ms) {
  Ctx& ctx = w->ctx;
  LSQ_HIP(hipEventRecord(w->ev[0], w->stream));
  frob_norms(ctx, M1, ld1, r1, c1, M2, ld2, r2, c2, v1, n1, v2, n2, w->matnorms);
  if (w->norm_scale != 1.0) scale_first(ctx, w->matnorms, 2, w->norm_scale);
  LSQ_HIP(hipEventRecord(w->ev[1], w->stream));
  LSQ_HIP(hipMemcpyAsync(w->pin, w->matnorms, 8 * sizeof(double), hipMemcpyDeviceToHost, w->stream));
  LSQ_HIP(hipStreamSynchronize(w->stream));
  bool finite = true;
  for (int k = 0; k < 4; ++k) {
    mx[k] = w->pin[4 + k];
    if (std::isnan(mx[k])) finite = false;
  }
  *ms = elapsed(w->ev[0], w->ev[1]);
  return finite;
}

void fill_best(lsq_result* res, int attempts, const BestIter& b, const RungOut& last) {
  if (!res) return;
  res->info = 3;
  res->prec_used = b.prec;
  res->solver_used = b.solver;
  res->attempts = attempts;
  res->ir_steps = b.steps;
  res->gmres_iters = b.inner;
  for (int q = 0; q < 3; ++q) res->berr[q] = b.berr[q];
  res->berr_max = b.berr_max;
  res->ms_convert = last.ms_convert;
  res->ms_factor = last.ms_factor;
  res->ms_refine = last.ms_refine;
}

void d2d(Worker* w, double* dst, const double* src, int n) {
  if (dst && n > 0)
    LSQ_HIP(hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToDevice, w->stream));
}

// The ladder for one LSE instance on worker w (arguments already checked).
int lse_solve_core(Worker* w, int m, int n, int p, const double* A, int lda, const double* B,
                   int ldb, const double* b, const double* d, double* x, double* r, double* v,
                   const lsq_opts& o_in, lsq_result* res, const float* sel_w) {
  Ctx& ctx = w->ctx;
  LseArgs a{m, n, p, A, B, b, d, lda, ldb};
  double mx[4];
  float ms_convert = 0.0f;
  RungOut ro;
  if (!ingest(w, A, lda, m, n, B, ldb, p, n, b, m, d, p, mx, &ms_convert)) {
    ro.ms_convert = ms_convert;
    fill_result(res, 5, 0, 0, 0, ro);
    return 5;
  }
  double* xi = ctx.ws->get<double>(n > 0 ? n : 1);
  double* ri = ctx.ws->get<double>(m > 0 ? m : 1);
  double* vi = ctx.ws->get<double>(p > 0 ? p : 1);
  double* xb = ctx.ws->get<double>(n > 0 ? n : 1);
  double* rb = ctx.ws->get<double>(m > 0 ? m : 1);
  double* vb = ctx.ws->get<double>(p > 0 ? p : 1);
  BestIter best;
  best.save = [&]() { d2d(w, xb, xi, n); d2d(w, rb, ri, m); d2d(w, vb, vi, p); };
  lsq_opts o = o_in;
  LseSolver pre;
  bool have_pre = false;
  int pre_code = 0;
  if (sel_w && (o.prec == LSQ_PREC_AUTO || o.solver == LSQ_SOLVER_AUTO)) {
    pre_code = lse_prefactor(w, a, kSelFactorPrec, o, pre, mx);
    have_pre = true;
    const Selection sl = select_run(w, LSQ_LSE, m, n, p, pre.fb, p, pre.fa, n - p, n, sel_w);
    if (o.prec == LSQ_PREC_AUTO) o.prec = pre_code == 0 ? class_prec(sl.cls[0]) : LSQ_PREC_FP64;
    if (o.solver == LSQ_SOLVER_AUTO) o.solver = class_solver(sl.cls[1]);
  }
  const auto rungs = ladder(o);
  w->history.clear();
  int used_p = 0, used_s = 0, attempts = 0, info = 3;
  for (size_t ri_ = 0; ri_ < rungs.size(); ++ri_) {
    const int prec = rungs[ri_].first;
    const std::vector<int>& solvers = rungs[ri_].second;
    w->more_rungs = ri_ + 1 < rungs.size();
    ro = lse_rung(w, a, prec, solvers, o, xi, ri, vi, attempts, used_s, mx, &best,
                  have_pre ? &pre : nullptr, pre_code);
    used_p = prec;
    if (ro.breakdown && prec == LSQ_PREC_FP64) { info = ro.breakdown; break; }
    if (ro.ok) { info = 0; break; }
    if (ro.singular) { info = ro.singular; break; }
  }
  w->more_rungs = false;
  ro.ms_convert = ms_convert;
  if (info == 0) {
    d2d(w, x, xi, n); d2d(w, r, ri, m); d2d(w, v, vi, p);
    fill_result(res, info, used_p, used_s, attempts, ro);
  } else if (info == 3) {
    if (!best.have) {
      // no rung produced a finite iterate: return x = 0 (r = v = 0) with its
      // backward error
      vec_zero(ctx, xb, 8, n); vec_zero(ctx, rb, 8, m); vec_zero(ctx, vb, 8, p);
      double* f1 = ctx.ws->get<double>(m > 0 ? m : 1);
      double* f2 = ctx.ws->get<double>(p > 0 ? p : 1);
      double* f3 = ctx.ws->get<double>(n > 0 ? n : 1);
      lse_residual(ctx, m, n, p, A, lda, B, ldb, b, d, xb, rb, vb, f1, f2, f3, w->matnorms, o.tol,
                   w->st_dev);
      read_status(w);
      for (int q = 0; q < 3; ++q) best.berr[q] = w->st_host->berr[q];
      best.berr_max = w->st_host->berr_max;
      best.prec = used_p;
      best.solver = used_s;
    }
    d2d(w, x, xb, n); d2d(w, r, rb, m); d2d(w, v, vb, p);
    fill_best(res, attempts, best, ro);
  } else {
    fill_result(res, info, used_p, used_s, attempts, ro);
  }
  LSQ_HIP(hipStreamSynchronize(w->stream));
  return info;
}

int gls_solve_core(Worker* w, int n, int m, int p, const double* W, int ldw, const double* V,
                   int ldv, const double* d, double* x, double* y, double* z, const lsq_opts& o_in,
                   lsq_result* res, const float* sel_w) {
  Ctx& ctx = w->ctx;
  GlsArgs a{n, m, p, W, V, d, ldw, ldv};
  double mx[4];
  float ms_convert = 0.0f;
  RungOut ro;
  if (!ingest(w, W, ldw, n, m, V, ldv, n, p, d, n, nullptr, 0, mx, &ms_convert)) {
    ro.ms_convert = ms_convert;
    fill_result(res, 5, 0, 0, 0, ro);
    return 5;
  }
  double* xi = ctx.ws->get<double>(m > 0 ? m : 1);
  double* yi = ctx.ws->get<double>(p > 0 ? p : 1);
  double* zi = ctx.ws->get<double>(n > 0 ? n : 1);
  double* xb = ctx.ws->get<double>(m > 0 ? m : 1);
  double* yb = ctx.ws->get<double>(p > 0 ? p : 1);
  double* zb = ctx.ws->get<double>(n > 0 ? n : 1);
  BestIter best;
  best.save = [&]() { d2d(w, xb, xi, m); d2d(w, yb, yi, p); d2d(w, zb, zi, n); };
  lsq_opts o = o_in;
  GlsSolver pre;
  bool have_pre = false;
  int pre_code = 0;
  if (sel_w && (o.prec == LSQ_PREC_AUTO || o.solver == LSQ_SOLVER_AUTO)) {
    pre_code = gls_prefactor(w, a, kSelFactorPrec, o, pre, mx);
    have_pre = true;
    const Selection sl = select_run(w, LSQ_GLS, m, n, p, pre.fw, m, pre.fv, n - m, n, sel_w);
    if (o.prec == LSQ_PREC_AUTO) o.prec = pre_code == 0 ? class_prec(sl.cls[0]) : LSQ_PREC_FP64;
    if (o.solver == LSQ_SOLVER_AUTO) o.solver = class_solver(sl.cls[1]);
  }
  const auto rungs = ladder(o);
  w->history.clear();
  int used_p = 0, used_s = 0, attempts = 0, info = 3;
  for (size_t ri_ = 0; ri_ < rungs.size(); ++ri_) {
    const int prec = rungs[ri_].first;
    const std::vector<int>& solvers = rungs[ri_].second;
    w->more_rungs = ri_ + 1 < rungs.size();
    ro = gls_rung(w, a, prec, solvers, o, xi, yi, zi, attempts, used_s, mx, &best,
                  have_pre ? &pre : nullptr, pre_code);
    used_p = prec;
    if (ro.breakdown && prec == LSQ_PREC_FP64) { info = ro.breakdown; break; }
    if (ro.ok) { info = 0; break; }
    if (ro.singular) { info = ro.singular; break; }
  }
  w->more_rungs = false;
  ro.ms_convert = ms_convert;
  if (info == 0) {
    d2d(w, x, xi, m); d2d(w, y, yi, p); d2d(w, z, zi, n);
    fill_result(res, info, used_p, used_s, attempts, ro);
  } else if (info == 3) {
    if (!best.have) {
      vec_zero(ctx, xb, 8, m); vec_zero(ctx, yb, 8, p); vec_zero(ctx, zb, 8, n);
      double* f1 = ctx.ws->get<double>(p > 0 ? p : 1);
      double* f2 = ctx.ws->get<double>(n > 0 ? n : 1);
      double* f3 = ctx.ws->get<double>(m > 0 ? m : 1);
      gls_residual(ctx, n, m, p, W, ldw, V, ldv, d, xb, yb, zb, f1, f2, f3, w->matnorms, o.tol,
                   w->st_dev);
      read_status(w);
      for (int q = 0; q < 3; ++q) best.berr[q] = w->st_host->berr[q];
      best.berr_max = w->st_host->berr_max;
      best.prec = used_p;
      best.solver = used_s;
    }
    d2d(w, x, xb, m); d2d(w, y, yb, p); d2d(w, z, zb, n);
    fill_best(res, attempts, best, ro);
  } else {
    fill_result(res, info, used_p, used_s, attempts, ro);
  }
  LSQ_HIP(hipStreamSynchronize(w->stream));
  return info;
}

int lse_check(int m, int n, int p, const double* A, int lda, const double* B, int ldb,
              const double* b, const double* d, const double* x, std::string* why) {
  auto bad = [&](int code, const char* msg) { if (why) *why = msg; return code; };
  if (m < 0) return bad(-2, "m < 0");
  if (n < 0 || n > m + p) return bad(-3, "n out of range (p <= n <= m + p)");
  if (p < 0 || p > n) return bad(-4, "p out of range (p <= n)");
  if (!A && m * n > 0) return bad(-5, "A is null");
  if (lda < (m > 1 ? m : 1)) return bad(-6, "lda < max(1, m)");
  if (!B && p * n > 0) return bad(-7, "B is null");
  if (ldb < (p > 1 ? p : 1)) return bad(-8, "ldb < max(1, p)");
  if (!b && m > 0) return bad(-9, "b is null");
  if (!d && p > 0) return bad(-10, "d is null");
  if (!x && n > 0) return bad(-11, "x is null");
  return 0;
}

int gls_check(int n, int m, int p, const double* W, int ldw, const double* V, int ldv,
              const double* d, const double* x, const double* y, std::string* why) {
  auto bad = [&](int code, const char* msg) { if (why) *why = msg; return code; };
  if (n < 0) return bad(-2, "n < 0");
  if (m < 0 || m > n) return bad(-3, "m out of range (m <= n)");
  if (p < 0 || n > m + p) return bad(-4, "p out of range (n <= m + p)");
  if (!W && n * m > 0) return bad(-5, "W is null");
  if (ldw < (n > 1 ? n : 1)) return bad(-6, "ldw < max(1, n)");
  if (!V && n * p > 0) return bad(-7, "V is null");
  if (ldv < (n > 1 ? n : 1)) return bad(-8, "ldv < max(1, n)");
  if (!d && n > 0) return bad(-9, "d is null");
  if (!x && m > 0) return bad(-10, "x is null");
  if (!y && p > 0) return bad(-11, "y is null");
  return 0;
}
}  // namespace

// Factors kept across calls: the solver object and the arena that holds its
// factors and prepared structures; ctx is the handle's context with this
// arena (its stream is refreshed from the handle at every call).
struct lsq_factors_st {
  lsq_handle owner = nullptr;
  int device = 0;
  int type = 0;
  int prec = 0;
  int m = 0, n = 0, p = 0, lda = 1, ldb = 1;
  const double* A = nullptr;
  const double* B = nullptr;
  Arena arena;
  Ctx ctx;
  LseSolver lse;
  GlsSolver gls;
};

namespace {

// The refinement solvers a factored solve runs: FP64 factors give the FP64
// direct solve; otherwise classical IR (IR or AUTO) or GMRES-IR.
bool factored_solvers(int prec, int solver, std::vector<int>& out) {
  out.clear();
  if (prec == LSQ_PREC_FP64) { out.push_back(LSQ_SOLVER_DIRECT); return true; }
  if (solver == LSQ_SOLVER_AUTO || solver == LSQ_SOLVER_IR) { out.push_back(LSQ_SOLVER_IR); return true; }
  if (solver == LSQ_SOLVER_GMRES_IR) { out.push_back(LSQ_SOLVER_GMRES_IR); return true; }
  return false;   // DIRECT needs FP64 factors
}

void factors_free(lsq_factors f) {
  if (!f) return;
  (void)hipSetDevice(f->device);
  f->arena.release();
  delete f;
}

}  // namespace

extern "C" {

int lse_solve(lsq_handle h, int m, int n, int p, const double* A, int lda, const double* B,
              int ldb, const double* b, const double* d, double* x, double* r, double* v,
              const lsq_opts* opts, lsq_result* res) {
  if (!h) return -1;
  std::string why;
  const int bad = lse_check(m, n, p, A, lda, B, ldb, b, d, x, &why);
  if (bad) return fail(h, bad, why);
  lsq_opts o;
  lsq_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0) || o.maxit < 0) return fail(h, -14, "invalid options");
  return guard(h, "lse_solve", [&]() -> int {
    return lse_solve_core(&h->w, m, n, p, A, lda, B, ldb, b, d, x, r, v, o, res, h->sel_w);
  });
}

int gls_solve(lsq_handle h, int n, int m, int p, const double* W, int ldw, const double* V,
              int ldv, const double* d, double* x, double* y, double* z, const lsq_opts* opts,
              lsq_result* res) {
  if (!h) return -1;
  std::string why;
  const int bad = gls_check(n, m, p, W, ldw, V, ldv, d, x, y, &why);
  if (bad) return fail(h, bad, why);
  lsq_opts o;
  lsq_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0) || o.maxit < 0) return fail(h, -13, "invalid options");
  return guard(h, "gls_solve", [&]() -> int {
    return gls_solve_core(&h->w, n, m, p, W, ldw, V, ldv, d, x, y, z, o, res, h->sel_w);
  });
}

// Complex problems through their real embedding: the complex LSE with A
// (m x n), B (p x n) is the real LSE with [Re A, -Im A; Im A, Re A] (2m x 2n),
// the same embedding of B (2p x 2n) and b, d, x, r, v as [Re; Im] (the
// embedding of A^H is the transpose of A's, so the augmented system, its
// residual blocks and the solution carry over exactly); GLS likewise.  The
// stop test uses the complex Frobenius norms (the embedding's divided by
// sqrt(2)) and the vector norms, which the embedding keeps, so berr is that
// of the complex problem.
namespace {
struct ComplexNorms {
  Worker* w;
  explicit ComplexNorms(Worker* w_) : w(w_) { w->norm_scale = std::sqrt(0.5); }
  ~ComplexNorms() { w->norm_scale = 1.0; }
};
}  // namespace

int zlse_solve(lsq_handle h, int m, int n, int p, const double* A, int lda, const double* B,
               int ldb, const double* b, const double* d, double* x, double* r, double* v,
               const lsq_opts* opts, lsq_result* res) {
  if (!h) return -1;
  std::string why;
  const int bad = lse_check(m, n, p, A, lda, B, ldb, b, d, x, &why);
  if (bad) return fail(h, bad, why);
  lsq_opts o;
  lsq_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0) || o.maxit < 0) return fail(h, -14, "invalid options");
  return guard(h, "zlse_solve", [&]() -> int {
    Worker* w = &h->w;
    Ctx& ctx = w->ctx;
    const int M = 2 * m, N = 2 * n, P = 2 * p;
    auto buf = [&](size_t len) { return ctx.ws->get<double>(len > 0 ? len : 1); };
    double* Ae = buf((size_t)M * N);
    double* Be = buf((size_t)P * N);
    double *be = buf(M), *de = buf(P), *xe = buf(N), *re = buf(M), *ve = buf(P);
    embed_mat(ctx, A, lda, m, n, Ae);
    embed_mat(ctx, B, ldb, p, n, Be);
    embed_vec(ctx, b, m, be);
    embed_vec(ctx, d, p, de);
    int info;
    {
      ComplexNorms cn(w);
      info = lse_solve_core(w, M, N, P, Ae, M > 1 ? M : 1, Be, P > 1 ? P : 1, be, de, xe, re, ve, o,
                            res, h->sel_w);
    }
    if (info == 0 || info == 3) {
      unembed_vec(ctx, xe, n, x);
      unembed_vec(ctx, re, m, r);
      unembed_vec(ctx, ve, p, v);
      LSQ_HIP(hipStreamSynchronize(w->stream));
    }
    return info;
  });
}

int zgls_solve(lsq_handle h, int n, int m, int p, const double* W, int ldw, const double* V,
               int ldv, const double* d, double* x, double* y, double* z, const lsq_opts* opts,
               lsq_result* res) {
  if (!h) return -1;
  std::string why;
  const int bad = gls_check(n, m, p, W, ldw, V, ldv, d, x, y, &why);
  if (bad) return fail(h, bad, why);
  lsq_opts o;
  lsq_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0) || o.maxit < 0) return fail(h, -13, "invalid options");
  return guard(h, "zgls_solve", [&]() -> int {
    Worker* w = &h->w;
    Ctx& ctx = w->ctx;
    const int Nn = 2 * n, Mm = 2 * m, P = 2 * p;
    auto buf = [&](size_t len) { return ctx.ws->get<double>(len > 0 ? len : 1); };
    double* We = buf((size_t)Nn * Mm);
    double* Ve = buf((size_t)Nn * P);
    double *de = buf(Nn), *xe = buf(Mm), *ye = buf(P), *ze = buf(Nn);
    embed_mat(ctx, W, ldw, n, m, We);
    embed_mat(ctx, V, ldv, n, p, Ve);
    embed_vec(ctx, d, n, de);
    int info;
    {
      ComplexNorms cn(w);
      info = gls_solve_core(w, Nn, Mm, P, We, Nn > 1 ? Nn : 1, Ve, Nn > 1 ? Nn : 1, de, xe, ye, ze,
                            o, res, h->sel_w);
    }
    if (info == 0 || info == 3) {
      unembed_vec(ctx, xe, m, x);
      unembed_vec(ctx, ye, p, y);
      unembed_vec(ctx, ze, n, z);
      LSQ_HIP(hipStreamSynchronize(w->stream));
    }
    return info;
  });
}

int lsq_solve_batched(lsq_handle h, int count, const lsq_problem* probs, const lsq_opts* opts,
                      lsq_result* res) {
  if (!h) return -1;
  if (count < 0) return fail(h, -2, "count < 0");
  if (count > 0 && !probs) return fail(h, -3, "problem array is null");
  lsq_opts o;
  lsq_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0) || o.maxit < 0) return fail(h, -4, "invalid options");
  std::vector<double> work(count);
  for (int i = 0; i < count; ++i) {
    const lsq_problem& q = probs[i];
    std::string why;
    int bad;
    if (q.type == LSQ_LSE)
      bad = lse_check(q.m, q.n, q.p, q.A, q.lda, q.B, q.ldb, q.b, q.d, q.x, &why);
    else if (q.type == LSQ_GLS)
      bad = gls_check(q.n, q.m, q.p, q.A, q.lda, q.B, q.ldb, q.d, q.x, q.y, &why);
    else
      bad = -1, why = "unknown problem type";
    if (bad) return fail(h, -3, "instance " + std::to_string(i) + ": " + why);
    // factorization flops (Section 3 cost model, leading terms) for the LPT order
    const double m = q.m, n = q.n, p = q.p;
    work[i] = q.type == LSQ_LSE ? 2 * m * n * n + 4 * m * n * p + 2 * n * p * p
                                : 2 * n * m * m + 4 * n * m * p + 2 * p * n * n;
  }
  h->last_error.clear();
  if (count == 0) return 0;
  // longest instances first; each worker thread takes the next one
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  const bool persistent =
      (h->batch_mode == LSQ_BATCH_AUTO || h->batch_mode == LSQ_BATCH_SEQUENTIAL) &&
      (o.solver == LSQ_SOLVER_AUTO || o.solver == LSQ_SOLVER_IR || o.solver == LSQ_SOLVER_DIRECT) &&
      (o.prec == LSQ_PREC_FP32 || o.prec == LSQ_PREC_FP64 || o.prec == LSQ_PREC_BF16 ||
       (o.prec == LSQ_PREC_AUTO && !h->sel_w));
  if (persistent) {
    const int first = (o.prec == LSQ_PREC_FP64 || o.solver == LSQ_SOLVER_DIRECT) ? LSQ_PREC_FP64
                      : o.prec == LSQ_PREC_BF16                                 ? LSQ_PREC_BF16
                                                                                : LSQ_PREC_FP32;
    try {
      LSQ_HIP(hipSetDevice(h->device));
      order = batch_persistent(h, probs, order, o, first, res);
    } catch (const HipError& e) {
      return fail(h, 4, std::string("lsq_solve_batched: ") + e.where + " failed");
    }
    if (order.empty()) return 0;
  }
  const int todo = (int)order.size();
  const int nw = std::min(h->batch_workers, todo);
  try {
    LSQ_HIP(hipSetDevice(h->device));
    LSQ_HIP(hipStreamSynchronize(h->w.stream));     // inputs produced on the caller's stream
    while ((int)h->pool.size() < nw) {
      auto wp = std::make_unique<Worker>();
      wp->init(h->device, h->num_cu, true);
      h->pool.push_back(std::move(wp));
    }
  } catch (const HipError& e) {
    return fail(h, 4, std::string("lsq_solve_batched: ") + e.where + " failed");
  }
  std::atomic<int> next{0}, nfail{0};
  std::vector<std::string> errs(nw);
  for (auto& wp : h->pool) wp->ctx.deterministic = h->w.ctx.deterministic;
  auto run = [&](int t) {
    Worker* w = h->pool[t].get();
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= todo) break;
      const int i = order[k];
      const lsq_problem& q = probs[i];
      lsq_result* ri = res ? &res[i] : nullptr;
      const int info = guard_w(w, &errs[t], "lsq_solve_batched", [&]() -> int {
        if (q.type == LSQ_LSE)
          return lse_solve_core(w, q.m, q.n, q.p, q.A, q.lda, q.B, q.ldb, q.b, q.d, q.x, nullptr,
                                nullptr, o, ri, h->sel_w);
        return gls_solve_core(w, q.n, q.m, q.p, q.A, q.lda, q.B, q.ldb, q.d, q.x, q.y, nullptr, o,
                              ri, h->sel_w);
      });
      if (info != 0) {
        nfail.fetch_add(1);
        if (ri && info == 4) ri->info = 4;
      }
    }
  };
  std::vector<std::thread> threads;
  for (int t = 1; t < nw; ++t) threads.emplace_back(run, t);
  run(0);
  for (auto& th : threads) th.join();
  for (auto& e : errs)
    if (!e.empty()) { h->last_error = e; break; }
  return nfail.load();
}

int lsq_batch_plan_create(lsq_handle h, int count, const lsq_problem* probs, const lsq_opts* opts,
                          lsq_batch_plan* plan_out) {
  if (!h) return -1;
  if (!plan_out) return fail(h, -2, "plan pointer is null");
  *plan_out = nullptr;
  if (count <= 0 || !probs) return fail(h, -2, "empty problem set");
  lsq_opts o;
  lsq_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0) || o.maxit < 0) return fail(h, -4, "invalid options");
  if (o.prec != LSQ_PREC_FP32 || !(o.solver == LSQ_SOLVER_IR || o.solver == LSQ_SOLVER_AUTO) || !o.escalate)
    return fail(h, -5, "a plan captures the FP32 rung with escalation to FP64 (prec FP32, solver IR, escalate 1)");
  if (h->batch_mode != LSQ_BATCH_AUTO || !h->w.ctx.side)
    return fail(h, -5, "a plan needs the concurrent persistent batch mode");
  std::vector<double> work(count);
  for (int i = 0; i < count; ++i) {
    const lsq_problem& q = probs[i];
    std::string why;
    int bad;
    if (q.type == LSQ_LSE)
      bad = lse_check(q.m, q.n, q.p, q.A, q.lda, q.B, q.ldb, q.b, q.d, q.x, &why);
    else if (q.type == LSQ_GLS)
      bad = gls_check(q.n, q.m, q.p, q.A, q.lda, q.B, q.ldb, q.d, q.x, q.y, &why);
    else
      bad = -1, why = "unknown problem type";
    if (bad) return fail(h, -3, "instance " + std::to_string(i) + ": " + why);
    const BatchProb bp{q.type == LSQ_LSE ? 0 : 1, q.m, q.n, q.p, q.A, q.B, q.b, q.d, q.lda, q.ldb, q.x, q.y};
    if (!batch_eligible(bp))
      return fail(h, -5, "instance " + std::to_string(i) + " exceeds the persistent kernel's sizes");
    const double m = q.m, n = q.n, p = q.p;
    work[i] = q.type == LSQ_LSE ? 2 * m * n * n + 4 * m * n * p + 2 * n * p * p
                                : 2 * n * m * m + 4 * n * m * p + 2 * p * n * n;
  }
  auto plan = std::make_unique<lsq_batch_plan_st>();
  plan->h = h;
  plan->probs.assign(probs, probs + count);
  plan->opts = o;
  plan->order.resize(count);
  for (int i = 0; i < count; ++i) plan->order[i] = i;
  std::stable_sort(plan->order.begin(), plan->order.end(), [&](int a, int b) { return work[a] > work[b]; });
  const int rc = guard(h, "lsq_batch_plan_create", [&]() -> int {
    LSQ_HIP(hipSetDevice(h->device));
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    (void)batch_persistent(h, plan->probs.data(), plan->order, o, LSQ_PREC_FP32, nullptr, plan.get());
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    return 0;
  });
  if (rc != 0) {
    plan->release();
    return rc;
  }
  *plan_out = plan.release();
  return 0;
}

int lsq_batch_plan_run(lsq_batch_plan plan, lsq_result* res) {
  if (!plan || !plan->h || !plan->exec) return -1;
  lsq_handle h = plan->h;
  std::vector<int> rest;
  const int rc = guard(h, "lsq_batch_plan_run", [&]() -> int {
    LSQ_HIP(hipSetDevice(h->device));
    rest = batch_persistent(h, plan->probs.data(), plan->order, plan->opts, LSQ_PREC_FP32, res, plan);
    return 0;
  });
  if (rc != 0 || rest.empty()) return rc;
  // what neither rung certified goes through the worker ladder, as in
  // lsq_solve_batched
  std::vector<lsq_problem> sub;
  for (int i : rest) sub.push_back(plan->probs[i]);
  std::vector<lsq_result> subres(sub.size());
  const int mode = h->batch_mode;
  h->batch_mode = LSQ_BATCH_WORKERS;
  const int r2 = lsq_solve_batched(h, (int)sub.size(), sub.data(), &plan->opts, subres.data());
  h->batch_mode = mode;
  if (res)
    for (size_t k = 0; k < rest.size(); ++k) res[rest[k]] = subres[k];
  return r2;
}

int lsq_batch_plan_destroy(lsq_batch_plan plan) {
  if (!plan) return 0;
  if (plan->h) {
    (void)hipSetDevice(plan->h->device);
    (void)hipStreamSynchronize(plan->h->w.stream);
    if (plan->h->w.ctx.side) (void)hipStreamSynchronize(plan->h->w.ctx.side);
  }
  plan->release();
  delete plan;
  return 0;
}

int lsq_selector_set(lsq_handle h, const float* weights, int count) {
  if (!h) return -1;
  if (!weights) {
    if (h->sel_w) (void)hipFree(h->sel_w);
    h->sel_w = nullptr;
    return 0;
  }
  if (count != kSelWeights) return fail(h, -3, "selector weight count mismatch");
  for (int i = 0; i < count; ++i)
    if (!std::isfinite(weights[i])) return fail(h, -2, "non-finite selector weight");
  for (int i = 0; i < kSelFeatures; ++i)
    if (!(weights[kSelFeatures + i] > 0.0f)) return fail(h, -2, "feature scales must be positive");
  try {
    LSQ_HIP(hipSetDevice(h->device));
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    for (auto& wp : h->pool) LSQ_HIP(hipStreamSynchronize(wp->stream));
    if (!h->sel_w) LSQ_HIP(hipMalloc(&h->sel_w, sizeof(float) * kSelWeights));
    LSQ_HIP(hipMemcpy(h->sel_w, weights, sizeof(float) * kSelWeights, hipMemcpyHostToDevice));
  } catch (const HipError& e) {
    return fail(h, 4, std::string("lsq_selector_set: ") + e.where + " failed");
  }
  return 0;
}

int lsq_selector_features(lsq_handle h, const lsq_problem* q, float* feats, float* logits, int* cls) {
  if (!h) return -1;
  if (!q) return -2;
  if (!feats) return -3;
  std::string why;
  int bad;
  if (q->type == LSQ_LSE)
    bad = lse_check(q->m, q->n, q->p, q->A, q->lda, q->B, q->ldb, q->b, q->d, q->x, &why);
  else if (q->type == LSQ_GLS)
    bad = gls_check(q->n, q->m, q->p, q->A, q->lda, q->B, q->ldb, q->d, q->x, q->y, &why);
  else
    bad = -1, why = "unknown problem type";
  if (bad) return fail(h, -2, why);
  if ((logits || cls) && !h->sel_w) return fail(h, -4, "no selector weights set");
  lsq_opts o;
  lsq_opts_default(&o);
  return guard(h, "lsq_selector_features", [&]() -> int {
    Worker* w = &h->w;
    Selection sl;
    if (q->type == LSQ_LSE) {
      LseArgs a{q->m, q->n, q->p, q->A, q->B, q->b, q->d, q->lda, q->ldb};
      frob_norms(w->ctx, q->A, q->lda, q->m, q->n, q->B, q->ldb, q->p, q->n, q->b, q->m, q->d, q->p,
                 w->matnorms);
      LseSolver sv;
      lse_prefactor(w, a, kSelFactorPrec, o, sv, nullptr);
      sl = select_run(w, LSQ_LSE, q->m, q->n, q->p, sv.fb, q->p, sv.fa, q->n - q->p, q->n, h->sel_w);
    } else {
      GlsArgs a{q->n, q->m, q->p, q->A, q->B, q->d, q->lda, q->ldb};
      frob_norms(w->ctx, q->A, q->lda, q->n, q->m, q->B, q->ldb, q->n, q->p, q->d, q->n, nullptr, 0,
                 w->matnorms);
      GlsSolver sv;
      gls_prefactor(w, a, kSelFactorPrec, o, sv, nullptr);
      sl = select_run(w, LSQ_GLS, q->m, q->n, q->p, sv.fw, q->m, sv.fv, q->n - q->m, q->n, h->sel_w);
    }
    for (int i = 0; i < kSelFeatures; ++i) feats[i] = sl.feats[i];
    if (logits)
      for (int i = 0; i < kSelOut; ++i) logits[i] = sl.logits[i];
    if (cls) { cls[0] = sl.cls[0]; cls[1] = sl.cls[1]; }
    return 0;
  });
}

int lse_factor(lsq_handle h, int m, int n, int p, const double* A, int lda, const double* B,
               int ldb, int prec, lsq_factors* factors) {
  if (!h) return -1;
  std::string why;
  static const double nonnull = 0.0;   // stands in for the vectors the shared check requires
  const int bad = lse_check(m, n, p, A, lda, B, ldb, &nonnull, &nonnull, &nonnull, &why);
  if (bad) return fail(h, bad, why);
  PrecSpec ps;
  if (prec == LSQ_PREC_AUTO || !prec_spec(prec, ps)) return fail(h, -9, "invalid precision");
  if (!factors) return fail(h, -10, "factors is null");
  *factors = nullptr;
  lsq_factors f = new lsq_factors_st();
  f->owner = h; f->device = h->w.device; f->type = LSQ_LSE; f->prec = prec;
  f->m = m; f->n = n; f->p = p; f->A = A; f->lda = lda; f->B = B; f->ldb = ldb;
  const int rc = guard(h, "lse_factor", [&]() -> int {
    double mx[4];
    float ms = 0.0f;
    if (!ingest(&h->w, A, lda, m, n, B, ldb, p, n, nullptr, 0, nullptr, 0, mx, &ms)) return 5;
    f->ctx = h->w.ctx;
    f->ctx.ws = &f->arena;
    LseSolver& sv = f->lse;
    sv.m = m; sv.n = n; sv.p = p; sv.k = n - p; sv.prec_id = prec; sv.ps = ps;
    sv.sA = pow2_scale(mx[0]);
    sv.sB = pow2_scale(mx[1]);
    // the factorization's temporaries go to the handle's arena
    // no early preparation: every prepared structure then sits above the mark
    // taken below, so a switch of solver kind rewinds all of it
    sv.factor(f->ctx, A, lda, B, ldb, kMaxNb, 0, &h->w.arena);
    const int sb = read_int(&h->w, sv.fb.status);
    const int sa = read_int(&h->w, sv.fa.status);
    sv.pmark = f->arena.mark();
    sv.has_pmark = true;
    return (sb || sa) ? 1 : 0;
  });
  if (rc != 0) {
    factors_free(f);
    if (rc == 1) h->last_error = "lse_factor: a panel factorization broke down at this precision";
    if (rc == 5) h->last_error = "lse_factor: a non-finite value in A or B";
    return rc;
  }
  *factors = f;
  return 0;
}

int gls_factor(lsq_handle h, int n, int m, int p, const double* W, int ldw, const double* V,
               int ldv, int prec, lsq_factors* factors) {
  if (!h) return -1;
  std::string why;
  static const double nonnull = 0.0;   // stands in for the vectors the shared check requires
  const int bad = gls_check(n, m, p, W, ldw, V, ldv, &nonnull, &nonnull, &nonnull, &why);
  if (bad) return fail(h, bad, why);
  PrecSpec ps;
  if (prec == LSQ_PREC_AUTO || !prec_spec(prec, ps)) return fail(h, -9, "invalid precision");
  if (!factors) return fail(h, -10, "factors is null");
  *factors = nullptr;
  lsq_factors f = new lsq_factors_st();
  f->owner = h; f->device = h->w.device; f->type = LSQ_GLS; f->prec = prec;
  f->m = m; f->n = n; f->p = p; f->A = W; f->lda = ldw; f->B = V; f->ldb = ldv;
  const int rc = guard(h, "gls_factor", [&]() -> int {
    double mx[4];
    float ms = 0.0f;
    if (!ingest(&h->w, W, ldw, n, m, V, ldv, n, p, nullptr, 0, nullptr, 0, mx, &ms)) return 5;
    f->ctx = h->w.ctx;
    f->ctx.ws = &f->arena;
    GlsSolver& sv = f->gls;
    sv.n = n; sv.m = m; sv.p = p; sv.k = n - m; sv.prec_id = prec; sv.ps = ps;
    sv.sW = pow2_scale(mx[0]);
    sv.sV = pow2_scale(mx[1]);
    // no early preparation: every prepared structure then sits above the mark
    // taken below, so a switch of solver kind rewinds all of it
    sv.factor(f->ctx, W, ldw, V, ldv, kMaxNb, 0, &h->w.arena);
    const int sw = read_int(&h->w, sv.fw.status);
    const int sv_ = read_int(&h->w, sv.fv.status);
    sv.pmark = f->arena.mark();
    sv.has_pmark = true;
    return (sw || sv_) ? 1 : 0;
  });
  if (rc != 0) {
    factors_free(f);
    if (rc == 1) h->last_error = "gls_factor: a panel factorization broke down at this precision";
    if (rc == 5) h->last_error = "gls_factor: a non-finite value in W or V";
    return rc;
  }
  *factors = f;
  return 0;
}

}  // extern "C"

// Argument checks shared by the two factored LSE entry points (0 or -k).
static int lse_factored_check(lsq_handle h, lsq_factors f, const double* b, const double* d,
                              const double* x, const lsq_opts* opts, lsq_opts& o,
                              std::vector<int>& solvers) {
  if (!f || f->type != LSQ_LSE) return fail(h, -2, "factors are not LSE factors");
  if (f->owner != h) return fail(h, -2, "factors belong to another handle");
  if (!b && f->m > 0) return fail(h, -3, "b is null");
  if (!d && f->p > 0) return fail(h, -4, "d is null");
  if (!x && f->n > 0) return fail(h, -5, "x is null");
  lsq_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0) || o.maxit < 0 || !factored_solvers(f->prec, o.solver, solvers))
    return fail(h, -8, "invalid options");
  return 0;
}

// Refinement of one right-hand side on stored LSE factors, on the handle's
// worker; its per-call temporaries come from the worker context's workspace.
static int lse_factored_run(Worker* w, lsq_factors f, const double* b, const double* d, double* x,
                            double* r, double* v, const lsq_opts& o, const std::vector<int>& solvers,
                            lsq_result* res) {
  const int m = f->m, n = f->n, p = f->p;
  Ctx& ctx = w->ctx;
  Arena* keep = f->ctx.ws;
  f->ctx = w->ctx;                     // the handle's current stream and events
  f->ctx.ws = keep;
  f->lse.pctx = &f->ctx;
  LseArgs a{m, n, p, f->A, f->B, b, d, f->lda, f->ldb};
  double mx[4];
  float ms_convert = 0.0f;
  RungOut ro;
  if (!ingest(w, f->A, f->lda, m, n, f->B, f->ldb, p, n, b, m, d, p, mx, &ms_convert)) {
    ro.ms_convert = ms_convert;
    fill_result(res, 5, f->prec, 0, 0, ro);
    return 5;
  }
  double* xi = ctx.ws->get<double>(n > 0 ? n : 1);
  double* ri = ctx.ws->get<double>(m > 0 ? m : 1);
  double* vi = ctx.ws->get<double>(p > 0 ? p : 1);
  double* xb = ctx.ws->get<double>(n > 0 ? n : 1);
  double* rb = ctx.ws->get<double>(m > 0 ? m : 1);
  double* vb = ctx.ws->get<double>(p > 0 ? p : 1);
  BestIter best;
  best.save = [&]() { d2d(w, xb, xi, n); d2d(w, rb, ri, m); d2d(w, vb, vi, p); };
  int attempts = 0, used_s = 0;
  w->history.clear();
  ro = lse_rung(w, a, f->prec, solvers, o, xi, ri, vi, attempts, used_s, nullptr, &best, &f->lse, 0);
  ro.ms_factor = 0.0f;
  ro.ms_convert = ms_convert;
  const int info = ro.ok ? 0 : 3;
  if (info == 0 || !best.have) {
    d2d(w, x, xi, n); d2d(w, r, ri, m); d2d(w, v, vi, p);
    fill_result(res, info, f->prec, used_s, attempts, ro);
  } else {
    d2d(w, x, xb, n); d2d(w, r, rb, m); d2d(w, v, vb, p);
    fill_best(res, attempts, best, ro);
  }
  LSQ_HIP(hipStreamSynchronize(w->stream));
  return info;
}

// Bytes of the per-call workspace of a classical-IR solve on stored LSE
// factors: the ingest scan's partial sums, the iterates and best iterate, the
// residual blocks, one residual evaluation's partial sums (returned to the
// workspace after each evaluation; hi and lo parts with the double-double
// residual), the previous x of the double-double mode and the pivot check of
// an FP64 solve that did not certify.  Each piece is rounded up to the
// workspace's 256-byte granularity.
static size_t lse_factored_ws_bytes(int m, int n, int p) {
  auto piece = [](size_t elems) { const size_t b = 8 * (elems > 0 ? elems : 1); return (b + 255) & ~size_t(255); };
  auto cd = [](long long a, long long q) { return (a + q - 1) / q; };
  size_t t = piece(16 * 512);                                  // ingest
  t += 2 * (piece(n) + piece(m) + piece(p));                   // iterate, best iterate
  t += piece(m) + piece(p) + piece(n);                         // f1, f2, f3
  // A's and B's partial sums: the rung's FP64 residual workspace, and hi and
  // lo parts besides it when the residual is double-double
  t += 3 * (piece((size_t)cd(n, 64) * m) + piece((size_t)cd(m, 256) * n));
  t += 3 * (piece((size_t)cd(n, 64) * p) + piece((size_t)cd(p, 256) * n));
  t += piece(n);                                               // previous x (double-double mode)
  const int len = std::max(std::max(m, n), p);
  t += 2 * piece((size_t)cd(len, 256) * kNormSlots);           // norm partials
  t += 2 * piece(2);                                           // pivot check of FP64 triangles
  return t;
}

// Cap of the allocation-free workspace in bytes (<= kScratchBytes; lowered
// only by the inspection entry point that tests the size check).
static size_t g_noalloc_cap = kScratchBytes;

extern "C" {

int lse_solve_factored(lsq_handle h, lsq_factors f, const double* b, const double* d, double* x,
                       double* r, double* v, const lsq_opts* opts, lsq_result* res) {
  if (!h) return -1;
  lsq_opts o;
  std::vector<int> solvers;
  if (const int bad = lse_factored_check(h, f, b, d, x, opts, o, solvers)) return bad;
  return guard(h, "lse_solve_factored", [&]() -> int {
    return lse_factored_run(&h->w, f, b, d, x, r, v, o, solvers, res);
  });
}

int lse_solve_factored_noalloc(lsq_handle h, lsq_factors f, const double* b, const double* d,
                               double* x, double* r, double* v, const lsq_opts* opts,
                               lsq_result* res) {
  if (!h) return -1;
  lsq_opts o;
  std::vector<int> solvers;
  if (const int bad = lse_factored_check(h, f, b, d, x, opts, o, solvers)) return bad;
  if (solvers.size() != 1 || solvers[0] == LSQ_SOLVER_GMRES_IR)
    return fail(h, -8, "the allocation-free solve runs classical IR (or the FP64 direct solve) only");
  const int tc = f->prec == LSQ_PREC_FP64 ? 8 : f->lse.ps.tc;
  if (f->lse.prepared_tc != tc)
    return fail(h, -2, "the factors are not prepared for classical refinement: "
                       "solve once with lse_solve_factored (solver IR) first");
  const size_t need = lse_factored_ws_bytes(f->m, f->n, f->p);
  if (need > g_noalloc_cap)
    return fail(h, -2, "the factors need " + std::to_string(need) +
                           " bytes of workspace per solve, more than the " +
                           std::to_string(g_noalloc_cap) + " bytes of the static scratch buffer");
  void* ptr = scratch_ptr(h->w.device);
  if (!ptr) return fail(h, 4, "no scratch buffer was set up on this device");
  Worker* w = &h->w;
  Arena fixed;
  fixed.adopt_fixed(ptr, g_noalloc_cap);
  Arena* prev = w->ctx.ws;
  w->ctx.ws = &fixed;
  w->arena.set_frozen(true);
  f->arena.set_frozen(true);
  const bool graphs = w->step_graphs;
  w->step_graphs = false;              // instantiating a graph allocates
  const int rc = guard(h, "lse_solve_factored_noalloc", [&]() -> int {
    return lse_factored_run(w, f, b, d, x, r, v, o, solvers, res);
  });
  w->step_graphs = graphs;
  w->ctx.ws = prev;
  w->arena.set_frozen(false);
  f->arena.set_frozen(false);
  return rc;
}

int gls_solve_factored(lsq_handle h, lsq_factors f, const double* d, double* x, double* y,
                       double* z, const lsq_opts* opts, lsq_result* res) {
  if (!h) return -1;
  if (!f || f->type != LSQ_GLS) return fail(h, -2, "factors are not GLS factors");
  if (f->owner != h) return fail(h, -2, "factors belong to another handle");
  const int n = f->n, m = f->m, p = f->p;
  if (!d && n > 0) return fail(h, -3, "d is null");
  if (!x && m > 0) return fail(h, -4, "x is null");
  if (!y && p > 0) return fail(h, -5, "y is null");
  lsq_opts o;
  lsq_opts_default(&o);
  if (opts) o = *opts;
  std::vector<int> solvers;
  if (!(o.tol >= 0) || o.maxit < 0 || !factored_solvers(f->prec, o.solver, solvers))
    return fail(h, -7, "invalid options");
  return guard(h, "gls_solve_factored", [&]() -> int {
    Worker* w = &h->w;
    Ctx& ctx = w->ctx;
    Arena* keep = f->ctx.ws;
    f->ctx = w->ctx;
    f->ctx.ws = keep;
    f->gls.pctx = &f->ctx;
    GlsArgs a{n, m, p, f->A, f->B, d, f->lda, f->ldb};
    double mx[4];
    float ms_convert = 0.0f;
    RungOut ro;
    if (!ingest(w, f->A, f->lda, n, m, f->B, f->ldb, n, p, d, n, nullptr, 0, mx, &ms_convert)) {
      ro.ms_convert = ms_convert;
      fill_result(res, 5, f->prec, 0, 0, ro);
      return 5;
    }
    double* xi = ctx.ws->get<double>(m > 0 ? m : 1);
    double* yi = ctx.ws->get<double>(p > 0 ? p : 1);
    double* zi = ctx.ws->get<double>(n > 0 ? n : 1);
    double* xb = ctx.ws->get<double>(m > 0 ? m : 1);
    double* yb = ctx.ws->get<double>(p > 0 ? p : 1);
    double* zb = ctx.ws->get<double>(n > 0 ? n : 1);
    BestIter best;
    best.save = [&]() { d2d(w, xb, xi, m); d2d(w, yb, yi, p); d2d(w, zb, zi, n); };
    int attempts = 0, used_s = 0;
    w->history.clear();
    ro = gls_rung(w, a, f->prec, solvers, o, xi, yi, zi, attempts, used_s, nullptr, &best, &f->gls, 0);
    ro.ms_factor = 0.0f;
    ro.ms_convert = ms_convert;
    const int info = ro.ok ? 0 : 3;
    if (info == 0 || !best.have) {
      d2d(w, x, xi, m); d2d(w, y, yi, p); d2d(w, z, zi, n);
      fill_result(res, info, f->prec, used_s, attempts, ro);
    } else {
      d2d(w, x, xb, m); d2d(w, y, yb, p); d2d(w, z, zb, n);
      fill_best(res, attempts, best, ro);
    }
    LSQ_HIP(hipStreamSynchronize(w->stream));
    return info;
  });
}

int lsq_dbg_factors_bytes(lsq_factors f, long long* in_use, long long* capacity) {
  if (!f) return -1;
  if (in_use) *in_use = (long long)f->arena.in_use();
  if (capacity) *capacity = (long long)f->arena.capacity();
  return 0;
}

int lsq_dbg_noalloc_bytes(lsq_factors f, long long* need, long long* cap) {
  if (!f || f->type != LSQ_LSE) return -1;
  if (need) *need = (long long)lse_factored_ws_bytes(f->m, f->n, f->p);
  if (cap) *cap = (long long)g_noalloc_cap;
  return 0;
}

int lsq_dbg_noalloc_cap(long long bytes) {
  if (bytes < 0 || bytes > (long long)kScratchBytes) return -1;
  g_noalloc_cap = bytes == 0 ? kScratchBytes : (size_t)bytes;
  return 0;
}

int lsq_factors_destroy(lsq_factors f) {
  factors_free(f);
  return 0;
}

int lse_solve_batched(lsq_handle h, int count, const lsq_problem* probs, const lsq_opts* opts,
                      lsq_result* res) {
  for (int i = 0; i < count; ++i)
    if (!probs || probs[i].type != LSQ_LSE) return -3;
  return lsq_solve_batched(h, count, probs, opts, res);
}

int gls_solve_batched(lsq_handle h, int count, const lsq_problem* probs, const lsq_opts* opts,
                      lsq_result* res) {
  for (int i = 0; i < count; ++i)
    if (!probs || probs[i].type != LSQ_GLS) return -3;
  return lsq_solve_batched(h, count, probs, opts, res);
}

// ------------------------------------------------------------ debug ABI --
int lsq_dbg_qr(lsq_handle h, int prec, int r, int c, const double* M, int ldm, const double* X,
               int ldx, int nx, double* R, double* Y1, double* Y2, double* Y3) {
  if (!h) return -1;
  PrecSpec ps;
  if (!prec_spec(prec, ps)) return -2;
  if (r < 0) return -3;
  if (c < 0) return -4;
  if (!M || ldm < (r > 1 ? r : 1)) return -5;
  if (nx > 0 && (!X || ldx < r)) return -7;
  return guard(h, "lsq_dbg_qr", [&]() -> int {
    Ctx& ctx = h->w.ctx;
    QRFactor f;
    qr_alloc(ctx, f, r, c, ps.tw, ps.mt, kMaxNb);
    mat_convert(ctx, f.M, ps.tw, f.ld, M, 8, ldm, r, c, false, false, false);
    qr_factor(ctx, f);
    if (R && f.k > 0) {
      void* tmp = ctx.ws->alloc((size_t)8 * r * c);
      mat_convert(ctx, tmp, 8, r, f.M, ps.tw, f.ld, r, c, false, false, false);
      // keep the upper trapezoid of the first k rows
      std::vector<double> host((size_t)r * c);
      LSQ_HIP(hipMemcpyAsync(host.data(), tmp, host.size() * 8, hipMemcpyDeviceToHost, h->w.stream));
      LSQ_HIP(hipStreamSynchronize(h->w.stream));
      std::vector<double> rk((size_t)f.k * c, 0.0);
      for (int j = 0; j < c; ++j)
        for (int i = 0; i < f.k && i <= j; ++i) rk[i + (size_t)j * f.k] = host[i + (size_t)j * r];
      LSQ_HIP(hipMemcpyAsync(R, rk.data(), rk.size() * 8, hipMemcpyHostToDevice, h->w.stream));
    }
    if (nx > 0) {
      void* Xw = ctx.ws->alloc((size_t)ps.tw * r * nx);
      if (Y1) {
        mat_convert(ctx, Xw, ps.tw, r, X, 8, ldx, r, nx, false, false, false);
        qr_apply_left_T(ctx, f, Xw, r, nx);
        mat_convert(ctx, Y1, 8, r, Xw, ps.tw, r, r, nx, false, false, false);
      }
      if (Y2 || Y3) {
        agg_prepare(ctx, f, ps.tc, kAggPanels);
        void* col = ctx.ws->alloc((size_t)ps.tc * (r > 0 ? r : 1));
        for (int j = 0; j < nx; ++j) {
          vec_convert(ctx, col, ps.tc, X + (size_t)j * ldx, 8, r, false);
          agg_apply(ctx, f, true, col, ps.tc);
          if (Y2) vec_convert(ctx, Y2 + (size_t)j * r, 8, col, ps.tc, r, false);
          if (Y3) {
            agg_apply(ctx, f, false, col, ps.tc);
            vec_convert(ctx, Y3 + (size_t)j * r, 8, col, ps.tc, r, false);
          }
        }
      }
    }
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    int st = 0;
    LSQ_HIP(hipMemcpy(&st, f.status, sizeof(int), hipMemcpyDeviceToHost));
    return st ? 1 : 0;
  });
}

int lsq_dbg_trsv(lsq_handle h, int prec, int tc64, int n, const double* U, int ldu, int trans,
                 const double* b, double* x) {
  if (!h) return -1;
  PrecSpec ps;
  if (!prec_spec(prec, ps)) return -2;
  if (n < 0) return -4;
  if (!U || ldu < (n > 1 ? n : 1)) return -5;
  return guard(h, "lsq_dbg_trsv", [&]() -> int {
    Ctx& ctx = h->w.ctx;
    QRFactor f;
    f.r = f.c = f.k = n; f.ld = n > 1 ? n : 1; f.tw = ps.tw; f.mt = ps.mt;
    f.M = ctx.ws->alloc((size_t)ps.tw * f.ld * (n > 0 ? n : 1));
    mat_convert(ctx, f.M, ps.tw, f.ld, U, 8, ldu, n, n, false, false, false);
    const int tc = tc64 ? 8 : ps.tc;
    TriBlock tb;
    trsv_prepare(ctx, tb, f, 0, n, tc);
    void* w = ctx.ws->alloc((size_t)tc * (n > 0 ? n : 1));
    vec_convert(ctx, w, tc, b, 8, n, false);
    trsv(ctx, tb, trans != 0, w);
    vec_convert(ctx, x, 8, w, tc, n, false);
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    return 0;
  });
}

static void status_out(lsq_handle h, double* out) {
  read_status(&h->w);
  const StopStatus& s = *h->w.st_host;
  for (int q = 0; q < 3; ++q) {
    out[q] = s.nf[q];
    out[3 + q] = s.scale[q];
    out[6 + q] = s.berr[q];
  }
  out[9] = s.berr_max;
}

int lsq_dbg_lse_residual(lsq_handle h, int m, int n, int p, const double* A, int lda,
                         const double* B, int ldb, const double* b, const double* d,
                         const double* x, const double* r, const double* v, double* f1,
                         double* f2, double* f3, double* out) {
  if (!h) return -1;
  return guard(h, "lsq_dbg_lse_residual", [&]() -> int {
    Ctx& ctx = h->w.ctx;
    frob_norms(ctx, A, lda, m, n, B, ldb, p, n, b, m, d, p, h->w.matnorms);
    lse_residual(ctx, m, n, p, A, lda, B, ldb, b, d, x, r, v, f1, f2, f3, h->w.matnorms, 1e-14,
                 h->w.st_dev, h->dbg_dd);
    if (out) status_out(h, out);
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    return 0;
  });
}

int lsq_dbg_gls_residual(lsq_handle h, int n, int m, int p, const double* W, int ldw,
                         const double* V, int ldv, const double* d, const double* x,
                         const double* y, const double* z, double* f1, double* f2, double* f3,
                         double* out) {
  if (!h) return -1;
  return guard(h, "lsq_dbg_gls_residual", [&]() -> int {
    Ctx& ctx = h->w.ctx;
    frob_norms(ctx, W, ldw, n, m, V, ldv, n, p, d, n, nullptr, 0, h->w.matnorms);
    gls_residual(ctx, n, m, p, W, ldw, V, ldv, d, x, y, z, f1, f2, f3, h->w.matnorms, 1e-14,
                 h->w.st_dev, h->dbg_dd);
    if (out) status_out(h, out);
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    return 0;
  });
}

int lsq_dbg_step_graph(lsq_handle h, int on) {
  if (!h) return -1;
  h->w.step_graphs = on != 0;
  return 0;
}

int lsq_dbg_residual_dd(lsq_handle h, int on) {
  if (!h) return -1;
  h->dbg_dd = on != 0;
  return 0;
}

int lsq_dbg_lse_correction(lsq_handle h, int prec, int m, int n, int p, const double* A, int lda,
                           const double* B, int ldb, const double* f1, const double* f2,
                           const double* f3, double* dr, double* dv, double* dx) {
  if (!h) return -1;
  PrecSpec ps;
  if (!prec_spec(prec, ps)) return -2;
  if (m < 0 || n < 0 || p < 0 || p > n || n > m + p) return -3;
  return guard(h, "lsq_dbg_lse_correction", [&]() -> int {
    Ctx& ctx = h->w.ctx;
    LseSolver sv;
    sv.m = m; sv.n = n; sv.p = p; sv.k = n - p; sv.ps = ps;
    sv.factor(ctx, A, lda, B, ldb, kMaxNb);
    sv.prepare(ctx, ps.tc);
    vec_zero(ctx, dr, 8, m);
    vec_zero(ctx, dv, 8, p);
    vec_zero(ctx, dx, 8, n);
    sv.correct(ctx, f1, f2, f3, dx, dr, dv);
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    return 0;
  });
}

int lsq_dbg_gls_correction(lsq_handle h, int prec, int n, int m, int p, const double* W, int ldw,
                           const double* V, int ldv, const double* f1, const double* f2,
                           const double* f3, double* dy, double* dz, double* dx) {
  if (!h) return -1;
  PrecSpec ps;
  if (!prec_spec(prec, ps)) return -2;
  if (m < 0 || n < 0 || p < 0 || m > n || n > m + p) return -3;
  return guard(h, "lsq_dbg_gls_correction", [&]() -> int {
    Ctx& ctx = h->w.ctx;
    GlsSolver sv;
    sv.n = n; sv.m = m; sv.p = p; sv.k = n - m; sv.ps = ps;
    sv.factor(ctx, W, ldw, V, ldv, kMaxNb);
    sv.prepare(ctx, ps.tc);
    vec_zero(ctx, dy, 8, p);
    vec_zero(ctx, dz, 8, n);
    vec_zero(ctx, dx, 8, m);
    sv.correct(ctx, f1, f2, f3, dx, dy, dz);
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    return 0;
  });
}

// ------------------------------------------------------------- timing --
static const char* const kKernelNames[kKCount] = {"panel_final_y", "panel_cholpass", "wy_t", "wy_u",
                                                  "dual_gemv", "batch_fp32", "batch_fp64", "agg_gemv",
                                                  "batch_esc"};

int lsq_dbg_timer_enable(lsq_handle h, const char* kernel) {
  if (!h) return -1;
  return guard(h, "lsq_dbg_timer_enable", [&]() -> int {
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    h->timer.used = 0;
    h->timer.flops = h->timer.bytes = 0.0;
    h->timer.target = -1;
    h->w.ctx.timer = nullptr;
    if (!kernel || !kernel[0]) return 0;
    for (int k = 0; k < kKCount; ++k)
      if (std::strcmp(kernel, kKernelNames[k]) == 0) h->timer.target = k;
    if (h->timer.target < 0) return fail(h, -2, std::string("unknown kernel name ") + kernel);
    h->w.ctx.timer = &h->timer;
    return 0;
  });
}

int lsq_dbg_timer_read(lsq_handle h, double* total_ms, int* launches, double* flops, double* bytes) {
  if (!h) return -1;
  return guard(h, "lsq_dbg_timer_read", [&]() -> int {
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    double tot = 0.0;
    for (int q = 0; q < h->timer.used; ++q) {
      float ms = 0.0f;
      LSQ_HIP(hipEventElapsedTime(&ms, h->timer.ev[2 * q], h->timer.ev[2 * q + 1]));
      tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = h->timer.used;
    if (flops) *flops = h->timer.flops;
    if (bytes) *bytes = h->timer.bytes;
    h->timer.used = 0;
    h->timer.flops = h->timer.bytes = 0.0;
    return 0;
  });
}

int lsq_dbg_copy(lsq_handle h, void* dst, const void* src, long long bytes) {
  if (!h) return -1;
  if (bytes < 0) return -4;
  if (bytes > 0 && (!dst || !src)) return -2;
  return guard(h, "lsq_dbg_copy", [&]() -> int {
    dev_copy(h->w.ctx, dst, src, (size_t)bytes);
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    return 0;
  });
}

// ------------------------------------------------- preconditioned operator --
int lsq_dbg_bd_apply_graph(lsq_handle h, int type, int prec, int m, int n, int p, const double* A,
                           int lda, const double* B, int ldb, double alpha, double beta,
                           const double* U, double* Y, int k, int* graph_used) {
  if (!h) return -1;
  if (type != LSQ_LSE && type != LSQ_GLS) return -2;
  PrecSpec ps;
  if (!prec_spec(prec, ps)) return -3;
  if (type == LSQ_LSE && !(p <= n && n <= m + p)) return -4;
  if (type == LSQ_GLS && !(m <= n && n <= m + p)) return -4;
  if (!(alpha > 0) || !(beta > 0)) return -11;
  if (k < 0) return -15;
  return guard(h, "lsq_dbg_bd_apply_graph", [&]() -> int {
    Ctx& ctx = h->w.ctx;
    bool used = false;
    if (type == LSQ_LSE) {
      LseSolver sv;
      sv.m = m; sv.n = n; sv.p = p; sv.k = n - p; sv.ps = ps;
      LseArgs a{m, n, p, A, B, nullptr, nullptr, lda, ldb};
      sv.factor(ctx, A, lda, B, ldb, kMaxNb);
      ensure_prepared(sv, ctx, 8, true);
      sv.alpha = alpha; sv.beta = beta; sv.sa = std::sqrt(alpha);
      std::function<void(const double*, double*)> op = [&](const double* u, double* y) {
        sv.m_right(ctx, u, sv.t1);
        sv.f_apply(ctx, a, sv.t1, sv.t2);
        sv.m_left(ctx, sv.t2, y);
      };
      graph_apply_columns(ctx, m + p + n, op, U, Y, k, &used);
    } else {
      GlsSolver sv;
      sv.n = n; sv.m = m; sv.p = p; sv.k = n - m; sv.ps = ps;
      GlsArgs a{n, m, p, A, B, nullptr, lda, ldb};
      sv.factor(ctx, A, lda, B, ldb, kMaxNb);
      ensure_prepared(sv, ctx, 8, true);
      sv.alpha = alpha; sv.beta = beta; sv.sa = std::sqrt(alpha);
      std::function<void(const double*, double*)> op = [&](const double* u, double* y) {
        sv.m_right(ctx, u, sv.t1);
        sv.f_apply(ctx, a, sv.t1, sv.t2);
        sv.m_left(ctx, sv.t2, y);
      };
      graph_apply_columns(ctx, p + n + m, op, U, Y, k, &used);
    }
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    if (graph_used) *graph_used = used ? 1 : 0;
    return 0;
  });
}

int lsq_dbg_bd_apply(lsq_handle h, int type, int prec, int m, int n, int p, const double* A, int lda,
                     const double* B, int ldb, double alpha, double beta, const double* u,
                     double* y) {
  if (!h) return -1;
  if (type != LSQ_LSE && type != LSQ_GLS) return -2;
  PrecSpec ps;
  if (!prec_spec(prec, ps)) return -3;
  if (type == LSQ_LSE && !(p <= n && n <= m + p)) return -4;
  if (type == LSQ_GLS && !(m <= n && n <= m + p)) return -4;
  if (!(alpha > 0) || !(beta > 0)) return -11;
  return guard(h, "lsq_dbg_bd_apply", [&]() -> int {
    Ctx& ctx = h->w.ctx;
    if (type == LSQ_LSE) {
      LseSolver sv;
      sv.m = m; sv.n = n; sv.p = p; sv.k = n - p; sv.ps = ps;
      LseArgs a{m, n, p, A, B, nullptr, nullptr, lda, ldb};
      sv.factor(ctx, A, lda, B, ldb, kMaxNb);
      ensure_prepared(sv, ctx, 8, true);
      sv.alpha = alpha; sv.beta = beta; sv.sa = std::sqrt(alpha);
      sv.m_right(ctx, u, sv.t1);
      sv.f_apply(ctx, a, sv.t1, sv.t2);
      sv.m_left(ctx, sv.t2, y);
    } else {
      GlsSolver sv;
      sv.n = n; sv.m = m; sv.p = p; sv.k = n - m; sv.ps = ps;
      GlsArgs a{n, m, p, A, B, nullptr, lda, ldb};
      sv.factor(ctx, A, lda, B, ldb, kMaxNb);
      ensure_prepared(sv, ctx, 8, true);
      sv.alpha = alpha; sv.beta = beta; sv.sa = std::sqrt(alpha);
      sv.m_right(ctx, u, sv.t1);
      sv.f_apply(ctx, a, sv.t1, sv.t2);
      sv.m_left(ctx, sv.t2, y);
    }
    LSQ_HIP(hipStreamSynchronize(h->w.stream));
    return 0;
  });
}

}  // extern "C"
