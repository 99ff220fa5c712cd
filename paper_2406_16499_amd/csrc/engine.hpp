// Host-side interfaces between liblsq's HIP translation units.
#pragma once
#include <initializer_list>
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <vector>
#include "common.hpp"

namespace lsq {

// ------------------------------------------------------------ workspace --
// Bump allocator over device chunks.  reset() rewinds without freeing, so a
// handle reuses the same memory across solves.  Pointers stay valid until the
// next reset().
class Arena {
 public:
  ~Arena();
  void* alloc(size_t bytes);
  template <typename T> T* get(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
  void reset();
  void release();
  // Position of the next allocation; rewind(mark) frees everything allocated
  // after it (the memory stays with the arena for reuse).
  struct Mark { size_t chunk = 0, used = 0; };
  Mark mark() const;
  void rewind(const Mark& m);
  size_t capacity() const;   // bytes held in chunks
  size_t in_use() const;     // bytes handed out since the last reset / rewind
  // Fixed mode: the arena hands out memory from [base, base + bytes) only,
  // which it does not own (release() leaves it alone), and an allocation that
  // does not fit throws instead of allocating a new chunk.
  void adopt_fixed(void* base, size_t bytes);
  // Frozen: every allocation throws (a caller that must not allocate).
  void set_frozen(bool f) { frozen_ = f; }
  bool frozen() const { return frozen_; }
  size_t high_water() const { return high_; }   // largest in_use() seen
 private:
  struct Chunk { char* base; size_t size; size_t used; bool owned; };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0;
  bool fixed_ = false, frozen_ = false;
  size_t high_ = 0;
};

// Optional timing of one kernel kind: HIP events on the context stream around
// each launch of that kind, with the launch's algorithmic flops and bytes.
enum KernelKind : int {
  kKPanelFinal = 0, kKPanelCholPass = 1, kKWyT = 2, kKWyU = 3, kKDualGemv = 4, kKBatch32 = 5,
  kKBatch64 = 6, kKAggGemv = 7, kKBatchEsc = 8, kKCount = 9
};
struct KernelTimer {
  int target = -1;
  std::vector<hipEvent_t> ev;   // 2 per launch
  int used = 0;                 // launches recorded
  double flops = 0.0, bytes = 0.0;
};

constexpr int kPinDoubles = 8192;   // size of the pinned host scratch of a context

struct Ctx {
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;        // second stream for look-ahead updates (null: none)
  Arena* ws = nullptr;
  int num_cu = 256;
  KernelTimer* timer = nullptr;
  double* pin = nullptr;             // pinned host scratch (kPinDoubles)
  std::vector<hipEvent_t>* events = nullptr;   // pool of timing-free events
  // Look-ahead in the blocked QR (next panel's columns first, the rest on the
  // side stream).  Off by default: the concurrent trailing updates take the
  // compute units the latency-bound panel kernels need, and the overlap
  // gains about 2% (6.27 vs 6.39 ms for the 4096 x 2048 FP32 factorization).
  bool lookahead = false;
  // Bitwise reproducible results: every sum that FP64 atomics would
  // accumulate in arrival order (panel Grams, skinny GEMVs) is formed in a
  // fixed order instead, at some cost in launches and traffic.
  bool deterministic = false;
};
// The i-th event of the context's pool (created on first use).
hipEvent_t ctx_event(Ctx& ctx, int i);

// Brackets one launch of kind `kind`; does nothing unless the timer targets it.
void ktimer_begin(Ctx& ctx, int kind, double flops, double bytes);
void ktimer_end(Ctx& ctx, int kind);
// The same on stream s (a launch on the side stream).
void ktimer_begin_on(Ctx& ctx, int kind, hipStream_t s, double flops, double bytes);
void ktimer_end_on(Ctx& ctx, int kind, hipStream_t s);
// Work of launches of kind `kind` known only once they have run.
void ktimer_add(Ctx& ctx, int kind, double flops, double bytes);

// ---------------------------------------------- Householder QR engine ----
// Aggregated compact-WY block over the panels starting at J0 (w columns):
// H = I - Y T Y^T with T (w x w, upper) = (striu(Y^T Y) + diag(Y^T Y) / 2)^{-1}.
struct AggBlock {
  int J0 = 0, w = 0;
  void* T = nullptr;            // w x w, column-major, compute precision
  size_t acc = 0;               // offset (elements) of the block's accumulators in agg_acc
};

// Blocked Householder QR of an r x c column-major matrix stored in Tw
// (float or double), k = min(r, c) reflectors in panels of nb columns.
// After factorization: R on and above the diagonal of M, the unit lower
// trapezoidal Householder vectors Y below it, and per panel the upper
// triangular T_j of the compact-WY form H_j = I - Y_j T_j Y_j^T, so that
// Q = H_0 H_1 ... H_{np-1}.
struct QRFactor {
  int r = 0, c = 0, k = 0, ld = 0, nb = 64, np = 0;
  int tw = 4;                   // sizeof(Tw): 4 (float) or 8 (double)
  int passes = 3;               // Cholesky QR passes per panel (3 for fp64, 2 otherwise)
  Mma mt = Mma::F32;
  void* M = nullptr;            // r x c, ld
  void* T = nullptr;            // np blocks of 64 x 64 (Tw), column-major ld 64
  void* Yhat = nullptr;         // per panel (r - j0) x 64 (Tw): Y_j T_j^T
  std::vector<size_t> yoff;     // element offset of panel j in Yhat
  int* status = nullptr;        // device: bit0 = a panel Cholesky broke down
  std::vector<AggBlock> agg;    // aggregated blocks for vector application
  int agg_tc = 0;
  // accumulators of the aggregated application, s = Y^T y (w) and t = op(T) s
  // (w) per block in compute precision; zero between applications
  void* agg_acc = nullptr;
  size_t agg_acc_len = 0;
};

void qr_alloc(Ctx& ctx, QRFactor& f, int r, int c, int tw, Mma mt, int nb);
void qr_factor(Ctx& ctx, QRFactor& f);
// C <- Q^T C for a column-major r x ncols matrix C (same Tw as the factor).
void qr_apply_left_T(Ctx& ctx, const QRFactor& f, void* C, int ldc, int ncols);

// Aggregated application: prepare blocks of `panels_per_block` panels (the
// Gram Y^T Y in FP64, T by triangular inversion) in compute precision tc, then
// y <- Q^T y (trans) or Q y with three parallel kernels per block and one
// fill that clears the accumulators after the last block.
void agg_prepare(Ctx& ctx, QRFactor& f, int tc, int panels_per_block);
void agg_apply(Ctx& ctx, const QRFactor& f, bool trans, void* y, int tc);
// Dense inverse X (nn x nn, ld nn, precision tc) of the upper triangular
// block f.M[o:o+nn, o:o+nn]; y = X x or X^T x.
void tri_inverse_factor(Ctx& ctx, const QRFactor& f, int o, int nn, void* X, int tc);
// y += op(X) x for a dense upper triangular X (nn x nn); y is not cleared.
void trmv_acc(Ctx& ctx, const void* X, int nn, bool trans, const void* x, void* y, int tc);

// ----------------------------------------------------- vector kernels ----
// Triangular solve with the upper triangular block U = f.M[o:o+nn, o:o+nn]:
// x <- U^{-1} x (trans = false) or U^{-T} x (trans = true), Tc precision,
// as a product with the inverse computed once by trsv_prepare.
struct TriBlock {
  const QRFactor* f = nullptr;
  int o = 0, nn = 0;
  void* inv = nullptr;          // nn x nn dense inverse (Tc)
  void* tmp = nullptr;          // nn (Tc), zero between solves
  int tc = 4;
};
void trsv_prepare(Ctx& ctx, TriBlock& tb, const QRFactor& f, int o, int nn, int tc);
void trsv(Ctx& ctx, const TriBlock& tb, bool trans, void* x);

// y[0:nr] += alpha * op(U) x, U = f.M[ro:ro+nr, co:co+nc] read with the upper
// mask of the factor (entries below its diagonal are zero); op(U) = U or U^T
// (for trans, y has length nc and x length nr).  Tc precision.
void gemv_upper(Ctx& ctx, const QRFactor& f, int ro, int co, int nr, int nc, bool trans,
                double alpha, const void* x, void* y, int tc);

// Elementwise helpers (n elements).  Types by size: 4 float, 8 double.
void vec_convert(Ctx& ctx, void* dst, int td, const void* src, int ts, int n, bool reverse,
                 double scale = 1.0);
void vec_axpy(Ctx& ctx, void* y, int ty, double a, const void* x, int tx, int n, bool reverse_x);
void vec_zero(Ctx& ctx, void* y, int ty, int n);
// dst = src, then src = 0 (same type t, n elements, no overlap).
void vec_move(Ctx& ctx, void* dst, void* src, int t, int n);

// Dense FP64 matrix -> Tw copy with optional transpose and index reversal:
// dst (dr x dc, ld ldd) [i][j] = scale * src[ri][ci] where (ri, ci) = trans ? (j, i) : (i, j),
// then ri, ci reversed when rev_r / rev_c (relative to src's own extents).
void mat_convert(Ctx& ctx, void* dst, int td, int ldd, const void* src, int ts, int lds,
                 int dr, int dc, bool trans, bool rev_rows_src, bool rev_cols_src,
                 double scale = 1.0);
// Multiplies the triangular factor of f (the entries on and above the
// diagonal of its first k rows) by s: undoes the power-of-two scale a matrix
// was factored with (exact in binary floating point).
void scale_upper(Ctx& ctx, QRFactor& f, double s);
// out[0] = min |diag|, out[1] = max |diag| of f.M[o:o+nn, o:o+nn] (synchronizes).
void diag_minmax(Ctx& ctx, const QRFactor& f, int o, int nn, double* out);

// ------------------------------------------------- FP64 residual sweep ----
// One pass over a column-major FP64 matrix M (rows x cols) yielding partial
// sums of M u (per column block) and M^T w (per row block).
struct DualParts {
  double* rowp = nullptr;  int ncb = 0;   // ncb x rows
  double* colp = nullptr;  int nrb = 0;   // nrb x cols
};
// Partial-sum buffers for a rows x cols matrix; dual_gemv allocates them
// itself when out.rowp is null, else reuses them (same shape required).
void dual_parts_alloc(Ctx& ctx, int rows, int cols, DualParts& out);
void dual_gemv(Ctx& ctx, const double* M, int ld, int rows, int cols, const double* u,
               const double* w, DualParts& out);

// Device status of the stop test (eq. lse-stop / eq. gls-stop).
struct StopStatus {
  double nf[3];       // ||f_i||
  double scale[3];    // right-hand sides without tol
  double berr[3];
  double berr_max;
  int converged;
  int nonfinite;
};
// Norm accumulation slots used by the residual kernels.
constexpr int kNormSlots = 12;

// Workspace of one FP64 residual evaluation, allocated once by the caller
// (for evaluations captured into a graph, whose addresses must stay fixed):
// the partial products of both matrices and the norm partials.
struct ResidualScratch {
  DualParts p1, p2;
  double* normp = nullptr;
};
// rows x cols of the two matrices of an LSE (A m x n, B p x n) or GLS
// (W n x m, V n x p) residual.
void residual_scratch_alloc(Ctx& ctx, int r1, int c1, int r2, int c2, int len, ResidualScratch& rs);

void lse_residual(Ctx& ctx, int m, int n, int p, const double* A, int lda, const double* B,
                  int ldb, const double* b, const double* d, const double* x, const double* r,
                  const double* v, double* f1, double* f2, double* f3, const double* matnorms,
                  double tol, StopStatus* st, bool dd = false, ResidualScratch* rs = nullptr);
void gls_residual(Ctx& ctx, int n, int m, int p, const double* W, int ldw, const double* V,
                  int ldv, const double* d, const double* x, const double* y, const double* z,
                  double* f1, double* f2, double* f3, const double* matnorms, double tol,
                  StopStatus* st, bool dd = false, ResidualScratch* rs = nullptr);
// dd: the residual in double-double (u_r = u^2) instead of FP64.  rs
// (FP64 only): preallocated workspace instead of the context's arena.
// matnorms[0..1] = ||A||_F, ||B||_F; matnorms[2..3] = ||b||, ||d|| (LSE) or ||d||, 0 (GLS);
// matnorms[4..7] = the largest magnitudes of the same four inputs, NaN for an
// input that holds a non-finite value.  Norms are exact to rounding over the
// whole FP64 range (no overflow or underflow of the squares).
// Plain copy of `bytes` bytes (16-byte vector loads/stores; calibration kernel).
void dev_copy(Ctx& ctx, void* dst, const void* src, size_t bytes);

void frob_norms(Ctx& ctx, const double* A, int lda, int ar, int ac, const double* B, int ldb,
                int br, int bc, const double* v1, int n1, const double* v2, int n2,
                double* matnorms);

// ------------------------------------------------------- complex data ----
// Real embedding of complex data (interleaved (re, im) pairs, column-major,
// ld in complex elements): E (2 rows x 2 cols, ld 2 rows) = [Re M, -Im M;
// Im M, Re M]; vectors as [Re u; Im u].  unembed_vec writes the interleaved
// vector back (nothing for a null u).
void embed_mat(Ctx& ctx, const double* M, int ld, int rows, int cols, double* E);
void embed_vec(Ctx& ctx, const double* u, int n, double* e);
void unembed_vec(Ctx& ctx, const double* e, int n, double* u);
// v[0:n] *= s (n <= 64)
void scale_first(Ctx& ctx, double* v, int n, double s);

// ------------------------------------------------------- FP64 Krylov ----
// One FP64 vector segment of vec_segs: dst[i] = c (a src[j] + b src2[j]),
// j = n - 1 - i if rev else i, the src2 term only for j >= lo, a null source
// contributing 0 (both null: a zero fill).  A reversed segment may not write
// over its sources.
struct VecSeg {
  double* dst;
  const double* src;
  const double* src2;
  int n, rev, lo;
  double a, b, c;
};
constexpr int kVecSegs = 6;
struct VecSegs {
  VecSeg s[kVecSegs];
  int count;
};
// Up to kVecSegs independent segments in one launch (segments with n <= 0
// are skipped).
void vec_segs(Ctx& ctx, std::initializer_list<VecSeg> segs);
inline VecSeg seg_copy(double* dst, const double* src, int n, bool rev = false, double c = 1.0) {
  return VecSeg{dst, src, nullptr, n, rev ? 1 : 0, 0, 1.0, 0.0, c};
}
inline VecSeg seg_zero(double* dst, int n) { return VecSeg{dst, nullptr, nullptr, n, 0, 0, 0.0, 0.0, 1.0}; }
// dst[i] = c (src[j] + b [j >= lo] src2[j])
inline VecSeg seg_add(double* dst, const double* src, const double* src2, int n, bool rev, int lo,
                      double b = 1.0, double c = 1.0) {
  return VecSeg{dst, src, src2, n, rev ? 1 : 0, lo, 1.0, b, c};
}
// Arguments of one combine (below); combine3 runs three in one launch.
struct CombineArgs {
  double* out;
  int n;
  double c0;
  const double* x0;
  double c1;
  const double* p1;
  int np1;
  double c2;
  const double* p2;
  int np2;
};
void combine3(Ctx& ctx, const CombineArgs& a0, const CombineArgs& a1, const CombineArgs& a2);
// out[i] = c0 x0[i] + c1 sum_q p1[q][i] + c2 sum_q p2[q][i] (null terms skipped),
// the parts being the partial products left by dual_gemv.
void combine(Ctx& ctx, double* out, int n, double c0, const double* x0, double c1, const double* p1,
             int np1, double c2, const double* p2, int np2);
double dev_norm2(Ctx& ctx, const double* x, int n);                 // synchronizes
double min_abs_diag(Ctx& ctx, const QRFactor& f, int o, int nn);   // synchronizes
// max |cur - old| / max |cur| over n elements (synchronizes; inf for NaN)
double rel_change(Ctx& ctx, const double* old, const double* cur, int n);

struct GmresOut {
  int iters = 0;
  bool converged = false;
  bool graph = false;          // the operator ran as a replayed HIP graph
  // the rate of the last restart cycle predicts more iterations than the
  // budget has left (only when give_up was set): GMRES stopped early
  bool hopeless = false;
};
// Restarted GMRES from x = 0 for apply(u) = M u (FP64, CGS2, Givens on the
// host).  With use_graph, apply (which must not synchronize the host) is
// captured once and replayed per iteration.  give_up: stop after a restart
// cycle whose residual reduction, extrapolated at the same rate, would not
// reach tol within maxit iterations.
GmresOut gmres(Ctx& ctx, int N, const std::function<void(const double*, double*)>& apply,
               const double* rhs, double* x, int restart, double tol, int maxit,
               bool use_graph = true, bool give_up = false);
// Y[:, j] = M U[:, j], j < k, by replays of the captured operator graph.
void graph_apply_columns(Ctx& ctx, int N, const std::function<void(const double*, double*)>& apply,
                         const double* U, double* Y, int k, bool* graph_used);

// ------------------------------------------------------------ selector ----
constexpr int kSelFeatures = 16, kSelHidden = 64, kSelOut = 7, kSelPrec = 5;
constexpr int kSelWeights = 2 * kSelFeatures + kSelHidden * kSelFeatures + kSelHidden +
                            kSelHidden * kSelHidden + kSelHidden + kSelOut * kSelHidden + kSelOut;
// out[0..2] = log10 max |d_i|, log10 min |d_i|, mean log10 |d_i| of diag f.M[o:o+nn, o:o+nn]
void diag_stats(Ctx& ctx, const QRFactor& f, int o, int nn, float* out);
void features(Ctx& ctx, int type, int m, int n, int p, const double* matnorms, const float* st1,
              const float* st2, const float* st3, float* feats);
// logits (7) and cls = {precision class 0..4, solver class 0..1}
void mlp_select(Ctx& ctx, const float* weights, const float* feats, float* logits, int* cls);

// ------------------------------------------------- persistent batch ----
// One instance of the persistent batched solver (type 0 = LSE with
// (m, n, p, A = A, B = B, b, d, x); type 1 = GLS with (n, m, p, A = W, B = V,
// d, x, y)).  Pointers are device pointers to FP64 column-major data.
constexpr int kBatchMaxDim = 1024;       // largest m, n, p of an instance
struct BatchProb {
  int type, m, n, p;
  const double *A, *B, *b, *d;
  int lda, ldb;
  double *x, *y;
};
struct BatchOut {
  int info;          // 0 converged, 3 no convergence, 5 non-finite iterate
  int steps;         // corrections after the initial solve
  double berr[3];
  double berr_max;
  // device wall clock (wall_clock64 ticks) when the work-group took the
  // instance, when its factorization was done and when its refinement ended
  unsigned long long t0, t1, t2;
};
// Device workspace bytes of one work-group for instance P (either precision).
size_t batch_ws_bytes(const BatchProb& P);
bool batch_eligible(const BatchProb& P);
// Resident work-groups per compute unit of the launch with element size tw.
int batch_blocks_per_cu(int tw);
// Householder flops of the factorization of instance P (the algorithmic work
// the kernel timer reports for a batch launch).
double batch_factor_flops(const BatchProb& P);
// One persistent launch over order[0:count) (indices into probs, device
// arrays); tw = 4 (FP32 factors and corrections) or 8 (FP64).  counter: one
// device int; ws: grid * ws_stride bytes; flops: algorithmic work of the
// launch, for the kernel timer.  fast_exit: a higher-precision rung follows,
// so an instance whose refinement contracts too slowly stops early, and one
// whose triangles show a diagonal ratio above route (> 0) skips refinement.
// lowp (tw = 4): the BF16 factorization (trailing updates and the
// application of the first factorization's Q^T with BF16 MFMA inputs).
void batch_launch(Ctx& ctx, int tw, const BatchProb* probs, const int* order, int count,
                  int* counter, char* ws, size_t ws_stride, int grid, double tol, int maxit, double polish,
                  bool fast_exit, double route, BatchOut* out, double flops, bool lowp = false);

// Escalation queues of the concurrent FP32 -> FP64 batch: the FP32 launch
// appends each instance that fails to queue 1 if it is among the first
// big_count of the order (the longest), else to queue 0, and counts every
// finished instance in done; an FP64 launch on the side stream takes slots
// from the heads, queue 1 first.  Device layout: this header, then per queue
// int slot[count], int ready[count] (all zero before the launches).
struct EscQueue {
  int tail[2], head[2], done, pad[3];
};
size_t esc_queue_bytes(int count);
// FP32 launch of `grid` work-groups over order[0:count) (as batch_launch,
// tw = 4, fast exit on) that pushes its failures to q; beside it on ctx.side
// an FP64 launch of grid64a work-groups, on the compute units the FP32 grid
// leaves free, solves the queued instances into out64 as they arrive, and
// grid64b more join after the FP32 launch (workspace ws64: grid64a +
// grid64b slots).  out64.info = -1 where an instance was not taken: a
// consumer that finds the queue empty for spin_ms while the FP32 launch is
// still running leaves, and the host runs what is left.  started (pinned
// host int, nullable): the consumers count themselves there and the FP32
// launch waits up to 20 ms for all grid64a of them.  big_count: see
// EscQueue.  pre: the first pre entries of the order go to the FP64 launch
// directly (queue 1, before any failure), and the FP32 launch starts after
// them.  lowp: the first launch factors in BF16 (as batch_launch).
// ctx.stream waits for all three launches.
void batch_launch_escalating(Ctx& ctx, const BatchProb* probs, const int* order, int count,
                             int* counter, char* ws, size_t ws_stride, int grid, char* ws64,
                             int grid64a, int grid64b, EscQueue* q, double tol, int maxit, double polish, double route,
                             BatchOut* out, BatchOut* out64, double flops, double spin_ms,
                             int* started, int big_count, int pre, bool lowp = false);
// The same sequence in a form a stream capture can record: fill kernels
// instead of memsets, the wait for the grid64a consumers on the device
// (started: a device int the consumers count themselves in, bounded at
// 20 ms), no kernel timer.  The FP32 results go to out, the FP64 ones to
// out64 (info -1: not taken).
void batch_capture_escalating(Ctx& ctx, const BatchProb* probs, const int* order, int count, int* counter,
                              char* ws, size_t ws_stride, int grid, char* ws64, int grid64a, int grid64b,
                              EscQueue* q, double tol, int maxit, double polish, double route, BatchOut* out,
                              BatchOut* out64, double spin_ms, int* started, int big_count, int pre);

}  // namespace lsq
