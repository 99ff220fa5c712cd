/*
 * lsq_debug.h -- inspection entry points of liblsq, one per step of the
 * refinement path, so that each step can be checked against an independent
 * implementation.  Same conventions as lsq.h: FP64 column-major device
 * buffers owned by the caller, work on the handle's stream, the call
 * synchronizes that stream before returning.  Return 0, -k for argument k,
 * or 4 for a HIP error.  `prec` is an lsq_prec value naming the storage /
 * MFMA precision of the factorization (Section 3, u_f).
 */
#ifndef LSQ_DEBUG_H
#define LSQ_DEBUG_H
#include "lsq.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Householder QR of M (r x c, assumption on xGEQRF of Section 4.1) at
 * precision prec.  Outputs, all FP64:
 *   R    (k x c, ld k, k = min(r,c)): the triangular factor (zeros below);
 *   Y1   (r x nx, ld r): Q^T X computed by the blocked matrix kernels;
 *   Y2   (r x nx, ld r): Q^T X computed column by column by the vector kernel;
 *   Y3   (r x nx, ld r): Q (Q^T X), both by the vector kernel.
 * Any output pointer may be NULL; X may be NULL when nx = 0. */
int lsq_dbg_qr(lsq_handle h, int prec, int r, int c, const double* M, int ldm,
               const double* X, int ldx, int nx, double* R, double* Y1, double* Y2, double* Y3);

/* Triangular solve with the upper triangle of U (n x n): x = U^{-1} b or
 * U^{-T} b (trans = 1), with U stored at precision prec and solved in FP32
 * (prec != FP64) or FP64 (prec = FP64); tc64 = 1 forces FP64 arithmetic. */
int lsq_dbg_trsv(lsq_handle h, int prec, int tc64, int n, const double* U, int ldu, int trans,
                 const double* b, double* x);

/* FP64 augmented residual of eq. aug-LSE at (x, r, v) and the stop-test
 * quantities of eq. lse-stop: out[0..2] = ||f_i||, out[3..5] = the right-hand
 * sides without tol, out[6..8] = blockwise backward errors, out[9] = their max
 * (host array of 10). */
int lsq_dbg_lse_residual(lsq_handle h, int m, int n, int p, const double* A, int lda,
                         const double* B, int ldb, const double* b, const double* d,
                         const double* x, const double* r, const double* v, double* f1,
                         double* f2, double* f3, double* out);

/* Same for eq. aug-GLS at (x, y, z) and eq. gls-stop (A = W, B = V). */
int lsq_dbg_gls_residual(lsq_handle h, int n, int m, int p, const double* A, int lda,
                         const double* B, int ldb, const double* d, const double* x,
                         const double* y, const double* z, double* f1, double* f2, double* f3,
                         double* out);

/* on = 0: classical refinement on the handle's stream runs each step kernel
 * by kernel instead of replaying it as a captured HIP graph (the default,
 * on != 0).  For comparing the two executions. */
int lsq_dbg_step_graph(lsq_handle h, int on);

/* on != 0: the two residual inspection entry points above evaluate the
 * residual in double-double (the opts->residual = 1 path), else in FP64. */
int lsq_dbg_residual_dd(lsq_handle h, int on);

/* Generalized RQ factorization of (B, A) at precision prec, then one call of
 * the LSE correction solver (Algorithm 1) on (f1, f2, f3): outputs dr (m),
 * dv (p), dx (n) with [[I,0,A],[0,0,B],[A^T,B^T,0]] [dr; -dv; dx] = f. */
int lsq_dbg_lse_correction(lsq_handle h, int prec, int m, int n, int p, const double* A, int lda,
                           const double* B, int ldb, const double* f1, const double* f2,
                           const double* f3, double* dr, double* dv, double* dx);

/* Generalized QR factorization of (W, V) = (A, B) at precision prec, then one
 * call of the GLS correction solver (Algorithm 3): outputs dy (p), dz (n),
 * dx (m) with [[I,V^T,0],[V,0,W],[0,W^T,0]] [dy; -dz; dx] = f. */
int lsq_dbg_gls_correction(lsq_handle h, int prec, int n, int m, int p, const double* A, int lda,
                           const double* B, int ldb, const double* f1, const double* f2,
                           const double* f3, double* dy, double* dz, double* dx);

/* The block-diagonal split-preconditioned operator of GMRES-IR applied to one
 * vector: y = M_l F~ M_r u (FP64 arithmetic) with the factors computed at
 * precision prec.  LSE (type LSQ_LSE, A m x n, B p x n): eq. lse-bdpre-mlarge
 * for m >= n, eq. lse-bdpre-nlarge for n > m; u and y of length m + p + n
 * ordered [r-block; v-block; x-block].  GLS (type LSQ_GLS, A = W n x m,
 * B = V n x p): eq. gls-bdpre-plarge for n <= p, eq. gls-bdpre-nlarge for
 * n > p; length p + n + m ordered [y; z; x].  alpha, beta > 0 are the
 * scalings of the augmented system (Section 5.1).  Returns -4 when the
 * problem's shape rule fails (LSE p <= n <= m + p, GLS m <= n <= m + p). */
int lsq_dbg_bd_apply(lsq_handle h, int type, int prec, int m, int n, int p, const double* A, int lda,
                     const double* B, int ldb, double alpha, double beta, const double* u,
                     double* y);

/* The same operator captured once as a HIP graph and replayed for each of
 * the k columns of U (N x k, column-major, N the augmented size): Y[:, j] =
 * M_l F~ M_r U[:, j].  The copies into and out of the graph's buffers run
 * eagerly between replays.  *graph_used (nullable) is 1 if the capture
 * succeeded (else the operator ran kernel by kernel).  Returns -15 for k < 0. */
int lsq_dbg_bd_apply_graph(lsq_handle h, int type, int prec, int m, int n, int p, const double* A,
                           int lda, const double* B, int ldb, double alpha, double beta,
                           const double* U, double* Y, int k, int* graph_used);

/* Kernel timing.  While enabled, HIP events are recorded on the stream of
 * every launch of the named kernel kind ("panel_final_y", "panel_cholpass",
 * "wy_t", "wy_u", "dual_gemv", and "batch_fp32" / "batch_fp64" for the
 * persistent batched solver, "batch_esc" for the launches of its concurrent
 * FP64 rung, "agg_gemv" for the two reflector-block GEMVs of each block of an
 * aggregated application of Q) around it, and the launch's algorithmic flops
 * and bytes are added up (the step each kernel carries out is the one cited
 * at its launch site: Householder QR panels and updates of Section 4.1, the
 * residual of eq. aug-LSE / eq. aug-GLS; for a batch launch the Householder
 * flops of the factorizations of the instances it solved).  NULL or "" disables; an unknown
 * name returns -2.  lsq_dbg_timer_read synchronizes the stream, returns the
 * summed event durations (ms), the launch count and the summed flops and
 * bytes since the last enable or read, and resets those counters.  Any output
 * pointer may be NULL. */
int lsq_dbg_timer_enable(lsq_handle h, const char* kernel);
int lsq_dbg_timer_read(lsq_handle h, double* total_ms, int* launches, double* flops, double* bytes);

/* Device-to-device copy of `bytes` bytes by a plain streaming kernel (16-byte
 * loads and stores), synchronized.  A calibration kernel of known traffic
 * for hardware byte counters; returns -4 for bytes < 0, -2 for a NULL
 * pointer with bytes > 0. */
int lsq_dbg_copy(lsq_handle h, void* dst, const void* src, long long bytes);

/* Bound (ms, default 50) on how long an FP64 work-group of the concurrent
   persistent batch waits for the FP32 launch to queue an instance; past it
   the work-group leaves, and the FP64 work-groups launched after the FP32
   launch (then the host, for anything still queued) solve the rest.  0 makes
   the early work-groups leave as soon as the queue is empty.  Returns -2
   outside [0, 1000]. */
int lsq_dbg_batch_wait(lsq_handle h, double ms);

/* Deterministic mode (1) or the default (0).  By default the panel Grams
   and the skinny GEMVs of the corrections add partial sums with FP64 atomics,
   so the last bits of a result depend on the order in which work-groups
   finish.  In the deterministic mode every such sum is formed in a fixed
   order (one Gram copy per row tile, summed in order; GEMV column blocks
   launched one after another), and the same input on the same device gives
   bitwise identical output from lse_solve, gls_solve, the complex and
   factored variants and the batched workers.  The persistent batched kernel
   is not covered.  Returns -2 outside 0..1. */
int lsq_dbg_deterministic(lsq_handle h, int on);

/* Per-step record of the last solve on the handle's own stream (lse_solve,
   gls_solve, the complex and factored variants; not the batched entry
   points): for step i < min(returned count, max_steps), berr[3 i .. 3 i + 2]
   = the three block backward errors of eq. lse-stop / gls-stop after that
   step, and (if rung is not NULL) rung[3 i .. 3 i + 2] = the precision and
   solver (lsq_prec, lsq_solver) of the rung and, for GMRES-IR, the inner
   iterations so far.  Steps of every rung the ladder ran are listed in
   order.  Returns the number of steps recorded, -2 for max_steps < 0 or a
   NULL berr with max_steps > 0. */
int lsq_dbg_history(lsq_handle h, int max_steps, double* berr, int* rung);

/* Route of the persistent batch's FP32 rung: when the FP64 rung follows, an
   instance whose FP32 triangles (R of B and T11 for the LSE, R of W and the
   leading (n - m) block of the second triangle for the GLS) show a largest to
   smallest diagonal magnitude ratio above `ratio` goes to the FP64 rung
   without refining.  0 turns the route off.  Returns -2 for a negative or
   NaN ratio. */
int lsq_dbg_batch_route(lsq_handle h, double ratio);

/* Share of the compute units on which the concurrent FP64 rung of the
   persistent batch starts beside the FP32 launch (default 0.25; the FP32
   launch takes the rest, and every unit joins the FP64 rung once the FP32
   launch ends).  Returns -2 outside (0, 1). */
int lsq_dbg_batch_split(lsq_handle h, double fp64_share);

/* Longest instances of the concurrent persistent batch (the head of its
   longest-first order), per work-group of the FP64 rung, that the rung solves
   in FP64 from the start (default 0; rounded to a count, at most 7/8 of the batch).
   The largest instances take about as long in FP32 as in FP64 on one
   work-group, so one that escalates would put both attempts on the launch's
   critical path.  Such an instance reports one attempt.  Returns -2 outside
   [0, 8]. */
int lsq_dbg_batch_pre(lsq_handle h, double per_wg);

/* The escalation fraction of the handle's last FP32-first persistent batch
   (the regime lsq_batch_tuning's esc_max compares against; 1 before any).
   Returns -2 for a NULL pointer. */
int lsq_dbg_batch_regime(lsq_handle h, double* last_escalation);

/* Schedule of the last persistent batched call (lsq_solve_batched and the
   typed variants, persistent modes), from the device wall clock: for each of
   the first `count` problems of that call, out[6 i .. 6 i + 5] = start,
   factored and end (ms from the earliest start) of its FP32 attempt, then of
   its FP64 attempt; NaN where an attempt did not run on the persistent path
   (or for i beyond that call).  Factored is the end of the conversions and
   the factorization; the refinement, initial solve included, runs from there
   to the end.  Returns -2 for count < 0 or a NULL out with count > 0. */
int lsq_dbg_batch_timeline(lsq_handle h, int count, double* out);

/* Device memory of a factors object (lse_factor / gls_factor): bytes in use
   and bytes held.  Returns -1 for NULL. */
int lsq_dbg_factors_bytes(lsq_factors factors, long long* in_use, long long* capacity);

/* Workspace of lse_solve_factored_noalloc: *need (nullable) receives the
   bytes one call on these factors takes from the static scratch array, *cap
   (nullable) the bytes the entry point accepts.  lsq_dbg_noalloc_cap lowers
   that cap to `bytes` (0 < bytes <= 64 MiB; 0 restores 64 MiB) so that the
   size check can be exercised on small problems; -1 outside that range. */
int lsq_dbg_noalloc_bytes(lsq_factors factors, long long* need, long long* cap);
int lsq_dbg_noalloc_cap(long long bytes);

/* Look-ahead of the blocked QR on the handle's factorizations: 0 off (the
   default), 1 the trailing updates after the next panel's columns on the
   side stream, overlapping the next panel.  -2 outside 0..1. */
int lsq_dbg_lookahead(lsq_handle h, int mode);

/* Text of the last error recorded on the handle ("" if none). */
const char* lsq_last_error(lsq_handle h);

#ifdef __cplusplus
}
#endif
#endif /* LSQ_DEBUG_H */
