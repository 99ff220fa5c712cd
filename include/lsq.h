/*
 * lsq.h -- C ABI of liblsq: mixed-precision iterative refinement for
 * equality-constrained least squares (LSE) and generalized least squares
 * (GLS) on AMD Instinct MI355X (gfx950).
 *
 * Method: Gao, Ma, Shao, "Mixed precision iterative refinement for least
 * squares with linear equality constraints and generalized least squares
 * problems" (arXiv 2406.16499).  The generalized RQ (LSE) or generalized QR
 * (GLS) factorization runs in a low precision u_f; the solution is then
 * refined on the 3-block augmented system with residuals in FP64 (Section 3),
 * either by classical refinement (Algorithms 2 and 4, correction solvers
 * Algorithms 1 and 3) or by GMRES with the block-diagonal split
 * preconditioners (Section 5: eq. lse-bdpre-mlarge / eq. lse-bdpre-nlarge
 * for LSE, eq. gls-bdpre-plarge / eq. gls-bdpre-nlarge for GLS, which
 * together cover every admissible shape).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrices and vectors are FP64, column-major, in GPU device memory.
 *   The caller owns every buffer; inputs are never modified (unlike LAPACK's
 *   xGGLSE / xGGGLM, which overwrite their inputs).
 * - Work is queued on the handle's stream (lsq_set_stream).  When a
 *   lsq_result pointer is given, the call synchronizes that stream once at
 *   the end to fill it.  Refinement decisions need the stop test on the
 *   host, so every solve synchronizes the stream at least once per
 *   refinement step.
 * - Return codes (LAPACK-style INFO):
 *      0   success: the returned iterate passes the stopping test with tol;
 *     -k   argument k is invalid (shape rule, leading dimension, null pointer);
 *      1   rank(B) < p (LSE) or rank(W) < m (GLS) (assumptions eq. assump:lse /
 *          eq. assump:gls): the FP64 factorization of B (LSE) or W (GLS) broke
 *          down, or the FP64 rung did not meet tol and that triangle R has a
 *          pivot ratio min|r_ii| / max|r_ii| <= 16 * 2^-53;
 *      2   T11 (LSE) or T22 (GLS) is singular, i.e. rank([A; B]) < n (LSE) or
 *          rank([W, V]) < n (GLS), the uniqueness condition of Section 1: the
 *          same two tests on the second FP64 factorization;
 *      3   no rung of the escalation ladder met tol; the iterate with the
 *          smallest backward error over all rungs is returned and its
 *          backward error reported (x = 0 and the backward error of x = 0 if
 *          no rung produced a finite iterate);
 *      4   HIP error or device allocation failure;
 *      5   a non-finite value (NaN or infinity) in A, B, b or d; nothing is
 *          factored and the outputs are not written.
 *   Outputs are written for codes 0 and 3 only.  A low-precision
 *   factorization never returns 1 or 2: near-singularity at u_f escalates to
 *   the next rung instead.
 * - Input scaling: every factorization works on its two matrices each
 *   scaled by the power of two that brings its largest magnitude into
 *   [1/2, 1), and scales the triangular factors back (exact in binary
 *   floating point).  The FP16 and BF16 MFMA inputs rounded from them stay
 *   inside the 16-bit range (Section 6.1 asks for scaling on the conversion
 *   to a lower precision), and the panels' Gram matrices cannot overflow.
 *   FP8 MFMA inputs are in addition scaled per tile.  The stop test's norms
 *   of A, B, b, d are exact to rounding over the whole FP64 range; those of
 *   the iterates are plain sums of squares (magnitudes up to about 1e150).
 * - Thread safety: a handle is used by one host thread at a time.
 */
#ifndef LSQ_H
#define LSQ_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsq_handle_st* lsq_handle;

/* Factorization precision u_f (Section 3: u_f >= u_s >= u >= u_r). */
typedef enum {
  LSQ_PREC_AUTO = 0,    /* learned selector when weights are set, else FP32      */
  LSQ_PREC_FP8E4M3 = 1, /* OCP e4m3 MFMA inputs, per-tile power-of-two scales */
  LSQ_PREC_BF16 = 2,    /* bf16 MFMA inputs, FP32 accumulation                    */
  LSQ_PREC_FP16 = 3,    /* fp16 MFMA inputs, FP32 accumulation                    */
  LSQ_PREC_FP32 = 4,    /* fp32 MFMA                                               */
  LSQ_PREC_FP64 = 5     /* fp64 MFMA: the all-FP64 direct path                     */
} lsq_prec;

typedef enum {
  LSQ_SOLVER_AUTO = 0,
  LSQ_SOLVER_IR = 1,       /* classical refinement, Algorithms 2 / 4              */
  LSQ_SOLVER_GMRES_IR = 2, /* GMRES with the block-diagonal split preconditioner */
  LSQ_SOLVER_DIRECT = 3    /* FP64 factorization + null-space / Paige solve,      */
                           /* certified by one FP64 residual evaluation           */
} lsq_solver;

typedef struct {
  int prec;            /* lsq_prec                                                  */
  int solver;          /* lsq_solver                                                */
  double tol;          /* threshold of eq. lse-stop / eq. gls-stop; default 1e-14   */
  int maxit;           /* refinement steps per rung; default 40 (Algorithms 2, 4)   */
  int gmres_restart;   /* default 30                                                */
  double gmres_tol;    /* inner relative tolerance of GMRES; default 1e-10          */
  int gmres_maxit;     /* total inner iterations per rung; default 300              */
  int escalate;        /* 1: on failure climb the ladder ending in FP64 direct      */
  double alpha, beta;  /* GMRES scaling (Section 5); <= 0 selects alpha = ||r0||    */
                       /* (LSE) or ||y0|| (GLS) and beta = 1                        */
  int nb;              /* panel width of the blocked factorization; 0 = default     */
  double polish;       /* after the stop test passes, one more correction while the */
                       /* backward error is above polish, toward the limiting       */
                       /* accuracy (forward error ~ cond u); default 8 * 2^-53;     */
                       /* <= 0 stops at once, as Algorithms 2 and 4 do              */
  int residual;        /* 0: FP64 residual (u_r = u, default); 1: double-double     */
                       /* residual (u_r = u^2, Table 2's extra-precise rows): the   */
                       /* refinement then goes on after the stop test passes while  */
                       /* the corrections change x (GLS: x and y) by more than 2u   */
                       /* relative and keep at least halving, so the forward error  */
                       /* reaches O(u) independently of the condition number        */
} lsq_opts;

typedef struct {
  int info;            /* as the return code                                        */
  int prec_used;       /* lsq_prec of the rung that produced the returned iterate   */
  int solver_used;     /* lsq_solver of that rung                                   */
  int attempts;        /* rungs tried                                               */
  int ir_steps;        /* corrections applied on the final rung                     */
  int gmres_iters;     /* total GMRES iterations on the final rung                  */
  double berr[3];      /* ||f_i|| / (right-hand side of the stop test without tol)  */
  double berr_max;
  /* stream time per phase: ms_convert the FP64 norm / magnitude / finiteness
     scan of the inputs (the down-conversions run inside the factorization and
     count in ms_factor); ms_factor and ms_refine those of the final rung     */
  float ms_convert, ms_factor, ms_refine;
} lsq_result;

/* Create a handle bound to GPU `device`; it owns a device workspace that grows
   on demand and is freed by lsq_destroy.  Returns 0 or 4. */
int lsq_create(lsq_handle* handle, int device);
int lsq_destroy(lsq_handle handle);
/* Queue all later work on `stream` (a hipStream_t; NULL = the default stream). */
int lsq_set_stream(lsq_handle handle, void* stream);
/* The defaults above (FP32 factorization, classical IR, tol 1e-14, the
   escalation ladder), each overridable from the environment for runs that
   cannot change the caller: LSQ_PREC (auto, fp8, bf16, fp16, fp32, fp64),
   LSQ_SOLVER (auto, ir, gmres, direct), LSQ_TOL (>= 0), LSQ_MAXIT (integer
   >= 0), LSQ_GMRES_MAXIT (integer >= 1), LSQ_ESCALATE (0 or 1), LSQ_RESIDUAL
   (0 or 1).  A value that does not parse or lies outside its range is
   ignored.  Needs no GPU. */
void lsq_opts_default(lsq_opts* opts);

/*
 * LSE (problem lse, Section 1):  min ||A x - b||_2  s.t.  B x = d,
 *   A: m x n (lda >= max(1,m)), B: p x n (ldb >= max(1,p)), b: m, d: p,
 *   with p <= n <= m + p.  Outputs: x (n); optionally r = b - A x (m) and the
 *   multiplier v (p) of eq. aug-LSE (pass NULL to skip).
 * Argument numbers for -k: 2 m, 3 n, 4 p, 5 A, 6 lda, 7 B, 8 ldb, 9 b, 10 d,
 * 11 x, 14 opts.
 */
int lse_solve(lsq_handle handle, int m, int n, int p,
              const double* A, int lda, const double* B, int ldb,
              const double* b, const double* d,
              double* x, double* r, double* v,
              const lsq_opts* opts, lsq_result* res);

/*
 * GLS (problem gls, Section 1):  min ||y||_2  s.t.  d = A x + B y,
 *   A = W: n x m (lda >= max(1,n)), B = V: n x p (ldb >= max(1,n)), d: n,
 *   with m <= n <= m + p.  Outputs: x (m), y (p); optionally the multiplier
 *   z (n) of eq. aug-GLS.
 * Argument numbers for -k: 2 n, 3 m, 4 p, 5 A, 6 lda, 7 B, 8 ldb, 9 d,
 * 10 x, 11 y, 13 opts.
 */
int gls_solve(lsq_handle handle, int n, int m, int p,
              const double* A, int lda, const double* B, int ldb,
              const double* d, double* x, double* y, double* z,
              const lsq_opts* opts, lsq_result* res);

/*
 * Complex LSE and GLS (Section 1 states both problems over C, with
 * Hermitian transposes): the same arguments as lse_solve / gls_solve, with
 * every matrix and vector complex, stored as interleaved (real, imaginary)
 * FP64 pairs (C99 double complex / LAPACK complex*16 layout), column-major
 * with lda, ldb counted in complex elements.  The solve runs on the real
 * embedding [Re M, -Im M; Im M, Re M] of each matrix (vectors [Re; Im]),
 * an LSE (GLS) of twice the sizes whose augmented system is the embedding
 * of the complex one, so its solution is the complex solution; the stop test
 * uses the complex Frobenius norms, so res->berr is the backward error of
 * the complex problem.  The solve holds the embedded copies (4 m n + 4 n p
 * doubles) in the handle's workspace.  Return codes and argument numbers as
 * lse_solve / gls_solve.
 */
int zlse_solve(lsq_handle handle, int m, int n, int p,
               const double* A, int lda, const double* B, int ldb,
               const double* b, const double* d, double* x, double* r, double* v,
               const lsq_opts* opts, lsq_result* res);
int zgls_solve(lsq_handle handle, int n, int m, int p,
               const double* A, int lda, const double* B, int ldb,
               const double* d, double* x, double* y, double* z,
               const lsq_opts* opts, lsq_result* res);

/*
 * Factor once, solve many right-hand sides.  lse_factor / gls_factor compute
 * the generalized RQ / QR factorization of the pair (Sections 3.1, 3.2) at
 * precision `prec` (an lsq_prec other than AUTO) into a new factors object,
 * which owns its own device memory.  The object keeps the pointers A and B:
 * the FP64 residual of every later solve reads them, so both must stay
 * allocated and unchanged until lsq_factors_destroy.  Returns 0 and sets
 * *factors, 1 if a panel factorization broke down at this precision (no
 * object is made), 5 for a non-finite value in A or B, 4 on a HIP error, or
 * -k for argument k (the numbers of lse_solve / gls_solve for the shared
 * arguments; 9 prec, 10 factors).  The factors are computed from
 * power-of-two scaled inputs as in lse_solve.
 */
typedef struct lsq_factors_st* lsq_factors;
int lse_factor(lsq_handle handle, int m, int n, int p,
               const double* A, int lda, const double* B, int ldb,
               int prec, lsq_factors* factors);
int gls_factor(lsq_handle handle, int n, int m, int p,
               const double* A, int lda, const double* B, int ldb,
               int prec, lsq_factors* factors);
/*
 * Refinement on stored factors (the correction solves of Algorithms 1 / 3,
 * or GMRES-IR of Section 5), with the right-hand sides b, d (LSE) or d (GLS)
 * of this call: opts->solver IR (or AUTO) or GMRES_IR; with FP64 factors the
 * FP64 direct solve.  The first solve of a kind also prepares the factors'
 * triangular inverses and aggregated blocks for it; later solves reuse them.
 * There is no escalation: a solve that does not certify returns 3 with the
 * iterate of smallest backward error; a non-finite value in b or d returns 5.
 * The prepared structures of one kind replace those of the other in the
 * factors' memory, which stays the same size over any number of switches.
 * res->ms_factor is 0.  Only the handle that made the factors may use them
 * (-2 otherwise).  Argument numbers for -k: 2 factors, 3 b, 4 d, 5 x, 8 opts
 * (LSE); 2 factors, 3 d, 4 x, 5 y, 7 opts (GLS).
 */
int lse_solve_factored(lsq_handle handle, lsq_factors factors,
                       const double* b, const double* d,
                       double* x, double* r, double* v,
                       const lsq_opts* opts, lsq_result* res);
int gls_solve_factored(lsq_handle handle, lsq_factors factors,
                       const double* d, double* x, double* y, double* z,
                       const lsq_opts* opts, lsq_result* res);
/*
 * Allocation-free variant of lse_solve_factored, for callers that cannot
 * allocate device memory during the call (tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, return codes and results as
 * lse_solve_factored with classical refinement (or, on FP64 factors, the
 * FP64 direct solve); the call itself allocates nothing: its per-call
 * workspace (ingest partial sums, iterates, residual blocks and the
 * residual's partial sums) lives in a static device array of 64 MiB, one per
 * GPU, held until the process ends.  Limits and errors:
 *   - -8 for opts->solver GMRES_IR (or invalid options);
 *   - -2 when the factors have not been prepared for classical refinement
 *     (solve once with lse_solve_factored and solver IR or AUTO first), and
 *     when the per-call workspace, about 24 (m n / 64 + m n / 256) + 32 (m +
 *     n + p) bytes, exceeds the 64 MiB;
 *   - 4 if the handle's device has no scratch address (lsq_create sets it up).
 * Every call on one GPU uses that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (two handles, two host threads, or
 * two streams) race and must be serialized by the caller.
 */
int lse_solve_factored_noalloc(lsq_handle handle, lsq_factors factors,
                               const double* b, const double* d,
                               double* x, double* r, double* v,
                               const lsq_opts* opts, lsq_result* res);
/* Frees the factors' device memory (NULL is a no-op).  Call it before
 * lsq_destroy of the handle that made them, with no solve in flight. */
int lsq_factors_destroy(lsq_factors factors);

/* One instance of a batch.  type: LSQ_LSE or LSQ_GLS; sizes and pointers as in
   lse_solve (m, n, p, A, B, b, d, x) or gls_solve (n, m, p with A = W, B = V,
   d, x, y).  Pointers are device pointers; b is ignored for GLS and y for LSE. */
enum { LSQ_LSE = 0, LSQ_GLS = 1 };
typedef struct {
  int type;
  int m, n, p;
  const double* A;
  const double* B;
  const double* b;
  const double* d;
  int lda, ldb;
  double* x;
  double* y;
} lsq_problem;

/* Solve `count` independent instances of uneven size.  `res` (host array of
   `count`, nullable) receives one record per instance.  Returns the number of
   instances with info != 0, or -k for an invalid argument (-3: a problem
   descriptor is invalid).  Work already queued on the handle's stream
   completes before the first instance starts, and every instance has
   finished when the call returns.
   Two executions (lsq_set_batch_mode):
   - persistent (LSQ_BATCH_AUTO, the default) for opts.prec FP32 or FP64 (or
     AUTO without selector weights) and opts.solver AUTO, IR or DIRECT: the
     instances with m, n, p in [1, 1024] are solved on the handle's stream by
     one launch with one work-group per instance (the longest first), which
     factors the pair (Section 3) and runs classical refinement (Algorithms 2
     and 4) entirely on the device: FP32 factors and corrections first, the
     instances that do not meet tol again with FP64 factors (reported as
     FP64 direct) when opts.escalate is set.  The FP64 rung runs beside the
     FP32 launch: each instance that fails is queued on the device (the
     longest first) and solved in FP64 by work-groups on a share of the
     compute units while the FP32 launch goes on (the rest join when it
     ends); the longest instances may go to that rung from the start (see
     lsq_batch_tuning), and report one attempt.  LSQ_BATCH_SEQUENTIAL runs the
     FP64 rung as a second launch after the FP32 one instead.  Instances that are not eligible or still fail
     continue on the batch workers below, with the full ladder.
   - batch workers (LSQ_BATCH_WORKERS, and every other option): the instances
     run concurrently on the handle's batch workers (streams of their own, one
     host thread each; see lsq_set_batch_workers), longest estimated
     factorization first, each as lse_solve / gls_solve would run it. */
int lsq_solve_batched(lsq_handle handle, int count, const lsq_problem* probs,
                      const lsq_opts* opts, lsq_result* res);

/* The persistent batch of lsq_solve_batched (opts.prec FP32, solver IR or
   AUTO, escalate set; concurrent mode) captured once for a fixed problem
   set, then replayed as one HIP graph.  A plan keeps the descriptors it was
   created with (the matrices and vectors they point to may change between
   runs, their sizes and addresses may not), their longest-first order, the
   launch shape in force at creation (route, FP64 share and FP64-first count
   of lsq_batch_tuning / the lsq_dbg_batch_* settings) and device buffers of
   its own; the handle must outlive it, and a plan runs on the handle's
   stream.  The graph holds the queue reset, the FP64 consumers on the side
   stream, a bounded device-side wait (at most 20 ms) until they are
   resident, the FP32 launch and the late consumers; it records no memset.
   lsq_batch_plan_create captures without running anything: returns -2 for a
   NULL plan pointer or an empty set, -3 for an invalid descriptor, -4 for
   invalid options, -5 when the set or the options are not of that form
   (another precision or solver, no escalation, another batch mode, an
   instance with m, n or p beyond 1024), 4 on a HIP error.
   lsq_batch_plan_run replays the graph, reads the results back and solves
   what no FP64 consumer took with an FP64 launch as lsq_solve_batched would;
   instances neither rung certifies continue on the batch workers.  `res`
   (nullable, `count` records in the order of creation) as for
   lsq_solve_batched; returns the number of instances with info != 0, -1 for
   a NULL plan.  Runs of plans on one handle must not overlap.
   lsq_batch_plan_destroy waits for the handle's streams and frees the plan
   (NULL is a no-op). */
typedef struct lsq_batch_plan_st* lsq_batch_plan;
int lsq_batch_plan_create(lsq_handle handle, int count, const lsq_problem* probs,
                          const lsq_opts* opts, lsq_batch_plan* plan);
int lsq_batch_plan_run(lsq_batch_plan plan, lsq_result* res);
int lsq_batch_plan_destroy(lsq_batch_plan plan);
/* Learned precision / solver selector (used when opts.prec is LSQ_PREC_AUTO
   or opts.solver is LSQ_SOLVER_AUTO; without weights AUTO means FP32 with
   classical IR).  An instance's features come from FP64 norms of its inputs
   and the diagonals of the triangles of its FP64 generalized factorization
   (Section 3), whose factors are kept when the selector picks FP64; an MLP
   16 -> 64 -> 64 -> 7 (ReLU, FP32) gives 5 precision logits {FP8-e4m3, BF16,
   FP16, FP32, FP64 direct} and 2 solver logits {IR, GMRES-IR}; the escalation
   ladder then starts at the chosen rung.
   lsq_selector_set copies LSQ_SELECTOR_WEIGHTS floats (host) in the order
   mean[16], std[16], W1[64][16], b1[64], W2[64][64], b2[64], W3[7][64], b3[7];
   NULL removes the selector.  Returns -3 for a wrong count, -2 for
   non-finite values or non-positive scales.
   lsq_selector_features computes the 16 features of one instance (host
   array) and, when weights are set, the 7 logits and the 2 chosen classes
   (either may be NULL; -4 without weights). */
#define LSQ_SELECTOR_FEATURES 16
#define LSQ_SELECTOR_WEIGHTS 5735
int lsq_selector_set(lsq_handle handle, const float* weights, int count);
int lsq_selector_features(lsq_handle handle, const lsq_problem* problem, float* feats,
                          float* logits, int* cls);

/* Number of concurrent workers of the batched entry points (1..64, default
   8).  Returns -2 outside that range. */
int lsq_set_batch_workers(lsq_handle handle, int workers);
/* Execution of the batched entry points (see lsq_solve_batched).  Returns -2
   for an unknown mode. */
enum { LSQ_BATCH_AUTO = 0, LSQ_BATCH_WORKERS = 1, LSQ_BATCH_SEQUENTIAL = 2 };
int lsq_set_batch_mode(lsq_handle handle, int mode);

/* Launch-shape table of the persistent batch, per size bucket and
   escalation regime, as written by the autotuner
   (paper_2406_16499_amd/autotune.py).  Entry i applies to a batch whose
   largest dimension max(m, n, p) is at most max_dim[i] while the escalation
   fraction of the handle's last FP32-first persistent batch (the share of the
   instances that tried the first rung and did not certify there; 1 before the
   first such batch and after every call of this function) is at most
   esc_max[i] in [0, 1] (NULL: all 1).  Of the entries that apply, the one
   with the smallest max_dim, then the smallest esc_max, wins.  route[i]
   (>= 0, 0 = off) is the diagonal-ratio route of the FP32 rung
   (lsq_dbg_batch_route), fp64_share[i] in (0, 1) the share of compute units
   the concurrent FP64 rung starts on (lsq_dbg_batch_split), pre[i] in [0, 8]
   the number of the longest instances, per work-group of that rung, that it
   solves in FP64 from the start instead of after an FP32 attempt
   (lsq_dbg_batch_pre; at most 7/8 of the batch's instances, so the FP32 rung
   always sees part of it).  A batch no entry covers uses those three settings.
   n = 0 clears the table.  Returns -2 for n < 0 or NULL arrays with n > 0,
   -3 for an entry out of range (the table is then unchanged). */
int lsq_batch_tuning(lsq_handle handle, int n, const int* max_dim, const double* route,
                     const double* fp64_share, const double* pre, const double* esc_max);

/* Same-type conveniences: every descriptor must carry the matching type. */
int lse_solve_batched(lsq_handle handle, int count, const lsq_problem* probs,
                      const lsq_opts* opts, lsq_result* res);
int gls_solve_batched(lsq_handle handle, int count, const lsq_problem* probs,
                      const lsq_opts* opts, lsq_result* res);

#ifdef __cplusplus
}
#endif
#endif /* LSQ_H */
