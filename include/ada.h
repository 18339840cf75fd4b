/*
 * ada.h -- C ABI of libada, an MI355X (gfx950) implementation of the adaptive
 * solver for square systems A X = B of Sanderson & Curtin, "An Adaptive Solver
 * for Systems of Linear Equations" (arXiv 2007.11208).
 *
 * What a solve computes (Section II of the paper):
 *   1. detection, in this order: banded (Section II-A: band widths from a
 *      column scan; banded when the band holds at most 25% of the n*n
 *      elements), upper or lower triangular (Section II-B), likely symmetric
 *      positive definite (Section II-C, Fig. 4); otherwise general;
 *   2. the matching factorise-and-solve: banded LU with partial pivoting,
 *      triangular substitution, Cholesky (whose failure re-routes to LU), or
 *      LU with partial pivoting (Section II-D);
 *   3. the reciprocal condition number (1-norm) of the routed factorisation;
 *   4. when a solver fails or rcond < threshold (default 0.5*eps, Section II-E)
 *      the minimum-norm least-squares solution from an SVD of the original A
 *      (here a one-sided Jacobi SVD), unless disabled.
 *
 * Conventions common to every entry point:
 *   - matrices are column-major FP64 in DEVICE memory owned by the caller;
 *     element (i,j) of a matrix with leading dimension ld is at M[i + j*ld];
 *   - A and B are never modified; X may not alias A or B;
 *   - the library never allocates device memory inside a solve: every scratch
 *     buffer comes from the caller's `work` area (size from ada_workspace_size);
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream); all
 *     device work is ordered on it. ada_solve blocks until its result is known;
 *   - return value: ADA_OK (0) or a negative ADA_ERR_* code; on error
 *     ada_last_error() names the cause (thread-local text);
 *   - a context may be shared by threads; a workspace or stream may not be
 *     shared by concurrent calls.
 */
#ifndef ADA_H
#define ADA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ADA_ABI_VERSION 1

/* return codes */
enum {
  ADA_OK = 0,
  ADA_PENDING = 1,                   /* ada_poll: the request has not completed yet */
  ADA_ERR_ARG = -1,                  /* bad n/nrhs/ld/layout/workspace, NULL pointer */
  ADA_ERR_NONFINITE = -2,            /* A or B holds NaN or Inf (rejected before any solve) */
  ADA_ERR_SINGULAR = -3,             /* fallback needed but opts.no_approx = 1; X holds the routed x */
  ADA_ERR_NOMEM = -4,                /* host allocation failed, or a server request larger than its arena */
  ADA_ERR_HIP = -5,                  /* a HIP runtime call failed, or a device wait timed out */
  ADA_ERR_FALLBACK_INFEASIBLE = -6   /* SVD fallback of a band-layout system too large to expand */
};

/* detected structure (Section II detection order; bit-exact with the definition) */
enum { ADA_CLASS_GENERAL = 0, ADA_CLASS_BANDED = 1, ADA_CLASS_TRI_UPPER = 2, ADA_CLASS_TRI_LOWER = 3,
       ADA_CLASS_SYMPD = 4,
       ADA_CLASS_SYM = 5 /* only with ADA_EXT_SYM: equal to its transpose, fails the Fig. 4 test */ };
/* solver whose x is returned */
enum { ADA_ROUTE_NONE = 0, ADA_ROUTE_BAND_LU = 1, ADA_ROUTE_TRI = 2, ADA_ROUTE_CHOL = 3, ADA_ROUTE_LU = 4,
       ADA_ROUTE_SVD = 5, ADA_ROUTE_LDLT = 6 };
/* A route the paper's conclusion (Section V) names as future work; off by default, so that the
   classes and routes are the paper's. Bits of ada_opts.extensions:
   ADA_EXT_SYM: a dense matrix exactly equal to its transpose that fails the sympd test of Fig. 4, or
     whose Cholesky factorisation fails, is solved by LDL^T with Bunch-Kaufman pivoting
     (P A P^T = L D L^T, D of 1x1 and 2x2 blocks) instead of LU; its condition estimate and the
     fallback rule are those of every route (an exactly singular D block is a solver failure).
   Tridiagonal matrices (the other case Section V names) take the band route at kl = ku = 1.
   ada_solve only (ada_solve_batched returns ADA_ERR_ARG when any bit is set). */
enum { ADA_EXT_SYM = 1 };
/* arithmetic of the LU / Cholesky factorisation. FP64: FP64 throughout. FP32_IR, BF16_IR: a
   factorisation in lower precision (ada_solve: the trailing-matrix updates take FP32 or BF16 operands
   with FP32 accumulation, panels and pivot search stay FP64; ada_solve_batched: FP32_IR only, the
   whole factorisation in FP32), then FP64 iterative refinement (FP64 residuals and corrections) until
   the backward error reaches sqrt(n)*eps. FP32: the correction is the solve with the FP32 factors;
   BF16: the correction equation is solved by GMRES (FP64 vectors, each right-hand side with its own
   Krylov basis of up to 50 vectors) preconditioned by the BF16 factors. When the refinement stalls,
   grows or needs more than 30 steps, or when the condition estimate of the low-precision factors is
   below 1e-9, the system is solved again by the FP64 route (the result's refine_iters is then
   negative; otherwise the number of refinement steps). Triangular, banded and SVD routes always run
   in FP64. */
enum { ADA_PREC_FP64 = 0, ADA_PREC_FP32_IR = 1, ADA_PREC_BF16_IR = 2 };
/* input layout */
enum { ADA_LAYOUT_DENSE = 0, ADA_LAYOUT_BAND = 1 };
/* why the SVD fallback ran (Section II-E): */
enum { ADA_FALLBACK_NONE = 0, ADA_FALLBACK_FAILURE = 1, ADA_FALLBACK_RCOND = 2, ADA_FALLBACK_RCOND_NAN = 3 };

typedef struct ada_ctx_s* ada_ctx;

typedef struct {
  uint32_t struct_size;     /* = sizeof(ada_opts); lets the ABI grow */
  int32_t no_approx;        /* 1: never run the SVD fallback (the optional argument of Section II-E);
                               the call then returns ADA_ERR_SINGULAR when the fallback is due */
  double rcond_threshold;   /* fallback when rcond < this; a negative value selects 0.5*eps */
  int32_t layout;           /* ADA_LAYOUT_DENSE, or ADA_LAYOUT_BAND: A holds LAPACK band storage,
                               A[ku_in + i - j + j*lda] = A(i,j) for max(0,j-ku_in) <= i <= min(n-1,j+kl_in),
                               lda >= kl_in+ku_in+1; entries outside the stored band are zero */
  int32_t kl_in, ku_in;     /* stored band widths for ADA_LAYOUT_BAND */
  int32_t force_general;    /* 1: skip detection, always LU (the paper's "standard" solver, Section III) */
  int32_t want_berr;        /* 1: compute result.berr (normwise backward error) on the device */
  int32_t precision;        /* ADA_PREC_* (default FP64) */
  int32_t extensions;       /* ADA_EXT_* bits (default 0: the paper's routes only) */
} ada_opts;

typedef struct {
  int32_t cls;              /* ADA_CLASS_*; GENERAL when force_general */
  int32_t kl, ku;           /* exact band widths of A (-1 when detection was skipped) */
  int32_t route;            /* ADA_ROUTE_* of the returned x */
  int32_t chol_failed;      /* 1 when Cholesky failed and the system was re-solved by LU */
  int32_t fallback;         /* ADA_FALLBACK_* */
  int32_t info;             /* 1-based column of the first zero pivot / zero diagonal / failed Cholesky pivot */
  int32_t rank;             /* SVD route: number of singular values > eps*sigma_max; else n */
  int32_t sweeps;           /* SVD route: Jacobi sweeps */
  int32_t nsolves;          /* solves spent by the condition estimate */
  int32_t refine_iters;     /* FP32_IR: refinement steps taken; < 0: the FP32 attempt did not converge
                               (-1: its factorisation failed, -1-k: stopped after k steps) and x comes
                               from the FP64 route; 0 otherwise */
  int32_t status;           /* per-system status of a batched solve (ADA_OK or ADA_ERR_*); ada_solve: ADA_OK */
  double rcond;             /* reciprocal 1-norm condition estimate of the routed factorisation; NaN if none */
  double berr;              /* max over columns of ||b-Ax||_inf / (||A||_inf ||x||_inf + ||b||_inf); NaN unless want_berr */
} ada_result;

/* Create a context bound to HIP device `device` (loads nothing else; cheap).
 * Returns ADA_OK or ADA_ERR_HIP / ADA_ERR_NOMEM. */
int ada_create(ada_ctx* out, int device);
void ada_destroy(ada_ctx ctx);

/* Thread-local description of the last error returned on this thread ("" if none). */
const char* ada_last_error(void);

/* Fill opts with the defaults (threshold 0.5*eps, dense layout, berr on). */
void ada_opts_default(ada_opts* opts);

/* Bytes of device workspace ada_solve needs for this shape and these options
 * (opts NULL = defaults). Returns 0 for invalid arguments. Pure host function. */
size_t ada_workspace_size(int n, int nrhs, const ada_opts* opts);

/* Adaptive solve of A X = B (Section II): detection, routed factorisation and
 * solve, condition estimate, SVD least-squares fallback.
 *   n >= 1, nrhs >= 1; A: device, lda >= n (dense) or per opts.layout;
 *   B: device n x nrhs, ldb >= n; X: device n x nrhs, ldx >= n (output);
 *   work: device, >= ada_workspace_size(n, nrhs, opts) bytes, 256-byte aligned;
 *   result: host pointer, filled on ADA_OK and on ADA_ERR_SINGULAR;
 *   stream: hipStream_t or NULL.
 * Blocking: returns after the result is known (X is complete on `stream`). */
int ada_solve(ada_ctx ctx, int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X,
              int ldx, void* work, size_t work_bytes, const ada_opts* opts, ada_result* result, void* stream);

/* ---- the same solve without a caller workspace ----
 * For callers that cannot allocate device memory or hand the library a
 * workspace (tight serving loops, harnesses that forbid allocation): ada_solve
 * with its workspace taken from a fixed array of ADA_NOALLOC_SCRATCH_BYTES in
 * the library's device memory. Every GPU the library is loaded on holds one
 * such array until the process ends; its address is taken once per device when
 * a context is created there. The call allocates nothing (no hipMalloc, no
 * hipFree, no events beyond those profiling already created). Arguments,
 * results, blocking and errors are those of ada_solve; a shape whose workspace
 * (ada_workspace_size) exceeds the fixed array returns ADA_ERR_ARG with the
 * sizes in ada_last_error (dense input with default options and one right-hand
 * side: n <= 3269).
 * All calls on one GPU share its array, which keeps the last call's contents
 * (each solve initialises what it reads): calls that overlap on one GPU, from
 * any thread or context, race and must be serialised by the caller. */
#define ADA_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int ada_solve_noalloc(ada_ctx ctx, int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X,
                      int ldx, const ada_opts* opts, ada_result* result, void* stream);

/* ---- batched solve: many independent small systems in one launch ----
 * Every system goes through the whole method of Section II (detection,
 * routed factorisation and solve, condition estimate, the rule of Section
 * II-E with the SVD least-squares fallback, backward error) inside one
 * workgroup on the device; workgroups take systems from a counter.
 * Supported per system: 1 <= n <= 256, 1 <= nrhs <= 8, dense column-major
 * input; others are reported with status ADA_ERR_ARG. A banded system is
 * factored by partial-pivoting elimination over the full matrix, which on a
 * band gives the band LU's pivots and factors. */
typedef struct {
  int32_t n, nrhs;          /* order and number of right-hand sides */
  int32_t lda, ldb, ldx;    /* leading dimensions, >= n */
  int32_t pad;
  int64_t a_off, b_off, x_off; /* element offsets of this system's A, B and X in the pools */
} ada_desc;

/* Bytes of device workspace ada_solve_batched needs for `count` systems. Pure host function. */
size_t ada_batched_workspace_size(int count);

/* Solve count systems. d_desc: device array of count descriptors; A_pool,
 * B_pool: device FP64 pools the offsets index (never modified); X_pool:
 * device FP64 pool for the solutions; work: device, >= the size above,
 * 256-byte aligned; opts: host pointer or NULL (layout must be dense;
 * no_approx, rcond_threshold, force_general, want_berr apply to every
 * system); d_results: device array of count results, filled with each
 * system's status. Asynchronous: returns once the work is enqueued on
 * `stream`; it enqueues kernels only (no host synchronisation, no memset,
 * no allocation), so it may be captured into a HIP graph and replayed.
 * Systems are taken largest first (a device-side ordering by n), in the
 * launch shape ctx keeps for the precision (ada_set_batched_shape,
 * ada_autotune_batched); each system's result depends neither on the
 * others in the batch nor on the shape.
 * Returns ADA_ERR_ARG for invalid arguments (nothing enqueued). */
int ada_solve_batched(ada_ctx ctx, int count, const ada_desc* d_desc, const double* A_pool, const double* B_pool,
                      double* X_pool, void* work, size_t work_bytes, const ada_opts* opts, ada_result* d_results,
                      void* stream);

/* Launch shape of ada_solve_batched. It changes the speed only: every valid shape gives
 * bit-identical results. The systems are split by order into `buckets` ranges launched one after
 * the other, largest orders first: range k holds the orders in (max_n[k+1], max_n[k]]
 * (max_n[buckets] = 0), with max_n[0] = 256 > max_n[1] > max_n[2] >= 16. Each launch sizes its LDS
 * for its largest order and runs wg_per_cu[k] workgroups per compute unit (1: the kernel variant
 * with 512 registers per lane; 2: the variant with 256, for ranges with max_n <= 96, whose LDS fits
 * twice) and workgroups[k] persistent workgroups in all (at most what the workspace of
 * ada_batched_workspace_size holds: 256 at max_n = 256). stage_cols: columns of a triangle held in
 * HBM (orders above 128) that a wave stages into LDS at a time, 4 or 8. The default: one launch,
 * 256 workgroups, stage_cols = 8. */
typedef struct {
  int32_t buckets;
  int32_t max_n[3];
  int32_t wg_per_cu[3];
  int32_t workgroups[3];
  int32_t stage_cols;
} ada_batched_shape;

/* Sets the shape ctx's ada_solve_batched calls use for `precision` (ADA_PREC_FP64 or
 * ADA_PREC_FP32_IR): shape (host pointer) is validated, ADA_ERR_ARG with the reason otherwise;
 * shape NULL restores the default. */
int ada_set_batched_shape(ada_ctx ctx, int precision, const ada_batched_shape* shape);
/* The shape ctx uses for `precision` (host pointer out). */
int ada_get_batched_shape(ada_ctx ctx, int precision, ada_batched_shape* shape);

/* Autotuner of the batched launch. Arguments as ada_solve_batched: the caller's own batch is solved
 * under each candidate shape and the fastest is kept in ctx for opts->precision. Candidates: one
 * launch, or launches split at orders 128, 96 or 64 (and 128 + 64, 96 + 48); for each range, one or
 * (max_n <= 96) two workgroups per compute unit; stage_cols 4 or 8. Each candidate runs once after a
 * warm-up, timed per range with events on `stream`; every range takes its fastest variant, the
 * split with the smallest sum wins, and the winner is timed once more. On return X_pool and
 * d_results hold the batch's solution (the same under every shape). Synchronises the stream;
 * allocates nothing but events. shape_out and ms_out (either may be NULL) receive the chosen shape
 * and its time per batch in ms. Returns ADA_OK, ADA_ERR_ARG or ADA_ERR_HIP. */
int ada_autotune_batched(ada_ctx ctx, int count, const ada_desc* d_desc, const double* A_pool,
                         const double* B_pool, double* X_pool, void* work, size_t work_bytes,
                         const ada_opts* opts, ada_result* d_results, void* stream, ada_batched_shape* shape_out,
                         double* ms_out);

/* ---- solve server: continuous batching over a caller-provided HBM arena ----
 * Requests are independent systems (each solved by the method of Section II, as ada_solve or, for
 * n <= 256 and nrhs <= 8, as ada_solve_batched). A request is admitted when its footprint fits in the
 * arena's free space and a worker is free, while earlier requests are still running: waiting small
 * systems are solved together by one batched launch, larger ones by solve workers that each have their
 * own context and stream, so that their kernels overlap on the device. Requests that reuse kept factors
 * start first; other requests start in arrival order, except that with two or more solve workers the
 * first of them takes only requests of order <= 1024 (a fast lane beside long factorisations and SVD
 * fallbacks). A request whose footprint cannot fit beside the server's fixed buffers is refused at
 * submission (ADA_ERR_NOMEM). A request may keep its factors resident (keep_factor = 1); later
 * requests that name the returned ada_factor (reuse) solve new right-hand sides with those factors
 * only, FP64-refined when the factors were mixed precision, until ada_factor_release.
 * Ownership: the arena, A, B and X are the caller's device memory; A and B must stay unchanged and X
 * untouched until the request's ada_poll returns a completion. The server copies A into the arena when
 * it keeps factors. Each server has one batch worker and `solve_workers` solve workers (host threads);
 * its calls are thread-safe. */
typedef struct ada_server_s* ada_server;
typedef uint64_t ada_ticket;
typedef uint64_t ada_factor;  /* 0 = none */
typedef struct {
  int32_t n, nrhs;           /* reuse: n = 0 or the factor's n; nrhs <= 8 */
  int32_t lda, ldb, ldx;     /* column-major leading dimensions (lda unused for reuse) */
  int32_t keep_factor;       /* 1: keep the factors resident and return them from ada_poll */
  const double* A;           /* device, n x n (NULL for reuse) */
  ada_factor reuse;          /* nonzero: solve with these kept factors (A unused) */
  const double* B;           /* device, n x nrhs */
  double* X;                 /* device, n x nrhs */
  ada_opts opts;             /* struct_size 0 = defaults; dense layout only; reuse takes the factor's */
} ada_request;

/* arena: device memory of arena_bytes (256-byte aligned), e.g. a torch allocation; solve_workers 1..8 */
int ada_server_create(ada_ctx ctx, void* arena, size_t arena_bytes, int solve_workers, ada_server* out);
/* Stops the workers after the requests they are running; queued requests are dropped. */
void ada_server_destroy(ada_server s);
/* Arena bytes the request holds while it runs (and, with keep_factor, until released); 0 for requests
 * the batch worker's fixed buffers serve and for reuse requests. Pure host function. */
size_t ada_request_footprint(const ada_request* r);
/* Queues the request and returns at once with its ticket (never waits for the device). */
int ada_submit(ada_server s, const ada_request* r, ada_ticket* out);
/* Waits up to timeout_us (< 0: without limit, 0: not at all) for the request. Returns ADA_PENDING if it
 * has not completed; otherwise its status (ADA_OK or ADA_ERR_*), fills *out (and *kept with the kept
 * factor, or 0) and retires the ticket. */
int ada_poll(ada_server s, ada_ticket t, ada_result* out, ada_factor* kept, int64_t timeout_us);
/* ada_poll that also reports the request's wait before it started and its latency from submission to
 * completion, in microseconds (either pointer may be NULL). */
int ada_poll_timed(ada_server s, ada_ticket t, ada_result* out, ada_factor* kept, int64_t timeout_us,
                   double* queue_us, double* total_us);
/* Frees the kept factors (after the requests that name them complete). */
int ada_factor_release(ada_server s, ada_factor f);
/* Arena bytes in use, requests waiting to start, factors kept. Any pointer may be NULL. */
int ada_server_usage(ada_server s, size_t* arena_used, int* queued, int* kept_factors);

/* ---- instrumentation (not part of the method) ----
 * When enabled, the library records HIP events on the solve's stream around
 * every launch of the kernel families below and accumulates, per family, the
 * launch count, the total device time between the events and the algorithmic
 * flops and HBM bytes of those launches (what the method must compute and
 * move, not what the kernel happens to do). Reading is per family. */
enum {
  ADA_KF_GEMM = 0,   /* trailing update of LU / Cholesky (FP64 MFMA) */
  ADA_KF_PANEL = 1,  /* LU panel with partial pivoting */
  ADA_KF_LASWP = 2,  /* row interchanges left and right of the panel */
  ADA_KF_TRSM_BLOCK = 3, /* block-row / block-column triangular solve inside a factorisation */
  ADA_KF_POTRF = 4,  /* Cholesky diagonal block */
  ADA_KF_TRSV = 5,   /* triangular solves (routed solves and estimator) */
  ADA_KF_GBTRF = 6,  /* band LU with partial pivoting */
  ADA_KF_GBTRS = 7,  /* band solves (one record per solve, several kernels) */
  ADA_KF_DETECT = 8, /* dense structure scan */
  ADA_KF_JACOBI = 9, /* one-sided Jacobi rounds */
  ADA_KF_COUNT = 10
};
/* Autotuner of the row-parallel band solve (band routes with n >= 512): times each candidate LDS
 * staging piece (8, 16, 32, 64 rows of a chunk at a time; those whose LDS fits) on a synthetic
 * band factor of order n with the given band widths and number of right-hand sides, on `stream`,
 * and keeps the fastest in ctx for every later band solve with the same kl + ku, one (nrhs = 1) or
 * several right-hand sides, and the same floor(log2 n) (the best piece depends on how many chunks
 * the order gives the compute units). The choice changes the speed only: every piece gives
 * bit-identical results. Allocates and frees its own device memory (about
 * 8 n (2kl+ku+1 + 2 nrhs + 5 (kl+ku)) bytes); synchronises the stream. 512 <= n <= 2^26,
 * 1 <= kl + ku <= 31, 1 <= nrhs <= 64. Returns ADA_OK, ADA_ERR_ARG, ADA_ERR_NOMEM or ADA_ERR_HIP;
 * *piece_out and *ms_out (either may be NULL) receive the chosen piece and its time per solve in ms. */
int ada_autotune_band(ada_ctx ctx, int n, int kl, int ku, int nrhs, void* stream, int* piece_out, double* ms_out);

/* Kernel-family timing: while on != 0, every later solve on ctx brackets each launch of a selected
 * family (see ada_profile_families) with two HIP events on the stream the launch goes to; the
 * durations accumulate per family until ada_profile_reset. Each event is a packet in the stream's
 * queue between dependent kernels, so timing slows the solves a little: select only the families
 * to be measured. Returns ADA_OK or ADA_ERR_ARG (ctx NULL). */
int ada_profile_enable(ada_ctx ctx, int on);
/* The families ada_profile_enable times: bit (1 << ADA_KF_*) set = timed. The default (and the
 * state after ada_create) is every family. Returns ADA_OK or ADA_ERR_ARG (ctx NULL). */
int ada_profile_families(ada_ctx ctx, unsigned mask);
/* kind: ADA_KF_*; any output pointer may be NULL. */
int ada_profile_read(ada_ctx ctx, int kind, int64_t* launches, double* total_ms, double* total_flops,
                     double* total_bytes);
int ada_profile_reset(ada_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* ADA_H */
