/*
 * caqr.h -- C ABI of the multilevel (tree) Householder QR library for one
 * AMD MI355X (gfx950).
 *
 * What it computes.  The QR factorization A = QR of an m-by-n real matrix,
 * m >= n, Q orthogonal and R upper triangular, obtained with Householder
 * reflections; Q is kept implicit in compact Y T Y^T form and the reflectors
 * are stored in the lower part of A along a reduction tree (paper, Section 3.1
 * "Multilevel QR factorization", and Algorithm 1, ML-CAQR(A, m, n, r, P)).
 *
 *   tsqr_factor : one panel (n <= 64): a reduction tree (arity 2 or 4) of
 *                 stacked-R eliminations over row blocks (the panel step of
 *                 Algorithm 1 and items 1(a)-1(b) of its description in
 *                 Section 3.1).
 *   caqr_factor : the panel loop of Algorithm 1: factor panel kk with the tree,
 *                 then update the trailing matrix with the leaf reflectors
 *                 (the MLUPFACT step) and the tree-node reflectors (the
 *                 MLUPELIM step).
 *   apply_q     : multiply by Q or Q^T using the stored tree of reflectors.
 *   ls_solve    : min ||A x - b||_2 via A = QR (the least-squares use named in
 *                 Section 3.1).
 *
 * Conventions shared by every call.
 *   - Matrices are column-major (Fortran order) FP64 with a leading
 *     dimension; all matrix pointers are DEVICE pointers of the handle's GPU.
 *   - Work is enqueued on the handle's stream and returns without waiting;
 *     caqr_sync() waits and reports asynchronous device errors.
 *   - Arguments are validated synchronously; on any error nothing is enqueued
 *     and no output is touched.
 *   - R is returned with a non-negative diagonal: the library records
 *     D = diag(sign(R_jj)) (sign(0) = +1) and folds it into Q, so that
 *     A = Q_thin R with Q_thin = Q_implicit(:, 0:n) D.  For full-rank A this R
 *     is unique, whatever the tree shape or leaf height.
 *   - Factorization never fails numerically: a rank-deficient A gives R_jj = 0
 *     and no error.  NaN/Inf in A propagate.
 *   - A handle is not thread-safe; use one handle per host thread.  Separate
 *     handles on separate streams may run concurrently.
 *
 * Storage of the factors.  A is overwritten: R in A(0:n, 0:n) (upper
 * triangle), leaf reflectors Y below the diagonal of each leaf block, and each
 * tree node's reflector block V (upper triangular, non-unit diagonal) over the
 * R slot of the row block it eliminated.  tau, T and D live in the factors
 * object.  The caller keeps A alive and unmodified while the factors are used.
 */
#ifndef CAQR_H
#define CAQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct caqr_handle_s *caqr_handle_t;   /* device, stream, workspace */
typedef struct caqr_factors_s *caqr_factors_t; /* tau/T/D buffers, tree metadata; references A */

typedef enum {
  CAQR_SUCCESS = 0,
  CAQR_ERR_INVALID_VALUE = 1, /* bad size, leading dimension, pointer or option */
  CAQR_ERR_ALLOC = 2,         /* device allocation failed or exceeds the workspace limit */
  CAQR_ERR_DEVICE = 3,        /* no usable GPU, or an asynchronous device error */
  CAQR_ERR_NOT_SUPPORTED = 4, /* valid request outside what is implemented (e.g. m < n) */
  CAQR_ERR_SINGULAR = 5,      /* ls_solve: R has an exactly zero diagonal entry */
  CAQR_ERR_NONFINITE = 6,     /* ls_solve: NaN/Inf in R's diagonal or in the solution */
  CAQR_ERR_NOT_CONVERGED = 7  /* ls_solve, mixed precision: refinement did not reach its tolerance */
} caqr_status_t;

typedef enum { CAQR_OP_N = 0, CAQR_OP_T = 1 } caqr_op_t;

/* Tree options (all fields 0 = library default).
 *   leaf_rows      rows per leaf block: 64, 128 or 256 (default 256).
 *   leaves_per_wg  leaves one workgroup factors and combines in its own
 *                  registers/LDS before the device-wide tree: 1, 2 or 4
 *                  (default 1), a power of the arity (2 needs arity 2, and
 *                  selects it when arity is 0).  A single panel with 128 or more
 *                  workgroups finishes the device-wide tree with one
 *                  launch per level instead of workgroups signalling each
 *                  other.
 *   inner_block    block size of the level below the panel (paper, Section
 *                  3.1, item 1(a): a level factors its part of a b_r-wide
 *                  panel with the next level's block size b_{r-1}): every
 *                  leaf and every stacked elimination is factored in inner
 *                  blocks of 16 or 32 columns, each finished block applied to
 *                  the columns right of it as one compact-WY transformation.
 *                  0 or 64: no inner blocking (default).  The reflectors are
 *                  the same as without it up to rounding, so Y, V, tau, T and
 *                  every other call are unchanged.  tsqr_factor and
 *                  caqr_factor only: the batched calls return
 *                  CAQR_ERR_NOT_SUPPORTED for a nonzero value.
 *   arity          members of every tree node: 2 (binary) or 4 (default 4;
 *                  2 when leaves_per_wg is 2).  Level s = arity^j groups
 *                  the row blocks (after the levels below) g, g + s, ...,
 *                  g + (arity - 1) s, g a multiple of arity * s, the lowest
 *                  index on top (for arity 2 the pairing of leaf i with leaf
 *                  i + 2^(k-1) at level k); a node with fewer members at the
 *                  end of a level eliminates those present.  A tree of arity
 *                  4 has about half the levels of the binary tree, so half
 *                  the sequential eliminations on the panel's critical
 *                  path.  Inner blocks need arity 2 (CAQR_ERR_NOT_SUPPORTED
 *                  otherwise).
 * leaves_per_wg only decides which levels run inside a workgroup, so R, Y, V
 * and tau are identical for every leaves_per_wg of one arity; different
 * arities give the same R up to rounding (different Y, V and tau). */
typedef struct {
  int32_t leaf_rows;
  int32_t leaves_per_wg;
  int32_t inner_block;
  int32_t arity; /* 0, 2 or 4 */
} caqr_tree_opts_t;

/* Summary of a factors object (host values). */
typedef struct {
  int64_t m, n, nb;       /* problem size and panel width */
  int64_t panels;         /* number of panels (1 for tsqr_factor with n <= 64) */
  int32_t leaf_rows;      /* leaf height used */
  int32_t leaves_per_wg;  /* leaves per workgroup used */
  int64_t leaves_panel0;  /* leaves of the first panel */
  int32_t depth_panel0;   /* tree levels of the first panel */
  int32_t t_formed;       /* 1 when the T factors are materialized */
  int32_t inner_block;    /* inner block used (0: none) */
  int32_t arity;          /* tree arity used (2 or 4) */
} caqr_factors_info_t;

/* Least-squares options and report.
 *   precision  CAQR_LS_F64 (0): the FP64 solve.  CAQR_LS_MIXED_F32 (1): the
 *              factorization's trailing-update products with the leaf
 *              reflectors (Y^T C and Y W) run on FP32 MFMA with FP32
 *              accumulation, while reflector generation, norms, the tree's
 *              R combines and node updates, the residuals and every step of
 *              the refinement stay FP64; the solution is refined in FP64 by
 *              CGLS on min ||b - A R~^-1 y||, x = R~^-1 y (R~ the computed R
 *              as a right preconditioner) until the backward-error bound
 *              ||A^T r|| / (a (a ||x|| + ||b||)) <= tol, a = max(||A||_F /
 *              sqrt(n), max_j ||A(:, j)||) <= ||A||_2 (so the reported bound
 *              is at least eta(x)), checked on a recomputed residual.
 *   max_iter   refinement iterations per right-hand side (0: 30).
 *   tol        target backward-error bound (0: 1e-12).
 *   no_fallback  0: when refinement does not reach tol (it stalls or runs out
 *              of iterations), the problem is solved again in FP64 from A
 *              and info->fallback is set; 1: return CAQR_ERR_NOT_CONVERGED
 *              with the last iterate in B.
 * With n <= 64 there is no trailing update, so the mixed solve is the FP64
 * one. */
typedef enum { CAQR_LS_F64 = 0, CAQR_LS_MIXED_F32 = 1 } caqr_ls_precision_t;

typedef struct {
  int32_t precision;   /* caqr_ls_precision_t */
  int32_t max_iter;    /* 0 = 30 */
  double tol;          /* 0 = 1e-12 */
  int32_t no_fallback; /* 0 or 1 */
  int32_t reserved;    /* 0 */
} caqr_ls_opts_t;

typedef struct {
  int32_t status;   /* caqr_status_t of the solve (valid after caqr_sync) */
  int64_t index;    /* first j with R_jj == 0 when status == CAQR_ERR_SINGULAR */
  int32_t iters;    /* mixed precision: refinement iterations (largest over the right-hand sides) */
  int32_t fallback; /* mixed precision: 1 when the FP64 solve replaced the refined one */
  double eta;       /* mixed precision: final backward-error bound (largest over the right-hand sides) */
} caqr_ls_info_t;

/* Argument checks run before the handle is inspected, so every size or
 * pointer error is reported identically whether or not a GPU is present; a
 * NULL handle with otherwise valid arguments is CAQR_ERR_INVALID_VALUE. */

/* ---------------------------------------------------------------- handles */

/* Create a handle on GPU `device` (its current stream is the null stream).
 * Returns CAQR_ERR_DEVICE if the device does not exist or no GPU is present;
 * *h is then set to NULL.  h must not be NULL. */
caqr_status_t caqr_create(caqr_handle_t *h, int device);

/* Destroy a handle and free its workspace (waits for its stream first). */
caqr_status_t caqr_destroy(caqr_handle_t h);

/* Set the stream (a hipStream_t passed as void*; NULL = null stream) on which
 * every later call of this handle enqueues its work. */
caqr_status_t caqr_set_stream(caqr_handle_t h, void *stream);
caqr_status_t caqr_get_stream(caqr_handle_t h, void **stream);

/* Upper bound, in bytes, on the device memory the library may hold for this
 * handle and for each factors object it creates (0 = unlimited).  A call that
 * would exceed it returns CAQR_ERR_ALLOC without enqueuing anything. */
caqr_status_t caqr_set_workspace_limit(caqr_handle_t h, size_t bytes);

/* Host-forced failure, for tests of error propagation through the ABI: with
 * k >= 1 the k-th library launch site this handle reaches from now on (a
 * panel, T formation, a trailing update or Q application, a back
 * substitution, a batched group) returns CAQR_ERR_DEVICE from the call that
 * reached it instead of enqueuing its kernel, as an asynchronous device error
 * would; the call releases what it allocated, and the handle stays usable.
 * Work enqueued before that site runs normally.  k = 0 switches it off.
 * Errors: CAQR_ERR_INVALID_VALUE for a NULL handle or k < 0. */
caqr_status_t caqr_debug_fail_at(caqr_handle_t h, int64_t k);

/* Wait for all work enqueued by this handle; report asynchronous errors. */
caqr_status_t caqr_sync(caqr_handle_t h);

/* Static English text for a status code. */
const char *caqr_status_string(caqr_status_t s);

/* Number of visible GPUs (0 when none); never fails. */
int caqr_device_count(void);

/* -------------------------------------------------------- factorizations */

/* QR of one tall-skinny panel by the binary reduction tree (n <= 64; larger
 * n is factored panel by panel as caqr_factor with nb = 64).
 *   m, n   sizes, m >= n >= 0 (m < n: CAQR_ERR_NOT_SUPPORTED).
 *   A      device, m-by-n, lda >= max(1, m); overwritten with R and the
 *          reflectors (see the storage note above).
 *   opts   NULL for defaults.
 *   F      receives a new factors object (owned by the caller, release with
 *          caqr_factors_destroy); it references A.
 * Only tau is stored; the T factors are formed on first use by apply_q. */
caqr_status_t tsqr_factor(caqr_handle_t h, int64_t m, int64_t n, double *A, int64_t lda,
                          const caqr_tree_opts_t *opts, caqr_factors_t *F);

/* QR of a general m-by-n matrix (m >= n) panel by panel, panel width nb
 * (1 <= nb <= 64; nb > n is clamped to n).  Each panel is factored by the
 * reduction tree and the trailing matrix is updated with the leaf and node
 * reflectors before the next panel.  Arguments as tsqr_factor. */
caqr_status_t caqr_factor(caqr_handle_t h, int64_t m, int64_t n, int64_t nb, double *A, int64_t lda,
                          const caqr_tree_opts_t *opts, caqr_factors_t *F);

/* C <- op(Q) C where Q is the m-by-m orthogonal factor of F (including the
 * sign matrix D), C is m-by-k in device memory with ldc >= max(1, m), k >= 0.
 * op = CAQR_OP_T gives Q^T C (so (Q^T A)(0:n, :) = R), op = CAQR_OP_N gives Q C
 * (so Q [I_n; 0] = Q_thin).  The handle must be on F's device. */
caqr_status_t apply_q(caqr_handle_t h, caqr_factors_t F, caqr_op_t op, int64_t k, double *C, int64_t ldc);

/* Release a factors object (does not touch A). */
caqr_status_t caqr_factors_destroy(caqr_factors_t F);

/* Host summary of F. */
caqr_status_t caqr_factors_get_info(caqr_factors_t F, caqr_factors_info_t *info);

/* Copy the recorded signs D (n doubles, each +1 or -1) to host memory. */
caqr_status_t caqr_factors_get_signs(caqr_handle_t h, caqr_factors_t F, double *d_host);

/* ------------------------------------------------------- least squares */

/* Solve min ||A x - b|| for each of the nrhs columns of B (m >= n).
 * FP64 (o NULL or o->precision == CAQR_LS_F64): A (m-by-n, lda) is
 * overwritten by its factorization, B (m-by-nrhs, ldb >= max(1, m)) by Q^T B
 * with the solutions in B(0:n, :).  Mixed precision: A is only read (the
 * library factors a copy, and the refinement needs A), B(0:n, :) receives
 * the solutions and the rest of B is left unspecified; the workspace (a copy
 * of A, the factors and the refinement's vectors) is allocated for the call.
 * The call waits for its stream and returns the numerical status:
 * CAQR_ERR_SINGULAR (info->index = first j with R_jj == 0) or
 * CAQR_ERR_NONFINITE (NaN/Inf in R's diagonal or in the solution); info (host
 * memory, may be NULL) receives the same status.  Argument errors are
 * reported before anything is enqueued. */
caqr_status_t ls_solve(caqr_handle_t h, int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *B,
                       int64_t ldb, const caqr_ls_opts_t *o, caqr_ls_info_t *info);

/* The solve of ls_solve without any device allocation, for callers that
 * cannot allocate (code running under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, results, statuses and the
 * waiting behaviour are those of ls_solve (no options).  The factors'
 * tau/D/T workspace, the ticket counters of the reduction trees and the
 * status words come from one static device array of 64 MiB that the library
 * holds on every GPU it runs on until the process ends (resolved per device
 * by caqr_create); the panel loop runs on the handle's stream alone (no
 * second stream), and the ticket counters are cleared by a kernel at the
 * start of every call.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (from several handles or threads) race and must be
 * serialized by the caller.  Problems whose workspace does not fit return
 * CAQR_ERR_NOT_SUPPORTED before anything is enqueued: about
 * 64 * ceil(m / 256) KiB for n <= 64 (m up to about 250,000 rows), and about
 * 128 * ceil(m_s / 256) KiB per 64-column panel beyond. */
caqr_status_t ls_solve_noalloc(caqr_handle_t h, int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda,
                               double *B, int64_t ldb, caqr_ls_info_t *info);

/* ------------------------------------------------------------- tracing */

/* Per-launch device timing (HIP events recorded on the handle's stream around
 * each kernel the library launches), for measurement tools.  Off by default. */
typedef enum {
  CAQR_TRACE_PANEL = 0,     /* panel factorization (leaf QR + reduction tree) */
  CAQR_TRACE_UPDATE_T = 1,  /* Q^T applied to a block of columns (trailing update) */
  CAQR_TRACE_UPDATE_N = 2,  /* Q applied to a block of columns */
  CAQR_TRACE_FORM_T = 3,    /* T factors formed after a factorization without them */
  CAQR_TRACE_OTHER = 4,     /* least-squares helpers */
  CAQR_TRACE_UPDATE_T_LEVELS = 5  /* trailing update of a factorization run as a leaf launch plus one
                                     launch per tree level (the columns beyond the next panel) */
} caqr_trace_kind_t;

typedef struct {
  int32_t kind;    /* caqr_trace_kind_t */
  int32_t panel;   /* panel index within its factorization */
  int64_t rows;    /* rows of the panel */
  int64_t cols;    /* panel width (PANEL, FORM_T) or columns updated (UPDATE_*) */
  int32_t width;   /* panel width b */
  int32_t leaves;  /* leaves of the panel's tree */
  double ms;       /* device time of the launch, milliseconds */
} caqr_trace_entry_t;

/* Enable (1) or disable (0) tracing of every kind; either call clears
 * recorded entries. */
caqr_status_t caqr_set_trace(caqr_handle_t h, int enable);

/* Trace only the kinds whose bit (1 << caqr_trace_kind_t) is set in mask
 * (0 disables tracing), so that a measurement brackets only the launches it
 * needs; clears recorded entries.  Errors: CAQR_ERR_INVALID_VALUE for a NULL
 * handle or bits above CAQR_TRACE_UPDATE_T_LEVELS. */
caqr_status_t caqr_set_trace_kinds(caqr_handle_t h, uint32_t mask);

/* Wait for the handle's stream and copy up to max entries (in launch order) to
 * host memory; *count receives the number recorded (may exceed max).  Entries
 * are cleared afterwards. */
caqr_status_t caqr_trace_read(caqr_handle_t h, caqr_trace_entry_t *out, int64_t max, int64_t *count);

/* ------------------------------------------------------------------------ */
/* Batched TSQR over independent problems of uneven sizes.                   */
/*                                                                           */
/* Each problem i is the panel factorization of Section 3.1 (Algorithm 1,    */
/* items 1(a)-1(b)) on its own: an m_i-by-n_i matrix (m_i >= n_i, n_i <= 64)  */
/* is split into leaves, each factored by Householder QR, and the leaf R      */
/* factors are eliminated along the tree of its plan's arity, exactly as      */
/* tsqr_factor does.  All problems run in one launch per (leaf height,        */
/* ceil(n_i/16), arity) group; the results of problem i are bitwise those of */
/* tsqr_factor on it with the same plan (leaf_rows, leaves_per_wg, arity).    */
/* CAQR_F32 runs the same steps in single                                     */
/* precision (float storage and arithmetic throughout); its results do not    */
/* depend on the other problems of the batch either.                          */
/* ------------------------------------------------------------------------ */

typedef enum { CAQR_F64 = 0, CAQR_F32 = 1 } caqr_dtype_t;

typedef struct caqr_batch_s *caqr_batch_t;

/* Factor `batch` problems.  m, n, lda: host arrays of length batch; A: host
   array of device pointers, A[i] column-major with leading dimension lda[i].
   On return A[i] holds R_i (top n_i-by-n_i upper triangle, non-negative
   diagonal) and the reflectors of problem i, as after tsqr_factor.  dt is the
   element type of every A[i]: CAQR_F64 (double) or CAQR_F32 (float).  opts:
   one plan for every problem, or NULL for the plans measured by
   caqr_tune_batched for dt (or a fixed size heuristic before any tuning).
   Errors: CAQR_ERR_INVALID_VALUE for a negative batch, missing arrays, an
   unknown dt, m_i < 0, lda_i < max(1, m_i), a null A[i] with n_i > 0 or
   invalid opts; CAQR_ERR_NOT_SUPPORTED for m_i < n_i,
   n_i > 64 or m_i > 2^31 - 1; CAQR_ERR_ALLOC; CAQR_ERR_DEVICE.  Arguments are checked before
   anything is enqueued.  Work is enqueued on the handle's stream; *F owns the
   per-problem tau, signs and workspace until caqr_batch_destroy (which waits
   for the device).  The caller keeps every A[i] alive while F is used. */
caqr_status_t tsqr_factor_batched(caqr_handle_t h, int64_t batch, const int64_t *m, const int64_t *n,
                                  void *const *A, const int64_t *lda, caqr_dtype_t dt,
                                  const caqr_tree_opts_t *opts, caqr_batch_t *F);

caqr_status_t caqr_batch_destroy(caqr_batch_t F);

/* The plan used for problem i (leaf_rows, leaves_per_wg, arity). */
caqr_status_t caqr_batch_get_plan(caqr_batch_t F, int64_t i, caqr_tree_opts_t *plan);

/* Signs D of problem i (n_i doubles, host memory, also for CAQR_F32 batches);
   waits for the factorization. */
caqr_status_t caqr_batch_get_signs(caqr_batch_t F, int64_t i, double *d);

/* Autotuner: for n in {8, 16, 32, 64} and m in each power-of-two bucket from
   256 to 65536, times every plan (leaf_rows 64/128/256 x (arity,
   leaves_per_wg) in (2, 1), (2, 2), (2, 4), (4, 1), (4, 4))
   on a batch of synthetic problems of element type dt filling the device, and
   keeps the fastest in the handle, one table per dt (launch time only, by HIP
   events).  Later batched calls of that dt with opts == NULL use it: a
   problem takes the plan of its n bucket (the smallest of 8/16/32/64 that is
   >= n_i) and of the power-of-two bucket of m_i (clamped to 256 .. 65536).
   Synchronous; uses a scratch buffer of 2^24 elements of dt (128 MiB for
   CAQR_F64).  Errors: CAQR_ERR_INVALID_VALUE for an unknown dt. */
caqr_status_t caqr_tune_batched(caqr_handle_t h, caqr_dtype_t dt);

/* The plan a batched call with opts == NULL would use for an m-by-n problem. */
caqr_status_t caqr_batch_plan_for(caqr_handle_t h, int64_t m, int64_t n, caqr_dtype_t dt, caqr_tree_opts_t *plan);

/* Batched least squares: min ||A_i X_i - B_i||_F for `batch` independent
   problems with n_i <= 64 (FP64).  A_i (m_i x n_i, lda_i) is factored in place
   by the batched TSQR (one launch per group, the plan of opts or the
   tuned/default plans); B_i (m_i x nrhs_i, ldb_i) is overwritten by Q_i^T B_i,
   its first n_i rows by X_i.  Q^T is applied with the stored reflectors one at
   a time in the order they were made (leaves, then the tree levels
   bottom-up), so X_i agrees with ls_solve's to rounding, not bitwise.  Waits
   for the device; info (host array of batch entries) receives each problem's
   status (CAQR_ERR_SINGULAR with the first zero pivot, CAQR_ERR_NONFINITE);
   the return value is CAQR_SUCCESS or the first such status.  Errors, before
   anything is enqueued: CAQR_ERR_INVALID_VALUE (negative sizes, leading
   dimensions below max(1, m_i), missing arrays or pointers, invalid opts);
   CAQR_ERR_NOT_SUPPORTED (m_i < n_i, n_i > 64, m_i > 2^31 - 1);
   CAQR_ERR_ALLOC; CAQR_ERR_DEVICE.  Problems with n_i = 0 or nrhs_i = 0 are
   left untouched. */
caqr_status_t ls_solve_batched(caqr_handle_t h, int64_t batch, const int64_t *m, const int64_t *n,
                               const int64_t *nrhs, double *const *A, const int64_t *lda, double *const *B,
                               const int64_t *ldb, const caqr_tree_opts_t *opts, caqr_ls_info_t *info);

/* ------------------------------------------------------------------------ */
/* Served least-squares stream.  Independent requests min ||A_i X_i - B_i||   */
/* (the solve of ls_solve, Section 3 of the paper for the factorization) are */
/* run concurrently on one GPU: `workers` host threads, each with its own    */
/* handle and non-blocking stream, take requests in arrival order as soon as */
/* one is free and the request's device footprint fits in the budget.  The   */
/* footprint is a copy of A (m x n), a copy of B (m x nrhs) and the factors' */
/* workspace, all carved from one device allocation made at creation, so no */
/* device memory is allocated or freed while serving.  A request's result is */
/* bitwise that of ls_solve on the same problem, whatever else is served.    */
/* Each worker drives two streams (its factorization's chain and the wide    */
/* trailing updates); the HIP runtime maps a process's streams onto         */
/* GPU_MAX_HW_QUEUES hardware queues (4 by default), and streams sharing a  */
/* queue run one after the other.  Start the serving process with at least  */
/* 2 x workers queues (e.g. GPU_MAX_HW_QUEUES=16 for 8 workers) for the      */
/* workers to overlap.                                                      */
/* ------------------------------------------------------------------------ */

typedef struct caqr_server_s *caqr_server_t;

typedef struct {
  int32_t device;        /* GPU ordinal */
  int32_t workers;       /* concurrent requests, 1 .. 64 */
  uint64_t budget_bytes; /* device memory for the requests in flight (>= 256) */
  int64_t reserved;      /* must be 0 */
} caqr_server_opts_t;

typedef struct {
  int64_t submit_ns; /* host steady clock (CLOCK_MONOTONIC on Linux), nanoseconds */
  int64_t start_ns;  /* admitted: a worker and the memory were free */
  int64_t end_ns;    /* X written and the request's stream idle */
} caqr_request_times_t;

/* Allocate the budget on the device, create the workers' handles and streams,
   start the workers.  Errors: CAQR_ERR_INVALID_VALUE (NULL arguments, workers
   outside 1..64, budget < 256, reserved != 0); CAQR_ERR_DEVICE (no such GPU);
   CAQR_ERR_ALLOC. */
caqr_status_t caqr_server_create(const caqr_server_opts_t *o, caqr_server_t *S);

/* Queue the solve of min ||A X - B||_F for an m-by-n A (m >= n, column-major,
   lda) and m-by-nrhs B (ldb); the n-by-nrhs solution goes to X (ldx >= n).
   A, B and X are device memory owned by the caller: A and B are only read (the
   server works on copies) and must stay valid and unchanged, and X unused,
   until caqr_server_wait returns for the ticket.  Ordering: `stream` (a
   hipStream_t passed as void*) is the caller's stream that produced A and B
   and last used X; an event recorded on it at submit orders the request's
   device work after everything enqueued there so far.  With stream == NULL
   the caller guarantees that A, B and X are complete on the device (e.g. the
   producing stream synchronized) before the call.  X is complete on the
   device when caqr_server_wait returns.  Returns at once.  Errors (nothing is
   queued): CAQR_ERR_INVALID_VALUE for negative sizes, leading dimensions
   below max(1, m) (max(1, n) for ldx), NULL pointers with nonzero sizes, a
   NULL ticket or server; CAQR_ERR_NOT_SUPPORTED for m < n; CAQR_ERR_ALLOC
   when the request's footprint exceeds the whole budget; CAQR_ERR_DEVICE when
   the ordering event cannot be recorded. */
caqr_status_t caqr_server_submit(caqr_server_t S, int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                 const double *B, int64_t ldb, double *X, int64_t ldx, void *stream,
                                 int64_t *ticket);

/* Block until the request has finished; fill info (status, and the first
   zero pivot for CAQR_ERR_SINGULAR) and times (either may be NULL), and
   release the ticket.  Returns the request's status (as ls_solve would), or
   CAQR_ERR_INVALID_VALUE for an unknown or already released ticket.  Only one
   wait may claim a ticket: a second wait on the same ticket, concurrent or
   later, returns CAQR_ERR_INVALID_VALUE and touches nothing. */
caqr_status_t caqr_server_wait(caqr_server_t S, int64_t ticket, caqr_ls_info_t *info, caqr_request_times_t *times);

/* Finish every queued request, stop the workers and free the server.
   caqr_server_submit and caqr_server_wait may be called from any host
   threads concurrently; caqr_server_destroy must not overlap any other call
   on S, and S is invalid afterwards (tickets not yet waited for are
   released with it). */
caqr_status_t caqr_server_destroy(caqr_server_t S);

#ifdef __cplusplus
}
#endif

#endif /* CAQR_H */
