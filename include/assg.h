/*
 * assg.h -- C ABI of the MI355X (gfx950) adaptive s-step conjugate gradient
 * library.
 *
 * The library solves A x = b for a sparse symmetric positive definite A
 * (Section 1 of Carson, "An adaptive s-step conjugate gradient algorithm with
 * dynamic basis updating") with the improved adaptive s-step CG of
 * Algorithm 5, and with Hestenes-Stiefel CG (Algorithm 1) as a comparator.
 * Every step of a solve runs in the library's HIP kernels on the GPU:
 * matrix powers (2.2)-(2.3), the Gram matrix G = Y^T Y (Section 2), the
 * s-selection (3.2), the inner coordinate updates, the Ritz estimates of
 * Algorithms 3-4, the adaptive c of (4.6), the break rule (4.7), the basis
 * parameter updates (2.7)/(2.8) and the recovery (2.6).
 *
 * Conventions
 *  - All functions return assg_status_t; nothing is thrown across the ABI.
 *    A solve that does not converge is not an error: see info->outcome.
 *  - "device" pointers are HIP device allocations on the handle's device,
 *    owned by the caller and never freed by the library.  "host" pointers are
 *    ordinary host memory owned by the caller.
 *  - Matrices are CSR with int32 row pointers and column indices, FP64
 *    values, both triangles stored, columns sorted within each row,
 *    nnz < 2^31.  The library reads A but never modifies it.
 *  - All work is enqueued on the handle's stream; functions that fill host
 *    results (solve, block controller, basis/Gram) return after that work has
 *    completed.  A handle may be used by one host thread at a time.
 *  - Dense small matrices returned to the host are row-major.  The s-step
 *    basis columns are in interleaved order [p0, r0, p1, r1, ..., p_{s-1},
 *    r_{s-1}, p_s] (the paper's [P, R] order, permuted so that Y_{k,l} is the
 *    leading 2l+1 columns).
 */
#ifndef ASSG_H
#define ASSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASSG_MAX_S 16                      /* largest sigma (s_max) supported  */
#define ASSG_MAX_COLS (2 * ASSG_MAX_S + 1) /* basis columns at s = ASSG_MAX_S  */

typedef struct assg_handle_s* assg_handle_t;

typedef enum {
  ASSG_OK = 0,
  ASSG_ERR_INVALID_ARG = -1,  /* bad pointer, size or option; nothing was enqueued   */
  ASSG_ERR_HIP = -2,          /* a HIP call failed; assg_last_error() has the text   */
  ASSG_ERR_ALLOC = -3,        /* device or pinned allocation failed                  */
  ASSG_ERR_UNSUPPORTED = -4,  /* no usable gfx950 device, or a storage A does not fit */
  ASSG_ERR_NOT_ANALYZED = -5  /* n, nnz, row_ptr or col_idx differ from the last analysis */
} assg_status_t;

/* Outcome of a solve (Section 5 reports converged, diverged "-" and
 * stagnated "- [res]" runs). */
typedef enum {
  ASSG_CONVERGED = 0,  /* true relative residual ||b - A x|| / ||b|| <= tol        */
  ASSG_STAGNATED = 1,  /* 5 failed confirmations without a 10% improvement        */
  ASSG_DIVERGED = 2,   /* a non-finite value appeared in G or in alpha/beta       */
  ASSG_BREAKDOWN = 3,  /* p'^T G B p' <= 0 or r'^T G r' <= 0 (A not SPD in effect) */
  ASSG_MAX_ITER = 4,   /* max_outer or max_iters reached                          */
  ASSG_RUNNING = 5     /* internal: never returned by a completed solve           */
} assg_outcome_t;

/* Polynomial basis of (2.3): monomial (theta=0, gamma=1, mu=0), Newton with
 * Leja-ordered shifts (2.7), or Chebyshev on [lambda_min, lambda_max] (2.8;
 * see assg_basis_params for the coefficients used). */
typedef enum {
  ASSG_BASIS_MONOMIAL = 0,
  ASSG_BASIS_NEWTON = 1,
  ASSG_BASIS_CHEBYSHEV = 2
} assg_basis_t;

/* Method run by assg_solve / assg_batch_solve: Algorithm 5 (default) or one
 * of the comparison methods of Section 5.  The monomial-basis methods
 * ignore opts.basis. */
typedef enum {
  ASSG_IMPROVED = 0,          /* Algorithm 5, c = xi~ of (4.6)                          */
  ASSG_IMPROVED_C_RATIO = 1,  /* Algorithm 5 with c = lambda~max / lambda~min (5.1)     */
  ASSG_IMPROVED_C_ONE = 2,    /* Algorithm 5 with c = 1 (Section 5.1)                   */
  ASSG_OLD_ADAPTIVE = 3,      /* Algorithm 2, monomial basis, constant c = opts.c_const: s~ by
                                 (3.2), break when kappa(Y_{k,s~}) >= eps* / (c eps rho_{j+1}) */
  ASSG_FIXED_SSTEP = 4        /* fixed s-step CG, monomial basis, s_k = sigma, no break   */
} assg_variant_t;

/* Sparse SPD matrix, CSR, all arrays device pointers (caller-owned). */
typedef struct {
  int64_t n;               /* rows = columns, 1 <= n < 2^31                      */
  int64_t nnz;             /* entries, 1 <= nnz < 2^31                           */
  const int32_t* row_ptr;  /* n + 1, row_ptr[0] = 0, row_ptr[n] = nnz            */
  const int32_t* col_idx;  /* nnz, in [0, n), sorted within each row              */
  const double* val;       /* nnz                                                 */
} assg_csr_t;

/* Inputs of Algorithm 5 besides A, b and x0. */
typedef struct {
  int32_t s_max;       /* sigma: largest s_k, 1..ASSG_MAX_S (default 10)          */
  int32_t s_init;      /* s-bar_0, 1..s_max; 0 (the default) means s_max          */
  int32_t growth;      /* f >= 1: s-bar_k = min(s_{k-1} + f, sigma); 0 (default): s_max */
  int32_t basis;       /* assg_basis_t (default ASSG_BASIS_CHEBYSHEV)             */
  double tol;          /* eps*: relative residual target, (0, 1) (default 1e-10)  */
  int64_t max_outer;   /* cap on outer loops; 0 -> max_iters                      */
  int64_t max_iters;   /* cap on total inner iterations; 0 -> 10 n               */
  int32_t record_trace;/* 1: keep one assg_trace_t per outer loop (assg_get_trace) */
  int32_t time_kernels;/* 1: time the matrix-powers kernels with HIP events       */
  int32_t variant;     /* assg_variant_t (default ASSG_IMPROVED)                  */
  int32_t pad0;
  double c_const;      /* c of ASSG_OLD_ADAPTIVE, > 0 (default 1)                 */
} assg_opts_t;

/* Result of a solve (host struct filled by the library). */
typedef struct {
  int32_t outcome;          /* assg_outcome_t                                     */
  int32_t pad0;
  int64_t outer_iters;      /* outer loops completed (= global synchronizations;  */
                            /* a loop ending in breakdown/divergence not counted) */
  int64_t total_iters;      /* inner iterations m                                 */
  double relres_updated;    /* (r'^T G r')^{1/2} / ||b|| at the end               */
  double relres_true;       /* ||b - A x|| / ||b|| of the returned x              */
  double lambda_min_est;    /* Algorithm 4 estimate                               */
  double lambda_max_est;    /* Algorithm 3 estimate                               */
  double c_last;            /* last c of (4.6)                                    */
  double solve_ms;          /* device time from first to last kernel (HIP events) */
  /* filled when opts.time_kernels = 1 (0 otherwise); loops after convergence
   * that were enqueued speculatively are excluded */
  double sweep_ms;          /* two-chain matrix-powers sweeps, levels >= 2        */
  int64_t sweep_launches;
  double sweep1_ms;         /* first sweep (no mu term)                           */
  int64_t sweep1_launches;
  double last_gram_ms;      /* last sweep fused with the Gram partial sums        */
  int64_t last_gram_launches;
  double other_ms;          /* Gram reduction + controller + recovery + checks    */
} assg_info_t;

/* One record per outer loop (opts.record_trace = 1). */
typedef struct {
  int32_t k;            /* outer loop index                                      */
  int32_t sbar;         /* s-bar_k: levels of the basis built                    */
  int32_t stilde;       /* s~_k from (3.2)                                       */
  int32_t sk;           /* s_k: inner iterations done                            */
  int64_t m;            /* iterations done before this loop                      */
  int32_t candidate;    /* 1: the updated residual reached tol in this loop      */
  int32_t flags;        /* bit0 breakdown, bit1 non-finite                       */
  double c_in;          /* c used by (3.2) in this loop                          */
  double thr;           /* tol / (c u ||r_m||/||b||)                             */
  double rho_m;         /* ||r_m|| / ||b|| from G                                */
  double phi;           /* max relative residual in the loop (4.7)               */
  double c;             /* c after the loop                                      */
  double lmin, lmax;    /* Ritz estimates after the loop                         */
  double psi;           /* psi after the loop (4.5)                              */
  double relres_updated;/* updated relative residual after the loop             */
  double relres_true;   /* true relative residual if checked (else -1)          */
  double kappa[ASSG_MAX_S]; /* kappa(Y_{k,l}) for l = 1..sbar (index l-1)        */
} assg_trace_t;

/* Carried state of Algorithm 5 between outer loops, for assg_block_controller. */
typedef struct {
  int64_t m;                 /* iterations done                                  */
  double c;                  /* current c (c_1 = u^{-1/2} before the first update) */
  double psi;                /* psi_m (4.5)                                      */
  double alpha_prev, beta_prev;
  double mt_max_omega, mt_max_h, mt_max_zeta;            /* Algorithm 3 state   */
  double mt_min_omega, mt_min_a, mt_min_d, mt_min_g, mt_min_h; /* Algorithm 4   */
  double lmin, lmax;         /* current estimates (NaN before the first update)  */
  double theta[ASSG_MAX_S], gamma[ASSG_MAX_S], mu[ASSG_MAX_S]; /* basis in use  */
} assg_block_state_t;

/* Result of one controller pass (one outer loop's small dense work). */
typedef struct {
  int32_t stilde, sk, candidate, flags;
  double thr, rho_m, phi, relres_updated;
  double kappa[ASSG_MAX_S];                  /* kappa(Y_{k,l}), l = 1..sbar      */
  double alpha[ASSG_MAX_S], beta[ASSG_MAX_S];/* coefficients of the sk steps     */
  double coef_x[ASSG_MAX_COLS];              /* x' (interleaved)                 */
  double coef_r[ASSG_MAX_COLS];              /* r'                               */
  double coef_p[ASSG_MAX_COLS];              /* p'                               */
} assg_block_result_t;

/* ---------------------------------------------------------------- basics */

/* Fills *o with the defaults listed in assg_opts_t.  Host only. */
assg_status_t assg_default_opts(assg_opts_t* o);

/* Static text for a status code.  Host only. */
const char* assg_status_string(assg_status_t s);

/* Text of the last HIP or validation error on this handle ("" if none). */
const char* assg_last_error(assg_handle_t h);

/* sizeof of the public structs, in the order assg_opts_t, assg_info_t,
 * assg_trace_t, assg_block_state_t, assg_block_result_t, assg_csr_t,
 * assg_tune_class_t; lets a binding check its layout.  Host only.  Returns
 * the count written (<= cap). */
int32_t assg_struct_sizes(int64_t* sizes, int32_t cap);

/* Creates a handle on the current HIP device.  ``stream`` is a hipStream_t
 * (NULL = the device's null stream); the caller's stream is only ordered
 * against (events), the library enqueues its kernels on a private
 * non-blocking stream of default priority.  Fails with ASSG_ERR_UNSUPPORTED
 * when no device is present. */
assg_status_t assg_create(assg_handle_t* h, void* stream);
assg_status_t assg_destroy(assg_handle_t h);
assg_status_t assg_set_stream(assg_handle_t h, void* stream);

/* Basis parameters the library uses (host, no GPU needed): writes s entries
 * of theta and gamma and s-1 of mu for the given kind and interval.
 *  - monomial: theta = 0, gamma = 1, mu = 0 (Section 2);
 *  - Newton (2.7): gamma = 1, mu = 0, theta_0 = lambda_max, theta_1 =
 *    lambda_min, theta_l = c + h t_l (c = (lmin+lmax)/2, h = (lmax-lmin)/2)
 *    with t_l the Leja points of [-1, 1] in the order of (2.7), a tie at
 *    equal products broken towards the smaller t;
 *  - Chebyshev (2.8) read as the Chebyshev recurrence of [lmin, lmax]:
 *    theta = (lmin+lmax)/2, gamma_0 = (lmax-lmin)/2, gamma_l = mu_l =
 *    (lmax-lmin)/4, so rho_l(z) = T_l(2 (z - theta)/(lmax - lmin)).
 * INVALID_ARG unless 1 <= s <= ASSG_MAX_S and lmin < lmax for Newton and
 * Chebyshev. */
assg_status_t assg_basis_params(int32_t kind, double lmin, double lmax, int32_t s,
                                double* theta, double* gamma, double* mu);

/* Device workspace needed by assg_solve / assg_hscg_solve for n rows and
 * sigma = s_max (the basis Y of (2.2): s_max pair vectors + one vector, plus
 * reduction partials).  Host only. */
assg_status_t assg_workspace_size(int64_t n, int32_t s_max, size_t* bytes);

/* Prepares A for the kernels: reads row_ptr once (device -> host) and cuts
 * the rows into the row blocks of the CSR-stream kernels (at most 256 rows
 * and 2048 nonzeros each; a longer row is a block of its own).  Checks
 * row_ptr (starts at 0, ends at nnz, nondecreasing) on the host and every
 * column index against [0, n) on the device; a failed check returns
 * ASSG_ERR_INVALID_ARG and leaves the handle with no analysis (solves then
 * return ASSG_ERR_NOT_ANALYZED).  Must be called again when the sparsity
 * pattern changes (row_ptr and col_idx must not change between analysis
 * and solve); values may change freely between solves. */
assg_status_t assg_analyze(assg_handle_t h, const assg_csr_t* A);

/* Storage the matrix-powers kernels read A from, chosen by the next
 * assg_analyze or assg_batch_analyze (a batch takes the diagonal storage
 * only when every system fits it, each system with its own diagonals):
 *  - ASSG_FORMAT_AUTO (the default): diagonal storage when every entry of A
 *    lies on one of at most 32 diagonals (i, i + off) and those diagonals
 *    hold at most 15% more positions than A has entries (stencil matrices),
 *    else CSR;
 *  - ASSG_FORMAT_CSR: CSR always;
 *  - ASSG_FORMAT_DIA: diagonal storage whatever its fill, or
 *    ASSG_ERR_UNSUPPORTED from the analysis when some entry lies off 32
 *    diagonals (the handle is then left with no analysis of that kind).
 * The diagonal storage is the library's copy of A's values, n per diagonal
 * (0 where A has no entry), allocated at analysis and refreshed from the CSR
 * values at the start of every solve and assg_basis_gram call, so values
 * may still change between calls.  It is read by the matrix-powers sweeps,
 * the last sweep with the Gram partials and HSCG's product A p; the setup,
 * the true-residual check, assg_spmv and the gradient scatter read CSR.
 * Each row's products are added in column order as in the CSR kernels, so
 * rows agree bit for bit; grid-wide sums agree too when both storages cut
 * the rows into the same 256-row blocks (at most 8 entries per row), and up
 * to rounding otherwise.  INVALID_ARG for another format value. */
typedef enum {
  ASSG_FORMAT_AUTO = 0,
  ASSG_FORMAT_CSR = 1,
  ASSG_FORMAT_DIA = 2
} assg_format_t;
assg_status_t assg_set_format(assg_handle_t h, int32_t format);

/* The storage the last successful analysis chose (ASSG_FORMAT_CSR or
 * ASSG_FORMAT_DIA); ASSG_ERR_NOT_ANALYZED when there is none. */
assg_status_t assg_get_format(assg_handle_t h, int32_t* format);

/* The storage the last batch analysis chose; ASSG_ERR_NOT_ANALYZED when
 * there is none. */
assg_status_t assg_batch_format(assg_handle_t h, int32_t* format);

/* ------------------------------------------------------------- the solves */

/* Algorithm 5: improved adaptive s-step CG (or a comparison method, see
 * opts.variant).  b (device, n) is read; x (device, n) holds x0 on entry and
 * the solution on return; b and x must not overlap (ASSG_ERR_INVALID_ARG).  ``workspace`` (device, >= assg_workspace_size
 * bytes) may be NULL, in which case the handle allocates and keeps one.
 * info (host) receives the outcome and iteration counts.  The relative
 * residual is ||b - A x|| / ||b||; with b = 0 the result is x = 0,
 * CONVERGED.  Every decision is taken on the device: the kernels of 4 outer
 * loops are captured once into a HIP graph (kept on the handle while the
 * pointers, sizes and s_max stay the same) and replayed, the host reading
 * the status word between replays; loops replayed after the end exit at
 * once.  With opts.time_kernels = 1 the same kernels are launched one by one
 * instead, with HIP events around the matrix-powers launches. */
assg_status_t assg_solve(assg_handle_t h, const assg_csr_t* A, const double* b, double* x,
                         const assg_opts_t* opts, void* workspace, size_t workspace_bytes,
                         assg_info_t* info);

/* assg_solve with the s-step schedule of its first loops given, for tests
 * that separate arithmetic from decisions.  Algorithm 5 compares
 * kappa(Y_{k,l}) and the residuals against thresholds ((3.2), (4.7), the
 * stopping test), so two correct implementations whose roundings differ can
 * take different s_k near a threshold and follow different trajectories;
 * replaying one schedule removes that freedom.  Loop k < nsk runs exactly
 * sk[k] inner steps (sk: host array of nsk >= 1 entries, 1 <= sk[k] <=
 * s-bar_k with s-bar_0 = s_init and s-bar_k = min(sk[k-1] + growth, s_max),
 * else ASSG_ERR_INVALID_ARG): the selection (3.2), the break (4.7) and the
 * in-loop stopping test are not applied there (kappa is still computed and
 * traced).  Loop nsk - 1 ends with the true-residual check; if it does not
 * confirm convergence the solve goes on as assg_solve would (opts.max_outer
 * and max_iters still apply).  Everything else, kernels included, is
 * assg_solve's; the handle keeps a device copy of the schedule. */
assg_status_t assg_solve_forced_schedule(assg_handle_t h, const assg_csr_t* A, const double* b,
                                         double* x, const assg_opts_t* opts, const int32_t* sk,
                                         int64_t nsk, void* workspace, size_t workspace_bytes,
                                         assg_info_t* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): assg_solve
 * with no workspace argument and no allocation of any kind inside the call.
 * The basis and the Gram partials live in a static device array of
 * ASSG_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU the library runs on holds
 * until the process ends; the call refuses (ASSG_ERR_INVALID_ARG) a system
 * whose assg_workspace_size(n, opts.s_max) exceeds it (about 354,000 rows at
 * s_max = 10), and opts.record_trace and opts.time_kernels must be 0.  The
 * handle (assg_create) and the analysis (assg_analyze) allocate as usual, so
 * they come before.  The outer loops are launched one by one (no graph
 * capture), with the same kernels and results as assg_solve.  Every call on
 * a GPU uses that GPU's one array: calls that overlap on one GPU (other
 * handles, other host threads, other streams) race and must not be issued;
 * nothing in the array needs to start at zero. */
#define ASSG_NOALLOC_SCRATCH_BYTES (64u << 20)
#define ASSG_MAX_DEVICES 64   /* devices with a scratch address table entry */
assg_status_t assg_solve_noalloc(assg_handle_t h, const assg_csr_t* A, const double* b, double* x,
                                 const assg_opts_t* opts, assg_info_t* info);

/* Algorithm 1 (HSCG) on the GPU: one SpMV with a fused p^T A p partial sum,
 * one update kernel with a fused r^T r partial sum and one direction update
 * per iteration; stopping as for assg_solve (updated residual <= tol, then
 * the true residual decides). */
assg_status_t assg_hscg_solve(assg_handle_t h, const assg_csr_t* A, const double* b, double* x,
                              double tol, int64_t max_iters, void* workspace,
                              size_t workspace_bytes, assg_info_t* info);

/* Copies the trace of the last assg_solve (opts.record_trace = 1) into host
 * memory: at most cap records, *count = records available. */
assg_status_t assg_get_trace(assg_handle_t h, assg_trace_t* host_buf, int64_t cap,
                             int64_t* count);

/* ---------------------------------------------------------------- batches */

#define ASSG_MAX_BATCH 2048   /* systems per batch */

/* Prepares a batch of nsys independent systems (A: host array of nsys CSR
 * descriptors of device matrices, each as for assg_analyze and checked the
 * same way, 1 <= nsys <= ASSG_MAX_BATCH, total rows and nonzeros < 2^31;
 * after a failed check the handle holds no batch).  The handle keeps one
 * block-diagonal copy of the patterns (the systems' rows and columns
 * concatenated; values are copied again at every solve), cuts row blocks
 * that never straddle systems, and picks the row-block shape of the
 * CSR-stream kernels for each size class of systems by timing products
 * (or from the process cache): see assg_batch_tuning.  Replaces any
 * previous batch of the handle; the single solve's analysis is kept. */
assg_status_t assg_batch_analyze(assg_handle_t h, int32_t nsys, const assg_csr_t* A);

/* Algorithm 5 on every system of the analyzed batch at once.  Each kernel
 * launch covers all systems; every system keeps its own control block
 * (s-bar, s~, s_k, coefficients, Ritz estimates, c, basis parameters,
 * stopping) and its blocks are skipped once it has stopped.  The outer loops
 * run from a captured HIP graph (4 loops per replay), so the host enqueues
 * one graph launch per 4 loops and reads the systems' states in between.
 * A, nsys: as given to assg_batch_analyze (same row_ptr pointers, values may
 * differ).  b, x: host arrays of nsys device pointers (n_i doubles each); x[i]
 * holds x0 on entry and the solution on return.  opts apply to every system
 * (record_trace must be 0, time_kernels is ignored).  info: host array of
 * nsys results; solve_ms is the time of the whole batch. */
assg_status_t assg_batch_solve(assg_handle_t h, int32_t nsys, const assg_csr_t* A,
                               const double* const* b, double* const* x, const assg_opts_t* opts,
                               assg_info_t* info);

/* The batch tuner.  Systems fall into size classes by rows (class 0: n <
 * 4,096; 1: < 65,536; 2: < 1,048,576; 3: larger).  For each class present,
 * assg_batch_analyze times one product over that class's systems with each
 * candidate row-block shape (rows per block / nonzero cap: 256/2048,
 * 256/1024, 128/2048, 128/1024, 64/1024, 64/512) and keeps the fastest; the
 * choice is cached for the process by (class, average nonzeros per row of
 * the class rounded to an integer), and a later analysis with the same key
 * reuses it without timing. */
#define ASSG_TUNE_CLASSES 4
#define ASSG_TUNE_SHAPES 6
typedef struct {
  int32_t systems;      /* systems of the batch in this class (0: none)               */
  int32_t rows;         /* chosen rows per block                                       */
  int32_t nnz_cap;      /* chosen nonzeros per block                                   */
  int32_t cached;       /* 1: taken from the process cache, candidate_us all 0         */
  double candidate_us[ASSG_TUNE_SHAPES]; /* product time of each candidate shape (us)  */
} assg_tune_class_t;

/* The tuner's result for the last assg_batch_analyze: classes (host) receives
 * ASSG_TUNE_CLASSES records, in class order. */
assg_status_t assg_batch_tuning(assg_handle_t h, assg_tune_class_t* classes);

/* ------------------------------------------------------- differentiation */

/* out[k] = alpha * u[row(k)] * v[col(k)] for every stored nonzero k of A:
 * the entries of alpha u v^T on A's sparsity pattern.  With x = A^{-1} b and
 * a loss L(x), the adjoint solution lambda = A^{-1} dL/dx (A is symmetric, so
 * the adjoint system has the same matrix) gives dL/db = lambda and
 * dL/dA_ij = -lambda_i x_j; with alpha = -1, u = lambda, v = x this call
 * writes the gradient with respect to A's stored values (every stored entry
 * counted as its own variable).  u, v (device, n), out (device, nnz; may not
 * alias u or v).  Returns after the kernel has completed. */
assg_status_t assg_csr_outer_on_pattern(assg_handle_t h, const assg_csr_t* A, const double* u,
                                        const double* v, double alpha, double* out);

/* ------------------------------------------ single steps of the hot path */

/* y = A x (device x, y; n each; x and y must not overlap). */
assg_status_t assg_spmv(assg_handle_t h, const assg_csr_t* A, const double* x, double* y);

/* The basis and Gram matrix of one outer loop with given parameters:
 * Y_{k,s} of (2.2) built by (2.3) from p and r (device, n each) with theta,
 * gamma (s entries) and mu (s-1 entries, host arrays), then G = Y^T Y.
 * Y_out (device, may be NULL) receives the 2s+1 columns column-major with
 * leading dimension n, interleaved order; G_out (host) the (2s+1)^2 matrix,
 * row-major, interleaved order.  Runs the same kernels as assg_solve. */
assg_status_t assg_basis_gram(assg_handle_t h, const assg_csr_t* A, const double* p,
                              const double* r, int32_t s, const double* theta,
                              const double* gamma, const double* mu, double* Y_out,
                              double* G_out);

/* One controller pass of Algorithm 5 (the device kernel assg_solve uses) on a
 * given Gram matrix: kappa of the leading blocks and s~ by (3.2), the inner
 * loop with alpha/beta through G, phi, psi, Algorithms 3/4, c (4.6), the
 * break (4.7) and the stopping candidate.  G (host) is (2 sbar+1)^2,
 * row-major, interleaved order; nb = ||b||; ``state`` (host) is read and
 * updated (m, c, psi, Ritz state; theta/gamma/mu are updated for the next
 * loop when m > 1, using ``basis`` and s_max).  ``res`` (host) receives s~,
 * s_k, the coefficients and the recovery coordinates. */
assg_status_t assg_block_controller(assg_handle_t h, const double* G, int32_t sbar, double nb,
                                    double tol, int32_t basis, int32_t s_max,
                                    assg_block_state_t* state, assg_block_result_t* res);

#ifdef __cplusplus
}
#endif

#endif /* ASSG_H */
