/*
 * tls.h -- C ABI of the MI355X total-least-squares library (libtls.so).
 *
 * The library solves the total least squares problem
 *     min ||[E, r]||_F  subject to  (A + E) x = b + r,   A m x n, m > n,
 * (Oktay & Carson, "Mixed Precision Rayleigh Quotient Iteration for Total
 * Least Squares Problems", abstract and Section 1) by Rayleigh quotient
 * iteration on [A, b] (Algorithm 2, RQI-PCGTLS), whose two inner solves
 * (A^T A - sigma^2 I) w = rhs run the preconditioned conjugate gradient
 * method PCGTLS (Algorithm 3) with an upper triangular factor R of A^T A.
 * The precisions follow Algorithm 4 (RQI-PCGTLS-MP): outer iteration in
 * u = FP64, PCGTLS in u_p, factor in u_q.
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless the comment says (host).
 *  - The caller owns all device memory: matrices, vectors and workspaces.
 *    The library never allocates device memory. Workspace sizes come from
 *    the *_workspace_size queries; workspaces must be 256-byte aligned.
 *  - Work is enqueued on the given stream. tls_factor_precond synchronizes
 *    it once per factorization attempt (breakdown and finite-input flags),
 *    and waits for the gate's runs only when a report is requested;
 *    tls_rqi_solve waits once per outer iteration for psi of eq. (4) (an
 *    event behind its copy; unless strict_pd is set, the iteration's two
 *    PCGTLS solves and update are enqueued before the wait, and the run
 *    past the last iteration is discarded) and synchronizes at the few
 *    decisions that need a value on the host; tls_pcg_step
 *    and tls_apply_precond are asynchronous unless a host trace is
 *    requested.
 *  - Every call returns a tls_status; no C++ exception crosses the ABI;
 *    tls_last_error() returns a thread-local message for the last failure.
 *  - Results are deterministic: reductions use a fixed order, so repeated
 *    calls on the same inputs give bitwise identical outputs.
 *  - Calls that share a workspace or a preconditioner must not overlap in
 *    time (they use synchronisation counters inside the workspace).
 *  - The gate of a low-precision factor (two Lanczos runs) executes on one
 *    library-owned stream per device (default priority, non-blocking,
 *    created on first use, kept until the process ends), forked from the
 *    caller's stream after the factorization. Its scalars come back through
 *    a small pinned host block per preconditioner (pooled per device, kept
 *    for reuse). See tls_factor_precond for when the caller may see the runs
 *    still going.
 */
#ifndef TLS_H
#define TLS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define TLS_API __attribute__((visibility("default")))
#else
#define TLS_API
#endif

/* Precisions (Table 2, plus bfloat16, which the paper does not use). */
/* TLS_BF16X3 (factor precision only, Cholesky route): each entry a of the
 * scaled A D^{-1} is split into two BF16 numbers, hi = bf16(a) and
 * lo = bf16(a - hi); the Gram matrix is hi^T hi + hi^T lo + lo^T hi on the
 * BF16 matrix cores with FP32 accumulation (lo^T lo, below 2^-16 relative,
 * is dropped) and the factor is computed and stored in FP32. Its unit
 * roundoff for the constraints of Section 3.1 is taken as 2^-16. */
typedef enum { TLS_FP64 = 0, TLS_FP32 = 1, TLS_FP16 = 2, TLS_BF16 = 3, TLS_BF16X3 = 4 } tls_prec;

/* Storage format of A. */
typedef enum { TLS_DENSE_COLMAJOR = 0, TLS_CSR = 1 } tls_format;

typedef enum {
  TLS_OK = 0,
  TLS_ERR_ARG = -1,            /* invalid argument (shape, null pointer, size)          */
  TLS_ERR_HIP = -2,            /* a HIP runtime call failed                             */
  TLS_ERR_NOT_SPD = -3,        /* Cholesky breakdown: non-positive pivot                */
  TLS_ERR_PRECISION = -4,      /* the u_q gate rejected the factor, escalation disabled  */
  TLS_ERR_INDEFINITE = -5,     /* delta_j <= 0 in PCGTLS with strict checking on        */
  TLS_ERR_NONUNIQUE = -6,      /* sigma_{n+1} estimate >= sigma'_n estimate (Section 2) */
  TLS_ERR_NO_CONVERGENCE = -7, /* kmax reached without the psi rule firing              */
  TLS_ERR_WORKSPACE = -8,      /* workspace too small or misaligned                     */
  TLS_ERR_NONFINITE = -9,      /* NaN or Inf in A or b                                  */
  TLS_ERR_SYNC_TIMEOUT = -10   /* an inter-workgroup wait exceeded its spin bound       */
} tls_status;

/* The data matrix A (m x n, m > n). Dense: column-major, element (i, j) at
 * val[i + j*ld], ld >= m. CSR: row_ptr[m+1] (row_ptr[0] = 0, nondecreasing,
 * row_ptr[m] = nnz), col_idx[nnz] in [0, n) strictly increasing within each
 * row, val[nnz]. tls_factor_precond checks this structure on the device
 * before any kernel uses the indices (one synchronization) and returns
 * TLS_ERR_ARG for a matrix that violates it; tls_rqi_solve accepts a CSR A
 * only with the same index arrays (pointers, m, nnz) the preconditioner was
 * built from. All arrays are device memory owned by the caller and must stay
 * valid and unchanged while a preconditioner built from A is in use. */
typedef struct {
  int32_t format;          /* tls_format */
  int32_t reserved;
  int64_t m, n;
  int64_t ld;              /* dense only */
  int64_t nnz;             /* CSR only   */
  const double *val;
  const int32_t *row_ptr;  /* CSR only   */
  const int32_t *col_idx;  /* CSR only   */
} tls_matrix;

/* Opaque preconditioner: a small host object owned by the library that
 * points into the caller's factor workspace (which must outlive it). */
typedef struct tls_precond_s *tls_precond;

/* Outcome of the per-instance check of the factorization precision u_q
 * against the constraints of Section 3.1 (the constants the paper drops
 * are taken as one). Estimates come from Lanczos on R^{-T} R^{-1}; they are
 * only as good as the factor, so with tls_rqi_solve's gate on, the factor is
 * also certified by Lanczos on R^{-T} A^T A R^{-1} (the operator whose
 * distance from I the analysis of Section 3.1 bounds). */
typedef struct {
  double kappa_est;        /* kappa(A D^{-1}) estimate (D = I when unscaled)   */
  double kappaF_est;       /* kappa_F(A D^{-1}) = ||A D^{-1}||_F / sigma_min    */
  double sigma_n_est;      /* sigma'_n(A) estimate                              */
  double sigma_1_est;      /* sigma'_1(A) estimate                              */
  double lam_min_H;        /* lambda_min(H), H = D^{-1} A^T A D^{-1}            */
  double bound5;           /* u_q <~ kappa^{-1}                    (eq. 5)       */
  double bound_chol;       /* u_q <~ kappa^{-2}        (Cholesky of fl(A^T A))   */
  double bound_wilkinson;  /* 1/(20 n^{3/2} kappa^2)                             */
  double bound_hp;         /* lam_min(H)/((2 lam_min(H) + n)(n+1))  (scaled)     */
  double bound6;           /* kappa_F^{-1}(1 - sigma_{n+1}^2/sigma'_n^2) (eq. 6);
                              filled by tls_rqi_solve, which knows b             */
  double u_q;              /* unit roundoff of the precision finally used        */
  double ctilde_min;       /* lambda_min estimate of C = I - s0^2 R^{-T}R^{-1}   */
  double quality_lo;       /* extreme Ritz values of R^{-T} A^T A R^{-1}: the    */
  double quality_hi;       /* a-posteriori certificate (six Lanczos steps,
                              products with A and R in FP64; for a dense A the
                              products ride on tls_rqi_solve's passes over A) */
  double cert_margin;      /* the window [1/2, 3/2] is narrowed by this much on
                              each side (0.05): Ritz values lie inside the
                              spectrum they estimate                           */
  int32_t requested;       /* tls_prec asked for                                 */
  int32_t used;            /* tls_prec actually used (after escalation)          */
  int32_t verdict;         /* bit 0: (5) holds, 1: kappa^-2 holds, 2: HP holds,
                              3: (6) holds, 4: a-posteriori certificate holds:
                              quality_lo - cert_margin >= 1/2 and quality_hi +
                              cert_margin <= 3/2 (the factor is within 50% of
                              A^T A in every direction),
                              5: the solve's sigma lies below the estimate of
                              sigma'_n (the smallest-root check)               */
  int32_t escalations;     /* times u_q was raised                               */
  int32_t chol_retries;    /* diagonal-shift retries after breakdown             */
  int32_t lanczos_steps;
  int32_t method;          /* 0: Cholesky of the Gram matrix, 1: Householder QR  */
  int32_t reserved;
} tls_gate_report;

#define TLS_MAX_ITERS 256

/* Warm-start network (a project addition; see tls_mlp_forward). */
#define TLS_MLP_IN 32
#define TLS_MLP_WIDTH 256
#define TLS_MLP_PARAMS 140289   /* 32*256+256 + 2*(256*256+256) + 256+1 */

/* Options of tls_rqi_solve. tls_default_opts() fills the plain FP64 path. */
typedef struct {
  int32_t u_p;             /* tls_prec of PCGTLS: TLS_FP64 or TLS_FP32            */
  int32_t kmax;            /* maximum RQI iterations, 1..TLS_MAX_ITERS            */
  int32_t stop_patience;   /* psi rule (eq. 4): stop after this many iterations
                              without a new smallest psi; 1 = stop at the first
                              increase, as printed. The loop also ends when psi
                              is 0 or exactly repeats the previous psi          */
  int32_t stop_ge;         /* 1: psi_{k+1} >= psi_k also counts (Example 2)      */
  int32_t ls_corrections;  /* corrections of x_LS by semi-normal equations        */
  int32_t strict_pd;       /* 1: delta_j <= 0 in PCGTLS is an error              */
  int32_t shift_clamp;     /* 1: shift = min(sigma_k^2, tau * sigma'_n estimate^2) */
  int32_t refine_sweeps;   /* final FP64 refinement RQI steps (explicit operator) */
  int32_t refine_pcg_steps;/* maximum PCG steps per refinement solve (it stops
                              earlier once r^T M r has fallen by 1e-26)           */
  int32_t allow_escalate;  /* raise u_q when the gate's certificate fails, or when
                              a gated solve on a low-precision factor ends
                              without convergence (see tls_rqi_solve)           */
  int32_t gate_enforce;    /* 1: run the b-dependent gate                         */
  int32_t features;        /* 1: compute the warm-start features (stats.features)
                              even when no warm start is requested                */
  int32_t min_inner_steps; /* the k-th PCGTLS runs take l = max(k, this) (l + 1
                              steps); 0 = l = k as in Algorithm 2. For starts
                              far above sigma_{n+1}, where k + 1 steps leave the
                              early Newton systems unsolved (0..4096)            */
  int32_t step_margin;     /* PCGTLS steps launched per run beyond those the
                              latest run read back executed (default 1; 0 =
                              launch all l + 1). Algorithm 3 ends a run early
                              at its exits, and the steps after its end cost a
                              short launch each; a run that ends within
                              e + step_margin steps is unchanged by the cap,
                              one that would run longer stops there (within
                              Algorithm 2's at most k + 1 steps), and a run
                              that used every step it was given lifts the cap
                              for the next (0..4096)                             */
  double shift_clamp_tau;  /* tau of the clamp (0 < tau < 1)                       */
  double sigma0_hint;      /* warm start from a given shift estimate sigma_hat
                              (<= 0: none; ignored when mlp_theta is set)         */
  double psi_tie;          /* the returned iterate is the latest x_k whose psi_k
                              is within this factor (>= 1; default 4) of the
                              smallest psi seen up to k: psi values that close
                              sit at the rounding floor of eq. (4), where psi no
                              longer tells iterates apart but RQI's iterates
                              still converge. 1 = the last one that attained the
                              minimum. A value below 1 is TLS_ERR_ARG.            */
  double *x_snapshots;     /* device, optional (kmax * n): x_k at each psi_k       */
  const float *mlp_theta;  /* device, optional: warm-start network parameters
                              (TLS_MLP_PARAMS floats); NULL = plain LS start      */
  const float *mlp_norm;   /* device: input standardisation [mean(32), scale(32)] */
} tls_rqi_opts;

/* Per-call record of the iteration (host). */
typedef struct {
  int32_t iters;           /* number of psi_k evaluated (k = 1..iters)            */
  int32_t k_best;          /* k of the returned iterate (smallest psi)            */
  int32_t pcg_steps;       /* PCGTLS steps launched per right-hand side (a run
                              executes fewer when it ends at its exits)          */
  int32_t warm_used;       /* 1 when the warm-start step was kept                 */
  int32_t stopped;         /* 0 psi rule, 1 kmax, 2 fixed point (psi == 0 or psi
                              repeated exactly)                                   */
  int32_t negative_delta;  /* PCGTLS steps that met delta_j < 0 in the last run
                              enqueued (with the lookahead, the discarded one)  */
  int32_t refine_steps;    /* refinement RQI steps taken                          */
  int32_t clamped;         /* iterations whose shift was clamped                  */
  int32_t gate_async;      /* 1: the gate's Lanczos runs were still in flight when
                              the iterations began (they overlapped the solve and
                              were read at a later host synchronisation)          */
  int32_t ls_refined;      /* != 0: the start was found outside the SPD region
                              and a second solve ran from x_LS recomputed to
                              convergence (|ls_refined| - 1 extra corrections);
                              > 0 its result is returned, < 0 the first one
                              (smaller sigma); see tls_rqi_solve                  */
  double sigma_ls;         /* sigma_0 = ||r_0|| / sqrt(1 + ||x_LS||^2)             */
  double psi[TLS_MAX_ITERS];
  double sigma[TLS_MAX_ITERS];
  double t_ms[TLS_MAX_ITERS]; /* host time since the call began when psi_k was read */
  double t_factor_ms;      /* time in escalation refactoring, if any               */
  double t_total_ms;
  double sigma_final;      /* sigma after the compensated residual                 */
  double sigma_hat;        /* warm-start shift estimate (0 when none)              */
  double psi_warm, psi_plain; /* psi at the warm and at the plain x_1 (warm start)  */
  double t_verdict_ms;     /* host time since the call began when the gate's
                              verdict (constraint (6) and the factor certificate)
                              was taken; an iterate is only usable from then on.
                              0 when no gate ran                                  */
  float features[TLS_MLP_IN]; /* warm-start features (when computed)              */
} tls_rqi_stats;

/* ---------------------------------------------------------------------------
 * Preconditioner (Section 2: Cholesky factor of A^T A, computed once;
 * Section 3.1: computed in precision u_q with two-sided diagonal scaling).
 * ------------------------------------------------------------------------- */

/* Bytes of workspace tls_factor_precond needs for A and u_q (covers every
 * escalation up to FP64). */
TLS_API size_t tls_factor_workspace_size(const tls_matrix *A, int32_t u_q);

/* Build R with R^T R ~ A^T A. With scaling = 1, D = diag(||A e_j||), the
 * columns of A D^{-1} are rounded to u_q, H = (A D^{-1})^T (A D^{-1}) is
 * accumulated in FP32 (FP64 when u_q = FP64), Cholesky gives R_hat, stored
 * in u_q, and R = R_hat D. scaling = 0 factors A^T A itself (FP64 only).
 * For u_q below FP64 the gate runs two Lanczos processes on the factor:
 * 8 steps on (R^T R)^{-1}, giving the estimates of kappa and sigma'_n behind
 * the A-only constraints of Section 3.1 (verdict bits 1, 2, 4), and 6 steps
 * on R^{-T} A^T A R^{-1}, whose extreme Ritz values (quality_lo, quality_hi)
 * are the a-posteriori certificate of the factor read by tls_rqi_solve.
 * The estimates run on a library side stream; the certificate runs beside
 * them on a second one (CSR) or rides on the solve's passes over the row
 * copy (dense, n <= 4096). With rep != NULL (host) the call waits for both
 * and fills *rep. With rep == NULL it returns while they may still run:
 * tls_rqi_solve then overlaps them with its iterations, and
 * tls_precond_info (with a report requested), tls_rqi_solve and
 * tls_precond_destroy wait for them; A and ws must stay valid until then.
 * allow_escalate applies to Cholesky breakdown (TLS_ERR_NOT_SPD): after the
 * diagonal shifts 2^j n u_q (j = 0, 1, 2) the factor is recomputed in the
 * next higher precision. A dense A with n <= 4096 also gets a row-major
 * FP64 copy in ws (read by every pass of the solve), made on the second
 * side stream beside the tail of the Cholesky chain; the call's stream
 * waits for it before the factorization's status is read, so it is
 * complete when the call returns. On success *out (host) receives a handle to
 * destroy with tls_precond_destroy. ws must hold
 * tls_factor_workspace_size() bytes. */
TLS_API tls_status tls_factor_precond(const tls_matrix *A, int32_t u_q, int32_t scaling,
                              int32_t allow_escalate, void *ws, size_t ws_bytes,
                              hipStream_t stream, tls_precond *out,
                              tls_gate_report *rep);

/* Bytes of workspace tls_factor_precond_qr needs for A and u_q (covers every
 * escalation up to FP64): the factor workspace of tls_factor_precond
 * without its dense cast buffer, plus the QR working matrix, FP64-sized,
 * (m + Np - n) x Np with Np = 64 ceil(n / 64), and 8 KiB of reflector
 * scratch per 256 rows of it. */
/* The Gram step alone (Section 2: the preconditioner is the Cholesky factor
 * of A^T A; Section 3.1: two-sided diagonal scaling and rounding to u_q):
 * G = Ahat^T Ahat with Ahat = fl_{u_q}(A D^{-1}), D = diag(||A e_j||_2)
 * when scaling (else D = I, FP64 only), computed exactly as
 * tls_factor_precond computes it before the Cholesky factorization: FP64
 * matrix cores on A (u_q = FP64); FP32 matrix cores on an FP32 cast (FP32);
 * 16-bit matrix cores with FP32 accumulation restarted every 128 rows and
 * row segments added in FP64 (FP16, BF16). Dense A only. G (device, n x n
 * column-major FP64) receives the upper triangle; the strict lower part is
 * not written. d (device, n, may be NULL) receives the diagonal of D. The
 * workspace is tls_factor_workspace_size(A, u_q) bytes. Asynchronous. */
TLS_API tls_status tls_gram(const tls_matrix *A, int32_t u_q, int32_t scaling, double *G, double *d,
                            void *ws, size_t ws_bytes, hipStream_t stream);

TLS_API size_t tls_factor_qr_workspace_size(const tls_matrix *A, int32_t u_q);

/* Build R with R^T R ~ A^T A from the Householder QR of A (Section 3: the
 * R-factor of A = Q [R; 0], computed in precision u_q; constraint (5) of
 * Section 3.1 asks u_q <~ kappa(A)^{-1}, against kappa(A)^{-2} for the
 * Cholesky factor of fl(A^T A)). With scaling = 1, D = diag(||A e_j||),
 * A D^{-1} is rounded to u_q (as in tls_factor_precond), its R-factor
 * R_hat is computed with every entry of the working matrix rounded to u_q
 * when stored (products and the block reflectors' intermediates in FP32;
 * everything in FP64 when u_q = FP64), its rows are given a nonnegative
 * diagonal and R = R_hat D. Q is not formed. A CSR A is
 * expanded into the dense working matrix. The gate, the handle and the
 * solve are those of tls_factor_precond (verdict bit 0, constraint (5),
 * is the a-priori condition that applies to this factor; bits 1 and 2
 * concern the Cholesky route and are reported for comparison). A zero or
 * non-finite pivot gives TLS_ERR_NOT_SPD, or, with allow_escalate, a
 * refactorization in the next higher precision. ws must hold
 * tls_factor_qr_workspace_size() bytes. */
TLS_API tls_status tls_factor_precond_qr(const tls_matrix *A, int32_t u_q, int32_t scaling,
                                 int32_t allow_escalate, void *ws, size_t ws_bytes,
                                 hipStream_t stream, tls_precond *out,
                                 tls_gate_report *rep);

/* Bytes of workspace tls_precond_import needs for order n. */
TLS_API size_t tls_precond_import_workspace_size(int64_t n);

/* Wrap a caller-supplied factor: R_host (host) is the n x n upper triangle,
 * column-major (entries below the diagonal ignored), d_host (host, may be
 * NULL = ones) the scaling with R = R_hat diag(d). R_hat is rounded to
 * `storage`. Used to run PCGTLS on a known factor. */
TLS_API tls_status tls_precond_import(int64_t n, const double *R_host, const double *d_host,
                              int32_t storage, void *ws, size_t ws_bytes,
                              hipStream_t stream, tls_precond *out);

TLS_API void tls_precond_destroy(tls_precond P);

/* Order n, storage precision and gate report of P (host outputs, each may
 * be NULL). Requesting the report waits for a gate still running. */
TLS_API tls_status tls_precond_info(const tls_precond P, int64_t *n, int32_t *storage,
                            tls_gate_report *rep);

/* How R^{-1} and R^{-T} are applied inside PCGTLS, the gate and x_LS:
 *   0 (default) GEMV with the explicit inverse X = R_hat^{-1}, formed once
 *     per factorization by recursive block inversion (stored in FP64 for an
 *     FP64 factor, FP32 otherwise);
 *   1 blocked forward/backward substitution with the stored tiles of R_hat
 *     (Table 1), one workgroup per 64-row block, inter-workgroup flags;
 *   2 the GEMV of mode 0 with one workgroup per 64-row block of the result
 *     (four waves stream the block row's tiles; no reduction across
 *     workgroups) instead of mode 0's split over N x ceil(N / c) workgroups
 *     (c = 4 tiles per workgroup up to N = 40, growing to 32 for large N;
 *     fixed-order reduction by the last workgroup of each block). It holds
 *     only N CUs, which suits work that runs beside a solve. */
TLS_API tls_status tls_precond_set_apply(tls_precond P, int32_t mode);

/* Copy R_hat (upper, column-major n x n, FP64) and d to host buffers. */
TLS_API tls_status tls_precond_export(const tls_precond P, double *R_host, double *d_host,
                              hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Algorithm 3: l-step PCGTLS for (A^T A - sigma2 I) w = rhs, using only R.
 * ------------------------------------------------------------------------- */

TLS_API size_t tls_pcg_workspace_size(const tls_precond P, int32_t nrhs, int32_t l);

/* Run j = 0..l on nrhs (1 or 2) right-hand sides sharing sigma2. A
 * right-hand side stops before step j when eta_j = 0 or, for j > 0,
 * eta_j <= u_p^2 eta_0 (2^-48 in FP32, 2^-106 in FP64: its residual is zero
 * in the working precision relative to the first), or when delta_j = 0 (the
 * printed condition) or
 * delta_j or alpha_j = eta_j / delta_j is not finite; a step runs whole or
 * not at all, so omega never takes a NaN from 0/0. rhs and omega are
 * n x nrhs column-major FP64 (device). u_p is the arithmetic precision
 * (TLS_FP64 or TLS_FP32). trace (host, may be NULL) receives, per
 * right-hand side r, 4*(l+2) doubles at offset 4*(l+2)*r:
 * eta_0..eta_{l+1}, delta_0..delta_{l+1}, alpha_0.., beta_0.. (NaN where a
 * value was not formed). delta_j < 0 is returned as TLS_ERR_INDEFINITE only
 * when strict_pd is set; otherwise the iteration continues as printed. */
TLS_API tls_status tls_pcg_step(const tls_precond P, double sigma2, int32_t nrhs,
                        const double *rhs, double *omega, int32_t l, int32_t u_p,
                        int32_t strict_pd, void *ws, size_t ws_bytes,
                        hipStream_t stream, double *trace);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as tls_pcg_step, with its workspace taken from a static device
 * array of TLS_PCG_NOALLOC_MAX_BYTES per GPU instead of a caller workspace.
 * The array is resolved to its device address on the first call on each
 * device (that device current) and held until the process ends. The call
 * allocates nothing itself (no hipMalloc/hipFree, no pinned memory); leave
 * tls_profile_start off around it, since the profiler creates events.
 * Calls whose tls_pcg_workspace_size(P, nrhs, l) exceeds the maximum return
 * TLS_ERR_WORKSPACE (e.g. n <= 8192 with l <= 1024 fits). Every call on one
 * GPU shares its array: calls that overlap in time on one GPU (two streams,
 * two threads) race and must be serialized by the caller. The state that
 * must start at zero is cleared by the call itself, on `stream`. */
#define TLS_PCG_NOALLOC_MAX_BYTES ((size_t)16 << 20)
TLS_API tls_status tls_pcg_step_noalloc(const tls_precond P, double sigma2, int32_t nrhs,
                        const double *rhs, double *omega, int32_t l, int32_t u_p,
                        int32_t strict_pd, hipStream_t stream, double *trace);

/* out = R^{-1} in (trans = 0) or R^{-T} in (trans = 1) for nrhs column-major
 * FP64 vectors, computed in u_p (forward/backward substitution, Table 1). */
TLS_API tls_status tls_apply_precond(const tls_precond P, int32_t trans, int32_t nrhs,
                             const double *in, double *out, int32_t u_p,
                             void *ws, size_t ws_bytes, hipStream_t stream);

/* y = A x (trans = 0, x n-vector, y m-vector) or y = A^T x (trans = 1), FP64.
 * For CSR, A^T x uses the CSC copy held by P (P may be NULL for trans = 0). */
TLS_API tls_status tls_matvec(const tls_matrix *A, const tls_precond P, int32_t trans,
                      const double *x, double *y, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Algorithms 2 / 4: RQI for TLS with PCGTLS inner solves.
 * ------------------------------------------------------------------------- */

TLS_API void tls_default_opts(tls_rqi_opts *o);

TLS_API size_t tls_rqi_workspace_size(const tls_matrix *A, const tls_precond P,
                              const tls_rqi_opts *o);

/* Solve the TLS problem for (A, b) with the preconditioner P built from the
 * same A. x (device, n, out) receives the iterate with the smallest psi (or
 * the refined one), *sigma (host) sigma_{n+1} from a compensated residual.
 * opts and stats are host structures (stats may be NULL).
 *
 * Gate (opts.gate_enforce, factor below FP64): after x_LS and sigma_0 the
 * bound of constraint (6) is formed with sigma_{n+1} <= sigma_0 (verdict bit
 * 8, reported) and the factor's certificate is read (bit 16: Ritz values of
 * R^{-T} A^T A R^{-1} within [0.5, 1.5]). Without bit 16 the call fails with
 * TLS_ERR_PRECISION, or, with opts.allow_escalate, refactors in the next
 * higher precision and solves again. If the certificate is still being
 * computed (tls_factor_precond called with rep == NULL) the iterations go
 * ahead meanwhile and the verdict is read at the first psi read-back after
 * it is done, or at the end (stats.gate_async = 1); a failed verdict then
 * discards the iterate and escalates as above, so the returned result is
 * the one the waiting order gives. The shift clamp waits for the estimates.
 * Start check (same condition, factor below FP64): a weak factor leaves the
 * corrected semi-normal equations short of x_LS, and the error can put
 * sigma_0 at or above sigma'_n, where A^T A - sigma^2 I is indefinite and RQI
 * may settle on a larger singular value. When the gate finds sigma_0 at or
 * above its estimate of sigma'_n (c~ <= 0 in (6)), a second solve runs on the
 * same factor from x_LS recomputed with corrections until the last is below
 * 1e-8 ||x|| (at most 64), and of the two converged results the one with
 * the smaller sigma is returned: every Rayleigh quotient bounds
 * sigma_{n+1} from above (stats.ls_refined). A problem whose own sigma_LS
 * exceeds sigma'_n is not helped by the second start (the shift clamp is the
 * remedy there), and keeps the first result.
 * A gated solve on a low-precision factor that reaches kmax before the psi
 * rule fires (TLS_ERR_NO_CONVERGENCE) escalates too when opts.allow_escalate
 * is set: a factor whose error exceeds the relative gap between sigma_{n+1}
 * and sigma'_n cannot steer RQI to the smallest root.
 *
 * Warm start (project addition; opts.mlp_theta or opts.sigma0_hint). After
 * x_0 = x_LS, u_0 = (R^T R)^{-1} x_0 and sigma_0 (the quantities of the
 * initial step of Algorithm 2), u_1 = (R^T R)^{-1} u_0 is formed and the
 * shift estimate lam = sigma_hat^2 of sigma_{n+1}^2 gives the candidate
 *   x_1w = x_0 + lam u_0 + lam^2 u_1
 * (the second-order truncation of x_TLS = (I - lam (A^T A)^{-1})^{-1} x_LS).
 * psi (eq. 4) is evaluated at x_1w and at the plain x_1 = x_0 + sigma_0^2 u_0;
 * the iteration starts from the one with the smaller psi (stats.warm_used).
 * The estimate of y = ln(1 - sigma_{n+1}^2 / sigma_0^2), the log of the
 * relative gap between the least-squares estimate and the answer, is
 * y_hat = feature 31 + net(features): a quadrature estimate of the gap
 * corrected by the network's output. Then sigma_hat^2 = sigma_0^2 (1 - exp(min(y_hat, 0))),
 * further clamped, with the shift clamp on, to tau times the sigma'_n
 * estimate squared.
 *
 * Features (stats.features, FP32, natural logarithms), from xx = x_0^T x_0,
 * xu = x_0^T u_0, uu = u_0^T u_0, uv = u_0^T u_1, vv = u_1^T u_1,
 * rr = ||b - A x_0||^2, t = sigma_0^2 xu / (1 + xx), the Ritz values
 * th_max >= th_min of (R^T R)^{-1} on span{x_0, u_0}, and d_j = ||A e_j||:
 *   0 ln m          1 ln n           2 ln ||A||_F     3 ln ||b||
 *   4 ln ||A^T b||  5 ln sigma_0     6 ln ||x_0||     7 ln ||r_0||
 *   8 ln(||r_0||/||b||)              9 ln t           10 ln(sqrt(uu/xx))
 *   11 -ln(th_max)/2  12 -ln(th_min)/2  13 ln sigma_0 + ln(th_max)/2
 *   14 sigma_0^2 th_max               15 t / (1 + t)
 *   16..19 min, max, mean, standard deviation of ln d_j
 *   20 ln(||A^T b|| / (||A||_F ||b||))  21 ln(1 + xx)  22 ln(uv xx / (xu uu))
 *   23 ln(uu xx / xu^2)  24 ln(||A||_F / sqrt(n)) - ln sigma_0
 *   25 ln(||b|| / sqrt(m))  26 ln(th_max / th_min) / 2
 *   27 ln(sigma_0^2 uv / uu)  28 ln(sigma_0^2 sqrt(vv / uu))
 *   29 ln(sigma_0^4 vv / xx) / 2  30 1
 *   31 ln(gap_G), gap_G = max(1 - lam_G / sigma_0^2, 1e-13), where lam_G solves
 *      lam (1 + q(lam)) = ||r_0||^2 (the secular form of eq. 2) with the
 *      quadratic form q(lam) = x_0^T (I - lam (A^T A)^{-1})^{-1} x_0 replaced
 *      by its two-point Gauss rule from two Lanczos steps on (R^T R)^{-1}
 *      started at x_0 (it uses the moments xx, xu, uu, uv) */
TLS_API tls_status tls_rqi_solve(const tls_matrix *A, const double *b, tls_precond P,
                         const tls_rqi_opts *opts, double *x, double *sigma,
                         tls_rqi_stats *stats, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/* out[i] = in[i] rounded to `prec` with round-to-nearest-even (IEEE 754),
 * returned as FP64: the rounding the scaled factor applies to A D^{-1}
 * (Section 3.1). count elements, device arrays. */
TLS_API tls_status tls_round(const double *in, int64_t count, int32_t prec, double *out,
                             hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Warm-start network (project addition, not in the paper): 32 -> 256 -> 256
 * -> 256 -> 1, exact GELU after each hidden layer, FP32, on the device.
 * theta: TLS_MLP_PARAMS floats, per layer W (out x in, row-major) then the
 * bias; norm: 64 floats [mean(32), scale(32)], inputs are (x - mean) * scale.
 * X: batch x 32 row-major. All arrays are device arrays owned by the caller;
 * the workspace (256-byte aligned) holds the batch activations. Results are
 * bitwise reproducible (fixed-order reductions).
 * ------------------------------------------------------------------------- */
TLS_API size_t tls_mlp_workspace_size(int64_t batch);

/* y (batch) = network(X). */
TLS_API tls_status tls_mlp_forward(const float *theta, const float *norm, const float *X,
                                   int64_t batch, float *y, void *ws, size_t ws_bytes,
                                   hipStream_t stream);

/* Mean squared error L = mean_b (y_b - t_b)^2 and its gradient: *loss
 * (device, 1 float), grad (device, TLS_MLP_PARAMS floats, overwritten). */
TLS_API tls_status tls_mlp_loss_grad(const float *theta, const float *norm, const float *X,
                                     const float *t, int64_t batch, float *grad, float *loss,
                                     void *ws, size_t ws_bytes, hipStream_t stream);

/* One Adam update (Kingma & Ba, Algorithm 1) of count parameters at step
 * number step >= 1: m, v (device) are the moment estimates, updated in place. */
TLS_API tls_status tls_mlp_adam(float *theta, float *m, float *v, const float *grad,
                                int64_t count, int64_t step, float lr, float beta1, float beta2,
                                float eps, hipStream_t stream);

/* Kernel-class timing. While profiling is on, the library records a pair of
 * HIP events on the caller's stream around every kernel it launches and
 * accumulates the elapsed time per kernel class. Process-wide state, not
 * thread-safe; meant for benchmarks. Classes (index: name):
 *   0 precond_apply  1 pcg_step  2 gram  3 chol_panel  4 chol_update
 *   5 residual  6 gradient  7 outer_scalars  8 setup  9 lanczos
 *   10 pack  11 residual_dd  12 invert  13 mlp
 *   14 gate: every launch on the library's side streams (the gate's Lanczos
 *      runs, which overlap the caller's stream), whatever its kernel.
 *   15 qr: the Householder QR factorization (tls_factor_precond_qr).
 * chol_panel counts the Cholesky step launches (each also carries the
 * previous step's trailing update); chol_update is no longer used. */
#define TLS_PROF_CLASSES 16
typedef struct {
  int32_t launches[TLS_PROF_CLASSES];
  double total_ms[TLS_PROF_CLASSES];
} tls_kernel_times;

TLS_API tls_status tls_profile_start(void);
/* Synchronizes the recorded events, fills *out (host) and stops profiling. */
TLS_API tls_status tls_profile_stop(tls_kernel_times *out);

/* Thread-local description of the last error (never NULL). */
TLS_API const char *tls_last_error(void);

/* Library version string. */
TLS_API const char *tls_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TLS_H */
