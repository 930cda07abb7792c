/*
 * msir.h -- C ABI of the MI355X multistage mixed precision iterative refinement
 * library (libmsir.so).
 *
 * The method is Algorithm 4 ("Multistage Iterative Refinement") of Oktay and
 * Carson, "Multistage Mixed Precision Iterative Refinement": an LU factorization
 * with partial pivoting in a low precision u_f is reused by a refinement loop
 * whose residual is computed in u_r; the correction comes from triangular solves
 * in u_f (SIR), from left-preconditioned GMRES with the preconditioned operator
 * applied in u (SGMRES-IR, Algorithm 3) or in u^2 (GMRES-IR, Algorithm 2); the
 * stopping criteria of Sec. 2.1.1 decide when to move to the next variant and,
 * after GMRES-IR, to raise u_f and refactor.
 *
 * Conventions for every entry point:
 *  - Matrices are column-major with an explicit leading dimension (LAPACK style).
 *  - Array arguments named d* are DEVICE pointers on the handle's device; the
 *    caller owns them.  Inputs are never modified.  Outputs are written only on
 *    success (return value >= 0).
 *  - Work is ordered on the handle's HIP stream; every call returns after its
 *    results are complete (host-visible where they are host outputs).
 *  - Return value: 0 success / converged; > 0 numerical outcome (MSIR_NOT_CONVERGED,
 *    MSIR_SINGULAR); < 0 error: -k means argument k (1-based) is invalid,
 *    MSIR_ERR_HIP a HIP runtime error, MSIR_ERR_ALLOC device memory could not be
 *    obtained within the handle's budget.  msir_status_string() names each code.
 *  - The library holds no global state besides the handles; distinct handles may
 *    be used from distinct host threads.  One handle must not be used by two
 *    threads at once.
 */
#ifndef MSIR_H
#define MSIR_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define MSIR_API __attribute__((visibility("default")))
#else
#define MSIR_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* Floating-point formats (Table 3; bf16 per Sec. 2.2; MSIR_DD = double-double,
 * the stand-in for quadruple precision, unit roundoff 2^-106).                  */
typedef enum { MSIR_FP16 = 0, MSIR_BF16 = 1, MSIR_FP32 = 2, MSIR_FP64 = 3, MSIR_DD = 4 } msir_prec;

/* Convergence detection (Sec. 2.1.1).  ESTIMATE: 0 <= phi <= sqrt(n) u_x
 * (eq. for the normwise error estimate).  BACKWARD: normwise backward error of
 * the iterate (inf-norm, residual in u_r) <= tol_nbe, tested at every residual.
 * TRUE: forward error (needs x_true) and normwise backward error <= the initial u,
 * the protocol of the paper's experiments (Sec. 3).  COMPONENTWISE: the
 * componentwise relative backward error max_i |b - A x|_i / (|A||x| + |b|)_i
 * (Sec. 2.1.2 measures; Sec. 2.1.1 notes componentwise measures as an
 * alternative test) <= tol_nbe, tested where BACKWARD tests; |b - A x| from a
 * double-double residual, |A||x| + |b| in float64.                               */
typedef enum { MSIR_CONV_ESTIMATE = 0, MSIR_CONV_BACKWARD = 1, MSIR_CONV_TRUE = 2,
               MSIR_CONV_COMPONENTWISE = 3 } msir_conv;

/* Scaling before a half-precision LU (Sec. 2.1.2).  AUTO: unscaled first, and
 * if the factors hold Inf/NaN, retry with two-sided power-of-two equilibration
 * plus a scalar mu.  ALWAYS: two-sided scaling from the start.  COLS: column
 * equilibration plus mu from the start.  Only applied when u_f is fp16.        */
typedef enum { MSIR_SCALE_NEVER = 0, MSIR_SCALE_AUTO = 1, MSIR_SCALE_ALWAYS = 2, MSIR_SCALE_COLS = 3 } msir_scale;

/* Solver parameters: the inputs of Algorithm 4 plus the readings listed in the
 * design notes.  Fill with msir_params_default() and override.                 */
typedef struct {
    msir_prec uf, u, ur;   /* initial (u_f, u, u_r); u in {FP32, FP64}; ur in {FP64, DD} */
    msir_prec ux;          /* storage precision of x: FP64 (default) or = u (paper mode:
                              x is stored in u, also after an escalation lowers u)     */
    int    i_max;          /* maximum refinement steps of each variant (>= 1)           */
    double tau;            /* GMRES relative preconditioned residual tolerance (> 0);
                              <= 0 selects 1e-6 for u = fp32 and 1e-10 for u = fp64   */
    double rho_thresh;     /* stopping parameter rho_thresh in (0, 1): 0.5 cautious,
                              0.9 aggressive (Sec. 2.1.1)                            */
    double k_max;          /* GMRES iterations per step; <= 0 selects 0.1 n           */
    int    restart;        /* GMRES restart length, 0 = none                          */
    msir_conv conv;        /* convergence detection mode                              */
    double tol_nbe;        /* tolerance of MSIR_CONV_BACKWARD and _COMPONENTWISE      */
    msir_scale scaling;    /* Sec. 2.1.2 scaling policy                               */
    int    nb;             /* LU panel width; 0 = automatic (see msir_nb_auto).  An
                              explicit width must suit every factor format the
                              escalation ladder can reach from uf (else -8)         */
    int    max_steps;      /* global cap on refinement steps (safety)                 */
    int    lu_update;      /* trailing update of fp16/bf16/fp32 factors: MSIR_LU_MFMA
                              (matrix cores, default) or MSIR_LU_FMA (sequential fp32
                              fused multiply-adds, k ascending: reproducible)       */
    int    gmres_op;       /* how GMRES applies U^{-1} L^{-1} in the operator precision
                              p in {FP32, FP64} (single-system solves; p = DD always
                              substitutes): MSIR_OP_INVERSE (default) multiplies by
                              the explicit inverses of L and U, formed once per
                              factorization in float64 and rounded to p;
                              MSIR_OP_SUBST substitutes row by row in p as the
                              method states (one dependent step per row)          */
} msir_params;

#define MSIR_LU_MFMA 0
#define MSIR_LU_FMA  1
#define MSIR_OP_INVERSE 0
#define MSIR_OP_SUBST   1

/* One refinement step (one residual + one correction), Alg. 4 loop body.       */
typedef struct {
    int level;              /* number of precision escalations so far            */
    int uf, u, ur;          /* msir_prec values in force for this step           */
    int stage;              /* 0 SIR, 1 SGMRES-IR, 2 GMRES-IR                     */
    int iter;               /* step index within the variant (1-based)           */
    int k_gmres;            /* GMRES iterations of this step, -1 for SIR          */
    int counted;            /* 0 for a SIR step discarded by the Inf/NaN check    */
    double z, v, rho_max, phi;  /* monitors of Sec. 2.1.1 (true correction)      */
    double rnorm;           /* ||r||_inf of the iterate the step started from    */
    double nbe;             /* its normwise backward error                       */
    unsigned events;        /* MSIR_EV_* bits                                    */
} msir_step;

#define MSIR_EV_NAN_D     1u   /* non-finite correction                          */
#define MSIR_EV_RESET_X0  2u   /* x reset to x0 (phi > phi_0)                    */
#define MSIR_EV_SWITCH    4u   /* moved to the next variant                      */
#define MSIR_EV_ESCALATE  8u   /* u_f raised and A refactored                    */
#define MSIR_EV_SCALED   16u   /* the factorization in use is scaled             */
#define MSIR_EV_NAN_X0   32u   /* x0 replaced by zero                            */
#define MSIR_EV_CONVERGED 64u

typedef struct {
    int    cged;            /* Alg. 4 output flag                                */
    int    status;          /* same code as the return value                     */
    int    steps;           /* refinement steps performed (history length)       */
    int    n_lu;            /* factorizations performed by this solve            */
    int    gmres_iters;     /* total GMRES iterations                            */
    int    final_uf, final_u, final_ur;
    double nbe;             /* final normwise backward error, residual in dd     */
    double ferr;            /* final forward error (NaN without x_true)          */
    double cbe;             /* final componentwise backward error                */
    double t_factor_ms, t_refine_ms;   /* device time split (HIP events)         */
} msir_result;

typedef struct msir_handle msir_handle;

/* Status codes */
#define MSIR_OK               0
#define MSIR_NOT_CONVERGED    1
#define MSIR_SINGULAR         2
#define MSIR_ERR_HIP       -100
#define MSIR_ERR_ALLOC     -101
#define MSIR_ERR_SIZE      -102   /* n outside [1, MSIR_MAX_N]                     */
#define MSIR_ERR_TIMEOUT   -103   /* a substitution launch's bounded wait expired;
                                     its results are invalid                      */
#define MSIR_MAX_N        16384   /* register-resident panel limit (see msir_nb_auto) */

/* Create a handle on HIP device `device`.  `stream` is a hipStream_t (NULL: the
 * null stream).  `hbm_budget_bytes` caps the workspace the handle may allocate
 * (0: no cap).  Errors: -1 h NULL, -2 bad device, MSIR_ERR_HIP.                */
MSIR_API int msir_create(msir_handle** h, int device, size_t hbm_budget_bytes, void* stream);
/* Release the handle and its workspace (NULL is accepted).                      */
MSIR_API int msir_destroy(msir_handle* h);
/* Paper defaults: (fp16, fp32, fp64), ux fp64, i_max 10, tau auto, rho 0.5,
 * k_max 0.1 n, restart 0, CONV_BACKWARD with tol 1e-15, SCALE_AUTO, nb auto.   */
MSIR_API void msir_params_default(msir_params* p);
/* Panel width used for an n x n factorization whose arithmetic is fp32 (fmt in
 * {FP16, BF16, FP32}) or fp64 (FP64): the panel is held in registers of one
 * compute unit, 64 (fp32) or 32 (fp64) values per thread over 1024 threads:
 * with R = ceil(n / 1024) rows per thread, nb = 64, 32, 16, 8, 4 for R <= 1, 2,
 * 4, 8, 16, halved for fp64.                                                    */
MSIR_API int msir_nb_auto(int n, msir_prec fmt);
/* Bytes of device workspace msir_solve needs for order n under params.          */
MSIR_API size_t msir_workspace_bytes(int n, const msir_params* p);
MSIR_API const char* msir_status_string(int status);

/* ---- Whole solve: Algorithm 4 ------------------------------------------------
 * Solve A x = b.  dA: n x n float64 (lda >= n).  db, dx: n float64.  dx_true:
 * NULL or the exact solution (enables ferr and CONV_TRUE).  params: NULL for
 * defaults.  out: NULL or result.  hist: NULL or caller host array of hist_cap
 * steps; *hist_len (may be NULL) receives the number of steps performed (it may
 * exceed hist_cap; only the first hist_cap are stored).
 * Returns MSIR_OK (converged), MSIR_NOT_CONVERGED (precision ladder exhausted or
 * max_steps reached; dx holds the last iterate), or an error (< 0).            */
MSIR_API int msir_solve(msir_handle* h, int n, const double* dA, int lda, const double* db, double* dx,
               const double* dx_true, const msir_params* params, msir_result* out,
               msir_step* hist, int hist_cap, int* hist_len);

/* Alg. 4 for a sparse A given in compressed sparse row form (Table 1's sparse
 * case): drowptr n+1 int32 row pointers (drowptr[0] = 0, drowptr[n] = nnz,
 * non-decreasing), dcolind nnz int32 column indices (strictly increasing within a
 * row, in [0, n)), dvals nnz float64 values; all device arrays owned by the caller.
 * The residual in u_r and A v inside GMRES use the CSR arrays (O(nnz) per product);
 * the LU, the norms and the final error figures use a dense copy held by the handle
 * (n^2 float64).  The pattern is validated on the device first: -12 when it is not
 * a valid n x n CSR pattern (nothing else runs).  Other arguments, results and
 * return values as for msir_solve.                                               */
MSIR_API int msir_solve_csr(msir_handle* h, int n, int nnz, const int* drowptr, const int* dcolind,
                   const double* dvals, const double* db, double* dx, const double* dx_true,
                   const msir_params* params, msir_result* out, msir_step* hist, int hist_cap, int* hist_len);

/* Least squares: min ||b - A x||_2, the extension of the multistage approach to
 * least squares problems that Sec. 4 names as future work.  Alg. 4 runs unchanged
 * on the augmented system [[alpha I, A], [A^T, 0]] [y; x] = [b; 0] of order
 * N = m + n, whose second block row is the normal equations A^T r = 0 for the
 * residual r = b - A x = alpha y.  dA: m x n float64 column-major (lda >= m),
 * m >= n, full column rank; db: m; dx: n (output); dr: NULL or m (output, the
 * residual alpha y).  alpha: 0 for the default (the largest power of two not above
 * max |a_ij|), else a positive power of two (alpha I and alpha y are then exact;
 * the augmented matrix is best conditioned near sigma_min(A) / sqrt(2));
 * *alpha_used (host, may be NULL) receives the value used.  The history, out
 * (nbe, cbe, ferr, n_lu) and the convergence test refer to the augmented system;
 * params as for msir_solve (CONV_TRUE is not available: -7).  The handle holds
 * the augmented matrix (N^2 float64).  Errors: -1 h NULL, MSIR_ERR_SIZE m or n < 1
 * or m + n > MSIR_MAX_N, -2 m < n, -3 dA NULL, -4 lda < m, -5 db NULL, -6 dx NULL,
 * -8 bad params, -9 alpha negative, not finite or not a power of two,
 * -11 hist_cap < 0; otherwise the return value of msir_solve on the augmented
 * system.                                                                       */
MSIR_API int msir_lstsq(msir_handle* h, int m, int n, const double* dA, int lda, const double* db, double alpha,
               double* dx, double* dr, double* alpha_used, const msir_params* params, msir_result* out,
               msir_step* hist, int hist_cap, int* hist_len);

/* GMRES-IR5: the five-precision GMRES-based refinement of Sec. 1 (u_f, u, u_r,
 * u_g, u_p), without the multistage controller.  One LU in params->uf (scaling
 * policy params->scaling), x0 from the factors, then steps: r = b - A x in
 * params->ur, r_hat = fl_ug(r / ||r||_inf), GMRES in ug with the preconditioned
 * matrix applied in up (explicit inverses for up in {FP32, FP64}, substitution for
 * DD), x <- fl_ux(x + fl_ux(||r|| d)).  Stops when the test of params->conv passes,
 * on a non-finite correction, or after params->i_max steps.  ug: FP32 or FP64,
 * not more precise than params->u (u_g >= u); up: FP32, FP64 or DD.  With
 * ug = up = u the steps are SGMRES-IR's (Alg. 3); ug = u, up = u^2 GMRES-IR's
 * (Alg. 2).  History entries are stage-2 steps of level 0.  Other arguments and
 * the return value as for msir_solve; -9: ug or up not allowed.                   */
MSIR_API int msir_gmres_ir5(msir_handle* h, int n, const double* dA, int lda, const double* db, double* dx,
                   const double* dx_true, const msir_params* params, msir_prec ug, msir_prec up,
                   msir_result* out, msir_step* hist, int hist_cap, int* hist_len);

/* nrhs right-hand sides of one A (Alg. 4 with several right-hand sides): an
 * independent controller per column (its own stages, triggers and escalations),
 * over a factor cache with one slot per factor format.  A level (u_f) is factored
 * by the first column that reaches it, together with the explicit inverses its
 * GMRES operator needs, and reused by every later column that reaches it; A's fp32
 * copy likewise.  Columns run one after another on the handle's stream.
 * dB, dX: n x nrhs column-major (ldb, ldx >= n).  dXt: NULL or the exact solutions
 * (ldxt >= n; enables ferr and CONV_TRUE).  outs: NULL or nrhs results; outs[j].n_lu
 * counts the factorizations performed while column j ran (0 when every level it
 * used was already cached), so their sum is the number of distinct levels reached.
 * hist: NULL or a host array of nrhs * hist_cap steps, column j's history from
 * hist + j * hist_cap; hist_len: NULL or nrhs counts (each may exceed hist_cap).
 * Returns the worst status over the columns, or an error (< 0): -10 CONV_TRUE
 * without dXt, -12 invalid params (as msir_solve's -8), -15 hist_cap < 0.        */
MSIR_API int msir_solve_multi(msir_handle* h, int n, int nrhs, const double* dA, int lda,
                     const double* dB, int ldb, double* dX, int ldx, const double* dXt, int ldxt,
                     const msir_params* params, msir_result* outs, msir_step* hist, int hist_cap,
                     int* hist_len);

/* Independent systems of uneven orders, Alg. 4 for each (the same controller,
 * parameters and results as msir_solve): system i has order n[i], matrix dA[i]
 * (lda[i]), right-hand side db[i], solution dx[i] and, when dxt is not NULL and
 * dxt[i] is not NULL, exact solution dxt[i] (host arrays of device pointers).
 * Systems of order <= 1024 run on batched kernels: one persistent launch factors all
 * of them (one workgroup per system, largest first), one persistent launch runs the
 * whole refinement of every system on the device (one workgroup per system, no host
 * round trip per step); systems that raise u_f are factored at the new level in one
 * more batched launch and resumed.  Their triangular solves (SIR and the GMRES
 * operator) are substitutions in the operator precision.  Larger systems are solved
 * one after another as by msir_solve.  outs: NULL or count results.  hist: NULL or a
 * host array of count * hist_cap steps (system i from hist + i * hist_cap); hist_len:
 * NULL or count lengths.  Returns the worst status, or an error: -3 a NULL array or
 * pointer, lda[i] < n[i]; -8 CONV_TRUE without dxt[i]; -9 invalid params (also
 * k_max above 256 for a system of order <= 1024); -12 hist_cap < 0; MSIR_ERR_SIZE an
 * order outside [1, MSIR_MAX_N].                                                 */
MSIR_API int msir_solve_batched(msir_handle* h, int count, const int* n, const double* const* dA,
                       const int* lda, const double* const* db, double* const* dx,
                       const double* const* dxt, const msir_params* params, msir_result* outs,
                       msir_step* hist, int hist_cap, int* hist_len);

/* ---- Serving: requests admitted as slots and device memory free up ----------
 * A server runs `slots` service slots, each a host thread with its own handle and
 * HIP stream (default priority).  A request is one A with nrhs right-hand sides,
 * solved by msir_solve_multi (Alg. 4 per column over one factor cache), with the
 * server's parameters.  Requests start first come, first served as soon as a slot
 * is free and the workspace estimate of the requests in service plus the new one
 * fits hbm_budget_bytes (0: no cap; the first request always starts); requests in service run
 * concurrently on their streams.  Slots keep their workspace between requests.
 * All pointers of a request are device pointers owned by the caller and must stay
 * valid until its completion has been returned by msir_server_poll.            */
typedef struct msir_server msir_server;
typedef struct {
    int id;                 /* caller's tag, returned with the completion        */
    int n, nrhs;
    const double* dA; int lda;
    const double* dB; int ldb;   /* n x nrhs right-hand sides                  */
    double* dX; int ldx;         /* n x nrhs solutions (written)               */
} msir_request;
typedef struct {
    int id, status;         /* status: worst msir_solve_multi status (or < 0)    */
    int nrhs, slot, n_lu, gmres_iters;
    double nbe_max;         /* largest final normwise backward error of the columns */
    double t_submit_ms, t_start_ms, t_end_ms;   /* host clock since server creation */
} msir_completion;
/* -1 s NULL, -2 bad device, -3 slots outside [1, 64], MSIR_ERR_HIP / ERR_ALLOC.  */
MSIR_API int msir_server_create(msir_server** s, int device, int slots, size_t hbm_budget_bytes,
                                const msir_params* params);
/* Queue a request (returns at once).  -2: invalid request fields.               */
MSIR_API int msir_server_submit(msir_server* s, const msir_request* r);
/* Move up to cap finished requests into out (*count of them), waiting up to
 * wait_ms for the first one (0: no wait, < 0: until one finishes).  Returns the
 * number of requests still queued, in service or finished and not yet returned. */
MSIR_API int msir_server_poll(msir_server* s, msir_completion* out, int cap, int* count, int wait_ms);
/* Stop: requests in service finish, queued ones are dropped; releases the slots. */
MSIR_API int msir_server_destroy(msir_server* s);

/* ---- Steps of the hot path (each call is one row of Algorithm 4) -------------
 * These are the building blocks msir_solve runs, exposed so each can be checked
 * on its own.  Matrices of format f are stored as: FP16/BF16 uint16 bit
 * patterns, FP32 float, FP64 double.                                             */

/* Round dA (n x n float64) to format `f` into dW (ldw >= n), directly and with
 * round-to-nearest-even (Alg. 4 first line: A held in u_f).  If scaling is
 * non-NULL it holds host arrays R[n], S[n] and scaling[2n] = mu, and dW receives
 * fl_f(mu R A S) (Sec. 2.1.2).  Returns 0 or < 0.                                 */
MSIR_API int msir_convert(msir_handle* h, int n, const double* dA, int lda, msir_prec f,
                 const double* R, const double* S, double mu, void* dW, int ldw);

/* Compute the scaling of Sec. 2.1.2 for dA: R (rows; all ones when rows == 0), S,
 * mu, written to host arrays R[n], S[n] and *mu.  f is the factor format.         */
MSIR_API int msir_scaling(msir_handle* h, int n, const double* dA, int lda, msir_prec f, int rows,
                 double* R, double* S, double* mu);

/* LU with partial pivoting in place on dW (format f, n x n, ldw), panel width nb
 * (0 = msir_nb_auto).  dipiv: n int32, LAPACK-style 0-based interchanges (rows j
 * and dipiv[j] swapped at step j).  *info: 0, or k+1 for the first zero pivot
 * column k.  Factors: unit lower L below the diagonal, U on and above, all in f,
 * computed as described for the blocked model (panel in fp32 or fp64 registers,
 * rank-1 updates by fused multiply-add).  update (fp16/bf16/fp32): MSIR_LU_MFMA
 * accumulates the trailing update on the matrix cores (fp32 accumulator, internal
 * summation order of the hardware); MSIR_LU_FMA with a sequential fp32 fused
 * multiply-add chain over k (bit-reproducible).  fp64 factors always use FMA.      */
MSIR_API int msir_getrf(msir_handle* h, int n, msir_prec f, void* dW, int ldw, int nb, int update, int* dipiv,
                        int* info);

/* Solve with stored factors: dy = mu S U^{-1} L^{-1} P R dt (Alg. 4 SIR solve and
 * the GMRES preconditioner), every solution component rounded to `comp`:
 * comp = f is the u_f-precision solve; comp in {FP32, FP64, DD} the operator
 * precision p.  dt, dy: n float64 (for DD, dt and dy point to 2n doubles: hi then
 * lo).  R, S: device arrays or NULL; mu scalar.  mode 0: row-by-row substitution
 * (the definition; components rounded to comp one at a time); mode 1 (comp FP32 or
 * FP64, ldw == n): through the explicit inverses of L and U, formed in float64 from
 * the stored factors and rounded to comp, as the GMRES operator applies them.    */
MSIR_API int msir_getrs(msir_handle* h, int n, msir_prec f, const void* dW, int ldw, const int* dipiv,
               const double* dR, const double* dS, double mu, msir_prec comp, int mode,
               const double* dt, double* dy);

/* fl_p(x) elementwise: each of the n float64 values in dx rounded to format p
 * (round to nearest, ties to even; magnitudes beyond the format's largest finite
 * value become infinities; NaN stays NaN), written as float64 to dy (may equal
 * dx).  p in FP16 / BF16 / FP32 / FP64 / DD (the last two leave values unchanged).
 * This is the rounding every fl_u(.) / fl_{u_f}(.) of the method uses (Sec. 2).  */
MSIR_API int msir_round(msir_handle* h, int n, msir_prec p, const double* dx, double* dy);

/* Residual r = b - A x in ur (FP64 or DD), s = ||r||_inf, and the scaled residual
 * r_hat = fl_u(r / s) (Alg. 4 residual line and Sec. 2.1.2).  drhat: n float64
 * holding u values.  *s receives s (host).                                        */
MSIR_API int msir_residual(msir_handle* h, int n, const double* dA, int lda, const double* dx,
                  const double* db, msir_prec ur, msir_prec u, double* drhat, double* s);

/* One GMRES correction (Alg. 2 / Alg. 3): d solves M^{-1} A d = M^{-1} rhat with
 * M = LU from msir_getrf, operator precision p (FP32: A rounded to fp32; FP64;
 * DD), working precision u, tolerance tau, at most ceil(k_max) iterations, restart
 * length restart (0 = none).  dd: n float64 (u values).  *k receives the number
 * of iterations.  R, S, mu as for msir_getrs.  For p in {FP32, FP64} the operator
 * uses the explicit inverses of L and U (msir_getrs mode 1); for DD substitution. */
MSIR_API int msir_gmres(msir_handle* h, int n, const double* dA, int lda, msir_prec f, const void* dW,
               int ldw, const int* dipiv, const double* dR, const double* dS, double mu,
               const double* drhat, msir_prec u, msir_prec p, double tau, double k_max,
               int restart, double* dd, int* k);

/* msir_residual for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with every scratch buffer (slice partial sums, r, block
 * maxima, the last-block counter) in one fixed device array of
 * MSIR_NOALLOC_SCRATCH_BYTES per GPU, held by the library until the process ends,
 * instead of the handle's workspace.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); the handle (created beforehand) supplies
 * the stream and its preallocated pinned memory for s.  Arguments, layout and return
 * values as for msir_residual; n up to MSIR_NOALLOC_MAX_N (else MSIR_ERR_SIZE);
 * MSIR_ERR_HIP if the array's address could not be obtained when the device's first
 * handle was created.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads, other handles) race and must be
 * serialized by the caller.                                                       */
#define MSIR_NOALLOC_MAX_N          8192
#define MSIR_NOALLOC_SCRATCH_BYTES  (2u << 20)
MSIR_API int msir_residual_noalloc(msir_handle* h, int n, const double* dA, int lda, const double* dx,
                                   const double* db, msir_prec ur, msir_prec u, double* drhat, double* s);

/* Normwise and componentwise backward errors of x (Sec. 2, error measures), the
 * residual formed in double-double: nbe = ||b-Ax||_inf/(||A||_inf ||x||_inf +
 * ||b||_inf), cbe = max_i |b-Ax|_i / (|A||x| + |b|)_i.                           */
MSIR_API int msir_backward_error(msir_handle* h, int n, const double* dA, int lda, const double* dx,
                        const double* db, double* nbe, double* cbe);

/* ---- Measurement -------------------------------------------------------------
 * Per kernel class device time: while enabled, every launch of an instrumented
 * kernel class on the handle's stream is bracketed by two HIP events; the sum of
 * their elapsed times and the launch count are kept per class.  Enabling resets
 * the counters.  Classes: */
typedef enum {
    MSIR_T_PANEL = 0,    /* LU panel (pivot search, scaling, rank-1 updates)    */
    MSIR_T_SWAP = 1,     /* row interchanges + U12 triangular solve              */
    MSIR_T_GEMM = 2,     /* LU trailing update (matrix cores)                    */
    MSIR_T_TRSV = 3,     /* forward + backward triangular solve                  */
    MSIR_T_MATVEC = 4,   /* A v inside GMRES, fp32 copy of A (partials + fold)    */
    MSIR_T_RESID = 5,    /* residual b - A x and its scaling                     */
    MSIR_T_ARNOLDI = 6,  /* modified Gram-Schmidt + Givens                       */
    MSIR_T_TRGEMV = 7,   /* one triangular product with an fp32 inverse factor   */
    MSIR_T_FOLD = 8,     /* fold of a product's slice partial sums into its output */
    MSIR_T_MATVEC64 = 9, /* A v inside GMRES with the float64 A (fp64 or dd)      */
    MSIR_T_TRGEMV64 = 10,/* one triangular product with an fp64 inverse factor   */
    MSIR_T_COUNT = 11
} msir_timer;
/* enable != 0: start timing (counters reset); 0: stop.                          */
MSIR_API int msir_timing(msir_handle* h, int enable);
/* Totals of class `cls` since timing was enabled (synchronizes the stream).     */
MSIR_API int msir_timing_get(msir_handle* h, int cls, long long* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* MSIR_H */
