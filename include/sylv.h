/*
 * sylv.h — C ABI of libsylv.so, a mixed-precision Schur-based solver for
 * the real Sylvester equation AX + XB = C and the real Lyapunov equation
 * AX + XA^T = C on one AMD Instinct MI355X (gfx950).
 *
 * Method (Dmytryshyn, Fasi, Higham, Liu, "Mixed-precision algorithms for
 * solving the Sylvester matrix equation"):
 *   - the problem statement is eq. (1.1) (Sylvester) and eq. (1.3)
 *     (Lyapunov, real case: A^* = A^T);
 *   - the real Schur factorisations of A and B are computed in low precision
 *     (Sec. 2.1, eq. (2.3): A ~ U T U^T with U orthogonal to u_low);
 *   - Bartels-Stewart transform / quasi-triangular solve / back-transform
 *     (Sec. 2.2.1) give the first iterate;
 *   - the stationary iteration of Sec. 3 (Alg. 3.1) refines it: each step
 *     solves the correction equation with the low-precision Schur factors
 *     while the residual R = C - AX - XB is formed in binary64 against the
 *     original coefficients (the original-basis form of eq. (3.2));
 *   - convergence is measured by the normwise relative residual, eq. (2.1),
 *     with Frobenius norms evaluated in binary64.
 * With low = SYLV_PREC_FP64 the library runs the plain binary64
 * Bartels-Stewart algorithm on the GPU (the baseline and the fallback).
 *
 * Conventions (all entry points):
 *   - Matrices are column-major with explicit leading dimensions; vec()
 *     stacks columns as in eq. (1.2).
 *   - Matrix arguments (A, B, C, X and the stage-level T, U, Y) are DEVICE
 *     pointers.  The caller owns them.  A, B and C are never modified; X is
 *     fully written.  Every other pointer argument (opts, size arrays,
 *     pointer arrays) is a HOST pointer; the per-equation sylv_info results
 *     may be in host or device memory.
 *   - `stream` is a hipStream_t passed as void*.  NULL means the default
 *     stream.  All work is enqueued on `stream`; the solve entry points make
 *     host decisions from device results (deflation points of the QR
 *     algorithm, residual norms), so they synchronise `stream` and return
 *     only when X and *info are final.
 *   - Workspace: `work`/`work_bytes` may provide device scratch of at least
 *     the size returned by the matching *_workspace_size call; with
 *     work == NULL the library allocates (and caches per device) what it
 *     needs.
 *   - Graph capture: the solve calls (sylv_solve, lyap_solve,
 *     sylv_solve_batched, sylv_solve_noalloc) check the stream first and,
 *     when it is being captured, return SYLV_ERR_CAPTURE_ALLOC (work ==
 *     NULL) or SYLV_ERR_CAPTURE without touching the stream: their stages
 *     take host decisions from device results (QR deflation points,
 *     residual norms).  The batched path records its own graph internally.
 *   - Return value (synchronous errors only): 0 = success; -i = the i-th
 *     argument is invalid (negative size, leading dimension too small, NULL
 *     pointer with a positive size, workspace too small); SYLV_ERR_HIP - k
 *     = HIP runtime error k; SYLV_ERR_ALLOC = device allocation failed;
 *     SYLV_ERR_NOGPU = no usable gfx950 device; SYLV_ERR_CAPTURE(_ALLOC) as
 *     above.
 *   - Numerical outcome is reported per equation in sylv_info.status.
 */
#ifndef SYLV_H
#define SYLV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SYLV_PREC_FP64 = 0, /* plain binary64 Bartels-Stewart (no refinement)          */
    SYLV_PREC_FP32 = 1, /* binary32 Schur/transforms/tri-solve + binary64 refinement */
    SYLV_PREC_BF16 = 2, /* as FP32, but every GEMM-shaped product (Hessenberg
                           trailing updates, off-window QR updates, transforms)
                           takes bfloat16-rounded inputs on BF16 MFMA; escalates
                           to FP32 and then FP64 when fallback is set             */
    SYLV_PREC_FP16 = 3, /* as BF16 with binary16 (IEEE half) operands on FP16 MFMA
                           (v_mfma_f32_16x16x32_f16, binary32 accumulation).
                           Binary16 has 5 exponent bits (Table 2.1), so every
                           operand is brought into its range by an exact power
                           of two: A and B before their factorisations (T
                           rescaled after), C and each residual before the
                           forward transform, the tri-solve output before the
                           back-transform; the powers are undone on the binary64
                           result.  Escalates like BF16.  Batched Lyapunov
                           equations skip the tri-solve scaling: a binary16
                           overflow there gives status NaN and escalates   */
    SYLV_PREC_AUTO = 4  /* per-equation choice by the learned selector (see
                           sylv_selector_set); needs installed weights          */
} sylv_prec;

typedef enum { SYLV_KIND_SYLV = 0, SYLV_KIND_LYAP = 1 } sylv_kind;

typedef struct {
    int    low;        /* sylv_prec: precision of the Schur factors and corrections (default FP32) */
    double tol;        /* target relative residual, eq. (2.1), Frobenius (default 1e-14)          */
    int    max_iter;   /* refinement cap (default 20, the cap used in the paper's experiments)    */
    int    fallback;   /* 1: on failure escalate to the plain binary64 path (default 1)           */
    int    orth_check; /* orthogonality of the low-precision Schur vectors (Sec. 2.1: ~u_low):
                          0 off; 1 (default) randomised estimate of ||U^T U - I||_F from 8
                          random sign probes, O(n^2) binary64 flops; 2 exact binary64
                          ||U^T U - I||_F by a full product, O(n^3); other values: -i  */
    int    alg;        /* SYLV_ALG_ORIG (default): refinement in the original basis (binary64
                          residual C - AX - XB, low-precision corrections); SYLV_ALG_ORTH: Alg. 4.1
                          (binary64-orthonormalised Schur vectors, Alg. 3.1 in the triangular basis
                          with binary64 tri-solves); SYLV_ALG_INV: Alg. 4.2 (the low-precision
                          Schur vectors with their binary64 inverses, same iteration);
                          SYLV_ALG_SYM: symmetric coefficients (Sec. 2.2.2, Hermitian case):
                          A = Q_A D_A Q_A^T and B = Q_B D_B Q_B^T by block Jacobi in the
                          precision `low` (FP64: plain binary64, no refinement), the
                          transformed equation solved elementwise, Y_ij = C~_ij / (d_i + e_j),
                          and the original-basis refinement; A and B must be symmetric to
                          ||A - A^T||_F <= 2^-26 ||A||_F (else -i for that argument); the
                          fallback is the general binary64 path.  ORTH/INV/SYM are
                          ignored by AUTO; ORTH/INV by FP64                                    */
} sylv_opts;

#define SYLV_ALG_ORIG 0
#define SYLV_ALG_ORTH 1
#define SYLV_ALG_INV  2
#define SYLV_ALG_SYM  3

typedef struct {
    double rel_res;     /* eq. (2.1) at exit, binary64, Frobenius norms                         */
    double orth_u;      /* ||U^T U - I||_F of the Schur vectors of A: the probe estimate
                           (orth_check 1) or the exact value (2); 0 if not checked              */
    double orth_v;      /* same for B (Lyapunov: equals orth_u)                                 */
    double sep_est;     /* min |lambda_i + mu_j| over the computed eigenvalues (estimate of sep) */
    double corr_ratio;  /* ||D||_F / ||X||_F of the last correction (stopping quantity of Alg. 3.1) */
    int    iterations;  /* refinement steps taken (corrections applied)                         */
    int    precision_used; /* sylv_prec of the path that produced X                             */
    int    fell_back;   /* 1 if the binary64 fallback produced X                                 */
    int    status;      /* SYLV_OK, or one of the SYLV_ST_* codes below                          */
    int    chosen;      /* SYLV_PREC_AUTO: class picked by the selector (0 BF16, 1 FP32, 2 FP64);
                           -1 otherwise                                                          */
} sylv_info;

#define SYLV_OK               0
#define SYLV_ST_PERTURBED     1  /* a near-singular pivot of the quasi-triangular solve was perturbed */
#define SYLV_ST_NOT_CONVERGED 2  /* tolerance not reached within max_iter and no fallback            */
#define SYLV_ST_NAN           3  /* NaN or Inf in the iterate or residual                            */
#define SYLV_ST_QR_FAILED     4  /* the QR algorithm hit its iteration cap                            */

#define SYLV_ERR_HIP     (-100)
#define SYLV_ERR_ALLOC   (-200)
#define SYLV_ERR_NOGPU   (-300)
/* below every SYLV_ERR_HIP - k (HIP error codes are < 1100) */
#define SYLV_ERR_SCRATCH (-2000)  /* sylv_solve_noalloc: workspace beyond its static scratch */
#define SYLV_ERR_NOINIT  (-2001)  /* sylv_solve_noalloc: sylv_init not called on this device */
#define SYLV_ERR_CAPTURE_ALLOC (-2002)  /* stream under graph capture and work == NULL           */
#define SYLV_ERR_CAPTURE (-2003)  /* stream under graph capture: the solves read device results on
                                     the host between stages, so they cannot be recorded        */

/* Fill *opts with the defaults listed in sylv_opts. */
void sylv_default_opts(sylv_opts *opts);

/* Device workspace in bytes that sylv_solve (lyap = 0) or lyap_solve
 * (lyap = 1, n ignored) needs for these sizes and options.  Returns 0 for
 * invalid arguments. */
size_t sylv_workspace_size(int m, int n, int lyap, const sylv_opts *opts);

/* Solve AX + XB = C (eq. (1.1)), A m x m, B n x n, C and X m x n.
 * opts may be NULL (defaults).  info (may be NULL) is host memory (pageable
 * or pinned) or device memory; a device info is filled by a copy on
 * `stream` before the call returns. */
int sylv_solve(int m, int n, const double *A, int lda, const double *B, int ldb,
               const double *C, int ldc, double *X, int ldx,
               const sylv_opts *opts, sylv_info *info,
               void *work, size_t work_bytes, void *stream);

/* Solve AX + XA^T = C (eq. (1.3), real case), A, C, X n x n, with one Schur
 * factorisation.  Arguments as sylv_solve. */
int lyap_solve(int n, const double *A, int lda, const double *C, int ldc,
               double *X, int ldx, const sylv_opts *opts, sylv_info *info,
               void *work, size_t work_bytes, void *stream);

/* Solve `batch` independent equations (kind[i] = SYLV_KIND_SYLV or
 * SYLV_KIND_LYAP; B[i] and n[i] ignored for Lyapunov, whose order is m[i]).
 * kind, m, n, lda, ldb, ldc, ldx and the pointer arrays A, B, C, X are HOST
 * arrays of length batch; the matrices they point to live in device memory
 * (column-major, binary64).  infos is a host or device array of length batch (may be
 * NULL).  Lyapunov equations of order 1..256 with low = SYLV_PREC_FP32
 * (or BF16, FP16, or AUTO with installed weights) are
 * solved together (Sec. 4 batched workloads): one workgroup per equation in
 * every stage, equations ordered longest first, Schur form, tri-solve and
 * corrections in binary32, residuals in binary64, per-equation convergence
 * control; an equation that misses the tolerance is re-solved in binary64
 * when opts->fallback is set (info.fell_back = 1).  With SYLV_PREC_AUTO the
 * selector's features are computed on the device for every equation of the
 * batch after its binary32 Schur form, one forward pass of the network over
 * the whole batch picks each equation's class (info.chosen): class 0 runs
 * its transforms on bfloat16 operands, class 1 on binary32, class 2 leaves
 * the batch for the single-equation binary64 path.  All other equations go
 * through sylv_solve / lyap_solve one after another.  work (device, may be
 * NULL: the library keeps its own) must hold sylv_batched_workspace_size
 * bytes; infos may also be a device array.  Returns 0, -i for an invalid
 * i-th argument (-15: work too small), or SYLV_ERR_*; synchronises the
 * stream before returning. */
int sylv_solve_batched(int batch, const int *kind, const int *m, const int *n,
                       const double *const *A, const int *lda,
                       const double *const *B, const int *ldb,
                       const double *const *C, const int *ldc,
                       double *const *X, const int *ldx,
                       const sylv_opts *opts, sylv_info *infos,
                       void *work, size_t work_bytes, void *stream);

/* Per-device set-up for the current device: pinned host staging, the
 * internal stream and events, and the device address of the static scratch
 * used by sylv_solve_noalloc.  Idempotent; other entry points do this set-up
 * themselves on first use.  Returns 0, SYLV_ERR_NOGPU, SYLV_ERR_ALLOC or
 * SYLV_ERR_HIP - k. */
int sylv_init(void);

/* Bytes of the static device scratch behind sylv_solve_noalloc (per GPU). */
#define SYLV_NOALLOC_SCRATCH_BYTES (32u << 20)

/* sylv_solve without any allocation, for callers that cannot allocate
 * device or pinned memory at solve time (code under stream capture, tight
 * serving loops, harnesses that forbid allocation).  Same arguments,
 * semantics and results as sylv_solve, with the workspace taken from a
 * static device array of SYLV_NOALLOC_SCRATCH_BYTES per GPU instead of a
 * `work` argument.  Requires a prior sylv_init() on the current device
 * (else SYLV_ERR_NOINIT).  Sizes whose sylv_workspace_size exceeds the
 * scratch return SYLV_ERR_SCRATCH (with the defaults: m = n up to about 430;
 * Lyapunov problems call it with B = A^T).  low = SYLV_PREC_AUTO returns -11
 * (the selector's device copy of its weights is made on first use).  Every
 * call on a GPU reuses that GPU's scratch, which keeps the last call's
 * contents; nothing in it needs to start at zero.  Calls from several host
 * threads are serialised by the library; work from several processes uses
 * separate copies. */
int sylv_solve_noalloc(int m, int n, const double *A, int lda, const double *B, int ldb,
                       const double *C, int ldc, double *X, int ldx,
                       const sylv_opts *opts, sylv_info *info, void *stream);

/* Device workspace in bytes that sylv_solve_batched needs for this batch
 * (host arrays as in sylv_solve_batched); 0 for invalid arguments. */
size_t sylv_batched_workspace_size(int batch, const int *kind, const int *m, const int *n,
                                   const sylv_opts *opts);

/* Tunables of the QR phase of the Schur factorisation for prec FP32 or
 * FP64 (process-wide; take effect at the next factorisation; the library's
 * defaults are the values its autotuner measured best on MI355X):
 *   nsmall  largest active block finished by one full-window LDS kernel,
 *   nw      aggressive-early-deflation window,
 *   nb      bulges per multishift sweep,
 *   adv     rows a bulge chain advances per LDS window phase,
 *   nibble  percentage of the window AED must deflate to skip the sweep,
 *   aed_waves    wavefronts of the AED kernel (4 or 7),
 *   chase_waves  wavefronts of the bulge-chase kernel (8 or 16),
 *   chains  bulge chains a sweep's nb bulges are split into (1..4): chain g
 *           enters one window width after chain g-1, and the chains' disjoint
 *           windows are chased side by side, one workgroup each (in exact
 *           arithmetic the same QR step: the chains' shift polynomials
 *           multiply to the sweep's).
 * A value <= 0 (nibble < 0) keeps the current one.  Returns 0, -1 for a bad
 * prec, -2 when the combination exceeds the LDS/workspace bounds
 * (FP32: nsmall, nw <= 140, nb <= 44, adv + 3 ceil(nb / chains) + 1 <= 141;
 * FP64: 98, 32 and 99; nsmall >= 16, nw >= 8, adv >= 4, nibble <= 100) or
 * names an unsupported wave or chain count. */
int sylv_schur_tune(int prec, int nsmall, int nw, int nb, int adv, int nibble, int aed_waves,
                    int chase_waves, int chains);
/* Current tunables (nsmall, nw, nb, adv, nibble, aed_waves, chase_waves,
 * chains) into vals[8] (host). */
int sylv_schur_tune_get(int prec, int *vals);

/* Tunables of the batched Lyapunov path (process-wide, next call on; the
 * defaults are the values the project's autotuner measured best on MI355X
 * for the 4096-equation batch of orders 16..256):
 *   hess_hi, hess_lo  Hessenberg kernel buckets: orders > hess_hi use the
 *                     1024-thread register kernel (capacity 256), orders in
 *                     (hess_lo, hess_hi] the 256-thread one of capacity 128,
 *                     the rest the 256-thread one of capacity 64
 *                     (1 <= hess_lo <= 64, hess_lo <= hess_hi <= 128);
 *   band1 > band2 > band3  band-QR LDS buckets below the top one (orders
 *                     256..band1+1, band1..band2+1, ...); each bucket's
 *                     launch reserves the band of its largest order, so
 *                     smaller buckets fit more workgroups per CU; 0 ends
 *                     the list (band1 < 256);
 *   graph_passes      refinement passes per captured graph (1..8).
 * Returns 0, or -1/-2/-3/-4 for an invalid hess_hi / hess_lo / band list /
 * graph_passes. */
int sylv_batched_tune(int hess_hi, int hess_lo, int band1, int band2, int band3, int graph_passes);
/* Current batched tunables (hess_hi, hess_lo, band1, band2, band3,
 * graph_passes) into vals[6] (host). */
int sylv_batched_tune_get(int *vals);

/* Text for a return value or a status code. */
const char *sylv_status_string(int code);

/* ------------------------------------------------------------------------
 * Stage-level entry points (used for stage-by-stage parity checks).
 * prec is SYLV_PREC_FP64 or SYLV_PREC_FP32; for FP32 the float arrays are
 * `float*` passed as void*.
 * ---------------------------------------------------------------------- */

/* Real Schur factorisation A = U T U^T (Sec. 2.1, eq. (2.3)): blocked
 * Householder reduction to Hessenberg form, then the multishift QR
 * algorithm.  A (n x n, lda) is read only; T (ldt) receives the upper
 * quasi-triangular factor (every 2x2 diagonal block holds a complex pair;
 * all other subdiagonal entries are exact zeros), U (ldu) the orthogonal
 * factor.  Element type per prec.  Returns 0 or a negative error; *status
 * (host, may be NULL) receives SYLV_OK or SYLV_ST_QR_FAILED. */
int sylv_schur(int n, const void *A, int lda, void *T, int ldt, void *U, int ldu,
               int prec, int *status, void *stream);

/* Symmetric eigen-decomposition S = Q diag(d) Q^T of the symmetric part
 * (S + S^T)/2 of S (n x n, lds, read only) -- the factorisation of the
 * symmetric-coefficient variant (Sec. 2.2.2) -- by two-sided block Jacobi
 * with a round-robin parallel ordering (Golub & Van Loan Sec. 8.5).  d
 * (device, n) receives the eigenvalues in no particular order, Q (ldq) the
 * orthonormal eigenvectors (column i belongs to d[i]).  Element type per
 * prec.  *sweeps (host, may be NULL): block sweeps taken; *status (host, may
 * be NULL): SYLV_OK, or SYLV_ST_QR_FAILED if the sweep cap (60) ran out. */
int sylv_sym_eig(int n, const void *S, int lds, void *d, void *Q, int ldq, int prec,
                 int *sweeps, int *status, void *stream);

/* Quasi-triangular equation TA Y + Y op(TB) = C (the Bartels-Stewart
 * substitution of Sec. 2.2.1): TA m x m and TB n x n upper quasi-triangular;
 * op(TB) = TB (trans_b = 0) or TB^T (trans_b = 1, the Lyapunov case).  C
 * (ldc) is overwritten by Y.  *perturbed (host, may be NULL) is set to 1 if
 * a near-singular block pivot was perturbed. */
int sylv_trsyl(int m, int n, const void *TA, int ldta, const void *TB, int ldtb,
               int trans_b, void *C, int ldc, int prec, int *perturbed, void *stream);

/* Binary64 QR factorisation of a nearly orthogonal square matrix by
 * CholQR2 (G = Q^T Q, R = chol(G), Q <- Q R^{-1}, twice), the binary64 QR
 * step of Alg. 4.1 applied to the low-precision Schur vectors: Q (n x n,
 * ldq, device, binary64) is overwritten by the Q factor with positive
 * diag(R); R (ldr, device, may be NULL) receives the upper triangular R
 * (zero below the diagonal) with Q_in = Q R.  *status (host, may be NULL):
 * SYLV_OK, or SYLV_ST_NOT_CONVERGED when a Cholesky pivot was not positive
 * (Q too far from orthogonal for a Cholesky QR).  Synchronises the stream. */
int sylv_cholqr(int n, double *Q, int ldq, double *R, int ldr, int *status, void *stream);

/* Binary64 residual R = C - A X - X op(B) with op(B) = B (lyap = 0) or A^T
 * (lyap = 1), and the relative residual of eq. (2.1) (Frobenius norms)
 * returned in *rel_res (host).  R (ldr) may be NULL. */
int sylv_residual(int m, int n, const double *A, int lda, const double *B, int ldb,
                  const double *C, int ldc, const double *X, int ldx,
                  double *R, int ldr, int lyap, double *rel_res, void *stream);

/* C = alpha op(A) op(B) + beta C with op = transpose when ta/tb = 1.
 * prec FP64: double operands (FP64 MFMA); FP32: float operands (FP32 MFMA);
 * BF16: float operands rounded to bfloat16 (nearest even) on load, BF16 MFMA
 * with binary32 accumulation (the GEMM-shaped updates of the BF16 option);
 * FP16: the same with binary16 (nearest even, no scaling) on FP16 MFMA.
 * op(A) is m x k, op(B) is k x n. */
int sylv_gemm(int prec, int ta, int tb, int m, int n, int k, double alpha,
              const void *A, int lda, const void *B, int ldb, double beta,
              void *C, int ldc, void *stream);

/* ------------------------------------------------------------------------
 * Learned precision selector (MLP 16-64-64-3, FP32).  Features are the 16
 * quantities listed in sylv_selector_features, read from the binary32 Schur
 * forms; classes are 0 = refinement with bfloat16-input transforms on those
 * forms, 1 = refinement with binary32 transforms, 2 = plain binary64.  The
 * residual test overrules the choice (0 -> 1 -> 2 on failure).
 * ---------------------------------------------------------------------- */

#define SYLV_NFEAT 16
#define SYLV_NCLASS 3
#define SYLV_MLP_NPARAM 5443

/* Forward pass: feats (device, n x 16 row-major, already standardised),
 * params (device, 5443 floats: W1 64x16, b1, W2 64x64, b2, W3 3x64, b3,
 * row-major weights), probs (device, n x 3 row-major). */
int sylv_mlp_forward(int n, const float *feats, const float *params, float *probs,
                     void *stream);

/* One training step on a mini-batch: forward, mean cross-entropy, backward
 * and an Adam update of params in place.  labels (device, int32, n);
 * adam_m/adam_v (device, 5443 floats each) are the moment estimates; t is
 * the 1-based step count; grad (device, 5443, may be NULL) receives the
 * gradient; loss (host, may be NULL) the mean loss of the batch. */
int sylv_mlp_train_step(int n, const float *feats, const int *labels, float *params,
                        float *adam_m, float *adam_v, int t, float lr, float *grad,
                        float *loss, void *stream);

/* Install selector weights (host: 5443 params followed by 16 feature means
 * and 16 feature standard deviations; all finite) used by SYLV_PREC_AUTO;
 * nvalues = 0 uninstalls them (AUTO is then an invalid option).  Returns 0,
 * -1 for a NULL or non-finite blob, -2 for a wrong length. */
int sylv_selector_set(const float *blob, int nvalues);

/* Install selector weights from a file written by the package's selector
 * module (little-endian: 8 bytes "SYLVSEL1", int32 5443, int32 16, int32 3,
 * then 5443 parameters, 16 feature means and 16 feature standard deviations
 * as binary32).  Returns 0, -1 if the file cannot be opened, -2 for a wrong
 * header or a short file, -3 for non-finite values. */
int sylv_selector_load(const char *path);

/* Training options of sylv_selector_train. */
typedef struct {
    int   epochs;   /* passes over the samples (default 30)          */
    int   batch;    /* mini-batch size (default 512)                 */
    float lr;       /* Adam step size (default 1e-3)                 */
    unsigned long long seed; /* initial weights and shuffling (default 0) */
} sylv_train_opts;

void sylv_default_train_opts(sylv_train_opts *opts);

/* Train the selector network on the GPU: feats (device, n_samples x 16
 * row-major, raw features as sylv_selector_features returns them), labels
 * (device, int32 class per sample).  The feature means and standard
 * deviations are computed on the device and the network is trained on the
 * standardised features by the library's forward/backward/Adam kernels
 * (He-normal initial weights, shuffled mini-batches, mean cross-entropy).
 * weights_out (device, 5443 + 32 floats) receives the blob sylv_selector_set
 * takes (params, means, standard deviations); loss_hist (host, `epochs`
 * floats, may be NULL) the mean batch loss of every epoch.  opts may be
 * NULL (defaults).  Allocates its own device scratch; synchronises the
 * stream.  Returns 0, -i for an invalid i-th argument, or SYLV_ERR_*. */
int sylv_selector_train(int n_samples, const float *feats, const int *labels,
                        const sylv_train_opts *opts, float *weights_out, float *loss_hist,
                        void *stream);

/* The 16 selector features of one equation (A, B, C device pointers,
 * binary64, column-major; B = NULL selects the Lyapunov equation
 * AX + XA^T = C, n ignored), computed from its binary32 Schur forms (the
 * forms SYLV_PREC_AUTO refines on): log2 m, log2 n, log10(||A||_F/sqrt m), log10(||B||_F/sqrt n),
 * log10(||C||_F/sqrt(mn)), log10 sep_est (sep_est = min |l_i + m_j| of the
 * computed spectra, Sec. 2.2), log10 kappa_est = log10((||A||_F+||B||_F)/sep_est),
 * Henrici departure ||N||_F/||T||_F of T_A and T_B, fraction of eigenvalues in
 * complex pairs (A, B), log10 relative minimum eigenvalue gap (A, B),
 * log10 of the probe estimates of ||U^T U - I||_F and ||V^T V - I||_F
 * (orth_check = 1), Lyapunov flag.  feats: host,
 * 16 floats.  Returns 0, -i for an invalid i-th argument, or SYLV_ERR_*. */
int sylv_selector_features(int m, int n, const double *A, int lda, const double *B, int ldb,
                           const double *C, int ldc, float *feats, void *stream);

/* ------------------------------------------------------------------------
 * Per-kernel timing (for roofline measurements).  sylv_profile_begin arms
 * one kernel family (ids: 1 gemm_kernel, 2 k_hess_col, 3 k_hess_gemv,
 * 4 k_aed, 5 k_chase, 6 k_trsyl_diag, 7 k_find_ktop, 8 k_cast,
 * 9 k_sumsq_partial, 10 k_bhess, 11 k_bschur, 12 k_btrsyl,
 * 13 gemm_batched_kernel, 14 k_jac_pairs, 15 k_jac_apply, 16 k_win_update); each later launch of that family is bracketed by two
 * HIP events recorded on its launch stream.  sylv_profile_end disarms,
 * waits for the events and returns the number of launches and the summed
 * durations in milliseconds, plus the algorithmic work the library
 * accounts for those launches (flops: gemm_kernel 2mnk; k_chase and k_aed
 * 12 flops per length-3 reflector application to a row or column; else 0)
 * (host pointers, may be NULL).
 * ---------------------------------------------------------------------- */
int sylv_profile_begin(int kernel_id);
int sylv_profile_end(long *launches, double *total_ms, double *work);
const char *sylv_kernel_name(int kernel_id);

#ifdef __cplusplus
}
#endif

#endif /* SYLV_H */
