/*
 * symstair.h - C ABI of the MI355X (gfx950) symmetric-stair PCG library.
 *
 * The library solves, for a batch of independent problems, the symmetric
 * positive-definite block-tridiagonal Schur-complement system S lambda = gamma
 * of a trajectory-optimization KKT system (Bu & Plancher, Sec. II-A,
 * Eq. (schur) and the theta/phi/zeta block definitions), with preconditioned
 * conjugate gradient (Sec. II-B) under one of these preconditioners:
 * block-Jacobi and scalar Jacobi (Sec. II-C, Eq. (jacobi)), the additive
 * stair preconditioner (Sec. III, Eqs. (stair), (stair_inv) and the additive
 * combination), the symmetric stair preconditioner (Sec. IV), and the
 * Neumann polynomials of degree 2 and 3 (Sec. II-C, Eq. (polynomial_precon)
 * with Psi = D).  The KKT step around the solve (ssp_kkt_rhs,
 * ssp_kkt_recover) forms gamma and recovers the primal step (Sec. II-A).
 *
 * The handle, layout, export, mapping, autotuning and diagnostic calls cite
 * no passage: the paper fixes what is computed, not how a GPU library holds
 * its batch, lays out its arrays or launches its kernels.  Their comments
 * state the contract instead.
 *
 * Conventions shared by every entry point
 *   - Problem p has N[p] >= 1 knots (block rows), state size nx[p] in [1, 64]
 *     and control size nu[p] in [0, 64].
 *   - S is the NEGATED (positive-definite) Schur complement of the paper's
 *     footnote: block row k = 0..N-1 has diagonal
 *       D_0 = Q_0^-1,
 *       D_k = Q_k^-1 + A_{k-1} Q_{k-1}^-1 A_{k-1}^T + B_{k-1} R_{k-1}^-1 B_{k-1}^T,
 *     and sub-diagonal L_k = S[k][k-1] = -A_{k-1} Q_{k-1}^-1 (k >= 1).  The
 *     returned lambda therefore equals minus the paper's lambda*.
 *   - Input arrays are DEVICE pointers to packed row-major FP64 blocks; the
 *     packing offsets are those returned by ssp_layout (problem after problem,
 *     knot after knot).  A[N-1], B[N-1] and R[N-1] are read-only padding: the
 *     last knot's dynamics do not enter S.
 *   - All calls are asynchronous on `stream` (a hipStream_t, NULL = default
 *     stream); outputs are valid after the stream is synchronised.  A handle
 *     must not be used from two host threads at once.
 *   - Numerical outcomes go to the per-problem status array and never fail
 *     the call; the call-level ssp_status reports argument, allocation or
 *     HIP runtime errors only.  No C++ exception crosses this interface.
 */
#ifndef SYMSTAIR_H
#define SYMSTAIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssp_batch ssp_batch; /* opaque; owns every device workspace */

typedef enum {
    SSP_OK = 0,
    SSP_ERR_ARG = 1,   /* invalid argument (null pointer, bad size, bad enum) */
    SSP_ERR_ALLOC = 2, /* device or host allocation failed */
    SSP_ERR_HIP = 3,   /* a HIP runtime call failed (message: ssp_last_error) */
    SSP_ERR_STATE = 4  /* call out of order (e.g. solve before build) */
} ssp_status;

/* Per-problem status codes (values of prob_status[p]). */
enum {
    SSP_P_OK = 0,
    SSP_P_NOT_SPD = 1,   /* a Q_k, R_k or D_k has a non-positive pivot */
    SSP_P_MAXITER = 2,   /* max_iter inner iterations or max refinement steps reached */
    SSP_P_NONFINITE = 3, /* NaN/Inf in gamma, lambda0 or a recurrence scalar */
    SSP_P_BREAKDOWN = 4, /* p^T S p <= 0 or r^T z <= 0 inside PCG */
    SSP_P_INACCURATE = 5, /* FP64 or FP32 without refinement: the inner solve met
                             rel_tol on its recurrence residual but the true FP64
                             residual did not (relres > rel_tol) */
    SSP_P_WARM_FALLBACK = 8, /* bit OR-ed onto the status: the warm start did not
                                reduce the residual and the solve started from 0 */
    SSP_P_PC_FALLBACK = 16   /* bit OR-ed onto the status (FP32 with refinement):
                                the float stair operator broke down, so the
                                refinement went on with block-Jacobi */
};

typedef enum {
    SSP_PC_BLOCK_JACOBI = 0, /* Phi^-1 = block-diag(D_k^-1)          Eq. (jacobi)   */
    SSP_PC_STAIR_ADD = 1,    /* Phi^-1 = (Psi_l^-1 + Psi_r^-1) / 2   Sec. III       */
    SSP_PC_SYM_STAIR = 2,    /* Phi^-1 = Psi_l^-1 + Psi_r^-1 - D^-1  Sec. IV        */
    SSP_PC_SCALAR_JACOBI = 3, /* Phi^-1 = diag(S)^-1                 Eq. (jacobi)   */
    SSP_PC_NEUMANN2 = 4,     /* Phi^-1 = (I + K + K^2) D^-1, K = D^-1 (D - S):     */
    SSP_PC_NEUMANN3 = 5      /* (I + K + K^2 + K^3) D^-1; Eq. (polynomial_precon)  */
                             /* with Psi = D (degree 1 is SSP_PC_SYM_STAIR)        */
} ssp_precon;

typedef enum {
    SSP_FP64 = 0,          /* S, Phi^-1 stored and applied in FP64             */
    SSP_FP32 = 1,          /* FP32 storage and PCG, one solve, FP64 true residual */
    SSP_FP32_REFINE64 = 2  /* FP32 inner PCG inside FP64 iterative refinement  */
} ssp_precision;

/* Create a batch handle on HIP device `device` for `nprob` >= 1 problems of
 * sizes N[p], nx[p], nu[p] (HOST arrays, copied).  Allocates the metadata;
 * matrix storage is allocated by the first ssp_build.  *out receives the
 * handle (NULL on failure).  SSP_ERR_ARG for N < 1, nx outside 1..64, nu
 * outside 0..64, more than 2^31 - 1 knots in all, or when the per-knot FP64
 * assembly's 8 (4 nx^2 + 2 nx nu + nu^2 + nx) bytes (largest nx, nu of the
 * batch) exceed 160 KiB of LDS (e.g. nx = 64 allows nu <= 26). */
ssp_status ssp_batch_create(int32_t nprob, const int32_t *N, const int32_t *nx, const int32_t *nu,
                            int device, ssp_batch **out);

/* Free every device and host resource of the handle (NULL is a no-op).
 * Synchronises the device first. */
ssp_status ssp_batch_destroy(ssp_batch *b);

/* Packing offsets (HOST int64 arrays of nprob + 1 entries, any may be NULL):
 * problem p's A and Q blocks start at element off_nn[p], its B blocks at
 * off_nu[p], its R blocks at off_uu[p], its gamma / lambda (and state
 * vector q, c, dx) entries at off_v[p], its control vectors (r, du: N nu
 * entries) at off_u[p]; entry nprob is the total element count of each
 * array.  The layout is the block structure of Sec. II-A: N block rows of
 * state size nx, N - 1 controls of size nu (the last control block is
 * padding). */
ssp_status ssp_layout(const ssp_batch *b, int64_t *off_nn, int64_t *off_nu, int64_t *off_uu,
                      int64_t *off_v, int64_t *off_u);

/* Build S and Phi^-1 (Sec. II-A block formulas; Sec. III / IV
 * preconditioners) from the per-knot blocks, entirely on the device in FP64,
 * then store them in the precision `prec` will solve in (FP32 storage keeps
 * the FP64 remainder of S as a second FP32 array for the refinement
 * residual).  A, Q, B, R: device FP64, layout of ssp_layout.  prob_status:
 * device int32[nprob], overwritten with SSP_P_OK or SSP_P_NOT_SPD.
 *
 * The build also decides which solve runs (see ssp_set_mapping, kernel 4):
 * the scaled solve, for which it writes, instead of D_k^-1, W_k = C_k^-1 with
 * C_k the Cholesky factor of D_k (D_k = C_k C_k^T), and Oh_k =
 * W_k L_k W_{k-1}^T, the off-diagonal blocks of W S W^T = I + Oh
 * (W = blockdiag(W_k)).  In that basis every preconditioner above except
 * scalar Jacobi is a polynomial in Oh (block-Jacobi W^T W, symmetric stair
 * W^T (I - Oh) W, additive stair W^T (I - Oh/2) W, Neumann degree m
 * W^T (sum_{i<=m} (-Oh)^i) W): the same operators, applied while streaming
 * one nx x nx block per knot (D_k^-1 = W_k^T W_k is formed when ssp_export
 * asks for it).  The
 * polynomial preconditioners SSP_PC_NEUMANN2/3 exist only there, and need
 * every problem's nx in {6, 14, 26, 36} with nu <= nx (else SSP_ERR_ARG).
 * With several state sizes in the batch the build's launches run on the
 * handle's internal streams, forked from `stream` and joined back into it:
 * the call is ordered on `stream` like a single launch (and can be captured
 * into a graph with it). */
ssp_status ssp_build(ssp_batch *b, ssp_precon pc, ssp_precision prec, const double *A,
                     const double *B, const double *Q, const double *R, int32_t *prob_status,
                     void *stream);

/* Build from a symmetric block-tridiagonal matrix given by its blocks
 * instead of the per-knot dynamics: D holds S[k][k] (k = 0..N-1) and Lsub
 * holds S[k][k-1] (k = 1..N-1; block 0 is not read), both device FP64
 * (preconditioners 0 - 3 only; not with kernel 4),
 * nx x nx row-major blocks at the problem's off_nn offsets of ssp_layout
 * (the layout of Q).  Each D_k is used as (D_k + D_k^T) / 2.  Stores S,
 * D_k^-1 and the preconditioner pc (Sec. II-C, III, IV) in the precision of
 * prec exactly as ssp_build does after assembling S, so ssp_solve,
 * ssp_export and the warm start work on the result unchanged.
 * prob_status: device int32[nprob], overwritten with SSP_P_OK or
 * SSP_P_NOT_SPD (some D_k is not positive definite).  Every D_k of an SPD S
 * is SPD, but not conversely: an S that is not SPD with SPD diagonal blocks
 * passes here and ssp_solve reports what its iteration meets (typically
 * SSP_P_BREAKDOWN or SSP_P_MAXITER). */
ssp_status ssp_build_from_blocks(ssp_batch *b, ssp_precon pc, ssp_precision prec, const double *D,
                                 const double *Lsub, int32_t *prob_status, void *stream);

/* Solve S lambda = gamma for every problem with PCG (Sec. II-B) to
 * ||gamma - S lambda||_2 <= rel_tol * ||gamma||_2, using the preconditioner
 * and precision of the last ssp_build.
 *   gamma:    device FP64 [off_v[nprob]] (read only)
 *   lambda:   device FP64, in = initial guess when use_lambda0 != 0,
 *             out = solution (always written)
 *   use_lambda0: 0 = start from zero; 1 = start from lambda (a non-finite
 *             entry gives SSP_P_NONFINITE); 2 = start from lambda unless its
 *             FP64 residual is not smaller than ||gamma|| (or not finite),
 *             in which case the solve starts from zero and the problem's
 *             status carries SSP_P_WARM_FALLBACK
 *   iters:    device int32[nprob], inner PCG iterations (S-products)
 *   relres:   device FP64[nprob], final true relative residual in FP64
 *   prob_status: device int32[nprob], in = build status (a problem whose
 *             status has low bits SSP_P_NOT_SPD is skipped: lambda = 0,
 *             iters = 0, relres = NaN; any other incoming value, e.g. an
 *             earlier solve's status, is ignored), out = solve status.
 *   max_iter: cap on the inner iterations per problem (<= 0: 10 * N * nx).
 * FP32_REFINE64 runs at most 5 refinement steps; the inner relative
 * tolerance of step j is clamp(0.5 * rel_tol * ||gamma|| / ||r_j||, t, 1) with
 * t = 1e-6, and t = min(1e-6, rel_tol / 2) in the scaled solve (kernel 4).
 * There a float breakdown only ends the inner solve; under a stair
 * preconditioner it also replaces it by block-Jacobi for the rest of the
 * solve (SSP_P_PC_FALLBACK, with a fresh budget of 5 refinement steps), and
 * under block-Jacobi SSP_P_BREAKDOWN is reported if the next FP64 residual
 * is not smaller.  With several state sizes in the batch the solve runs one
 * launch per state size on the handle's internal streams, forked from
 * `stream` and joined back into it (ordered on `stream` like one launch). */
ssp_status ssp_solve(ssp_batch *b, double rel_tol, int32_t max_iter, const double *gamma,
                     double *lambda, int use_lambda0, int32_t *iters, double *relres,
                     int32_t *prob_status, void *stream);

/* ssp_solve for callers that cannot allocate device memory at call time
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, kernels and results, but the solve workspace
 * (the persistent grid's work counter, the FP64 residual vectors and the
 * seven inner-precision vectors, about 72 bytes per entry of lambda in FP64
 * storage, 44 in FP32 storage) lives in one fixed array of
 * SSP_NOALLOC_SCRATCH_BYTES per device, held from the library's first use
 * on that device to the end of the process.  The call itself allocates
 * nothing: no hipMalloc, hipFree or allocating library routine.
 * Errors: SSP_ERR_ARG (checked first) when the batch needs more workspace
 * than the array holds; SSP_ERR_STATE as for ssp_solve, and when the
 * explicit-block kernel would first have to allocate its stair blocks (run
 * one ssp_solve or ssp_export with the handle before).  Every call on a
 * device shares that device's array (the work counter is reset by a fill
 * kernel at each call; the vectors are written before they are read): calls
 * whose execution overlaps on one device, from any handle, thread or
 * stream, race and give undefined results. */
#define SSP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ssp_status ssp_solve_noalloc(ssp_batch *b, double rel_tol, int32_t max_iter, const double *gamma,
                             double *lambda, int use_lambda0, int32_t *iters, double *relres,
                             int32_t *prob_status, void *stream);

/* The KKT step around the solve (Sec. II-A, Eq. (schur) and the zeta blocks).
 * The KKT system is [G C^T; C 0] [dz; lambda*] = [g; c] with
 * G = blkdiag(Q_0, R_0, ..., R_{N-2}, Q_{N-1}), g = (q_0, r_0, ..., q_{N-1}) and
 * C the dynamics constraints (block row 0: +I on x_0; block row k + 1:
 * -A_k, -B_k, +I on x_k, u_k, x_{k+1}), the sign the paper's block form of
 * gamma fixes.  Both calls need the Q_k^-1, R_k^-1 of the preceding ssp_build
 * of this handle (SSP_ERR_STATE after ssp_build_from_blocks, before any
 * build, or after a build with ssp_set_keep_inverses(b, 0)) and take the same A, B device arrays; all vectors are device FP64
 * in the layout of ssp_layout (q, c, gamma, lambda, dx: off_v; r, du:
 * off_u).  Numerically they follow the build: a problem flagged NOT_SPD
 * there gets meaningless values.
 *
 * ssp_kkt_rhs: gamma = c - C G^-1 g, i.e. gamma_0 = c_0 - Q_0^-1 q_0 and
 * gamma_k = c_k + zeta_{k-1} with zeta_k = A_k Q_k^-1 q_k + B_k R_k^-1 r_k
 * - Q_{k+1}^-1 q_{k+1}; r's last block per problem is not read. */
ssp_status ssp_kkt_rhs(ssp_batch *b, const double *A, const double *B, const double *q, const double *r,
                       const double *c, double *gamma, void *stream);
/* ssp_kkt_recover: dz* = G^-1 (g - C^T lambda*) for the solution lambda of
 * ssp_solve (lambda* = -lambda):
 *   dx_k = Q_k^-1 (q_k + lambda_k - A_k^T lambda_{k+1})  (k = N-1: no lambda_N term),
 *   du_k = R_k^-1 (r_k - B_k^T lambda_{k+1})             (k <= N-2; du_{N-1} = 0). */
ssp_status ssp_kkt_recover(ssp_batch *b, const double *A, const double *B, const double *q, const double *r,
                           const double *lambda, double *dx, double *du, void *stream);

/* Refinement steps (outer FP64 residual corrections) each problem took in
 * the last ssp_solve: copied into the caller's device int32[nprob]. */
ssp_status ssp_solve_outer(const ssp_batch *b, int32_t *outer, void *stream);

/* Copy the stored matrices out as FP64 blocks (device pointers, N blocks of
 * nx x nx per problem at offsets off_nn): which = 0 -> S (diag = D_k,
 * off = L_k, FP32 storage returns hi + lo), which = 1 -> Phi^-1 (diag =
 * D_k^-1, off = Phi^-1[k][k-1], zero for block-Jacobi), which = 2 -> S as the
 * PCG reads it (the FP32 hi part only under FP32 storage).  which = 1
 * computes the explicit stair blocks if the last build did not (SSP_ERR_ARG
 * for the polynomial preconditioners, which are not block tridiagonal);
 * which = 3 -> the scaled basis of the last build (diag = W_k, off = Oh_k;
 * SSP_ERR_STATE if it was not built). */
ssp_status ssp_export(ssp_batch *b, int which, double *diag, double *off, void *stream);

/* Kernel-mapping knobs of the batched PCG kernel (the autotuner sets them):
 * threads per workgroup (64, 128, 256 or 512), the LDS staging budget in
 * bytes per workgroup (0 = library default) and the kernel:
 *   0 = automatic (default): a batch of one problem with N >= 24 knots runs
 *       the cooperative solve when its grid fits on the device at once, any
 *       other batch the fused kernel;
 *   1 = two sweeps per iteration over the explicitly stored stair blocks;
 *   2 = the fused kernel: one sweep per iteration applying
 *       Phi^-1 = D^-1 - c D^-1 O D^-1 (O = S - D; c = 1 symmetric stair,
 *       1/2 additive stair, 0 block-Jacobi) from the stored D^-1 and S, one
 *       workgroup per problem;
 *   3 = the cooperative solve for a batch of one problem of any length whose
 *       grid fits (else as 0): the same method with the problem's knots
 *       spread over the grid, four per workgroup, and grid-wide barriers;
 *   4 = the scaled solve: one persistent grid for the whole batch, problems
 *       taken largest first from a device queue, each PCG pass streaming the
 *       Oh_k blocks of the congruence basis (see ssp_build).  With kernel 0
 *       the build chooses it for the polynomial preconditioners and for
 *       block-Jacobi and both stairs under FP32 storage (except a single
 *       problem of N >= 24 knots, which runs the cooperative solve).
 * The choice takes effect at the next build.
 * The fused kernel is built for 128 and 256 threads and for knots that fit
 * its LDS rings; otherwise the explicit kernel runs.  Returns SSP_ERR_ARG for
 * an unknown value or a budget that cannot hold one knot of the largest nx. */
ssp_status ssp_set_mapping(ssp_batch *b, int32_t threads, int32_t lds_bytes, int32_t kernel);

/* ---------------------------------------------------------------------------
 * Learned warm start (per-knot network).
 *
 * For a knot k of a problem with state size nx the network reads
 *   x_k = [vec D_k, vec L_k, gamma_k]   (2 nx^2 + nx inputs, row-major blocks
 *                                        as stored by the last ssp_build,
 *                                        L_0 = 0),
 * standardises it, (x_k - mu) * inv_sd, applies two hidden layers of width H
 * with the exact GELU and a linear output layer, and scales the output by
 * y_scale to give lambda0_k.  FP32 throughout (matrix cores).  Parameters are
 * one float vector: W1 (nin x H, row-major), b1 (H), W2 (H x H), b2, W3
 * (H x nx), b3 (nx), nin = 2 nx^2 + nx.  Training minimises, over a range of
 * problems, the mean of || S_p (lambda0_p - lambda*_p) ||^2, i.e. the squared
 * residual of the warm start when lambda* is the exact solution; optimiser
 * Adam.  One network serves one state size.  All pointers are device
 * pointers unless stated; calls are asynchronous on `stream` unless stated.
 * ------------------------------------------------------------------------- */
typedef struct ssp_mlp ssp_mlp;

/* Number of parameters for state size nx and hidden width H (-1 if invalid). */
int64_t ssp_mlp_num_params(int32_t nx, int32_t hidden);
/* New network for state size nx in [1, 64], hidden width a multiple of 16 in
 * [16, 512]; parameters zero, mu = 0, inv_sd = 1, y_scale = 1. */
ssp_status ssp_mlp_create(int32_t nx, int32_t hidden, int device, ssp_mlp **out);
ssp_status ssp_mlp_destroy(ssp_mlp *m);
/* Copy parameters in (resets the Adam moments and step count) / out.
 * get_params copies the parameters and/or the last gradient (either may be
 * NULL, not both). */
ssp_status ssp_mlp_set_params(ssp_mlp *m, const float *theta, void *stream);
ssp_status ssp_mlp_get_params(const ssp_mlp *m, float *theta, float *grad, void *stream);
/* Standardisation: mu, inv_sd: float[nin]; y_scale > 0 (host value). */
ssp_status ssp_mlp_set_scaling(ssp_mlp *m, const float *mu, const float *inv_sd, float y_scale, void *stream);
ssp_status ssp_mlp_get_scaling(const ssp_mlp *m, float *mu, float *inv_sd, float *y_scale, void *stream);
/* Fit the standardisation to every knot of the batch's problems with this
 * network's nx: per-input mean and 1 / max(population std, 1e-6), and
 * y_scale = root mean square of lambda_star there.  The batch must be built;
 * gamma, lambda_star: FP64 vector layout.  Synchronises the stream. */
ssp_status ssp_mlp_fit_scaling(ssp_mlp *m, ssp_batch *b, const double *gamma, const double *lambda_star,
                               void *stream);
/* Write lambda0 (FP64 vector layout) at every knot of the batch's problems
 * with this network's nx; other problems' entries are left untouched.  Pass
 * lambda0 to ssp_solve with use_lambda0 = 2 to keep zero as the fallback. */
ssp_status ssp_mlp_predict(ssp_mlp *m, ssp_batch *b, const double *gamma, double *lambda0, void *stream);
/* Loss and gradient over problems [p0, p1) of a built batch (all of this
 * network's nx): the gradient stays in the handle for ssp_mlp_adam; loss
 * (FP64[1], may be NULL) receives the mean squared warm-start residual. */
ssp_status ssp_mlp_loss_grad(ssp_mlp *m, ssp_batch *b, int32_t p0, int32_t p1, const double *gamma,
                             const double *lambda_star, double *loss, void *stream);
/* One Adam step (Kingma & Ba, bias-corrected) with the last gradient. */
ssp_status ssp_mlp_adam(ssp_mlp *m, float lr, float beta1, float beta2, float eps, void *stream);
/* Optimiser state for checkpoint / resume: the Adam first and second moments
 * (device float[num_params] each, either may be NULL on get) and the number
 * of Adam steps taken (host).  set_state after set_params (which resets
 * them) continues training exactly where get_state left it. */
ssp_status ssp_mlp_get_state(const ssp_mlp *m, float *m1, float *m2, int64_t *steps, void *stream);
ssp_status ssp_mlp_set_state(ssp_mlp *m, const float *m1, const float *m2, int64_t steps, void *stream);
/* FP32 matrix-core GEMM the network uses, C = op(A) op(B) (row-major, op =
 * transpose when trans_* != 0); exposed for tests. */
ssp_status ssp_gemm_f32(int32_t M, int32_t N, int32_t K, const float *A, int32_t lda, int32_t trans_a,
                        const float *B, int32_t ldb, int32_t trans_b, float *C, int32_t ldc, void *stream);

/* Autotuner of the fused kernel's mapping.  The batch's problems are solved
 * in groups of one state size, each group launched on its own stream with its
 * own workgroup size and LDS budget (the budget sets the knots per pipeline
 * step, hence workgroups per CU).  ssp_autotune times every candidate
 * mapping (128 or 256 threads; the largest step and two shorter ones) on
 * each group alone with this batch's last build and keeps the fastest; it
 * then solves the whole batch once, so the outputs (same meaning as in
 * ssp_solve, zero start, max_iter = 10 N nx) hold valid results.  It
 * synchronises the stream and must not be captured into a graph.
 * ssp_set_mapping clears the tuned choice.  With nothing to tune (the
 * explicit kernel, the cooperative solve) it only solves once. */
ssp_status ssp_autotune(ssp_batch *b, double rel_tol, const double *gamma, double *lambda, int32_t *iters,
                        double *relres, int32_t *prob_status, void *stream);
/* Set the fused kernel's mapping of the solve group with state size nx
 * (e.g. a mapping the autotuner found earlier): threads 128 or 256 and an
 * LDS budget that holds at least one pipeline step; 0, 0 restores the
 * default.  The storage precision of the next ssp_build must be the one the
 * budget was checked for (checked against the current storage).
 * SSP_ERR_ARG for an unknown nx or an unusable mapping. */
ssp_status ssp_set_group_mapping(ssp_batch *b, int32_t nx, int32_t threads, int32_t lds_bytes);
/* The mapping in use per solve group (largest total work first): up to
 * max_groups entries of state size, threads, LDS bytes and the autotuner's
 * best time in ms (0 if not tuned), host arrays (any may be NULL); the group
 * count goes to *ngroups. */
ssp_status ssp_get_mapping(const ssp_batch *b, int32_t max_groups, int32_t *nx, int32_t *threads,
                           int32_t *lds_bytes, float *tuned_ms, int32_t *ngroups);

/* Whether ssp_build stores Q_k^-1 and R_k^-1 for the KKT step: on = 1
 * (default) stores them in the handle's FP64 workspace, on = 0 does not
 * (a caller that only solves saves their HBM traffic; ssp_kkt_rhs and
 * ssp_kkt_recover then return SSP_ERR_STATE until a build that keeps them).
 * The stored S, preconditioner and scaled basis are the same either way.
 * Takes effect at the next ssp_build. */
ssp_status ssp_set_keep_inverses(ssp_batch *b, int32_t on);

/* Accumulation of the PCG inner products (r.u, w.u, r.r; Sec. II-B) in the
 * scaled solve under FP32 storage: on = 0 (default) sums the FP32 products
 * in FP32 (per-lane partial sums, then a fixed-order workgroup tree), on = 1
 * sums the same FP32 products in FP64 and rounds the totals to FP32.  FP64
 * storage always sums in FP64; the fused, cooperative and explicit solves
 * sum in their storage type.  Takes effect at the next solve. */
ssp_status ssp_set_reduction_fp64(ssp_batch *b, int32_t on);

/* Mapping of the scaled solve (kernel 4): threads 128 or 256 and the LDS
 * budget per workgroup (0 = the largest pipeline step of every state size);
 * 0, 0 restores the defaults.  ssp_autotune tunes both when the last build
 * chose the scaled solve.  SSP_ERR_ARG if some state size of the batch gets
 * no pipeline step from the budget. */
ssp_status ssp_set_scaled_mapping(ssp_batch *b, int32_t threads, int32_t lds_bytes);
/* The scaled solve's mapping: threads, LDS bytes, workgroups of each
 * persistent grid on this device (min(resident workgroups, nprob); one grid
 * runs per state size of the batch) and the autotuner's best time in ms (0 if
 * not tuned); any pointer may be NULL. */
ssp_status ssp_get_scaled_mapping(const ssp_batch *b, int32_t *threads, int32_t *lds_bytes, int32_t *grid,
                                  float *tuned_ms);
/* The largest horizon N whose six PCG recurrence vectors the scaled solve
 * keeps in the workgroup's LDS instead of HBM, for state size nx,
 * preconditioner pc, storage precision prec and a mapping of threads (128
 * or 256) and lds_bytes (as ssp_get_scaled_mapping reports it): problems
 * with N <= *max_n stream only the Oh blocks per pass.  0 = none (state
 * sizes above 14 never).  A pure function of its arguments (no device call);
 * SSP_ERR_ARG for a NULL max_n or an unknown pc or prec. */
ssp_status ssp_scaled_onchip_horizon(int32_t nx, ssp_precon pc, ssp_precision prec, int32_t threads,
                                     int32_t lds_bytes, int32_t *max_n);

/* The kernel the last ssp_solve (or ssp_autotune) of this batch enqueued:
 * 1 explicit two-sweep, 2 fused (one workgroup per problem), 3 cooperative
 * (one problem over the whole grid), 4 scaled (a persistent grid per state
 * size); 0 before
 * any solve.  *W and *G (may be
 * NULL) receive the cooperative plan: own knots per workgroup and
 * workgroups (0 for the other kernels). */
ssp_status ssp_solve_kernel(const ssp_batch *b, int32_t *kernel, int32_t *W, int32_t *G);

/* Human-readable text of a call-level status, and of the last HIP error seen
 * by this thread (static storage, never NULL). */
/* Device-to-device copy of `bytes` bytes (a multiple of 16; src and dst
 * 16-byte aligned, not overlapping) with a plain streaming kernel, on
 * `stream`.  It is the library's own measure of the practical HBM rate that
 * the solve's measured traffic is compared with; the library itself never
 * calls it. */
ssp_status ssp_copy_bytes(const void *src, void *dst, int64_t bytes, void *stream);

const char *ssp_status_str(ssp_status s);
const char *ssp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SYMSTAIR_H */
