/*
 * CPU oracle for symmetric-stair preconditioned CG on the trajectory-
 * optimization Schur complement.  TEST INFRASTRUCTURE ONLY: tests, the smoke
 * check and the benchmark's CPU-baseline leg call it; the library never does.
 * It shares no code with the GPU library (no headers, helpers or tables).
 *
 * Everything here is plain, unblocked, obviously-correct loop code in FP64
 * (the FP32 inner solve of the mixed-precision mode runs in float on purpose).
 *
 * Paper passages followed (Bu & Plancher, "Symmetric Stair Preconditioning of
 * Linear Systems for Parallel Trajectory Optimization"):
 *   Sec. II-A, Eq. (schur) and the theta/phi block definitions: the Schur
 *     complement S of the KKT system, block tridiagonal.  The paper's S is
 *     negative definite; its footnote negates it, and we store that negated
 *     SPD matrix, so lambda here is minus the paper's lambda*.
 *   Sec. II-C, Eq. (jacobi): block-Jacobi Phi = block-diag(S).
 *   Sec. III, Eq. (stair) and Eq. (stair_inv): left/right stair splittings and
 *     their inverses Psi^-1 = D^-1 (2D - Psi) D^-1, explicit blocks.
 *   Sec. III, additive stair Phi_add^-1 = (Psi_l^-1 + Psi_r^-1) / 2.
 *   Sec. IV, symmetric stair Phi_sym^-1 = Psi_l^-1 + Psi_r^-1 - D^-1 and its
 *     explicit block form.
 *   Sec. II-B: PCG needs only products with S and Phi^-1 plus reductions (the
 *     recurrences are the textbook preconditioned CG the paper cites).
 *   Sec. II-C, Eq. (jacobi): scalar Jacobi Phi = diag(S).
 *   Sec. II-C, Eq. (polynomial_precon): with the splitting S = Psi - P,
 *     Psi = D (block diagonal) and P = D - S, the degree-m preconditioner is
 *     (I + Psi^-1 P + ... + (Psi^-1 P)^m) Psi^-1; it is applied by the Horner
 *     recurrence z_0 = D^-1 r, z_{j+1} = D^-1 (r - O z_j) with O = S - D.
 *   Sec. II-A, Eq. (schur) and the zeta block definitions: the right-hand
 *     side gamma = c - C G^-1 g and the recovery dz = G^-1 (g - C^T lambda*).
 *
 * Indexing reading (N knots -> N block rows k = 0..N-1):
 *   D_0 = Q_0^-1
 *   D_k = Q_k^-1 + A_{k-1} Q_{k-1}^-1 A_{k-1}^T + B_{k-1} R_{k-1}^-1 B_{k-1}^T
 *   L_k = S[k][k-1] = -A_{k-1} Q_{k-1}^-1                    (k >= 1)
 * i.e. the paper's off-diagonal O between block rows k-1 and k is L_k^T.
 * The preconditioner's sub-diagonal block Phi^-1[k][k-1] is
 *   sym: -D_k^-1 L_k D_{k-1}^-1,   add: half of that,   block-Jacobi: 0.
 * The stored arrays are D, L, Dinv, M (N blocks each, L_0 = M_0 = 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* status codes (per problem); kept numerically equal to the library's */
#define OR_OK 0
#define OR_NOT_SPD 1
#define OR_MAXITER 2
#define OR_NONFINITE 3
#define OR_BREAKDOWN 4
#define OR_WARM_FALLBACK 8 /* OR-ed: the warm start was replaced by zero */
#define OR_PC_FALLBACK 16  /* OR-ed: the solve went on with block-Jacobi after a float breakdown */

#define OR_INACCURATE 5 /* one solve without refinement: recurrence met tol, true residual did not */

#define OR_PC_BJ 0
#define OR_PC_ADD 1
#define OR_PC_SYM 2
#define OR_PC_JACOBI 3 /* scalar Jacobi: Phi = diag(S) */
#define OR_PC_POLY2 4  /* Neumann polynomial of degree 2 in Psi^-1 P, Psi = D */
#define OR_PC_POLY3 5  /* ... of degree 3 */

#define OR_FP64 0
#define OR_FP32 1
#define OR_FP32_REFINE64 2

/* ---------------------------------------------------------------- dense --- */

/* A = L L^T with L lower triangular (row-major n x n).  Returns 1 if a pivot
 * is not positive (A not SPD). */
static int chol(int n, const double *A, double *L) {
    memset(L, 0, sizeof(double) * (size_t)n * n);
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) return 1;
        double d = sqrt(s);
        L[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / d;
        }
    }
    return 0;
}

/* Solve L L^T x = b in place. */
static void chol_solve(int n, const double *L, double *x) {
    for (int i = 0; i < n; ++i) {
        double t = x[i];
        for (int k = 0; k < i; ++k) t -= L[i * n + k] * x[k];
        x[i] = t / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = x[i];
        for (int k = i + 1; k < n; ++k) t -= L[k * n + i] * x[k];
        x[i] = t / L[i * n + i];
    }
}

/* Ainv = A^-1 for SPD A via Cholesky, column by column, then symmetrised.
 * Returns 1 if A is not SPD. */
static int spd_inv(int n, const double *A, double *Ainv) {
    double *L = malloc(sizeof(double) * (size_t)n * n);
    double *col = malloc(sizeof(double) * (size_t)n);
    int bad = chol(n, A, L);
    if (!bad) {
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < n; ++i) col[i] = (i == j) ? 1.0 : 0.0;
            chol_solve(n, L, col);
            for (int i = 0; i < n; ++i) Ainv[i * n + j] = col[i];
        }
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                double s = 0.5 * (Ainv[i * n + j] + Ainv[j * n + i]);
                Ainv[i * n + j] = s;
                Ainv[j * n + i] = s;
            }
    }
    free(L);
    free(col);
    return bad;
}

/* C (m x n) = X (m x k) * Y (k x n), or with Y^T when ty = 1 (Y is n x k). */
static void matmul(int m, int k, int n, const double *X, const double *Y, int ty, double *C) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) s += X[i * k + l] * (ty ? Y[j * k + l] : Y[l * n + j]);
            C[i * n + j] = s;
        }
}

/* ---------------------------------------------------------------- build --- */

/* The preconditioner of a block-tridiagonal S given by its diagonal blocks D
 * and sub-diagonal blocks L (N blocks nx x nx each, L[0] unused): Dinv =
 * D_k^-1 (Eq. jacobi; also the diagonal blocks of both stair forms) and
 * M = Phi^-1[k][k-1] (Eq. stair_inv and the Sec. IV form; zero for
 * block-Jacobi, M[0] = 0).  Returns OR_NOT_SPD if some D_k is not SPD. */
int ssp_oracle_precond(int N, int nx, int pc, const double *D, const double *L, double *Dinv, double *M) {
    const size_t nn = (size_t)nx * nx;
    double *T1 = malloc(sizeof(double) * nn), *T2 = malloc(sizeof(double) * nn);
    int st = OR_OK;

    /* D_k^-1: block-Jacobi inverse and the diagonal of both stair forms */
    for (int k = 0; k < N && st == OR_OK; ++k)
        if (spd_inv(nx, D + k * nn, Dinv + k * nn)) st = OR_NOT_SPD;

    /* scalar Jacobi (Eq. jacobi with Phi = diag(S)): Dinv holds 1 / S_ii */
    if (st == OR_OK && pc == OR_PC_JACOBI)
        for (int k = 0; k < N; ++k)
            for (int i = 0; i < nx; ++i)
                for (int j = 0; j < nx; ++j)
                    Dinv[k * nn + i * nx + j] = (i == j) ? 1.0 / D[k * nn + i * nx + i] : 0.0;

    /* sub-diagonal blocks of Phi^-1 (Eq. stair_inv and the Sec. IV form);
     * zero for block-Jacobi, scalar Jacobi and the polynomial forms, which
     * are not block tridiagonal and are applied by their recurrence */
    if (st == OR_OK) {
        memset(M, 0, sizeof(double) * nn);
        for (int k = 1; k < N; ++k) {
            double *Mk = M + k * nn;
            if (pc != OR_PC_ADD && pc != OR_PC_SYM) { memset(Mk, 0, sizeof(double) * nn); continue; }
            matmul(nx, nx, nx, Dinv + k * nn, L + k * nn, 0, T1);       /* D_k^-1 L_k */
            matmul(nx, nx, nx, T1, Dinv + (k - 1) * nn, 0, T2);         /* ... D_{k-1}^-1 */
            double scale = (pc == OR_PC_ADD) ? -0.5 : -1.0;
            for (size_t e = 0; e < nn; ++e) Mk[e] = scale * T2[e];
        }
    }
    free(T1); free(T2);
    return st;
}

/* Assemble S (D, L) and the preconditioner (Dinv, M) of one problem.
 * A, Q: N blocks nx x nx; B: N blocks nx x nu; R: N blocks nu x nu.
 * D, L, Dinv, M: N blocks nx x nx each (L[0] = M[0] = 0).
 * Returns OR_NOT_SPD if any Q_k, R_k or D_k is not SPD, else OR_OK. */
int ssp_oracle_build(int N, int nx, int nu, const double *A, const double *B, const double *Q,
                     const double *R, int pc, double *D, double *L, double *Dinv, double *M) {
    const size_t nn = (size_t)nx * nx, nuu = (size_t)nu * nu;
    double *Qinv = malloc(sizeof(double) * nn * (size_t)N);
    double *Rinv = malloc(sizeof(double) * (nuu ? nuu : 1));
    double *T1 = malloc(sizeof(double) * nn), *T2 = malloc(sizeof(double) * nn);
    double *BR = malloc(sizeof(double) * (size_t)nx * (nu ? nu : 1));
    int st = OR_OK;

    /* Q_k^-1 for every knot */
    for (int k = 0; k < N && st == OR_OK; ++k)
        if (spd_inv(nx, Q + k * nn, Qinv + k * nn)) st = OR_NOT_SPD;

    /* diagonal blocks D_k and sub-diagonal blocks L_k */
    if (st == OR_OK) {
        memcpy(D, Qinv, sizeof(double) * nn);
        memset(L, 0, sizeof(double) * nn);
    }
    for (int k = 1; k < N && st == OR_OK; ++k) {
        const double *Ak = A + (k - 1) * nn, *Bk = B + (size_t)(k - 1) * nx * nu;
        const double *Qi = Qinv + (k - 1) * nn;
        if (nu > 0 && spd_inv(nu, R + (k - 1) * nuu, Rinv)) { st = OR_NOT_SPD; break; }
        /* phi = A Q^-1 ; L_k = -phi */
        matmul(nx, nx, nx, Ak, Qi, 0, T1);
        for (size_t e = 0; e < nn; ++e) L[k * nn + e] = -T1[e];
        /* A Q^-1 A^T */
        matmul(nx, nx, nx, T1, Ak, 1, T2);
        for (size_t e = 0; e < nn; ++e) D[k * nn + e] = Qinv[k * nn + e] + T2[e];
        if (nu > 0) {
            /* B R^-1 B^T */
            matmul(nx, nu, nu, Bk, Rinv, 0, BR);
            matmul(nx, nu, nx, BR, Bk, 1, T2);
            for (size_t e = 0; e < nn; ++e) D[k * nn + e] += T2[e];
        }
    }

    if (st == OR_OK) st = ssp_oracle_precond(N, nx, pc, D, L, Dinv, M);
    free(Qinv); free(Rinv); free(T1); free(T2); free(BR);
    return st;
}

/* ---------------------------------------------------- block tridiagonal --- */

/* y = T x for the symmetric block-tridiagonal T with diagonal blocks Dg and
 * sub-diagonal blocks Sb (Sb[0] unused): y_k = Dg_k x_k + Sb_k x_{k-1} + Sb_{k+1}^T x_{k+1}. */
void ssp_oracle_btmv(int N, int nx, const double *Dg, const double *Sb, const double *x, double *y) {
    const size_t nn = (size_t)nx * nx;
    for (int k = 0; k < N; ++k)
        for (int i = 0; i < nx; ++i) {
            double s = 0.0;
            for (int j = 0; j < nx; ++j) s += Dg[k * nn + i * nx + j] * x[k * nx + j];
            if (k > 0)
                for (int j = 0; j < nx; ++j) s += Sb[k * nn + i * nx + j] * x[(k - 1) * nx + j];
            if (k + 1 < N)
                for (int j = 0; j < nx; ++j) s += Sb[(k + 1) * nn + j * nx + i] * x[(k + 1) * nx + j];
            y[k * nx + i] = s;
        }
}

static void btmv_f(int N, int nx, const float *Dg, const float *Sb, const float *x, float *y) {
    const size_t nn = (size_t)nx * nx;
    for (int k = 0; k < N; ++k)
        for (int i = 0; i < nx; ++i) {
            float s = 0.0f;
            for (int j = 0; j < nx; ++j) s += Dg[k * nn + i * nx + j] * x[k * nx + j];
            if (k > 0)
                for (int j = 0; j < nx; ++j) s += Sb[k * nn + i * nx + j] * x[(k - 1) * nx + j];
            if (k + 1 < N)
                for (int j = 0; j < nx; ++j) s += Sb[(k + 1) * nn + j * nx + i] * x[(k + 1) * nx + j];
            y[k * nx + i] = s;
        }
}

/* z = Phi^-1 r.  poly = 0: Phi^-1 is the block-tridiagonal matrix with
 * diagonal blocks Dinv and sub-diagonal blocks M (block-Jacobi, scalar
 * Jacobi, both stairs).  poly = m >= 1: the Neumann polynomial
 * sum_{i=0..m} (D^-1 P)^i D^-1 of Eq. (polynomial_precon) with Psi = D,
 * P = D - S = -O, by Horner: z = D^-1 r, then m times z = D^-1 (r - O z).
 * L holds S's sub-diagonal blocks (O's); t: one scratch vector. */
static void apply_precond(int N, int nx, const double *Dinv, const double *M, const double *L, int poly,
                          const double *r, double *z, double *t) {
    const size_t nn = (size_t)nx * nx;
    if (poly == 0) { ssp_oracle_btmv(N, nx, Dinv, M, r, z); return; }
    for (int k = 0; k < N; ++k)
        for (int i = 0; i < nx; ++i) {
            double s = 0.0;
            for (int j = 0; j < nx; ++j) s += Dinv[k * nn + i * nx + j] * r[k * nx + j];
            z[k * nx + i] = s;
        }
    for (int it = 0; it < poly; ++it) {
        /* t = r - O z, with O z the block-tridiagonal product with zero diagonal */
        for (int k = 0; k < N; ++k)
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                if (k > 0)
                    for (int j = 0; j < nx; ++j) s += L[k * nn + i * nx + j] * z[(k - 1) * nx + j];
                if (k + 1 < N)
                    for (int j = 0; j < nx; ++j) s += L[(k + 1) * nn + j * nx + i] * z[(k + 1) * nx + j];
                t[k * nx + i] = r[k * nx + i] - s;
            }
        for (int k = 0; k < N; ++k)
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int j = 0; j < nx; ++j) s += Dinv[k * nn + i * nx + j] * t[k * nx + j];
                z[k * nx + i] = s;
            }
    }
}

/* Exported for tests: z = Phi^-1 r as the PCG applies it. */
void ssp_oracle_apply_precond(int N, int nx, const double *Dinv, const double *M, const double *L, int poly,
                              const double *r, double *z) {
    double *t = malloc(sizeof(double) * (size_t)N * nx);
    apply_precond(N, nx, Dinv, M, L, poly, r, z, t);
    free(t);
}

/* The same in float (the inner solve of mixed precision). */
static void apply_precond_f(int N, int nx, const float *Dinv, const float *M, const float *L, int poly,
                            const float *r, float *z, float *t) {
    const size_t nn = (size_t)nx * nx;
    if (poly == 0) { btmv_f(N, nx, Dinv, M, r, z); return; }
    for (int k = 0; k < N; ++k)
        for (int i = 0; i < nx; ++i) {
            float s = 0.0f;
            for (int j = 0; j < nx; ++j) s += Dinv[k * nn + i * nx + j] * r[k * nx + j];
            z[k * nx + i] = s;
        }
    for (int it = 0; it < poly; ++it) {
        for (int k = 0; k < N; ++k)
            for (int i = 0; i < nx; ++i) {
                float s = 0.0f;
                if (k > 0)
                    for (int j = 0; j < nx; ++j) s += L[k * nn + i * nx + j] * z[(k - 1) * nx + j];
                if (k + 1 < N)
                    for (int j = 0; j < nx; ++j) s += L[(k + 1) * nn + j * nx + i] * z[(k + 1) * nx + j];
                t[k * nx + i] = r[k * nx + i] - s;
            }
        for (int k = 0; k < N; ++k)
            for (int i = 0; i < nx; ++i) {
                float s = 0.0f;
                for (int j = 0; j < nx; ++j) s += Dinv[k * nn + i * nx + j] * t[k * nx + j];
                z[k * nx + i] = s;
            }
    }
}

static double dot(size_t n, const double *a, const double *b) {
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static float dot_f(size_t n, const float *a, const float *b) {
    float s = 0.0f;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static int all_finite(size_t n, const double *a) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* ------------------------------------------------------------------ PCG --- */

/* Textbook preconditioned CG on S lam = gamma (FP64).
 * lam: in = initial guess, out = solution.  Stop when ||r||_2 <= tol ||gamma||_2
 * on the recurrence residual, checked before every S-product.  *iters counts
 * the S-products after the initial residual.  Returns a status code. */
int ssp_oracle_pcg(int N, int nx, const double *D, const double *L, const double *Dinv,
                   const double *M, int poly, const double *gamma, double tol, int max_iter, double *lam,
                   int *iters) {
    const size_t n = (size_t)N * nx;
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    double *t = malloc(sizeof(double) * n);
    int st = OR_OK, it = 0;
    *iters = 0;
    if (!all_finite(n, gamma) || !all_finite(n, lam)) { st = OR_NONFINITE; goto done; }
    const double gnorm = sqrt(dot(n, gamma, gamma));
    if (gnorm == 0.0) { memset(lam, 0, sizeof(double) * n); goto done; }
    ssp_oracle_btmv(N, nx, D, L, lam, q);
    for (size_t i = 0; i < n; ++i) r[i] = gamma[i] - q[i];
    apply_precond(N, nx, Dinv, M, L, poly, r, z, t);
    memcpy(p, z, sizeof(double) * n);
    double rz = dot(n, r, z);
    for (;;) {
        double rnorm = sqrt(dot(n, r, r));
        if (!isfinite(rnorm)) { st = OR_NONFINITE; break; }
        if (rnorm <= tol * gnorm) break;
        if (it >= max_iter) { st = OR_MAXITER; break; }
        ssp_oracle_btmv(N, nx, D, L, p, q);
        ++it;
        double pq = dot(n, p, q);
        if (!(pq > 0.0) || !(rz > 0.0)) { st = isfinite(pq) ? OR_BREAKDOWN : OR_NONFINITE; break; }
        double alpha = rz / pq;
        for (size_t i = 0; i < n; ++i) { lam[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        apply_precond(N, nx, Dinv, M, L, poly, r, z, t);
        double rz_new = dot(n, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        for (size_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
done:
    *iters = it;
    free(r); free(z); free(p); free(q); free(t);
    return st;
}

/* The same recurrences in float, on float copies of S and Phi^-1, solving
 * S d = rhs from d = 0 to ||r|| <= tol ||rhs||.  The right-hand side is
 * scaled to unit 2-norm in FP64 before rounding to float (so tiny or huge
 * residuals neither underflow nor overflow) and d is scaled back in FP64.
 * Used as the inner solve of mixed precision. */
static int pcg_f32(int N, int nx, const float *D, const float *L, const float *Dinv, const float *M, int poly,
                   const double *rhs, double tol, int max_iter, double *d_out, int *iters) {
    const size_t n = (size_t)N * nx;
    float *r = malloc(sizeof(float) * n), *z = malloc(sizeof(float) * n);
    float *p = malloc(sizeof(float) * n), *q = malloc(sizeof(float) * n);
    float *d = calloc(n, sizeof(float)), *t = malloc(sizeof(float) * n);
    int st = OR_OK, it = 0;
    const double scale = sqrt(dot(n, rhs, rhs));
    for (size_t i = 0; i < n; ++i) r[i] = (float)(rhs[i] / scale);
    const float bnorm = sqrtf(dot_f(n, r, r));
    apply_precond_f(N, nx, Dinv, M, L, poly, r, z, t);
    memcpy(p, z, sizeof(float) * n);
    float rz = dot_f(n, r, z);
    for (;;) {
        float rnorm = sqrtf(dot_f(n, r, r));
        if (!isfinite(rnorm)) { st = OR_NONFINITE; break; }
        if (rnorm <= (float)tol * bnorm) break;
        if (it >= max_iter) { st = OR_MAXITER; break; }
        btmv_f(N, nx, D, L, p, q);
        ++it;
        float pq = dot_f(n, p, q);
        if (!(pq > 0.0f) || !(rz > 0.0f)) { st = isfinite(pq) ? OR_BREAKDOWN : OR_NONFINITE; break; }
        float alpha = rz / pq;
        for (size_t i = 0; i < n; ++i) { d[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        apply_precond_f(N, nx, Dinv, M, L, poly, r, z, t);
        float rz_new = dot_f(n, r, z);
        float beta = rz_new / rz;
        rz = rz_new;
        for (size_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    for (size_t i = 0; i < n; ++i) d_out[i] = scale * (double)d[i];
    *iters = it;
    free(r); free(z); free(p); free(q); free(d); free(t);
    return st;
}

/* Mixed precision: textbook iterative refinement around the float PCG.
 *   r_j = gamma - S lam_j in FP64; stop when ||r_j|| <= tol ||gamma||;
 *   inner float PCG on S d = r_j to relative tolerance
 *     tau_j = clamp(theta * tol * ||gamma|| / ||r_j||, tau_min, 1);
 *   lam_{j+1} = lam_j + d in FP64.
 * refine = 0 runs one inner solve only (plain FP32 mode).
 * refine = 0 ends with OR_INACCURATE if the true residual then misses tol.
 * Under refinement an inner breakdown (p^T S p <= 0 or r^T z <= 0 in float,
 * a loss of float accuracy for an SPD S) ends that inner solve; the step
 * still updates lam and the loop goes on.  Under a stair or polynomial
 * preconditioner (M != 0 or poly > 0) the breakdown also replaces it by
 * block-Jacobi (M = 0, poly = 0), whose
 * float operator stays positive definite far longer, for the rest of the
 * solve, with a fresh budget of refinement steps; the status then carries
 * OR_PC_FALLBACK.  Under block-Jacobi, BREAKDOWN is reported if the next FP64
 * residual is not smaller than the one before that step.
 * *iters is the total number of inner S-products, *outer the refinement
 * steps taken. */
int ssp_oracle_pcg_mixed(int N, int nx, const double *D, const double *L, const double *Dinv,
                         const double *M, int poly, const double *gamma, double tol, int max_iter,
                         int refine, int max_outer, double theta, double tau_min, double *lam,
                         int *iters, int *outer) {
    const size_t n = (size_t)N * nx, nb = (size_t)N * nx * nx;
    float *Df = malloc(sizeof(float) * nb), *Lf = malloc(sizeof(float) * nb);
    float *DIf = malloc(sizeof(float) * nb), *Mf = malloc(sizeof(float) * nb);
    double *r = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n);
    int st = OR_OK, total = 0, steps = 0, broke = 0, base = 0, fell = 0, stair = 0;
    double prev = INFINITY;
    for (size_t e = 0; e < nb; ++e) {
        Df[e] = (float)D[e]; Lf[e] = (float)L[e]; DIf[e] = (float)Dinv[e]; Mf[e] = (float)M[e];
        if (M[e] != 0.0) stair = 1;
    }
    if (poly > 0) stair = 1;
    *iters = 0;
    *outer = 0;
    if (!all_finite(n, gamma) || !all_finite(n, lam)) { st = OR_NONFINITE; goto done; }
    const double gnorm = sqrt(dot(n, gamma, gamma));
    if (gnorm == 0.0) { memset(lam, 0, sizeof(double) * n); goto done; }
    for (;;) {
        ssp_oracle_btmv(N, nx, D, L, lam, r);
        for (size_t i = 0; i < n; ++i) r[i] = gamma[i] - r[i];
        double rnorm = sqrt(dot(n, r, r));
        if (!isfinite(rnorm)) { st = OR_NONFINITE; break; }
        if (rnorm <= tol * gnorm) break;
        if (steps > 0 && !refine) { st = OR_INACCURATE; break; }
        if (broke && !(rnorm < prev)) { st = OR_BREAKDOWN; break; }
        if (steps - base >= max_outer) { st = OR_MAXITER; break; }
        prev = rnorm;
        double tau = refine ? theta * tol * gnorm / rnorm : tol * gnorm / rnorm;
        if (refine && tau < tau_min) tau = tau_min;
        if (tau > 1.0) tau = 1.0;
        int it = 0;
        int ist = pcg_f32(N, nx, Df, Lf, DIf, Mf, poly, r, tau, max_iter - total, d, &it);
        total += it;
        ++steps;
        for (size_t i = 0; i < n; ++i) lam[i] += d[i];
        broke = refine && ist == OR_BREAKDOWN;
        if (broke && stair && !fell) {
            memset(Mf, 0, sizeof(float) * nb);  /* go on with block-Jacobi */
            poly = 0;
            fell = OR_PC_FALLBACK;
            broke = 0;
            base = steps;
        }
        if (ist == OR_NONFINITE || (ist == OR_BREAKDOWN && !refine)) { st = ist; break; }
        if (ist == OR_MAXITER) { st = OR_MAXITER; break; }
    }
done:
    *iters = total;
    *outer = steps;
    free(Df); free(Lf); free(DIf); free(Mf); free(r); free(d);
    return st | fell;
}

/* ||gamma - S lam||_2 / ||gamma||_2 in FP64 (0 when gamma = 0). */
double ssp_oracle_relres(int N, int nx, const double *D, const double *L, const double *gamma,
                         const double *lam) {
    const size_t n = (size_t)N * nx;
    double *y = malloc(sizeof(double) * n);
    ssp_oracle_btmv(N, nx, D, L, lam, y);
    double rr = 0.0, gg = dot(n, gamma, gamma);
    for (size_t i = 0; i < n; ++i) { double t = gamma[i] - y[i]; rr += t * t; }
    free(y);
    return gg > 0.0 ? sqrt(rr / gg) : sqrt(rr);
}

/* ------------------------------------------------------- direct solve --- */

/* Block-tridiagonal Cholesky (block Thomas) solve of S lam = gamma:
 *   C_0 = D_0, C_k = D_k - L_k C_{k-1}^-1 L_k^T,
 *   y_0 = gamma_0, y_k = gamma_k - L_k C_{k-1}^-1 y_{k-1},
 *   lam_{N-1} = C_{N-1}^-1 y_{N-1}, lam_k = C_k^-1 (y_k - L_{k+1}^T lam_{k+1}).
 * Returns OR_NOT_SPD if a pivot block is not SPD. */
int ssp_oracle_direct(int N, int nx, const double *D, const double *L, const double *gamma,
                      double *lam) {
    const size_t nn = (size_t)nx * nx;
    double *Cf = malloc(sizeof(double) * nn * (size_t)N);   /* Cholesky factors of C_k */
    double *C = malloc(sizeof(double) * nn), *W = malloc(sizeof(double) * nn);
    double *y = malloc(sizeof(double) * (size_t)N * nx), *t = malloc(sizeof(double) * nx);
    int st = OR_OK;
    for (int k = 0; k < N; ++k) {
        memcpy(C, D + k * nn, sizeof(double) * nn);
        memcpy(y + k * nx, gamma + k * nx, sizeof(double) * nx);
        if (k > 0) {
            /* W = C_{k-1}^-1 L_k^T, column by column */
            for (int j = 0; j < nx; ++j) {
                for (int i = 0; i < nx; ++i) t[i] = L[k * nn + j * nx + i];
                chol_solve(nx, Cf + (k - 1) * nn, t);
                for (int i = 0; i < nx; ++i) W[i * nx + j] = t[i];
            }
            for (int i = 0; i < nx; ++i)
                for (int j = 0; j < nx; ++j) {
                    double s = 0.0;
                    for (int l = 0; l < nx; ++l) s += L[k * nn + i * nx + l] * W[l * nx + j];
                    C[i * nx + j] -= s;
                }
            /* y_k -= L_k C_{k-1}^-1 y_{k-1} */
            memcpy(t, y + (k - 1) * nx, sizeof(double) * nx);
            chol_solve(nx, Cf + (k - 1) * nn, t);
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int l = 0; l < nx; ++l) s += L[k * nn + i * nx + l] * t[l];
                y[k * nx + i] -= s;
            }
        }
        for (int i = 0; i < nx; ++i)
            for (int j = i + 1; j < nx; ++j) {
                double s = 0.5 * (C[i * nx + j] + C[j * nx + i]);
                C[i * nx + j] = C[j * nx + i] = s;
            }
        if (chol(nx, C, Cf + k * nn)) { st = OR_NOT_SPD; goto done; }
    }
    for (int k = N - 1; k >= 0; --k) {
        memcpy(t, y + k * nx, sizeof(double) * nx);
        if (k + 1 < N)
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int l = 0; l < nx; ++l) s += L[(k + 1) * nn + l * nx + i] * lam[(k + 1) * nx + l];
                t[i] -= s;
            }
        chol_solve(nx, Cf + k * nn, t);
        memcpy(lam + k * nx, t, sizeof(double) * nx);
    }
done:
    free(Cf); free(C); free(W); free(y); free(t);
    return st;
}

/* ------------------------------------------------------------ KKT step --- */

/* The paper writes the KKT system of the QP as [G C^T; C 0] [dz; lambda*] =
 * [g; c] (Eq. schur: S = -C G^-1 C^T, gamma = c - C G^-1 g,
 * dz* = G^-1 (g - C^T lambda*)), with G = blkdiag(Q_0, R_0, ..., R_{N-2},
 * Q_{N-1}) and g = (q_0, r_0, ..., r_{N-2}, q_{N-1}).  Its block form of
 * gamma, c + (-Q_0^-1 q_0, zeta_0, zeta_1, ...) with
 * zeta_k = A_k Q_k^-1 q_k + B_k R_k^-1 r_k - Q_{k+1}^-1 q_{k+1}, fixes the
 * sign of C: block row 0 is +I on x_0 and block row k + 1 is
 * (-A_k, -B_k, +I) on (x_k, u_k, x_{k+1}).  (S does not depend on that
 * sign.)  The library's lambda solves the negated system, lambda = -lambda*.
 *
 * gamma (N nx) from q (N nx), r (N nu; block N-1 unused) and c (N nx):
 *   gamma_0 = c_0 - Q_0^-1 q_0,   gamma_k = c_k + zeta_{k-1}  (k >= 1).
 * Returns OR_NOT_SPD if a Q_k or R_k (k <= N-2) is not SPD. */
int ssp_oracle_kkt_rhs(int N, int nx, int nu, const double *A, const double *B, const double *Q,
                       const double *R, const double *q, const double *r, const double *c, double *gamma) {
    const size_t nn = (size_t)nx * nx, nuu = (size_t)nu * nu;
    double *Qi = malloc(sizeof(double) * nn), *Ri = malloc(sizeof(double) * (nuu ? nuu : 1));
    double *v = malloc(sizeof(double) * nx), *w = malloc(sizeof(double) * (nu ? nu : 1));
    int st = OR_OK;
    for (int k = 0; k < N * nx; ++k) gamma[k] = c[k];
    for (int k = 0; k < N && st == OR_OK; ++k) {
        /* -Q_k^-1 q_k enters row k */
        if (spd_inv(nx, Q + k * nn, Qi)) { st = OR_NOT_SPD; break; }
        for (int i = 0; i < nx; ++i) {
            double t = 0.0;
            for (int j = 0; j < nx; ++j) t += Qi[i * nx + j] * q[k * nx + j];
            v[i] = t;
            gamma[k * nx + i] -= t;
        }
        if (k + 1 >= N) break;
        /* A_k Q_k^-1 q_k + B_k R_k^-1 r_k enters row k + 1 */
        if (nu > 0) {
            if (spd_inv(nu, R + k * nuu, Ri)) { st = OR_NOT_SPD; break; }
            for (int i = 0; i < nu; ++i) {
                double t = 0.0;
                for (int j = 0; j < nu; ++j) t += Ri[i * nu + j] * r[(size_t)k * nu + j];
                w[i] = t;
            }
        }
        for (int i = 0; i < nx; ++i) {
            double t = 0.0;
            for (int j = 0; j < nx; ++j) t += A[k * nn + i * nx + j] * v[j];
            for (int j = 0; j < nu; ++j) t += B[(size_t)k * nx * nu + i * nu + j] * w[j];
            gamma[(k + 1) * nx + i] += t;
        }
    }
    free(Qi); free(Ri); free(v); free(w);
    return st;
}

/* dz* = G^-1 (g - C^T lambda*) with lambda* = -lam:
 *   dx_k = Q_k^-1 (q_k + lam_k - A_k^T lam_{k+1})   (no lam_N term at k = N-1),
 *   du_k = R_k^-1 (r_k - B_k^T lam_{k+1})           (k <= N-2; du_{N-1} = 0).
 * dx: N nx, du: N nu.  Returns OR_NOT_SPD as kkt_rhs does. */
int ssp_oracle_kkt_recover(int N, int nx, int nu, const double *A, const double *B, const double *Q,
                           const double *R, const double *q, const double *r, const double *lam,
                           double *dx, double *du) {
    const size_t nn = (size_t)nx * nx, nuu = (size_t)nu * nu;
    double *Mi = malloc(sizeof(double) * (nn > nuu ? nn : (nuu ? nuu : 1)));
    double *t = malloc(sizeof(double) * (nx > nu ? nx : (nu ? nu : 1)));
    int st = OR_OK;
    for (int k = 0; k < N && st == OR_OK; ++k) {
        for (int i = 0; i < nx; ++i) {
            double s = q[k * nx + i] + lam[k * nx + i];
            if (k + 1 < N)
                for (int j = 0; j < nx; ++j) s -= A[k * nn + j * nx + i] * lam[(k + 1) * nx + j];
            t[i] = s;
        }
        if (spd_inv(nx, Q + k * nn, Mi)) { st = OR_NOT_SPD; break; }
        for (int i = 0; i < nx; ++i) {
            double s = 0.0;
            for (int j = 0; j < nx; ++j) s += Mi[i * nx + j] * t[j];
            dx[k * nx + i] = s;
        }
        for (int i = 0; i < nu; ++i) du[(size_t)k * nu + i] = 0.0;
        if (k + 1 >= N || nu == 0) continue;
        for (int i = 0; i < nu; ++i) {
            double s = r[(size_t)k * nu + i];
            for (int j = 0; j < nx; ++j) s -= B[(size_t)k * nx * nu + j * nu + i] * lam[(k + 1) * nx + j];
            t[i] = s;
        }
        if (spd_inv(nu, R + k * nuu, Mi)) { st = OR_NOT_SPD; break; }
        for (int i = 0; i < nu; ++i) {
            double s = 0.0;
            for (int j = 0; j < nu; ++j) s += Mi[i * nu + j] * t[j];
            du[(size_t)k * nu + i] = s;
        }
    }
    free(Mi); free(t);
    return st;
}

/* --------------------------------------------------------------- batch --- */

/* OpenMP threads of the batch drivers (n >= 1; used to time one core). */
void ssp_oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int ssp_oracle_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* The build alone for every problem of a packed batch (the first half of
 * ssp_oracle_solve_batch, timed on its own); per-problem build status. */
void ssp_oracle_build_batch(int P, const int *Ns, const int *nxs, const int *nus, const int64_t *off_nn,
                            const int64_t *off_nu, const int64_t *off_uu, const double *A, const double *B,
                            const double *Q, const double *R, int pc, int *status) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < P; ++p) {
        const int N = Ns[p], nx = nxs[p], nu = nus[p];
        const size_t nb = (size_t)N * nx * nx;
        double *D = malloc(sizeof(double) * nb), *L = malloc(sizeof(double) * nb);
        double *Di = malloc(sizeof(double) * nb), *M = malloc(sizeof(double) * nb);
        status[p] = ssp_oracle_build(N, nx, nu, A + off_nn[p], B + off_nu[p], Q + off_nn[p], R + off_uu[p], pc,
                                     D, L, Di, M);
        free(D); free(L); free(Di); free(M);
    }
}

/* Build and solve every problem of a packed ragged batch, one problem per
 * OpenMP task.  Offsets are per problem (see the generator's layout):
 * off_nn for A, Q and the nx x nx block arrays, off_nu for B, off_uu for R,
 * off_v for gamma / lambda.  lam holds the initial guess on entry.
 * precision: OR_FP64, OR_FP32 (one float inner solve) or OR_FP32_REFINE64.
 * Per-problem outputs: iters, outer steps, true relres, status. */
void ssp_oracle_solve_batch(int P, const int *Ns, const int *nxs, const int *nus,
                            const int64_t *off_nn, const int64_t *off_nu, const int64_t *off_uu,
                            const int64_t *off_v, const double *A, const double *B, const double *Q,
                            const double *R, const double *gamma, int pc, int precision,
                            double tol, int max_iter, int max_outer, double theta, double tau_min,
                            int warm_fallback, double *lam, int *iters, int *outer, double *relres,
                            int *status) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < P; ++p) {
        const int N = Ns[p], nx = nxs[p], nu = nus[p];
        const size_t nb = (size_t)N * nx * nx;
        double *D = malloc(sizeof(double) * nb), *L = malloc(sizeof(double) * nb);
        double *Di = malloc(sizeof(double) * nb), *M = malloc(sizeof(double) * nb);
        const double *g = gamma + off_v[p];
        double *x = lam + off_v[p];
        int it = 0, ou = 0;
        int st = ssp_oracle_build(N, nx, nu, A + off_nn[p], B + off_nu[p], Q + off_nn[p],
                                  R + off_uu[p], pc, D, L, Di, M);
        const int poly = pc == OR_PC_POLY2 ? 2 : pc == OR_PC_POLY3 ? 3 : 0;
        int fell_back = 0;
        if (st == OR_OK && warm_fallback) {
            /* a warm start whose residual is not below ||gamma|| is replaced by zero */
            const double rr = ssp_oracle_relres(N, nx, D, L, g, x);
            if (!(rr < 1.0)) {
                memset(x, 0, sizeof(double) * (size_t)N * nx);
                fell_back = OR_WARM_FALLBACK;
            }
        }
        if (st == OR_OK) {
            if (precision == OR_FP64) {
                st = ssp_oracle_pcg(N, nx, D, L, Di, M, poly, g, tol, max_iter, x, &it);
                ou = 1;
            } else {
                st = ssp_oracle_pcg_mixed(N, nx, D, L, Di, M, poly, g, tol, max_iter,
                                          precision == OR_FP32_REFINE64, max_outer, theta, tau_min,
                                          x, &it, &ou);
            }
            relres[p] = ssp_oracle_relres(N, nx, D, L, g, x);
            /* one FP64 solve: the recurrence residual met tol, the true one must too */
            if (precision == OR_FP64 && st == OR_OK && relres[p] > tol) st = OR_INACCURATE;
        } else {
            relres[p] = NAN;
        }
        iters[p] = it;
        outer[p] = ou;
        status[p] = st | fell_back;
        free(D); free(L); free(Di); free(M);
    }
}
