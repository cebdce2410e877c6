/* Exercises the oracle's C entry points on small seeded problems so that a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer can check its
 * memory accesses (test infrastructure: run by tests/test_oracle_sanitizers.py).
 * Exit status 0 when every call returned and every status is as expected. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void ssp_oracle_solve_batch(int P, const int *Ns, const int *nxs, const int *nus, const int64_t *off_nn,
                            const int64_t *off_nu, const int64_t *off_uu, const int64_t *off_v, const double *A,
                            const double *B, const double *Q, const double *R, const double *gamma, int pc,
                            int precision, double tol, int max_iter, int max_outer, double theta, double tau_min,
                            int warm_fallback, double *lam, int *iters, int *outer, double *relres, int *status);
void ssp_oracle_build_batch(int P, const int *Ns, const int *nxs, const int *nus, const int64_t *off_nn,
                            const int64_t *off_nu, const int64_t *off_uu, const double *A, const double *B,
                            const double *Q, const double *R, int pc, int *status);
int ssp_oracle_build(int N, int nx, int nu, const double *A, const double *B, const double *Q, const double *R,
                     int pc, double *D, double *L, double *Dinv, double *M);
int ssp_oracle_direct(int N, int nx, const double *D, const double *L, const double *gamma, double *lam);
int ssp_oracle_kkt_rhs(int N, int nx, int nu, const double *A, const double *B, const double *Q, const double *R,
                       const double *q, const double *r, const double *c, double *gamma);
int ssp_oracle_kkt_recover(int N, int nx, int nu, const double *A, const double *B, const double *Q,
                           const double *R, const double *q, const double *r, const double *lam, double *dx,
                           double *du);

static uint64_t state = 88172645463325252ull;
static double unif(void) {  /* xorshift64, uniform in (-1, 1) */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 4503599627370496.0 - 1.0;
}

/* SPD block: I + G G^T / n */
static void spd(int n, double *M) {
    double *G = malloc(sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) G[i] = unif();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int l = 0; l < n; ++l) s += G[i * n + l] * G[j * n + l] / n;
            M[i * n + j] = s;
        }
    free(G);
}

int main(void) {
    enum { P = 5 };
    const int Ns[P] = {1, 2, 7, 13, 4}, nxs[P] = {3, 5, 6, 4, 2}, nus[P] = {2, 0, 3, 4, 1};
    int64_t onn[P + 1] = {0}, onu[P + 1] = {0}, ouu[P + 1] = {0}, ov[P + 1] = {0}, ou[P + 1] = {0};
    for (int p = 0; p < P; ++p) {
        onn[p + 1] = onn[p] + (int64_t)Ns[p] * nxs[p] * nxs[p];
        onu[p + 1] = onu[p] + (int64_t)Ns[p] * nxs[p] * nus[p];
        ouu[p + 1] = ouu[p] + (int64_t)Ns[p] * nus[p] * nus[p];
        ov[p + 1] = ov[p] + (int64_t)Ns[p] * nxs[p];
        ou[p + 1] = ou[p] + (int64_t)Ns[p] * nus[p];
    }
    double *A = malloc(sizeof(double) * onn[P]), *Q = malloc(sizeof(double) * onn[P]);
    double *B = malloc(sizeof(double) * (onu[P] + 1)), *R = malloc(sizeof(double) * (ouu[P] + 1));
    double *g = malloc(sizeof(double) * ov[P]), *lam = malloc(sizeof(double) * ov[P]);
    for (int p = 0; p < P; ++p) {
        const int N = Ns[p], nx = nxs[p], nu = nus[p];
        for (int k = 0; k < N; ++k) {
            double *a = A + onn[p] + (int64_t)k * nx * nx;
            for (int i = 0; i < nx * nx; ++i) a[i] = (i % (nx + 1) == 0 ? 1.0 : 0.0) + 0.05 * unif();
            spd(nx, Q + onn[p] + (int64_t)k * nx * nx);
            for (int i = 0; i < nx * nu; ++i) B[onu[p] + (int64_t)k * nx * nu + i] = 0.1 * unif();
            if (nu) spd(nu, R + ouu[p] + (int64_t)k * nu * nu);
        }
    }
    for (int64_t i = 0; i < ov[P]; ++i) g[i] = unif();
    int it[P], outer[P], st[P], bst[P];
    double rr[P];
    int bad = 0;
    for (int pc = 0; pc <= 5; ++pc)
        for (int prec = 0; prec <= 2; ++prec)
            for (int warm = 0; warm <= 1; ++warm) {
                for (int64_t i = 0; i < ov[P]; ++i) lam[i] = warm ? 0.5 * unif() : 0.0;
                ssp_oracle_solve_batch(P, Ns, nxs, nus, onn, onu, ouu, ov, A, B, Q, R, g, pc, prec,
                                       prec == 1 ? 1e-5 : 1e-8, 2000, 5, 0.5, 1e-6, warm, lam, it, outer, rr, st);
                for (int p = 0; p < P; ++p) bad += (st[p] & 7) == 1 || (st[p] & 7) == 3;
            }
    ssp_oracle_build_batch(P, Ns, nxs, nus, onn, onu, ouu, A, B, Q, R, 2, bst);
    for (int p = 0; p < P; ++p) {
        bad += bst[p] != 0;
        const int N = Ns[p], nx = nxs[p], nu = nus[p];
        const size_t nb = (size_t)N * nx * nx;
        double *D = malloc(sizeof(double) * nb), *L = malloc(sizeof(double) * nb);
        double *Di = malloc(sizeof(double) * nb), *M = malloc(sizeof(double) * nb);
        double *x = malloc(sizeof(double) * N * nx), *q = malloc(sizeof(double) * N * nx);
        double *c = malloc(sizeof(double) * N * nx), *gm = malloc(sizeof(double) * N * nx);
        double *dx = malloc(sizeof(double) * N * nx);
        double *r = malloc(sizeof(double) * (N * nu + 1)), *du = malloc(sizeof(double) * (N * nu + 1));
        for (int i = 0; i < N * nx; ++i) q[i] = unif(), c[i] = unif();
        for (int i = 0; i < N * nu; ++i) r[i] = unif();
        bad += ssp_oracle_build(N, nx, nu, A + onn[p], B + onu[p], Q + onn[p], R + ouu[p], 2, D, L, Di, M) != 0;
        bad += ssp_oracle_direct(N, nx, D, L, g + ov[p], x) != 0;
        bad += ssp_oracle_kkt_rhs(N, nx, nu, A + onn[p], B + onu[p], Q + onn[p], R + ouu[p], q, r, c, gm) != 0;
        bad += ssp_oracle_kkt_recover(N, nx, nu, A + onn[p], B + onu[p], Q + onn[p], R + ouu[p], q, r, x, dx,
                                      du) != 0;
        free(D); free(L); free(Di); free(M); free(x); free(q); free(c); free(gm); free(dx); free(r); free(du);
    }
    free(A); free(Q); free(B); free(R); free(g); free(lam);
    printf("oracle driver: %d unexpected statuses\n", bad);
    return bad != 0;
}
