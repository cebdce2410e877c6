// The KKT step around the Schur-complement solve (Sec. II-A, Eq. (schur) and
// the zeta block definitions), in FP64, knot-parallel.
//
// The KKT system of the QP is [G C^T; C 0] [dz; lambda*] = [g; c] with
// G = blkdiag(Q_0, R_0, ..., R_{N-2}, Q_{N-1}), g = (q_0, r_0, ..., q_{N-1});
// the paper's block form of gamma, c + (-Q_0^-1 q_0, zeta_0, zeta_1, ...) with
// zeta_k = A_k Q_k^-1 q_k + B_k R_k^-1 r_k - Q_{k+1}^-1 q_{k+1}, fixes C's block
// rows: +I on x_0, and (-A_k, -B_k, +I) on (x_k, u_k, x_{k+1}).  The library
// solves the negated Schur complement, so its lambda is -lambda*:
//   right-hand side   gamma_0 = c_0 - Q_0^-1 q_0,
//                     gamma_k = c_k + A_{k-1} Q_{k-1}^-1 q_{k-1} + B_{k-1} R_{k-1}^-1 r_{k-1} - Q_k^-1 q_k,
//   recovery          dx_k = Q_k^-1 (q_k + lambda_k - A_k^T lambda_{k+1})   (no lambda_N term),
//                     du_k = R_k^-1 (r_k - B_k^T lambda_{k+1})   (k <= N-2; du_{N-1} = 0).
// Q_k^-1 and R_k^-1 are the FP64 inverses the last ssp_build left in its
// workspaces.  One wavefront per knot, lane i = row i; the small vectors
// (Q^-1 q, R^-1 r, the bracketed terms) pass through LDS.
#include "ssp_device.h"
#include "ssp_host.h"

namespace ssp {

namespace {

constexpr int kKnotsPerGroup = 4;  // wavefronts (knots) per 256-thread workgroup

struct KnotRef {
    int p, k, N, nx, nu;
    bool ok;
};

__device__ __forceinline__ KnotRef knot_ref(const BuildArgs &a, int64_t knots) {
    KnotRef r;
    const int64_t g = (int64_t)blockIdx.x * kKnotsPerGroup + (threadIdx.x >> 6);
    r.ok = g < knots;
    const int64_t gg = r.ok ? g : 0;
    r.p = a.knot_prob[gg];
    r.k = (int)(gg - a.koff[r.p]);
    r.N = a.N[r.p];
    r.nx = a.nx[r.p];
    r.nu = a.nu[r.p];
    return r;
}

// y_i = sum_j M[i][j] v[j] (M row-major n x m in global memory, v in LDS)
__device__ __forceinline__ double row_mv(const double *__restrict__ M, int i, int m, const double *v) {
    double s0 = 0.0, s1 = 0.0;
    int j = 0;
    for (; j + 2 <= m; j += 2) {
        s0 += M[(int64_t)i * m + j] * v[j];
        s1 += M[(int64_t)i * m + j + 1] * v[j + 1];
    }
    if (j < m) s0 += M[(int64_t)i * m + j] * v[j];
    return s0 + s1;
}

// y_i = sum_j M[j][i] v[j] (column i of the n x m row-major M, v of length n in LDS)
__device__ __forceinline__ double col_mv(const double *__restrict__ M, int i, int n, int m, const double *v) {
    double s0 = 0.0, s1 = 0.0;
    int j = 0;
    for (; j + 2 <= n; j += 2) {
        s0 += M[(int64_t)j * m + i] * v[j];
        s1 += M[(int64_t)(j + 1) * m + i] * v[j + 1];
    }
    if (j < n) s0 += M[(int64_t)j * m + i] * v[j];
    return s0 + s1;
}

}  // namespace

// gamma for every knot of the batch (vector layouts off_v for q, c, gamma,
// off_u for r).
__global__ __launch_bounds__(64 * kKnotsPerGroup) void k_kkt_rhs(BuildArgs a, const int64_t *off_v,
                                                               const int64_t *off_u, const double *q,
                                                               const double *r, const double *c, double *gamma,
                                                               int64_t knots) {
    __shared__ double sm[kKnotsPerGroup][3 * 64];
    const KnotRef kr = knot_ref(a, knots);
    const int i = threadIdx.x & 63;
    double *vq = sm[threadIdx.x >> 6], *vp = vq + 64, *wp = vp + 64;
    const int nx = kr.nx, nu = kr.nu, k = kr.k, p = kr.p;
    const int64_t ov = off_v[p], onn = a.off_nn[p], onu = a.off_nu[p], ouu = a.off_uu[p], ou = off_u[p];
    // q_k and, for k >= 1, q_{k-1}, r_{k-1} into LDS
    if (kr.ok && i < nx) {
        vq[i] = q[ov + (int64_t)k * nx + i];
        if (k > 0) vp[i] = q[ov + (int64_t)(k - 1) * nx + i];
    }
    if (kr.ok && k > 0 && i < nu) wp[i] = r[ou + (int64_t)(k - 1) * nu + i];
    wave_sync();
    double y = 0.0, yp = 0.0, wr = 0.0;
    if (kr.ok && i < nx) {
        y = row_mv(a.Qinv + onn + (int64_t)k * nx * nx, i, nx, vq);                  // (Q_k^-1 q_k)_i
        if (k > 0) yp = row_mv(a.Qinv + onn + (int64_t)(k - 1) * nx * nx, i, nx, vp);  // (Q_{k-1}^-1 q_{k-1})_i
    }
    if (kr.ok && k > 0 && i < nu) wr = row_mv(a.Rinv + ouu + (int64_t)(k - 1) * nu * nu, i, nu, wp);
    wave_sync();  // vp, wp are read above before they are overwritten
    if (kr.ok && k > 0) {
        if (i < nx) vp[i] = yp;
        if (i < nu) wp[i] = wr;
    }
    wave_sync();
    if (kr.ok && i < nx) {
        double g = c[ov + (int64_t)k * nx + i] - y;
        if (k > 0) {
            g += row_mv(a.A + onn + (int64_t)(k - 1) * nx * nx, i, nx, vp);
            if (nu > 0) g += row_mv(a.B + onu + (int64_t)(k - 1) * nx * nu, i, nu, wp);
        }
        gamma[ov + (int64_t)k * nx + i] = g;
    }
}

// dx, du for every knot of the batch from lambda (the library's sign).
__global__ __launch_bounds__(64 * kKnotsPerGroup) void k_kkt_recover(BuildArgs a, const int64_t *off_v,
                                                                   const int64_t *off_u,
                                                                   const double *q, const double *r,
                                                                   const double *lam, double *dx, double *du,
                                                                   int64_t knots) {
    __shared__ double sm[kKnotsPerGroup][3 * 64];
    const KnotRef kr = knot_ref(a, knots);
    const int i = threadIdx.x & 63;
    double *ln = sm[threadIdx.x >> 6], *tx = ln + 64, *tu = tx + 64;
    const int nx = kr.nx, nu = kr.nu, k = kr.k, p = kr.p, N = kr.N;
    const int64_t ov = off_v[p], onn = a.off_nn[p], onu = a.off_nu[p], ouu = a.off_uu[p], ou = off_u[p];
    const bool next = k + 1 < N;
    if (kr.ok && next && i < nx) ln[i] = lam[ov + (int64_t)(k + 1) * nx + i];
    wave_sync();
    // t = q_k + lambda_k - A_k^T lambda_{k+1};  s = r_k - B_k^T lambda_{k+1}
    if (kr.ok && i < nx) {
        double t = q[ov + (int64_t)k * nx + i] + lam[ov + (int64_t)k * nx + i];
        if (next) t -= col_mv(a.A + onn + (int64_t)k * nx * nx, i, nx, nx, ln);
        tx[i] = t;
    }
    if (kr.ok && next && i < nu) {
        double s = r[ou + (int64_t)k * nu + i];
        s -= col_mv(a.B + onu + (int64_t)k * nx * nu, i, nx, nu, ln);
        tu[i] = s;
    }
    wave_sync();
    if (kr.ok && i < nx) dx[ov + (int64_t)k * nx + i] = row_mv(a.Qinv + onn + (int64_t)k * nx * nx, i, nx, tx);
    if (kr.ok && i < nu)
        du[ou + (int64_t)k * nu + i] = next ? row_mv(a.Rinv + ouu + (int64_t)k * nu * nu, i, nu, tu) : 0.0;
}

hipError_t launch_kkt_rhs(const BuildArgs &a, const int64_t *off_v, const int64_t *off_u, const double *q,
                          const double *r, const double *c, double *gamma, int64_t knots, hipStream_t s) {
    if (knots == 0) return hipSuccess;
    const int64_t groups = (knots + kKnotsPerGroup - 1) / kKnotsPerGroup;
    hipLaunchKernelGGL(k_kkt_rhs, dim3((unsigned)groups), dim3(64 * kKnotsPerGroup), 0, s, a, off_v, off_u, q, r, c,
                       gamma, knots);
    return hipGetLastError();
}

hipError_t launch_kkt_recover(const BuildArgs &a, const int64_t *off_v, const int64_t *off_u, const double *q,
                              const double *r, const double *lam, double *dx, double *du, int64_t knots,
                              hipStream_t s) {
    if (knots == 0) return hipSuccess;
    const int64_t groups = (knots + kKnotsPerGroup - 1) / kKnotsPerGroup;
    hipLaunchKernelGGL(k_kkt_recover, dim3((unsigned)groups), dim3(64 * kKnotsPerGroup), 0, s, a, off_v, off_u, q, r,
                       lam, dx, du, knots);
    return hipGetLastError();
}

}  // namespace ssp
