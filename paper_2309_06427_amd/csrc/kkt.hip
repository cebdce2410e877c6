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
//
// The step reads each knot's blocks once and does nx^2 multiply-adds per
// block, so it is bound by HBM.  For nx = 6, 14, 26 with nu <= nx / 2 a wave
// takes 8, 4 or 1 consecutive knots of one problem (8 or 16 lanes per knot
// for the small sizes), first copies all their blocks into LDS (contiguous
// wave-wide loads, all issued before the first LDS write) and multiplies
// from there; a lane reading its own matrix row from HBM would touch up to
// nx cache lines per load instruction.  Other sizes run one generic kernel
// that reads the rows from HBM directly.
#include "ssp_device.h"
#include "ssp_host.h"

namespace ssp {

namespace {

constexpr int kKnotsPerGroup = 4;  // wavefronts (knots) per 256-thread workgroup (generic kernels)

struct KnotRef {
    int p, k, N, nx, nu;
    bool ok;
};

// the knot of this wave: entry g of the list of (problem, knot) pairs (g >= n: none)
__device__ __forceinline__ KnotRef knot_ref(const BuildArgs &a, const int2 *list, int64_t g, int64_t n) {
    KnotRef r;
    r.ok = g < n;
    const int2 e = list[r.ok ? g : 0];
    r.p = e.x;
    r.k = e.y;
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

// ---- staged kernels (compiled state sizes) ----

template <int NX>
struct KktGeo {
    static constexpr int NUM = NX / 2;  // largest control size of the class
    static constexpr int NN = NX * NX;
    // knots per wave (consecutive knots of one problem) and lanes per knot
    static constexpr int KP = NX <= 8 ? 8 : NX <= 16 ? 4 : 1;
    static constexpr int RL = 64 / KP;
    // nx x nx blocks sit in LDS with an odd row stride (in doubles), so
    // that lanes reading their own rows hit distinct banks
    static constexpr int LD = NX | 1;
    static constexpr int NNP = NX * LD;
    // LDS doubles per wave: KP + 1 Q^-1 blocks, KP blocks of A, B, R^-1,
    // three vectors of RL entries per knot
    static constexpr int PW = (2 * KP + 1) * NNP + KP * (NX * NUM + NUM * NUM) + 3 * 64;
    static constexpr int WAVES = KP == 8 ? 4 : 1;  // waves per workgroup
};

// Workgroup index in an order that hands each XCD a contiguous run: the
// dispatcher deals workgroups to the 8 XCDs in turn, so workgroups b and
// b + 8 share an L2; they get consecutive indices here.
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t q = nb >> 3, rem = nb & 7, x = b & 7;
    return x * q + min(x, rem) + (b >> 3);
}

template <int MAXN>
constexpr int regs_for() { return (MAXN + 63) / 64; }

// n <= MAXN contiguous doubles from src into registers, lane ln taking
// elements ln, ln + 64, ...; indices past n repeat element n - 1 (src must
// hold at least one element, also for n = 0)
template <int MAXN>
__device__ __forceinline__ void ld_range(double (&v)[regs_for<MAXN>()], const double *__restrict__ src, int n,
                                         int ln) {
    const int last = max(n, 1) - 1;
#pragma unroll
    for (int t = 0; t < regs_for<MAXN>(); ++t) v[t] = src[min(t * 64 + ln, last)];
}

template <int MAXN>
__device__ __forceinline__ void st_range(double *dst, const double (&v)[regs_for<MAXN>()], int n, int ln) {
#pragma unroll
    for (int t = 0; t < regs_for<MAXN>(); ++t) {
        const int e = t * 64 + ln;
        if (e < n) dst[e] = v[t];
    }
}

// the same for consecutive row-major blocks of NC columns, stored with row
// stride LD (element e at e + (e / NC) (LD - NC))
template <int MAXN, int NC, int LD>
__device__ __forceinline__ void st_rows(double *dst, const double (&v)[regs_for<MAXN>()], int n, int ln) {
#pragma unroll
    for (int t = 0; t < regs_for<MAXN>(); ++t) {
        const int e = t * 64 + ln;
        if (e < n) dst[e + (e / NC) * (LD - NC)] = v[t];
    }
}

// sum_j M[i][j] v[j], j < NC (compile time), M row-major with row stride ld in LDS
template <int NC>
__device__ __forceinline__ double lds_row(const double *M, int ld, int i, const double *v) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) (j & 1 ? s1 : s0) += M[i * ld + j] * v[j];
    return s0 + s1;
}

// the same with a run-time column count m <= NC
template <int NC>
__device__ __forceinline__ double lds_row_n(const double *M, int ld, int i, const double *v, int m) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j)
        if (j < m) (j & 1 ? s1 : s0) += M[i * ld + j] * v[j];
    return s0 + s1;
}

// sum_j M[j][i] v[j], j < NR (compile time), M row-major with row stride ld in LDS
template <int NR>
__device__ __forceinline__ double lds_col(const double *M, int ld, int i, const double *v) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int j = 0; j < NR; ++j) (j & 1 ? s1 : s0) += M[j * ld + i] * v[j];
    return s0 + s1;
}

}  // namespace

// One wave per work item (p, k0): the knots k0 .. k0 + nk - 1 of problem p
// (nk = min(KP, N - k0)), RL lanes per knot, lane i of a knot = row i.  The
// wave issues every block load of the item before its first LDS write.

template <int NX>
__global__ __launch_bounds__(64 * KktGeo<NX>::WAVES) void k_kkt_rhs_nx(BuildArgs a, const KktRec *recs, int64_t n,
                                                                     const double *q, const double *r,
                                                                     const double *c, double *gamma) {
    using G = KktGeo<NX>;
    constexpr int NN = G::NN, NUM = G::NUM, LD = G::LD, NNP = G::NNP, KP = G::KP, RL = G::RL;
    __shared__ double sm[G::WAVES][G::PW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
    // item j + 1 reads the last Q^-1 block of item j: neighbours share an XCD
    const int64_t g = xcd_block() * G::WAVES + w;
    if (g >= n) return;  // whole wave; the kernel uses no workgroup barrier
    const KktRec it = recs[g];
    const int k0 = it.k0, N = it.N, nu = it.nu;
    const int nk = min(KP, N - k0);
    const int64_t ov = it.ov, ou = it.ou, onn = it.onn;
    // blocks in LDS: Q^-1_{k0-1+j} in Q slot j (j = 0 .. nk), and A_{k-1},
    // B_{k-1}, R^-1_{k-1} of knot k = k0 + s in slot s; k0 = 0 has no Q
    // slot 0 and no slot 0 of the others
    const int h = k0 > 0 ? 0 : 1;         // first slot present
    const int na = nk - h;                // knots k >= 1 among the item
    const int nb = nu > 0 ? na * NX * nu : 0, nr = nu > 0 ? na * nu * nu : 0;
    double *sQ = sm[w], *sA = sQ + (KP + 1) * NNP, *sB = sA + KP * NNP, *sR = sB + KP * NX * NUM;
    double *vq = sR + KP * NUM * NUM, *vp = vq + 64, *wp = vp + 64;
    const double *any = a.Qinv + onn;  // a valid address for empty ranges
    const int64_t kb = k0 - 1 + h;     // first block of the A, B, R^-1 ranges
    double rq[regs_for<(KP + 1) * NN>()], ra[regs_for<KP * NN>()], rb[regs_for<KP * NX * NUM>()],
        rr[regs_for<KP * NUM * NUM>()];
    ld_range<(KP + 1) * NN>(rq, a.Qinv + onn + (int64_t)(k0 - 1 + h) * NN, (nk + 1 - h) * NN, ln);
    ld_range<KP * NN>(ra, na ? a.A + onn + kb * NN : any, na * NN, ln);
    ld_range<KP * NX * NUM>(rb, nb ? a.B + it.onu + kb * NX * nu : any, nb, ln);
    ld_range<KP * NUM * NUM>(rr, nr ? a.Rinv + it.ouu + kb * nu * nu : any, nr, ln);
    // this lane's knot k = k0 + s and row i (clamped for the idle lanes)
    const int s = min(ln / RL, nk - 1), i = min(ln % RL, NX - 1), iu = min(ln % RL, max(nu, 1) - 1);
    const int k = k0 + s;
    const bool prev = k > 0, row = ln / RL < nk && ln % RL < NX, urow = ln / RL < nk && ln % RL < nu;
    const double qk = q[ov + (int64_t)k * NX + i];
    const double qp = prev ? q[ov + (int64_t)(k - 1) * NX + i] : 0.0;
    const double rp = prev && nu > 0 ? r[ou + (int64_t)(k - 1) * nu + iu] : 0.0;
    const double ck = c[ov + (int64_t)k * NX + i];
    st_rows<(KP + 1) * NN, NX, LD>(sQ + h * NNP, rq, (nk + 1 - h) * NN, ln);
    st_rows<KP * NN, NX, LD>(sA + h * NNP, ra, na * NN, ln);
    st_range<KP * NX * NUM>(sB + h * NX * nu, rb, nb, ln);
    st_range<KP * NUM * NUM>(sR + h * nu * nu, rr, nr, ln);
    double *vqs = vq + s * RL, *vps = vp + s * RL, *wps = wp + s * RL;
    if (row) {
        vq[ln] = qk;
        vp[ln] = qp;
    }
    if (urow) wp[ln] = rp;
    wave_sync();
    const double y = lds_row<NX>(sQ + (s + 1) * NNP, LD, i, vqs);  // (Q_k^-1 q_k)_i
    const double yp = lds_row<NX>(sQ + s * NNP, LD, i, vps);       // (Q_{k-1}^-1 q_{k-1})_i
    const double wr = lds_row_n<NUM>(sR + s * nu * nu, nu, iu, wps, nu);  // (R_{k-1}^-1 r_{k-1})_i
    wave_sync();  // vp, wp are read above before they are overwritten
    if (row) vp[ln] = prev ? yp : 0.0;
    if (urow) wp[ln] = prev ? wr : 0.0;
    wave_sync();
    const double ga = lds_row<NX>(sA + s * NNP, LD, i, vps) + lds_row_n<NUM>(sB + s * NX * nu, nu, i, wps, nu);
    if (row) gamma[ov + (int64_t)k * NX + i] = ck - y + (prev ? ga : 0.0);
}

template <int NX>
__global__ __launch_bounds__(64 * KktGeo<NX>::WAVES) void k_kkt_recover_nx(BuildArgs a, const KktRec *recs,
                                                                         int64_t n, const double *q,
                                                                         const double *r, const double *lam,
                                                                         double *dx, double *du) {
    using G = KktGeo<NX>;
    constexpr int NN = G::NN, NUM = G::NUM, LD = G::LD, NNP = G::NNP, KP = G::KP, RL = G::RL;
    __shared__ double sm[G::WAVES][G::PW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * G::WAVES + w;
    if (g >= n) return;  // whole wave; the kernel uses no workgroup barrier
    const KktRec it = recs[g];
    const int k0 = it.k0, N = it.N, nu = it.nu;
    const int nk = min(KP, N - k0);
    const int64_t ov = it.ov, ou = it.ou, onn = it.onn;
    // Q^-1_k, A_k, B_k, R^-1_k of knot k = k0 + s in slot s; the last knot
    // of the problem has no A, B, R^-1 term
    const int na = min(nk, N - 1 - k0);
    const int nb = nu > 0 ? na * NX * nu : 0, nr = nu > 0 ? na * nu * nu : 0;
    double *sQ = sm[w], *sA = sQ + KP * NNP, *sB = sA + KP * NNP, *sR = sB + KP * NX * NUM;
    double *ls = sR + KP * NUM * NUM, *tx = ls + 64, *tu = tx + 64;
    const double *any = a.Qinv + onn;
    double rq[regs_for<KP * NN>()], ra[regs_for<KP * NN>()], rb[regs_for<KP * NX * NUM>()],
        rr[regs_for<KP * NUM * NUM>()];
    ld_range<KP * NN>(rq, a.Qinv + onn + (int64_t)k0 * NN, nk * NN, ln);
    ld_range<KP * NN>(ra, na ? a.A + onn + (int64_t)k0 * NN : any, na * NN, ln);
    ld_range<KP * NX * NUM>(rb, nb ? a.B + it.onu + (int64_t)k0 * NX * nu : any, nb, ln);
    ld_range<KP * NUM * NUM>(rr, nr ? a.Rinv + it.ouu + (int64_t)k0 * nu * nu : any, nr, ln);
    const int s = min(ln / RL, nk - 1), i = min(ln % RL, NX - 1), iu = min(ln % RL, max(nu, 1) - 1);
    const int k = k0 + s;
    const bool next = k + 1 < N, row = ln / RL < nk && ln % RL < NX, urow = ln / RL < nk && ln % RL < nu;
    const double lnext = next ? lam[ov + (int64_t)(k + 1) * NX + i] : 0.0;
    const double t0 = q[ov + (int64_t)k * NX + i] + lam[ov + (int64_t)k * NX + i];
    const double s0 = next && nu > 0 ? r[ou + (int64_t)k * nu + iu] : 0.0;
    st_rows<KP * NN, NX, LD>(sQ, rq, nk * NN, ln);
    st_rows<KP * NN, NX, LD>(sA, ra, na * NN, ln);
    st_range<KP * NX * NUM>(sB, rb, nb, ln);
    st_range<KP * NUM * NUM>(sR, rr, nr, ln);
    double *lss = ls + s * RL, *txs = tx + s * RL, *tus = tu + s * RL;
    if (row) ls[ln] = lnext;
    wave_sync();
    // t = q_k + lambda_k - A_k^T lambda_{k+1};  s = r_k - B_k^T lambda_{k+1}
    const double ta = lds_col<NX>(sA + s * NNP, LD, i, lss);
    const double sb = lds_col<NX>(sB + s * NX * nu, nu, iu, lss);
    if (row) tx[ln] = next ? t0 - ta : t0;
    if (urow) tu[ln] = next ? s0 - sb : 0.0;
    wave_sync();
    const double dxi = lds_row<NX>(sQ + s * NNP, LD, i, txs);
    const double dui = lds_row_n<NUM>(sR + s * nu * nu, nu, iu, tus, nu);
    if (row) dx[ov + (int64_t)k * NX + i] = dxi;
    if (urow) du[ou + (int64_t)k * nu + iu] = next ? dui : 0.0;
}

// ---- generic kernels (any nx, nu <= 64) ----

// gamma for the knots of the list (vector layouts off_v for q, c, gamma,
// off_u for r).
__global__ __launch_bounds__(64 * kKnotsPerGroup) void k_kkt_rhs(BuildArgs a, const int2 *list, int64_t knots,
                                                               const int64_t *off_v, const int64_t *off_u,
                                                               const double *q, const double *r, const double *c,
                                                               double *gamma) {
    __shared__ double sm[kKnotsPerGroup][3 * 64];
    const KnotRef kr = knot_ref(a, list, (int64_t)blockIdx.x * kKnotsPerGroup + (threadIdx.x >> 6), knots);
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

// dx, du for the knots of the list from lambda (the library's sign).
__global__ __launch_bounds__(64 * kKnotsPerGroup) void k_kkt_recover(BuildArgs a, const int2 *list, int64_t knots,
                                                                   const int64_t *off_v, const int64_t *off_u,
                                                                   const double *q, const double *r,
                                                                   const double *lam, double *dx, double *du) {
    __shared__ double sm[kKnotsPerGroup][3 * 64];
    const KnotRef kr = knot_ref(a, list, (int64_t)blockIdx.x * kKnotsPerGroup + (threadIdx.x >> 6), knots);
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

const int kKktSizes[kKktClasses] = {6, 14, 26};

int kkt_class_of(int nx, int nu) {
    for (int c = 0; c < kKktClasses; ++c)
        if (nx == kKktSizes[c] && nu <= nx / 2) return c;
    return -1;
}

int kkt_knots_per_item(int cls) {
    switch (cls) {
    case 0: return KktGeo<6>::KP;
    case 1: return KktGeo<14>::KP;
    case 2: return KktGeo<26>::KP;
    default: return 1;
    }
}

namespace {

template <int NX>
int64_t kkt_grid(int64_t n) {
    return (n + KktGeo<NX>::WAVES - 1) / KktGeo<NX>::WAVES;
}

}  // namespace

hipError_t launch_kkt_rhs(int cls, const BuildArgs &a, const int2 *items, const KktRec *recs, int64_t n,
                          const int64_t *off_v, const int64_t *off_u, const double *q, const double *r,
                          const double *c, double *gamma, hipStream_t s) {
    if (n == 0) return hipSuccess;
    switch (cls) {
#define SSP_KKT_RHS(C, NX)                                                                                        \
    case C:                                                                                                       \
        hipLaunchKernelGGL(k_kkt_rhs_nx<NX>, dim3((unsigned)kkt_grid<NX>(n)), dim3(64 * KktGeo<NX>::WAVES), 0, s, \
                           a, recs, n, q, r, c, gamma);                                                            \
        break;
        SSP_KKT_RHS(0, 6)
        SSP_KKT_RHS(1, 14)
        SSP_KKT_RHS(2, 26)
#undef SSP_KKT_RHS
    default:
        hipLaunchKernelGGL(k_kkt_rhs, dim3((unsigned)((n + kKnotsPerGroup - 1) / kKnotsPerGroup)),
                           dim3(64 * kKnotsPerGroup), 0, s, a, items, n, off_v, off_u, q, r, c, gamma);
    }
    return hipGetLastError();
}

hipError_t launch_kkt_recover(int cls, const BuildArgs &a, const int2 *items, const KktRec *recs, int64_t n,
                              const int64_t *off_v, const int64_t *off_u, const double *q, const double *r,
                              const double *lam, double *dx, double *du, hipStream_t s) {
    if (n == 0) return hipSuccess;
    switch (cls) {
#define SSP_KKT_REC(C, NX)                                                                                  \
    case C:                                                                                                 \
        hipLaunchKernelGGL(k_kkt_recover_nx<NX>, dim3((unsigned)kkt_grid<NX>(n)), dim3(64 * KktGeo<NX>::WAVES), \
                           0, s, a, recs, n, q, r, lam, dx, du);                                             \
        break;
        SSP_KKT_REC(0, 6)
        SSP_KKT_REC(1, 14)
        SSP_KKT_REC(2, 26)
#undef SSP_KKT_REC
    default:
        hipLaunchKernelGGL(k_kkt_recover, dim3((unsigned)((n + kKnotsPerGroup - 1) / kKnotsPerGroup)),
                           dim3(64 * kKnotsPerGroup), 0, s, a, items, n, off_v, off_u, q, r, lam, dx, du);
    }
    return hipGetLastError();
}

}  // namespace ssp
