// Assembly of S and Phi^-1 with the matrices held in registers, one lane
// per matrix row, for state sizes compiled in (nx = 6, 14, 26, 36).
//
// A wavefront holds kw = floor(64 / nx) knots; lane l works on row l % nx of
// knot l / nx, so all rows of a knot live in one wave and exchange data
// through a per-knot LDS buffer under wave-local ordering only.  Workgroups
// walk a list of (problem, first knot) items of one state size.
//
// Phase 1: Q_k^-1, R_k^-1 (Sec. II-A block entries).
// Phase 2: L_k = -A_{k-1} Q_{k-1}^-1,
//          D_k = Q_k^-1 + A_{k-1} Q_{k-1}^-1 A_{k-1}^T + B_{k-1} R_{k-1}^-1 B_{k-1}^T
//          (negated Eq. (schur) blocks), D_k^-1 (the block-Jacobi inverse,
//          Eq. (jacobi)), stored interleaved per knot as D_k, L_k, D_k^-1.
// SPD inverses are Gauss-Jordan eliminations without pivoting: for an SPD
// matrix every pivot is a positive Schur-complement diagonal, so a
// non-positive pivot flags the matrix as not positive definite.
//
// Scaled basis (when asked for): in phase 2, instead of D_k^-1, the inverse
// W_k = C_k^-1 of the Cholesky factor C_k of D_k (D_k = C_k C_k^T, W_k lower
// triangular), and in phase 3 the off-diagonal blocks Oh_k = W_k L_k W_{k-1}^T
// of the congruence W S W^T = I + Oh (W = blockdiag(W_k)), which the scaled
// solve streams instead of D, L, D^-1.
#include "ssp_device.h"
#include "ssp_host.h"
#include "ssp_sweep.h"

namespace ssp {

namespace {

constexpr int kThreads = 128;
constexpr int kGjBlock = 2;  // pivots per LDS exchange of the Gauss-Jordan inverses

typedef double f64x2 __attribute__((ext_vector_type(2)));

// per-lane place in the knot mapping
template <int NX>
struct Lane {
    static constexpr int KW = 64 / NX;       // knots per wave
    static constexpr int NP = (NX + 1) & ~1;  // LDS row pitch (16-byte rows)
    int g, i, knot;                           // knot slot in the workgroup, row, knot index
    bool row;                                 // this lane holds a row of a real knot
};

template <int NX>
__device__ __forceinline__ Lane<NX> lane_of(int k0, int N) {
    Lane<NX> L;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kl = lane / NX;
    // the spare lanes at the top of a wave (kl == KW) share the wave's last
    // knot buffer: they never write LDS or memory and their flags are unused
    L.g = w * Lane<NX>::KW + (kl < Lane<NX>::KW ? kl : Lane<NX>::KW - 1);
    L.i = lane - kl * NX;
    L.knot = k0 + L.g;
    L.row = kl < Lane<NX>::KW && L.knot < N;
    return L;
}

// LDS of one knot: an NX x NX matrix (row pitch NP) and a pivot row.
template <int NX>
constexpr int knot_lds_doubles() {
    return NX * Lane<NX>::NP + Lane<NX>::NP;
}

// Read n = NX doubles of an LDS row (16-byte aligned) into registers.
template <int NX>
__device__ __forceinline__ void lds_row(const double *p, double (&r)[NX]) {
    static_for<0, NX / 2>([&](auto hc) {
        constexpr int j = 2 * decltype(hc)::value;
        const f64x2 v = *(const f64x2 *)(p + j);
        r[j] = v.x;
        r[j + 1] = v.y;
    });
    if constexpr (NX % 2) r[NX - 1] = p[NX - 1];
}

template <int NX>
__device__ __forceinline__ void lds_put_row(double *p, const double (&r)[NX]) {
    static_for<0, NX / 2>([&](auto hc) {
        constexpr int j = 2 * decltype(hc)::value;
        f64x2 v;
        v.x = r[j];
        v.y = r[j + 1];
        *(f64x2 *)(p + j) = v;
    });
    if constexpr (NX % 2) p[NX - 1] = r[NX - 1];
}

// Gauss-Jordan inverse of the n x n SPD matrix (n <= NX) whose row i this
// lane holds in a[] (lanes i >= n of the knot only take part in the
// ordering).  M: the knot's LDS buffer, used for the pivot row.  Returns
// false if a pivot is not positive.
template <int NX>
__device__ __forceinline__ bool gj_inverse(double (&a)[NX], int i, bool row, int n, double *M) {
    constexpr int NP = Lane<NX>::NP;
    double *prow = M + NX * NP;
    bool ok = true;
    static_for<0, NX>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (k < n) {
            if (row && i == k) lds_put_row<NX>(prow, a);
            wave_sync();
            double pr[NX];
            lds_row<NX>(prow, pr);
            wave_sync();  // the pivot row is read before the next one is written
            const double inv = 1.0 / pr[k];
            if (!(pr[k] > 0.0)) ok = false;
            if (i == k) {
                static_for<0, NX>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    a[j] = j == k ? inv : pr[j] * inv;
                });
            } else {
                const double g = a[k] * inv;  // row multiple of the unscaled pivot row
                static_for<0, NX>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    a[j] = j == k ? -g : fma(-g, pr[j], a[j]);
                });
            }
        }
    });
    return ok;
}

// The same inverse with BK pivots per exchange: the pivot lanes of a block
// k0 .. k0+bk-1 publish their rows in LDS once; every lane inverts the bk x bk
// pivot block B itself (Gauss-Jordan on scalars, the same pivots as the
// one-at-a-time elimination, checked for positivity) and applies the whole
// block: a non-pivot row becomes a - c P with c = a_K B^-1 (P: the pivot
// rows, K: the block's columns, which become -c), pivot row m becomes
// (B^-1 P)_m (its K columns (B^-1)_m), written as a - g P with
// g = e_m - (B^-1)_m since a = P_m.  M: the knot's LDS buffer, whose first
// BK rows hold the pivot rows.  Returns false if a pivot is not positive.
template <int NX, int BK>
__device__ __forceinline__ bool gj_inverse_blocked(double (&a)[NX], int i, bool row, int n, double *M) {
    constexpr int NP = Lane<NX>::NP;
    bool ok = true;
    static_for<0, (NX + BK - 1) / BK>([&](auto bc) {
        constexpr int k0 = decltype(bc)::value * BK;
        constexpr int bk = NX - k0 < BK ? NX - k0 : BK;
        if (k0 < n) {
            const int me = (row && i >= k0 && i < k0 + bk && i < n) ? i - k0 : -1;
            if (me >= 0) lds_put_row<NX>(M + me * NP, a);
            wave_sync();
            // B^-1 of the valid part of the block (m < n - k0); the rest acts as identity
            double B[bk][bk];
            static_for<0, bk>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                static_for<0, bk>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    const bool v = k0 + m < n && k0 + q < n;
                    B[m][q] = v ? M[m * NP + k0 + q] : (m == q ? 1.0 : 0.0);
                });
            });
            static_for<0, bk>([&](auto pc) {
                constexpr int pv = decltype(pc)::value;
                if (!(B[pv][pv] > 0.0)) ok = false;
                const double inv = 1.0 / B[pv][pv];
                static_for<0, bk>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    B[pv][q] = q == pv ? inv : B[pv][q] * inv;
                });
                static_for<0, bk>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    if (m != pv) {
                        const double f = B[m][pv];
                        static_for<0, bk>([&](auto qc) {
                            constexpr int q = decltype(qc)::value;
                            B[m][q] = q == pv ? -f * inv : fma(-f, B[pv][q], B[m][q]);
                        });
                    }
                });
            });
            // g: c = a_K B^-1 for a non-pivot row, e_me - (B^-1)_me for pivot row me
            double g[bk], kc[bk];
            static_for<0, bk>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                double c = 0.0;
                static_for<0, bk>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    c = fma(a[k0 + q], B[q][m], c);
                });
                double bm = 0.0;  // (B^-1)[me][m]
                static_for<0, bk>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    if (me == q) bm = B[q][m];
                });
                g[m] = me >= 0 ? ((me == m ? 1.0 : 0.0) - bm) : c;
                kc[m] = me >= 0 ? bm : -c;  // the new K column m of this row
                if (k0 + m >= n) g[m] = 0.0;
            });
            // a_j -= sum_m g_m P_mj outside the block's columns, read two entries at a time
            static_for<0, NX / 2>([&](auto hc) {
                constexpr int j = 2 * decltype(hc)::value;
                double s0 = a[j], s1 = a[j + 1];
                static_for<0, bk>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    const f64x2 v = *(const f64x2 *)(M + m * NP + j);
                    s0 = fma(-g[m], v.x, s0);
                    s1 = fma(-g[m], v.y, s1);
                });
                a[j] = s0;
                a[j + 1] = s1;
            });
            if constexpr (NX % 2) {
                constexpr int j = NX - 1;
                double s0 = a[j];
                static_for<0, bk>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    s0 = fma(-g[m], M[m * NP + j], s0);
                });
                a[j] = s0;
            }
            static_for<0, bk>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                if (k0 + m < n) a[k0 + m] = kc[m];
            });
            wave_sync();  // the pivot rows are read before the next block's are written
        }
    });
    return ok;
}

// W = C^-1 for the Cholesky factor C of the SPD matrix (A = C C^T) whose
// row i this lane holds in a[] (every lane of the knot holds one row), in
// place: afterwards a[] is row i of W (lower triangular).  Forward Gaussian
// elimination of [A | I] without pivoting (stable for SPD A): at step j the
// pivot lane publishes its row, lanes below subtract f = a_ij / u_jj times
// it, which leaves U (upper, pivots u_jj on its diagonal) on the right and
// E = L^-1 (unit lower) on the left of the same row storage (entry j of a
// lower row becomes -f, E's new entry; its other entries update alike).
// With A = L diag(u) L^T, W = diag(u)^-1/2 L^-1.  M: the knot's LDS buffer
// (pivot row).  Returns false if a pivot is not positive.
template <int NX>
__device__ __forceinline__ bool lower_inverse_rows(double (&a)[NX], int i, bool row, double *M) {
    constexpr int NP = Lane<NX>::NP;
    double *prow = M + NX * NP;
    bool ok = true;
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (row && i == j) lds_put_row<NX>(prow, a);
        wave_sync();
        double pr[NX];
        lds_row<NX>(prow, pr);
        wave_sync();  // the pivot row is read before the next one is written
        if (!(pr[j] > 0.0)) ok = false;
        if (i > j) {
            const double f = a[j] / pr[j];
            static_for<0, NX>([&](auto lc) {
                constexpr int l = decltype(lc)::value;
                if constexpr (l != j) a[l] = fma(-f, pr[l], a[l]);
            });
            a[j] = -f;
        }
    });
    // this lane's pivot u_ii sits at a[i]; scale E's row by u_ii^-1/2
    double u = 0.0;
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j == i) u = a[j];
    });
    const double s = 1.0 / sqrt(u);
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        a[j] = j < i ? a[j] * s : (j == i ? s : 0.0);
    });
    return ok;
}

// out = x M (M: n x NX in LDS, rows of pitch NP), x: this lane's row.
template <int NX>
__device__ __forceinline__ void row_times(const double (&x)[NX], const double *M, int n, double (&out)[NX]) {
    constexpr int NP = Lane<NX>::NP;
    static_for<0, NX>([&](auto jc) { out[decltype(jc)::value] = 0.0; });
    static_for<0, NX>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        if (l < n) {
            double m[NX];
            lds_row<NX>(M + l * NP, m);
            static_for<0, NX>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                out[j] += x[l] * m[j];
            });
        }
    });
}

// out[j] += sum_{l < n} x[l] M[j][l] for j < NX (x M^T, M: NX x n in LDS).
template <int NX>
__device__ __forceinline__ void row_times_t(const double (&x)[NX], const double *M, int n, double (&out)[NX]) {
    constexpr int NP = Lane<NX>::NP;
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        double m[NX];
        lds_row<NX>(M + j * NP, m);
        double s = 0.0;
        static_for<0, NX>([&](auto lc) {
            constexpr int l = decltype(lc)::value;
            if (l < n) s += x[l] * m[l];
        });
        out[j] += s;
    });
}

// Replace a[] (row i of a matrix that should be symmetric) by row i of
// (M + M^T) / 2 through the knot's LDS buffer.
template <int NX>
__device__ __forceinline__ void symmetrise(double (&a)[NX], int i, bool row, double *M) {
    constexpr int NP = Lane<NX>::NP;
    wave_sync();
    if (row) lds_put_row<NX>(M + i * NP, a);
    wave_sync();
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        a[j] = 0.5 * (a[j] + M[j * NP + i]);
    });
    wave_sync();
}

// Load n entries of a global row into registers (entries >= n set to 0).
template <int NX>
__device__ __forceinline__ void load_row(const double *__restrict__ src, int n, double (&r)[NX]) {
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        r[j] = j < n ? src[j] : 0.0;
    });
}

// Load a full row of NX entries of the storage type into FP64 registers.
template <typename TM, int NX>
__device__ __forceinline__ void load_row_t(const TM *__restrict__ src, double (&r)[NX]) {
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        r[j] = (double)src[j];
    });
}

template <int NX>
__device__ __forceinline__ void store_row(double *__restrict__ dst, int n, const double (&r)[NX]) {
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j < n) dst[j] = r[j];
    });
}

// Store a row in the storage type (scale applied), with its FP32 remainder.
template <typename TM, int NX>
__device__ __forceinline__ void store_split_row(TM *__restrict__ hi, float *__restrict__ lo, const double (&r)[NX],
                                                double scale) {
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        const double v = scale * r[j];
        const TM h = (TM)v;
        hi[j] = h;
        if (lo) lo[j] = (float)(v - (double)h);
    });
}

// Store the upper-triangle part (j >= i) of row i of a symmetric matrix into
// its packed form (entry (i, j) at packed_row(i) + j), with the FP32 remainder.
template <typename TM, int NX>
__device__ __forceinline__ void store_split_packed_row(TM *__restrict__ hi, float *__restrict__ lo, int i,
                                                       const double (&r)[NX]) {
    const int base = packed_row(i, NX);
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j >= i) {
            const double v = r[j];
            const TM h = (TM)v;
            hi[base + j] = h;
            if (lo) lo[base + j] = (float)(v - (double)h);
        }
    });
}

}  // namespace

// Phase 1 for one state size: Q_k^-1 for every knot and R_k^-1 for k < N-1
// (requires nu <= NX).
template <int NX>
__global__ __launch_bounds__(kThreads) void k_build_inv_nx(BuildArgs a, const int2 *items) {
    constexpr int KN = (kThreads / 64) * Lane<NX>::KW;  // knots per workgroup
    __shared__ __align__(16) double sm[KN * knot_lds_doubles<NX>()];
    const int2 it = items[blockIdx.x];
    const int p = it.x, N = a.N[p], nu = a.nu[p];
    const Lane<NX> ln = lane_of<NX>(it.y, N);
    double *M = sm + ln.g * knot_lds_doubles<NX>();
    const int nn = NX * NX;
    bool ok = true;
    double r[NX];
    const int64_t oq = a.off_nn[p] + (int64_t)ln.knot * nn + ln.i * NX;
    if (ln.row) load_row<NX>(a.Q + oq, NX, r);
    ok = gj_inverse_blocked<NX, kGjBlock>(r, ln.i, ln.row, NX, M) && ok;
    if (ln.row) store_row<NX>(a.Qinv + oq, NX, r);
    if (nu > 0) {
        const bool rrow = ln.row && ln.knot < N - 1 && ln.i < nu;
        const int64_t orr = a.off_uu[p] + (int64_t)ln.knot * nu * nu + ln.i * nu;
        if (rrow) load_row<NX>(a.R + orr, nu, r);
        const bool okr = gj_inverse_blocked<NX, kGjBlock>(r, ln.i, rrow, nu, M);
        if (ln.knot < N - 1) ok = okr && ok;
        if (rrow) store_row<NX>(a.Rinv + orr, nu, r);
    }
    if (ln.row && !ok) atomicOr(a.status + p, kNotSpd);
}

// Phase 2 for one state size: D_k, L_k (storage type, FP32 remainder under
// FP32 storage) and D_k^-1, interleaved per knot (D_k and D_k^-1 packed).
template <typename TM, int NX>
__global__ __launch_bounds__(kThreads) void k_build_asm_nx(BuildArgs a, const int2 *items) {
    constexpr int KN = (kThreads / 64) * Lane<NX>::KW;
    constexpr int NP = Lane<NX>::NP;
    __shared__ __align__(16) double sm[KN * knot_lds_doubles<NX>()];
    const int2 it = items[blockIdx.x];
    const int p = it.x, N = a.N[p], nu = a.nu[p];
    const Lane<NX> ln = lane_of<NX>(it.y, N);
    double *M = sm + ln.g * knot_lds_doubles<NX>();
    const int nn = NX * NX, k = ln.knot, i = ln.i;
    const int bs = block_stride(NX, sizeof(TM)), bp = packed_stride(NX, sizeof(TM));
    TM *blk = (TM *)a.B3 + a.off_b3[p] + (int64_t)k * (2 * bp + bs);  // D_k (packed), L_k, D_k^-1 (packed)
    const int64_t ol = a.off_blk[p] + (int64_t)k * bs;               // remainder of L_k
    const int64_t od = a.off_pk[p] + (int64_t)k * bp;                // remainder of D_k (packed)
    const bool prev = ln.row && k > 0;

    double d[NX], t[NX];
    if (ln.row) load_row<NX>(a.Qinv + a.off_nn[p] + (int64_t)k * nn + i * NX, NX, d);  // Q_k^-1
    // L_k = -A_{k-1} Q_{k-1}^-1 ; D_k += A_{k-1} Q_{k-1}^-1 A_{k-1}^T
    wave_sync();
    if (prev) store_row<NX>(M + i * NP, NX, *(const double(*)[NX])(a.Qinv + a.off_nn[p] + (int64_t)(k - 1) * nn +
                                                                       i * NX));
    wave_sync();
    double x[NX];
    if (prev) load_row<NX>(a.A + a.off_nn[p] + (int64_t)(k - 1) * nn + i * NX, NX, x);
    row_times<NX>(x, M, NX, t);  // t = row i of A Q^-1 (= phi)
    if (!prev) static_for<0, NX>([&](auto jc) { t[decltype(jc)::value] = 0.0; });  // L_0 = 0
    wave_sync();
    if (prev) lds_put_row<NX>(M + i * NP, x);  // rows of A_{k-1}
    wave_sync();
    if (prev) row_times_t<NX>(t, M, NX, d);
    if (ln.row) store_split_row<TM, NX>(blk + bp + i * NX, a.SLlo ? a.SLlo + ol + i * NX : nullptr, t, -1.0);
    // D_k += B_{k-1} R_{k-1}^-1 B_{k-1}^T
    if (nu > 0) {
        wave_sync();
        if (prev && i < nu)
            store_row<NX>(M + i * NP, nu,
                          *(const double(*)[NX])(a.Rinv + a.off_uu[p] + (int64_t)(k - 1) * nu * nu + i * nu));
        wave_sync();
        if (prev) load_row<NX>(a.B + a.off_nu[p] + (int64_t)(k - 1) * NX * nu + i * nu, nu, x);
        row_times<NX>(x, M, nu, t);  // t = row i of B R^-1 (first nu entries)
        wave_sync();
        if (prev) lds_put_row<NX>(M + i * NP, x);  // rows of B_{k-1} (nu entries each)
        wave_sync();
        if (prev) row_times_t<NX>(t, M, nu, d);
    }
    symmetrise<NX>(d, i, ln.row, M);  // exactly symmetric before the upper triangle is kept
    if (ln.row) store_split_packed_row<TM, NX>(blk, a.SDlo ? a.SDlo + od : nullptr, i, d);
    bool ok;
    if (a.Zs) {
        // scaled basis: W_k = C_k^-1 instead of D_k^-1, stored full (zeros
        // above the diagonal) in the storage type; D_k^-1 = W_k^T W_k is
        // formed only on demand
        ok = lower_inverse_rows<NX>(d, i, ln.row, M);
        if (ln.row) store_split_row<TM, NX>((TM *)a.Zs + ol + i * NX, (float *)nullptr, d, 1.0);
    } else {
        ok = gj_inverse_blocked<NX, kGjBlock>(d, i, ln.row, NX, M);
        symmetrise<NX>(d, i, ln.row, M);
        if (ln.row) store_split_packed_row<TM, NX>(blk + bp + bs, (float *)nullptr, i, d);
    }
    if (ln.row && !ok) atomicOr(a.status + p, kNotSpd);
}

// Phase 3 of the scaled basis: Oh_k = W_k L_k W_{k-1}^T (k >= 1, Oh_0 = 0)
// in FP64 from the stored W and L_k (storage type: the block the solve
// applies is rounded to that type anyway, and the transforms use the same
// stored W), stored in the storage type.  Both products are row-times-transpose
// dot products against LDS rows: X = L_k W_{k-1}^T with the rows of W_{k-1}
// in LDS, then row i of W_k X = sum_l W_k[i][l] X[l][:] with X^T in LDS
// (lane i stores its row of X as LDS column i) and row i of W_k in registers.
template <typename TM, int NX>
__global__ __launch_bounds__(kThreads) void k_build_ohat_nx(BuildArgs a, const int2 *items) {
    constexpr int KN = (kThreads / 64) * Lane<NX>::KW;
    constexpr int NP = Lane<NX>::NP;
    __shared__ __align__(16) double sm[KN * knot_lds_doubles<NX>()];
    const int2 it = items[blockIdx.x];
    const int p = it.x, N = a.N[p];
    const Lane<NX> ln = lane_of<NX>(it.y, N);
    double *M = sm + ln.g * knot_lds_doubles<NX>();
    const int nn = NX * NX, k = ln.knot, i = ln.i;
    const int bs = block_stride(NX, sizeof(TM)), bp = packed_stride(NX, sizeof(TM));
    const int64_t ol = a.off_blk[p] + (int64_t)k * bs;
    const bool prev = ln.row && k > 0;
    double x[NX], t[NX];
    static_for<0, NX>([&](auto jc) { t[decltype(jc)::value] = 0.0; });
    if (prev) {
        load_row_t<TM, NX>((const TM *)a.Zs + ol - bs + i * NX, x);  // row i of W_{k-1}
        wave_sync();
        lds_put_row<NX>(M + i * NP, x);
        wave_sync();
        // row i of L_k
        load_row_t<TM, NX>((const TM *)a.B3 + a.off_b3[p] + (int64_t)k * (2 * bp + bs) + bp + i * NX, x);
        row_times_t<NX>(x, M, NX, t);  // t = row i of X = L_k W_{k-1}^T
        wave_sync();
        static_for<0, NX>([&](auto jc) {  // X^T: LDS column i
            constexpr int j = decltype(jc)::value;
            M[j * NP + i] = t[j];
        });
        wave_sync();
        load_row_t<TM, NX>((const TM *)a.Zs + ol + i * NX, x);  // row i of W_k
        static_for<0, NX>([&](auto jc) { t[decltype(jc)::value] = 0.0; });
        row_times_t<NX>(x, M, NX, t);  // row i of W_k X
    } else {
        // knot 0 (Oh_0 = 0) or a lane without a row: the same ordering points
        wave_sync();
        wave_sync();
        wave_sync();
        wave_sync();
    }
    if (ln.row) store_split_row<TM, NX>((TM *)a.OH + ol + i * NX, (float *)nullptr, t, 1.0);
}

template <int NX>
static hipError_t launch_nx(const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_inv_nx<NX>, dim3(nitems), dim3(kThreads), 0, s, a, items);
    hipError_t e = hipGetLastError();
    if (e) return e;
    if (fp32)
        hipLaunchKernelGGL((k_build_asm_nx<float, NX>), dim3(nitems), dim3(kThreads), 0, s, a, items);
    else
        hipLaunchKernelGGL((k_build_asm_nx<double, NX>), dim3(nitems), dim3(kThreads), 0, s, a, items);
    return hipGetLastError();
}

template <int NX>
static hipError_t launch_ohat_nx(const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL((k_build_ohat_nx<float, NX>), dim3(nitems), dim3(kThreads), 0, s, a, items);
    else
        hipLaunchKernelGGL((k_build_ohat_nx<double, NX>), dim3(nitems), dim3(kThreads), 0, s, a, items);
    return hipGetLastError();
}

hipError_t launch_build_ohat(int cls, const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s) {
    switch (cls) {
        case 0: return launch_ohat_nx<6>(a, items, nitems, fp32, s);
        case 1: return launch_ohat_nx<14>(a, items, nitems, fp32, s);
        case 2: return launch_ohat_nx<26>(a, items, nitems, fp32, s);
        case 3: return launch_ohat_nx<36>(a, items, nitems, fp32, s);
        case 4: return launch_dpp_ohat<6>(a, items, nitems, fp32, s);
        case 5: return launch_dpp_ohat<14>(a, items, nitems, fp32, s);
        case 6: return launch_dpp_ohat<26>(a, items, nitems, fp32, s);
    }
    return hipErrorInvalidValue;
}

// classes 0-3: the LDS kernels above (any nu <= nx); 4-6: the DPP-broadcast
// kernels, for nu = nx / 2.  At nx = 6 a knot fills 6 lanes of a 16-lane DPP
// row, and the LDS kernels (ten knots per wave) are faster, so class 4 is
// compiled but not chosen.
const int kBuildSizes[kBuildClasses] = {6, 14, 26, 36, 6, 14, 26};

int build_class_of(int nx, int nu) {
    for (int c = 5; c < kBuildClasses; ++c)
        if (nx == kBuildSizes[c] && 2 * nu == nx) return c;
    for (int c = 0; c < 4; ++c)
        if (nx == kBuildSizes[c] && nu <= nx) return c;
    return -1;
}

int build_knots_per_item(int cls) { return cls >= 4 ? dpp_knots_per_item() : (kThreads / 64) * (64 / kBuildSizes[cls]); }

hipError_t launch_build_class(int cls, const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s) {
    switch (cls) {
        case 0: return launch_nx<6>(a, items, nitems, fp32, s);
        case 1: return launch_nx<14>(a, items, nitems, fp32, s);
        case 2: return launch_nx<26>(a, items, nitems, fp32, s);
        case 3: return launch_nx<36>(a, items, nitems, fp32, s);
        case 4: return launch_dpp_class<6>(a, items, nitems, fp32, s);
        case 5: return launch_dpp_class<14>(a, items, nitems, fp32, s);
        case 6: return launch_dpp_class<26>(a, items, nitems, fp32, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace ssp
