// Assembly of S and the scaled basis for the compiled state sizes up to 32,
// with every broadcast operand folded into the FP64 multiply-add.
//
// Mapping: one knot per 16-lane row of a wavefront, one wave (4 knots) per
// workgroup and work item.  A matrix is held R = 1 (nx <= 16) or R = 2 rows
// per lane: lane p < P = ceil(nx / R) of the knot's row holds matrix rows p
// and p + P in its slots 0 and 1.  Row l of such a matrix sits in lane l % P,
// slot l / P; the FP64 multiply-add with DPP row_newbcast:(l % P) reads that
// lane's register for every lane of the row (v_fmac_f64_dpp).  Products and
// elimination steps therefore take no LDS traffic and no extra instruction
// per operand: an LDS broadcast read feeds one FP64 multiply-add per 8 bytes
// and runs at half the FP64 rate, the folded broadcast at the full rate.
//
// The phases and their arithmetic are those of the LDS kernels of the same
// assembly (Sec. II-A blocks, Eq. (jacobi), the scaled basis): Q_k^-1 and
// R_k^-1 by Gauss-Jordan without pivoting (a non-positive pivot flags the
// matrix as not positive definite), L_k = -A_{k-1} Q_{k-1}^-1,
// D_k = Q_k^-1 + A_{k-1} Q_{k-1}^-1 A_{k-1}^T + B_{k-1} R_{k-1}^-1 B_{k-1}^T,
// then W_k = C_k^-1 (D_k = C_k C_k^T) and Oh_k = W_k L_k W_{k-1}^T, or D_k^-1.
// Sums run in a different order.  Two differences of form: the Gauss-Jordan
// pivot row is scaled by its pivot's inverse once at the end instead of at its
// step (the row stays a fixed multiple of the usual one in between), and D_k
// is made symmetric by copying its upper triangle onto the lower one (the
// upper triangle is what is stored).
//
// Memory: the assembly kernel (which forms the inverses in registers, see
// k_bdpp_asm) moves blocks between HBM and LDS only in wave-wide copies of
// contiguous ranges, and lanes read their rows
// from LDS (a lane that loads or stores its own rows touches a separate cache
// line per lane and instruction, which bounded an earlier version in the
// memory pipeline); the Oh kernel, with few loads per knot, reads its rows
// directly.
//
// A DPP read of a VGPR needs two wait states after a VALU write to it, which
// the compiler cannot see inside the asm: every block of multiply-adds starts
// with s_nop 1 and reads no register that an earlier instruction of the block
// writes.  The blocks are not volatile, so the compiler schedules the operand
// loads ahead of them; results that only a masked store uses are pinned in
// wave-uniform code first (keep()), so no block runs with lanes masked off.
#include "ssp_device.h"
#include "ssp_host.h"
#include "ssp_sweep.h"

namespace ssp {

namespace {

constexpr int kThreadsD = 64;             // one wave
constexpr int kKnotsD = kThreadsD / 16;   // one knot per 16-lane row

template <int NX>
struct RowGeo {
    static constexpr int R = NX > 16 ? 2 : 1;      // matrix rows per lane
    static constexpr int P = (NX + R - 1) / R;     // lanes per knot
};

template <int L>
__device__ __forceinline__ double bcast(double v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + L, 0xf, 0xf, true);  // row_newbcast:L
}

#define SSP_FMAC(d, s, x, l) "v_fmac_f64_dpp %" #d ", %" #s ", %" #x " row_newbcast:%" #l " row_mask:0xf bank_mask:0xf\n\t"

// a_t += bcast_L(s_t) * x, one broadcast lane
template <int L>
__device__ __forceinline__ void fmac_l8(double &a0, double &a1, double &a2, double &a3, double &a4, double &a5,
                                        double &a6, double &a7, double s0, double s1, double s2, double s3, double s4,
                                        double s5, double s6, double s7, double x) {
    asm("s_nop 1\n\t" SSP_FMAC(0, 8, 16, 17) SSP_FMAC(1, 9, 16, 17) SSP_FMAC(2, 10, 16, 17)
                     SSP_FMAC(3, 11, 16, 17) SSP_FMAC(4, 12, 16, 17) SSP_FMAC(5, 13, 16, 17) SSP_FMAC(6, 14, 16, 17)
                         SSP_FMAC(7, 15, 16, 17)
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                 : "v"(s0), "v"(s1), "v"(s2), "v"(s3), "v"(s4), "v"(s5), "v"(s6), "v"(s7), "v"(x), "n"(L));
}
template <int L>
__device__ __forceinline__ void fmac_l4(double &a0, double &a1, double &a2, double &a3, double s0, double s1, double s2,
                                        double s3, double x) {
    asm("s_nop 1\n\t" SSP_FMAC(0, 4, 8, 9) SSP_FMAC(1, 5, 8, 9) SSP_FMAC(2, 6, 8, 9) SSP_FMAC(3, 7, 8, 9)
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
                 : "v"(s0), "v"(s1), "v"(s2), "v"(s3), "v"(x), "n"(L));
}
template <int L>
__device__ __forceinline__ void fmac_l2(double &a0, double &a1, double s0, double s1, double x) {
    asm("s_nop 1\n\t" SSP_FMAC(0, 2, 4, 5) SSP_FMAC(1, 3, 4, 5)
                 : "+v"(a0), "+v"(a1)
                 : "v"(s0), "v"(s1), "v"(x), "n"(L));
}
template <int L>
__device__ __forceinline__ void fmac_l1(double &a0, double s0, double x) {
    asm("s_nop 1\n\t" SSP_FMAC(0, 1, 2, 3) : "+v"(a0) : "v"(s0), "v"(x), "n"(L));
}

// a_t += bcast_{L_t}(s_t) * x, one broadcast lane per multiply-add
template <int L0, int L1, int L2, int L3, int L4, int L5, int L6, int L7>
__device__ __forceinline__ void fmac_j8(double &a0, double &a1, double &a2, double &a3, double &a4, double &a5,
                                        double &a6, double &a7, double s0, double s1, double s2, double s3, double s4,
                                        double s5, double s6, double s7, double x) {
    asm("s_nop 1\n\t" SSP_FMAC(0, 8, 16, 17) SSP_FMAC(1, 9, 16, 18) SSP_FMAC(2, 10, 16, 19)
                     SSP_FMAC(3, 11, 16, 20) SSP_FMAC(4, 12, 16, 21) SSP_FMAC(5, 13, 16, 22) SSP_FMAC(6, 14, 16, 23)
                         SSP_FMAC(7, 15, 16, 24)
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                 : "v"(s0), "v"(s1), "v"(s2), "v"(s3), "v"(s4), "v"(s5), "v"(s6), "v"(s7), "v"(x), "n"(L0),
                   "n"(L1), "n"(L2), "n"(L3), "n"(L4), "n"(L5), "n"(L6), "n"(L7));
}
template <int L0, int L1, int L2, int L3>
__device__ __forceinline__ void fmac_j4(double &a0, double &a1, double &a2, double &a3, double s0, double s1, double s2,
                                        double s3, double x) {
    asm("s_nop 1\n\t" SSP_FMAC(0, 4, 8, 9) SSP_FMAC(1, 5, 8, 10) SSP_FMAC(2, 6, 8, 11) SSP_FMAC(3, 7, 8, 12)
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
                 : "v"(s0), "v"(s1), "v"(s2), "v"(s3), "v"(x), "n"(L0), "n"(L1), "n"(L2), "n"(L3));
}
template <int L0, int L1>
__device__ __forceinline__ void fmac_j2(double &a0, double &a1, double s0, double s1, double x) {
    asm("s_nop 1\n\t" SSP_FMAC(0, 2, 4, 5) SSP_FMAC(1, 3, 4, 6)
                 : "+v"(a0), "+v"(a1)
                 : "v"(s0), "v"(s1), "v"(x), "n"(L0), "n"(L1));
}

#undef SSP_FMAC

__device__ __forceinline__ void keep1(double v) { asm volatile("" ::"v"(v)); }

// Settle a pivot test here: otherwise the compiler sinks the comparisons to
// the flag's last use and holds every pivot in registers until then.
__device__ __forceinline__ bool settle(bool f) {
    int v = f;
    asm volatile("" : "+v"(v));
    return v != 0;
}

// Make every value of a[][] be computed here (in wave-uniform code).
template <int R, int N>
__device__ __forceinline__ void keep(const double (&a)[R][N]) {
    static_for<0, R>([&](auto s_) {
        static_for<0, N>([&](auto jc) { keep1(a[decltype(s_)::value][decltype(jc)::value]); });
    });
}

// An empty asm that makes v depend on w: reads addressed through v stay below
// the computation of w.
__device__ __forceinline__ void tie(int &v, double w) { asm("" : "+v"(v) : "v"(w)); }

// Runs step(l, x) for l = 0 .. NL-1 with x[s] = blk[ro[s] + l] (0 where
// !live), the LDS reads of step l + 1 issued at the start of step l: the row
// offsets are tied to step l - 1's result dep(s), so the compiler cannot
// hoist the reads of all steps to the top (and spill what they occupy).
template <int NL, int R, typename T, typename Step, typename Dep>
__device__ __forceinline__ void lds_steps(const T *blk, int (&ro)[R], bool live, Step &&step, Dep &&dep) {
    double xn[R];
    static_for<0, R>([&](auto s_) { xn[decltype(s_)::value] = (double)blk[ro[decltype(s_)::value]]; });
    static_for<0, NL>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        double xc[R];
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            xc[s] = live ? xn[s] : 0.0;
        });
        if constexpr (l + 1 < NL)
            static_for<0, R>([&](auto s_) {
                constexpr int s = decltype(s_)::value;
                xn[s] = (double)blk[ro[s] + l + 1];
            });
        step(lc, xc);
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            tie(ro[s], dep(s_));
        });
    });
}

// acc[j] += bcast_L(src[j]) * x for J0 <= j < J1 (src: the same row slot in
// every lane, read from lane L)
template <int L, int J0, int J1, int N>
__device__ __forceinline__ void row_l(double (&acc)[N], const double (&src)[N], double x) {
    constexpr int c = J1 - J0;
    if constexpr (c >= 8) {
        fmac_l8<L>(acc[J0], acc[J0 + 1], acc[J0 + 2], acc[J0 + 3], acc[J0 + 4], acc[J0 + 5], acc[J0 + 6], acc[J0 + 7],
                   src[J0], src[J0 + 1], src[J0 + 2], src[J0 + 3], src[J0 + 4], src[J0 + 5], src[J0 + 6],
                   src[J0 + 7], x);
        row_l<L, J0 + 8, J1>(acc, src, x);
    } else if constexpr (c >= 4) {
        fmac_l4<L>(acc[J0], acc[J0 + 1], acc[J0 + 2], acc[J0 + 3], src[J0], src[J0 + 1], src[J0 + 2], src[J0 + 3], x);
        row_l<L, J0 + 4, J1>(acc, src, x);
    } else if constexpr (c >= 2) {
        fmac_l2<L>(acc[J0], acc[J0 + 1], src[J0], src[J0 + 1], x);
        row_l<L, J0 + 2, J1>(acc, src, x);
    } else if constexpr (c == 1) {
        fmac_l1<L>(acc[J0], src[J0], x);
    }
}

// acc[j] += bcast_{j % P}(m[j / P][E]) * x for J0 <= j < J1: element E of
// row j of a matrix held R rows per lane (the transposed product)
template <int P, int E, int J0, int J1, int R, int N, int M>
__device__ __forceinline__ void row_t(double (&acc)[N], const double (&m)[R][M], double x) {
    constexpr int c = J1 - J0;
    if constexpr (c >= 8) {
        fmac_j8<J0 % P, (J0 + 1) % P, (J0 + 2) % P, (J0 + 3) % P, (J0 + 4) % P, (J0 + 5) % P, (J0 + 6) % P,
                (J0 + 7) % P>(acc[J0], acc[J0 + 1], acc[J0 + 2], acc[J0 + 3], acc[J0 + 4], acc[J0 + 5], acc[J0 + 6],
                              acc[J0 + 7], m[J0 / P][E], m[(J0 + 1) / P][E], m[(J0 + 2) / P][E],
                              m[(J0 + 3) / P][E], m[(J0 + 4) / P][E], m[(J0 + 5) / P][E], m[(J0 + 6) / P][E],
                              m[(J0 + 7) / P][E], x);
        row_t<P, E, J0 + 8, J1>(acc, m, x);
    } else if constexpr (c >= 4) {
        fmac_j4<J0 % P, (J0 + 1) % P, (J0 + 2) % P, (J0 + 3) % P>(acc[J0], acc[J0 + 1], acc[J0 + 2], acc[J0 + 3],
                                                                  m[J0 / P][E], m[(J0 + 1) / P][E],
                                                                  m[(J0 + 2) / P][E], m[(J0 + 3) / P][E], x);
        row_t<P, E, J0 + 4, J1>(acc, m, x);
    } else if constexpr (c >= 2) {
        fmac_j2<J0 % P, (J0 + 1) % P>(acc[J0], acc[J0 + 1], m[J0 / P][E], m[(J0 + 1) / P][E], x);
        row_t<P, E, J0 + 2, J1>(acc, m, x);
    } else if constexpr (c == 1) {
        fmac_l1<J0 % P>(acc[J0], m[J0 / P][E], x);
    }
}

// Gauss-Jordan inverse, without pivoting, of the n x n SPD matrix (n <= NC)
// held RS rows per lane in a[][] (rows >= n: identity rows).  At step k every
// other row subtracts a_ik / a_kk times the broadcast pivot row and takes
// -a_ik / a_kk in column k; the pivot row keeps its values and takes 1 in
// column k, and is scaled by 1 / a_kk after the last step.  Returns false if
// a pivot is not positive.
template <int P, int RS, int NC>
__device__ __forceinline__ bool gj_dpp(double (&a)[RS][NC], int p, int n) {
    bool ok = true;
    double sc[RS];
    static_for<0, RS>([&](auto sc_) { sc[decltype(sc_)::value] = 1.0; });
    static_for<0, NC>([&](auto kc) {
        constexpr int k = decltype(kc)::value, Lk = k % P, Sk = k / P;
        if (k < n) {
            const double piv = bcast<Lk>(a[Sk][k]);
            if (!(piv > 0.0)) ok = false;
            const double inv = 1.0 / piv;
            double ng[RS];
            static_for<0, RS>([&](auto s_) {
                constexpr int s = decltype(s_)::value;
                if constexpr (s == Sk) {
                    const bool me = p == Lk;  // this lane holds the pivot row
                    ng[s] = me ? 0.0 : -a[s][k] * inv;
                    sc[s] = me ? inv : sc[s];
                } else {
                    ng[s] = -a[s][k] * inv;
                }
            });
            // the other slots first, then the pivot's slot (whose pivot row stays as it is)
            static_for<0, RS>([&](auto s_) {
                constexpr int s = decltype(s_)::value;
                if constexpr (s != Sk) {
                    row_l<Lk, 0, k>(a[s], a[Sk], ng[s]);
                    row_l<Lk, k + 1, NC>(a[s], a[Sk], ng[s]);
                }
            });
            row_l<Lk, 0, k>(a[Sk], a[Sk], ng[Sk]);
            row_l<Lk, k + 1, NC>(a[Sk], a[Sk], ng[Sk]);
            static_for<0, RS>([&](auto s_) {
                constexpr int s = decltype(s_)::value;
                if constexpr (s == Sk)
                    a[s][k] = p == Lk ? 1.0 : ng[s];
                else
                    a[s][k] = ng[s];
            });
        }
    });
    static_for<0, RS>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        static_for<0, NC>([&](auto jc) { a[s][decltype(jc)::value] *= sc[s]; });
    });
    return ok;
}

// W = C^-1 for the Cholesky factor C of the SPD matrix held R rows per lane
// in a[][] (A = C C^T), in place: forward elimination of [A | I] without
// pivoting, rows below the pivot subtracting f = a_ij / u_jj times the
// broadcast pivot row and taking -f in column j, leaves E = L^-1 on the left
// and U's pivots u_ii on the diagonal; W = diag(u)^-1/2 E.  Returns false if a
// pivot is not positive.
template <int P, int R, int NX>
__device__ __forceinline__ bool lower_inverse_dpp(double (&a)[R][NX], int p) {
    bool ok = true;
    static_for<0, NX>([&](auto jc) {
        constexpr int j = decltype(jc)::value, Lj = j % P, Sj = j / P;
        const double piv = bcast<Lj>(a[Sj][j]);
        if (!(piv > 0.0)) ok = false;
        const double inv = 1.0 / piv;
        double ng[R];
        bool below[R];
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            below[s] = p + s * P > j;
            ng[s] = below[s] ? -a[s][j] * inv : 0.0;
        });
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            if constexpr (s != Sj) {
                row_l<Lj, 0, j>(a[s], a[Sj], ng[s]);
                row_l<Lj, j + 1, NX>(a[s], a[Sj], ng[s]);
            }
        });
        row_l<Lj, 0, j>(a[Sj], a[Sj], ng[Sj]);
        row_l<Lj, j + 1, NX>(a[Sj], a[Sj], ng[Sj]);
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            if (below[s]) a[s][j] = ng[s];
        });
    });
    static_for<0, R>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        const int i = p + s * P;
        double u = 1.0;
        static_for<0, NX>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if (j == i) u = a[s][j];
        });
        const double sc = 1.0 / sqrt(u);
        static_for<0, NX>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            a[s][j] = j < i ? a[s][j] * sc : (j == i ? sc : 0.0);
        });
    });
    return ok;
}

// per-lane place: knot slot g in the workgroup, lane p of the knot
template <int NX>
struct Dl {
    int g, p, knot;
    bool act;  // lane p < P of a knot < N
    __device__ int row(int s) const { return p + s * RowGeo<NX>::P; }
    __device__ bool has(int s) const { return act && row(s) < NX; }
};

template <int NX>
__device__ __forceinline__ Dl<NX> dl_of(int k0, int N) {
    Dl<NX> d;
    d.g = threadIdx.x >> 4;
    d.p = threadIdx.x & 15;
    d.knot = k0 + d.g;
    d.act = d.p < RowGeo<NX>::P && d.knot < N;
    return d;
}

// Global memory is only touched by these wave-wide copies of contiguous
// ranges (consecutive lanes, consecutive elements); lanes read and write
// their matrix rows in LDS.  A lane that loads or stores its own rows in
// global memory touches a separate cache line per lane and instruction, and
// the memory pipeline, not the arithmetic, then bounds the assembly.
// The lane index, opaque to the compiler: a copy's element addresses are
// formed where the copy runs instead of once for all copies (and held in
// registers through every phase between them).
__device__ __forceinline__ int lane_here() {
    int l = threadIdx.x;
    asm volatile("" : "+v"(l));
    return l;
}

// Into LDS: n <= MAXN contiguous elements, every load of the range in flight
// before the first write (source indices clamped to the range, so no load is
// masked; lanes past the range write their copy to a spare slot).  The
// copy's loads are issued where it is called, so only one staged range
// occupies registers at a time.
template <int MAXN, typename TD, typename TS>
__device__ __forceinline__ void stage_in(TD *dst, const TS *__restrict__ src, int n, TD *spare) {
    constexpr int B = (MAXN + kThreadsD - 1) / kThreadsD;
    asm volatile("" ::: "memory");  // the loads of this copy stay here (not hoisted into earlier phases)
    const int ln = lane_here();
    TS v[B];
    static_for<0, B>([&](auto ic) { v[decltype(ic)::value] = src[min(decltype(ic)::value * kThreadsD + ln, n - 1)]; });
    static_for<0, B>([&](auto ic) {
        const int e = decltype(ic)::value * kThreadsD + ln;
        *(e < n ? dst + e : spare) = (TD)v[decltype(ic)::value];
    });
}

// Out of LDS: n <= MAXN contiguous elements, eight per lane at a time; only a
// partial last chunk tests each element.
template <int MAXN, typename TD, typename TS>
__device__ __forceinline__ void copy_out(TD *__restrict__ dst, const TS *src, int n) {
    constexpr int B = 8, CH = B * kThreadsD;
    const int ln = lane_here();
    static_for<0, (MAXN + CH - 1) / CH>([&](auto cc) {
        constexpr int base = decltype(cc)::value * CH;
        if (base + CH <= n) {
            static_for<0, B>([&](auto ic) {
                const int e = base + decltype(ic)::value * kThreadsD + ln;
                dst[e] = (TD)src[e];
            });
        } else if (base < n) {
            static_for<0, B>([&](auto ic) {
                const int e = base + decltype(ic)::value * kThreadsD + ln;
                if (e < n) dst[e] = (TD)src[e];
            });
        }
    });
}

// rows p + s P of an LDS block of nrows x ld doubles into slots (rows clamped
// to the block)
template <int NX, int RS, int NC>
__device__ __forceinline__ void lds_rows(const double *blk, int ld, int nrows, int p, double (&a)[RS][NC]) {
    static_for<0, RS>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        const int r = min(p + s * RowGeo<NX>::P, nrows - 1);
        static_for<0, NC>([&](auto jc) { a[s][decltype(jc)::value] = blk[r * ld + decltype(jc)::value]; });
    });
}

// rows p + s P of a row-major NX x NX block in global memory into slots
// (rows clamped), converted to FP64
template <typename TM, int NX>
__device__ __forceinline__ void load_slots_t(const TM *__restrict__ src, int p, double (&a)[RowGeo<NX>::R][NX]) {
    static_for<0, RowGeo<NX>::R>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        const int r = min(p + s * RowGeo<NX>::P, NX - 1);
        static_for<0, NX>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            a[s][j] = (double)src[r * NX + j];
        });
    });
}

// rows that are not this lane's real rows become identity rows.  The row
// index is made opaque to the compiler, so each call forms its own identity
// values: shared between calls, they were held (and spilled) across the
// whole assembly, and reloaded one dependent scratch load at a time.
template <int NX, int RS, int NC>
__device__ __forceinline__ void identity_outside(double (&a)[RS][NC], int p, bool live, int n) {
    static_for<0, RS>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        int r = p + s * RowGeo<NX>::P;
        asm volatile("" : "+v"(r));
        const bool real = live && r < n;
        static_for<0, NC>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            a[s][j] = real ? a[s][j] : (j == r ? 1.0 : 0.0);
        });
    });
}

// this lane's real rows (r < n) into an LDS block of n x n elements
template <int NX, typename T, int RS, int NC>
__device__ __forceinline__ void rows_to_lds(T *blk, int n, bool live, int p, const double (&a)[RS][NC], double scale) {
    static_for<0, RS>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        const int r = p + s * RowGeo<NX>::P;
        if (live && r < n)
            static_for<0, NC>([&](auto jc) { blk[r * n + decltype(jc)::value] = (T)(scale * a[s][decltype(jc)::value]); });
    });
}

// The same with the FP32 remainder v - (TM)v into a second block.
template <int NX, typename TM>
__device__ __forceinline__ void split_rows_to_lds(TM *hi, float *lo, bool live, int p,
                                                  const double (&a)[RowGeo<NX>::R][NX], double scale) {
    static_for<0, RowGeo<NX>::R>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        const int r = p + s * RowGeo<NX>::P;
        if (live && r < NX)
            static_for<0, NX>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const double v = scale * a[s][j];
                const TM h = (TM)v;
                hi[r * NX + j] = h;
                if (lo) lo[r * NX + j] = (float)(v - (double)h);
            });
    });
}

// upper triangle (j >= r) of this lane's rows into packed LDS blocks
template <int NX, typename TM>
__device__ __forceinline__ void split_packed_to_lds(TM *hi, float *lo, bool live, int p,
                                                    const double (&a)[RowGeo<NX>::R][NX]) {
    static_for<0, RowGeo<NX>::R>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        const int r = p + s * RowGeo<NX>::P;
        if (live && r < NX) {
            const int base = packed_row(r, NX);
            static_for<0, NX>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                if (j >= r) {
                    const double v = a[s][j];
                    const TM h = (TM)v;
                    hi[base + j] = h;
                    if (lo) lo[base + j] = (float)(v - (double)h);
                }
            });
        }
    });
}

// this lane's real rows (scale applied) into a row-major NX x NX block in
// global memory, with the FP32 remainder under FP32 storage
template <typename TM, int NX>
__device__ __forceinline__ void store_split_slots(TM *__restrict__ hi, float *__restrict__ lo, const Dl<NX> &d,
                                                  const double (&a)[RowGeo<NX>::R][NX], double scale) {
    static_for<0, RowGeo<NX>::R>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        const int r = d.row(s);
        if (d.has(s))
            static_for<0, NX>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const double v = scale * a[s][j];
                const TM h = (TM)v;
                hi[r * NX + j] = h;
                if (lo) lo[r * NX + j] = (float)(v - (double)h);
            });
    });
}

// Copy the upper triangle of the matrix held in a[][] onto its lower triangle
// through the knot's LDS buffer (P rows of NX doubles), one slot at a time:
// upper entries are never changed, so every copy reads original values.
template <int NX>
__device__ __forceinline__ void lower_from_upper(double (&a)[RowGeo<NX>::R][NX], int p, double *buf) {
    constexpr int R = RowGeo<NX>::R, P = RowGeo<NX>::P;
    static_for<0, R>([&](auto t_) {
        constexpr int t = decltype(t_)::value;  // source slot: rows q + t P
        wave_sync();
        if (p < P) static_for<0, NX>([&](auto jc) { buf[p * NX + decltype(jc)::value] = a[t][decltype(jc)::value]; });
        wave_sync();
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            const int i = min(p + s * P, NX - 1);
            static_for<0, P>([&](auto qc) {
                constexpr int j = decltype(qc)::value + t * P;  // row j of the source slot
                if constexpr (j < NX) {
                    const double v = buf[decltype(qc)::value * NX + i];  // entry (j, i)
                    if (j < i) a[s][j] = v;
                }
            });
        });
    });
    wave_sync();
}

}  // namespace

// One knot's blocks of S and of the scaled basis from the inputs A, B, Q, R:
// D_k, L_k (storage type, FP32 remainder under FP32 storage) and then W_k
// (SCALED: the scaled basis) or D_k^-1 (nu = NX / 2).  One wave, knots
// k0 .. k0 + 3; at least two waves per SIMD (the compiler keeps the kernel
// within 256 registers).
//
// The inverses Q_{k-1}^-1, R_{k-1}^-1 and Q_k^-1 are formed in registers
// from the staged inputs, so every Q_k is inverted twice (by the rows of
// knots k and k + 1).  That is a fifth more FP64 work than reading a stored
// Q^-1, R^-1 back, and saves their store and both reads, which bound the
// assembly in HBM.  With keep_qr set the knot's Q_k^-1 and R_{k-1}^-1 are
// also stored (the KKT step reads them); items cover disjoint knot ranges,
// so each block is stored once.
template <typename TM, int NX, bool SCALED>
__global__ __launch_bounds__(kThreadsD) __attribute__((amdgpu_waves_per_eu(2))) void k_bdpp_asm(BuildArgs a,
                                                                                              const int2 *items) {
    constexpr int R = RowGeo<NX>::R, P = RowGeo<NX>::P, NN = NX * NX, NU = NX / 2, UU = NU * NU, XU = NX * NU;
    constexpr int RU = (NU + P - 1) / P, PK = NX * (NX + 1) / 2;
    __shared__ __align__(16) double sm[kKnotsD * NN + 2];
    double *spare = sm + kKnotsD * NN;  // sink of staged copies past their range
    const BuildRec it = a.brec[blockIdx.x];  // the item items[blockIdx.x] with its problem's offsets
    const int pr = it.pr, N = it.N, k0 = it.k0, nk = min(kKnotsD, N - k0);
    const int64_t oblk = sizeof(TM) == 4 ? it.oblk32 : it.oblk64, ob3 = sizeof(TM) == 4 ? it.ob3_32 : it.ob3_64;
    const Dl<NX> d = dl_of<NX>(k0, N);
    const int k = d.knot, kc = min(k, N - 1), km = max(kc - 1, 0);
    const bool prev = d.act && k > 0;
    const bool keep = a.keep_qr != 0;
    // blocks k-1 of the knots k0 .. k0+nk-1 (knot 0 reads block 0 with a zero multiplier)
    const int ks = max(k0 - 1, 0), ke = max(k0 + nk - 1, ks + 1), gm = km - ks, gc = kc - k0;
    const int bs = block_stride(NX, sizeof(TM)), bp = packed_stride(NX, sizeof(TM)), kst = 2 * bp + bs;
    TM *b3 = (TM *)a.B3 + ob3 + (int64_t)k0 * kst;  // per knot: D_k (packed), L_k, D_k^-1 (packed)
    int rw[R];
    static_for<0, R>([&](auto s_) { rw[decltype(s_)::value] = min(d.row(decltype(s_)::value), NX - 1); });

    // m = Q_{k-1}^-1 (identity where the knot has no predecessor)
    double m[R][NX], t[R][NX];
    stage_in<kKnotsD * NN>(sm, a.Q + it.onn + (int64_t)ks * NN, (ke - ks) * NN, spare);
    wave_sync();
    lds_rows<NX>(sm + gm * NN, NX, NX, d.p, m);
    identity_outside<NX>(m, d.p, prev, NX);
    (void)gj_dpp<P, R, NX>(m, d.p, NX);  // Q_{k-1} is checked by the row of knot k-1
    wave_sync();
    // t = A_{k-1} Q_{k-1}^-1 (rows of Q^-1 broadcast)
    stage_in<kKnotsD * NN>(sm, a.A + it.onn + (int64_t)ks * NN, (ke - ks) * NN, spare);
    wave_sync();
    int ro[R];  // this lane's rows in the staged block
    static_for<0, R>([&](auto s_) { ro[decltype(s_)::value] = gm * NN + rw[decltype(s_)::value] * NX; });
    static_for<0, R>([&](auto s_) { static_for<0, NX>([&](auto jc) { t[decltype(s_)::value][decltype(jc)::value] = 0.0; }); });
    lds_steps<NX>(sm, ro, prev, [&](auto lc, const double (&x)[R]) {
        constexpr int l = decltype(lc)::value;
        static_for<0, R>([&](auto s_) { row_l<l % P, 0, NX>(t[decltype(s_)::value], m[l / P], x[decltype(s_)::value]); });
    }, [&](auto s_) { return t[decltype(s_)::value][NX - 1]; });
    // D_k = A t^T (rows of t broadcast), + B u^T, + Q_k^-1 below
    double dk[R][NX];
    static_for<0, R>([&](auto s_) { static_for<0, NX>([&](auto jc) { dk[decltype(s_)::value][decltype(jc)::value] = 0.0; }); });
    lds_steps<NX>(sm, ro, prev, [&](auto lc, const double (&x)[R]) {
        constexpr int l = decltype(lc)::value;
        static_for<0, R>([&](auto s_) { row_t<P, l, 0, NX>(dk[decltype(s_)::value], t, x[decltype(s_)::value]); });
    }, [&](auto s_) { return dk[decltype(s_)::value][NX - 1]; });
    // L_k = -t
    {
        wave_sync();
        TM *hi = (TM *)sm;
        float *lo = sizeof(TM) == 4 && a.SLlo ? (float *)(hi + kKnotsD * NN) : nullptr;
        split_rows_to_lds<NX, TM>(hi + d.g * NN, lo ? lo + d.g * NN : nullptr, d.act, d.p, t, -1.0);
        wave_sync();
        for (int g = 0; g < nk; ++g) {
            copy_out<NN>(b3 + (int64_t)g * kst + bp, hi + g * NN, NN);
            if (lo) copy_out<NN>(a.SLlo + oblk + (int64_t)(k0 + g) * bs, lo + g * NN, NN);
        }
        wave_sync();
    }
    bool ok = true;
    // D_k += B u^T with u = B_{k-1} R_{k-1}^-1
    {
        double *Rb = sm, *Bb = sm + kKnotsD * UU;
        stage_in<kKnotsD * UU>(Rb, a.R + it.ouu + (int64_t)ks * UU, (ke - ks) * UU, spare);
        stage_in<kKnotsD * XU>(Bb, a.B + it.onu + (int64_t)ks * XU, (ke - ks) * XU, spare);
        wave_sync();
        double ri[RU][NU], u[R][NU];
        lds_rows<NX>(Rb + gm * UU, NU, NU, d.p, ri);
        // R_{N-1} has no inverse in the method; knots without a predecessor
        // (zero multiplier) take the identity
        identity_outside<NX>(ri, d.p, prev, NU);
        const bool okr = settle(gj_dpp<P, RU, NU>(ri, d.p, NU));
        if (prev) ok = okr;
        if (keep) {  // R_{k-1}^-1 of the knots k0-1 .. k0+nk-2 (from 0)
            wave_sync();
            rows_to_lds<NX>(Rb + gm * UU, NU, prev, d.p, ri, 1.0);
            wave_sync();
            const int nr = k0 + nk - 1 - ks;
            if (nr > 0) copy_out<kKnotsD * UU>(a.Rinv + it.ouu + (int64_t)ks * UU, Rb, nr * UU);
        }
        static_for<0, R>([&](auto s_) { static_for<0, NU>([&](auto jc) { u[decltype(s_)::value][decltype(jc)::value] = 0.0; }); });
        int rb[R];
        static_for<0, R>([&](auto s_) { rb[decltype(s_)::value] = gm * XU + rw[decltype(s_)::value] * NU; });
        lds_steps<NU>(Bb, rb, prev, [&](auto lc, const double (&x)[R]) {
            constexpr int l = decltype(lc)::value;
            static_for<0, R>([&](auto s_) { row_l<l % P, 0, NU>(u[decltype(s_)::value], ri[l / P], x[decltype(s_)::value]); });
        }, [&](auto s_) { return u[decltype(s_)::value][NU - 1]; });
        lds_steps<NU>(Bb, rb, prev, [&](auto lc, const double (&x)[R]) {
            constexpr int l = decltype(lc)::value;
            static_for<0, R>([&](auto s_) { row_t<P, l, 0, NX>(dk[decltype(s_)::value], u, x[decltype(s_)::value]); });
        }, [&](auto s_) { return dk[decltype(s_)::value][NX - 1]; });
        wave_sync();
    }
    // D_k += Q_k^-1
    {
        stage_in<kKnotsD * NN>(sm, a.Q + it.onn + (int64_t)k0 * NN, nk * NN, spare);
        wave_sync();
        double q[R][NX];
        lds_rows<NX>(sm + gc * NN, NX, NX, d.p, q);
        identity_outside<NX>(q, d.p, d.act, NX);
        // D_k's rows wait in the knot's LDS block while Q_k is inverted (both
        // in registers at once would not fit)
        double *park = sm + d.g * NN;
        wave_sync();
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            if (d.p < P) static_for<0, NX>([&](auto jc) { park[rw[s] * NX + decltype(jc)::value] = dk[s][decltype(jc)::value]; });
        });
        ok = settle(gj_dpp<P, R, NX>(q, d.p, NX)) && ok;
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            static_for<0, NX>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                dk[s][j] = park[rw[s] * NX + j] + q[s][j];
            });
        });
        if (keep) {  // Q_k^-1 of the knots k0 .. k0+nk-1
            wave_sync();
            rows_to_lds<NX>(sm + d.g * NN, NX, d.act, d.p, q, 1.0);
            wave_sync();
            copy_out<kKnotsD * NN>(a.Qinv + it.onn + (int64_t)k0 * NN, sm, nk * NN);
        }
    }
    lower_from_upper<NX>(dk, d.p, sm + d.g * P * NX);
    // D_k (packed upper triangle)
    {
        TM *hi = (TM *)sm;
        float *lo = sizeof(TM) == 4 && a.SDlo ? (float *)(hi + kKnotsD * PK) : nullptr;
        split_packed_to_lds<NX, TM>(hi + d.g * PK, lo ? lo + d.g * PK : nullptr, d.act, d.p, dk);
        wave_sync();
        for (int g = 0; g < nk; ++g) {
            copy_out<PK>(b3 + (int64_t)g * kst, hi + g * PK, PK);
            if (lo) copy_out<PK>(a.SDlo + it.opk + (int64_t)(k0 + g) * bp, lo + g * PK, PK);
        }
        wave_sync();
    }
    bool okd;
    if constexpr (SCALED) {
        // scaled basis: W_k = C_k^-1, stored full (zeros above the diagonal)
        okd = lower_inverse_dpp<P, R, NX>(dk, d.p);
        TM *w = (TM *)sm;
        split_rows_to_lds<NX, TM>(w + d.g * NN, nullptr, d.act, d.p, dk, 1.0);
        wave_sync();
        for (int g = 0; g < nk; ++g) copy_out<NN>((TM *)a.Zs + oblk + (int64_t)(k0 + g) * bs, w + g * NN, NN);
    } else {
        okd = gj_dpp<P, R, NX>(dk, d.p, NX);
        TM *di = (TM *)sm;
        split_packed_to_lds<NX, TM>(di + d.g * PK, nullptr, d.act, d.p, dk);
        wave_sync();
        for (int g = 0; g < nk; ++g) copy_out<PK>(b3 + (int64_t)g * kst + bp + bs, di + g * PK, PK);
    }
    if (d.act && !(ok && okd)) atomicOr(a.status + pr, kNotSpd);
}

// Oh_k = W_k L_k W_{k-1}^T (k >= 1, Oh_0 = 0) in FP64 from the stored W and
// L_k (storage type): X = L_k W_{k-1}^T with the rows of W_{k-1} broadcast,
// then W_k X with the rows of X broadcast.  Each lane reads its own rows from
// global memory: few loads per knot, all issued at the start, which here
// beats staging the blocks through LDS.
template <typename TM, int NX>
__global__ __launch_bounds__(kThreadsD) void k_bdpp_ohat(BuildArgs a, const int2 *items) {
    constexpr int R = RowGeo<NX>::R, P = RowGeo<NX>::P;
    const BuildRec it = a.brec[blockIdx.x];  // the item items[blockIdx.x] with its problem's offsets
    const int N = it.N;
    const int64_t oblk = sizeof(TM) == 4 ? it.oblk32 : it.oblk64, ob3 = sizeof(TM) == 4 ? it.ob3_32 : it.ob3_64;
    const Dl<NX> d = dl_of<NX>(it.k0, N);
    const int k = d.knot, kc = min(k, N - 1), km = max(kc - 1, 0);
    const bool prev = d.act && k > 0;
    const int bs = block_stride(NX, sizeof(TM)), bp = packed_stride(NX, sizeof(TM));
    const TM *Z = (const TM *)a.Zs + oblk;
    const TM *Lk = (const TM *)a.B3 + ob3 + (int64_t)kc * (2 * bp + bs) + bp;
    int rw[R];
    static_for<0, R>([&](auto s_) { rw[decltype(s_)::value] = min(d.row(decltype(s_)::value), NX - 1); });
    double w[R][NX], x[R][NX];
    load_slots_t<TM, NX>(Z + (int64_t)km * bs, d.p, w);
    static_for<0, R>([&](auto s_) { static_for<0, NX>([&](auto jc) { x[decltype(s_)::value][decltype(jc)::value] = 0.0; }); });
    static_for<0, NX>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            const double lv = (double)Lk[rw[s] * NX + l], v = prev ? lv : 0.0;
            row_t<P, l, 0, NX>(x[s], w, v);
        });
    });
    const TM *Wk = Z + (int64_t)kc * bs;
    double o[R][NX];
    static_for<0, R>([&](auto s_) { static_for<0, NX>([&](auto jc) { o[decltype(s_)::value][decltype(jc)::value] = 0.0; }); });
    static_for<0, NX>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        static_for<0, R>([&](auto s_) {
            constexpr int s = decltype(s_)::value;
            const double v = (double)Wk[rw[s] * NX + l];
            row_l<l % P, 0, NX>(o[s], x[l / P], v);
        });
    });
    keep(o);
    store_split_slots<TM, NX>((TM *)a.OH + oblk + (int64_t)kc * bs, (float *)nullptr, d, o, 1.0);
}

template <int NX>
hipError_t launch_dpp_class(const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    const bool sc = a.Zs != nullptr;
    const dim3 g(nitems), t(kThreadsD);
    if (fp32 && sc)
        hipLaunchKernelGGL((k_bdpp_asm<float, NX, true>), g, t, 0, s, a, items);
    else if (fp32)
        hipLaunchKernelGGL((k_bdpp_asm<float, NX, false>), g, t, 0, s, a, items);
    else if (sc)
        hipLaunchKernelGGL((k_bdpp_asm<double, NX, true>), g, t, 0, s, a, items);
    else
        hipLaunchKernelGGL((k_bdpp_asm<double, NX, false>), g, t, 0, s, a, items);
    return hipGetLastError();
}

template <int NX>
hipError_t launch_dpp_ohat(const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL((k_bdpp_ohat<float, NX>), dim3(nitems), dim3(kThreadsD), 0, s, a, items);
    else
        hipLaunchKernelGGL((k_bdpp_ohat<double, NX>), dim3(nitems), dim3(kThreadsD), 0, s, a, items);
    return hipGetLastError();
}

int dpp_knots_per_item() { return kKnotsD; }

template hipError_t launch_dpp_class<6>(const BuildArgs &, const int2 *, int, bool, hipStream_t);
template hipError_t launch_dpp_class<14>(const BuildArgs &, const int2 *, int, bool, hipStream_t);
template hipError_t launch_dpp_class<26>(const BuildArgs &, const int2 *, int, bool, hipStream_t);
template hipError_t launch_dpp_ohat<6>(const BuildArgs &, const int2 *, int, bool, hipStream_t);
template hipError_t launch_dpp_ohat<14>(const BuildArgs &, const int2 *, int, bool, hipStream_t);
template hipError_t launch_dpp_ohat<26>(const BuildArgs &, const int2 *, int, bool, hipStream_t);

}  // namespace ssp
