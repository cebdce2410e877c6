// Device pieces shared by the fused PCG passes: 16-byte vector types, LDS
// ring slots, block-row and block-column dot products against LDS vector
// windows, and the pipelined FP64 true residual r = gamma - S lambda.
#pragma once

#include <math.h>

#include <type_traits>

#include "ssp_device.h"
#include "ssp_sweep.h"

namespace ssp {

namespace {

// Native clang vector types (LLVM first-class vectors, unlike HIP's struct
// float4) so that arrays of them are split into registers.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename TM>
struct Vec16;
template <>
struct Vec16<float> {
    using T = f32x4;
    static constexpr int V = 4;
};
template <>
struct Vec16<double> {
    using T = f64x2;
    static constexpr int V = 2;
};

// slot of knot k0 + d in a ring of R slots whose knot k0 sits at slot sb
// (-R < d < 2R)
__device__ __forceinline__ int slot_of(int sb, int d, int R) {
    int s = sb + d;
    if (s < 0) s += R;
    if (s >= R) s -= R;
    if (s >= R) s -= R;
    return s;
}

// Dot products of a column (stride NX) or a row of an NX x NX LDS block with
// an LDS vector window, for a compile-time NX: 8 terms at a time (x and row
// entries read in aligned pairs), four partial sums.  NX = 0: runtime size,
// plain loops.
constexpr int kChunk = 8;

template <int NX, bool COL, typename T>
__device__ __forceinline__ T block_dot(const T *__restrict__ blk, int i, const T *__restrict__ x, int nrt) {
    if constexpr (NX > 0) {
        static_assert(NX % 2 == 0, "compiled state sizes are even");
        using P2 = typename std::conditional<sizeof(T) == 4, f32x2, f64x2>::type;
        T s[4] = {T(0), T(0), T(0), T(0)};
        constexpr int CH = sizeof(T) == 4 ? kChunk : kChunk / 2;  // FP64: half the registers per chunk
        static_for<0, (NX + CH - 1) / CH>([&](auto cc) {
            constexpr int j0 = decltype(cc)::value * CH;
            constexpr int jn = NX - j0 < CH ? NX - j0 : CH;
            T xr[jn], ar[jn];
            static_for<0, jn / 2>([&](auto hc) {
                constexpr int j = 2 * decltype(hc)::value;
                const P2 v = *(const P2 *)(x + j0 + j);
                xr[j] = v.x;
                xr[j + 1] = v.y;
                if constexpr (!COL) {
                    const P2 w = *(const P2 *)(blk + i * NX + j0 + j);
                    ar[j] = w.x;
                    ar[j + 1] = w.y;
                }
            });
            if constexpr (COL) {
                static_for<0, jn>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    ar[j] = blk[(j0 + j) * NX + i];
                });
            }
            static_for<0, jn>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                s[(j0 + j) % 4] += ar[j] * xr[j];
            });
        });
        return (s[0] + s[1]) + (s[2] + s[3]);
    } else {
        T s0 = T(0), s1 = T(0);
        int j = 0;
        for (; j + 2 <= nrt; j += 2) {
            if (COL) {
                s0 += blk[j * nrt + i] * x[j];
                s1 += blk[(j + 1) * nrt + i] * x[j + 1];
            } else {
                s0 += blk[i * nrt + j] * x[j];
                s1 += blk[i * nrt + j + 1] * x[j + 1];
            }
        }
        if (j < nrt) s0 += (COL ? blk[j * nrt + i] : blk[i * nrt + j]) * x[j];
        return s0 + s1;
    }
}

// Column i of an nx x nx LDS block (row-major) times x.
template <int NX, typename T>
__device__ __forceinline__ T col_dot(const T *__restrict__ blk, int i, const T *__restrict__ x, int nrt) {
    return block_dot<NX, true>(blk, i, x, nrt);
}

// Row i of an nx x nx LDS block times x.
template <int NX, typename T>
__device__ __forceinline__ T row_dot(const T *__restrict__ blk, int i, const T *__restrict__ x, int nrt) {
    return block_dot<NX, false>(blk, i, x, nrt);
}

// Row i (= column i) of a symmetric block stored packed in LDS (upper
// triangle by rows) times x: entry (j, i) sits at packed_row(j) + i for
// j <= i and at packed_row(i) + j above.  Chunks of 8 terms, four partial
// sums, as in block_dot.
template <int NX, typename T>
__device__ __forceinline__ T sym_dot(const T *__restrict__ P, int i, const T *__restrict__ x, int nrt) {
    if constexpr (NX > 0) {
        using P2 = typename std::conditional<sizeof(T) == 4, f32x2, f64x2>::type;
        constexpr int CH = sizeof(T) == 4 ? kChunk : kChunk / 2;
        const int ri = packed_row(i, NX);
        T s[4] = {T(0), T(0), T(0), T(0)};
        static_for<0, (NX + CH - 1) / CH>([&](auto cc) {
            constexpr int j0 = decltype(cc)::value * CH;
            constexpr int jn = NX - j0 < CH ? NX - j0 : CH;
            T xr[jn], ar[jn];
            static_for<0, jn / 2>([&](auto hc) {
                constexpr int j = 2 * decltype(hc)::value;
                const P2 v = *(const P2 *)(x + j0 + j);
                xr[j] = v.x;
                xr[j + 1] = v.y;
            });
            static_for<0, jn>([&](auto jc) {
                constexpr int j = j0 + decltype(jc)::value;
                ar[decltype(jc)::value] = P[j <= i ? packed_row(j, NX) + i : ri + j];
            });
            static_for<0, jn>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                s[(j0 + j) % 4] += ar[j] * xr[j];
            });
        });
        return (s[0] + s[1]) + (s[2] + s[3]);
    } else {
        T s0 = T(0), s1 = T(0);
        int j = 0;
        for (; j + 2 <= nrt; j += 2) {
            s0 += P[packed_index(i, j, nrt)] * x[j];
            s1 += P[packed_index(i, j + 1, nrt)] * x[j + 1];
        }
        if (j < nrt) s0 += P[packed_index(i, j, nrt)] * x[j];
        return s0 + s1;
    }
}

// Lean forms of the dot products for passes that must stay within few
// registers: a loop over pairs of terms (x and row entries read as aligned
// pairs), partially unrolled, so that the loads in flight are bounded by the
// unroll factor instead of the whole row.  NX even.
template <int NX, bool COL, typename T>
__device__ __forceinline__ T lean_dot(const T *__restrict__ blk, int i, const T *__restrict__ x) {
    static_assert(NX % 2 == 0, "compiled state sizes are even");
    using P2 = typename std::conditional<sizeof(T) == 4, f32x2, f64x2>::type;
    T s0 = T(0), s1 = T(0);
#pragma unroll 4
    for (int j = 0; j < NX; j += 2) {
        const P2 v = *(const P2 *)(x + j);
        T a0, a1;
        if constexpr (COL) {
            a0 = blk[j * NX + i];
            a1 = blk[(j + 1) * NX + i];
        } else {
            const P2 w = *(const P2 *)(blk + i * NX + j);
            a0 = w.x;
            a1 = w.y;
        }
        s0 += a0 * v.x;
        s1 += a1 * v.y;
    }
    return s0 + s1;
}

// Row i of a packed symmetric block (upper triangle by rows) times x, lean:
// entries (j, i) for j < i down the column part, then row i from the diagonal.
template <int NX, typename T>
__device__ __forceinline__ T lean_sym_dot(const T *__restrict__ P, int i, const T *__restrict__ x) {
    T s0 = T(0), s1 = T(0);
    int pj = i;  // packed index of (0, i), then (j, i) = packed_row(j) + i
#pragma unroll 2
    for (int j = 0; j < i; ++j) {
        s0 += P[pj] * x[j];
        pj += NX - 1 - j;
    }
    const int ri = packed_row(i, NX);
#pragma unroll 2
    for (int j = i; j < NX; ++j) s1 += P[ri + j] * x[j];
    return s0 + s1;
}

}  // namespace

// 16-byte prefetch registers of the residual pass per array (FP32 storage
// loads hi and lo vectors, FP64 storage hi only)
template <typename TM>
constexpr int residual_slots() { return sizeof(TM) == 4 ? 8 : 16; }

// Knots per step of the pipelined FP64 residual pass for a compiled state
// size (< 1: it cannot run and the staged sweep is used).  LDS: a ring of
// C + 1 knots of D (packed) and L in FP64 and a lambda window of C + 2 knots.
template <typename TM>
__host__ __device__ inline int residual_knots_per_step(int nx, int block, int lds_bytes) {
    const int V = 16 / (int)sizeof(TM);
    const int per = packed_stride(nx, sizeof(TM)) + block_stride(nx, sizeof(TM));  // D and L of a knot
    const int nxp = (nx + 1) & ~1;
    int C = (block / 64) * (64 / nx);
    const int Cp = (residual_slots<TM>() * block * V) / per;
    if (Cp < C) C = Cp;
    const int Cl = (lds_bytes / 8 - nxp) / (per + nxp) - 1;
    if (Cl < C) C = Cl;
    return C;
}

// This thread's parts of ||r||^2 and ||gamma||^2 from one residual pass,
// both summed over the same rows in the same order, so that a start whose
// residual is exactly gamma (lambda = 0) gives two equal norms.
struct ResNorms {
    double rr, gg;
};

// r = gamma - S lambda in FP64 with S read as hi + lo (FP32 storage) or
// FP64, pipelined like the fused pass: the next step's D and L blocks are
// prefetched into registers while the current step computes, then stored
// into an LDS ring as FP64.  Step c stores knots [k0, k1) and forms r one
// knot behind (r_k needs L_{k+1}).  Writes r64, returns this thread's parts
// of ||r||^2 and ||gamma||^2.  The same wave mapping as the fused pass
// (lane -> knot, row).
template <typename TM, int BLOCK, int NX>
__device__ __forceinline__ ResNorms residual_pass(int N, int C, const TM *__restrict__ B3,
                                                const float *__restrict__ Dlo, const float *__restrict__ Llo,
                                                const double *__restrict__ lam, const double *__restrict__ gam,
                                                double *__restrict__ r64, double *smem) {
    using VT = typename Vec16<TM>::T;
    constexpr int V = Vec16<TM>::V;
    constexpr int KP = residual_slots<TM>();
    constexpr bool LO = sizeof(TM) == 4;
    constexpr int W = BLOCK / 64, KW = 64 / NX, NXP = (NX + 1) & ~1;
    constexpr int BS = (NX * NX + V - 1) / V * V;                // full block stride of the storage
    constexpr int BP = (NX * (NX + 1) / 2 + V - 1) / V * V;      // packed block stride
    constexpr int KS = 2 * BP + BS;                              // knot stride: D, L, D^-1
    constexpr int VPK = (BP + BS) / V;                           // 16-byte vectors of D and L per knot
    const int R = C + 1, RL = C + 2, ss = BP + BS;
    double *ring = smem, *win = smem + R * ss;  // slot: D (packed, BP doubles), then L
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kloc = lane / NX, i = lane - kloc * NX;
    const bool lane_ok = kloc < KW;
    const int kme = wv * KW + kloc, group = W * KW;
    VT hi[KP];
    f32x4 lo[LO ? KP : 1];
    double lamv = 0.0;

    auto issue = [&](int k0, int kc) {
        const int nvec = kc * VPK;
        static_for<0, KP>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            int q = threadIdx.x + m * BLOCK;
            if (q >= nvec) q = 0;  // surplus slots re-read the first vector
            const int kk = q / VPK, e = (q - kk * VPK) * V;
            const int64_t k = k0 + kk;
            hi[m] = *(const VT *)(B3 + k * KS + e);
            if constexpr (LO) {
                const float *src = e < BP ? Dlo + k * BP + e : Llo + k * BS + (e - BP);
                lo[m] = *(const f32x4 *)src;
            }
        });
        const bool lead = lane_ok && kme < kc;
        lamv = lam[lead ? (int64_t)(k0 + kme) * NX + i : 0];
    };
    auto store = [&](int kc, int sb) {
        const int nvec = kc * VPK;
        static_for<0, KP>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int q = threadIdx.x + m * BLOCK;
            if (q < nvec) {
                const int kk = q / VPK, e = (q - kk * VPK) * V;
                int s = sb + kk;
                if (s >= R) s -= R;
                double *dst = ring + s * ss + e;
                if constexpr (LO) {
                    const f32x4 h = hi[m], l = lo[m];
                    f64x2 a, b;
                    a.x = (double)h.x + (double)l.x;
                    a.y = (double)h.y + (double)l.y;
                    b.x = (double)h.z + (double)l.z;
                    b.y = (double)h.w + (double)l.w;
                    *(f64x2 *)dst = a;
                    *(f64x2 *)(dst + 2) = b;
                } else {
                    *(f64x2 *)dst = hi[m];
                }
            }
        });
    };

    double rr = 0.0, gg = 0.0;
    const int nsteps = (N + C - 1) / C;
    __syncthreads();  // lambda rows were just updated by other threads
    issue(0, min(C, N));
    int sb = 0, sw = 0;  // ring slot and window slot of knot k0
    for (int c = 0; c < nsteps; ++c) {
        const int k0 = c * C, kc = min(C, N - k0), k1 = k0 + kc;
        const bool last = k1 == N;
        __syncthreads();  // every reader of the slots refilled below is done
        store(kc, sb);
        if (lane_ok && kme < kc) win[slot_of(sw, kme, RL) * NXP + i] = lamv;
        if (!last) issue(k1, min(C, N - k1));
        __syncthreads();
        const int klo = max(k0 - 1, 0), khi = last ? N : k1 - 1;
        for (int kk = kme; kk < khi - klo; kk += group) {
            if (!lane_ok) break;
            const int k = klo + kk, dk = k - k0;
            const double *Dk = ring + slot_of(sb, dk, R) * ss;
            double y = lean_sym_dot<NX>(Dk, i, win + slot_of(sw, dk, RL) * NXP);  // D_k (packed)
            if (k > 0) y += lean_dot<NX, false>(Dk + BP, i, win + slot_of(sw, dk - 1, RL) * NXP);
            if (k + 1 < N)
                y += lean_dot<NX, true>(ring + slot_of(sb, dk + 1, R) * ss + BP, i, win + slot_of(sw, dk + 1, RL) * NXP);
            const double gv = gam[(int64_t)k * NX + i];
            const double r = gv - y;
            r64[(int64_t)k * NX + i] = r;
            rr += r * r;
            gg += gv * gv;
        }
        sb += C;
        if (sb >= R) sb -= R;
        sw += C;
        if (sw >= RL) sw -= RL;
    }
    return ResNorms{rr, gg};
}

}  // namespace ssp
