// Batched PCG in the block-Jacobi congruence basis, one persistent grid.
//
// With D_k = C_k C_k^T (Cholesky) and W_k = C_k^-1, the congruence
// W S W^T = I + Oh (W = blockdiag(W_k)) has identity diagonal blocks and the
// off-diagonal blocks Oh_k = W_k L_k W_{k-1}^T (below) and Oh_k^T (above),
// with O = S - D and W O W^T = Oh; D^-1 = W^T W.  The preconditioners of the
// paper become polynomials in Oh:
//   block-Jacobi (Eq. (jacobi)):          D^-1                 = W^T W,
//   symmetric stair (Sec. IV):            D^-1 - D^-1 O D^-1   = W^T (I - Oh) W,
//   additive stair (Sec. III):            D^-1 - D^-1 O D^-1/2 = W^T (I - Oh/2) W,
//   Neumann polynomial of degree m (Eq. (polynomial_precon), Psi = D,
//   P = D - S = -O):  sum_{i<=m} (D^-1 P)^i D^-1 = W^T (sum_{i<=m} (-Oh)^i) W
// (the stair identities are those of Eq. (stair_inv) with S = Psi_l + Psi_r - D).
// PCG on S lambda = gamma with Phi^-1 = W^T q(Oh) W is therefore PCG on
// (I + Oh) lh = W gamma with the preconditioner q(Oh) and lambda = W^T lh:
// the same iterates in exact arithmetic, with residuals rh = W r.  Each PCG
// pass streams Oh_k only (nx^2 elements per knot instead of D_k, L_k and
// D_k^-1), and the float operator I + Oh is as well conditioned as
// block-Jacobi-preconditioned S, whatever the conditioning of the D_k.
//
// The refinement loop stays in the original basis: each outer step forms the
// true residual r = gamma - S lambda in FP64 from D, L (hi + lo), maps it to
// rh = W r, runs the float PCG on (I + Oh) d = rh / ||rh|| (stopping on the
// recurrence residual in the scaled basis) and adds ||rh|| W^T d to lambda in
// FP64.  FP64 storage runs the same loop in FP64 (further outer steps restart
// the FP64 iteration from the true residual).
//
// Per pass the single-reduction recurrences of the fused kernel are used:
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s,
//   u = q(Oh) r, w = (I + Oh) u, gamma = r.u, delta = w.u, rho = r.r,
// with u by Horner, h_0 = r, h_j = r - c Oh h_{j-1} (j = 1..m), u = h_m.  The
// pass walks the knots in steps of C: step c updates the lead knots [k0, k1)
// and writes r into window 0, computes h_j j knots behind the lead (Oh couples
// neighbours) and w m + 1 knots behind; the last step drains the tail.  The
// Oh blocks of a step arrive in registers (16-byte loads issued one step
// ahead) and are stored into an LDS ring.
//
// Scheduling: one launch for the whole ragged batch.  Workgroups take
// problems from a device queue ordered by decreasing work N nx^2, so the long
// problems start first and the short ones fill in at the end; each problem
// runs the code compiled for its state size.
#include <math.h>

#include "ssp_device.h"
#include "ssp_fused.h"
#include "ssp_host.h"
#include "ssp_sweep.h"

namespace ssp {

namespace {

template <typename TM>
constexpr int vlen() { return 16 / (int)sizeof(TM); }
template <typename TM, int NX>
constexpr int bstride() { return (NX * NX + vlen<TM>() - 1) / vlen<TM>() * vlen<TM>(); }
template <typename TM, int NX>
constexpr int vstride() { return (NX + vlen<TM>() - 1) / vlen<TM>() * vlen<TM>(); }
template <int BLOCK, int NX>
constexpr int max_step() { return (BLOCK / 64) * (64 / NX); }

// 16-byte prefetch registers per thread: one step of the largest step the
// wave mapping allows (capped; the LDS budget may shorten the step further)
template <typename TM, int BLOCK, int NX>
constexpr int pf3_slots() {
    constexpr int n = (max_step<BLOCK, NX>() * bstride<TM, NX>() / vlen<TM>() + BLOCK - 1) / BLOCK;
    constexpr int cap = sizeof(TM) == 4 ? 12 : 8;
    return n < cap ? n : cap;
}

// Knots per step for an LDS budget: the Oh ring and m + 1 vector windows
// (r, h_1 .. h_{m-1}, u) of R = C + m + 2 slots each, plus a 16-byte spot.
template <typename TM, int BLOCK, int NX>
__host__ __device__ inline int knots3(int lds_bytes, int m) {
    int C = max_step<BLOCK, NX>();
    const int Cp = pf3_slots<TM, BLOCK, NX>() * BLOCK * vlen<TM>() / bstride<TM, NX>();
    if (Cp < C) C = Cp;
    const int per = (bstride<TM, NX>() + (m + 1) * vstride<TM, NX>()) * (int)sizeof(TM);
    const int Cl = (lds_bytes - 16) / per - (m + 2);
    if (Cl < C) C = Cl;
    return C;
}

template <typename TM, int BLOCK, int NX>
__host__ __device__ inline int lds3_for(int C, int m) {
    return (C + m + 2) * (bstride<TM, NX>() + (m + 1) * vstride<TM, NX>()) * (int)sizeof(TM) + 16;
}

// The six recurrence vectors of a problem of N knots stay in the
// workgroup's LDS, behind the pass's ring, windows and spare spot, when
// they fit in the budget: the passes then stream only the Oh blocks from
// HBM.  Returns their byte offset in the dynamic LDS, or -1 if they do not
// fit.  Compiled for the small state sizes only (at nx 26 a budget that
// keeps three workgroups per CU holds no horizon of the workloads).
template <typename TM, int BLOCK, int NX>
__host__ __device__ inline int vectors3_offset(int N, int lds_bytes, int m) {
    if constexpr (NX > 14) {
        return -1;
    } else {
        const int C = knots3<TM, BLOCK, NX>(lds_bytes, m);
        if (C < 1) return -1;
        const int off = (lds3_for<TM, BLOCK, NX>(C, m) + 15) & ~15;
        return (int64_t)off + 6 * (int64_t)N * NX * (int64_t)sizeof(TM) <= lds_bytes ? off : -1;
    }
}

// Knots per step of residual_lean for an LDS budget: C + 1 knot slots of D
// (packed) and L in FP64 and a lambda window of C + 2 knots.
template <typename TM, int NX>
__host__ __device__ inline int residual3_knots(int lds_bytes) {
    constexpr int V = vlen<TM>();
    constexpr int SS = (NX * (NX + 1) / 2 + V - 1) / V * V + bstride<TM, NX>(), NXP = (NX + 1) & ~1;
    int C = (lds_bytes / 8 - NXP) / (SS + NXP) - 1;
    return C < 64 ? C : 64;
}

template <typename TI>
struct Vecs3 {
    TI *u, *w, *p, *s, *x, *r;
};

// Per-lane partial inner products of one pass: in the storage type, or (the
// FP64-accumulation option) the same storage-type products summed in FP64.
template <typename TI>
struct Dots3 {
    TI gam, del, rho;
    double g64 = 0.0, d64 = 0.0, r64 = 0.0;
};

// Register prefetch of one step: the step's Oh blocks (one contiguous chunk,
// 16-byte loads, surplus slots re-read the first vector so that every load is
// unconditional) and the six recurrence vectors of this thread's lead row
// (the init pass: the FP64 right-hand side of that row instead).
template <typename TM, int BLOCK, int NX>
struct Prefetch3 {
    using VT = typename Vec16<TM>::T;
    static constexpr int V = Vec16<TM>::V;
    static constexpr int BS = bstride<TM, NX>();
    static constexpr int kPF = pf3_slots<TM, BLOCK, NX>();
    VT reg[kPF];
    TM vec[6];
    double res = 0;

    __device__ __forceinline__ void issue(const TM *OH, int k0, int kc, bool init, int lead_row, const double *rhs,
                                          const Vecs3<TM> vs) {
        const int nvec = kc * BS / V;
        const VT *src = (const VT *)(OH + (int64_t)k0 * BS);
        static_for<0, kPF>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            int q = threadIdx.x + m * BLOCK;
            if (q >= nvec) q = 0;
            reg[m] = src[q];
        });
        const int row = lead_row >= 0 ? lead_row : 0;
        if (init) {
            res = rhs[row];
        } else {
            vec[0] = vs.u[row];
            vec[1] = vs.w[row];
            vec[2] = vs.p[row];
            vec[3] = vs.s[row];
            vec[4] = vs.x[row];
            vec[5] = vs.r[row];
        }
    }

    // chunk -> ring slots sb, sb + 1, ... (mod R); surplus vectors (a
    // partial slot, or whole slots of a short step) go to the 16-byte spot
    // `dummy`.  Every register is stored on every path, so the next issue
    // finds no load still pending on them and need not wait for memory.
    __device__ __forceinline__ void store(TM *ring, int kc, int sb, int R, TM *dummy) const {
        const int nvec = kc * BS / V;
        const int wrap = R * BS, base = sb * BS;
        static_for<0, kPF>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int q = threadIdx.x + m * BLOCK;
            int off = base + q * V;
            if (off >= wrap) off -= wrap;
            *(VT *)(q < nvec ? ring + off : dummy) = reg[m];
        });
    }
};

// Workgroup sums of a pass's partial inner products (fixed-order trees; in
// FP64 under the FP64-accumulation option, then rounded to the storage type).
template <typename TI, int BLOCK>
__device__ __forceinline__ Dots3<TI> reduce_dots(Dots3<TI> dt, bool acc64, double *red64, TI *redT) {
    if (acc64) {
        block_sum2<BLOCK>(dt.g64, dt.d64, red64);
        dt.r64 = block_sum<BLOCK>(dt.r64, red64 + 2 * (BLOCK / kWave));
        return Dots3<TI>{uniform((TI)dt.g64), uniform((TI)dt.d64), uniform((TI)dt.r64)};
    }
    block_sum2<BLOCK>(dt.gam, dt.del, redT);
    dt.rho = block_sum<BLOCK>(dt.rho, redT + 2 * (BLOCK / kWave));
    return Dots3<TI>{uniform(dt.gam), uniform(dt.del), uniform(dt.rho)};
}

struct Geo3 {
    int N, C, R, m;  // knots, knots per step, ring slots, Horner steps
    bool acc64;      // accumulate the inner products in FP64
};

// One pass over the knots (see the file comment).  init: the pass that starts
// an inner solve (r = rhs * inv_s, x = 0); first: the first update pass
// (p = u, s = w).
template <typename TI, int BLOCK, int NX>
__device__ __forceinline__ Dots3<TI> scaled_pass(const Geo3 &g, bool init, bool first, TI alpha, TI beta, TI cc,
                                                 double inv_s, const double *__restrict__ rhs,
                                                 const TI *__restrict__ OH, const Vecs3<TI> v, TI *smem) {
    constexpr int W = BLOCK / 64, KW = 64 / NX, BS = bstride<TI, NX>(), NXP = vstride<TI, NX>();
    const int N = g.N, C = g.C, R = g.R, m = g.m;
    TI *ring = smem;             // R slots of BS
    TI *win = ring + R * BS;     // window j (R slots of NXP) at win + j R NXP: 0 = r, m = u
    TI *dummy = win + (m + 1) * R * NXP;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kloc = lane / NX, i = lane - kloc * NX;
    const bool lane_ok = kloc < KW;
    const int kme = wv * KW + kloc, group = W * KW;
    Dots3<TI> d{TI(0), TI(0), TI(0)};

    Prefetch3<TI, BLOCK, NX> pf;
    const int nsteps = (N + C - 1) / C;
    auto lead_row = [&](int k0, int kc) { return (lane_ok && kme < kc) ? (k0 + kme) * NX + i : -1; };
    pf.issue(OH, 0, min(C, N), init, lead_row(0, min(C, N)), rhs, v);
    int sb = 0;  // ring slot of knot k0
    for (int c = 0; c < nsteps; ++c) {
        const int k0 = c * C, kc = min(C, N - k0), k1 = k0 + kc;
        const bool last = k1 == N;
        __syncthreads();  // every reader of the slots refilled below is done
        pf.store(ring, kc, sb, R, dummy);
        TI cur[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) cur[e] = pf.vec[e];
        const double res = pf.res;
        if (!last) pf.issue(OH, k1, min(C, N - k1), init, lead_row(k1, min(C, N - k1)), rhs, v);

        // A: recurrence updates on the lead rows, r into window 0
        if (lane_ok && kme < kc) {
            const int row = (k0 + kme) * NX + i;
            TI r;
            if (init) {
                r = (TI)(res * inv_s);
                v.x[row] = TI(0);
            } else {
                const TI pv = first ? cur[0] : cur[0] + beta * cur[2];
                const TI sv = first ? cur[1] : cur[1] + beta * cur[3];
                v.p[row] = pv;
                v.s[row] = sv;
                v.x[row] = cur[4] + alpha * pv;
                r = cur[5] - alpha * sv;
            }
            v.r[row] = r;
            win[slot_of(sb, kme, R) * NXP + i] = r;
            const TI rr = r * r;
            if (g.acc64)
                d.r64 += (double)rr;
            else
                d.rho += rr;
            if (m == 0) {  // block-Jacobi: u = r
                v.u[row] = r;
                if (g.acc64)
                    d.g64 += (double)rr;
                else
                    d.gam += rr;
            }
        }
        __syncthreads();  // ring blocks and window 0 come from every wave

        // H_j: h_j = r - c Oh h_{j-1}, j knots behind the lead
        for (int j = 1; j <= m; ++j) {
            const TI *hin = win + (j - 1) * R * NXP;
            TI *hout = win + j * R * NXP;
            const int lo = max(k0 - j, 0), hi = last ? N : k1 - j;
            for (int kk = kme; kk < hi - lo; kk += group) {
                if (!lane_ok) break;
                const int k = lo + kk, dk = k - k0;
                const int s = slot_of(sb, dk, R);
                TI t = TI(0);
                if (k > 0) t += lean_dot<NX, false>(ring + s * BS, i, hin + slot_of(sb, dk - 1, R) * NXP);
                if (k + 1 < N) {
                    const int sp = slot_of(sb, dk + 1, R);
                    t += lean_dot<NX, true>(ring + sp * BS, i, hin + sp * NXP);
                }
                const TI rk = win[s * NXP + i];
                const TI h = rk - cc * t;
                hout[s * NXP + i] = h;
                if (j == m) {
                    if (g.acc64)
                        d.g64 += (double)(rk * h);
                    else
                        d.gam += rk * h;
                    v.u[k * NX + i] = h;
                }
            }
            __syncthreads();
        }

        // W: w = u + Oh u, m + 1 knots behind the lead
        {
            const TI *u = win + m * R * NXP;
            const int lo = max(k0 - m - 1, 0), hi = last ? N : k1 - m - 1;
            for (int kk = kme; kk < hi - lo; kk += group) {
                if (!lane_ok) break;
                const int k = lo + kk, dk = k - k0;
                const int s = slot_of(sb, dk, R);
                const TI uk = u[s * NXP + i];
                TI w = uk;
                if (k > 0) w += lean_dot<NX, false>(ring + s * BS, i, u + slot_of(sb, dk - 1, R) * NXP);
                if (k + 1 < N) {
                    const int sp = slot_of(sb, dk + 1, R);
                    w += lean_dot<NX, true>(ring + sp * BS, i, u + sp * NXP);
                }
                if (g.acc64)
                    d.d64 += (double)(w * uk);
                else
                    d.del += w * uk;
                v.w[k * NX + i] = w;
            }
        }
        sb += C;
        if (sb >= R) sb -= R;
    }
    return d;
}

// r = gamma - S lambda in FP64 with S read as D (packed) and L in the
// storage type plus their FP32 remainders (or FP64), in steps of C knots:
// the step's D, L (and L of the next knot) are converted to FP64 into LDS
// with 16-byte loads, lambda of knots k0 - 1 .. k1 into a window, then r is
// formed for knots [k0, k1).  No loads cross a step, so the pass needs few
// registers (it runs once per outer step).  Returns this thread's parts of
// ||r||^2 and ||gamma||^2, summed over the same rows in the same order.
template <typename TM, int BLOCK, int NX>
__device__ __forceinline__ ResNorms residual_lean(int N, int C, const TM *__restrict__ B3,
                                                  const float *__restrict__ Dlo, const float *__restrict__ Llo,
                                                  const double *__restrict__ lam, const double *__restrict__ gam,
                                                  double *__restrict__ r64, double *smem) {
    constexpr int V = vlen<TM>(), KW = 64 / NX, W = BLOCK / 64, NXP = (NX + 1) & ~1;
    constexpr int BS = bstride<TM, NX>(), BP = (NX * (NX + 1) / 2 + V - 1) / V * V, KS = 2 * BP + BS;
    constexpr int SS = BP + BS;  // FP64 slot: D packed, then L
    constexpr bool LO = sizeof(TM) == 4;
    double *ring = smem, *win = smem + (C + 1) * SS;  // C + 1 knot slots, C + 2 window slots
    const int lane = threadIdx.x & 63, kloc = lane / NX, i = lane - kloc * NX;
    const bool lane_ok = kloc < KW;
    const int kme = (threadIdx.x >> 6) * KW + kloc, group = W * KW;
    double rr = 0.0, gg = 0.0;
    __syncthreads();  // lambda rows were just written by other threads
    for (int k0 = 0; k0 < N; k0 += C) {
        const int k1 = min(k0 + C, N), kl = min(k1 + 1, N);  // blocks of knots [k0, kl)
        const int nv = (kl - k0) * (SS / V);
        for (int q = threadIdx.x; q < nv; q += BLOCK) {
            const int kk = q / (SS / V), e = (q - kk * (SS / V)) * V;
            const int64_t k = k0 + kk;
            const TM *src = B3 + k * KS + e;  // D packed then L: the first SS elements of the knot
            double *dst = ring + kk * SS + e;
            if constexpr (LO) {
                const f32x4 h = *(const f32x4 *)src;
                const f32x4 l = *(const f32x4 *)(e < BP ? Dlo + k * BP + e : Llo + k * BS + (e - BP));
                dst[0] = (double)h.x + (double)l.x;
                dst[1] = (double)h.y + (double)l.y;
                dst[2] = (double)h.z + (double)l.z;
                dst[3] = (double)h.w + (double)l.w;
            } else {
                const f64x2 h = *(const f64x2 *)src;
                dst[0] = h.x;
                dst[1] = h.y;
            }
        }
        const int lo = max(k0 - 1, 0), nl = (kl - lo) * NX;
        for (int q = threadIdx.x; q < nl; q += BLOCK) {
            const int kk = q / NX, j = q - kk * NX;
            win[kk * NXP + j] = lam[(int64_t)lo * NX + q];
        }
        __syncthreads();
        for (int kk = kme; kk < k1 - k0; kk += group) {
            if (!lane_ok) break;
            const int k = k0 + kk, wk = k - lo;  // window slot of knot k
            const double *Dk = ring + kk * SS;
            double y = lean_sym_dot<NX>(Dk, i, win + wk * NXP);
            if (k > 0) y += lean_dot<NX, false>(Dk + BP, i, win + (wk - 1) * NXP);
            if (k + 1 < N) y += lean_dot<NX, true>(ring + (kk + 1) * SS + BP, i, win + (wk + 1) * NXP);
            const double gv = gam[(int64_t)k * NX + i];
            const double r = gv - y;
            r64[(int64_t)k * NX + i] = r;
            rr += r * r;
            gg += gv * gv;
        }
        __syncthreads();
    }
    return ResNorms{rr, gg};
}

// rh = W r on every knot (W_k stored full, zero above the diagonal);
// returns this thread's part of ||rh||^2.
template <typename TM, int BLOCK, int NX>
__device__ __forceinline__ double zt_apply(int N, const TM *__restrict__ Z, const double *__restrict__ r,
                                           double *__restrict__ rh) {
    constexpr int KW = 64 / NX, BS = bstride<TM, NX>(), group = (BLOCK / 64) * KW;
    const int lane = threadIdx.x & 63, kloc = lane / NX, i = lane - kloc * NX;
    const int kme = (threadIdx.x >> 6) * KW + kloc;
    double acc = 0.0;
    __syncthreads();  // r rows come from other threads
    if (kloc < KW) {
        for (int k = kme; k < N; k += group) {
            const TM *zk = Z + (int64_t)k * BS;
            const double *rk = r + (int64_t)k * NX;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
            for (int l = 0; l < NX; l += 2) {
                s0 += (double)zk[i * NX + l] * rk[l];
                s1 += (double)zk[i * NX + l + 1] * rk[l + 1];
            }
            const double s = s0 + s1;
            rh[(int64_t)k * NX + i] = s;
            acc += s * s;
        }
    }
    return acc;
}

// lam += scale * W^T x on every knot.
template <typename TM, typename TI, int BLOCK, int NX>
__device__ __forceinline__ void z_apply_add(int N, const TM *__restrict__ Z, const TI *__restrict__ x, double scale,
                                            double *__restrict__ lam) {
    constexpr int KW = 64 / NX, BS = bstride<TM, NX>(), group = (BLOCK / 64) * KW;
    const int lane = threadIdx.x & 63, kloc = lane / NX, i = lane - kloc * NX;
    const int kme = (threadIdx.x >> 6) * KW + kloc;
    __syncthreads();  // x rows come from other threads
    if (kloc < KW) {
        for (int k = kme; k < N; k += group) {
            const TM *zk = Z + (int64_t)k * BS + i;
            const TI *xk = x + (int64_t)k * NX;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
            for (int l = 0; l < NX; l += 2) {
                s0 += (double)zk[l * NX] * (double)xk[l];
                s1 += (double)zk[(l + 1) * NX] * (double)xk[l + 1];
            }
            lam[(int64_t)k * NX + i] += scale * (s0 + s1);
        }
    }
    __syncthreads();  // lambda rows are read by other threads next
}

template <typename TI>
struct Prob3 {
    int N, max_iter;
    double gnorm;
    const TI *B3;  // D (packed), L, D^-1 (packed) per knot: the true residual reads D and L
    const float *SDlo, *SLlo;
    const TI *OH, *Z;
    double *lam, *r64, *rh64;
    const double *gam;
    Vecs3<TI> v;
};

struct Outcome3 {
    int st = kOk, total = 0, steps = 0;
    bool fallback = false, pc_fallback = false;
    double rnorm = 0.0;
};

// VL: the recurrence vectors live in LDS (vectors3_offset), a separate
// instantiation so that the compiler sees LDS pointers there and global
// pointers in the other (a pointer that may be either would turn every
// access into a flat one, whose waits also hold the LDS traffic).
template <typename TI, int BLOCK, int NX, bool ACC, bool VL>
__device__ __forceinline__ Outcome3 solve_scaled(const SolveArgs &a, const Prob3<TI> &q, unsigned char *smem_raw,
                                                 double *red64, TI *redT) {
    const int N = q.N, n = N * NX, tid = threadIdx.x;
    Outcome3 o;
    Geo3 g;
    g.N = N;
    g.m = a.poly;
    g.acc64 = ACC;
    g.C = knots3<TI, BLOCK, NX>(a.lds_bytes, g.m);
    g.R = g.C + g.m + 2;
    Vecs3<TI> vv = q.v;
    if constexpr (VL) {
        TI *vb = (TI *)(smem_raw + vectors3_offset<TI, BLOCK, NX>(N, a.lds_bytes, g.m));
        vv = Vecs3<TI>{vb + 1 * n, vb + 2 * n, vb + 3 * n, vb + 4 * n, vb + 5 * n, vb};
    }
    const int Cres = residual3_knots<TI, NX>(a.lds_bytes);
    const TI cc = (TI)a.pc_c;
    int pending = kOk, base = 0;
    int mcur = g.m;  // block-Jacobi (m = 0) after a float breakdown of the polynomial
    bool broke = false;
    double prev = INFINITY, gsame = q.gnorm;
    const double *rsrc = q.r64;
    for (;;) {
        if (o.steps == 0 && a.use_lambda0 == 0) {
            rsrc = q.gam;
            o.rnorm = q.gnorm;
        } else {
            ResNorms nr = residual_lean<TI, BLOCK, NX>(N, Cres, q.B3, q.SDlo, q.SLlo, q.lam, q.gam, q.r64,
                                                       (double *)smem_raw);
            block_sum2<BLOCK>(nr.rr, nr.gg, red64);
            o.rnorm = uniform(sqrt(nr.rr));
            gsame = uniform(sqrt(nr.gg));
            rsrc = q.r64;
        }
        // a warm start is kept only if its residual is strictly below
        // ||gamma||, both norms summed in the same order
        if (o.steps == 0 && a.use_lambda0 == 2 && !(o.rnorm < gsame)) {
            for (int row = tid; row < n; row += BLOCK) q.lam[row] = 0.0;
            o.rnorm = q.gnorm;
            o.fallback = true;
            rsrc = q.gam;
            __syncthreads();
        }
        if (!isfinite(o.rnorm)) {
            o.st = kNonFinite;
            break;
        }
        if (pending != kOk) {
            o.st = pending;
            break;
        }
        if (o.rnorm <= a.tol * q.gnorm) break;
        if (o.steps > 0 && !a.refine) {
            o.st = kInaccurate;
            break;
        }
        if (broke && !(o.rnorm < prev)) {
            o.st = kBreakdown;
            break;
        }
        if (o.steps - base >= a.max_outer) {
            o.st = kMaxIter;
            break;
        }
        prev = o.rnorm;
        double tau = a.theta * a.tol * q.gnorm / o.rnorm;
        if (tau < a.tau_min) tau = a.tau_min;
        if (tau > 1.0) tau = 1.0;

        // the right-hand side in the scaled basis, rh = W r
        double hh = zt_apply<TI, BLOCK, NX>(N, q.Z, rsrc, q.rh64);
        hh = block_sum<BLOCK>(hh, red64);
        const double hn = uniform(sqrt(hh));
        if (!(hn > 0.0) || !isfinite(hn)) {
            o.st = kNonFinite;
            break;
        }
        Geo3 gc = g;
        gc.m = mcur;
        gc.R = g.C + mcur + 2;
        int it = 0, ist = kOk;
        Dots3<TI> dt = scaled_pass<TI, BLOCK, NX>(gc, true, false, TI(0), TI(0), cc, 1.0 / hn, q.rh64, q.OH, vv,
                                                  (TI *)smem_raw);
        dt = reduce_dots<TI, BLOCK>(dt, gc.acc64, red64, redT);
        const TI bnorm = sqrt(dt.rho);
        const TI tauT = (TI)tau;
        TI gam_prev = TI(0), alpha = TI(0), beta = TI(0);
        for (;;) {
            const TI rn = sqrt(dt.rho);
            if (!isfinite(rn)) {
                ist = kNonFinite;
                break;
            }
            if (rn <= tauT * bnorm) break;
            if (o.total + it >= q.max_iter) {
                ist = kMaxIter;
                break;
            }
            TI den;
            if (it == 0) {
                den = dt.del;
                beta = TI(0);
            } else {
                beta = dt.gam / gam_prev;
                den = dt.del - beta * dt.gam / alpha;
            }
            if (!(den > TI(0)) || !(dt.gam > TI(0))) {
                ist = (isfinite(den) && isfinite(dt.gam)) ? kBreakdown : kNonFinite;
                break;
            }
            alpha = dt.gam / den;
            gam_prev = dt.gam;
            dt = scaled_pass<TI, BLOCK, NX>(gc, false, it == 0, alpha, beta, cc, 0.0, q.rh64, q.OH, vv,
                                            (TI *)smem_raw);
            dt = reduce_dots<TI, BLOCK>(dt, gc.acc64, red64, redT);
            ++it;
        }
        o.total += it;
        ++o.steps;
        z_apply_add<TI, TI, BLOCK, NX>(N, q.Z, vv.x, hn, q.lam);
        // under refinement a float breakdown only ends the inner solve; with a
        // polynomial in Oh it also hands the rest of the solve to block-Jacobi
        broke = a.refine && ist == kBreakdown;
        if (broke && mcur != 0) {
            mcur = 0;
            o.pc_fallback = true;
            broke = false;
            base = o.steps;
        }
        if (ist != kOk && !broke && !(a.refine && ist == kBreakdown)) pending = ist;
    }
    return o;
}

template <typename TI, int BLOCK, int NX, bool ACC>
__device__ __forceinline__ void solve_one3(const SolveArgs &a, int p, Prob3<TI> &q, unsigned char *smem_raw,
                                           double *red64, TI *redT) {
    const int tid = threadIdx.x;
    const int N = q.N, n = N * NX;
    const int64_t ob = a.off_blk[p], ov = a.off_v[p];
    q.B3 = (const TI *)a.B3 + a.off_b3[p];
    q.SDlo = a.SDlo ? a.SDlo + a.off_pk[p] : nullptr;
    q.SLlo = a.SLlo ? a.SLlo + ob : nullptr;
    q.OH = (const TI *)a.OH + ob;
    q.Z = (const TI *)a.Z + ob;
    TI *Wk = (TI *)a.work;
    q.v = Vecs3<TI>{Wk + 1 * a.tot_v + ov, Wk + 2 * a.tot_v + ov, Wk + 3 * a.tot_v + ov, Wk + 4 * a.tot_v + ov,
                    Wk + 5 * a.tot_v + ov, Wk + 0 * a.tot_v + ov};

    double gg = 0.0, bad = 0.0;
    for (int row = tid; row < n; row += BLOCK) {
        const double gv = q.gam[row];
        gg += gv * gv;
        if (a.use_lambda0 == 1) {
            if (!isfinite(q.lam[row])) bad = 1.0;
        } else if (a.use_lambda0 == 0) {
            q.lam[row] = 0.0;
        }
    }
    block_sum2<BLOCK>(gg, bad, red64);
    gg = uniform(gg);
    bad = uniform(bad);
    q.gnorm = sqrt(gg);
    Outcome3 o;
    if (!isfinite(q.gnorm) || bad != 0.0) {
        o.st = kNonFinite;
        o.rnorm = NAN;
    } else if (gg == 0.0) {
        for (int row = tid; row < n; row += BLOCK) q.lam[row] = 0.0;
    } else {
        if (vectors3_offset<TI, BLOCK, NX>(N, a.lds_bytes, a.poly) >= 0)
            o = solve_scaled<TI, BLOCK, NX, ACC, NX <= 14>(a, q, smem_raw, red64, redT);
        else
            o = solve_scaled<TI, BLOCK, NX, ACC, false>(a, q, smem_raw, red64, redT);
    }
    if (tid == 0) {
        a.iters[p] = o.total;
        a.outer[p] = o.steps;
        a.relres[p] = gg == 0.0 ? 0.0 : o.rnorm / q.gnorm;
        a.status[p] = o.st | (o.fallback ? kWarmFallback : 0) | (o.pc_fallback ? kPcFallback : 0);
    }
}


// One problem from start to status, for state size NX.  Every path ends at
// the caller's workgroup barrier (no early return: a divergent-looking exit
// next to the queue's single-thread fetch lets the compiler thread it back
// to the loop head without that fetch).
template <typename TI, int BLOCK, int NX, bool ACC>
__device__ __forceinline__ void run_problem3(const SolveArgs &a, int p, int st_in, unsigned char *smem_raw,
                                             double *red64, TI *redT) {
    const int tid = threadIdx.x;
    const int N = a.N[p], n = N * NX;
    const int64_t ob = a.off_blk[p], ov = a.off_v[p];
    Prob3<TI> q;
    q.N = N;
    q.max_iter = a.max_iter > 0 ? a.max_iter : 10 * n;
    q.lam = a.lambda + ov;
    q.gam = a.gamma + ov;
    q.r64 = a.r64 + ov;
    q.rh64 = a.rh64 + ov;
    if (build_failed(st_in)) {
        for (int row = tid; row < n; row += BLOCK) q.lam[row] = 0.0;
        if (tid == 0) {
            a.iters[p] = 0;
            a.outer[p] = 0;
            a.relres[p] = NAN;
        }
    } else {
        solve_one3<TI, BLOCK, NX, ACC>(a, p, q, smem_raw, red64, redT);
    }
}

}  // namespace

// Persistent solve of every problem: workgroups take queue positions from a
// device counter until the queue is empty (every workgroup reaches the exit
// test after each problem).
// The queue position, problem, state size and incoming status are read
// into scalar registers (readfirstlane), so every branch on them is uniform
// for the compiler too: each workgroup barrier is then reached the same
// number of times by every wave.
// One persistent grid for the problems of one compiled state size NX (a
// kernel instance per size keeps each size's register allocation to
// itself).  ACC: sum the inner products in FP64 (the option; FP32 storage
// only).
template <typename TI, int BLOCK, int NX, bool ACC>
__global__ __launch_bounds__(BLOCK, 3) void k_pcg3(SolveArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red64[3 * (BLOCK / kWave)];
    __shared__ TI redT[3 * (BLOCK / kWave)];
    __shared__ int s_next;
    if (threadIdx.x == 0) s_next = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    int qi = __builtin_amdgcn_readfirstlane(s_next);
    while (qi < a.nprob) {
        const int p = __builtin_amdgcn_readfirstlane(a.order[qi]);
        const int nx = __builtin_amdgcn_readfirstlane(a.nx[p]);
        const int st_in = __builtin_amdgcn_readfirstlane(a.status[p]);
        if (nx == NX) {
            run_problem3<TI, BLOCK, NX, ACC>(a, p, st_in, smem_raw, red64, redT);
        } else if (threadIdx.x == 0) {  // the host queues only problems of this size
            a.status[p] = kNonFinite;
            a.relres[p] = NAN;
            a.iters[p] = 0;
            a.outer[p] = 0;
        }
        __syncthreads();  // the problem is done: s_next, the LDS and the reduction scratch are free
        if (threadIdx.x == 0) s_next = (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        qi = __builtin_amdgcn_readfirstlane(s_next);
    }
}

namespace {

template <typename TI>
int knots3_rt(int nx, int threads, int lds_bytes, int m) {
    switch (threads * 100 + nx) {
        case 25606: return knots3<TI, 256, 6>(lds_bytes, m);
        case 25614: return knots3<TI, 256, 14>(lds_bytes, m);
        case 25626: return knots3<TI, 256, 26>(lds_bytes, m);
        case 25636: return knots3<TI, 256, 36>(lds_bytes, m);
        case 12806: return knots3<TI, 128, 6>(lds_bytes, m);
        case 12814: return knots3<TI, 128, 14>(lds_bytes, m);
        case 12826: return knots3<TI, 128, 26>(lds_bytes, m);
        case 12836: return knots3<TI, 128, 36>(lds_bytes, m);
    }
    return 0;
}

template <typename TI>
int lds3_rt(int nx, int threads, int m) {
    int C = knots3_rt<TI>(nx, threads, 1 << 30, m);
    if (C < 1) return 0;
    switch (threads * 100 + nx) {
        case 25606: return lds3_for<TI, 256, 6>(C, m);
        case 25614: return lds3_for<TI, 256, 14>(C, m);
        case 25626: return lds3_for<TI, 256, 26>(C, m);
        case 25636: return lds3_for<TI, 256, 36>(C, m);
        case 12806: return lds3_for<TI, 128, 6>(C, m);
        case 12814: return lds3_for<TI, 128, 14>(C, m);
        case 12826: return lds3_for<TI, 128, 26>(C, m);
        case 12836: return lds3_for<TI, 128, 36>(C, m);
    }
    return 0;
}

template <typename TI, int BLOCK, bool ACC>
const void *pcg3_fn(int nx) {
    switch (nx) {
        case 6: return (const void *)k_pcg3<TI, BLOCK, 6, ACC>;
        case 14: return (const void *)k_pcg3<TI, BLOCK, 14, ACC>;
        case 26: return (const void *)k_pcg3<TI, BLOCK, 26, ACC>;
        case 36: return (const void *)k_pcg3<TI, BLOCK, 36, ACC>;
    }
    return nullptr;
}

const void *pcg3_kernel(bool fp32, int threads, bool acc, int nx) {
    if (fp32 && acc) return threads == 128 ? pcg3_fn<float, 128, true>(nx) : pcg3_fn<float, 256, true>(nx);
    if (fp32) return threads == 128 ? pcg3_fn<float, 128, false>(nx) : pcg3_fn<float, 256, false>(nx);
    return threads == 128 ? pcg3_fn<double, 128, false>(nx) : pcg3_fn<double, 256, false>(nx);
}

hipError_t allow_lds(const void *f) {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, f);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)fa.sharedSizeBytes);
}

}  // namespace

int pcg3_residual_steps(int nx, bool fp32, int lds_bytes) {
    switch (nx) {
        case 6: return fp32 ? residual3_knots<float, 6>(lds_bytes) : residual3_knots<double, 6>(lds_bytes);
        case 14: return fp32 ? residual3_knots<float, 14>(lds_bytes) : residual3_knots<double, 14>(lds_bytes);
        case 26: return fp32 ? residual3_knots<float, 26>(lds_bytes) : residual3_knots<double, 26>(lds_bytes);
        case 36: return fp32 ? residual3_knots<float, 36>(lds_bytes) : residual3_knots<double, 36>(lds_bytes);
    }
    return 0;
}

template <typename TI>
int onchip3_rt(int nx, int threads, int lds_bytes, int m) {
    // the largest N whose vectors vectors3_offset keeps in LDS (0: none)
    int lo = 0;
    for (int N = 1; N <= 4096; ++N) {
        int off = -1;
        switch (threads * 100 + nx) {
            case 25606: off = vectors3_offset<TI, 256, 6>(N, lds_bytes, m); break;
            case 25614: off = vectors3_offset<TI, 256, 14>(N, lds_bytes, m); break;
            case 12806: off = vectors3_offset<TI, 128, 6>(N, lds_bytes, m); break;
            case 12814: off = vectors3_offset<TI, 128, 14>(N, lds_bytes, m); break;
        }
        if (off < 0) break;
        lo = N;
    }
    return lo;
}

int pcg3_onchip_horizon(int nx, bool fp32, int threads, int lds_bytes, int m) {
    return fp32 ? onchip3_rt<float>(nx, threads, lds_bytes, m) : onchip3_rt<double>(nx, threads, lds_bytes, m);
}

int pcg3_steps_for(int nx, bool fp32, int threads, int lds_bytes, int m) {
    return fp32 ? knots3_rt<float>(nx, threads, lds_bytes, m) : knots3_rt<double>(nx, threads, lds_bytes, m);
}

int pcg3_lds(int nx, bool fp32, int threads, int m) {
    int l = fp32 ? lds3_rt<float>(nx, threads, m) : lds3_rt<double>(nx, threads, m);
    if (l == 0) return 0;
    if (l > kFusedLdsCap) {
        // shrink to the cap
        l = kFusedLdsCap;
        if (pcg3_steps_for(nx, fp32, threads, l, m) < 1) return 0;
    }
    return l;
}

int pcg3_occupancy(bool fp32, int threads, int lds_bytes, int *cus, bool acc, int nx) {
    int dev = 0, n = 0;
    if (cus) *cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    const void *f = pcg3_kernel(fp32, threads, acc, nx);
    if (!f) return 0;
    if (allow_lds(f) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, threads, (size_t)lds_bytes) != hipSuccess) return 0;
    if (cus) {
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return 0;
        *cus = pr.multiProcessorCount;
    }
    return n;
}

hipError_t launch_pcg3(const SolveArgs &a, bool fp32, int threads, int nx, int grid, hipStream_t s) {
    if (a.nprob == 0) return hipSuccess;
    if (threads != 128 && threads != 256) return hipErrorInvalidValue;
    const bool acc = fp32 && a.acc64 != 0;
    const void *f = pcg3_kernel(fp32, threads, acc, nx);
    if (!f) return hipErrorInvalidValue;
    // per kernel instance: the LDS opt-in once, and the resident workgroups
    // for an LDS budget queried once per process (no runtime query inside a
    // graph capture after the first eager solve)
    struct Entry {
        const void *f;
        int lds, grid;
    };
    static Entry cache[64];
    static int used = 0, next = 0;
    int hit = -1;
    for (int c = 0; c < used; ++c)
        if (cache[c].f == f && cache[c].lds == a.lds_bytes) hit = c;
    if (hit < 0) {
        hipError_t e = allow_lds(f);
        if (e != hipSuccess) return e;
        int cus = 0;
        const int occ = pcg3_occupancy(fp32, threads, a.lds_bytes, &cus, acc, nx);
        if (occ < 1 || cus < 1) return hipErrorInvalidConfiguration;
        hit = used < 64 ? used++ : (next++ % 64);
        cache[hit] = Entry{f, a.lds_bytes, occ * cus};
    }
    if (grid <= 0) grid = cache[hit].grid;
    if (grid > a.nprob) grid = a.nprob;
    SolveArgs arg = a;
    void *args[] = {(void *)&arg};
    hipError_t e = hipLaunchKernel(f, dim3(grid), dim3(threads), args, (size_t)a.lds_bytes, s);
    return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace ssp
