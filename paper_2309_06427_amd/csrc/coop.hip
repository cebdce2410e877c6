// Cooperative solve of one long problem: its knots are spread over the whole
// grid, W knots per workgroup (one wavefront per knot, lane i on row i), so a
// horizon of N knots runs on N / W workgroups at once instead of one.  The
// method is the fused kernel's (Sec. II-B PCG with Phi^-1 = D^-1 - c D^-1 O
// D^-1, the single-reduction recurrences, FP64 iterative refinement with the
// block-Jacobi fallback); what changes is how the knots talk to each other.
//
// One grid-wide synchronisation per PCG iteration.  An iteration needs, at
// knot k, y = D^-1 r at k-2 .. k+2 (for t = O y at k-1 .. k+1, for
// u = y - c D^-1 t there, for w = S u at k) and then the three dot products.
// So every workgroup also carries two ghost knots on each side (their L_k and
// D_k^-1 in LDS) and keeps r and the search direction s = S p of the ghosts
// itself, with the same recurrences, in the same order, as their owners:
// their values are bit-identical to the owners'.  The only remote input of an
// iteration is w at the ghosts, which the owners publish together with their
// partial sums before the one synchronisation.  The refinement's FP64
// residual (a few times per solve) exchanges lambda and r64 the same way.
//
// Synchronisation.  Every value that crosses workgroups is written and read
// with agent-scope atomics, which are coherent across the chiplets' L2s
// without cache maintenance.  The per-iteration exchange needs no separate
// barrier: each 64-bit word carries 32 bits of payload and a 32-bit tag, the
// running count of grid sums (continued across launches from a counter kept
// in device memory, so a tag never repeats and nothing has to be cleared), so
// a reader knows a word is current when its tag matches.  A workgroup
// publishes its w rows and then its partial sums; wave 0 of every workgroup
// polls all partial-sum records, the ghost waves poll their w rows.  Records
// and w rows alternate between two buffers by sum parity, so a fast
// workgroup cannot overwrite a value before every reader has it.  The FP64
// residual of the refinement (a few times per solve) also needs lambda of
// the neighbours first: a plain grid barrier (arrival words) does that.
// Every wait is bounded: a workgroup that waits too long raises an error
// flag that ends every other wait, so the grid always drains.  The launch is
// cooperative (the whole grid resident or the launch fails).
#include <math.h>

#include "ssp_device.h"
#include "ssp_host.h"
#include "ssp_sweep.h"

namespace ssp {

namespace {

constexpr int kGh = 2;                // ghost knots on each side
constexpr int kMaxW = 4;              // own knots per workgroup at most
constexpr int kMaxSlots = kMaxW + 2 * kGh;
constexpr int kCoopThreads = 64 * kMaxSlots;
constexpr unsigned kSpin = 1u << 22;  // polls before a wait gives up
// flags[kTagBase]: tag counter kept across launches; flags[kErr]: error flag;
// flags[kFlag0 + g]: arrivals of workgroup g at the plain barrier
constexpr int kTagBase = 0, kErr = 63, kFlag0 = 64;

typedef unsigned long long u64;

struct CoopArgs {
    SolveArgs s;
    unsigned *flags;  // kFlag0 + G words; [kErr, kFlag0 + G) zero at launch
    u64 *rec;         // partial-sum records: 2 parities x G x 6 words
    u64 *wtag;        // tagged w rows: 2 parities x n x (sizeof(TI) / 4) words
    int G, W;         // workgroups, own knots per workgroup
};

template <typename T>
__device__ __forceinline__ void put(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T get(T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// tagged values: one word per float, two per double (low, high halves)
__device__ __forceinline__ void put_tagged(u64 *p, float v, unsigned tag) {
    put(p, ((u64)tag << 32) | __float_as_uint(v));
}
__device__ __forceinline__ void put_tagged(u64 *p, double v, unsigned tag) {
    const u64 b = (u64)__double_as_longlong(v);
    put(p, ((u64)tag << 32) | (b & 0xffffffffull));
    put(p + 1, ((u64)tag << 32) | (b >> 32));
}
__device__ __forceinline__ bool get_tagged(u64 *p, float &v, unsigned tag) {
    const u64 a = get(p);
    v = __uint_as_float((unsigned)a);
    return (unsigned)(a >> 32) == tag;
}
__device__ __forceinline__ bool get_tagged(u64 *p, double &v, unsigned tag) {
    const u64 a = get(p), b = get(p + 1);
    v = __longlong_as_double((long long)((b << 32) | (a & 0xffffffffull)));
    return (unsigned)(a >> 32) == tag && (unsigned)(b >> 32) == tag;
}

// spin accounting of a wave's bounded wait; false once it has to give up
__device__ __forceinline__ bool keep_waiting(unsigned *flags, unsigned spins) {
    if (spins > kSpin || ((spins & 63) == 63 && __any(get(flags + kErr) != 0u))) {
        if ((threadIdx.x & 63) == 0) put(flags + kErr, 1u);
        return false;
    }
    return true;
}

// Plain grid barrier (every thread of every workgroup calls it): arrival
// words counted up to `gen`.  Returns false once any workgroup has given up.
__device__ __forceinline__ bool grid_sync(unsigned *flags, int G, unsigned &gen, int *s_ok) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this thread's stores are visible
    __syncthreads();
    ++gen;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        if (lane == 0) put(flags + kFlag0 + blockIdx.x, gen);
        int ok = 1;
        for (unsigned spins = 0;; ++spins) {
            bool here = true;
            for (int h = lane; h < G; h += 64) here = here && (int)(get(flags + kFlag0 + h) - gen) >= 0;
            if (__all(here)) break;
            if (!keep_waiting(flags, spins)) {
                ok = 0;
                break;
            }
        }
        if (lane == 0) *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

template <typename T>
__device__ __forceinline__ T dot_row(const T *M, int i, const T *x, int nx) {  // row i of a full block
    T s = T(0);
#pragma unroll 4
    for (int j = 0; j < nx; ++j) s += M[i * nx + j] * x[j];
    return s;
}
template <typename T>
__device__ __forceinline__ T dot_col(const T *M, int i, const T *x, int nx) {  // column i of a full block
    T s = T(0);
#pragma unroll 4
    for (int j = 0; j < nx; ++j) s += M[j * nx + i] * x[j];
    return s;
}
template <typename T>
__device__ __forceinline__ T dot_sym(const T *P, int i, const T *x, int nx) {  // row i of a packed symmetric block
    T s = T(0);
#pragma unroll 4
    for (int j = 0; j < nx; ++j) s += P[packed_index(i, j, nx)] * x[j];
    return s;
}

// 16-byte vector of T (LDS windows are 16-byte aligned and padded to it)
template <typename T>
struct V16;
template <>
struct V16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};
template <>
struct V16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};

// sum_j m[j] x[j] for a row m held in registers and a vector x in LDS
template <int NX, typename T>
__device__ __forceinline__ T dot_reg(const T (&m)[NX], const T *x) {
    using VT = typename V16<T>::type;
    constexpr int V = V16<T>::n;
    T s = T(0);
#pragma unroll
    for (int j0 = 0; j0 < NX; j0 += V) {
        const VT v = *(const VT *)(x + j0);
#pragma unroll
        for (int q = 0; q < V; ++q)
            if (j0 + q < NX) s += m[j0 + q] * v[q];
    }
    return s;
}

// LDS elements of the block area: ghost slots hold [L_k, D_k^-1 packed],
// own slots the whole knot run [D_k packed, L_k, D_k^-1 packed].
__host__ __device__ inline int coop_block_elems(int W, int bs, int bp) {
    return 2 * kGh * (bs + bp) + W * (2 * bp + bs);
}

}  // namespace

// NX > 0: the state size is NX, known at compile time; with REG the lane's
// rows of D_k^-1, D_k, L_k and L_{k+1}^T also sit in registers.
template <typename TI, int NX>
__global__ __launch_bounds__(kCoopThreads) void k_coop(CoopArgs ca) {
    using TM = TI;
    constexpr bool REG = NX > 0 && 4 * NX * (int)sizeof(TI) <= 640;  // at most 160 VGPRs of rows
    constexpr int RN = REG ? NX : 1;
    const SolveArgs &a = ca.s;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[3 * kMaxSlots];
    __shared__ double sums[2][3];
    __shared__ int s_ok, s_sum_ok[2];
    const int p = a.order[0];
    const int N = a.N[p], nx = NX > 0 ? NX : a.nx[p], n = N * nx;
    const int G = ca.G, W = ca.W, S = W + 2 * kGh, g = blockIdx.x;
    const int sl = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane;
    const int k0 = g * W, k = k0 - kGh + sl;
    const bool is_own = sl >= kGh && sl < kGh + W;
    const bool row = k >= 0 && k < N && lane < nx;  // this lane holds a row of a knot
    const bool own = row && is_own;
    const bool inner = sl >= 1 && sl <= W + 2;      // t and u are formed at own knots +- 1
    const int bs = block_stride(nx, sizeof(TM)), bp = packed_stride(nx, sizeof(TM)), ks = 2 * bp + bs,
              gks = bs + bp;
    const int nxp = (nx + 3) & ~3;
    const int64_t ov = a.off_v[p];
    const TM *B3 = (const TM *)a.B3 + a.off_b3[p];
    const float *SDlo = a.SDlo ? a.SDlo + a.off_pk[p] : nullptr;
    const float *SLlo = a.SLlo ? a.SLlo + a.off_blk[p] : nullptr;
    double *lam = a.lambda + ov;
    const double *gam = a.gamma + ov;
    double *r64g = a.r64 + ov;   // FP64 residual rows (published by their owners)
    constexpr int TW = sizeof(TI) / 4;  // tagged words per value
    unsigned gen = 0;                   // plain barriers passed
    const unsigned tag0 = get(ca.flags + kTagBase);  // tags of this launch: tag0 + 1, tag0 + 2, ...
    unsigned nsum = 0;                  // grid sums done
    const int e = k * nx + i;    // this lane's element of the problem's vectors (when row)

    TM *blk = (TM *)smem_raw;
    auto base = [&](int q) -> TM * {
        return q < kGh ? blk + q * gks
                       : (q < kGh + W ? blk + kGh * gks + (q - kGh) * ks
                                      : blk + kGh * gks + W * ks + (q - kGh - W) * gks);
    };
    auto Lof = [&](int q) -> const TM * { return base(q) + ((q >= kGh && q < kGh + W) ? bp : 0); };
    auto Diof = [&](int q) -> const TM * { return base(q) + ((q >= kGh && q < kGh + W) ? bp + bs : bs); };
    TI *Yw = (TI *)(blk + coop_block_elems(W, bs, bp));     // y of every slot (S x nxp)
    TI *Uw = Yw + S * nxp;                                   // u of every slot
    TI *Rw = Uw + S * nxp;                                   // per-slot window (r, then t)
    double *lw = (double *)(Rw + S * nxp) + sl * 3 * nxp;  // FP64 lambda at k-1, k, k+1
    TI *wr = Rw + sl * nxp;
    for (int q = 0; q < S; ++q) {
        const int kq = k0 - kGh + q;
        if (kq < 0 || kq >= N) continue;
        const bool o = q >= kGh && q < kGh + W;
        const int cnt = o ? ks : gks;
        const TM *src = B3 + (int64_t)kq * ks + (o ? 0 : bp);
        TM *dst = base(q);
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) dst[t] = src[t];
    }
    // a workgroup that starts after another one has already given up (the
    // launch has failed) publishes nothing, so no stale tag can outlive it
    if (threadIdx.x == 0) s_ok = get(ca.flags + kErr) == 0u;
    __syncthreads();
    const bool started_ok = s_ok != 0;
    const TM *Dk = base(sl), *Lk = Lof(sl), *Dik = Diof(sl);
    const TM *Lk1 = sl + 1 < S ? Lof(sl + 1) : nullptr;  // L_{k+1}
    TM rdi[RN], rd[RN], rl0[RN], rl1[RN];
    if constexpr (REG) {
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            rdi[j] = row ? Dik[packed_index(i, j, NX)] : TM(0);
            rd[j] = own ? Dk[packed_index(i, j, NX)] : TM(0);
            rl0[j] = (row && k > 0) ? Lk[i * NX + j] : TM(0);
            rl1[j] = (row && k + 1 < N && Lk1) ? Lk1[j * NX + i] : TM(0);
        }
    }
    // row i of D_k^-1, D_k, L_k and L_{k+1}^T times a vector in LDS
    auto mv_dinv = [&](const TI *x) -> TI {
        if constexpr (REG) return dot_reg<RN>(rdi, x);
        else return dot_sym(Dik, i, x, nx);
    };
    auto mv_d = [&](const TI *x) -> TI {
        if constexpr (REG) return dot_reg<RN>(rd, x);
        else return dot_sym(Dk, i, x, nx);
    };
    auto mv_l0 = [&](const TI *x) -> TI {
        if constexpr (REG) return dot_reg<RN>(rl0, x);
        else return dot_row(Lk, i, x, nx);
    };
    auto mv_l1 = [&](const TI *x) -> TI {
        if constexpr (REG) return dot_reg<RN>(rl1, x);
        else return dot_col(Lk1, i, x, nx);
    };

    // Grid-wide sums of three values over the own knots (fixed order: wave
    // butterflies, own slots in order, then workgroups as below).  Before it
    // publishes its record a workgroup has published its w rows (tagged like
    // the record) and, with FENCE, completed its other stores.  Ghost waves
    // with `wslot` wait for their row of w and return it in `wv`.
    auto grid_sum3 = [&](double v0, double v1, double v2, double out[3], bool fence, u64 *wslot, TI &wv) -> bool {
        ++nsum;
        const unsigned tag = tag0 + nsum, par = nsum & 1;
        v0 = wave_sum(v0);
        v1 = wave_sum(v1);
        v2 = wave_sum(v2);
        if (lane == 0) {
            red[sl * 3 + 0] = v0;
            red[sl * 3 + 1] = v1;
            red[sl * 3 + 2] = v2;
        }
        if (threadIdx.x == 0) s_sum_ok[par] = 1;
        if (fence) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        u64 *rb = ca.rec + (size_t)par * G * 6;
        if (threadIdx.x < 3) {
            double t = 0.0;
            for (int q = kGh; q < kGh + W; ++q) t += red[q * 3 + threadIdx.x];
            put_tagged(rb + g * 6 + 2 * threadIdx.x, t, tag);
        }
        if (sl == 0) {
            // every workgroup sums the G records the same way: lane h takes
            // workgroups h, h + 64, ... in order, then the wave butterfly
            double t0, t1, t2;
            for (unsigned spins = 0;; ++spins) {
                bool here = true;
                t0 = t1 = t2 = 0.0;
                for (int h = lane; h < G; h += 64) {
                    double x0, x1, x2;
                    const bool h0 = get_tagged(rb + h * 6 + 0, x0, tag);
                    const bool h1 = get_tagged(rb + h * 6 + 2, x1, tag);
                    const bool h2 = get_tagged(rb + h * 6 + 4, x2, tag);
                    here = here && h0 && h1 && h2;
                    t0 += x0;
                    t1 += x1;
                    t2 += x2;
                }
                if (__all(here)) break;
                if (!keep_waiting(ca.flags, spins)) {
                    s_sum_ok[par] = 0;
                    break;
                }
            }
            t0 = wave_sum(t0);
            t1 = wave_sum(t1);
            t2 = wave_sum(t2);
            if (lane == 0) {
                sums[par][0] = t0;
                sums[par][1] = t1;
                sums[par][2] = t2;
            }
        }
        if (wslot) {
            for (unsigned spins = 0;; ++spins) {
                TI x;
                const bool here = !row || get_tagged(wslot, x, tag);
                if (row) wv = x;
                if (__all(here)) break;
                if (!keep_waiting(ca.flags, spins)) {
                    s_sum_ok[par] = 0;
                    break;
                }
            }
        }
        __syncthreads();
        out[0] = sums[par][0];
        out[1] = sums[par][1];
        out[2] = sums[par][2];
        return s_sum_ok[par] != 0;
    };
    TI wdummy = TI(0);

    const bool failed_build = build_failed(a.status[p]);
    int st = failed_build ? kNotSpd : kOk;
    int total = 0, steps = 0;
    double rnorm = 0.0, gnorm = 0.0;
    bool fallback = false, pc_fallback = false, alive = true;
    // ||gamma|| and finiteness of the inputs
    {
        double gg = 0.0, bad = 0.0;
        if (own) {
            const double gv = gam[e];
            gg = gv * gv;
            if (a.use_lambda0 == 1 && !isfinite(get(lam + e))) bad = 1.0;
            if (a.use_lambda0 == 0) put(lam + e, 0.0);
        }
        double t[3] = {0.0, 0.0, 0.0};
        alive = started_ok && grid_sum3(gg, bad, 0.0, t, false, nullptr, wdummy);
        gnorm = sqrt(t[0]);
        if (st == kOk && (!isfinite(gnorm) || t[1] != 0.0)) {
            st = kNonFinite;
            rnorm = NAN;
        }
    }
    if (st == kOk && alive && gnorm == 0.0) {
        if (own) put(lam + e, 0.0);
    } else if (st == kOk && alive) {
        const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * n;
        int pcur = a.pc, base_step = 0, pending = kOk;
        bool broke = false;
        double prev = INFINITY;
        double r64 = 0.0;  // this lane's FP64 residual row (own and ghost knots)
        for (;;) {
            // true residual r = gamma - S lambda in FP64 (hi + lo under FP32 storage)
            if (steps == 0 && a.use_lambda0 == 0) {
                r64 = row ? gam[e] : 0.0;
                rnorm = gnorm;
            } else {
                if (!grid_sync(ca.flags, G, gen, &s_ok)) {  // lambda of the neighbours is final
                    alive = false;
                    break;
                }
                if (is_own && lane < nx) {
                    lw[lane] = (k > 0 && k < N) ? get(lam + e - nx) : 0.0;
                    lw[nxp + lane] = k < N ? get(lam + e) : 0.0;
                    lw[2 * nxp + lane] = (k + 1 < N) ? get(lam + e + nx) : 0.0;
                }
                wave_sync();
                double rr = 0.0;
                if (own) {
                    const int64_t kd = (int64_t)k * bp, kl = (int64_t)k * bs, kl1 = (int64_t)(k + 1) * bs;
                    double y = 0.0;
#pragma unroll 2
                    for (int j = 0; j < nx; ++j) {
                        const int pi = packed_index(i, j, nx);
                        y += ((double)Dk[pi] + (SDlo ? (double)SDlo[kd + pi] : 0.0)) * lw[nxp + j];
                    }
                    if (k > 0)
#pragma unroll 2
                        for (int j = 0; j < nx; ++j)
                            y += ((double)Lk[i * nx + j] + (SLlo ? (double)SLlo[kl + i * nx + j] : 0.0)) * lw[j];
                    if (k + 1 < N)
#pragma unroll 2
                        for (int j = 0; j < nx; ++j)
                            y += ((double)Lk1[j * nx + i] + (SLlo ? (double)SLlo[kl1 + j * nx + i] : 0.0)) *
                                 lw[2 * nxp + j];
                    r64 = gam[e] - y;
                    rr = r64 * r64;
                    put(r64g + e, r64);
                }
                double t[3];
                if (!grid_sum3(rr, 0.0, 0.0, t, true, nullptr, wdummy)) {  // r64 rows are visible
                    alive = false;
                    break;
                }
                rnorm = sqrt(t[0]);
                if (row && !is_own) r64 = get(r64g + e);  // ghosts: the owners' rows
                if (steps == 0 && a.use_lambda0 == 2 && !(rnorm < gnorm)) {
                    // a warm start that does not reduce the residual is replaced by zero
                    if (own) put(lam + e, 0.0);
                    r64 = row ? gam[e] : 0.0;
                    rnorm = gnorm;
                    fallback = true;
                }
            }
            if (!isfinite(rnorm)) {
                st = kNonFinite;
                break;
            }
            if (pending != kOk) {
                st = pending;
                break;
            }
            if (rnorm <= a.tol * gnorm) break;
            if (steps > 0 && !a.refine) {
                st = kInaccurate;
                break;
            }
            if (broke && !(rnorm < prev)) {
                st = kBreakdown;
                break;
            }
            if (steps - base_step >= a.max_outer) {
                st = kMaxIter;
                break;
            }
            prev = rnorm;
            double tau = (a.refine ? a.theta : 1.0) * a.tol * gnorm / rnorm;
            if (a.refine && tau < a.tau_min) tau = a.tau_min;
            if (tau > 1.0) tau = 1.0;
            const TI c2 = pcur == 2 ? TI(1) : TI(0.5);

            // inner single-reduction PCG on S d = r / ||r|| from d = 0; r and
            // s = S p are kept at the own and the ghost knots, p and x at the own
            TI r = row ? (TI)(r64 / rnorm) : TI(0);
            TI x = TI(0), pv = TI(0), sv = TI(0);
            int it = 0, ist = kOk;
            TI alpha = TI(0), gam_prev = TI(0);
            TI bnorm = TI(0);
            for (;;) {
                // y = D^-1 r at every slot; t = O y, u = y - c D^-1 t at own +- 1
                if (lane < nx) wr[lane] = r;
                wave_sync();
                const TI y = row ? mv_dinv(wr) : TI(0);
                TI u = y;
                if (pcur != 0) {
                    if (lane < nx) Yw[sl * nxp + lane] = y;
                    __syncthreads();
                    TI t = TI(0);
                    if (row && inner) {
                        if (k > 0) t += mv_l0(Yw + (sl - 1) * nxp);
                        if (k + 1 < N) t += mv_l1(Yw + (sl + 1) * nxp);
                    }
                    if (lane < nx) wr[lane] = t;  // t replaces r in the window
                    wave_sync();
                    if (row && inner) u = y - c2 * mv_dinv(wr);
                }
                if (lane < nx) Uw[sl * nxp + lane] = u;
                __syncthreads();
                // w = S u at the own knots, published for the neighbours' ghosts
                TI w = TI(0);
                if (own) {
                    w = mv_d(Uw + sl * nxp);
                    if (k > 0) w += mv_l0(Uw + (sl - 1) * nxp);
                    if (k + 1 < N) w += mv_l1(Uw + (sl + 1) * nxp);
                }
                // this sum's tag and buffer: the next grid sum's
                u64 *wslot = ca.wtag + ((size_t)((nsum + 1) & 1) * n + (row ? e : 0)) * TW;
                if (own) put_tagged(wslot, w, tag0 + nsum + 1);
                double t3[3];
                if (!grid_sum3(own ? (double)(r * u) : 0.0, own ? (double)(w * u) : 0.0,
                               own ? (double)(r * r) : 0.0, t3, false, is_own ? nullptr : wslot, w)) {
                    alive = false;
                    break;
                }
                const TI dgam = (TI)t3[0], ddel = (TI)t3[1], drho = (TI)t3[2];
                if (it == 0) bnorm = sqrt(drho);
                const TI rn = sqrt(drho);
                if (!isfinite(rn)) {
                    ist = kNonFinite;
                    break;
                }
                if (rn <= (TI)tau * bnorm) break;
                if (total + it >= max_iter) {
                    ist = kMaxIter;
                    break;
                }
                TI den, beta;
                if (it == 0) {
                    den = ddel;
                    beta = TI(0);
                } else {
                    beta = dgam / gam_prev;
                    den = ddel - beta * dgam / alpha;
                }
                if (!(den > TI(0)) || !(dgam > TI(0))) {
                    ist = (isfinite(den) && isfinite(dgam)) ? kBreakdown : kNonFinite;
                    break;
                }
                alpha = dgam / den;
                gam_prev = dgam;
                // p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s
                // (one code path for own and ghost knots)
                pv = it == 0 ? u : u + beta * pv;
                sv = it == 0 ? w : w + beta * sv;
                x += alpha * pv;
                r -= alpha * sv;
                ++it;
            }
            if (!alive) break;
            total += it;
            ++steps;
            if (own) put(lam + e, get(lam + e) + rnorm * (double)x);
            broke = a.refine && ist == kBreakdown;
            if (broke && pcur != 0) {
                pcur = 0;
                pc_fallback = true;
                broke = false;
                base_step = steps;
            }
            if (ist != kOk && !broke && !(a.refine && ist == kBreakdown)) pending = ist;
        }
    }
    if (!alive) st = kNonFinite;  // a wait gave up: report the problem as failed
    if (failed_build && own) put(lam + e, 0.0);
    // The next launch's tags start after every tag this one may have used:
    // a workgroup publishes sum s + 1 only after it has seen workgroup 0's
    // record of sum s, so no tag beyond tag0 + nsum + 1 was written (also
    // after a failed wait).  Every workgroup read tag0 before its first record.
    if (g == 0 && threadIdx.x == 0) put(ca.flags + kTagBase, tag0 + nsum + 2);
    if (g == 0 && threadIdx.x == 0) {
        a.iters[p] = total;
        a.outer[p] = steps;
        a.relres[p] = failed_build ? NAN : (gnorm == 0.0 ? 0.0 : rnorm / gnorm);
        a.status[p] = st | (fallback ? kWarmFallback : 0) | (pc_fallback ? kPcFallback : 0);
    }
}

int coop_lds(int nx, bool fp32, int W) {
    const int eb = fp32 ? 4 : 8;
    const int bs = block_stride(nx, eb), bp = packed_stride(nx, eb), nxp = (nx + 3) & ~3, S = W + 2 * kGh;
    return eb * (coop_block_elems(W, bs, bp) + 3 * S * nxp) + 8 * S * 3 * nxp + 16;
}

int coop_flag_words(int N) { return kFlag0 + N; }
int coop_clear_first() { return kErr; }
size_t coop_rec_words(int N) { return (size_t)12 * N; }
size_t coop_wtag_words(int N, int nx) { return (size_t)4 * N * nx; }

namespace {

using CoopKernel = void (*)(CoopArgs);

// state sizes with a compiled-in specialisation
template <typename TI>
CoopKernel coop_kernel(int nx) {
    switch (nx) {
        case 6: return k_coop<TI, 6>;
        case 14: return k_coop<TI, 14>;
        case 26: return k_coop<TI, 26>;
        case 36: return k_coop<TI, 36>;
        default: return k_coop<TI, 0>;
    }
}

CoopKernel coop_kernel(int nx, bool fp32) { return fp32 ? coop_kernel<float>(nx) : coop_kernel<double>(nx); }

}  // namespace

bool coop_plan(int N, int nx, bool fp32, int device, int *W_out, int *G_out) {
    if (N < 1 || nx < 1 || nx > 64) return false;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return false;
    const void *f = (const void *)coop_kernel(nx, fp32);
    for (int W = kMaxW; W >= 2; --W) {
        const int lds = coop_lds(nx, fp32, W);
        if (lds > kFusedLdsCap) continue;
        int blocks = 0;
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return false;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, 64 * (W + 2 * kGh), lds) != hipSuccess)
            return false;
        const int G = (N + W - 1) / W;
        if (G <= blocks * cus) {
            *W_out = W;
            *G_out = G;
            return true;
        }
    }
    return false;
}

hipError_t launch_coop(const SolveArgs &a, unsigned *flags, u64 *rec, u64 *wtag, int nx, int W, int G, bool fp32,
                       hipStream_t s) {
    if (W < 2 || W > kMaxW || G < 1) return hipErrorInvalidValue;
    CoopArgs ca;
    ca.s = a;
    ca.flags = flags;
    ca.rec = rec;
    ca.wtag = wtag;
    ca.G = G;
    ca.W = W;
    const void *f = (const void *)coop_kernel(nx, fp32);
    const int lds = coop_lds(nx, fp32, W);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    void *args[] = {&ca};
    return hipLaunchCooperativeKernel(f, dim3(G), dim3(64 * (W + 2 * kGh)), args, lds, s);
}

}  // namespace ssp
