// Batched preconditioned conjugate gradient on S lambda = gamma.
//
// One workgroup owns one problem for the whole solve (largest problems are
// dispatched first).  Every product with S or Phi^-1 is a sweep over the
// problem's knots in chunks: the chunk's nx x nx blocks and its slice of the
// input vector (plus one halo knot on each side) are staged in LDS with
// coalesced loads, then each thread produces one row
//   y_k = Dg_k x_k + Sb_k x_{k-1} + Sb_{k+1}^T x_{k+1}
// (Sec. II-A block-tridiagonal form; the symmetric-stair Phi^-1 of Sec. IV
// and the additive stair of Sec. III have the same stencil, block-Jacobi has
// no off-diagonal term).  The PCG recurrences are the textbook ones the paper
// relies on in Sec. II-B; reductions are fixed-order wave butterflies plus a
// sequential sum over waves, so results are bitwise reproducible.
//
// Precision: the outer loop is FP64 iterative refinement.  Each step forms
// the true residual r = gamma - S lambda in FP64 (S = hi + lo under FP32
// storage), stops at ||r|| <= tol ||gamma||, else solves S d = r / ||r|| with
// the inner PCG in the storage precision and adds ||r|| d to lambda in FP64.
// FP64 and plain FP32 modes run exactly one inner solve.
#include <math.h>

#include "ssp_device.h"
#include "ssp_host.h"

namespace ssp {

namespace {

// Staging geometry of one sweep.  Rows of a staged block are padded to
// nx + 1 elements (odd for even nx) so that row-wise LDS reads by
// consecutive lanes fall in distinct banks.
struct Geo {
    int nx, ldx, blk, nn, C;
    uint64_t mg;  // magic for division by nx
};

template <typename TS>
__device__ __forceinline__ Geo make_geo(int nx, bool has_sub, int lds_bytes, int block) {
    Geo g;
    g.nx = nx;
    g.ldx = nx + 1;
    g.blk = nx * g.ldx;
    g.nn = nx * nx;
    g.mg = div_magic(nx);
    const int per_knot = (has_sub ? 2 : 1) * g.blk + nx;
    const int fixed = (has_sub ? g.blk : 0) + 2 * nx;
    int C = block / nx;
    const int Cl = (lds_bytes / (int)sizeof(TS) - fixed) / per_knot;
    if (Cl < C) C = Cl;
    g.C = C < 1 ? 1 : C;
    return g;
}

// One block-tridiagonal product over a problem of N knots.
//   Dg, Sb: diagonal and sub-diagonal blocks (storage TM, row-major, Sb[0]
//   ignored); Dlo/Slo optional FP32 remainders added during staging.
//   xval(row): value of the input vector at a row of the problem (it may be
//   called for halo rows owned by other threads).
//   epi(row, y, x): called once per row by the row's owner with the product
//   row y and the staged input x.
template <typename TS, typename TM, int BLOCK, typename XF, typename EF>
__device__ __forceinline__ void bt_sweep(int N, const Geo &g, const TM *__restrict__ Dg,
                                         const float *__restrict__ Dlo, const TM *__restrict__ Sb,
                                         const float *__restrict__ Slo, bool has_sub, TS *smem, XF &&xval,
                                         EF &&epi) {
    const int tid = threadIdx.x;
    const int nx = g.nx, ldx = g.ldx, blk = g.blk, nn = g.nn, C = g.C;
    TS *Ds = smem;
    TS *Ss = Ds + C * blk;
    TS *xs = Ss + (has_sub ? (C + 1) * blk : 0);
    for (int k0 = 0; k0 < N; k0 += C) {
        const int kc = min(C, N - k0);
        __syncthreads();
        {
            const TM *src = Dg + (int64_t)k0 * nn;
            const float *srl = Dlo ? Dlo + (int64_t)k0 * nn : nullptr;
            const int cnt = kc * nn;
            for (int e = tid; e < cnt; e += BLOCK) {
                TS v = (TS)src[e];
                if (srl) v += (TS)srl[e];
                Ds[e + fast_div(e, g.mg)] = v;
            }
        }
        if (has_sub) {
            const int ks = min(kc + 1, N - k0);
            const TM *src = Sb + (int64_t)k0 * nn;
            const float *srl = Slo ? Slo + (int64_t)k0 * nn : nullptr;
            const int cnt = ks * nn;
            for (int e = tid; e < cnt; e += BLOCK) {
                TS v = (TS)src[e];
                if (srl) v += (TS)srl[e];
                Ss[e + fast_div(e, g.mg)] = v;
            }
        }
        {
            const int cnt = (kc + 2) * nx;
            const int base = (k0 - 1) * nx;
            for (int t = tid; t < cnt; t += BLOCK) {
                const int row = base + t;
                xs[t] = (row >= 0 && row < N * nx) ? xval(row) : TS(0);
            }
        }
        __syncthreads();
        if (tid < kc * nx) {
            const int kk = fast_div(tid, g.mg), i = tid - kk * nx, k = k0 + kk;
            const TS *dcol = Ds + kk * blk + i;  // column i of the symmetric Dg_k
            const TS *xk = xs + (kk + 1) * nx;
            TS y = TS(0);
            for (int j = 0; j < nx; ++j) y += dcol[j * ldx] * xk[j];
            if (has_sub) {
                if (k > 0) {
                    const TS *lrow = Ss + kk * blk + i * ldx;  // row i of Sb_k
                    const TS *xm = xs + kk * nx;
                    for (int j = 0; j < nx; ++j) y += lrow[j] * xm[j];
                }
                if (k + 1 < N) {
                    const TS *lcol = Ss + (kk + 1) * blk + i;  // column i of Sb_{k+1}
                    const TS *xp = xs + (kk + 2) * nx;
                    for (int j = 0; j < nx; ++j) y += lcol[j * ldx] * xp[j];
                }
            }
            epi(k * nx + i, y, xk[i]);
        }
    }
}

}  // namespace

template <typename TI, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_pcg(SolveArgs a) {
    using TM = TI;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red64[2 * (BLOCK / kWave)];
    __shared__ TI redT[2 * (BLOCK / kWave)];
    const int tid = threadIdx.x;
    const int p = a.order[blockIdx.x];
    const int N = a.N[p], nx = a.nx[p];
    const int n = N * nx;
    const int64_t onn = a.off_nn[p], ov = a.off_v[p];
    double *lam = a.lambda + ov;
    const double *gam = a.gamma + ov;
    double *r64 = a.r64 + ov;

    int st = a.status[p];
    if (st != kOk) {
        for (int row = tid; row < n; row += BLOCK) lam[row] = 0.0;
        if (tid == 0) {
            a.iters[p] = 0;
            a.outer[p] = 0;
            a.relres[p] = NAN;
        }
        return;
    }
    const bool has_M = a.PM != nullptr;
    const TM *SD = (const TM *)a.SD + onn, *SL = (const TM *)a.SL + onn;
    const float *SDlo = a.SDlo ? a.SDlo + onn : nullptr, *SLlo = a.SLlo ? a.SLlo + onn : nullptr;
    const TM *PD = (const TM *)a.PD + onn, *PM = has_M ? (const TM *)a.PM + onn : nullptr;
    TI *W = (TI *)a.work;
    TI *R[2] = {W + 0 * a.tot_v + ov, W + 1 * a.tot_v + ov};
    TI *Pv[2] = {W + 2 * a.tot_v + ov, W + 3 * a.tot_v + ov};
    TI *Qv = W + 4 * a.tot_v + ov, *Zv = W + 5 * a.tot_v + ov, *Dv = W + 6 * a.tot_v + ov;
    const int max_iter = a.max_iter > 0 ? a.max_iter : 10 * n;

    // ||gamma||, finiteness of gamma and lambda0
    double gg = 0.0, bad = 0.0;
    for (int row = tid; row < n; row += BLOCK) {
        const double gv = gam[row];
        gg += gv * gv;
        if (a.use_lambda0) {
            if (!isfinite(lam[row])) bad = 1.0;
        } else {
            lam[row] = 0.0;
        }
    }
    block_sum2<BLOCK>(gg, bad, red64);
    int total = 0, steps = 0;
    double rnorm = 0.0;
    const double gnorm = sqrt(gg);
    if (!isfinite(gnorm) || bad != 0.0) {
        st = kNonFinite;
        rnorm = NAN;
    } else if (gg == 0.0) {
        for (int row = tid; row < n; row += BLOCK) lam[row] = 0.0;
    } else {
        const Geo g64 = make_geo<double>(nx, true, a.lds_bytes, BLOCK);
        const Geo gS = make_geo<TI>(nx, true, a.lds_bytes, BLOCK);
        const Geo gP = make_geo<TI>(nx, has_M, a.lds_bytes, BLOCK);
        int pending = kOk;
        for (;;) {
            // true residual r = gamma - S lambda in FP64
            double rr64 = 0.0;
            bt_sweep<double, TM, BLOCK>(
                N, g64, SD, SDlo, SL, SLlo, true, (double *)smem_raw, [&](int row) { return lam[row]; },
                [&](int row, double y, double) {
                    const double r = gam[row] - y;
                    r64[row] = r;
                    rr64 += r * r;
                });
            rr64 = block_sum<BLOCK>(rr64, red64);
            rnorm = sqrt(rr64);
            if (!isfinite(rnorm)) {
                st = kNonFinite;
                break;
            }
            if (pending != kOk) {
                st = pending;
                break;
            }
            if (rnorm <= a.tol * gnorm) break;
            if (steps > 0 && !a.refine) break;
            if (steps >= a.max_outer) {
                st = kMaxIter;
                break;
            }
            double tau = (a.refine ? a.theta : 1.0) * a.tol * gnorm / rnorm;
            if (a.refine && tau < a.tau_min) tau = a.tau_min;
            if (tau > 1.0) tau = 1.0;
            const double inv_s = 1.0 / rnorm;

            // inner PCG on S d = r / ||r|| from d = 0
            int rc = 0, pc = 0, it = 0, ist = kOk;
            TI rz = TI(0), rr = TI(0), beta = TI(0), alpha = TI(0);
            bt_sweep<TI, TM, BLOCK>(
                N, gP, PD, nullptr, PM, nullptr, has_M, (TI *)smem_raw,
                [&](int row) { return (TI)(r64[row] * inv_s); },
                [&](int row, TI y, TI x) {
                    Zv[row] = y;
                    R[rc][row] = x;
                    Dv[row] = TI(0);
                    rz += x * y;
                    rr += x * x;
                });
            block_sum2<BLOCK>(rz, rr, redT);
            const TI bnorm = sqrt(rr);
            const TI tauT = (TI)tau;
            for (;;) {
                const TI rn = sqrt(rr);
                if (!isfinite(rn)) {
                    ist = kNonFinite;
                    break;
                }
                if (rn <= tauT * bnorm) break;
                if (total + it >= max_iter) {
                    ist = kMaxIter;
                    break;
                }
                // q = S p with p = z + beta p_old (p = z on the first pass)
                TI pq = TI(0);
                const bool first = (it == 0);
                TI *Pold = Pv[pc], *Pnew = Pv[pc ^ 1];
                bt_sweep<TI, TM, BLOCK>(
                    N, gS, SD, nullptr, SL, nullptr, true, (TI *)smem_raw,
                    [&](int row) { return first ? Zv[row] : Zv[row] + beta * Pold[row]; },
                    [&](int row, TI y, TI x) {
                        Qv[row] = y;
                        Pnew[row] = x;
                        pq += x * y;
                    });
                pq = block_sum<BLOCK>(pq, redT);
                pc ^= 1;
                ++it;
                if (!(pq > TI(0)) || !(rz > TI(0))) {
                    ist = isfinite(pq) ? kBreakdown : kNonFinite;
                    break;
                }
                alpha = rz / pq;
                // r -= alpha q ; d += alpha p ; z = Phi^-1 r
                TI rzn = TI(0);
                rr = TI(0);
                TI *Rold = R[rc], *Rnew = R[rc ^ 1], *Pcur = Pv[pc];
                bt_sweep<TI, TM, BLOCK>(
                    N, gP, PD, nullptr, PM, nullptr, has_M, (TI *)smem_raw,
                    [&](int row) { return Rold[row] - alpha * Qv[row]; },
                    [&](int row, TI y, TI x) {
                        Zv[row] = y;
                        Rnew[row] = x;
                        Dv[row] += alpha * Pcur[row];
                        rzn += x * y;
                        rr += x * x;
                    });
                block_sum2<BLOCK>(rzn, rr, redT);
                rc ^= 1;
                beta = rzn / rz;
                rz = rzn;
            }
            total += it;
            ++steps;
            __syncthreads();
            for (int row = tid; row < n; row += BLOCK) lam[row] += rnorm * (double)Dv[row];
            if (ist != kOk) pending = ist;
        }
    }
    if (tid == 0) {
        a.iters[p] = total;
        a.outer[p] = steps;
        a.relres[p] = gg == 0.0 ? 0.0 : rnorm / gnorm;
        a.status[p] = st;
    }
}

int pcg_min_lds(int nx_max, bool has_sub) {
    const int blk = nx_max * (nx_max + 1);
    const int per_knot = (has_sub ? 2 : 1) * blk + nx_max;
    const int fixed = (has_sub ? blk : 0) + 2 * nx_max;
    return (int)sizeof(double) * (per_knot + fixed);
}

int pcg_default_lds(int nx_max, bool fp32, int threads) {
    const int blk = nx_max * (nx_max + 1);
    const int C = threads / nx_max < 1 ? 1 : threads / nx_max;
    const int elem = fp32 ? 4 : 8;
    int want = elem * (C * (2 * blk + nx_max) + blk + 2 * nx_max);
    const int lo = pcg_min_lds(nx_max, true);
    const int cap = lo > 64 * 1024 ? lo : 64 * 1024;
    if (want > cap) want = cap;
    if (want < lo) want = lo;
    return want;
}

template <typename TI, int BLOCK>
static hipError_t launch_t(const SolveArgs &a, int nprob, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void *)k_pcg<TI, BLOCK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       a.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_pcg<TI, BLOCK>), dim3(nprob), dim3(BLOCK), a.lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_pcg(const SolveArgs &a, int nprob, bool fp32, int threads, hipStream_t s) {
    if (nprob == 0) return hipSuccess;
    if (fp32) {
        switch (threads) {
            case 64: return launch_t<float, 64>(a, nprob, s);
            case 128: return launch_t<float, 128>(a, nprob, s);
            case 256: return launch_t<float, 256>(a, nprob, s);
            case 512: return launch_t<float, 512>(a, nprob, s);
        }
    } else {
        switch (threads) {
            case 64: return launch_t<double, 64>(a, nprob, s);
            case 128: return launch_t<double, 128>(a, nprob, s);
            case 256: return launch_t<double, 256>(a, nprob, s);
            case 512: return launch_t<double, 512>(a, nprob, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace ssp
