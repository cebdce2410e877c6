// Batched preconditioned conjugate gradient on S lambda = gamma, explicit form:
// the preconditioner's stored blocks are streamed in a sweep of their own.
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
// FP64 and plain FP32 modes run exactly one inner solve.  Under refinement
// a float breakdown (p^T S p <= 0 or r^T z <= 0) only ends the inner solve;
// it is reported when the next FP64 residual has not decreased.
#include <math.h>

#include "ssp_device.h"
#include "ssp_host.h"
#include "ssp_sweep.h"

namespace ssp {

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
    const int64_t onn = a.off_blk[p], ov = a.off_v[p];
    const int bs = block_stride(nx, sizeof(TM));
    double *lam = a.lambda + ov;
    const double *gam = a.gamma + ov;
    double *r64 = a.r64 + ov;

    int st = kOk;
    if (build_failed(a.status[p])) {
        for (int row = tid; row < n; row += BLOCK) lam[row] = 0.0;
        if (tid == 0) {
            a.iters[p] = 0;
            a.outer[p] = 0;
            a.relres[p] = NAN;
        }
        return;
    }
    bool has_M = a.PM != nullptr;
    const int bp = packed_stride(nx, sizeof(TM)), ks3 = 2 * bp + bs;  // knot stride
    const TM *SD = (const TM *)a.B3 + a.off_b3[p], *SL = SD + bp, *PD = SD + bp + bs;  // D, D^-1 packed
    const float *SDlo = a.SDlo ? a.SDlo + a.off_pk[p] : nullptr, *SLlo = a.SLlo ? a.SLlo + onn : nullptr;
    const TM *PM = has_M ? (const TM *)a.PM + onn : nullptr;
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
        if (a.use_lambda0 == 1) {
            if (!isfinite(lam[row])) bad = 1.0;
        } else if (a.use_lambda0 == 0) {
            lam[row] = 0.0;
        }
    }
    block_sum2<BLOCK>(gg, bad, red64);
    int total = 0, steps = 0;
    bool fallback = false;     // the warm start was dropped for lambda = 0
    bool pc_fallback = false;  // block-Jacobi took over after a float breakdown
    double rnorm = 0.0;
    const double gnorm = sqrt(gg);
    if (!isfinite(gnorm) || bad != 0.0) {
        st = kNonFinite;
        rnorm = NAN;
    } else if (gg == 0.0) {
        for (int row = tid; row < n; row += BLOCK) lam[row] = 0.0;
    } else {
        const Geo g64 = make_geo<double>(nx, bs, true, a.lds_bytes, BLOCK);
        const Geo gS = make_geo<TI>(nx, bs, true, a.lds_bytes, BLOCK);
        const Geo gP = make_geo<TI>(nx, bs, has_M, a.lds_bytes, BLOCK);
        int pending = kOk, base = 0;
        bool broke = false;  // last inner solve ended in a float breakdown (refinement only)
        double prev = INFINITY;
        for (;;) {
            // true residual r = gamma - S lambda in FP64
            double rr64 = 0.0, gg64 = 0.0;  // ||r||^2 and ||gamma||^2 over the same rows in the same order
            bt_sweep<double, TM, BLOCK, 0>(
                N, g64, SD, ks3, SDlo, bp, SL, ks3, SLlo, true, (double *)smem_raw, [&](int row) { return lam[row]; },
                [&](int row, double y, double) {
                    const double gv = gam[row];
                    const double r = gv - y;
                    r64[row] = r;
                    rr64 += r * r;
                    gg64 += gv * gv;
                });
            block_sum2<BLOCK>(rr64, gg64, red64);
            rnorm = sqrt(rr64);
            // kept only if strictly below ||gamma|| (lambda0 = 0 ties and falls back)
            if (steps == 0 && a.use_lambda0 == 2 && !(rnorm < sqrt(gg64))) {
                // a warm start that does not reduce the residual is replaced by zero
                for (int row = tid; row < n; row += BLOCK) {
                    lam[row] = 0.0;
                    r64[row] = gam[row];
                }
                rnorm = gnorm;
                fallback = true;
                __syncthreads();
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
            if (steps - base >= a.max_outer) {
                st = kMaxIter;
                break;
            }
            prev = rnorm;
            double tau = (a.refine ? a.theta : 1.0) * a.tol * gnorm / rnorm;
            if (a.refine && tau < a.tau_min) tau = a.tau_min;
            if (tau > 1.0) tau = 1.0;
            const double inv_s = 1.0 / rnorm;

            // inner PCG on S d = r / ||r|| from d = 0
            int rc = 0, pc = 0, it = 0, ist = kOk;
            TI rz = TI(0), rr = TI(0), beta = TI(0), alpha = TI(0);
            bt_sweep<TI, TM, BLOCK, 0>(
                N, gP, PD, ks3, nullptr, bp, PM, bs, nullptr, has_M, (TI *)smem_raw,
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
                bt_sweep<TI, TM, BLOCK, 0>(
                    N, gS, SD, ks3, nullptr, bp, SL, ks3, nullptr, true, (TI *)smem_raw,
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
                bt_sweep<TI, TM, BLOCK, 0>(
                    N, gP, PD, ks3, nullptr, bp, PM, bs, nullptr, has_M, (TI *)smem_raw,
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
            // under refinement a float breakdown only ends the inner solve; under a
            // stair preconditioner it also hands the rest of the solve to
            // block-Jacobi (the float stair operator lost definiteness)
            broke = a.refine && ist == kBreakdown;
            if (broke && has_M) {
                has_M = false;
                pc_fallback = true;
                broke = false;
                base = steps;
            }
            if (ist != kOk && !broke && !(a.refine && ist == kBreakdown)) pending = ist;
        }
    }
    if (tid == 0) {
        a.iters[p] = total;
        a.outer[p] = steps;
        a.relres[p] = gg == 0.0 ? 0.0 : rnorm / gnorm;
        a.status[p] = st | (fallback ? kWarmFallback : 0) | (pc_fallback ? kPcFallback : 0);
    }
}

int pcg_min_lds(int nx_max, bool has_sub) { return bt_sweep_min_lds(nx_max, has_sub, sizeof(double)); }

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
