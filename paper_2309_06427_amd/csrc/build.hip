// Assembly of S and Phi^-1 from per-knot blocks, in FP64 on the device.
//
// Three knot-parallel phases (a launch boundary between phases supplies the
// neighbour knot's results):
//   1. Q_k^-1 and R_k^-1                      (Sec. II-A block entries)
//   2. D_k = Q_k^-1 + A_{k-1} Q_{k-1}^-1 A_{k-1}^T + B_{k-1} R_{k-1}^-1 B_{k-1}^T,
//      L_k = -A_{k-1} Q_{k-1}^-1, D_k^-1          (negated Eq. (schur) blocks;
//      D^-1 is the block-Jacobi inverse, Eq. (jacobi))
//   3. Phi^-1[k][k-1] = -D_k^-1 L_k D_{k-1}^-1 (symmetric stair, Sec. IV),
//      half of it for the additive stair (Sec. III), nothing for block-Jacobi.
// Phases 1 and 2 here are the generic form for any state size: one 64-lane
// workgroup per knot with its matrices in LDS (the compiled state sizes use
// the register-resident kernels instead).  Phase 3 reads the stored blocks.  SPD
// inverses use Gauss-Jordan elimination without pivoting: for an SPD matrix
// every pivot is a positive Schur-complement diagonal, so a non-positive
// pivot flags the matrix as not positive definite.
#include "ssp_device.h"
#include "ssp_host.h"
#include "ssp_sweep.h"

namespace ssp {

namespace {

constexpr int T = kWave;  // threads per knot team

// In-place inverse of the SPD n x n matrix a (row-major, LDS).  col: n
// doubles of LDS.  Returns false if a pivot is not positive (uniform).
__device__ bool team_spd_inverse(double *a, double *col, int n) {
    const int lane = threadIdx.x;
    bool ok = true;
    for (int k = 0; k < n; ++k) {
        __syncthreads();
        const double piv = a[k * n + k];
        if (!(piv > 0.0)) ok = false;
        const double inv = 1.0 / piv;
        for (int i = lane; i < n; i += T) col[i] = a[i * n + k];
        __syncthreads();
        for (int j = lane; j < n; j += T) a[k * n + j] = (j == k ? 1.0 : a[k * n + j]) * inv;
        __syncthreads();
        for (int e = lane; e < n * n; e += T) {
            const int i = e / n, j = e - i * n;
            if (i != k) a[e] = (j == k ? 0.0 : a[e]) - col[i] * a[k * n + j];
        }
    }
    __syncthreads();
    // symmetrise (the exact inverse is symmetric)
    for (int e = lane; e < n * n; e += T) {
        const int i = e / n, j = e - i * n;
        if (i < j) {
            const double s = 0.5 * (a[i * n + j] + a[j * n + i]);
            a[i * n + j] = s;
            a[j * n + i] = s;
        }
    }
    __syncthreads();
    return ok;
}

// C (m x n) = X (m x k) * Y, Y stored k x n (ty = 0) or n x k (ty = 1, i.e. Y^T).
__device__ void team_gemm(int m, int k, int n, const double *X, const double *Y, bool ty, double *Cm) {
    for (int e = threadIdx.x; e < m * n; e += T) {
        const int i = e / n, j = e - i * n;
        double s = 0.0;
        if (ty)
            for (int l = 0; l < k; ++l) s += X[i * k + l] * Y[j * k + l];
        else
            for (int l = 0; l < k; ++l) s += X[i * k + l] * Y[l * n + j];
        Cm[e] = s;
    }
    __syncthreads();
}

__device__ void team_load(double *dst, const double *src, int cnt) {
    for (int e = threadIdx.x; e < cnt; e += T) dst[e] = src[e];
}

__device__ void team_store(double *dst, const double *src, int cnt) {
    for (int e = threadIdx.x; e < cnt; e += T) dst[e] = src[e];
}

template <typename TM>
__device__ void store_split(TM *hi, float *lo, const double *src, int cnt, double scale) {
    for (int e = threadIdx.x; e < cnt; e += T) {
        const double v = scale * src[e];
        const TM h = (TM)v;
        hi[e] = h;
        if (lo) lo[e] = (float)(v - (double)h);
    }
}

// Upper triangle of the symmetric n x n matrix src (row-major, LDS) into
// packed form, with the FP32 remainder.
template <typename TM>
__device__ void store_split_packed(TM *hi, float *lo, const double *src, int n) {
    for (int e = threadIdx.x; e < n * n; e += T) {
        const int r = e / n, c = e - r * n;
        if (c >= r) {
            const double v = src[e];
            const TM h = (TM)v;
            hi[packed_row(r, n) + c] = h;
            if (lo) lo[packed_row(r, n) + c] = (float)(v - (double)h);
        }
    }
}

__device__ __forceinline__ void knot_of(const BuildArgs &a, int &p, int &k) {
    const int g = blockIdx.x;
    p = a.knot_prob[g];
    k = g - (int)a.koff[p];
}

// knot of a generic-assembly workgroup
__device__ __forceinline__ void listed_knot_of(const BuildArgs &a, int &p, int &k) {
    const int g = a.knot_list[blockIdx.x];
    p = a.knot_prob[g];
    k = g - (int)a.koff[p];
}

// full n x n matrix in LDS from its packed upper triangle
template <typename TM>
__device__ void team_load_packed(double *dst, const TM *src, int n) {
    for (int e = threadIdx.x; e < n * n; e += T) {
        const int r = e / n, c = e - r * n;
        dst[e] = (double)src[packed_index(r, c, n)];
    }
}

template <typename TM>
__device__ void team_load_lo(double *dst, const TM *src, const float *lo, int cnt, double scale) {
    for (int e = threadIdx.x; e < cnt; e += T) dst[e] = scale * ((double)src[e] + (lo ? (double)lo[e] : 0.0));
}

}  // namespace

// Phase 1: Q_k^-1 (every knot) and R_k^-1 (k < N-1).
__global__ __launch_bounds__(T) void k_build_inv(BuildArgs a) {
    extern __shared__ double sm[];
    int p, k;
    listed_knot_of(a, p, k);
    const int N = a.N[p], nx = a.nx[p], nu = a.nu[p];
    double *m = sm, *col = sm + a.mx * a.mx;
    team_load(m, a.Q + a.off_nn[p] + (int64_t)k * nx * nx, nx * nx);
    bool ok = team_spd_inverse(m, col, nx);
    team_store(a.Qinv + a.off_nn[p] + (int64_t)k * nx * nx, m, nx * nx);
    if (k < N - 1 && nu > 0) {
        __syncthreads();
        team_load(m, a.R + a.off_uu[p] + (int64_t)k * nu * nu, nu * nu);
        ok = team_spd_inverse(m, col, nu) && ok;
        team_store(a.Rinv + a.off_uu[p] + (int64_t)k * nu * nu, m, nu * nu);
    }
    if (!ok && threadIdx.x == 0) atomicOr(a.status + p, kNotSpd);
}

// Phase 2: D_k, L_k (stored in TM, plus the FP32 remainder for FP32 storage)
// and D_k^-1.
template <typename TM>
__global__ __launch_bounds__(T) void k_build_S(BuildArgs a) {
    extern __shared__ double sm[];
    int p, k;
    listed_knot_of(a, p, k);
    const int nx = a.nx[p], nu = a.nu[p];
    const int nn = nx * nx;
    const int64_t o = a.off_nn[p] + (int64_t)k * nn;
    const int bs = block_stride(nx, sizeof(TM)), bp = packed_stride(nx, sizeof(TM));
    const int64_t os = a.off_blk[p] + (int64_t)k * bs;  // remainder of L_k
    const int64_t od = a.off_pk[p] + (int64_t)k * bp;   // remainder of D_k (packed)
    TM *blk = (TM *)a.B3 + a.off_b3[p] + (int64_t)k * (2 * bp + bs);  // D_k (packed), L_k, D_k^-1 (packed)
    double *Dm = sm, *Am = Dm + nn, *Qp = Am + nn, *T1 = Qp + nn, *Bm = T1 + nn;
    double *Rm = Bm + nx * nu, *BR = Rm + nu * nu, *col = BR + nx * nu;
    team_load(Dm, a.Qinv + o, nn);
    if (k > 0) {
        const int64_t om = o - nn;
        team_load(Am, a.A + om, nn);
        team_load(Qp, a.Qinv + om, nn);
        __syncthreads();
        team_gemm(nx, nx, nx, Am, Qp, false, T1);  // A Q^-1 (= phi, L_k = -phi)
        for (int e = threadIdx.x; e < nn; e += T) {
            double s = 0.0;
            const int i = e / nx, j = e - i * nx;
            for (int l = 0; l < nx; ++l) s += T1[i * nx + l] * Am[j * nx + l];  // A Q^-1 A^T
            Dm[e] += s;
        }
        if (nu > 0) {
            const int64_t ob = a.off_nu[p] + (int64_t)(k - 1) * nx * nu;
            const int64_t ou = a.off_uu[p] + (int64_t)(k - 1) * nu * nu;
            team_load(Bm, a.B + ob, nx * nu);
            team_load(Rm, a.Rinv + ou, nu * nu);
            __syncthreads();
            team_gemm(nx, nu, nu, Bm, Rm, false, BR);  // B R^-1
            for (int e = threadIdx.x; e < nn; e += T) {
                double s = 0.0;
                const int i = e / nx, j = e - i * nx;
                for (int l = 0; l < nu; ++l) s += BR[i * nu + l] * Bm[j * nu + l];  // B R^-1 B^T
                Dm[e] += s;
            }
        }
        __syncthreads();
        store_split(blk + bp, a.SLlo ? a.SLlo + os : nullptr, T1, nn, -1.0);
    } else {
        for (int e = threadIdx.x; e < nn; e += T) {
            blk[bp + e] = (TM)0;
            if (a.SLlo) a.SLlo[os + e] = 0.f;
        }
    }
    __syncthreads();
    // exact symmetry of the stored D (the PCG kernel reads D by columns)
    for (int e = threadIdx.x; e < nn; e += T) {
        const int i = e / nx, j = e - i * nx;
        if (i < j) {
            const double s = 0.5 * (Dm[i * nx + j] + Dm[j * nx + i]);
            Dm[i * nx + j] = s;
            Dm[j * nx + i] = s;
        }
    }
    __syncthreads();
    store_split_packed(blk, a.SDlo ? a.SDlo + od : nullptr, Dm, nx);
    __syncthreads();
    const bool ok = team_spd_inverse(Dm, col, nx);
    store_split_packed(blk + bp + bs, (float *)nullptr, Dm, nx);
    if (!ok && threadIdx.x == 0) atomicOr(a.status + p, kNotSpd);
}

// S given directly by its blocks (D_k, and L_k = S[k][k-1] for k >= 1, FP64
// row-major at the problem's off_nn): stores D_k (symmetrised) and L_k like
// phase 2, and D_k^-1.  One workgroup per knot of the batch.
template <typename TM>
__global__ __launch_bounds__(T) void k_build_blocks(BuildArgs a, const double *D, const double *Lsub) {
    extern __shared__ double sm[];
    int p, k;
    knot_of(a, p, k);
    const int nx = a.nx[p], nn = nx * nx;
    const int64_t o = a.off_nn[p] + (int64_t)k * nn;
    const int bs = block_stride(nx, sizeof(TM)), bp = packed_stride(nx, sizeof(TM));
    const int64_t os = a.off_blk[p] + (int64_t)k * bs;  // remainder of L_k
    const int64_t od = a.off_pk[p] + (int64_t)k * bp;   // remainder of D_k (packed)
    TM *blk = (TM *)a.B3 + a.off_b3[p] + (int64_t)k * (2 * bp + bs);  // D_k (packed), L_k, D_k^-1 (packed)
    double *Dm = sm, *col = sm + nn;
    team_load(Dm, D + o, nn);
    if (k > 0) {
        store_split(blk + bp, a.SLlo ? a.SLlo + os : nullptr, Lsub + o, nn, 1.0);
    } else {
        for (int e = threadIdx.x; e < nn; e += T) {
            blk[bp + e] = (TM)0;
            if (a.SLlo) a.SLlo[os + e] = 0.f;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nn; e += T) {
        const int i = e / nx, j = e - i * nx;
        if (i < j) {
            const double s = 0.5 * (Dm[i * nx + j] + Dm[j * nx + i]);
            Dm[i * nx + j] = s;
            Dm[j * nx + i] = s;
        }
    }
    __syncthreads();
    store_split_packed(blk, a.SDlo ? a.SDlo + od : nullptr, Dm, nx);
    __syncthreads();
    const bool ok = team_spd_inverse(Dm, col, nx);
    store_split_packed(blk + bp + bs, (float *)nullptr, Dm, nx);
    if (!ok && threadIdx.x == 0) atomicOr(a.status + p, kNotSpd);
}

// Phase 3 (explicit stair blocks, built only when asked for): the
// sub-diagonal blocks of Phi^-1 in TM, from the stored D^-1 and L (with
// L's FP32 remainder), multiplied in FP64.
template <typename TM>
__global__ __launch_bounds__(T) void k_build_phi(BuildArgs a) {
    extern __shared__ double sm[];
    int p, k;
    knot_of(a, p, k);
    const int nx = a.nx[p];
    const int nn = nx * nx, bs = block_stride(nx, sizeof(TM)), bp = packed_stride(nx, sizeof(TM));
    const int ks = 2 * bp + bs;
    const int64_t os = a.off_blk[p] + (int64_t)k * bs;
    const TM *blk = (const TM *)a.B3 + a.off_b3[p] + (int64_t)k * ks;  // D_k (packed), L_k, D_k^-1 (packed)
    double *Di = sm, *Lm = Di + nn, *Dp = Lm + nn, *T1 = Dp + nn, *T2 = T1 + nn;
    if (k == 0 || (a.pc != 1 && a.pc != 2)) {  // block-diagonal preconditioners (and k = 0)
        for (int e = threadIdx.x; e < nn; e += T) ((TM *)a.PM)[os + e] = (TM)0;
        return;
    }
    team_load_packed(Di, blk + bp + bs, nx);                                // D_k^-1
    team_load_lo(Lm, blk + bp, a.SLlo ? a.SLlo + os : nullptr, nn, -1.0);  // +phi = -L_k
    team_load_packed(Dp, blk - ks + bp + bs, nx);                           // D_{k-1}^-1
    __syncthreads();
    team_gemm(nx, nx, nx, Di, Lm, false, T1);
    team_gemm(nx, nx, nx, T1, Dp, false, T2);
    // -D_k^-1 L_k D_{k-1}^-1 = +D_k^-1 phi D_{k-1}^-1 ; additive stair halves it
    store_split((TM *)a.PM + os, (float *)nullptr, T2, nn, a.pc == 1 ? 0.5 : 1.0);
}

// Export kernel: one workgroup per knot copies one block kind from the
// stored layout to the caller's full FP64 blocks (which: 0 D, 1 L, 2 D^-1,
// 3 explicit stair blocks), adding the FP32 remainder lo when given.
template <typename TM>
__global__ void k_export(BuildArgs a, int which, const TM *hi, const float *lo, double *dst) {
    int p, k;
    knot_of(a, p, k);
    const int nx = a.nx[p], nn = nx * nx, bs = block_stride(nx, sizeof(TM)), bp = packed_stride(nx, sizeof(TM));
    const int64_t o = a.off_nn[p] + (int64_t)k * nn;
    const int64_t kb = a.off_b3[p] + (int64_t)k * (2 * bp + bs);
    for (int e = threadIdx.x; e < nn; e += T) {
        const int r = e / nx, c = e - r * nx;
        double v;
        if (which == 0) {
            const int pi = packed_index(r, c, nx);
            v = (double)hi[kb + pi] + (lo ? (double)lo[a.off_pk[p] + (int64_t)k * bp + pi] : 0.0);
        } else if (which == 1) {
            v = (double)hi[kb + bp + e] + (lo ? (double)lo[a.off_blk[p] + (int64_t)k * bs + e] : 0.0);
        } else if (which == 2) {
            v = (double)hi[kb + bp + bs + packed_index(r, c, nx)];
        } else {
            v = (double)hi[a.off_blk[p] + (int64_t)k * bs + e];
        }
        dst[o + e] = v;
    }
}

// D_k^-1 = W_k^T W_k (W_k = C_k^-1, D_k = C_k C_k^T) into the stored D_k^-1
// slot, from the stored W (storage type, block stride bs); one workgroup per
// knot, W_k in LDS in FP64.
template <typename TM>
__global__ void k_dinv_from_w(BuildArgs a) {
    extern __shared__ double sm[];
    int p, k;
    knot_of(a, p, k);
    const int nx = a.nx[p], nn = nx * nx, bs = block_stride(nx, sizeof(TM)), bp = packed_stride(nx, sizeof(TM));
    TM *blk = (TM *)a.B3 + a.off_b3[p] + (int64_t)k * (2 * bp + bs);
    const TM *W = (const TM *)a.Zs + a.off_blk[p] + (int64_t)k * bs;
    for (int e = threadIdx.x; e < nn; e += T) sm[e] = (double)W[e];
    __syncthreads();
    for (int e = threadIdx.x; e < nn; e += T) {
        const int r = e / nx, c = e - r * nx;
        if (r > c) continue;
        double v = 0.0;
        for (int l = 0; l < nx; ++l) v += sm[l * nx + r] * sm[l * nx + c];
        blk[bp + bs + packed_index(r, c, nx)] = (TM)v;
    }
}

// Scalar Jacobi (Eq. (jacobi) with Phi = diag(S)): replace the stored D_k^-1
// of every knot by diag(1 / (D_k)_ii), (D_k)_ii read as stored hi + lo.  One
// workgroup per knot.
template <typename TM>
__global__ void k_jacobi_diag(BuildArgs a) {
    int p, k;
    knot_of(a, p, k);
    const int nx = a.nx[p], bs = block_stride(nx, sizeof(TM)), bp = packed_stride(nx, sizeof(TM));
    TM *blk = (TM *)a.B3 + a.off_b3[p] + (int64_t)k * (2 * bp + bs);
    const float *lo = a.SDlo ? a.SDlo + a.off_pk[p] + (int64_t)k * bp : nullptr;
    for (int e = threadIdx.x; e < nx * nx; e += T) {
        const int r = e / nx, c = e - r * nx;
        if (r > c) continue;
        const int pi = packed_index(r, c, nx);
        double v = 0.0;
        if (r == c) v = 1.0 / ((double)blk[pi] + (lo ? (double)lo[pi] : 0.0));
        blk[bp + bs + pi] = (TM)v;
    }
}

__global__ void k_fill_i32(int32_t *dst, int32_t v, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = v;
}

__global__ void k_fill_f64(double *dst, double v, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = v;
}

// ------------------------------------------------------------- launchers ---

static size_t lds_phase1(int mx) { return sizeof(double) * (mx * mx + mx); }
static size_t lds_phase2(int nx, int nu) { return sizeof(double) * (4 * nx * nx + 2 * nx * nu + nu * nu + nx); }
static size_t lds_phase3(int nx) { return sizeof(double) * 5 * nx * nx; }

hipError_t launch_build(const BuildArgs &a, int64_t knots, int nx_max, int nu_max, bool fp32, hipStream_t s) {
    if (knots == 0) return hipSuccess;
    const dim3 grid((unsigned)knots), block(T);
    const size_t l1 = lds_phase1(a.mx), l2 = lds_phase2(nx_max, nu_max);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_build_inv, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l1)))
        return e;
    hipLaunchKernelGGL(k_build_inv, grid, block, l1, s, a);
    if ((e = hipGetLastError())) return e;
    const void *f2 = fp32 ? (const void *)k_build_S<float> : (const void *)k_build_S<double>;
    if ((e = hipFuncSetAttribute(f2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l2))) return e;
    if (fp32)
        hipLaunchKernelGGL(k_build_S<float>, grid, block, l2, s, a);
    else
        hipLaunchKernelGGL(k_build_S<double>, grid, block, l2, s, a);
    return hipGetLastError();
}

hipError_t launch_build_blocks(const BuildArgs &a, const double *D, const double *Lsub, int64_t knots, bool fp32,
                              hipStream_t s) {
    if (knots == 0) return hipSuccess;
    const size_t l1 = lds_phase1(a.mx);
    const void *f = fp32 ? (const void *)k_build_blocks<float> : (const void *)k_build_blocks<double>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l1);
    if (e) return e;
    if (fp32)
        hipLaunchKernelGGL(k_build_blocks<float>, dim3((unsigned)knots), dim3(T), l1, s, a, D, Lsub);
    else
        hipLaunchKernelGGL(k_build_blocks<double>, dim3((unsigned)knots), dim3(T), l1, s, a, D, Lsub);
    return hipGetLastError();
}

hipError_t launch_build_phi(const BuildArgs &a, int64_t knots, int nx_max, bool fp32, hipStream_t s) {
    if (knots == 0) return hipSuccess;
    const size_t l3 = lds_phase3(nx_max);
    const void *f3 = fp32 ? (const void *)k_build_phi<float> : (const void *)k_build_phi<double>;
    hipError_t e = hipFuncSetAttribute(f3, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l3);
    if (e) return e;
    if (fp32)
        hipLaunchKernelGGL(k_build_phi<float>, dim3((unsigned)knots), dim3(T), l3, s, a);
    else
        hipLaunchKernelGGL(k_build_phi<double>, dim3((unsigned)knots), dim3(T), l3, s, a);
    return hipGetLastError();
}

hipError_t launch_export(const BuildArgs &a, int which, const void *hi, const float *lo, bool fp32, double *dst,
                         int64_t knots, hipStream_t s) {
    if (knots == 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k_export<float>, dim3((unsigned)knots), dim3(T), 0, s, a, which, (const float *)hi, lo, dst);
    else
        hipLaunchKernelGGL(k_export<double>, dim3((unsigned)knots), dim3(T), 0, s, a, which, (const double *)hi, lo,
                           dst);
    return hipGetLastError();
}

hipError_t launch_dinv_from_w(const BuildArgs &a, int64_t knots, int nx_max, bool fp32, hipStream_t s) {
    if (knots == 0) return hipSuccess;
    const size_t l = sizeof(double) * nx_max * nx_max;
    if (fp32)
        hipLaunchKernelGGL(k_dinv_from_w<float>, dim3((unsigned)knots), dim3(T), l, s, a);
    else
        hipLaunchKernelGGL(k_dinv_from_w<double>, dim3((unsigned)knots), dim3(T), l, s, a);
    return hipGetLastError();
}

hipError_t launch_jacobi_diag(const BuildArgs &a, int64_t knots, bool fp32, hipStream_t s) {
    if (knots == 0) return hipSuccess;
    if (fp32)
        hipLaunchKernelGGL(k_jacobi_diag<float>, dim3((unsigned)knots), dim3(T), 0, s, a);
    else
        hipLaunchKernelGGL(k_jacobi_diag<double>, dim3((unsigned)knots), dim3(T), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *dst, int32_t v, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, s, dst, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *dst, double v, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks), dim3(256), 0, s, dst, v, n);
    return hipGetLastError();
}

}  // namespace ssp
