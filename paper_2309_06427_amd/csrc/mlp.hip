// Learned per-knot warm start: a network with two GELU hidden layers maps
// each knot's stored blocks D_k, L_k (Sec. II-A, Eq. (schur)) and its slice of
// gamma to a guess of that knot's part of lambda.  Inference and training
// (forward, residual loss, backward, Adam) run in these kernels.
//
// Every product is an FP32 GEMM on the matrix cores
// (v_mfma_f32_16x16x4_f32): 64 x 64 output tiles per 256-thread workgroup,
// each wave a 32 x 32 quarter as 2 x 2 MFMA tiles, K staged through LDS 16 at
// a time.  Operand loaders read the network inputs straight from the stored
// blocks (no feature matrix is materialised) and the epilogues fuse bias,
// GELU and its derivative.  Weight gradients reduce over the knots with a
// fixed K split and a fixed-order sum, so training steps are reproducible.
#include <math.h>

#include "ssp_device.h"
#include "ssp_mlp.h"
#include "ssp_sweep.h"

namespace ssp {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, GT = 256, PADL = 4;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// ---------------------------------------------------------------- loaders ---
// A loader returns element (m, k) of op(A) (0 outside M x K); kFast tells the
// tile loop to walk k fastest (row-major A) or m fastest (column access).

struct RowA {  // A(m, k) = p[m * ld + k]
    static constexpr bool kFast = true;
    const float *p;
    int ld, M, K;
    __device__ float operator()(int m, int k) const { return (m < M && k < K) ? p[(int64_t)m * ld + k] : 0.f; }
};

struct ColA {  // A(m, k) = p[k * ld + m]
    static constexpr bool kFast = false;
    const float *p;
    int ld, M, K;
    __device__ float operator()(int m, int k) const { return (m < M && k < K) ? p[(int64_t)k * ld + m] : 0.f; }
};

struct RowB {  // B(k, n) = p[k * ld + n]
    static constexpr bool kFast = false;
    const float *p;
    int ld, K, N;
    __device__ float operator()(int k, int n) const { return (k < K && n < N) ? p[(int64_t)k * ld + n] : 0.f; }
};

struct ColB {  // B(k, n) = p[n * ld + k]
    static constexpr bool kFast = true;
    const float *p;
    int ld, K, N;
    __device__ float operator()(int k, int n) const { return (k < K && n < N) ? p[(int64_t)n * ld + k] : 0.f; }
};

// Raw input f of knot m: vec D_k (row-major, read from the packed upper
// triangle), then vec L_k (zero at the first knot), then gamma_k.
template <typename TM>
__device__ __forceinline__ float raw_feature(const FeatSrc &s, const KnotInfo &q, int f) {
    const int nn = s.nx * s.nx;
    const TM *B3 = (const TM *)s.B3;
    if (f < nn) {
        const int r = f / s.nx, c = f - r * s.nx;
        return (float)B3[q.blk + packed_index(r, c, s.nx)];
    }
    if (f < 2 * nn) return q.first ? 0.f : (float)B3[q.blk + s.lofs + (f - nn)];
    return (float)s.gamma[q.vec + (f - 2 * nn)];
}

template <typename TM>
struct FeatA {  // A(m, f) = standardised input f of knot m
    static constexpr bool kFast = true;
    FeatSrc s;
    const float *mu, *isd;
    int K;
    __device__ float operator()(int m, int f) const {
        if (m >= s.M || f >= K) return 0.f;
        return (raw_feature<TM>(s, s.ki[m], f) - mu[f]) * isd[f];
    }
};

template <typename TM>
struct FeatAT {  // A(f, m) = standardised input f of knot m (transposed features)
    static constexpr bool kFast = false;
    FeatA<TM> a;
    __device__ float operator()(int f, int m) const { return a(m, f); }
};

// -------------------------------------------------------------- epilogues ---

struct EpStore {  // C[z][m][n] = v  (z: K-split index)
    float *c;
    int ld;
    int64_t zstride;
    __device__ void operator()(int m, int n, int z, float v) const { c[z * zstride + (int64_t)m * ld + n] = v; }
};

struct EpBiasGelu {
    const float *b;
    float *z, *h;
    int ld;
    __device__ void operator()(int m, int n, int, float v) const {
        const float zz = v + b[n];
        if (z) z[(int64_t)m * ld + n] = zz;
        h[(int64_t)m * ld + n] = gelu(zz);
    }
};

struct EpOut {  // network output (+ lambda0 = y_scale * o at the knot's rows)
    const float *b;
    float *o;
    int ld;
    const KnotInfo *ki;
    double *lam;
    float ys;
    __device__ void operator()(int m, int n, int, float v) const {
        const float oo = v + b[n];
        if (o) o[(int64_t)m * ld + n] = oo;
        if (lam) lam[ki[m].vec + n] = (double)(ys * oo);
    }
};

struct EpGeluBack {  // dZ = v * gelu'(Z)
    const float *z;
    float *dz;
    int ld;
    __device__ void operator()(int m, int n, int, float v) const {
        dz[(int64_t)m * ld + n] = v * gelu_grad(z[(int64_t)m * ld + n]);
    }
};

// ------------------------------------------------------------------- GEMM ---
// C = op(A) op(B) over k in [z * kspl, min(K, (z + 1) * kspl)), z = blockIdx.z.
template <class AL, class BL, class EP>
__global__ __launch_bounds__(GT) void k_gemm(int M, int N, int K, int kspl, AL al, BL bl, EP ep) {
    __shared__ float As[BK][BM + PADL];
    __shared__ float Bs[BK][BN + PADL];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN, z = blockIdx.z;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int kb = z * kspl, ke = min(K, kb + kspl);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < (BM * BK) / GT; ++e) {
            const int idx = t + GT * e;
            int mm, kk;
            if constexpr (AL::kFast) {
                mm = idx / BK;
                kk = idx % BK;
            } else {
                kk = idx / BM;
                mm = idx % BM;
            }
            As[kk][mm] = (k0 + kk < ke) ? al(m0 + mm, k0 + kk) : 0.f;
            int nn, kk2;
            if constexpr (BL::kFast) {
                nn = idx / BK;
                kk2 = idx % BK;
            } else {
                kk2 = idx / BN;
                nn = idx % BN;
            }
            Bs[kk2][nn] = (k0 + kk2 < ke) ? bl(k0 + kk2, n0 + nn) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int sub = 0; sub < BK / 4; ++sub) {
            const int kr = 4 * sub + (lane >> 4), c = lane & 15;
            const float a0 = As[kr][wm + c], a1 = As[kr][wm + 16 + c];
            const float b0 = Bs[kr][wn + c], b1 = Bs[kr][wn + 16 + c];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    // lane l holds rows 4 (l / 16) + r, column l % 16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r, n = n0 + wn + 16 * j + (lane & 15);
                if (m < M && n < N) ep(m, n, z, acc[i][j][r]);
            }
}

template <class AL, class BL, class EP>
hipError_t gemm(int M, int N, int K, int splits, const AL &al, const BL &bl, const EP &ep, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (splits < 1) splits = 1;
    int kspl = (K + splits - 1) / splits;
    kspl = (kspl + BK - 1) / BK * BK;
    if (kspl < BK) kspl = BK;
    const int nz = K > 0 ? (K + kspl - 1) / kspl : 1;
    hipLaunchKernelGGL((k_gemm<AL, BL, EP>), dim3((M + BM - 1) / BM, (N + BN - 1) / BN, nz), dim3(GT), 0, s, M, N, K,
                       kspl, al, bl, ep);
    return hipGetLastError();
}

// First layer, z = standardised inputs x W1 + b1, h = gelu(z), for 64 knots
// by up to 128 hidden units per workgroup (4 waves, each 16 knots x 128
// units as 8 MFMA tiles), K in steps of 32 through two LDS buffers.  A
// thread gathers eight consecutive raw inputs of one knot per step through a
// table of input offsets built in LDS at the start (D_k from its packed upper
// triangle, L_k, gamma_k); the step's 32 means and inverse deviations go to
// LDS beside the tile and standardise each A operand as it is read (features
// past nin get inverse deviation 0, so they add nothing; rows past M only
// feed outputs that are not stored).  The next step's loads are issued
// before this step's products, at clamped addresses and without branches,
// so that no wait separates them.
constexpr int kL1N = 128, kL1K = 32;
constexpr int kFeatL = 1, kFeatG = 2;  // input kinds in the table's top bits (0: D_k)
constexpr int kL1MaxIn = 3136;         // table entries (the static tiles leave room for these)

template <typename TM>
__global__ __launch_bounds__(GT) void k_layer1(FeatSrc s, const float *__restrict__ W1, const float *__restrict__ b1,
                                               const float *__restrict__ mu, const float *__restrict__ isd, int nin,
                                               int H, float *__restrict__ Z, float *__restrict__ Hout) {
    __shared__ float As[2][kL1K][BM + PADL];
    __shared__ float Bs[2][kL1K][kL1N + PADL];
    __shared__ float Ms[2][2][kL1K];  // mean, inverse deviation of the step's inputs
    __shared__ int foff[kL1MaxIn];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * kL1N;
    const int nx = s.nx, nn = nx * nx;
    for (int f = t; f < nin; f += GT) {
        int v;
        if (f < nn) {
            const int r = f / nx, c = f - r * nx;
            v = packed_index(r, c, nx);
        } else if (f < 2 * nn) {
            v = (kFeatL << 30) | (s.lofs + f - nn);
        } else {
            v = (kFeatG << 30) | (f - 2 * nn);
        }
        foff[f] = v;
    }
    // this thread's A row and its eight inputs of each step
    const int am = t >> 2, aq = (t & 3) * 8;
    const KnotInfo q = s.ki[min(m0 + am, s.M - 1)];  // rows past M: a valid knot (outputs not stored)
    const TM *src = (const TM *)s.B3 + q.blk;
    const double *gsrc = s.gamma + q.vec;
    // B tile: row t / 8 of the step, sixteen columns from 16 (t % 8); the
    // first 64 threads also fetch the step's scaling (t < 32 means, else
    // inverse deviations)
    const int bk = t >> 3, bn = (t & 7) * 16;
    const int nlast = nin - 1;
    f32x4 acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the next step's raw loads and their 0/1 weights: combined only when
    // they are stored, so that the loads stay in flight over this step's
    // products.  Both input loads are kept (weighted rather than selected) so
    // that the compiler issues them unconditionally; they read finite inputs
    // at valid addresses.
    TM rd[8];
    double rg[8];
    float wd[8], wg[8], wb[4], rs, ws;
    f32x4 rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int fc = min(k0 + aq + j, nlast);
            const int e = foff[fc], kind = (int)((unsigned)e >> 30), o = e & 0x3fffffff;
            rd[j] = src[kind == kFeatG ? 0 : o];
            rg[j] = gsrc[kind == kFeatG ? o : 0];
            wd[j] = (kind == kFeatG || (kind == kFeatL && q.first)) ? 0.f : 1.f;
            wg[j] = kind == kFeatG ? 1.f : 0.f;
        }
        const int kr = k0 + bk;
        const float *wrow = W1 + (int64_t)min(kr, nlast) * H;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int n = n0 + bn + 4 * c;
            rb[c] = *(const f32x4 *)(wrow + min(n, H - 4));
            wb[c] = (kr < nin && n < H) ? 1.f : 0.f;
        }
        const int fs = k0 + (t & 31);
        rs = (t < 32 ? mu : isd)[min(fs, nlast)];
        ws = (t < 32 || fs < nin) ? 1.f : 0.f;
    };
    __syncthreads();  // the input table is complete
    load(0);
    for (int k0 = 0, buf = 0; k0 < nin; k0 += kL1K, buf ^= 1) {
#pragma unroll
        for (int j = 0; j < 8; ++j) As[buf][aq + j][am] = (float)rd[j] * wd[j] + (float)rg[j] * wg[j];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) Bs[buf][bk][bn + 4 * c + r] = rb[c][r] * wb[c];
        if (t < 64) Ms[buf][t >> 5][t & 31] = rs * ws;
        __syncthreads();  // this buffer is full; the other one's readers are done (they passed this barrier)
        load(k0 + kL1K);  // past nin: clamped addresses, zero scaling
#pragma unroll
        for (int sub = 0; sub < kL1K / 4; ++sub) {
            const int kr = 4 * sub + (lane >> 4), c = lane & 15;
            const float a = (As[buf][kr][16 * w + c] - Ms[buf][0][kr]) * Ms[buf][1][kr];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Bs[buf][kr][16 * j + c], acc[j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = m0 + 16 * w + 4 * (lane >> 4) + r, n = n0 + 16 * j + (lane & 15);
            if (m < s.M && n < H) {
                const float z = acc[j][r] + b1[n];
                if (Z) Z[(int64_t)m * H + n] = z;
                Hout[(int64_t)m * H + n] = gelu(z);
            }
        }
}

// number of K splits gemm() will use (the partial buffer holds that many)
int split_count(int K, int splits) {
    if (splits < 1) splits = 1;
    int kspl = (K + splits - 1) / splits;
    kspl = (kspl + BK - 1) / BK * BK;
    if (kspl < BK) kspl = BK;
    return K > 0 ? (K + kspl - 1) / kspl : 1;
}

// ------------------------------------------------------------ small kernels ---

__global__ void k_knot_info(const int32_t *knot_prob, const int64_t *koff, const int32_t *N, const int64_t *off_b3,
                            const int64_t *off_v, const int32_t *list, int64_t g0, int M, int nx, int ks,
                            KnotInfo *out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int64_t g = list ? (int64_t)list[m] : g0 + m;
    const int p = knot_prob[g];
    const int k = (int)(g - koff[p]);
    KnotInfo q;
    q.blk = off_b3[p] + (int64_t)k * ks;
    q.vec = off_v[p] + (int64_t)k * nx;
    q.first = k == 0;
    q.last = k == N[p] - 1;
    out[m] = q;
}

// column sums of a row-major M x n matrix into out[0..n) (fixed order)
__global__ __launch_bounds__(256) void k_colsum(const float *x, int M, int n, float *out) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6, col = blockIdx.x * 64 + c;
    float s = 0.f;
    if (col < n)
        for (int m = r; m < M; m += 4) s += x[(int64_t)m * n + col];
    red[r][c] = s;
    __syncthreads();
    if (r == 0 && col < n) out[col] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

// out[i] = sum_z part[z * cnt + i] (fixed order)
__global__ void k_sum_splits(const float *part, int nz, int64_t cnt, float *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < nz; ++z) s += part[z * cnt + i];
        out[i] = s;
    }
}

// Partial sums (x - shift) and (x - shift)^2 over knots for 64 features per
// block column; blockIdx.y strides the knots.  Features f < nin are network
// inputs, f >= nin are label entries lam[vec + f - nin].
template <typename TM>
__global__ __launch_bounds__(256) void k_stats_part(FeatSrc s, const double *lam, int nin, int nf, double *part) {
    __shared__ double r1[4][64], r2[4][64];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6, f = blockIdx.x * 64 + c;
    double a = 0.0, b = 0.0;
    if (f < nf) {
        auto val = [&](int m) -> double {
            const KnotInfo q = s.ki[m];
            return f < nin ? (double)raw_feature<TM>(s, q, f) : lam[q.vec + (f - nin)];
        };
        const double shift = val(0);
        for (int m = blockIdx.y * 4 + r; m < s.M; m += 4 * gridDim.y) {
            const double d = val(m) - shift;
            a += d;
            b += d * d;
        }
    }
    r1[r][c] = a;
    r2[r][c] = b;
    __syncthreads();
    if (r == 0 && f < nf) {
        part[(int64_t)blockIdx.y * 2 * nf + f] = (r1[0][c] + r1[1][c]) + (r1[2][c] + r1[3][c]);
        part[(int64_t)blockIdx.y * 2 * nf + nf + f] = (r2[0][c] + r2[1][c]) + (r2[2][c] + r2[3][c]);
    }
}

template <typename TM>
__global__ __launch_bounds__(256) void k_stats_final(FeatSrc s, const double *lam, int nin, int nf, int ny,
                                                     const double *part, float *mu, float *isd, float *ys) {
    __shared__ double red[256];
    double lab = 0.0;  // this thread's share of sum over label features of E[x^2]
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
        double a = 0.0, b = 0.0;
        for (int y = 0; y < ny; ++y) {
            a += part[(int64_t)y * 2 * nf + f];
            b += part[(int64_t)y * 2 * nf + nf + f];
        }
        const KnotInfo q = s.ki[0];
        const double shift = f < nin ? (double)raw_feature<TM>(s, q, f) : lam[q.vec + (f - nin)];
        const double mean_d = a / s.M;
        double var = b / s.M - mean_d * mean_d;
        if (var < 0.0) var = 0.0;
        const double mean = shift + mean_d;
        if (f < nin) {
            mu[f] = (float)mean;
            const double sd = sqrt(var);
            isd[f] = (float)(1.0 / (sd > 1e-6 ? sd : 1e-6));
        } else {
            lab += var + mean * mean;
        }
    }
    red[threadIdx.x] = lab;
    __syncthreads();
    if (threadIdx.x == 0 && nf > nin) {
        double t = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += red[i];
        *ys = (float)sqrt(t / (nf - nin));
    }
}

// E = ys * O - lam*
__global__ void k_err(const KnotInfo *ki, int M, int nx, const float *O, float ys, const double *lam, float *E) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * nx) return;
    const int m = (int)(e / nx), i = (int)(e - (int64_t)m * nx);
    E[e] = ys * O[e] - (float)lam[ki[m].vec + i];
}

// Y = scale * S X over whole problems (rows of knot m in X, Y at m * nx);
// part[block] = sum of Y^2 over the block (when part != null).
template <typename TM>
__global__ __launch_bounds__(256) void k_smul(FeatSrc s, const float *X, float scale, float *Y, double *part) {
    __shared__ double red[4];
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int nx = s.nx;
    double sq = 0.0;
    if (e < (int64_t)s.M * nx) {
        const int m = (int)(e / nx), i = (int)(e - (int64_t)m * nx);
        const KnotInfo q = s.ki[m];
        const TM *B3 = (const TM *)s.B3;
        const TM *Dp = B3 + q.blk;  // D_k packed
        const float *x = X + (int64_t)m * nx;
        float y = 0.f;
        for (int j = 0; j < nx; ++j) y += (float)Dp[packed_index(i, j, nx)] * x[j];
        if (!q.first) {
            const TM *Lr = B3 + q.blk + s.lofs + i * nx;  // row i of L_k
            for (int j = 0; j < nx; ++j) y += (float)Lr[j] * x[j - nx];
        }
        if (!q.last) {
            const TM *Ln = B3 + s.ki[m + 1].blk + s.lofs;  // column i of L_{k+1}
            for (int j = 0; j < nx; ++j) y += (float)Ln[j * nx + i] * x[nx + j];
        }
        y *= scale;
        Y[e] = y;
        sq = (double)y * y;
    }
    if (part) {
        sq = wave_sum(sq);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
        __syncthreads();
        if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

__global__ __launch_bounds__(256) void k_loss_final(const double *part, int n, double scale, double *loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 256; ++i) t += red[i];
        *loss = t * scale;
    }
}

__global__ void k_adam(float *theta, const float *grad, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float g = grad[i];
        const float mi = b1 * m[i] + (1.f - b1) * g;
        const float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

int grid_for(int64_t n, int block) {
    const int64_t g = (n + block - 1) / block;
    return (int)(g < 65535 ? (g > 0 ? g : 1) : 65535);
}

template <typename TM>
hipError_t forward_t(const FeatSrc &f, const NetView &w, const float *mu, const float *isd, float ys, float *Z1,
                     float *H1, float *Z2, float *H2, float *O, double *lam, hipStream_t s) {
    hipError_t e;
    if (w.nin <= kL1MaxIn && w.H % 4 == 0) {
        hipLaunchKernelGGL(k_layer1<TM>, dim3((f.M + BM - 1) / BM, (w.H + kL1N - 1) / kL1N), dim3(GT), 0, s, f, w.W1,
                           w.b1, mu, isd, w.nin, w.H, Z1, H1);
        if ((e = hipGetLastError())) return e;
    } else {
        FeatA<TM> fa{f, mu, isd, w.nin};
        if ((e = gemm(f.M, w.H, w.nin, 1, fa, RowB{w.W1, w.H, w.nin, w.H}, EpBiasGelu{w.b1, Z1, H1, w.H}, s)))
            return e;
    }
    if ((e = gemm(f.M, w.H, w.H, 1, RowA{H1, w.H, f.M, w.H}, RowB{w.W2, w.H, w.H, w.H}, EpBiasGelu{w.b2, Z2, H2, w.H},
                  s)))
        return e;
    return gemm(f.M, w.nx, w.H, 1, RowA{H2, w.H, f.M, w.H}, RowB{w.W3, w.nx, w.H, w.nx},
                EpOut{w.b3, O, w.nx, f.ki, lam, ys}, s);
}

// weight gradient op(A)^T-style product with a K split over the knots,
// summed into dst
template <class AL, class BL>
hipError_t wgrad(int M, int N, int K, const AL &al, const BL &bl, float *split, int splits, float *dst,
                 hipStream_t s) {
    const int nz = split_count(K, splits);
    hipError_t e = gemm(M, N, K, splits, al, bl, EpStore{split, N, (int64_t)M * N}, s);
    if (e) return e;
    hipLaunchKernelGGL(k_sum_splits, dim3(grid_for((int64_t)M * N, 256)), dim3(256), 0, s, split, nz,
                       (int64_t)M * N, dst);
    return hipGetLastError();
}

template <typename TM>
hipError_t backward_t(const FeatSrc &f, const NetView &w, const float *mu, const float *isd, const float *Z1,
                      const float *H1, const float *Z2, const float *H2, const float *dO, float *dZ2, float *dZ1,
                      float *grad, float *split, int splits, hipStream_t s) {
    const int M = f.M, H = w.H, nx = w.nx, nin = w.nin;
    float *gW1 = grad, *gb1 = gW1 + (int64_t)nin * H, *gW2 = gb1 + H, *gb2 = gW2 + (int64_t)H * H, *gW3 = gb2 + H,
          *gb3 = gW3 + (int64_t)H * nx;
    hipError_t e;
    // layer 3: dW3 = H2^T dO, db3 = colsum dO, dZ2 = (dO W3^T) * gelu'(Z2)
    if ((e = wgrad(H, nx, M, ColA{H2, H, H, M}, RowB{dO, nx, M, nx}, split, splits, gW3, s))) return e;
    hipLaunchKernelGGL(k_colsum, dim3((nx + 63) / 64), dim3(256), 0, s, dO, M, nx, gb3);
    if ((e = gemm(M, H, nx, 1, RowA{dO, nx, M, nx}, ColB{w.W3, nx, nx, H}, EpGeluBack{Z2, dZ2, H}, s))) return e;
    // layer 2
    if ((e = wgrad(H, H, M, ColA{H1, H, H, M}, RowB{dZ2, H, M, H}, split, splits, gW2, s))) return e;
    hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(256), 0, s, dZ2, M, H, gb2);
    if ((e = gemm(M, H, H, 1, RowA{dZ2, H, M, H}, ColB{w.W2, H, H, H}, EpGeluBack{Z1, dZ1, H}, s))) return e;
    // layer 1 (inputs re-read from the stored blocks)
    FeatAT<TM> ft{FeatA<TM>{f, mu, isd, nin}};
    if ((e = wgrad(nin, H, M, ft, RowB{dZ1, H, M, H}, split, splits, gW1, s))) return e;
    hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(256), 0, s, dZ1, M, H, gb1);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_knot_info(const int32_t *knot_prob, const int64_t *koff, const int32_t *N, const int64_t *off_b3,
                            const int64_t *off_v, const int32_t *list, int64_t g0, int M, int nx, int ks,
                            KnotInfo *out, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_knot_info, dim3((M + 255) / 256), dim3(256), 0, s, knot_prob, koff, N, off_b3, off_v, list,
                       g0, M, nx, ks, out);
    return hipGetLastError();
}

hipError_t launch_feature_stats(const FeatSrc &f, const double *lam, float *mu, float *inv_sd, float *y_scale,
                                double *part, hipStream_t s) {
    if (f.M <= 0) return hipErrorInvalidValue;
    const int nin = 2 * f.nx * f.nx + f.nx, nf = nin + (lam ? f.nx : 0), ny = 64;
    const dim3 g1((nf + 63) / 64, ny);
    if (f.fp32) {
        hipLaunchKernelGGL(k_stats_part<float>, g1, dim3(256), 0, s, f, lam, nin, nf, part);
        hipLaunchKernelGGL(k_stats_final<float>, dim3(1), dim3(256), 0, s, f, lam, nin, nf, ny, part, mu, inv_sd,
                           y_scale);
    } else {
        hipLaunchKernelGGL(k_stats_part<double>, g1, dim3(256), 0, s, f, lam, nin, nf, part);
        hipLaunchKernelGGL(k_stats_final<double>, dim3(1), dim3(256), 0, s, f, lam, nin, nf, ny, part, mu, inv_sd,
                           y_scale);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const FeatSrc &f, const NetView &w, const float *mu, const float *inv_sd, float y_scale,
                              float *Z1, float *H1, float *Z2, float *H2, float *O, double *lambda, hipStream_t s) {
    if (f.M <= 0) return hipSuccess;
    return f.fp32 ? forward_t<float>(f, w, mu, inv_sd, y_scale, Z1, H1, Z2, H2, O, lambda, s)
                  : forward_t<double>(f, w, mu, inv_sd, y_scale, Z1, H1, Z2, H2, O, lambda, s);
}

hipError_t launch_mlp_loss(const FeatSrc &f, const float *O, float y_scale, const double *lam_star, int nprob,
                           float *E, float *R, float *dO, double *part, double *loss, hipStream_t s) {
    if (f.M <= 0 || nprob <= 0) return hipErrorInvalidValue;
    const int64_t n = (int64_t)f.M * f.nx;
    const int g = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_err, dim3(g), dim3(256), 0, s, f.ki, f.M, f.nx, O, y_scale, lam_star, E);
    if (f.fp32) {
        hipLaunchKernelGGL(k_smul<float>, dim3(g), dim3(256), 0, s, f, E, 1.0f, R, part);
        hipLaunchKernelGGL(k_smul<float>, dim3(g), dim3(256), 0, s, f, R, y_scale * 2.0f / nprob, dO,
                           (double *)nullptr);
    } else {
        hipLaunchKernelGGL(k_smul<double>, dim3(g), dim3(256), 0, s, f, E, 1.0f, R, part);
        hipLaunchKernelGGL(k_smul<double>, dim3(g), dim3(256), 0, s, f, R, y_scale * 2.0f / nprob, dO,
                           (double *)nullptr);
    }
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, part, g, 1.0 / nprob, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const FeatSrc &f, const NetView &w, const float *mu, const float *inv_sd,
                               const float *Z1, const float *H1, const float *Z2, const float *H2, const float *dO,
                               float *dZ2, float *dZ1, float *grad, float *split, int splits, hipStream_t s) {
    if (f.M <= 0) return hipErrorInvalidValue;
    return f.fp32 ? backward_t<float>(f, w, mu, inv_sd, Z1, H1, Z2, H2, dO, dZ2, dZ1, grad, split, splits, s)
                  : backward_t<double>(f, w, mu, inv_sd, Z1, H1, Z2, H2, dO, dZ2, dZ1, grad, split, splits, s);
}

hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int64_t n, float lr, float beta1,
                       float beta2, float eps, float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n, 256)), dim3(256), 0, s, theta, grad, m, v, n, lr, beta1, beta2, eps,
                       bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_gemm_f32(int M, int N, int K, const float *A, int lda, bool ta, const float *B, int ldb, bool tb,
                           float *C, int ldc, hipStream_t s) {
    const EpStore ep{C, ldc, 0};
    if (!ta && !tb) return gemm(M, N, K, 1, RowA{A, lda, M, K}, RowB{B, ldb, K, N}, ep, s);
    if (!ta && tb) return gemm(M, N, K, 1, RowA{A, lda, M, K}, ColB{B, ldb, K, N}, ep, s);
    if (ta && !tb) return gemm(M, N, K, 1, ColA{A, lda, M, K}, RowB{B, ldb, K, N}, ep, s);
    return gemm(M, N, K, 1, ColA{A, lda, M, K}, ColB{B, ldb, K, N}, ep, s);
}

}  // namespace ssp
