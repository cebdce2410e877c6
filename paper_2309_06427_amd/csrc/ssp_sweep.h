// Chunked block-tridiagonal product staged through LDS (one workgroup).
#pragma once

#include "ssp_device.h"

namespace ssp {

// Stored blocks of one problem are nx*nx elements at a stride of bs elements
// (nx*nx rounded up to 16 bytes) so that every block starts 16-byte aligned.
__host__ __device__ inline int block_stride(int nx, int elem_bytes) {
    const int v = 16 / elem_bytes;
    return (nx * nx + v - 1) / v * v;
}

// The symmetric blocks D_k and D_k^-1 are stored packed: the upper triangle
// row by row, entry (r, c) with r <= c at packed_row(r, nx) + c, padded to
// 16 bytes.
__host__ __device__ constexpr int packed_row(int r, int nx) { return r * nx - r * (r + 1) / 2; }
__host__ __device__ inline int packed_stride(int nx, int elem_bytes) {
    const int v = 16 / elem_bytes;
    return (nx * (nx + 1) / 2 + v - 1) / v * v;
}
// packed index of entry (i, j) of a symmetric block
__host__ __device__ inline int packed_index(int i, int j, int nx) {
    return i <= j ? packed_row(i, nx) + j : packed_row(j, nx) + i;
}
// One knot of the solve array: D_k (packed), L_k (full), D_k^-1 (packed).
__host__ __device__ inline int knot_stride(int nx, int elem_bytes) {
    return 2 * packed_stride(nx, elem_bytes) + block_stride(nx, elem_bytes);
}

// Staging geometry of one sweep.  Rows of a staged block are padded to
// nx + 1 elements (odd for even nx) so that row-wise LDS reads by
// consecutive lanes fall in distinct banks.
struct Geo {
    int nx, ldx, blk, nn, bs, C;
    uint64_t mg, mgb, mgn;  // division magics for nx, bs and nx * nx
};

template <typename TS>
__device__ __forceinline__ Geo make_geo(int nx, int bs, bool has_sub, int lds_bytes, int block) {
    Geo g;
    g.nx = nx;
    g.ldx = nx + 1;
    g.blk = nx * g.ldx;
    g.nn = nx * nx;
    g.bs = bs;
    g.mg = div_magic(nx);
    g.mgb = div_magic(bs);
    g.mgn = div_magic(nx * nx);
    const int per_knot = (has_sub ? 2 : 1) * g.blk + nx;
    const int fixed = (has_sub ? g.blk : 0) + 2 * nx;
    int C = block / nx;
    const int Cl = (lds_bytes / (int)sizeof(TS) - fixed) / per_knot;
    if (Cl < C) C = Cl;
    g.C = C < 1 ? 1 : C;
    return g;
}

// Bytes of LDS bt_sweep needs for one knot per chunk in element type TS.
inline int bt_sweep_min_lds(int nx, bool has_sub, int elem_bytes) {
    const int blk = nx * (nx + 1);
    return elem_bytes * ((has_sub ? 2 : 1) * blk + nx + (has_sub ? blk : 0) + 2 * nx);
}

// Copy the blocks [k0, k0 + kc) of a stored array (block k at src + k * ks,
// its FP32 remainder at lo + k * los) into LDS rows padded to ldx.  packed:
// the stored blocks are symmetric and packed (upper triangle) and are
// unpacked to full rows here.
template <typename TS, typename TM, int BLOCK>
__device__ __forceinline__ void stage_blocks(TS *dst, const TM *__restrict__ src, int ks,
                                             const float *__restrict__ lo, int los, bool packed, int k0, int kc,
                                             const Geo &g) {
    if (!packed) {
        const int cnt = kc * g.bs;
        for (int e = threadIdx.x; e < cnt; e += BLOCK) {
            const int kk = fast_div(e, g.mgb), f = e - kk * g.bs;
            if (f < g.nn) {
                TS v = (TS)src[(int64_t)(k0 + kk) * ks + f];
                if (lo) v += (TS)lo[(int64_t)(k0 + kk) * los + f];
                dst[kk * g.blk + f + fast_div(f, g.mg)] = v;
            }
        }
    } else {
        const int cnt = kc * g.nn;
        for (int e = threadIdx.x; e < cnt; e += BLOCK) {
            const int kk = fast_div(e, g.mgn), f = e - kk * g.nn;
            const int r = fast_div(f, g.mg), c = f - r * g.nx;
            const int pi = packed_index(r, c, g.nx);
            TS v = (TS)src[(int64_t)(k0 + kk) * ks + pi];
            if (lo) v += (TS)lo[(int64_t)(k0 + kk) * los + pi];
            dst[kk * g.blk + r * g.ldx + c] = v;
        }
    }
}

// sum_j a[j * stride] * x[j] over n terms (n = NX when it is a compile-time
// constant), four partial sums so that the LDS reads are issued together.
template <int NX, typename T>
__device__ __forceinline__ T strided_dot(const T *__restrict__ a, int stride, const T *__restrict__ x, int nrt) {
    const int n = NX > 0 ? NX : nrt;
    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
    int j = 0;
#pragma unroll 2
    for (; j + 4 <= n; j += 4) {
        a0 += a[(j + 0) * stride] * x[j + 0];
        a1 += a[(j + 1) * stride] * x[j + 1];
        a2 += a[(j + 2) * stride] * x[j + 2];
        a3 += a[(j + 3) * stride] * x[j + 3];
    }
#pragma unroll
    for (; j < n; ++j) a0 += a[j * stride] * x[j];
    return (a0 + a1) + (a2 + a3);
}

// One block-tridiagonal product over a problem of N knots,
//   y_k = Dg_k x_k + Sb_k x_{k-1} + Sb_{k+1}^T x_{k+1},
// with Dg symmetric and stored packed.  Dg, Sb: stored blocks at knot
// strides dks, sks (Sb[0] ignored); Dlo / Slo: optional FP32 remainders
// (strides dlos, bs) added while staging.  xval(row) gives the input
// vector (it may be called for halo rows of other threads); epi(row, y, x) is
// called once per row by the row's owner.
// NX: compile-time state size (0 = runtime g.nx).
template <typename TS, typename TM, int BLOCK, int NX, typename XF, typename EF>
__device__ __forceinline__ void bt_sweep(int N, const Geo &g, const TM *__restrict__ Dg, int dks,
                                         const float *__restrict__ Dlo, int dlos, const TM *__restrict__ Sb,
                                         int sks, const float *__restrict__ Slo, bool has_sub, TS *smem,
                                         XF &&xval, EF &&epi) {
    const int tid = threadIdx.x;
    const int nx = NX > 0 ? NX : g.nx, ldx = nx + 1, blk = nx * ldx, C = g.C;
    TS *Ds = smem;
    TS *Ss = Ds + C * blk;
    TS *xs = Ss + (has_sub ? (C + 1) * blk : 0);
    for (int k0 = 0; k0 < N; k0 += C) {
        const int kc = min(C, N - k0);
        __syncthreads();
        stage_blocks<TS, TM, BLOCK>(Ds, Dg, dks, Dlo, dlos, true, k0, kc, g);
        if (has_sub) stage_blocks<TS, TM, BLOCK>(Ss, Sb, sks, Slo, g.bs, false, k0, min(kc + 1, N - k0), g);
        {
            const int cnt = (kc + 2) * nx;
            const int base = (k0 - 1) * nx;
            for (int t = tid; t < cnt; t += BLOCK) {
                const int row = base + t;
                xs[t] = (row >= 0 && row < N * nx) ? xval(row) : TS(0);
            }
        }
        __syncthreads();
        for (int t = tid; t < kc * nx; t += BLOCK) {
            const int kk = NX > 0 ? t / NX : fast_div(t, g.mg), i = t - kk * nx, k = k0 + kk;
            const TS *xk = xs + (kk + 1) * nx;
            TS y = strided_dot<NX>(Ds + kk * blk + i, ldx, xk, nx);  // column i of the symmetric Dg_k
            if (has_sub) {
                if (k > 0) y += strided_dot<NX>(Ss + kk * blk + i * ldx, 1, xs + kk * nx, nx);  // row i of Sb_k
                if (k + 1 < N)
                    y += strided_dot<NX>(Ss + (kk + 1) * blk + i, ldx, xs + (kk + 2) * nx, nx);  // col i of Sb_{k+1}
            }
            epi(k * nx + i, y, xk[i]);
        }
    }
}

}  // namespace ssp
