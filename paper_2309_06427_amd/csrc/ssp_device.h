// Device-side helpers shared by the library's kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ssp {

constexpr int kWave = 64;

// Per-problem status codes (numerically equal to the public SSP_P_* values).
constexpr int kOk = 0, kNotSpd = 1, kMaxIter = 2, kNonFinite = 3, kBreakdown = 4;
// one inner solve without refinement met the tolerance on its recurrence
// residual but not on the true FP64 residual
constexpr int kInaccurate = 5;
constexpr int kWarmFallback = 8;  // OR-ed flag: the warm start was replaced by zero
constexpr int kPcFallback = 16;   // OR-ed flag: block-Jacobi took over after a float breakdown

// A solve skips a problem only when its incoming status says the build found
// a block that is not positive definite; every other code (an earlier
// solve's iteration limit, breakdown or fallback flags) starts a fresh solve.
__host__ __device__ inline bool build_failed(int st) { return (st & 7) == kNotSpd; }

// A value every lane of the wave holds equally (a workgroup sum, a queue
// position), moved into scalar registers: branches on it are then uniform
// for the compiler, which keeps loops that contain workgroup barriers from
// being restructured around lanes it would otherwise treat as divergent.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Butterfly sum over the 64 lanes of a wavefront.  Every lane ends with the
// same bits: each stage adds the same two operands on both partner lanes.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Workgroup sum in a fixed order (wave butterflies, then waves 0..W-1 in
// sequence), returned to every thread.  `red` holds BLOCK/64 entries of LDS.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
    v = wave_sum(v);
    if constexpr (BLOCK == kWave) {
        return v;
    } else {
        const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
        if (l == 0) red[w] = v;
        __syncthreads();
        T s = red[0];
#pragma unroll
        for (int i = 1; i < BLOCK / kWave; ++i) s += red[i];
        __syncthreads();
        return s;
    }
}

// Two sums in one pass over the LDS scratch (2 * BLOCK/64 entries).
template <int BLOCK, typename T>
__device__ __forceinline__ void block_sum2(T &a, T &b, T *red) {
    a = wave_sum(a);
    b = wave_sum(b);
    if constexpr (BLOCK > kWave) {
        constexpr int W = BLOCK / kWave;
        const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
        if (l == 0) {
            red[w] = a;
            red[W + w] = b;
        }
        __syncthreads();
        T sa = red[0], sb = red[W];
#pragma unroll
        for (int i = 1; i < W; ++i) {
            sa += red[i];
            sb += red[W + i];
        }
        __syncthreads();
        a = sa;
        b = sb;
    }
}

// e / d for 0 <= e < 2^31 / d: (e * m) >> 32 with m = ceil(2^32 / d) (exact
// because e * (m d - 2^32) < e d < 2^32).
__host__ __device__ inline uint64_t div_magic(int d) { return ((1ull << 32) + (uint64_t)d - 1) / (uint64_t)d; }
__device__ __forceinline__ int fast_div(int e, uint64_t m) { return (int)(((uint64_t)(uint32_t)e * m) >> 32); }

// Calls f(std::integral_constant<int, I>) for I = B .. E-1, so that arrays
// indexed by I are addressed with constants from the start (and live in
// registers rather than scratch).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Wave-local LDS ordering: a wavefront's LDS operations execute in program
// order, so when every thread involved belongs to one wave this only has to
// stop the compiler from moving LDS accesses across the point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace ssp
