// A plain streaming copy, the library's own measure of the practical HBM rate
// that the solve's measured traffic is compared with: one 16-byte load and
// store per thread over a grid that covers the buffer, so the workgroups in
// flight at any time touch one contiguous stretch of memory (a grid-stride
// loop with a few thousand workgroups scatters them and streams 20-25 %
// slower on this GPU).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/symstair.h"
#include "ssp_batch.h"

namespace {

constexpr int kCopyThreads = 256;

__global__ __launch_bounds__(kCopyThreads) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                        int64_t n16) {
    const int64_t i = (int64_t)blockIdx.x * kCopyThreads + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

}  // namespace

ssp_status ssp_copy_bytes(const void *src, void *dst, int64_t bytes, void *stream) {
    if (!src || !dst || bytes < 0 || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return SSP_ERR_ARG;
    if (bytes == 0) return SSP_OK;
    const int64_t n16 = bytes / 16;
    const int64_t blocks = (n16 + kCopyThreads - 1) / kCopyThreads;
    if (blocks > 0x7fffffff) return SSP_ERR_ARG;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kCopyThreads), 0, (hipStream_t)stream,
                       (const uint4 *)src, (uint4 *)dst, n16);
    SSP_HIP(hipGetLastError());
    return SSP_OK;
}
