// The allocation-free solve: ssp_solve with its workspace (the persistent
// grid's work counter, the FP64 residuals and the inner-precision vectors)
// in a fixed device array of the library instead of the handle's buffers.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/symstair.h"
#include "ssp_batch.h"
#include "ssp_host.h"

using namespace ssp_host;

namespace {

constexpr size_t kScratchBytes = SSP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

struct DeviceScratch {
    bool looked_up = false;
    hipError_t err = hipSuccess;
    void *ptr = nullptr;  // device address of `scratch` on this device
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

}  // namespace

// One copy per device, held from the code object's load to the process end.
// Host code must use the address hipGetSymbolAddress returns, never this name.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

ssp_status ssp_host::scratch_init(int device, void **ptr) {
    if (device < 0 || device >= kMaxDevices) {
        g_last_error = "device ordinal beyond the fixed-workspace table";
        return SSP_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceScratch &d = g_dev[device];
    if (!d.looked_up) {
        void *p = nullptr;
        d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        d.ptr = d.err == hipSuccess ? p : nullptr;
        d.looked_up = true;
    }
    if (d.err != hipSuccess) return hip_fail(d.err, "hipGetSymbolAddress(scratch)");
    if (ptr) *ptr = d.ptr;
    return SSP_OK;
}

extern "C" ssp_status ssp_solve_noalloc(ssp_batch *b, double rel_tol, int32_t max_iter, const double *gamma,
                                        double *lambda, int use_lambda0, int32_t *iters, double *relres,
                                        int32_t *prob_status, void *stream) {
    if (!b) return SSP_ERR_ARG;
    const size_t need = solve_scratch_bytes(b);
    if (need > kScratchBytes) {
        g_last_error = "ssp_solve_noalloc: the batch needs " + std::to_string(need) +
                       " bytes of solve workspace, the fixed array holds " + std::to_string(kScratchBytes);
        return SSP_ERR_ARG;
    }
    void *base = nullptr;
    {
        DevGuard g(b->device);
        const ssp_status rc = scratch_init(b->device, &base);  // recorded at ssp_batch_create
        if (rc != SSP_OK) return rc;
    }
    const SolveScratch sc = carve_solve_scratch(b, base);
    return solve_impl(b, rel_tol, max_iter, gamma, lambda, use_lambda0, iters, relres, prob_status, stream, &sc);
}
