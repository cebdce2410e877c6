// Host-side state of a batch handle and helpers shared by the host sources.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/symstair.h"
#include "ssp_host.h"

namespace ssp_host {

extern thread_local std::string g_last_error;

inline ssp_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return SSP_ERR_HIP;
}

#define SSP_HIP(call)                                               \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return ssp_host::hip_fail(e_, #call); \
    } while (0)

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

// Solve workspace of one call: the handle's own, or the library's fixed
// device array (the allocation-free entry point).
struct SolveScratch {
    unsigned *queue = nullptr;  // persistent grid's work counter (1 word)
    double *r64 = nullptr;      // FP64 residual, tot_v long
    double *rh64 = nullptr;     // FP64 residual in the scaled basis, tot_v long
    void *work = nullptr;       // 7 vectors of the storage precision, tot_v long each
};

}  // namespace ssp_host

struct ssp_batch {
    int device = 0;
    int P = 0;
    std::vector<int32_t> N, nx, nu;
    std::vector<int64_t> off_nn, off_nu, off_uu, off_v, off_u, koff;  // off_u: control vectors (N nu)
    std::vector<int64_t> off_blk32, off_blk64;  // full-block offsets (padded stride bs)
    std::vector<int64_t> off_b3_32, off_b3_64;  // solve-array offsets (knot stride)
    std::vector<int64_t> off_pk32;              // packed-block offsets (D remainders, FP32 storage)
    int nx_max = 1, nu_max = 0;
    int64_t knots = 0;
    // device metadata
    int32_t *dN = nullptr, *dnx = nullptr, *dnu = nullptr, *dorder = nullptr, *dknot = nullptr;
    // assembly work lists: per compiled state size, (problem, first knot)
    // items at ditems + item_off[c]; knots of the other problems in dgeneric
    int2 *ditems = nullptr;
    int32_t *dgeneric = nullptr;
    int item_off[ssp::kBuildClasses + 1] = {};
    // KKT step: work items (problem, first knot) by kernel class
    // (ssp::kkt_class_of), the generic class last, at dkkt + kkt_off[c]
    int2 *dkkt = nullptr;
    ssp::KktRec *dkktrec = nullptr;
    ssp::BuildRec *ditemrec = nullptr;  // the assembly work items with their problem's horizon and offsets  // the same items with their problem's sizes and offsets
    int64_t kkt_off[ssp::kKktClasses + 2] = {};
    int64_t n_generic = 0;
    int gen_nx_max = 1, gen_nu_max = 0;
    // global knot lists per state size (built on first use by the warm start)
    std::vector<std::pair<int, std::pair<int32_t *, int64_t>>> nx_knots;
    int64_t *doff_nn = nullptr, *doff_nu = nullptr, *doff_uu = nullptr, *doff_v = nullptr, *dkoff = nullptr;
    int64_t *doff_u = nullptr;
    int64_t *doff_blk32 = nullptr, *doff_blk64 = nullptr;
    int64_t *doff_b3_32 = nullptr, *doff_b3_64 = nullptr, *doff_pk32 = nullptr;
    // FP64 build workspaces
    double *Qinv = nullptr, *Rinv = nullptr;
    // stored matrices
    bool fp32 = false;
    bool have_storage = false;
    void *B3 = nullptr;  // per knot: D_k (packed), L_k, D_k^-1 (packed), storage type
    void *PM = nullptr;  // explicit stair blocks, built on demand
    float *SDlo = nullptr, *SLlo = nullptr;
    // solve workspace
    void *work = nullptr;
    double *r64 = nullptr;
    int32_t *douter = nullptr;
    // scaled basis (built when the scaled solve will run): Z_k, Oh_k in the
    // storage type (full blocks, stride bs), Z_k in FP64 (build only), the
    // scaled residual and the persistent grid's queue counter
    void *Zs = nullptr, *OH = nullptr;
    double *rh64 = nullptr;
    unsigned *dqueue = nullptr;
    bool have_scaled = false;  // Zs/OH/Zw/rh64 allocated for the current storage precision
    bool scaled = false;       // the last build wrote the scaled basis: ssp_solve runs the scaled kernel
    bool dinv_valid = false;   // the stored D_k^-1 matches the last build (a scaled build leaves it out)
    int s3_threads = 256, s3_lds = 0;  // mapping of the scaled kernel (0: default budget)
    float s3_tuned_ms = 0.0f;
    // state
    bool built = false;
    bool have_qr = false;  // Q^-1, R^-1 of the last build are in Qinv, Rinv (ssp_build, not from blocks)
    bool m_valid = false;  // explicit stair blocks PM match the last build
    ssp_precon pc = SSP_PC_SYM_STAIR;
    ssp_precision prec = SSP_FP64;
    int threads = 128;
    int lds_bytes = 0;  // 0: default
    int kernel = 0;     // 0 auto, 1 explicit, 2 batched fused, 3 cooperative (one problem), 4 scaled
    // cooperative solve of a single problem: barrier words and partial sums
    unsigned *dbar = nullptr;
    unsigned long long *drec = nullptr, *dwtag = nullptr;
    int coop_key = -1, coop_W = 0, coop_G = 0;  // cached plan (key: storage precision)
    int keep_qr = 1;                              // builds store Q^-1, R^-1 for the KKT step
    int acc64 = 0;                                // scaled solve: FP64 sums of the FP32 inner products
    int last_kernel = 0;                          // kernel of the last solve: 1 explicit, 2 fused, 3 cooperative, 4 scaled
    // Fused solve groups: the problems of one state size, largest first,
    // launched on their own stream with their own workgroup size and LDS
    // budget (0: derived from threads / lds_bytes above).
    struct Group {
        int nx = 0, count = 0, offset = 0;  // problems dgorder[offset .. offset + count)
        double work = 0;                    // sum of N nx^2 (launch order: largest first)
        int threads = 0, lds = 0;
        float tuned_ms = 0.0f;  // best solve time the autotuner measured (0: not tuned)
    };
    std::vector<Group> groups;
    int32_t *dgorder = nullptr;
    std::vector<hipStream_t> gstreams;
    std::vector<hipEvent_t> gevents;  // one per group, plus the fork event at the end
};

namespace ssp_host {

// Bytes of solve workspace the batch needs (FP64 sizes before a build).
size_t solve_scratch_bytes(const ssp_batch *b);
// The workspace pointers inside a region of solve_scratch_bytes(b) bytes
// at base (256-byte aligned).
SolveScratch carve_solve_scratch(const ssp_batch *b, void *base);
// ssp_solve with the workspace of sc (nullptr: the handle's own).
ssp_status solve_impl(ssp_batch *b, double rel_tol, int32_t max_iter, const double *gamma, double *lambda,
                      int use_lambda0, int32_t *iters, double *relres, int32_t *prob_status, void *stream,
                      const SolveScratch *sc);
// Looks up the device address of the fixed workspace array on `device`
// (the current device) once; later calls return the recorded result (the
// address into *ptr when ptr is not null).
ssp_status scratch_init(int device, void **ptr = nullptr);

}  // namespace ssp_host
