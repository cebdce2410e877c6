// Host side of the C ABI declared in include/symstair.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/symstair.h"
#include "ssp_batch.h"
#include "ssp_host.h"
#include "ssp_sweep.h"

using namespace ssp_host;

thread_local std::string ssp_host::g_last_error = "no error";

namespace {

void free_scaled(ssp_batch *b) {
    for (void *p : {b->Zs, b->OH, (void *)b->rh64})
        if (p) (void)hipFree(p);
    b->Zs = b->OH = nullptr;
    b->rh64 = nullptr;
    b->have_scaled = false;
    b->scaled = false;
}

void free_storage(ssp_batch *b) {
    for (void *p : {b->B3, b->PM, (void *)b->SDlo, (void *)b->SLlo, b->work})
        if (p) (void)hipFree(p);
    b->B3 = b->PM = b->work = nullptr;
    b->SDlo = b->SLlo = nullptr;
    b->have_storage = false;
    b->m_valid = false;
    free_scaled(b);
}

// Storage of the scaled basis for the current storage precision.
ssp_status alloc_scaled(ssp_batch *b) {
    if (b->have_scaled) return SSP_OK;
    const size_t elem = b->fp32 ? sizeof(float) : sizeof(double);
    const size_t nn = (size_t)(b->fp32 ? b->off_blk32 : b->off_blk64)[b->P];
    if (hipMalloc(&b->Zs, std::max<size_t>(nn, 1) * elem) != hipSuccess ||
        hipMalloc(&b->OH, std::max<size_t>(nn, 1) * elem) != hipSuccess ||
        dalloc(&b->rh64, (size_t)b->off_v[b->P]) != hipSuccess) {
        free_scaled(b);
        g_last_error = "hipMalloc of scaled-basis storage failed";
        return SSP_ERR_ALLOC;
    }
    b->have_scaled = true;
    return SSP_OK;
}

// Horner steps of the preconditioner polynomial in the scaled basis and
// the coefficient of each step.
int poly_steps(ssp_precon pc) {
    switch (pc) {
        case SSP_PC_BLOCK_JACOBI: return 0;
        case SSP_PC_STAIR_ADD:
        case SSP_PC_SYM_STAIR: return 1;
        case SSP_PC_NEUMANN2: return 2;
        case SSP_PC_NEUMANN3: return 3;
        default: return 0;
    }
}

// every problem has a compiled state size (the register-resident assembly,
// which also builds the scaled basis, and the scaled solve exist for those)
bool scaled_possible(const ssp_batch *b) {
    for (int p = 0; p < b->P; ++p)
        if (ssp::build_class_of(b->nx[p], b->nu[p]) < 0) return false;
    return true;
}

// LDS budget of the scaled kernel: the largest step of every state size in
// the batch (or the tuned / set budget), at least what the FP64 residual's
// staged fallback needs.
int scaled_lds(const ssp_batch *b, int threads, int m) {
    int need = 0;
    for (const auto &g : b->groups) need = std::max(need, ssp::pcg3_lds(g.nx, b->fp32, threads, m));
    int l = b->s3_lds > 0 ? b->s3_lds : need;
    // the FP64 residual needs one knot per step of every state size
    for (const auto &g : b->groups)
        while (l < ssp::kFusedLdsCap && ssp::pcg3_residual_steps(g.nx, b->fp32, l) < 1) l += 256;
    return std::min(l, ssp::kFusedLdsCap);
}

// the scaled kernel can run every state size of the batch with this budget
bool scaled_fits(const ssp_batch *b, int threads, int lds, int m) {
    for (const auto &g : b->groups)
        if (ssp::pcg3_steps_for(g.nx, b->fp32, threads, lds, m) < 1 || ssp::pcg3_residual_steps(g.nx, b->fp32, lds) < 1)
            return false;
    return true;
}

ssp_status alloc_storage(ssp_batch *b, bool fp32) {
    if (b->have_storage && b->fp32 == fp32) return SSP_OK;
    free_storage(b);
    const size_t elem = fp32 ? sizeof(float) : sizeof(double);
    const size_t nn = (size_t)(fp32 ? b->off_blk32 : b->off_blk64)[b->P];
    const size_t n3 = (size_t)(fp32 ? b->off_b3_32 : b->off_b3_64)[b->P];
    const size_t nv = (size_t)b->off_v[b->P];
    if (hipMalloc(&b->B3, std::max<size_t>(n3, 1) * elem) != hipSuccess) {
        free_storage(b);
        g_last_error = "hipMalloc of matrix storage failed";
        return SSP_ERR_ALLOC;
    }
    if (fp32) {
        if (dalloc(&b->SDlo, (size_t)b->off_pk32[b->P]) != hipSuccess || dalloc(&b->SLlo, nn) != hipSuccess) {
            free_storage(b);
            g_last_error = "hipMalloc of FP32 remainder storage failed";
            return SSP_ERR_ALLOC;
        }
    }
    if (hipMalloc(&b->work, std::max<size_t>(7 * nv, 1) * elem) != hipSuccess) {
        free_storage(b);
        g_last_error = "hipMalloc of solve workspace failed";
        return SSP_ERR_ALLOC;
    }
    b->fp32 = fp32;
    b->have_storage = true;
    return SSP_OK;
}


// Workgroup size and LDS bytes of the fused kernel for one solve group, or
// lds = 0 if its knots do not fit the fused kernel's registers or LDS.
void group_mapping(const ssp_batch *b, const ssp_batch::Group &g, int *threads, int *lds) {
    const int t = g.threads > 0 ? g.threads : b->threads;
    *threads = t;
    *lds = 0;
    if (!ssp::pcg2_threads_ok(t)) return;
    const int need = ssp::pcg2_lds(g.nx, b->fp32, t);
    if (need == 0) return;
    int l = g.lds > 0 ? g.lds : (b->lds_bytes > 0 ? b->lds_bytes : need);
    l = std::max(l, ssp::bt_sweep_min_lds(g.nx, true, 8));
    if (l > ssp::kFusedLdsCap) return;
    if (ssp::pcg2_steps_for(g.nx, b->fp32, t, l) < 1) return;
    *lds = l;
}

// knots from which a single problem runs the cooperative solve by default
constexpr int kCoopMinKnots = 24;

// a single problem long enough to spread over the grid, whose grid fits on
// the device at once (the plan is cached per storage precision)
bool use_coop(ssp_batch *b) {
    if (b->P != 1 || !b->dbar || !(b->kernel == 3 || (b->kernel == 0 && b->N[0] >= kCoopMinKnots))) return false;
    const int key = b->fp32 ? 1 : 0;
    if (b->coop_key != key) {
        b->coop_key = key;
        if (!ssp::coop_plan(b->N[0], b->nx[0], b->fp32, b->device, &b->coop_W, &b->coop_G)) b->coop_W = 0;
    }
    return b->coop_W > 0;
}

// every group can run the fused kernel
bool fused_ok(const ssp_batch *b) {
    for (const auto &g : b->groups) {
        int t, l;
        group_mapping(b, g, &t, &l);
        if (l == 0) return false;
    }
    return true;
}

int explicit_lds(const ssp_batch *b) {
    if (b->lds_bytes > 0) return b->lds_bytes;
    return ssp::pcg_default_lds(b->nx_max, b->fp32, b->threads);
}

ssp::BuildArgs build_args(const ssp_batch *b) {
    ssp::BuildArgs a{};
    a.N = b->dN;
    a.nx = b->dnx;
    a.nu = b->dnu;
    a.off_nn = b->doff_nn;
    a.off_nu = b->doff_nu;
    a.off_uu = b->doff_uu;
    a.off_blk = b->fp32 ? b->doff_blk32 : b->doff_blk64;
    a.off_b3 = b->fp32 ? b->doff_b3_32 : b->doff_b3_64;
    a.off_pk = b->doff_pk32;
    a.knot_prob = b->dknot;
    a.koff = b->dkoff;
    a.knot_list = b->dgeneric;
    a.Qinv = b->Qinv;
    a.Rinv = b->Rinv;
    a.B3 = b->B3;
    a.SDlo = b->fp32 ? b->SDlo : nullptr;
    a.SLlo = b->fp32 ? b->SLlo : nullptr;
    a.PM = b->PM;
    a.Zs = a.OH = nullptr;
    a.pc = (int)b->pc;
    a.mx = std::max(b->nx_max, b->nu_max);
    a.keep_qr = b->keep_qr;
    return a;
}

// D_k^-1 = W_k^T W_k into the stored blocks after a scaled build, on demand
ssp_status ensure_dinv(ssp_batch *b, hipStream_t s) {
    if (b->dinv_valid) return SSP_OK;
    ssp::BuildArgs a = build_args(b);
    a.Zs = b->Zs;
    SSP_HIP(ssp::launch_dinv_from_w(a, b->knots, b->nx_max, b->fp32, s));
    b->dinv_valid = true;
    return SSP_OK;
}

// explicit stair blocks, built on demand from the stored D^-1 and L
ssp_status ensure_m(ssp_batch *b, hipStream_t s) {
    if (b->m_valid) return SSP_OK;
    {
        ssp_status rc = ensure_dinv(b, s);
        if (rc != SSP_OK) return rc;
    }
    if (!b->PM) {
        const size_t elem = b->fp32 ? sizeof(float) : sizeof(double);
        const size_t nn = (size_t)(b->fp32 ? b->off_blk32 : b->off_blk64)[b->P];
        if (hipMalloc(&b->PM, std::max<size_t>(nn, 1) * elem) != hipSuccess) {
            b->PM = nullptr;
            g_last_error = "hipMalloc of explicit preconditioner blocks failed";
            return SSP_ERR_ALLOC;
        }
    }
    ssp::BuildArgs a = build_args(b);
    SSP_HIP(ssp::launch_build_phi(a, b->knots, b->nx_max, b->fp32, s));
    b->m_valid = true;
    return SSP_OK;
}

ssp::SolveArgs solve_args(const ssp_batch *b, double rel_tol, int32_t max_iter, const double *gamma,
                          double *lambda, int use_lambda0, int32_t *iters, double *relres, int32_t *prob_status) {
    ssp::SolveArgs a{};
    a.order = b->dorder;
    a.N = b->dN;
    a.nx = b->dnx;
    a.off_blk = b->fp32 ? b->doff_blk32 : b->doff_blk64;
    a.off_b3 = b->fp32 ? b->doff_b3_32 : b->doff_b3_64;
    a.off_pk = b->doff_pk32;
    a.off_v = b->doff_v;
    a.status = prob_status;
    a.B3 = b->B3;
    a.SDlo = b->fp32 ? b->SDlo : nullptr;
    a.SLlo = b->fp32 ? b->SLlo : nullptr;
    // the classic kernels apply scalar Jacobi as block-diagonal (its stored
    // D^-1 blocks are diagonal); the scaled kernel reads poly / pc_c below
    a.pc = b->pc == SSP_PC_SCALAR_JACOBI ? (int)SSP_PC_BLOCK_JACOBI : (int)b->pc;
    a.gamma = gamma;
    a.lambda = lambda;
    a.use_lambda0 = use_lambda0;
    a.tol = rel_tol;
    a.max_iter = max_iter;
    a.refine = b->prec == SSP_FP32_REFINE64 ? 1 : 0;
    a.max_outer = a.refine ? 5 : 1;
    a.theta = 0.5;
    a.tau_min = 1e-6;
    a.iters = iters;
    a.outer = b->douter;
    a.relres = relres;
    a.work = b->work;
    a.r64 = b->r64;
    a.tot_v = b->off_v[b->P];
    a.OH = b->OH;
    a.Z = b->Zs;
    a.rh64 = b->rh64;
    a.queue = b->dqueue;
    a.nprob = b->P;
    a.poly = poly_steps(b->pc);
    a.pc_c = b->pc == SSP_PC_STAIR_ADD ? 0.5 : 1.0;
    a.acc64 = b->acc64;
    return a;
}

// The scaled solve: refinement in FP64 around the float inner solve, or
// FP64 restarts from the true residual under FP64 storage.
ssp_status launch_scaled(ssp_batch *b, ssp::SolveArgs a, hipStream_t s) {
    const int t = b->s3_threads;
    a.lds_bytes = scaled_lds(b, t, a.poly);
    if (!scaled_fits(b, t, a.lds_bytes, a.poly)) {
        g_last_error = "scaled solve: the LDS budget holds no pipeline step of some state size";
        return SSP_ERR_ARG;
    }
    a.refine = b->prec == SSP_FP32 ? 0 : 1;
    a.max_outer = a.refine ? 5 : 1;
    a.theta = 0.5;
    // the float operator I + Oh is as well conditioned as block-Jacobi
    // preconditioned S, so the first inner solve may aim at theta tol itself
    // (no floor above it): one outer step then suffices for most problems
    a.tau_min = b->prec == SSP_FP64 ? 1e-15 : std::min(1e-6, a.theta * a.tol);
    // one persistent grid per state size (largest total work first), each
    // with its own queue counter, on internal streams forked from and joined
    // back into s: a grid whose queue is empty retires and the next size's
    // workgroups take its place
    const int ng = (int)b->groups.size();
    SSP_HIP(ssp::launch_fill_i32((int32_t *)a.queue, 0, ng, s));
    const bool fork = ng > 1;
    if (fork) {
        SSP_HIP(hipEventRecord(b->gevents[ng], s));
        for (int i = 0; i < ng; ++i) SSP_HIP(hipStreamWaitEvent(b->gstreams[i], b->gevents[ng], 0));
    }
    for (int i = 0; i < ng; ++i) {
        const auto &g = b->groups[i];
        ssp::SolveArgs ga = a;
        ga.order = b->dgorder + g.offset;
        ga.nprob = g.count;
        ga.queue = a.queue + i;
        SSP_HIP(ssp::launch_pcg3(ga, b->fp32, t, g.nx, 0, fork ? b->gstreams[i] : s));
    }
    if (fork) {
        for (int i = 0; i < ng; ++i) {
            SSP_HIP(hipEventRecord(b->gevents[i], b->gstreams[i]));
            SSP_HIP(hipStreamWaitEvent(s, b->gevents[i], 0));
        }
    }
    b->last_kernel = 4;
    return SSP_OK;
}

// Candidate LDS budgets of the autotuner for a group at `threads`: the
// fused kernel's largest step and two shorter ones (more workgroups per CU).
std::vector<int> lds_candidates(const ssp_batch *b, int nx, int threads) {
    std::vector<int> out;
    const int need = ssp::pcg2_lds(nx, b->fp32, threads);
    if (need == 0) return out;
    const int cmax = ssp::pcg2_steps_for(nx, b->fp32, threads, need);
    const int eb = b->fp32 ? 4 : 8, V = 16 / eb;
    const int ks = ssp::knot_stride(nx, eb), nxp = (nx + V - 1) / V * V;
    const int per = (ks + 4 * nxp) * eb;
    const int lo = ssp::bt_sweep_min_lds(nx, true, 8);
    for (int c : {cmax, cmax - 1, (cmax + 1) / 2}) {
        if (c < 1) continue;
        const int l = std::max((c + 2) * per + nxp * eb + 16, lo);
        if (l <= ssp::kFusedLdsCap && ssp::pcg2_steps_for(nx, b->fp32, threads, l) >= 1 &&
            std::find(out.begin(), out.end(), l) == out.end())
            out.push_back(l);
    }
    return out;
}

// Fused solve of every group (which < 0) or of group `which` alone, each
// group on its own stream, forked from and joined back into s.
ssp_status launch_groups(ssp_batch *b, ssp::SolveArgs a, int which, hipStream_t s) {
    const int ng = (int)b->groups.size();
    const bool fork = which < 0 && ng > 1;
    if (fork) {
        SSP_HIP(hipEventRecord(b->gevents[ng], s));
        for (int i = 0; i < ng; ++i) SSP_HIP(hipStreamWaitEvent(b->gstreams[i], b->gevents[ng], 0));
    }
    for (int i = 0; i < ng; ++i) {
        if (which >= 0 && i != which) continue;
        const auto &g = b->groups[i];
        int t, l;
        group_mapping(b, g, &t, &l);
        ssp::SolveArgs ga = a;
        ga.order = b->dgorder + g.offset;
        ga.lds_bytes = l;
        SSP_HIP(ssp::launch_pcg2(ga, g.count, b->fp32, t, g.nx, fork ? b->gstreams[i] : s));
    }
    if (fork) {
        for (int i = 0; i < ng; ++i) {
            SSP_HIP(hipEventRecord(b->gevents[i], b->gstreams[i]));
            SSP_HIP(hipStreamWaitEvent(s, b->gevents[i], 0));
        }
    }
    return SSP_OK;
}

// Autotuner of the scaled solve: workgroup size and LDS budget (the budget
// sets the knots per pipeline step of every state size and the workgroups
// resident per CU).  Each candidate solves the whole batch once untimed and
// once timed; the fastest is kept and the batch is solved once more with it.
ssp_status autotune_scaled(ssp_batch *b, double rel_tol, const double *gamma, double *lambda, int32_t *iters,
                           double *relres, int32_t *prob_status, void *stream) {
    DevGuard dg(b->device);
    hipStream_t s = (hipStream_t)stream;
    int32_t *st0 = nullptr;
    if (dalloc(&st0, (size_t)b->P) != hipSuccess) {
        g_last_error = "hipMalloc of status copy failed";
        return SSP_ERR_ALLOC;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ssp_status rc = SSP_OK;
    hipError_t e;
    auto fail = [&](hipError_t err, const char *what) {
        if (rc == SSP_OK) rc = hip_fail(err, what);
    };
    if ((e = hipMemcpyAsync(st0, prob_status, sizeof(int32_t) * b->P, hipMemcpyDeviceToDevice, s))) fail(e, "status copy");
    if (rc == SSP_OK && ((e = hipEventCreate(&e0)) || (e = hipEventCreate(&e1)))) fail(e, "hipEventCreate");
    const ssp::SolveArgs a = solve_args(b, rel_tol, 0, gamma, lambda, 0, iters, relres, prob_status);
    const int m = poly_steps(b->pc);
    int best_t = 0, best_l = 0;
    float best = 0.0f;
    for (int t : {256, 128}) {
        b->s3_threads = t;
        b->s3_lds = 0;
        const int base = scaled_lds(b, t, m);
        for (double f : {1.0, 1.25, 1.5, 0.8}) {
            const int l = std::min((int)(base * f) / 16 * 16, ssp::kFusedLdsCap);
            if (!scaled_fits(b, t, l, m) || (f != 1.0 && l == base)) continue;
            b->s3_lds = l;
            float ms = 0.0f;
            for (int rep = 0; rep < 2 && rc == SSP_OK; ++rep) {
                if ((e = hipMemcpyAsync(prob_status, st0, sizeof(int32_t) * b->P, hipMemcpyDeviceToDevice, s))) {
                    fail(e, "status restore");
                    break;
                }
                if ((e = hipEventRecord(e0, s))) fail(e, "hipEventRecord");
                if (rc == SSP_OK && (rc = launch_scaled(b, a, s)) != SSP_OK) break;
                if ((e = hipEventRecord(e1, s)) || (e = hipEventSynchronize(e1)) || (e = hipEventElapsedTime(&ms, e0, e1)))
                    fail(e, "autotune timing");
            }
            if (rc != SSP_OK) break;
            if (best_t == 0 || ms < best) {
                best = ms;
                best_t = t;
                best_l = l;
            }
        }
        if (rc != SSP_OK) break;
    }
    if (best_t) {
        b->s3_threads = best_t;
        b->s3_lds = best_l;
        b->s3_tuned_ms = best;
    } else {
        b->s3_threads = 256;
        b->s3_lds = 0;
    }
    if (rc == SSP_OK &&
        (e = hipMemcpyAsync(prob_status, st0, sizeof(int32_t) * b->P, hipMemcpyDeviceToDevice, s)))
        fail(e, "status restore");
    if (rc == SSP_OK) rc = launch_scaled(b, a, s);
    if (rc == SSP_OK && (e = hipStreamSynchronize(s))) fail(e, "hipStreamSynchronize");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(st0);
    return rc;
}

}  // namespace

extern "C" {

const char *ssp_status_str(ssp_status s) {
    switch (s) {
        case SSP_OK: return "ok";
        case SSP_ERR_ARG: return "invalid argument";
        case SSP_ERR_ALLOC: return "allocation failed";
        case SSP_ERR_HIP: return "HIP runtime error";
        case SSP_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

const char *ssp_last_error(void) { return ssp_host::g_last_error.c_str(); }

ssp_status ssp_batch_create(int32_t nprob, const int32_t *N, const int32_t *nx, const int32_t *nu, int device,
                            ssp_batch **out) {
    if (!out) return SSP_ERR_ARG;
    *out = nullptr;
    if (nprob < 1 || !N || !nx || !nu) return SSP_ERR_ARG;
    int ndev = 0;
    SSP_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return SSP_ERR_ARG;
    for (int p = 0; p < nprob; ++p)
        if (N[p] < 1 || nx[p] < 1 || nx[p] > 64 || nu[p] < 0 || nu[p] > 64) return SSP_ERR_ARG;

    ssp_batch *b = new (std::nothrow) ssp_batch();
    if (!b) return SSP_ERR_ALLOC;
    b->device = device;
    b->P = nprob;
    b->N.assign(N, N + nprob);
    b->nx.assign(nx, nx + nprob);
    b->nu.assign(nu, nu + nprob);
    b->off_nn.assign(nprob + 1, 0);
    b->off_nu.assign(nprob + 1, 0);
    b->off_uu.assign(nprob + 1, 0);
    b->off_v.assign(nprob + 1, 0);
    b->off_u.assign(nprob + 1, 0);
    b->koff.assign(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        const int64_t n = N[p], x = nx[p], u = nu[p];
        b->off_nn[p + 1] = b->off_nn[p] + n * x * x;
        b->off_nu[p + 1] = b->off_nu[p] + n * x * u;
        b->off_uu[p + 1] = b->off_uu[p] + n * u * u;
        b->off_v[p + 1] = b->off_v[p] + n * x;
        b->off_u[p + 1] = b->off_u[p] + n * u;
        b->koff[p + 1] = b->koff[p] + n;
        b->nx_max = std::max(b->nx_max, (int)x);
        b->nu_max = std::max(b->nu_max, (int)u);
    }
    b->off_blk32.assign(nprob + 1, 0);
    b->off_blk64.assign(nprob + 1, 0);
    b->off_b3_32.assign(nprob + 1, 0);
    b->off_b3_64.assign(nprob + 1, 0);
    b->off_pk32.assign(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        b->off_blk32[p + 1] = b->off_blk32[p] + (int64_t)N[p] * ssp::block_stride(nx[p], 4);
        b->off_blk64[p + 1] = b->off_blk64[p] + (int64_t)N[p] * ssp::block_stride(nx[p], 8);
        b->off_b3_32[p + 1] = b->off_b3_32[p] + (int64_t)N[p] * ssp::knot_stride(nx[p], 4);
        b->off_b3_64[p + 1] = b->off_b3_64[p] + (int64_t)N[p] * ssp::knot_stride(nx[p], 8);
        b->off_pk32[p + 1] = b->off_pk32[p] + (int64_t)N[p] * ssp::packed_stride(nx[p], 4);
    }
    b->knots = b->koff[nprob];
    // the per-knot FP64 assembly keeps 4 nx^2 + 2 nx nu + nu^2 + nx doubles in LDS
    const int64_t asm_bytes = 8 * (4ll * b->nx_max * b->nx_max + 2ll * b->nx_max * b->nu_max +
                                   (int64_t)b->nu_max * b->nu_max + b->nx_max);
    if (b->knots > INT32_MAX || asm_bytes > 160 * 1024) {
        g_last_error = b->knots > INT32_MAX ? "more than 2^31 - 1 knots in the batch"
                                            : "nx_max, nu_max: the per-knot FP64 assembly needs more than 160 KiB of LDS";
        delete b;
        return SSP_ERR_ARG;
    }
    // problem order: largest N * nx^2 first, ties by index
    std::vector<int32_t> order(nprob);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
        return (int64_t)N[a] * nx[a] * nx[a] > (int64_t)N[c] * nx[c] * nx[c];
    });
    // fused solve groups by state size, largest total work first
    {
        std::vector<int> sizes(b->nx.begin(), b->nx.end());
        std::sort(sizes.begin(), sizes.end());
        sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
        for (int x : sizes) {
            ssp_batch::Group g;
            g.nx = x;
            for (int p = 0; p < nprob; ++p)
                if (nx[p] == x) g.work += (double)N[p] * x * x;
            b->groups.push_back(g);
        }
        std::stable_sort(b->groups.begin(), b->groups.end(),
                         [](const ssp_batch::Group &u, const ssp_batch::Group &v) { return u.work > v.work; });
    }
    std::vector<int32_t> gorder;
    for (auto &g : b->groups) {
        g.offset = (int)gorder.size();
        for (int32_t p : order)
            if (nx[p] == g.nx) gorder.push_back(p);
        g.count = (int)gorder.size() - g.offset;
    }
    std::vector<int32_t> knot_prob((size_t)b->knots);
    for (int p = 0; p < nprob; ++p)
        std::fill(knot_prob.begin() + b->koff[p], knot_prob.begin() + b->koff[p + 1], p);
    // assembly work lists (largest problems first within a class)
    std::vector<int2> items;
    std::vector<int32_t> generic;
    for (int c = 0; c < ssp::kBuildClasses; ++c) {
        b->item_off[c] = (int)items.size();
        const int per = ssp::build_knots_per_item(c);
        for (int32_t p : order)
            if (ssp::build_class_of(nx[p], nu[p]) == c)
                for (int k0 = 0; k0 < N[p]; k0 += per) items.push_back(make_int2(p, k0));
    }
    b->item_off[ssp::kBuildClasses] = (int)items.size();
    std::vector<ssp::BuildRec> itemrec(items.size());
    for (size_t j = 0; j < items.size(); ++j) {
        const int p = items[j].x;
        itemrec[j] = ssp::BuildRec{p, items[j].y, N[p], 0, b->off_nn[p], b->off_nu[p], b->off_uu[p], b->off_pk32[p],
                                   b->off_blk32[p], b->off_blk64[p], b->off_b3_32[p], b->off_b3_64[p]};
    }
    for (int p = 0; p < nprob; ++p) {
        if (ssp::build_class_of(nx[p], nu[p]) >= 0) continue;
        for (int64_t g = b->koff[p]; g < b->koff[p + 1]; ++g) generic.push_back((int32_t)g);
        b->gen_nx_max = std::max(b->gen_nx_max, (int)nx[p]);
        b->gen_nu_max = std::max(b->gen_nu_max, (int)nu[p]);
    }
    b->n_generic = (int64_t)generic.size();
    // KKT work items, one list per kernel class, the generic class last
    std::vector<int2> kkt;
    kkt.reserve((size_t)b->knots);
    for (int c = 0; c <= ssp::kKktClasses; ++c) {
        b->kkt_off[c] = (int64_t)kkt.size();
        const int want = c < ssp::kKktClasses ? c : -1, per = ssp::kkt_knots_per_item(want);
        for (int p = 0; p < nprob; ++p)
            if (ssp::kkt_class_of(nx[p], nu[p]) == want)
                for (int k0 = 0; k0 < N[p]; k0 += per) kkt.push_back(make_int2(p, k0));
    }
    b->kkt_off[ssp::kKktClasses + 1] = (int64_t)kkt.size();
    std::vector<ssp::KktRec> kktrec(kkt.size());
    for (size_t j = 0; j < kkt.size(); ++j) {
        const int p = kkt[j].x;
        kktrec[j] = ssp::KktRec{p, kkt[j].y, N[p], nu[p], b->off_nn[p], b->off_v[p], b->off_u[p], b->off_nu[p],
                                b->off_uu[p], 0};
    }

    DevGuard g(device);
    ssp_status rc = SSP_OK;
    auto up = [&](auto **dst, const auto *src, size_t cnt) {
        if (rc != SSP_OK) return;
        if (dalloc(dst, cnt) != hipSuccess) {
            rc = SSP_ERR_ALLOC;
            return;
        }
        if (cnt == 0) return;
        hipError_t e = hipMemcpy(*dst, src, cnt * sizeof(**dst), hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy metadata");
    };
    up(&b->dN, b->N.data(), nprob);
    up(&b->dnx, b->nx.data(), nprob);
    up(&b->dnu, b->nu.data(), nprob);
    up(&b->dorder, order.data(), nprob);
    up(&b->dgorder, gorder.data(), gorder.size());
    if (rc == SSP_OK && b->groups.size() > 1) {
        for (size_t i = 0; i < b->groups.size(); ++i) {
            hipStream_t st;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                rc = SSP_ERR_HIP;
                break;
            }
            b->gstreams.push_back(st);
        }
        for (size_t i = 0; rc == SSP_OK && i <= b->groups.size(); ++i) {
            hipEvent_t ev;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                rc = SSP_ERR_HIP;
                break;
            }
            b->gevents.push_back(ev);
        }
        if (rc != SSP_OK) g_last_error = "stream/event creation failed";
    }
    up(&b->dknot, knot_prob.data(), knot_prob.size());
    up(&b->ditems, items.data(), items.size());
    up(&b->ditemrec, itemrec.data(), itemrec.size());
    up(&b->dgeneric, generic.data(), generic.size());
    up(&b->dkkt, kkt.data(), kkt.size());
    up(&b->dkktrec, kktrec.data(), kktrec.size());
    up(&b->doff_nn, b->off_nn.data(), nprob + 1);
    up(&b->doff_nu, b->off_nu.data(), nprob + 1);
    up(&b->doff_uu, b->off_uu.data(), nprob + 1);
    up(&b->doff_v, b->off_v.data(), nprob + 1);
    up(&b->doff_u, b->off_u.data(), nprob + 1);
    up(&b->dkoff, b->koff.data(), nprob + 1);
    up(&b->doff_blk32, b->off_blk32.data(), nprob + 1);
    up(&b->doff_blk64, b->off_blk64.data(), nprob + 1);
    up(&b->doff_b3_32, b->off_b3_32.data(), nprob + 1);
    up(&b->doff_b3_64, b->off_b3_64.data(), nprob + 1);
    up(&b->doff_pk32, b->off_pk32.data(), nprob + 1);
    if (rc == SSP_OK && nprob == 1) {
        if (dalloc(&b->dbar, ssp::coop_flag_words(N[0])) != hipSuccess ||
            dalloc(&b->drec, ssp::coop_rec_words(N[0])) != hipSuccess ||
            dalloc(&b->dwtag, ssp::coop_wtag_words(N[0], nx[0])) != hipSuccess)
            rc = SSP_ERR_ALLOC;
        else if (hipMemset(b->dbar, 0, sizeof(unsigned) * ssp::coop_flag_words(N[0])) != hipSuccess ||
                 hipMemset(b->drec, 0, 8 * ssp::coop_rec_words(N[0])) != hipSuccess ||
                 hipMemset(b->dwtag, 0, 8 * ssp::coop_wtag_words(N[0], nx[0])) != hipSuccess ||
                 hipDeviceSynchronize() != hipSuccess)
            rc = SSP_ERR_HIP;
    }
    if (rc == SSP_OK) {
        const size_t nn = b->off_nn[nprob], uu = b->off_uu[nprob], nv = b->off_v[nprob];
        if (dalloc(&b->Qinv, nn) != hipSuccess || dalloc(&b->Rinv, uu) != hipSuccess ||
            dalloc(&b->r64, nv) != hipSuccess || dalloc(&b->douter, (size_t)nprob) != hipSuccess ||
            dalloc(&b->dqueue, std::max<size_t>(b->groups.size(), 1)) != hipSuccess)
            rc = SSP_ERR_ALLOC;
    }
    if (rc != SSP_OK) {
        if (rc == SSP_ERR_ALLOC) g_last_error = "hipMalloc of batch metadata/workspace failed";
        ssp_batch_destroy(b);
        return rc;
    }
    {
        // device address of this device's fixed solve workspace (the
        // allocation-free solve entry point), looked up once per device
        DevGuard g(device);
        (void)scratch_init(device);
    }
    *out = b;
    return SSP_OK;
}

ssp_status ssp_batch_destroy(ssp_batch *b) {
    if (!b) return SSP_OK;
    {
        DevGuard g(b->device);
        (void)hipDeviceSynchronize();
        free_storage(b);
        for (auto &kl : b->nx_knots)
            if (kl.second.first) (void)hipFree(kl.second.first);
        for (hipStream_t st : b->gstreams) (void)hipStreamDestroy(st);
        for (hipEvent_t ev : b->gevents) (void)hipEventDestroy(ev);
        if (b->dgorder) (void)hipFree(b->dgorder);
        for (void *p : {(void *)b->dN, (void *)b->dnx, (void *)b->dnu, (void *)b->dorder, (void *)b->dknot,
                        (void *)b->ditems, (void *)b->ditemrec, (void *)b->dgeneric, (void *)b->dkkt, (void *)b->dkktrec, (void *)b->doff_nn, (void *)b->doff_nu, (void *)b->doff_uu, (void *)b->doff_v,
                        (void *)b->dkoff, (void *)b->doff_blk32, (void *)b->doff_blk64, (void *)b->doff_b3_32, (void *)b->doff_b3_64,
                        (void *)b->doff_pk32, (void *)b->dbar, (void *)b->drec, (void *)b->dwtag, (void *)b->Qinv, (void *)b->Rinv,
                        (void *)b->r64, (void *)b->douter, (void *)b->dqueue, (void *)b->doff_u})
            if (p) (void)hipFree(p);
    }
    delete b;
    return SSP_OK;
}

ssp_status ssp_layout(const ssp_batch *b, int64_t *off_nn, int64_t *off_nu, int64_t *off_uu, int64_t *off_v,
                      int64_t *off_u) {
    if (!b) return SSP_ERR_ARG;
    const size_t cnt = (size_t)b->P + 1;
    if (off_u) std::memcpy(off_u, b->off_u.data(), cnt * sizeof(int64_t));
    if (off_nn) std::memcpy(off_nn, b->off_nn.data(), cnt * sizeof(int64_t));
    if (off_nu) std::memcpy(off_nu, b->off_nu.data(), cnt * sizeof(int64_t));
    if (off_uu) std::memcpy(off_uu, b->off_uu.data(), cnt * sizeof(int64_t));
    if (off_v) std::memcpy(off_v, b->off_v.data(), cnt * sizeof(int64_t));
    return SSP_OK;
}

ssp_status ssp_set_mapping(ssp_batch *b, int32_t threads, int32_t lds_bytes, int32_t kernel) {
    if (!b) return SSP_ERR_ARG;
    if (threads != 64 && threads != 128 && threads != 256 && threads != 512) return SSP_ERR_ARG;
    if (lds_bytes < 0 || lds_bytes > 160 * 1024) return SSP_ERR_ARG;
    if (kernel < 0 || kernel > 4) return SSP_ERR_ARG;
    if (lds_bytes > 0 && lds_bytes < ssp::pcg_min_lds(b->nx_max, true)) return SSP_ERR_ARG;
    b->threads = threads;
    b->lds_bytes = lds_bytes;
    b->kernel = kernel;
    for (auto &g : b->groups) g.threads = g.lds = 0;
    return SSP_OK;
}

ssp_status ssp_build(ssp_batch *b, ssp_precon pc, ssp_precision prec, const double *A, const double *B,
                     const double *Q, const double *R, int32_t *prob_status, void *stream) {
    if (!b || !A || !Q || !prob_status) return SSP_ERR_ARG;
    if (b->nu_max > 0 && (!B || !R)) return SSP_ERR_ARG;
    if (pc < SSP_PC_BLOCK_JACOBI || pc > SSP_PC_NEUMANN3) return SSP_ERR_ARG;
    if (prec < SSP_FP64 || prec > SSP_FP32_REFINE64) return SSP_ERR_ARG;
    // which solve will run: the scaled one for the polynomial forms, for the
    // block preconditioners under FP32 storage, and when asked for (kernel 4)
    const bool poly = pc == SSP_PC_NEUMANN2 || pc == SSP_PC_NEUMANN3;
    const bool one_long = b->P == 1 && b->N[0] >= 24;  // the cooperative solve's case
    bool scaled = b->kernel == 4 || poly ||
                  (b->kernel == 0 && prec != SSP_FP64 && pc != SSP_PC_SCALAR_JACOBI && !one_long);
    if (pc == SSP_PC_SCALAR_JACOBI) {
        if (b->kernel == 4) {
            g_last_error = "scalar Jacobi has no scaled-basis form (use kernel 0, 1 or 2)";
            return SSP_ERR_ARG;
        }
        scaled = false;
    }
    if (scaled && !scaled_possible(b)) {
        if (poly || b->kernel == 4) {
            g_last_error = "the scaled solve (and the polynomial preconditioners) need state sizes 6, 14, 26 or 36 "
                           "with nu <= nx";
            return SSP_ERR_ARG;
        }
        scaled = false;
    }
    if (poly && (b->kernel == 1 || b->kernel == 2 || b->kernel == 3)) {
        g_last_error = "the polynomial preconditioners run in the scaled solve only (kernel 0 or 4)";
        return SSP_ERR_ARG;
    }
    DevGuard g(b->device);
    hipStream_t s = (hipStream_t)stream;
    const bool fp32 = prec != SSP_FP64;
    ssp_status rc = alloc_storage(b, fp32);
    if (rc != SSP_OK) return rc;
    if (scaled && (rc = alloc_scaled(b)) != SSP_OK) return rc;
    b->built = false;
    b->m_valid = false;
    b->pc = pc;
    b->prec = prec;
    b->scaled = scaled;
    b->dinv_valid = !scaled;
    b->have_qr = b->keep_qr != 0;
    SSP_HIP(ssp::launch_fill_i32(prob_status, 0, b->P, s));
    ssp::BuildArgs a = build_args(b);
    a.A = A;
    a.B = B;
    a.Q = Q;
    a.R = R;
    a.status = prob_status;
    if (scaled) {
        a.Zs = b->Zs;
        a.OH = b->OH;
    }
    // The classes are independent (disjoint problems): each class's chain (inverse, assembly, Oh) runs on the
    // internal stream of its state size, forked from and joined back into the caller's stream, so the small
    // classes' launches overlap the large ones' instead of queueing behind them.
    const int ng = (int)b->groups.size();
    const bool fork = ng > 1 && (int)b->gstreams.size() == ng;
    if (fork) {
        SSP_HIP(hipEventRecord(b->gevents[ng], s));
        for (int i = 0; i < ng; ++i) SSP_HIP(hipStreamWaitEvent(b->gstreams[i], b->gevents[ng], 0));
    }
    for (int c = 0; c < ssp::kBuildClasses; ++c) {
        const int n = b->item_off[c + 1] - b->item_off[c];
        if (n == 0) continue;
        hipStream_t cs = s;
        if (fork)
            for (int i = 0; i < ng; ++i)
                if (b->groups[i].nx == ssp::kBuildSizes[c]) cs = b->gstreams[i];
        a.brec = b->ditemrec + b->item_off[c];
        SSP_HIP(ssp::launch_build_class(c, a, b->ditems + b->item_off[c], n, fp32, cs));
        if (scaled) SSP_HIP(ssp::launch_build_ohat(c, a, b->ditems + b->item_off[c], n, fp32, cs));
    }
    SSP_HIP(ssp::launch_build(a, b->n_generic, b->gen_nx_max, b->gen_nu_max, fp32, s));
    if (fork)
        for (int i = 0; i < ng; ++i) {
            SSP_HIP(hipEventRecord(b->gevents[i], b->gstreams[i]));
            SSP_HIP(hipStreamWaitEvent(s, b->gevents[i], 0));
        }
    if (pc == SSP_PC_SCALAR_JACOBI) SSP_HIP(ssp::launch_jacobi_diag(a, b->knots, fp32, s));
    b->built = true;
    return SSP_OK;
}

ssp_status ssp_build_from_blocks(ssp_batch *b, ssp_precon pc, ssp_precision prec, const double *D,
                                 const double *Lsub, int32_t *prob_status, void *stream) {
    if (!b || !D || !Lsub || !prob_status) return SSP_ERR_ARG;
    if (pc < SSP_PC_BLOCK_JACOBI || pc > SSP_PC_SCALAR_JACOBI) return SSP_ERR_ARG;
    if (prec < SSP_FP64 || prec > SSP_FP32_REFINE64) return SSP_ERR_ARG;
    if (b->kernel == 4) {
        g_last_error = "the scaled solve needs the assembly from dynamics (ssp_build)";
        return SSP_ERR_ARG;
    }
    DevGuard g(b->device);
    hipStream_t s = (hipStream_t)stream;
    const bool fp32 = prec != SSP_FP64;
    ssp_status rc = alloc_storage(b, fp32);
    if (rc != SSP_OK) return rc;
    b->built = false;
    b->m_valid = false;
    b->pc = pc;
    b->prec = prec;
    b->scaled = false;
    b->dinv_valid = true;
    b->have_qr = false;
    SSP_HIP(ssp::launch_fill_i32(prob_status, 0, b->P, s));
    ssp::BuildArgs a = build_args(b);
    a.status = prob_status;
    SSP_HIP(ssp::launch_build_blocks(a, D, Lsub, b->knots, fp32, s));
    if (pc == SSP_PC_SCALAR_JACOBI) SSP_HIP(ssp::launch_jacobi_diag(a, b->knots, fp32, s));
    b->built = true;
    return SSP_OK;
}

}  // extern "C"

// ssp_solve and the allocation-free solve share this body
size_t ssp_host::solve_scratch_bytes(const ssp_batch *b) {
    const size_t nv = (size_t)b->off_v[b->P];
    const size_t elem = b->built && b->fp32 ? sizeof(float) : sizeof(double);
    auto up = [](size_t n) { return (n + 255) / 256 * 256; };
    return 256 + 2 * up(nv * sizeof(double)) + up(7 * nv * elem);
}

ssp_host::SolveScratch ssp_host::carve_solve_scratch(const ssp_batch *b, void *base) {
    const size_t nv = (size_t)b->off_v[b->P];
    auto up = [](size_t n) { return (n + 255) / 256 * 256; };
    char *p = (char *)base;
    SolveScratch sc;
    sc.queue = (unsigned *)p;
    sc.r64 = (double *)(p + 256);
    sc.rh64 = (double *)(p + 256 + up(nv * sizeof(double)));
    sc.work = p + 256 + 2 * up(nv * sizeof(double));
    return sc;
}

ssp_status ssp_host::solve_impl(ssp_batch *b, double rel_tol, int32_t max_iter, const double *gamma,
                                double *lambda, int use_lambda0, int32_t *iters, double *relres,
                                int32_t *prob_status, void *stream, const SolveScratch *sc) {
    if (!b || !gamma || !lambda || !iters || !relres || !prob_status) return SSP_ERR_ARG;
    if (!(rel_tol >= 0.0) || use_lambda0 < 0 || use_lambda0 > 2) return SSP_ERR_ARG;
    if (!b->built) return SSP_ERR_STATE;
    DevGuard g(b->device);
    hipStream_t s = (hipStream_t)stream;
    ssp::SolveArgs a = solve_args(b, rel_tol, max_iter, gamma, lambda, use_lambda0, iters, relres, prob_status);
    if (sc) {
        a.work = sc->work;
        a.r64 = sc->r64;
        a.rh64 = sc->rh64;
        a.queue = sc->queue;
    }
    if (b->scaled) return launch_scaled(b, a, s);
    if (use_coop(b)) {
        // one long problem: spread its knots over the whole grid
        const int c0 = ssp::coop_clear_first();
        SSP_HIP(ssp::launch_fill_i32((int32_t *)b->dbar + c0, 0, ssp::coop_flag_words(b->N[0]) - c0, s));
        SSP_HIP(ssp::launch_coop(a, b->dbar, b->drec, b->dwtag, b->nx[0], b->coop_W, b->coop_G, b->fp32, s));
        b->last_kernel = 3;
        return SSP_OK;
    }
    if (b->kernel != 1 && fused_ok(b)) {
        b->last_kernel = 2;
        return launch_groups(b, a, -1, s);
    } else {
        b->last_kernel = 1;
        // explicit stored stair blocks (also the fallback when a knot does not
        // fit the fused kernel's registers or LDS)
        if (sc && b->pc != SSP_PC_BLOCK_JACOBI && !b->PM) {
            g_last_error = "the explicit kernel's stair blocks are not allocated yet (a first ssp_solve or "
                           "ssp_export allocates them)";
            return SSP_ERR_STATE;
        }
        if (b->pc != SSP_PC_BLOCK_JACOBI) {
            ssp_status rc = ensure_m(b, s);
            if (rc != SSP_OK) return rc;
            a.PM = b->PM;
        }
        a.lds_bytes = explicit_lds(b);
        SSP_HIP(ssp::launch_pcg(a, b->P, b->fp32, b->threads, s));
    }
    return SSP_OK;
}

extern "C" {

ssp_status ssp_solve(ssp_batch *b, double rel_tol, int32_t max_iter, const double *gamma, double *lambda,
                     int use_lambda0, int32_t *iters, double *relres, int32_t *prob_status, void *stream) {
    return solve_impl(b, rel_tol, max_iter, gamma, lambda, use_lambda0, iters, relres, prob_status, stream,
                      nullptr);
}

ssp_status ssp_solve_outer(const ssp_batch *b, int32_t *outer, void *stream) {
    if (!b || !outer) return SSP_ERR_ARG;
    if (!b->built) return SSP_ERR_STATE;
    DevGuard g(b->device);
    SSP_HIP(hipMemcpyAsync(outer, b->douter, sizeof(int32_t) * b->P, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SSP_OK;
}

ssp_status ssp_export(ssp_batch *b, int which, double *diag, double *off, void *stream) {
    if (!b || !diag || !off || which < 0 || which > 3) return SSP_ERR_ARG;
    if (which == 3) {
        if (!b->built) return SSP_ERR_STATE;
        if (!b->scaled) {
            g_last_error = "the last build did not write the scaled basis";
            return SSP_ERR_STATE;
        }
        DevGuard g(b->device);
        hipStream_t s = (hipStream_t)stream;
        ssp::BuildArgs a = build_args(b);
        SSP_HIP(ssp::launch_export(a, 3, b->Zs, nullptr, b->fp32, diag, b->knots, s));
        SSP_HIP(ssp::launch_export(a, 3, b->OH, nullptr, b->fp32, off, b->knots, s));
        return SSP_OK;
    }
    if (!b->built) return SSP_ERR_STATE;
    if (which == 1 && (b->pc == SSP_PC_NEUMANN2 || b->pc == SSP_PC_NEUMANN3)) {
        g_last_error = "a polynomial preconditioner of degree >= 2 is not block tridiagonal";
        return SSP_ERR_ARG;
    }
    DevGuard g(b->device);
    hipStream_t s = (hipStream_t)stream;
    ssp::BuildArgs a = build_args(b);
    if (which == 1) {
        ssp_status rd = ensure_dinv(b, s);
        if (rd != SSP_OK) return rd;
        SSP_HIP(ssp::launch_export(a, 2, b->B3, nullptr, b->fp32, diag, b->knots, s));
        ssp_status rc = ensure_m(b, s);
        if (rc != SSP_OK) return rc;
        a = build_args(b);
        SSP_HIP(ssp::launch_export(a, 3, b->PM, nullptr, b->fp32, off, b->knots, s));
    } else {
        const bool lo = which == 0 && b->fp32;
        SSP_HIP(ssp::launch_export(a, 0, b->B3, lo ? b->SDlo : nullptr, b->fp32, diag, b->knots, s));
        SSP_HIP(ssp::launch_export(a, 1, b->B3, lo ? b->SLlo : nullptr, b->fp32, off, b->knots, s));
    }
    return SSP_OK;
}

ssp_status ssp_autotune(ssp_batch *b, double rel_tol, const double *gamma, double *lambda, int32_t *iters,
                        double *relres, int32_t *prob_status, void *stream) {
    if (!b || !gamma || !lambda || !iters || !relres || !prob_status || !(rel_tol >= 0.0)) return SSP_ERR_ARG;
    if (!b->built) return SSP_ERR_STATE;
    if (b->scaled) return autotune_scaled(b, rel_tol, gamma, lambda, iters, relres, prob_status, stream);
    if (b->kernel == 1 || !fused_ok(b) || use_coop(b))  // only the batched fused kernel has a mapping to tune
        return ssp_solve(b, rel_tol, 0, gamma, lambda, 0, iters, relres, prob_status, stream);
    DevGuard dg(b->device);
    hipStream_t s = (hipStream_t)stream;
    int32_t *st0 = nullptr;
    if (dalloc(&st0, (size_t)b->P) != hipSuccess) {
        g_last_error = "hipMalloc of status copy failed";
        return SSP_ERR_ALLOC;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ssp_status rc = SSP_OK;
    auto fail = [&](hipError_t e, const char *what) {
        if (rc == SSP_OK) rc = hip_fail(e, what);
    };
    hipError_t e = hipMemcpyAsync(st0, prob_status, sizeof(int32_t) * b->P, hipMemcpyDeviceToDevice, s);
    if (e) fail(e, "status copy");
    if (rc == SSP_OK && ((e = hipEventCreate(&e0)) || (e = hipEventCreate(&e1)))) fail(e, "hipEventCreate");
    const ssp::SolveArgs a = solve_args(b, rel_tol, 0, gamma, lambda, 0, iters, relres, prob_status);
    for (size_t gi = 0; rc == SSP_OK && gi < b->groups.size(); ++gi) {
        auto &g = b->groups[gi];
        int best_t = 0, best_l = 0;
        float best = 0.0f;
        for (int t : {128, 256}) {
            for (int l : lds_candidates(b, g.nx, t)) {
                g.threads = t;
                g.lds = l;
                float ms = 0.0f;
                for (int rep = 0; rep < 2 && rc == SSP_OK; ++rep) {  // warm-up, then timed
                    if ((e = hipMemcpyAsync(prob_status, st0, sizeof(int32_t) * b->P, hipMemcpyDeviceToDevice, s))) {
                        fail(e, "status restore");
                        break;
                    }
                    if ((e = hipEventRecord(e0, s))) fail(e, "hipEventRecord");
                    if (rc == SSP_OK && (rc = launch_groups(b, a, (int)gi, s)) != SSP_OK) break;
                    if ((e = hipEventRecord(e1, s)) || (e = hipEventSynchronize(e1)) ||
                        (e = hipEventElapsedTime(&ms, e0, e1)))
                        fail(e, "autotune timing");
                }
                if (rc != SSP_OK) break;
                if (best_t == 0 || ms < best) {
                    best = ms;
                    best_t = t;
                    best_l = l;
                }
            }
            if (rc != SSP_OK) break;
        }
        g.threads = best_t;
        g.lds = best_l;
        g.tuned_ms = best;
    }
    // leave valid results of the chosen mapping in the outputs
    if (rc == SSP_OK &&
        (e = hipMemcpyAsync(prob_status, st0, sizeof(int32_t) * b->P, hipMemcpyDeviceToDevice, s)))
        fail(e, "status restore");
    if (rc == SSP_OK) rc = launch_groups(b, a, -1, s);
    if (rc == SSP_OK && (e = hipStreamSynchronize(s))) fail(e, "hipStreamSynchronize");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(st0);
    return rc;
}

ssp_status ssp_set_group_mapping(ssp_batch *b, int32_t nx, int32_t threads, int32_t lds_bytes) {
    if (!b) return SSP_ERR_ARG;
    for (auto &g : b->groups) {
        if (g.nx != nx) continue;
        if (threads == 0 && lds_bytes == 0) {
            g.threads = g.lds = 0;
            return SSP_OK;
        }
        if (!ssp::pcg2_threads_ok(threads) || lds_bytes < ssp::bt_sweep_min_lds(nx, true, 8) ||
            lds_bytes > ssp::kFusedLdsCap || ssp::pcg2_steps_for(nx, b->fp32, threads, lds_bytes) < 1)
            return SSP_ERR_ARG;
        g.threads = threads;
        g.lds = lds_bytes;
        g.tuned_ms = 0.0f;
        return SSP_OK;
    }
    return SSP_ERR_ARG;
}

ssp_status ssp_get_mapping(const ssp_batch *b, int32_t max_groups, int32_t *nx, int32_t *threads,
                           int32_t *lds_bytes, float *tuned_ms, int32_t *ngroups) {
    if (!b || !ngroups || max_groups < 0) return SSP_ERR_ARG;
    const int ng = (int)b->groups.size();
    *ngroups = ng;
    for (int i = 0; i < ng && i < max_groups; ++i) {
        int t, l;
        group_mapping(b, b->groups[i], &t, &l);
        if (nx) nx[i] = b->groups[i].nx;
        if (threads) threads[i] = t;
        if (lds_bytes) lds_bytes[i] = l;
        if (tuned_ms) tuned_ms[i] = b->groups[i].tuned_ms;
    }
    return SSP_OK;
}

ssp_status ssp_kkt_rhs(ssp_batch *b, const double *A, const double *B, const double *q, const double *r,
                       const double *c, double *gamma, void *stream) {
    if (!b || !A || !q || !c || !gamma) return SSP_ERR_ARG;
    if (b->nu_max > 0 && (!B || !r)) return SSP_ERR_ARG;
    if (!b->built || !b->have_qr) {
        g_last_error = "ssp_kkt_rhs needs a preceding ssp_build that kept Q^-1, R^-1 (ssp_set_keep_inverses)";
        return SSP_ERR_STATE;
    }
    DevGuard g(b->device);
    ssp::BuildArgs a = build_args(b);
    a.A = A;
    a.B = B;
    for (int cls = 0; cls <= ssp::kKktClasses; ++cls)
        SSP_HIP(ssp::launch_kkt_rhs(cls < ssp::kKktClasses ? cls : -1, a, b->dkkt + b->kkt_off[cls],
                                    b->dkktrec + b->kkt_off[cls], b->kkt_off[cls + 1] - b->kkt_off[cls], b->doff_v,
                                    b->doff_u, q, r, c, gamma,
                                    (hipStream_t)stream));
    return SSP_OK;
}

ssp_status ssp_kkt_recover(ssp_batch *b, const double *A, const double *B, const double *q, const double *r,
                           const double *lambda, double *dx, double *du, void *stream) {
    if (!b || !A || !q || !lambda || !dx) return SSP_ERR_ARG;
    if (b->nu_max > 0 && (!B || !r || !du)) return SSP_ERR_ARG;
    if (!b->built || !b->have_qr) {
        g_last_error = "ssp_kkt_recover needs a preceding ssp_build that kept Q^-1, R^-1 (ssp_set_keep_inverses)";
        return SSP_ERR_STATE;
    }
    DevGuard g(b->device);
    ssp::BuildArgs a = build_args(b);
    a.A = A;
    a.B = B;
    for (int cls = 0; cls <= ssp::kKktClasses; ++cls)
        SSP_HIP(ssp::launch_kkt_recover(cls < ssp::kKktClasses ? cls : -1, a, b->dkkt + b->kkt_off[cls],
                                        b->dkktrec + b->kkt_off[cls], b->kkt_off[cls + 1] - b->kkt_off[cls],
                                        b->doff_v, b->doff_u, q, r, lambda, dx,
                                        du, (hipStream_t)stream));
    return SSP_OK;
}

ssp_status ssp_set_keep_inverses(ssp_batch *b, int32_t on) {
    if (!b || (on != 0 && on != 1)) return SSP_ERR_ARG;
    b->keep_qr = on;
    return SSP_OK;
}

ssp_status ssp_set_reduction_fp64(ssp_batch *b, int32_t on) {
    if (!b || (on != 0 && on != 1)) return SSP_ERR_ARG;
    b->acc64 = on;
    return SSP_OK;
}

ssp_status ssp_set_scaled_mapping(ssp_batch *b, int32_t threads, int32_t lds_bytes) {
    if (!b) return SSP_ERR_ARG;
    if (threads == 0 && lds_bytes == 0) {
        b->s3_threads = 256;
        b->s3_lds = 0;
        b->s3_tuned_ms = 0.0f;
        return SSP_OK;
    }
    if ((threads != 128 && threads != 256) || lds_bytes < 0 || lds_bytes > ssp::kFusedLdsCap) return SSP_ERR_ARG;
    const int m = poly_steps(b->pc);
    const int l = lds_bytes > 0 ? lds_bytes : 0;
    const int prev_t = b->s3_threads, prev_l = b->s3_lds;
    b->s3_threads = threads;
    b->s3_lds = l;
    if (!scaled_possible(b) || !scaled_fits(b, threads, scaled_lds(b, threads, m), m)) {
        b->s3_threads = prev_t;
        b->s3_lds = prev_l;
        return SSP_ERR_ARG;
    }
    b->s3_tuned_ms = 0.0f;
    return SSP_OK;
}

ssp_status ssp_scaled_onchip_horizon(int32_t nx, ssp_precon pc, ssp_precision prec, int32_t threads,
                                     int32_t lds_bytes, int32_t *max_n) {
    if (!max_n || pc < SSP_PC_BLOCK_JACOBI || pc > SSP_PC_NEUMANN3) return SSP_ERR_ARG;
    if (prec < SSP_FP64 || prec > SSP_FP32_REFINE64) return SSP_ERR_ARG;
    // scalar Jacobi never runs the scaled solve
    *max_n = pc == SSP_PC_SCALAR_JACOBI ? 0
                                        : ssp::pcg3_onchip_horizon(nx, prec != SSP_FP64, threads, lds_bytes, poly_steps(pc));
    return SSP_OK;
}

ssp_status ssp_get_scaled_mapping(const ssp_batch *b, int32_t *threads, int32_t *lds_bytes, int32_t *grid,
                                  float *tuned_ms) {
    if (!b) return SSP_ERR_ARG;
    const int t = b->s3_threads, m = poly_steps(b->pc);
    const int l = scaled_lds(b, t, m);
    if (threads) *threads = t;
    if (lds_bytes) *lds_bytes = l;
    if (tuned_ms) *tuned_ms = b->s3_tuned_ms;
    if (grid) {
        DevGuard g(b->device);
        int cus = 0;
        const int occ = ssp::pcg3_occupancy(b->fp32, t, l, &cus, b->fp32 && b->acc64, b->groups[0].nx);
        *grid = std::min(occ * cus, b->P);
    }
    return SSP_OK;
}

ssp_status ssp_solve_kernel(const ssp_batch *b, int32_t *kernel, int32_t *W, int32_t *G) {
    if (!b || !kernel) return SSP_ERR_ARG;
    *kernel = b->last_kernel;
    if (W) *W = b->last_kernel == 3 ? b->coop_W : 0;
    if (G) *G = b->last_kernel == 3 ? b->coop_G : 0;
    return SSP_OK;
}

}  // extern "C"
