// Host side of the warm-start network entry points of include/symstair.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/symstair.h"
#include "ssp_batch.h"
#include "ssp_mlp.h"
#include "ssp_sweep.h"

using namespace ssp_host;

struct ssp_mlp {
    int device = 0;
    int nx = 0, H = 0, nin = 0;
    int64_t np = 0;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *mu = nullptr, *isd = nullptr;
    float *ys_dev = nullptr;
    float ys = 1.0f;
    int64_t t = 0;  // Adam steps taken
    // scratch sized for `cap` knots
    int cap = 0, splits = 16;
    ssp::KnotInfo *ki = nullptr;
    float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *dZ1 = nullptr, *dZ2 = nullptr;
    float *O = nullptr, *E = nullptr, *R = nullptr, *dO = nullptr, *split = nullptr;
    double *part = nullptr, *loss = nullptr;
};

namespace {

constexpr int kPredictChunk = 65536;  // knots per inference pass (bounds the activation scratch)

void free_scratch(ssp_mlp *m) {
    for (void *p : {(void *)m->ki, (void *)m->Z1, (void *)m->H1, (void *)m->Z2, (void *)m->H2, (void *)m->dZ1,
                    (void *)m->dZ2, (void *)m->O, (void *)m->E, (void *)m->R, (void *)m->dO, (void *)m->split,
                    (void *)m->part})
        if (p) (void)hipFree(p);
    m->ki = nullptr;
    m->Z1 = m->H1 = m->Z2 = m->H2 = m->dZ1 = m->dZ2 = m->O = m->E = m->R = m->dO = m->split = nullptr;
    m->part = nullptr;
    m->cap = 0;
}

ssp_status ensure_scratch(ssp_mlp *m, int knots) {
    if (knots <= m->cap) return SSP_OK;
    // the stream may still use the old buffers
    SSP_HIP(hipDeviceSynchronize());
    free_scratch(m);
    const size_t M = (size_t)knots, H = m->H, nx = m->nx;
    const size_t big = std::max({(size_t)m->nin * H, H * H, H * nx});
    const size_t npart = std::max((M * nx + 255) / 256 + 1, (size_t)2 * 64 * (m->nin + nx));
    bool ok = dalloc(&m->ki, M) == hipSuccess;
    for (float **p : {&m->Z1, &m->H1, &m->Z2, &m->H2, &m->dZ1, &m->dZ2}) ok = ok && dalloc(p, M * H) == hipSuccess;
    for (float **p : {&m->O, &m->E, &m->R, &m->dO}) ok = ok && dalloc(p, M * nx) == hipSuccess;
    ok = ok && dalloc(&m->split, (size_t)m->splits * big) == hipSuccess;
    ok = ok && dalloc(&m->part, npart) == hipSuccess;
    if (!ok) {
        free_scratch(m);
        g_last_error = "hipMalloc of warm-start scratch failed";
        return SSP_ERR_ALLOC;
    }
    m->cap = knots;
    return SSP_OK;
}

ssp::NetView view(const ssp_mlp *m) {
    ssp::NetView w;
    w.nin = m->nin;
    w.H = m->H;
    w.nx = m->nx;
    w.W1 = m->theta;
    w.b1 = w.W1 + (int64_t)m->nin * m->H;
    w.W2 = w.b1 + m->H;
    w.b2 = w.W2 + (int64_t)m->H * m->H;
    w.W3 = w.b2 + m->H;
    w.b3 = w.W3 + (int64_t)m->H * m->nx;
    return w;
}

// device list of the global knots of problems with state size nx (cached)
ssp_status nx_knots(ssp_batch *b, int nx, const int32_t **list, int64_t *count) {
    for (auto &e : b->nx_knots)
        if (e.first == nx) {
            *list = e.second.first;
            *count = e.second.second;
            return SSP_OK;
        }
    std::vector<int32_t> ks;
    for (int p = 0; p < b->P; ++p)
        if (b->nx[p] == nx)
            for (int64_t g = b->koff[p]; g < b->koff[p + 1]; ++g) ks.push_back((int32_t)g);
    int32_t *d = nullptr;
    if (!ks.empty()) {
        if (dalloc(&d, ks.size()) != hipSuccess) {
            g_last_error = "hipMalloc of knot list failed";
            return SSP_ERR_ALLOC;
        }
        SSP_HIP(hipMemcpy(d, ks.data(), ks.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    b->nx_knots.push_back({nx, {d, (int64_t)ks.size()}});
    *list = d;
    *count = (int64_t)ks.size();
    return SSP_OK;
}

ssp::FeatSrc feat_src(const ssp_batch *b, const ssp_mlp *m, const double *gamma, int M) {
    ssp::FeatSrc f;
    f.B3 = b->B3;
    f.fp32 = b->fp32;
    f.gamma = gamma;
    f.ki = m->ki;
    f.M = M;
    f.nx = m->nx;
    f.lofs = ssp::packed_stride(m->nx, b->fp32 ? 4 : 8);  // L_k after the packed D_k
    return f;
}

ssp_status knot_info(const ssp_batch *b, ssp_mlp *m, const int32_t *list, int64_t g0, int M, hipStream_t s) {
    SSP_HIP(ssp::launch_knot_info(b->dknot, b->dkoff, b->dN, b->fp32 ? b->doff_b3_32 : b->doff_b3_64, b->doff_v,
                                  list, g0, M, m->nx, ssp::knot_stride(m->nx, b->fp32 ? 4 : 8), m->ki, s));
    return SSP_OK;
}

}  // namespace

extern "C" {

int64_t ssp_mlp_num_params(int32_t nx, int32_t hidden) {
    if (nx < 1 || nx > 64 || hidden < 1) return -1;
    const int64_t nin = 2ll * nx * nx + nx, H = hidden;
    return nin * H + H + H * H + H + H * nx + nx;
}

ssp_status ssp_mlp_create(int32_t nx, int32_t hidden, int device, ssp_mlp **out) {
    if (!out) return SSP_ERR_ARG;
    *out = nullptr;
    if (nx < 1 || nx > 64 || hidden < 16 || hidden > 512 || hidden % 16) return SSP_ERR_ARG;
    int ndev = 0;
    SSP_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return SSP_ERR_ARG;
    ssp_mlp *m = new (std::nothrow) ssp_mlp();
    if (!m) return SSP_ERR_ALLOC;
    m->device = device;
    m->nx = nx;
    m->H = hidden;
    m->nin = 2 * nx * nx + nx;
    m->np = ssp_mlp_num_params(nx, hidden);
    DevGuard g(device);
    bool ok = true;
    for (float **p : {&m->theta, &m->m, &m->v, &m->grad}) ok = ok && dalloc(p, (size_t)m->np) == hipSuccess;
    ok = ok && dalloc(&m->mu, (size_t)m->nin) == hipSuccess && dalloc(&m->isd, (size_t)m->nin) == hipSuccess;
    ok = ok && dalloc(&m->ys_dev, 1) == hipSuccess && dalloc(&m->loss, 1) == hipSuccess;
    if (ok) {
        ok = hipMemset(m->theta, 0, m->np * 4) == hipSuccess && hipMemset(m->m, 0, m->np * 4) == hipSuccess &&
             hipMemset(m->v, 0, m->np * 4) == hipSuccess && hipMemset(m->mu, 0, m->nin * 4) == hipSuccess;
        std::vector<float> one((size_t)m->nin, 1.0f);
        ok = ok && hipMemcpy(m->isd, one.data(), m->nin * 4, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        g_last_error = "hipMalloc of warm-start network failed";
        ssp_mlp_destroy(m);
        return SSP_ERR_ALLOC;
    }
    *out = m;
    return SSP_OK;
}

ssp_status ssp_mlp_destroy(ssp_mlp *m) {
    if (!m) return SSP_OK;
    {
        DevGuard g(m->device);
        (void)hipDeviceSynchronize();
        free_scratch(m);
        for (void *p : {(void *)m->theta, (void *)m->m, (void *)m->v, (void *)m->grad, (void *)m->mu, (void *)m->isd,
                        (void *)m->ys_dev, (void *)m->loss})
            if (p) (void)hipFree(p);
    }
    delete m;
    return SSP_OK;
}

ssp_status ssp_mlp_set_params(ssp_mlp *m, const float *theta, void *stream) {
    if (!m || !theta) return SSP_ERR_ARG;
    DevGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    SSP_HIP(hipMemcpyAsync(m->theta, theta, m->np * 4, hipMemcpyDeviceToDevice, s));
    SSP_HIP(hipMemsetAsync(m->m, 0, m->np * 4, s));
    SSP_HIP(hipMemsetAsync(m->v, 0, m->np * 4, s));
    m->t = 0;
    return SSP_OK;
}

ssp_status ssp_mlp_get_params(const ssp_mlp *m, float *theta, float *grad, void *stream) {
    if (!m || (!theta && !grad)) return SSP_ERR_ARG;
    DevGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    if (theta) SSP_HIP(hipMemcpyAsync(theta, m->theta, m->np * 4, hipMemcpyDeviceToDevice, s));
    if (grad) SSP_HIP(hipMemcpyAsync(grad, m->grad, m->np * 4, hipMemcpyDeviceToDevice, s));
    return SSP_OK;
}

ssp_status ssp_mlp_set_scaling(ssp_mlp *m, const float *mu, const float *inv_sd, float y_scale, void *stream) {
    if (!m || !mu || !inv_sd || !(y_scale > 0.0f)) return SSP_ERR_ARG;
    DevGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    SSP_HIP(hipMemcpyAsync(m->mu, mu, m->nin * 4, hipMemcpyDeviceToDevice, s));
    SSP_HIP(hipMemcpyAsync(m->isd, inv_sd, m->nin * 4, hipMemcpyDeviceToDevice, s));
    m->ys = y_scale;
    return SSP_OK;
}

ssp_status ssp_mlp_get_scaling(const ssp_mlp *m, float *mu, float *inv_sd, float *y_scale, void *stream) {
    if (!m || !mu || !inv_sd || !y_scale) return SSP_ERR_ARG;
    DevGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    SSP_HIP(hipMemcpyAsync(mu, m->mu, m->nin * 4, hipMemcpyDeviceToDevice, s));
    SSP_HIP(hipMemcpyAsync(inv_sd, m->isd, m->nin * 4, hipMemcpyDeviceToDevice, s));
    *y_scale = m->ys;
    return SSP_OK;
}

ssp_status ssp_mlp_fit_scaling(ssp_mlp *m, ssp_batch *b, const double *gamma, const double *lambda_star,
                               void *stream) {
    if (!m || !b || !gamma || !lambda_star) return SSP_ERR_ARG;
    if (!b->built || b->device != m->device) return SSP_ERR_STATE;
    DevGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    const int32_t *list = nullptr;
    int64_t cnt = 0;
    ssp_status rc = nx_knots(b, m->nx, &list, &cnt);
    if (rc != SSP_OK) return rc;
    if (cnt == 0 || cnt > INT32_MAX) return SSP_ERR_ARG;
    // knot info for every knot of the class (one pass; the scratch grows to hold it)
    if ((rc = ensure_scratch(m, (int)std::min<int64_t>(cnt, kPredictChunk))) != SSP_OK) return rc;
    ssp::KnotInfo *all = nullptr;
    if (dalloc(&all, (size_t)cnt) != hipSuccess) {
        g_last_error = "hipMalloc of knot info failed";
        return SSP_ERR_ALLOC;
    }
    SSP_HIP(ssp::launch_knot_info(b->dknot, b->dkoff, b->dN, b->fp32 ? b->doff_b3_32 : b->doff_b3_64, b->doff_v,
                                  list, 0, (int)cnt, m->nx, ssp::knot_stride(m->nx, b->fp32 ? 4 : 8), all, s));
    ssp::FeatSrc f = feat_src(b, m, gamma, (int)cnt);
    f.ki = all;
    hipError_t e = ssp::launch_feature_stats(f, lambda_star, m->mu, m->isd, m->ys_dev, m->part, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&m->ys, m->ys_dev, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(all);
    if (e != hipSuccess) return hip_fail(e, "feature statistics");
    return SSP_OK;
}

ssp_status ssp_mlp_predict(ssp_mlp *m, ssp_batch *b, const double *gamma, double *lambda0, void *stream) {
    if (!m || !b || !gamma || !lambda0) return SSP_ERR_ARG;
    if (!b->built || b->device != m->device) return SSP_ERR_STATE;
    DevGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    const int32_t *list = nullptr;
    int64_t cnt = 0;
    ssp_status rc = nx_knots(b, m->nx, &list, &cnt);
    if (rc != SSP_OK) return rc;
    if (cnt == 0) return SSP_OK;
    if ((rc = ensure_scratch(m, (int)std::min<int64_t>(cnt, kPredictChunk))) != SSP_OK) return rc;
    const ssp::NetView w = view(m);
    for (int64_t c0 = 0; c0 < cnt; c0 += m->cap) {
        const int M = (int)std::min<int64_t>(m->cap, cnt - c0);
        if ((rc = knot_info(b, m, list + c0, 0, M, s)) != SSP_OK) return rc;
        SSP_HIP(ssp::launch_mlp_forward(feat_src(b, m, gamma, M), w, m->mu, m->isd, m->ys, nullptr, m->H1, nullptr,
                                        m->H2, nullptr, lambda0, s));
    }
    return SSP_OK;
}

ssp_status ssp_mlp_loss_grad(ssp_mlp *m, ssp_batch *b, int32_t p0, int32_t p1, const double *gamma,
                             const double *lambda_star, double *loss, void *stream) {
    if (!m || !b || !gamma || !lambda_star) return SSP_ERR_ARG;
    if (!b->built || b->device != m->device) return SSP_ERR_STATE;
    if (p0 < 0 || p1 > b->P || p0 >= p1) return SSP_ERR_ARG;
    for (int p = p0; p < p1; ++p)
        if (b->nx[p] != m->nx) return SSP_ERR_ARG;
    const int64_t M64 = b->koff[p1] - b->koff[p0];
    if (M64 > (1 << 24)) return SSP_ERR_ARG;
    const int M = (int)M64;
    DevGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    ssp_status rc = ensure_scratch(m, M);
    if (rc != SSP_OK) return rc;
    if ((rc = knot_info(b, m, nullptr, b->koff[p0], M, s)) != SSP_OK) return rc;
    const ssp::FeatSrc f = feat_src(b, m, gamma, M);
    const ssp::NetView w = view(m);
    SSP_HIP(ssp::launch_mlp_forward(f, w, m->mu, m->isd, m->ys, m->Z1, m->H1, m->Z2, m->H2, m->O, nullptr, s));
    SSP_HIP(ssp::launch_mlp_loss(f, m->O, m->ys, lambda_star, p1 - p0, m->E, m->R, m->dO, m->part, m->loss, s));
    SSP_HIP(ssp::launch_mlp_backward(f, w, m->mu, m->isd, m->Z1, m->H1, m->Z2, m->H2, m->dO, m->dZ2, m->dZ1, m->grad,
                                     m->split, m->splits, s));
    if (loss) SSP_HIP(hipMemcpyAsync(loss, m->loss, sizeof(double), hipMemcpyDeviceToDevice, s));
    return SSP_OK;
}

ssp_status ssp_mlp_adam(ssp_mlp *m, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!m || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return SSP_ERR_ARG;
    DevGuard g(m->device);
    m->t += 1;
    const double bc1 = 1.0 - std::pow((double)beta1, (double)m->t), bc2 = 1.0 - std::pow((double)beta2, (double)m->t);
    SSP_HIP(ssp::launch_adam(m->theta, m->grad, m->m, m->v, m->np, lr, beta1, beta2, eps, (float)bc1, (float)bc2,
                             (hipStream_t)stream));
    return SSP_OK;
}

ssp_status ssp_mlp_get_state(const ssp_mlp *m, float *m1, float *m2, int64_t *steps, void *stream) {
    if (!m || !steps) return SSP_ERR_ARG;
    DevGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    if (m1) SSP_HIP(hipMemcpyAsync(m1, m->m, sizeof(float) * m->np, hipMemcpyDeviceToDevice, s));
    if (m2) SSP_HIP(hipMemcpyAsync(m2, m->v, sizeof(float) * m->np, hipMemcpyDeviceToDevice, s));
    *steps = m->t;
    return SSP_OK;
}

ssp_status ssp_mlp_set_state(ssp_mlp *m, const float *m1, const float *m2, int64_t steps, void *stream) {
    if (!m || !m1 || !m2 || steps < 0) return SSP_ERR_ARG;
    DevGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    SSP_HIP(hipMemcpyAsync(m->m, m1, sizeof(float) * m->np, hipMemcpyDeviceToDevice, s));
    SSP_HIP(hipMemcpyAsync(m->v, m2, sizeof(float) * m->np, hipMemcpyDeviceToDevice, s));
    m->t = steps;
    return SSP_OK;
}

ssp_status ssp_gemm_f32(int32_t M, int32_t N, int32_t K, const float *A, int32_t lda, int32_t trans_a,
                        const float *B, int32_t ldb, int32_t trans_b, float *C, int32_t ldc, void *stream) {
    if (M < 0 || N < 0 || K < 0 || !A || !B || !C) return SSP_ERR_ARG;
    SSP_HIP(ssp::launch_gemm_f32(M, N, K, A, lda, trans_a != 0, B, ldb, trans_b != 0, C, ldc, (hipStream_t)stream));
    return SSP_OK;
}

}  // extern "C"
