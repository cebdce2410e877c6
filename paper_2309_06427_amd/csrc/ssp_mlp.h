// Warm-start network kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssp {

// One knot of a feature set: element offset of its run in the stored array
// (D_k packed, then L_k at +lofs), offset of its rows in the vector layout,
// and whether it is the first / last knot of its problem.
struct KnotInfo {
    int64_t blk;
    int64_t vec;
    int32_t first, last;
};

// Knots whose inputs are read: M knots of state size nx from the stored
// blocks (storage type float when fp32, else double; L_k at lofs after the
// start of a knot's run).
struct FeatSrc {
    const void *B3;
    bool fp32;
    const double *gamma;
    const KnotInfo *ki;
    int M, nx, lofs;
};

// Parameter layout (floats): W1 (nin x H), b1, W2 (H x H), b2, W3 (H x nx), b3.
struct NetView {
    int nin, H, nx;
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};

// knot_prob / koff / N / off_b3 / off_v: batch metadata (device); ks: knot
// stride of the stored array.  Knot m is list[m] when list != null, else g0 + m.
hipError_t launch_knot_info(const int32_t *knot_prob, const int64_t *koff, const int32_t *N, const int64_t *off_b3,
                            const int64_t *off_v, const int32_t *list, int64_t g0, int M, int nx, int ks,
                            KnotInfo *out, hipStream_t s);

// Per-feature mean and 1 / max(std, 1e-6) of the inputs of f's knots, and the
// root mean square of the labels lam (vector layout) at those knots.
// part: 2 * 64 * (nin + nx) doubles of scratch.
hipError_t launch_feature_stats(const FeatSrc &f, const double *lam, float *mu, float *inv_sd, float *y_scale,
                                double *part, hipStream_t s);

// Forward pass.  Z1/Z2 (pre-activations, may be null when not training),
// H1/H2: M x H.  O: M x nx network outputs (may be null); lambda: when not
// null, y_scale * O is written to lambda at each knot's rows (FP64).
hipError_t launch_mlp_forward(const FeatSrc &f, const NetView &w, const float *mu, const float *inv_sd, float y_scale,
                              float *Z1, float *H1, float *Z2, float *H2, float *O, double *lambda, hipStream_t s);

// Residual loss and output gradient over whole problems: E = y_scale O - lam*,
// R = S E, loss += sum R^2 / nprob (into loss[0], FP64), dO = y_scale (2 / nprob) S R.
// E, R, dO: M x nx; part: >= ceil(M * nx / 256) doubles.
hipError_t launch_mlp_loss(const FeatSrc &f, const float *O, float y_scale, const double *lam_star, int nprob,
                           float *E, float *R, float *dO, double *part, double *loss, hipStream_t s);

// Backward pass into grad (parameter layout); dZ2, dZ1: M x H scratch;
// split: K-split partials, 'splits' * (nin * H) floats.
hipError_t launch_mlp_backward(const FeatSrc &f, const NetView &w, const float *mu, const float *inv_sd,
                               const float *Z1, const float *H1, const float *Z2, const float *H2, const float *dO,
                               float *dZ2, float *dZ1, float *grad, float *split, int splits, hipStream_t s);

hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int64_t n, float lr, float beta1,
                       float beta2, float eps, float bc1, float bc2, hipStream_t s);

// Plain FP32 GEMM C (M x N) = op(A) op(B) with A, B row-major (test hook).
hipError_t launch_gemm_f32(int M, int N, int K, const float *A, int lda, bool ta, const float *B, int ldb, bool tb,
                           float *C, int ldc, hipStream_t s);

}  // namespace ssp
