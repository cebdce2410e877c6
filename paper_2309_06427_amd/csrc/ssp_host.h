// Kernel argument blocks and launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssp {

struct BuildArgs {
    const int32_t *N, *nx, *nu;
    const int64_t *off_nn, *off_nu, *off_uu;
    const int32_t *knot_prob;  // global knot index -> problem
    const int64_t *koff;       // problem -> first global knot
    const double *A, *B, *Q, *R;
    double *Qinv, *Rinv, *L64, *Dinv64;  // FP64 workspaces (layout of A/Q, R)
    void *SD, *SL;                       // S diagonal / sub-diagonal blocks (storage type)
    float *SDlo, *SLlo;                  // FP64 remainders under FP32 storage (else null)
    void *PD, *PM;                       // Phi^-1 diagonal / sub-diagonal (PM null: block-Jacobi)
    int32_t *status;
    int pc;  // 0 block-Jacobi, 1 additive stair, 2 symmetric stair
    int mx;  // max(nx, nu) over the batch
};

struct SolveArgs {
    const int32_t *order;  // workgroup -> problem (largest first)
    const int32_t *N, *nx;
    const int64_t *off_nn, *off_v;
    int32_t *status;
    const void *SD, *SL;
    const float *SDlo, *SLlo;
    const void *PD, *PM;
    const double *gamma;
    double *lambda;
    int use_lambda0;
    double tol;
    int max_iter;  // <= 0: 10 * N * nx
    int max_outer;
    int refine;
    double theta, tau_min;
    int32_t *iters, *outer;
    double *relres;
    void *work;    // 7 vectors of the inner precision, each tot_v long
    double *r64;   // FP64 residual, tot_v long
    int64_t tot_v;
    int lds_bytes;
};

hipError_t launch_build(const BuildArgs &a, int64_t knots, int nx_max, int nu_max, bool fp32, hipStream_t s);
hipError_t launch_export(const void *hi, const float *lo, bool fp32, double *dst, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t *dst, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double *dst, double v, int64_t n, hipStream_t s);
hipError_t launch_pcg(const SolveArgs &a, int nprob, bool fp32, int threads, hipStream_t s);

// Smallest LDS budget the PCG kernel accepts for a batch whose largest state
// size is nx_max (one knot staged in FP64 plus the neighbour blocks).
int pcg_min_lds(int nx_max, bool has_sub);
// Default LDS budget for a mapping.
int pcg_default_lds(int nx_max, bool fp32, int threads);

}  // namespace ssp
