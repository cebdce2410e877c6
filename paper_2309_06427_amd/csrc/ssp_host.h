// Kernel argument blocks and launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssp {

// One work item (problem, first knot) of the DPP assembly kernels with its
// problem's horizon and offsets, so that a wave's first loads depend on one
// round of scalar loads (the offsets are not looked up through the problem
// index); both storage precisions' block offsets are kept.
struct alignas(16) BuildRec {
    int32_t pr, k0, N, pad;
    int64_t onn, onu, ouu, opk, oblk32, oblk64, ob3_32, ob3_64;
};

struct BuildArgs {
    const int32_t *N, *nx, *nu;
    const int64_t *off_nn, *off_nu, *off_uu;  // input (caller) layout
    const int64_t *off_blk;                   // full-block layout: sum of N bs (L remainders, explicit blocks)
    const int64_t *off_b3;                    // solve array: sum of N knot_stride
    const int64_t *off_pk;                    // packed-block layout: sum of N packed_stride (D remainders)
    const int32_t *knot_prob;                 // global knot index -> problem
    const int64_t *koff;                      // problem -> first global knot
    const int32_t *knot_list;                 // generic assembly: workgroup -> global knot
    const double *A, *B, *Q, *R;
    double *Qinv, *Rinv;  // FP64 workspaces (layout of Q, R)
    void *B3;            // per knot k: D_k (packed), L_k (full), D_k^-1 (packed), storage type
    float *SDlo, *SLlo;  // FP64 remainders of D_k (packed stride), L_k (stride bs) under FP32 storage
    void *PM;           // explicit Phi^-1[k][k-1] blocks (stride bs; null: not built)
    // scaled basis (null: not built): W_k = C_k^-1 with D_k = C_k C_k^T
    // (lower triangular) and Oh_k = W_k L_k W_{k-1}^T (stride bs, storage
    // type); the stored D_k^-1 is then not written
    void *Zs, *OH;
    int32_t *status;
    int pc;  // 0 block-Jacobi, 1 additive stair, 2 symmetric stair, 3 scalar Jacobi, 4/5 Neumann degree 2/3
    int mx;  // max(nx, nu) over the batch
    int keep_qr;  // store Q_k^-1, R_k^-1 in Qinv, Rinv (the KKT step reads them)
    const BuildRec *brec;  // DPP classes: the launched class's item records, in the order of its items
};

struct SolveArgs {
    const int32_t *order;  // workgroup -> problem (largest first)
    const int32_t *N, *nx;
    const int64_t *off_blk, *off_v;  // full-block layout (L remainders, explicit blocks), vectors
    const int64_t *off_b3, *off_pk;  // solve array, packed-block layout (D remainders)
    int32_t *status;
    const void *B3;            // per knot: D (packed), L, D^-1 (packed)
    const float *SDlo, *SLlo;  // FP64 remainders of D (packed stride), L (stride bs)
    const void *PM;            // explicit sub-diagonal blocks (explicit kernel only)
    int pc;               // 0 block-Jacobi, 1 additive stair, 2 symmetric stair
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
    // scaled solve (congruence basis, persistent grid)
    const void *OH, *Z;  // Oh_k and W_k blocks (stride bs, full-block layout off_blk)
    double *rh64;        // FP64 residual in the scaled basis, W r, tot_v long
    unsigned *queue;     // next position in `order` (zeroed before every launch)
    int nprob;           // problems in the queue
    int poly;            // Horner steps m of the preconditioner polynomial in Oh (0: block-Jacobi)
    double pc_c;         // coefficient of each Horner step (1; 1/2 for the additive stair)
    int acc64;           // scaled solve: sum the FP32 inner products in FP64
};

// Generic assembly (any nx <= 64), one 64-lane workgroup per knot of
// a.knot_list[0 .. knots).
hipError_t launch_build(const BuildArgs &a, int64_t knots, int nx_max, int nu_max, bool fp32, hipStream_t s);
// Register-resident assembly for the state sizes kBuildSizes: class
// build_class_of(nx, nu) (-1: the generic kernels); a work item (problem,
// first knot) of class c covers build_knots_per_item(c) knots.
constexpr int kBuildClasses = 7;
extern const int kBuildSizes[kBuildClasses];
int build_class_of(int nx, int nu);
int build_knots_per_item(int cls);
hipError_t launch_build_class(int cls, const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s);
// Scaled basis for one class, after launch_build_class wrote W_k (a.Zs) and
// L_k: Oh_k = W_k L_k W_{k-1}^T for the same work items.
hipError_t launch_build_ohat(int cls, const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s);
// The same two steps with DPP-broadcast kernels (state sizes up to 32, one
// knot per 16-lane row, dpp_knots_per_item() knots per work item).
int dpp_knots_per_item();
template <int NX>
hipError_t launch_dpp_class(const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s);
template <int NX>
hipError_t launch_dpp_ohat(const BuildArgs &a, const int2 *items, int nitems, bool fp32, hipStream_t s);
// D_k^-1 = W_k^T W_k into the stored D_k^-1 slots after a scaled build
// (from the FP64 W of a.Zw), for the consumers of D^-1 (export, explicit
// stair blocks).
hipError_t launch_dinv_from_w(const BuildArgs &a, int64_t knots, int nx_max, bool fp32, hipStream_t s);
// Scalar Jacobi: overwrite every stored D_k^-1 with diag(1 / (D_k)_ii).
hipError_t launch_jacobi_diag(const BuildArgs &a, int64_t knots, bool fp32, hipStream_t s);
// S from caller-given blocks D_k, L_k (every knot of the batch): stored D,
// L and D^-1 as the assembly stores them.
hipError_t launch_build_blocks(const BuildArgs &a, const double *D, const double *Lsub, int64_t knots, bool fp32,
                               hipStream_t s);
// Explicit stair blocks from the stored D^-1 and L (every knot of the batch).
hipError_t launch_build_phi(const BuildArgs &a, int64_t knots, int nx_max, bool fp32, hipStream_t s);
// Copy one stored block kind to the caller's FP64 layout (full nx x nx
// blocks at off_nn): which = 0 D_k (+ packed remainder lo), 1 L_k (+ lo),
// 2 D_k^-1, 3 the explicit stair blocks (array `hi`, stride bs).
hipError_t launch_export(const BuildArgs &a, int which, const void *hi, const float *lo, bool fp32, double *dst,
                         int64_t knots, hipStream_t s);
hipError_t launch_fill_i32(int32_t *dst, int32_t v, int64_t n, hipStream_t s);

// KKT step around the solve (FP64): gamma from q, r, c, and dx, du from
// lambda, with the Q^-1, R^-1 of the last build (a.Qinv, a.Rinv) and the
// caller's A, B (a.A, a.B), for the n work items (problem p, first knot k0)
// of `items`: the knots k0 .. min(k0 + kkt_knots_per_item(cls), N) - 1.
// Vector offsets: off_v (state, N nx per problem), off_u (control, N nu
// per problem).  Class kkt_class_of(nx, nu) of every item's problem picks
// the kernel compiled for state size kKktSizes[cls] (nu <= nx / 2), -1 the
// generic one (any nx, nu <= 64; one knot per item).
// One work item of the staged KKT kernels with everything a wave needs
// before its block loads: one 64-byte record, a single scalar load (the
// problem's sizes and offsets are not looked up through the problem index).
struct alignas(16) KktRec {
    int32_t p, k0, N, nu;
    int64_t onn, ov, ou, onu, ouu, pad;
};
constexpr int kKktClasses = 3;
extern const int kKktSizes[kKktClasses];
int kkt_class_of(int nx, int nu);
int kkt_knots_per_item(int cls);
hipError_t launch_kkt_rhs(int cls, const BuildArgs &a, const int2 *list, const KktRec *recs, int64_t n,
                          const int64_t *off_v, const int64_t *off_u, const double *q, const double *r,
                          const double *c, double *gamma, hipStream_t s);
hipError_t launch_kkt_recover(int cls, const BuildArgs &a, const int2 *list, const KktRec *recs, int64_t n,
                              const int64_t *off_v, const int64_t *off_u, const double *q, const double *r,
                              const double *lam, double *dx, double *du, hipStream_t s);
hipError_t launch_fill_f64(double *dst, double v, int64_t n, hipStream_t s);

// Explicit two-sweep PCG (stored Phi^-1 blocks).
hipError_t launch_pcg(const SolveArgs &a, int nprob, bool fp32, int threads, hipStream_t s);
int pcg_min_lds(int nx_max, bool has_sub);
int pcg_default_lds(int nx_max, bool fp32, int threads);

// Cooperative solve of a batch of one problem (N knots of state size nx):
// W own knots per workgroup, G workgroups (coop_plan picks them, or returns
// false when no such grid can be resident on `device` at once).  flags:
// coop_flag_words(N) unsigned words, all zero when allocated, words from
// coop_clear_first() on zeroed before every launch; rec, wtag:
// coop_rec_words(N) and coop_wtag_words(N, nx) 64-bit words, zero when
// allocated and never cleared again.  The problem's r64 row is used as an
// exchange buffer.
bool coop_plan(int N, int nx, bool fp32, int device, int *W, int *G);
int coop_flag_words(int N);
int coop_clear_first();
size_t coop_rec_words(int N);
size_t coop_wtag_words(int N, int nx);
hipError_t launch_coop(const SolveArgs &a, unsigned *flags, unsigned long long *rec, unsigned long long *wtag, int nx,
                       int W, int G, bool fp32, hipStream_t s);

// Dynamic LDS the fused kernel may ask for (a CU's 160 KB less room for
// the kernel's own static arrays).
constexpr int kFusedLdsCap = 160 * 1024 - 256;

// Fused single-sweep PCG with the preconditioner applied from D^-1 and S.
hipError_t launch_pcg2(const SolveArgs &a, int nprob, bool fp32, int threads, int nx, hipStream_t s);
int pcg2_lds(int nx_max, bool fp32, int threads);  // 0 if the mapping cannot hold one knot
// Knots per step the fused kernel uses for state size nx (< 1: cannot run).
int pcg2_steps_for(int nx, bool fp32, int threads, int lds_bytes);
// Workgroup sizes the fused kernel is compiled for (128, 256).
bool pcg2_threads_ok(int threads);

// Scaled solve of the problems order[0 .. nprob) (all of state size nx, one
// of kBuildSizes): one persistent grid of the kernel instance compiled for
// nx, problems taken from the device queue counter a.queue.  `grid`:
// workgroups to launch (<= 0: as many as fit on the device at once).
hipError_t launch_pcg3(const SolveArgs &a, bool fp32, int threads, int nx, int grid, hipStream_t s);
// LDS bytes for the largest pipeline step of state size nx at `threads`
// with m Horner steps (0 if it cannot run), and the knots per step a budget
// gives (< 1: cannot run).
int pcg3_lds(int nx, bool fp32, int threads, int m);
int pcg3_steps_for(int nx, bool fp32, int threads, int lds_bytes, int m);
// largest horizon whose recurrence vectors the scaled solve keeps in LDS
int pcg3_onchip_horizon(int nx, bool fp32, int threads, int lds_bytes, int m);
// Knots per step of the scaled solve's FP64 residual for a budget (< 1: none).
int pcg3_residual_steps(int nx, bool fp32, int lds_bytes);
// Workgroups of k_pcg3 for state size nx resident per CU with this LDS
// budget, and CUs.
int pcg3_occupancy(bool fp32, int threads, int lds_bytes, int *cus, bool acc, int nx);

}  // namespace ssp
