// Batched PCG with one fused sweep per iteration.
//
// The preconditioners are applied from D^-1 and S without stored stair
// blocks.  From Eq. (stair_inv), Psi^-1 = D^-1 (2D - Psi) D^-1 for either
// stair; with S = Psi_l + Psi_r - D (Sec. III) this gives
//   symmetric stair (Sec. IV):  Phi^-1 = Psi_l^-1 + Psi_r^-1 - D^-1
//                                      = 2 D^-1 - D^-1 S D^-1 = D^-1 - D^-1 O D^-1,
//   additive stair (Sec. III):  Phi^-1 = (Psi_l^-1 + Psi_r^-1) / 2
//                                      = D^-1 - 0.5 D^-1 O D^-1,
//   block-Jacobi (Eq. (jacobi)): Phi^-1 = D^-1,
// with O = S - D the off-diagonal blocks.  So u = Phi^-1 r is y = D^-1 r,
// t = O y, u = y - c D^-1 t (the O form avoids forming D^-1 D y, which
// cancels badly in FP32 when D_k is ill-conditioned), and every
// preconditioner streams the same three block arrays (D, L, D^-1) per
// iteration.
//
// The CG recurrences are rearranged so that one pass over the knots applies
// both the preconditioner and S (the single-reduction form of Chronopoulos
// and Gear; in exact arithmetic its iterates are those of textbook PCG):
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//   u = Phi^-1 r,  w = S u,  gamma = r.u,  delta = w.u,  rho = r.r,
//   beta' = gamma' / gamma,  alpha' = gamma' / (delta' - beta' gamma' / alpha).
// The pass walks the knots in steps of C: step c updates the lead knots
// [k0, k1) and computes y there, t and u one knot behind, and w two knots
// behind (S couples neighbours), so the last step also drains the tail.
// Blocks and vector windows live in LDS rings of C + 2 knots; the next
// step's blocks are fetched into registers with 16-byte loads while the
// current step computes.
#include <math.h>

#include <type_traits>

#include "ssp_device.h"
#include "ssp_fused.h"
#include "ssp_host.h"
#include "ssp_sweep.h"

namespace ssp {

namespace {

// 16-byte prefetch registers per thread (fewer for FP64, whose arithmetic
// needs twice the registers)
template <typename TM>
constexpr int prefetch_slots() { return sizeof(TM) == 4 ? 12 : 8; }

// The six recurrence vectors of a problem.
template <typename TI>
struct Vecs {
    TI *u, *w, *p, *s, *x, *r;
};

// Geometry of the fused pass for one problem.  Knots are mapped to
// wavefronts: a wave holds kw = floor(64 / nx) knots, lane l of wave w works
// on row l % nx of knot w * kw + l / nx, so all rows of a knot sit in one
// wave.  A step covers C <= waves * kw knots.
struct Geo2 {
    int N, nx, nn, bs, bp, ks, nxp;  // knots, state size, block elements, full / packed block stride,
                                     // knot stride, vector slot stride
    int C, R, RU;            // knots per step, block/vector ring slots, u ring slots
    int kw;                  // knots per wave
};

// Knots per step that fit the wave mapping, the prefetch registers and the
// LDS budget.  Ring slot: one knot's D, L, D^-1 (knot stride) and the r, y, t, u vector
// windows (4 nxp), plus one extra u slot.
template <typename TM>
__host__ __device__ inline int pcg2_knots_per_step(int nx, int block, int lds_bytes) {
    const int V = 16 / (int)sizeof(TM);
    const int ks = knot_stride(nx, sizeof(TM));
    const int nxp = (nx + V - 1) / V * V;
    int C = (block / 64) * (64 / nx);
    const int Cp = (prefetch_slots<TM>() * block * V) / ks;
    if (Cp < C) C = Cp;
    const int per = (ks + 4 * nxp) * (int)sizeof(TM);
    const int Cl = (lds_bytes - nxp * (int)sizeof(TM) - 16) / per - 2;  // + one u slot + 16-byte spot
    if (Cl < C) C = Cl;
    return C;  // may be < 1: the mapping cannot run this nx
}

// Register prefetch of one step: the step's D, L and D^-1 blocks (16-byte
// loads) and the six recurrence vectors of this thread's lead row.  Every
// load is issued unconditionally (surplus slots re-read the step's first
// vector), so the compiler can count outstanding loads and the compute
// phases never wait on them.
template <typename TM, int BLOCK>
struct Prefetch {
    using VT = typename Vec16<TM>::T;
    static constexpr int V = Vec16<TM>::V;
    static constexpr int kPF = prefetch_slots<TM>();
    VT reg[kPF];
    TM vec[6];       // u, w, p, s, x, r of this thread's lead row
    double res = 0;  // init pass: the FP64 residual of that row instead

    __device__ __forceinline__ void issue(const TM *B3, int k0, int kc, int ks, bool init, int lead_row,
                                          const double *r64, const Vecs<TM> vs) {
        // the step's D, L, D^-1 blocks: one contiguous chunk of kc knot strides
        const int nvec = kc * ks / V;
        const VT *src = (const VT *)(B3 + (int64_t)k0 * ks);
        static_for<0, kPF>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            int q = threadIdx.x + m * BLOCK;
            if (q >= nvec) q = 0;
            reg[m] = src[q];
        });
        const int row = lead_row >= 0 ? lead_row : 0;
        if (init) {
            res = r64[row];
        } else {
            vec[0] = vs.u[row];
            vec[1] = vs.w[row];
            vec[2] = vs.p[row];
            vec[3] = vs.s[row];
            vec[4] = vs.x[row];
            vec[5] = vs.r[row];
        }
    }

    // Copy the prefetched chunk into the block ring (one knot stride per slot,
    // in the same D, L, D^-1 order): register m lands at
    // (ring slot of k0) * ks + its offset in the chunk, modulo the ring.
    // Slots wholly past the chunk are skipped by a uniform branch; in the
    // partial slot the surplus lanes write a 16-byte scratch spot (dummy)
    // instead of branching.
    __device__ __forceinline__ void store(TM *ring, int kc, int sb, int ks, int R, TM *dummy) const {
        const int nvec = kc * ks / V;
        const int wrap = R * ks;
        const int base = sb * ks;
        static_for<0, kPF>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            if (m * BLOCK < nvec) {
                const int q = threadIdx.x + m * BLOCK;
                int off = base + q * V;
                if (off >= wrap) off -= wrap;
                *(VT *)(q < nvec ? ring + off : dummy) = reg[m];
            }
        });
    }
};

}  // namespace

// Per-thread partial sums of one pass.
template <typename TI>
struct Dots {
    TI gam, del, rho;
};

// One fused pass over the knots (see the file comment).  init: the pass that
// starts an inner solve (r = r64 / ||r64||, x = 0); first: the first update
// pass (p = u, s = w).
template <typename TI, int BLOCK, int NX>
__device__ __forceinline__ Dots<TI> fused_pass(const Geo2 &g, int pc, bool init, bool first, TI alpha, TI beta,
                                               double inv_s, const double *__restrict__ r64,
                                               const TI *__restrict__ B3, TI *Rv, TI *Uv, TI *Wv, TI *Pv, TI *Sv,
                                               TI *Xv, TI *smem) {
    using TM = TI;
    constexpr int W = BLOCK / 64;
    const int nx = NX > 0 ? NX : g.nx, bs = g.bs, bp = g.bp, ks = g.ks, nxp = g.nxp;
    const int N = g.N, C = g.C, R = g.R, RU = g.RU, kw = g.kw;
    TM *ring = smem;  // slot s: D (packed) at s * ks, L at + bp, D^-1 (packed) at + bp + bs
    TM *rD = ring, *rL = ring + bp, *rDi = ring + bp + bs;
    const int ss = ks;  // slot stride of the block ring
    TI *vr = ring + R * ss, *vy = vr + R * nxp, *vt = vy + R * nxp, *vu = vt + R * nxp;
    const bool bj = pc == 0;
    const TI c2 = pc == 2 ? TI(1) : TI(0.5);
    const Vecs<TI> vsrc{Uv, Wv, Pv, Sv, Xv, Rv};
    Dots<TI> d{TI(0), TI(0), TI(0)};

    // this thread's place in the wave mapping
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kloc = NX > 0 ? lane / NX : lane / nx;
    const int i = lane - kloc * nx;
    const bool lane_ok = kloc < kw;
    const int kme = wv * kw + kloc;  // knot offset handled in a knot range
    const int group = W * kw;        // knots covered by one sweep of the block

    // row i of (S x)_k (diag) or (O x)_k, from ring blocks and a ring window
    // (xb, slots sx / sxm / sxp of knots k / k - 1 / k + 1, -1 if absent),
    // s / sp: block-ring slots of k / k + 1
    auto s_row = [&](const TI *xb, int sx, int sxm, int sxp, int s, int sp, bool diag) -> TI {
        TI y = TI(0);
        if (diag) y += sym_dot<NX>(rD + s * ss, i, xb + sx * nxp, nx);        // D_k (packed)
        if (sxm >= 0) y += row_dot<NX>(rL + s * ss, i, xb + sxm * nxp, nx);   // row i of L_k
        if (sxp >= 0) y += col_dot<NX>(rL + sp * ss, i, xb + sxp * nxp, nx);  // column i of L_{k+1}
        return y;
    };

    // results of the previous step, written at the start of the next one
    TI oP = TI(0), oS = TI(0), oX = TI(0), oR = TI(0), oU = TI(0), oW = TI(0);
    int rowA = -1, rowU = -1, rowW = -1;

    Prefetch<TM, BLOCK> pf;
    const int nsteps = (N + C - 1) / C;
    auto lead_row = [&](int k0, int kc) { return (lane_ok && kme < kc) ? (k0 + kme) * nx + i : -1; };
    pf.issue(B3, 0, min(C, N), ks, init, lead_row(0, min(C, N)), r64, vsrc);
    int sb = 0, sbu = 0;  // ring slots of knot k0
    for (int c = 0; c < nsteps; ++c) {
        const int k0 = c * C, kc = min(C, N - k0), k1 = k0 + kc;
        const bool last = k1 == N;
        __syncthreads();  // every reader of the slots about to be refilled is done
        pf.store(ring, kc, sb, ks, R, vu + RU * nxp);
        TM cur[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) cur[v] = pf.vec[v];
        const double res = pf.res;
        // write back the previous step's rows before the next loads go out
        if (rowA >= 0) {
            if (!init) {
                Pv[rowA] = oP;
                Sv[rowA] = oS;
            }
            Xv[rowA] = oX;
            Rv[rowA] = oR;
        }
        if (rowU >= 0) Uv[rowU] = oU;
        if (rowW >= 0) Wv[rowW] = oW;
        rowA = rowU = rowW = -1;
        if (!last) pf.issue(B3, k1, min(C, N - k1), ks, init, lead_row(k1, min(C, N - k1)), r64, vsrc);

        const bool lead = lane_ok && kme < kc;
        const int sl = slot_of(sb, kme, R);
        // A: recurrence updates on the lead rows
        if (lead) {
            TI r;
            if (init) {
                r = (TI)(res * inv_s);
                oX = TI(0);
            } else {
                const TI pv = first ? cur[0] : cur[0] + beta * cur[2];
                const TI sv = first ? cur[1] : cur[1] + beta * cur[3];
                oP = pv;
                oS = sv;
                oX = cur[4] + alpha * pv;
                r = cur[5] - alpha * sv;
            }
            oR = r;
            rowA = (k0 + kme) * nx + i;
            vr[sl * nxp + i] = r;
            d.rho += r * r;
        }
        __syncthreads();  // the ring blocks stored above come from every wave
        // B: y = D^-1 r on the lead knots (u itself for block-Jacobi)
        if (lead) {
            const TI *rk = vr + sl * nxp;
            const TI y = sym_dot<NX>(rDi + sl * ss, i, rk, nx);
            if (bj) {
                vu[slot_of(sbu, kme, RU) * nxp + i] = y;
                oU = y;
                rowU = (k0 + kme) * nx + i;
                d.gam += rk[i] * y;
            } else {
                vy[sl * nxp + i] = y;
            }
        }
        __syncthreads();
        int wlo, whi;  // knots that receive w in this step
        if (!bj) {
            // C: t = O y one knot behind the lead; D: u = y - c D^-1 t (same wave)
            const int tlo = max(k0 - 1, 0), thi = last ? N : k1 - 1;
            for (int kk = kme; kk < thi - tlo; kk += group) {
                if (!lane_ok) break;
                const int k = tlo + kk, dk = k - k0;
                const int s = slot_of(sb, dk, R);
                const int sm = k > 0 ? slot_of(sb, dk - 1, R) : -1;
                const int sp = k + 1 < N ? slot_of(sb, dk + 1, R) : -1;
                vt[s * nxp + i] = s_row(vy, s, sm, sp, s, sp, false);
            }
            wave_sync();
            for (int kk = kme; kk < thi - tlo; kk += group) {
                if (!lane_ok) break;
                const int k = tlo + kk, dk = k - k0;
                const int s = slot_of(sb, dk, R);
                const TI z = sym_dot<NX>(rDi + s * ss, i, vt + s * nxp, nx);
                const TI u = vy[s * nxp + i] - c2 * z;
                vu[slot_of(sbu, dk, RU) * nxp + i] = u;
                d.gam += vr[s * nxp + i] * u;
                if (last) {
                    Uv[k * nx + i] = u;
                } else {
                    oU = u;
                    rowU = k * nx + i;
                }
            }
            __syncthreads();
            wlo = max(k0 - 2, 0);
            whi = last ? N : k1 - 2;
        } else {
            wlo = max(k0 - 1, 0);
            whi = last ? N : k1 - 1;
        }
        // E: w = S u behind the u front
        for (int kk = kme; kk < whi - wlo; kk += group) {
            if (!lane_ok) break;
            const int k = wlo + kk, dk = k - k0;
            const int s = slot_of(sb, dk, R);
            const int su = slot_of(sbu, dk, RU);
            const int sm = k > 0 ? slot_of(sbu, dk - 1, RU) : -1;
            const int sp = k + 1 < N ? slot_of(sbu, dk + 1, RU) : -1;
            const TI w = s_row(vu, su, sm, sp, s, k + 1 < N ? slot_of(sb, dk + 1, R) : -1, true);
            d.del += w * vu[su * nxp + i];
            if (last) {
                Wv[k * nx + i] = w;
            } else {
                oW = w;
                rowW = k * nx + i;
            }
        }
        sb += C;
        if (sb >= R) sb -= R;
        sbu += C;
        if (sbu >= RU) sbu -= RU;
    }
    if (rowA >= 0) {
        if (!init) {
            Pv[rowA] = oP;
            Sv[rowA] = oS;
        }
        Xv[rowA] = oX;
        Rv[rowA] = oR;
    }
    if (rowU >= 0) Uv[rowU] = oU;
    if (rowW >= 0) Wv[rowW] = oW;
    return d;
}

// Pointers of one problem inside the batch buffers.
template <typename TI>
struct Prob {
    int N, bs, bp, ks, max_iter;
    double gnorm;
    const TI *B3;  // per knot: D (packed), L, D^-1 (packed), knot stride ks
    const float *SDlo, *SLlo;
    double *lam, *r64;
    const double *gam;
    TI *Rv, *Uv, *Wv, *Pv, *Sv, *Xv;
};

// Outcome of one problem's solve.
struct Outcome {
    int st = kOk, total = 0, steps = 0;
    bool fallback = false;     // the warm start was dropped for lambda = 0
    bool pc_fallback = false;  // block-Jacobi took over after a float breakdown
    double rnorm = 0.0;
};

// FP64 refinement loop around the fused inner PCG, for state size NX
// (0 = runtime nx).
template <typename TI, int BLOCK, int NX>
__device__ __forceinline__ Outcome solve_problem(const SolveArgs &a, const Prob<TI> q, int nx_rt,
                                              unsigned char *smem_raw, double *red64, TI *redT) {
    using TM = TI;
    const int nx = NX > 0 ? NX : nx_rt;
    const int N = q.N, n = N * nx, tid = threadIdx.x;
    Outcome o;
    Geo2 g;
    g.N = N;
    g.nx = nx;
    g.nn = nx * nx;
    g.bs = q.bs;
    g.bp = q.bp;
    g.ks = q.ks;
    g.nxp = (nx + Vec16<TM>::V - 1) / Vec16<TM>::V * Vec16<TM>::V;
    g.kw = 64 / nx;
    g.C = pcg2_knots_per_step<TM>(nx, BLOCK, a.lds_bytes);
    g.R = g.C + 2;
    g.RU = g.C + 3;
    const Geo g64 = make_geo<double>(nx, q.bs, true, a.lds_bytes, BLOCK);
    const int Cres = NX > 0 ? residual_knots_per_step<TM>(nx, BLOCK, a.lds_bytes) : 0;
    int pending = kOk;
    int pcur = a.pc;     // block-Jacobi after a stair breakdown (refinement only)
    int base = 0;        // refinement steps before that switch
    bool broke = false;  // last inner solve ended in a float breakdown (refinement only)
    double prev = INFINITY;
    double gsame = q.gnorm;      // ||gamma|| summed like the last residual norm
    const double *rsrc = q.r64;  // where the next inner solve reads its right-hand side
    for (;;) {
        if (o.steps == 0 && a.use_lambda0 == 0) {
            // lambda = 0: the residual is gamma itself, no sweep needed
            rsrc = q.gam;
            o.rnorm = q.gnorm;
        } else {
            // true residual r = gamma - S lambda in FP64
            ResNorms nr{0.0, 0.0};
            if (NX > 0 && Cres >= 1) {
                nr = residual_pass<TM, BLOCK, (NX > 0 ? NX : 2)>(N, Cres, q.B3, q.SDlo, q.SLlo, q.lam, q.gam,
                                                                 q.r64, (double *)smem_raw);
            } else {
                bt_sweep<double, TM, BLOCK, NX>(
                    N, g64, q.B3, q.ks, q.SDlo, q.bp, q.B3 + q.bp, q.ks, q.SLlo, true, (double *)smem_raw,
                    [&](int row) { return q.lam[row]; },
                    [&](int row, double y, double) {
                        const double gv = q.gam[row];
                        const double r = gv - y;
                        q.r64[row] = r;
                        nr.rr += r * r;
                        nr.gg += gv * gv;
                    });
            }
            block_sum2<BLOCK>(nr.rr, nr.gg, red64);
            o.rnorm = sqrt(nr.rr);
            gsame = sqrt(nr.gg);
            rsrc = q.r64;
        }
        // the start is kept only if its residual is strictly below ||gamma||,
        // both norms summed in the same order (lambda0 = 0 gives a tie and
        // falls back)
        if (o.steps == 0 && a.use_lambda0 == 2 && !(o.rnorm < gsame)) {
            // a warm start that does not reduce the residual is replaced by zero
            for (int row = tid; row < n; row += BLOCK) {
                q.lam[row] = 0.0;
                q.r64[row] = q.gam[row];
            }
            o.rnorm = q.gnorm;
            o.fallback = true;
            rsrc = q.gam;
            __syncthreads();
        }
        if (!isfinite(o.rnorm)) {
            o.st = kNonFinite;
            break;
        }
        if (pending != kOk) {
            o.st = pending;
            break;
        }
        if (o.rnorm <= a.tol * q.gnorm) break;
        if (o.steps > 0 && !a.refine) {
            o.st = kInaccurate;
            break;
        }
        if (broke && !(o.rnorm < prev)) {
            o.st = kBreakdown;
            break;
        }
        if (o.steps - base >= a.max_outer) {
            o.st = kMaxIter;
            break;
        }
        prev = o.rnorm;
        double tau = (a.refine ? a.theta : 1.0) * a.tol * q.gnorm / o.rnorm;
        if (a.refine && tau < a.tau_min) tau = a.tau_min;
        if (tau > 1.0) tau = 1.0;
        const double inv_s = 1.0 / o.rnorm;

        // inner PCG on S d = r / ||r|| from d = 0
        int it = 0, ist = kOk;
        Dots<TI> dt = fused_pass<TI, BLOCK, NX>(g, pcur, true, false, TI(0), TI(0), inv_s, rsrc, q.B3, q.Rv, q.Uv,
                                                q.Wv, q.Pv, q.Sv, q.Xv, (TI *)smem_raw);
        block_sum2<BLOCK>(dt.gam, dt.del, redT);
        dt.rho = block_sum<BLOCK>(dt.rho, redT + 2 * (BLOCK / kWave));
        const TI bnorm = sqrt(dt.rho);
        const TI tauT = (TI)tau;
        TI gam_prev = TI(0), alpha = TI(0), beta = TI(0);
        for (;;) {
            const TI rn = sqrt(dt.rho);
            if (!isfinite(rn)) {
                ist = kNonFinite;
                break;
            }
            if (rn <= tauT * bnorm) break;
            if (o.total + it >= q.max_iter) {
                ist = kMaxIter;
                break;
            }
            // alpha_j = gamma_j / p_j^T S p_j, with p^T S p from the recurrences
            TI den;
            if (it == 0) {
                den = dt.del;
                beta = TI(0);
            } else {
                beta = dt.gam / gam_prev;
                den = dt.del - beta * dt.gam / alpha;
            }
            if (!(den > TI(0)) || !(dt.gam > TI(0))) {
                ist = (isfinite(den) && isfinite(dt.gam)) ? kBreakdown : kNonFinite;
                break;
            }
            alpha = dt.gam / den;
            gam_prev = dt.gam;
            dt = fused_pass<TI, BLOCK, NX>(g, pcur, false, it == 0, alpha, beta, 0.0, q.r64, q.B3, q.Rv, q.Uv, q.Wv,
                                           q.Pv, q.Sv, q.Xv, (TI *)smem_raw);
            block_sum2<BLOCK>(dt.gam, dt.del, redT);
            dt.rho = block_sum<BLOCK>(dt.rho, redT + 2 * (BLOCK / kWave));
            ++it;
        }
        o.total += it;
        ++o.steps;
        __syncthreads();
        for (int row = tid; row < n; row += BLOCK) q.lam[row] += o.rnorm * (double)q.Xv[row];
        // under refinement a float breakdown only ends the inner solve; under a
        // stair preconditioner it also hands the rest of the solve to
        // block-Jacobi (the float stair operator lost definiteness)
        broke = a.refine && ist == kBreakdown;
        if (broke && pcur != 0) {
            pcur = 0;
            o.pc_fallback = true;
            broke = false;
            base = o.steps;
        }
        if (ist != kOk && !broke && !(a.refine && ist == kBreakdown)) pending = ist;
    }
    return o;
}

// One launch per solve group; NX > 0: every problem of the launch has state
// size NX (compiled in), NX = 0: any state size.
template <typename TI, int BLOCK, int NX>
__global__ __launch_bounds__(BLOCK, 2) void k_pcg2(SolveArgs a) {
    using TM = TI;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red64[2 * (BLOCK / kWave)];
    __shared__ TI redT[3 * (BLOCK / kWave)];
    const int tid = threadIdx.x;
    const int p = a.order[blockIdx.x];
    const int N = a.N[p], nx = NX > 0 ? NX : a.nx[p];
    const int n = N * nx;
    const int64_t ob = a.off_blk[p], ov = a.off_v[p];
    Prob<TI> q;
    q.N = N;
    q.bs = block_stride(nx, sizeof(TM));
    q.bp = packed_stride(nx, sizeof(TM));
    q.ks = 2 * q.bp + q.bs;
    q.max_iter = a.max_iter > 0 ? a.max_iter : 10 * n;
    q.lam = a.lambda + ov;
    q.gam = a.gamma + ov;
    q.r64 = a.r64 + ov;

    Outcome o;
    if (build_failed(a.status[p])) {
        for (int row = tid; row < n; row += BLOCK) q.lam[row] = 0.0;
        if (tid == 0) {
            a.iters[p] = 0;
            a.outer[p] = 0;
            a.relres[p] = NAN;
        }
        return;
    }
    q.B3 = (const TM *)a.B3 + a.off_b3[p];
    q.SDlo = a.SDlo ? a.SDlo + a.off_pk[p] : nullptr;
    q.SLlo = a.SLlo ? a.SLlo + ob : nullptr;
    TI *W = (TI *)a.work;
    q.Rv = W + 0 * a.tot_v + ov;
    q.Uv = W + 1 * a.tot_v + ov;
    q.Wv = W + 2 * a.tot_v + ov;
    q.Pv = W + 3 * a.tot_v + ov;
    q.Sv = W + 4 * a.tot_v + ov;
    q.Xv = W + 5 * a.tot_v + ov;

    double gg = 0.0, bad = 0.0;
    for (int row = tid; row < n; row += BLOCK) {
        const double gv = q.gam[row];
        gg += gv * gv;
        if (a.use_lambda0 == 1) {
            if (!isfinite(q.lam[row])) bad = 1.0;
        } else if (a.use_lambda0 == 0) {
            q.lam[row] = 0.0;
        }
    }
    block_sum2<BLOCK>(gg, bad, red64);
    q.gnorm = sqrt(gg);
    if (!isfinite(q.gnorm) || bad != 0.0) {
        o.st = kNonFinite;
        o.rnorm = NAN;
    } else if (gg == 0.0) {
        for (int row = tid; row < n; row += BLOCK) q.lam[row] = 0.0;
    } else {
        o = solve_problem<TI, BLOCK, NX>(a, q, nx, smem_raw, red64, redT);
    }
    if (tid == 0) {
        a.iters[p] = o.total;
        a.outer[p] = o.steps;
        a.relres[p] = gg == 0.0 ? 0.0 : o.rnorm / q.gnorm;
        a.status[p] = o.st | (o.fallback ? kWarmFallback : 0) | (o.pc_fallback ? kPcFallback : 0);
    }
}

int pcg2_steps_for(int nx, bool fp32, int threads, int lds_bytes) {
    return fp32 ? pcg2_knots_per_step<float>(nx, threads, lds_bytes)
                : pcg2_knots_per_step<double>(nx, threads, lds_bytes);
}

int pcg2_lds(int nx_max, bool fp32, int threads) {
    // ring budget for C knots of the largest nx, at least the FP64 residual sweep
    const int eb = fp32 ? 4 : 8;
    int C = fp32 ? pcg2_knots_per_step<float>(nx_max, threads, 1 << 30)
                 : pcg2_knots_per_step<double>(nx_max, threads, 1 << 30);
    if (C < 1) return 0;
    const int V = 16 / eb;
    const int ks = knot_stride(nx_max, eb), nxp = (nx_max + V - 1) / V * V;
    const int per = (ks + 4 * nxp) * eb;
    int bytes = (C + 2) * per + nxp * eb + 16;
    const int res = bt_sweep_min_lds(nx_max, true, 8);
    if (bytes < res) bytes = res;
    if (bytes > kFusedLdsCap) {
        // shrink the step to the LDS limit
        C = (kFusedLdsCap - nxp * eb - 16) / per - 2;
        if (C < 1 || res > kFusedLdsCap) return 0;
        bytes = (C + 2) * per + nxp * eb + 16;
        if (bytes < res) bytes = res;
    }
    return bytes;
}

template <typename TI, int BLOCK, int NX>
static hipError_t launch2_t(const SolveArgs &a, int nprob, hipStream_t s) {
    // all the LDS a workgroup may have is allowed once; each launch asks for
    // its own size (launches of other sizes may be in flight on other streams)
    static int allowed = 0;
    const void *f = (const void *)k_pcg2<TI, BLOCK, NX>;
    if (allowed == 0) {
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, f);
        if (e != hipSuccess) return e;
        const int cap = 160 * 1024 - (int)fa.sharedSizeBytes;
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
        if (e != hipSuccess) return e;
        allowed = cap;
    }
    if (a.lds_bytes > allowed) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_pcg2<TI, BLOCK, NX>), dim3(nprob), dim3(BLOCK), a.lds_bytes, s, a);
    return hipGetLastError();
}

template <typename TI, int BLOCK>
static hipError_t launch2_nx(const SolveArgs &a, int nprob, int nx, hipStream_t s) {
    switch (nx) {  // state sizes with a compiled-in specialisation; others use the runtime path
        case 6: return launch2_t<TI, BLOCK, 6>(a, nprob, s);
        case 14: return launch2_t<TI, BLOCK, 14>(a, nprob, s);
        case 26: return launch2_t<TI, BLOCK, 26>(a, nprob, s);
        case 36: return launch2_t<TI, BLOCK, 36>(a, nprob, s);
        default: return launch2_t<TI, BLOCK, 0>(a, nprob, s);
    }
}

bool pcg2_threads_ok(int threads) { return threads == 128 || threads == 256; }

hipError_t launch_pcg2(const SolveArgs &a, int nprob, bool fp32, int threads, int nx, hipStream_t s) {
    if (nprob == 0) return hipSuccess;
    if (fp32) {
        switch (threads) {
            case 128: return launch2_nx<float, 128>(a, nprob, nx, s);
            case 256: return launch2_nx<float, 256>(a, nprob, nx, s);
        }
    } else {
        switch (threads) {
            case 128: return launch2_nx<double, 128>(a, nprob, nx, s);
            case 256: return launch2_nx<double, 256>(a, nprob, nx, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace ssp
