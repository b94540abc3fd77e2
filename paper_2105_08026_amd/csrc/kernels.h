// Kernels of the sampler.
//
//  sweep_kernel     one RAM sweep of every object (Sec. 2.2) fused with the
//                   per-tile FP64 partial sums the theta step consumes, and
//                   the selection quadrature for the pending theta'
//                   (workgroup 0).
//  epilogue_kernel  one workgroup per dataset: fixed-order reduction of the partials,
//                   then the theta Metropolis-Hastings step (fused cycles)
//                   and the next proposal.  Kept out of the sweep kernel:
//                   a cross-workgroup release inside it would write back
//                   the XCD's L2 once per workgroup.
//  theta_kernel     the theta step on its own (plain cycle).
//  poplik_kernel    sum_i log f(chi_i; theta) - N ln Z(theta) for a given theta.
//  init kernels   derived per-object data, factors, quadrature tables.
#pragma once

#include "models.h"

namespace hbm {

// Values an epilogue needs that do not depend on the tile reduction.  The
// sweep kernel's workgroup 0 computes them while the object tiles run (and
// set_theta_kernel for a theta set from the host), one wavefront each:
//   wave 0: the expensive per-theta scalars of the proposal just judged
//           (lnGamma(beta' + 1) ...);
//   wave 1: the standard normals of the next proposal (Philox blocks
//           (0, k + 1, 1, b));
//   wave 2: ln u of the theta accept test (block (0, k, 2, 0)) and the log
//           prior of the judged proposal;
//   wave 3: eta of the next sweep.
struct Precomp {
    double z[kMaxP];
    double aux_used[2];
    double lprior_used;
    double ln_u;
    double eta_next;
    double zraw;      // quadrature sum of ln Z at the judged proposal (before its shift)
    double logz_used; // ln Z at the judged proposal (0 without selection or support)
    double dconst;    // N times the object-independent part of its log f change (dlf_const)
};
static_assert(sizeof(Precomp) % 8 == 0, "Precomp is copied in 8-byte words");

// Arguments of the sweep kernel.  Arrays of the packed datasets are
// component-major with stride n_total; per-dataset tables are indexed by the
// dataset (quadrature tables with stride nq, theta traces with stride
// trace_stride rows of p).
template <typename T>
struct SweepArgs {
    T *chi;
    T *chol;
    uint32_t *acc;
    const T *dd;               // derived per-object data [MD][n_total]
    T *snaps;                  // latent snapshots [snap][D][n_total] or nullptr
    T *trace;                  // [3 + D][n_total] or nullptr
    double *partials;          // [3][n_tiles_total]: sum log f, sum of log f changes, accepted moves
    Precomp *side;             // [n_ds] values for the epilogue, written by the side workgroups
    CycleState *cs;            // [n_ds]
    const Statics *st;         // [n_ds]
    const double *qx, *qw, *qeps;   // [n_ds][nq]
    const int32_t *tile_ds;    // dataset of each tile, -1 for an unused tile
    int64_t n_total;
    int32_t n_tiles_total;
    int32_t n_ds;
    int32_t nq;
};

// ---------------------------------------------------------------------------
// Theta-chain arithmetic (FP64).  The state is staged in LDS by one
// workgroup; lane 0 runs the sequential parts on that copy.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stage_in(CycleState &dst, const CycleState *src)
{
    const uint64_t *s = reinterpret_cast<const uint64_t *>(src);
    uint64_t *d = reinterpret_cast<uint64_t *>(&dst);
    for (int j = threadIdx.x; j < static_cast<int>(sizeof(CycleState) / 8); j += blockDim.x) d[j] = s[j];
    __syncthreads();
}

__device__ __forceinline__ void stage_out(CycleState *dst, const CycleState &src)
{
    __syncthreads();
    const uint64_t *s = reinterpret_cast<const uint64_t *>(&src);
    uint64_t *d = reinterpret_cast<uint64_t *>(dst);
    for (int j = threadIdx.x; j < static_cast<int>(sizeof(CycleState) / 8); j += blockDim.x) d[j] = s[j];
}


// k: the sweep whose theta step follows; judged: the proposal that sweep's
// sums refer to (nullptr when there is none to judge).  The draws (the next
// proposal's normals, ln u, the next step size) depend on k alone
// (precompute_draws), the rest on the judged proposal (precompute_judged);
// each value is one lane's, whichever wavefront computes it.
template <class M>
__device__ __forceinline__ void precompute_draws(Precomp &pc, int64_t k, const Statics &s)
{
    constexpr int NB = (M::P + 3) / 4;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    if (wave == 1 && lane < NB) {
        const Block4 blk = philox(0u, static_cast<uint32_t>(k + 1), 1u, static_cast<uint32_t>(lane), s.key0, s.key1);
        double z4[4];
        normals<double, 4>(blk, z4);
        for (int j = 0; j < 4; ++j)
            if (4 * lane + j < kMaxP) pc.z[4 * lane + j] = z4[j];
    }
    if (wave == 2 && lane == 0) {
        const Block4 ub = philox(0u, static_cast<uint32_t>(k), 2u, 0u, s.key0, s.key1);
        pc.ln_u = log(uniform24<double>(ub, 4));
    }
    if (wave == 3 && lane == 0) pc.eta_next = pow(static_cast<double>(k + 2), -s.gamma);
}

template <class M>
__device__ __forceinline__ void precompute_judged(Precomp &pc, const double *judged, bool judged_valid)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    if (wave == 0 && lane == 0) {
        if (judged_valid) M::aux(judged, pc.aux_used);
        else pc.aux_used[0] = pc.aux_used[1] = 0.0;
    }
    if (wave == 2 && lane == 0) pc.lprior_used = judged_valid ? M::log_prior(judged) : -HUGE_VAL;
}

template <class M>
__device__ __forceinline__ void precompute(Precomp &pc, int64_t k, const double *judged, bool judged_valid,
                                           const Statics &s)
{
    if (judged != nullptr) precompute_judged<M>(pc, judged, judged_valid);
    precompute_draws<M>(pc, k, s);
}

// Draws the proposal theta' = theta + S_theta z for sweep k + 1 (c.k == k)
// and derives the constants that sweep needs (lane 0).
template <class M>
__device__ void prepare_next(CycleState &c, const Statics &s, const Precomp &pc)
{
    using T = typename M::T;
    constexpr int P = M::P;
    for (int r = 0; r < P; ++r) {
        double v = c.theta[r];
        for (int q = 0; q <= r; ++q) v += c.chol_theta[r * P + q] * pc.z[q];
        c.prop[r] = v;
        c.zprop[r] = pc.z[r];
    }
    c.prop_valid = M::in_support(c.prop);
    const double *tp = c.prop_valid ? c.prop : c.theta;
    M::derive_kc(c.theta, tp, c.aux_cur, s, kc_of<T>(&c));
    M::z_consts(tp, c.zc_prop);
    c.eta_next = pc.eta_next;
}

// Turns the reduced sums of sweep c.k + 1 into the quantities its theta step
// judges (lane 0): the proposal the sweep used, its ln Z, log prior and
// aux scalars, and sum_i [log f(chi_i; theta') - log f(chi_i; theta)].
template <class M, bool kStats = false>
__device__ void finish_sweep(CycleState &c, const Statics &s, const double *v, const Precomp &pc)
{
    c.k += 1;
    c.sum_lf = v[0];
    if constexpr (kStats) {
        for (int j = 0; j < M::NS; ++j) c.stats[j] = v[1 + j];
        c.sum_dlf_raw = 0.0;
        c.n_acc_last = v[1 + M::NS];
    } else {
        c.sum_dlf_raw = v[1];
        c.n_acc_last = v[2];
    }
    for (int r = 0; r < M::P; ++r) {
        c.used_prop[r] = c.prop[r];
        c.used_z[r] = c.zprop[r];
    }
    c.used_valid = c.prop_valid;
    c.aux_used[0] = pc.aux_used[0];
    c.aux_used[1] = pc.aux_used[1];
    c.lprior_used = pc.lprior_used;
    // ln Z(theta') and N dlf_const come from the sweep's side workgroup
    c.logZ_used = pc.logz_used;
    c.sum_dlf = v[1];
    if (c.used_valid) {
        if (M::kSelection && !(c.logZ_used > -HUGE_VAL && c.logZ_used < HUGE_VAL)) c.flags |= kFlagBadZ;
        if constexpr (!kStats) c.sum_dlf = v[1] - pc.dconst;
    }
    if constexpr (kStats) c.sum_dlf = 0.0;
    c.eta_used = c.eta_next;
    c.sums_ready = 1;
}

// Metropolis-Hastings step of cycle k on theta (lane 0).
template <class M>
__device__ void theta_mh(CycleState &c, const Statics &s, double *theta_trace, double ln_u)
{
    constexpr int P = M::P;
    double delta = -HUGE_VAL;
    if (c.used_valid) {
        delta = c.sum_dlf - static_cast<double>(s.n) * (c.logZ_used - c.logZ_cur) + (c.lprior_used - c.lprior_cur);
        if (delta != delta) delta = -HUGE_VAL;
    }
    const double alpha = delta >= 0.0 ? 1.0 : exp(delta);
    const bool accepted = ln_u < delta;
    if (accepted) {
        for (int r = 0; r < P; ++r) c.theta[r] = c.used_prop[r];
        c.logZ_cur = c.logZ_used;
        c.lprior_cur = c.lprior_used;
        c.aux_cur[0] = c.aux_used[0];
        c.aux_cur[1] = c.aux_used[1];
    }
    if (s.adapt_theta) {
        double L[P * (P + 1) / 2], zz[P];
        for (int r = 0, e = 0; r < P; ++r)
            for (int q = 0; q <= r; ++q, ++e) L[e] = c.chol_theta[r * P + q];
        for (int r = 0; r < P; ++r) zz[r] = c.used_z[r];
        ram_adapt<double, P>(L, zz, c.eta_used * (alpha - s.alpha_star_theta));
        for (int r = 0, e = 0; r < P; ++r)
            for (int q = 0; q <= r; ++q, ++e) c.chol_theta[r * P + q] = L[e];
    }
    if (c.n_theta < s.trace_cap) {
        // (a null trace: a copy of the chain whose trace another workgroup writes)
        if (theta_trace != nullptr)
            for (int r = 0; r < P; ++r) theta_trace[c.n_theta * P + r] = c.theta[r];
        c.n_theta += 1;
    } else {
        c.flags |= kFlagTraceFull;
    }
    c.sums_ready = 0;
    c.delta_last = delta;
    c.alpha_last = alpha;
    c.accepted_last = accepted;
    if (c.budget > 0 && c.n_theta >= c.budget) c.active = 0;
}

template <class M>
__device__ __forceinline__ double block_log_z(const double *zc, const double *qx, const double *qw,
                                              const double *qeps, int nq, double (*red)[kBlock]);

// The theta step from the sweep's sufficient statistics: K = s.substeps
// Metropolis steps on theta given chi, K >= 1, every thread of the
// workgroup taking part.  Sub-step j of cycle k draws its proposal normals
// from Philox blocks (j, k, 1, b) and its uniform from (j, k, 2, 0);
// sub-step 0 judges the proposal the sweep was prepared with (its ln Z and
// per-theta scalars come from the sweep's side workgroup).  The change of
// sum_i log f between any two theta follows from the statistics in O(1);
// the theta RAM adapts with eta_n, n = (k - 1) K + j + 1.
//
// Only the chain itself is sequential.  The draws, the step sizes eta and
// (per step) the proposal's ln Z, lnGamma-type scalars and log prior do not
// depend on the accept decisions that precede them in the same way: the
// draws and eta for all K steps come first, one lane each; then each step's
// proposal is formed by lane 0, and while the workgroup sums its selection
// normaliser, lane 64 evaluates its per-theta scalars.
constexpr int kMaxSubsteps = 64;

// The per-theta scalars of a model (lnGamma ...) called out of line: inlined
// into the sub-step loop they would spill the workgroup's registers.
template <class M>
__device__ __attribute__((noinline)) void aux_out_of_line(const double *th, double *a)
{
    M::aux(th, a);
}

template <class M>
__device__ void theta_substeps(CycleState &c, const Statics &s, double *theta_trace, const Precomp &pc,
                               const double *qx, const double *qw, const double *qeps, int nq,
                               double (*red)[kBlock])
{
    constexpr int P = M::P, NB = (P + 3) / 4;
    constexpr int kAuxLane = kWave;               // first lane of the second wavefront
    __shared__ double sh_z[kMaxSubsteps][kMaxP];
    __shared__ double sh_lnu[kMaxSubsteps], sh_eta[kMaxSubsteps];
    __shared__ double sh_prop[kMaxP], sh_ap[2], sh_lp;
    __shared__ int32_t sh_valid;
    const int K = s.substeps;
    for (int j = threadIdx.x; j < K; j += kBlock) {
        if (j == 0) {
            for (int r = 0; r < P; ++r) sh_z[0][r] = c.used_z[r];
            sh_lnu[0] = pc.ln_u;
        } else {
            for (int b = 0; b < NB; ++b) {
                const Block4 blk = philox(static_cast<uint32_t>(j), static_cast<uint32_t>(c.k), 1u,
                                          static_cast<uint32_t>(b), s.key0, s.key1);
                double z4[4];
                normals<double, 4>(blk, z4);
                for (int q = 0; q < 4; ++q)
                    if (4 * b + q < P) sh_z[j][4 * b + q] = z4[q];
            }
            const Block4 ub = philox(static_cast<uint32_t>(j), static_cast<uint32_t>(c.k), 2u, 0u, s.key0, s.key1);
            sh_lnu[j] = log(uniform24<double>(ub, 4));
        }
        sh_eta[j] = pow(static_cast<double>((c.k - 1) * K + j + 2), -s.gamma);
    }
    double t0[kMaxP], a0[2];
    for (int r = 0; r < P; ++r) t0[r] = c.theta[r];
    a0[0] = c.aux_cur[0];
    a0[1] = c.aux_cur[1];
    const double n = static_cast<double>(s.n);
    double d_cur = 0.0;                 // sum log f(theta_j) - sum log f(theta_0)
    int n_acc = 0;
    double delta = -HUGE_VAL, alpha = 0.0;
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        if (threadIdx.x == 0) {
            if (j == 0) {
                for (int r = 0; r < P; ++r) sh_prop[r] = c.used_prop[r];
                sh_valid = c.used_valid;
            } else {
                for (int r = 0; r < P; ++r) {
                    double v = c.theta[r];
                    for (int q = 0; q <= r; ++q) v += c.chol_theta[r * P + q] * sh_z[j][q];
                    sh_prop[r] = v;
                }
                sh_valid = M::in_support(sh_prop);
            }
        }
        __syncthreads();
        double zraw = 0.0;
        if (j > 0 && sh_valid) {
            if (threadIdx.x == kAuxLane) {
                double ap[2];
                aux_out_of_line<M>(sh_prop, ap);
                sh_ap[0] = ap[0];
                sh_ap[1] = ap[1];
                sh_lp = M::log_prior(sh_prop);
            }
            if constexpr (M::kSelection) {
                double zc[4];
                M::z_consts(sh_prop, zc);
                zraw = block_log_z<M>(zc, qx, qw, qeps, nq, red);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double ap[2] = {0.0, 0.0}, lp = -HUGE_VAL, lz = 0.0, d_prop = 0.0;
            delta = -HUGE_VAL;
            if (sh_valid) {
                if (j == 0) {
                    ap[0] = c.aux_used[0];
                    ap[1] = c.aux_used[1];
                    lp = c.lprior_used;
                    lz = c.logZ_used;
                } else {
                    ap[0] = sh_ap[0];
                    ap[1] = sh_ap[1];
                    lp = sh_lp;
                    if (M::kSelection) {
                        lz = zraw - M::logz_shift(ap);
                        if (!(lz > -HUGE_VAL && lz < HUGE_VAL)) c.flags |= kFlagBadZ;
                    }
                }
                d_prop = M::stats_dlf(t0, sh_prop, a0, ap, c.stats, n, s);
                delta = (d_prop - d_cur) - n * (lz - c.logZ_cur) + (lp - c.lprior_cur);
                if (delta != delta) delta = -HUGE_VAL;
            }
            alpha = delta >= 0.0 ? 1.0 : exp(delta);
            if (sh_lnu[j] < delta) {
                for (int r = 0; r < P; ++r) c.theta[r] = sh_prop[r];
                c.logZ_cur = lz;
                c.lprior_cur = lp;
                c.aux_cur[0] = ap[0];
                c.aux_cur[1] = ap[1];
                d_cur = d_prop;
                n_acc += 1;
            }
            if (s.adapt_theta) {
                double L[P * (P + 1) / 2], zz[P];
                for (int r = 0, e = 0; r < P; ++r)
                    for (int q = 0; q <= r; ++q, ++e) L[e] = c.chol_theta[r * P + q];
                for (int r = 0; r < P; ++r) zz[r] = sh_z[j][r];
                ram_adapt<double, P>(L, zz, sh_eta[j] * (alpha - s.alpha_star_theta));
                for (int r = 0, e = 0; r < P; ++r)
                    for (int q = 0; q <= r; ++q, ++e) c.chol_theta[r * P + q] = L[e];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (c.n_theta < s.trace_cap) {
            if (theta_trace != nullptr)
                for (int r = 0; r < P; ++r) theta_trace[c.n_theta * P + r] = c.theta[r];
            c.n_theta += 1;
        } else {
            c.flags |= kFlagTraceFull;
        }
        c.sums_ready = 0;
        c.delta_last = delta;
        c.alpha_last = alpha;
        c.accepted_last = n_acc;
        if (c.budget > 0 && c.n_theta >= c.budget) c.active = 0;
    }
}

// Node j's term of the selection quadrature, rounded on its own: the sums
// below add it without a fused multiply-add, so whichever thread computes it
// the total is the same.
template <class M>
__device__ __forceinline__ double quad_term(const double *zc, const double *qx, const double *qw,
                                            const double *qeps, int j)
{
    const double t = (qw[j] * exp(M::zlog(zc, qx[j]))) * qeps[j];
    return t;
}

// ln of the selection quadrature sum_j w_j g(x_j; theta) eps_j over the fixed
// ln L rule, where g is the luminosity PDF in x = ln L without its
// normaliser (the model's zlog; the normaliser is applied by the caller
// through logz_shift); lane t of one 256-thread workgroup adds nodes t,
// t + 256, ... in that order, then the block sum.  Valid in thread 0.
template <class M>
__device__ __forceinline__ double block_log_z(const double *zc, const double *qx, const double *qw,
                                              const double *qeps, int nq, double (*red)[kBlock])
{
    double v[1] = {0.0};
    for (int j = threadIdx.x; j < nq; j += kBlock) {
        const double t = quad_term<M>(zc, qx, qw, qeps, j);
        v[0] = v[0] + t;
    }
    block_sum<1>(v, red);
    return log(v[0]);
}

// The per-dataset scalars a tile needs, read together right after the
// tile's dataset is known (one round of scalar loads, not a chain).
template <typename T>
struct TileView {
    int64_t k;                 // sweep being done
    int64_t obj_start, n;
    int64_t snap_cap;
    uint32_t key0, key1;
    int32_t thin;
    int32_t active;
    int32_t snap_ring;         // snapshots wrap around the snap_cap rows (streamed runs)
    T eta, astar;
};

template <class M>
__device__ __forceinline__ TileView<typename M::T> tile_view(const SweepArgs<typename M::T> &a, int ds)
{
    using T = typename M::T;
    const CycleState &c = a.cs[ds];
    const Statics &s = a.st[ds];
    return TileView<T>{c.k + 1, s.obj_start, s.n, s.snap_cap, s.key0, s.key1, s.thin, c.active, s.snap_ring,
                       static_cast<T>(c.eta_next), static_cast<T>(s.alpha_star)};
}

// One object's RAM step and its contributions to the tile sums, from the
// object's state already loaded into registers; returns whether the move
// was accepted.  i: position in the packed arrays; il: index within its
// dataset (the random-number counter).
template <class M, bool kTrace, bool kStats = false>
__device__ __forceinline__ bool step_object(const SweepArgs<typename M::T> &a, int ds, const TileView<typename M::T> &tv,
                                            int64_t il, int64_t i, typename M::T *x, typename M::T *S, uint32_t nacc,
                                            const typename M::Obj &o, double *v, bool valid = true,
                                            const typename M::T *kc_in = nullptr)
{
    using T = typename M::T;
    constexpr int D = M::D, NC = M::NC;
    const CycleState *cs = a.cs + ds;
    const Statics &st = a.st[ds];
    const int64_t n = a.n_total;
    const int64_t k = tv.k;
    // the sweep's constants: the dataset's state, or a copy the caller holds
    const T *kc = kc_in != nullptr ? kc_in : kc_of<T>(const_cast<CycleState *>(cs));
    const T eta = tv.eta;
    const T astar = tv.astar;
    T U[D], y[D];
    const Block4 b = philox(static_cast<uint32_t>(il), static_cast<uint32_t>(k), 0u, 0u, tv.key0, tv.key1);
    normals<T, D>(b, U);
#pragma unroll
    for (int r = 0; r < D; ++r) {
        T acc_r = x[r];
#pragma unroll
        for (int q = 0; q <= r; ++q) acc_r += S[r * (r + 1) / 2 + q] * U[q];
        y[r] = acc_r;
    }
    const Eval<T> ex = M::eval(o, x, kc, st);
    const Eval<T> ey = M::eval(o, y, kc, st);
    const T neg_inf = -static_cast<T>(HUGE_VAL);
    const T delta = (ey.lpv > neg_inf) ? ey.lpv - ex.lpv : neg_inf;
    const bool accept = ln_uniform(b, T(0)) < delta;
    const T alpha = accept_prob(delta);
    if (accept) {
#pragma unroll
        for (int j = 0; j < D; ++j) x[j] = y[j];
        nacc += 1u;
    }
    const Eval<T> en = accept ? ey : ex;
    ram_adapt<T, D>(S, U, eta * (alpha - astar));
    v[0] = valid ? static_cast<double>(en.lf) : 0.0;
    if constexpr (kStats) {
        T sv[M::NS > 0 ? M::NS : 1];
        M::stats(o, x, en, kc, st, sv);
#pragma unroll
        for (int j = 0; j < M::NS; ++j) v[1 + j] = valid ? static_cast<double>(sv[j]) : 0.0;
    } else {
        v[1] = valid ? static_cast<double>(M::dlf(o, x, en, kc, st)) : 0.0;
    }
    if (!valid) return false;
#pragma unroll
    for (int j = 0; j < D; ++j) a.chi[j * n + i] = x[j];
#pragma unroll
    for (int e = 0; e < NC; ++e) a.chol[e * n + i] = S[e];
    a.acc[i] = nacc;
    if (!(ex.lpv > neg_inf)) atomicOr(&a.cs[ds].flags, kFlagNonFiniteState);
    if (kTrace) {
        a.trace[i] = ex.lp;
        a.trace[n + i] = ey.lp;
        a.trace[2 * n + i] = accept ? static_cast<T>(1) : static_cast<T>(0);
#pragma unroll
        for (int j = 0; j < D; ++j) a.trace[(3 + j) * n + i] = y[j];
    }
    if (a.snaps != nullptr && tv.thin > 0 && k % tv.thin == 0) {
        int64_t snap = k / tv.thin - 1;
        if (tv.snap_ring && tv.snap_cap > 0) snap %= tv.snap_cap;
        if (snap < tv.snap_cap) {
#pragma unroll
            for (int j = 0; j < D; ++j) a.snaps[(snap * D + j) * n + i] = x[j];
        }
    }
    return accept;
}

// The values of the theta step that the objects do not decide, for the
// proposal c.prop that the sweep k = c.k + 1 prepares (what a side workgroup
// computes while the tiles run): the selection quadrature and per-theta
// scalars of the proposal, the accept uniform, the next proposal's normals and
// step size, and (off the epilogue's serial path) ln Z of the proposal and N
// times the object-independent part of its log f change.  The whole
// workgroup takes part; the result goes to out.  draws_done: the draws are
// in sd already (precompute_draws for sweep c.k + 1).
template <class M>
__device__ __forceinline__ void side_values(const CycleState &cs, const Statics &st, const double *qx, const double *qw,
                            const double *qeps, int32_t nq, Precomp &sd, double (*zred)[kBlock], Precomp *out,
                            bool draws_done = false)
{
    const bool valid = cs.prop_valid != 0;
    double judged[kMaxP];
    for (int r = 0; r < M::P; ++r) judged[r] = cs.prop[r];
    double zraw = 0.0;
    if constexpr (M::kSelection) {
        if (valid) {
            double zc[4] = {cs.zc_prop[0], cs.zc_prop[1], cs.zc_prop[2], cs.zc_prop[3]};
            zraw = block_log_z<M>(zc, qx, qw, qeps, nq, zred);
        }
    }
    if (draws_done) precompute_judged<M>(sd, judged, valid);
    else precompute<M>(sd, cs.k + 1, judged, valid, st);
    if (threadIdx.x == 0) sd.zraw = zraw;
    __syncthreads();
    // the judged proposal's ln Z and constant log f change, off the
    // epilogue's serial path (they need its aux scalars from wave 0)
    if (threadIdx.x == 0) {
        sd.logz_used = (valid && M::kSelection) ? zraw - M::logz_shift(sd.aux_used) : 0.0;
        sd.dconst = valid ? static_cast<double>(st.n) * M::dlf_const(cs.theta, judged, cs.aux_cur, sd.aux_used) : 0.0;
    }
    __syncthreads();
    const uint64_t *src = reinterpret_cast<const uint64_t *>(&sd);
    uint64_t *dst = reinterpret_cast<uint64_t *>(out);
    for (int j = threadIdx.x; j < static_cast<int>(sizeof(Precomp) / 8); j += kBlock) dst[j] = src[j];
}

// ---------------------------------------------------------------------------
// The sweep.  Workgroups 0 .. n_ds-1 are side workgroups, one per dataset:
// ln Z at its pending proposal and every FP64 value of its theta step that
// the objects do not decide.  Every other workgroup updates TPW consecutive
// tiles of 256 objects (lane t takes object t of each) and writes one set of
// FP64 partial sums per tile, reduced in the same fixed order whatever TPW
// is, so the launch shape never changes a result.  No workgroup waits on
// another: the epilogue kernel that follows on the stream reduces the
// partials.
// ---------------------------------------------------------------------------
// kSingle: the context holds one dataset covering every position (object i
// of the dataset at position i), so tiles need no table and no per-dataset
// placement.
// kStats: the tiles reduce the model's sufficient statistics at the new
// state instead of the change of log f for the pending proposal.
template <class M, bool kTrace, int TPW, bool kSingle, bool kStats = false>
__global__ __launch_bounds__(kBlock) void sweep_kernel(SweepArgs<typename M::T> a)
{
    constexpr int kCols = kStats ? 1 + M::NS : 2;     // FP64 sums per tile besides the accepted count
    __shared__ double red[kCols * TPW][kBlock];
    __shared__ uint32_t nacc_w[TPW][kWavesPerBlock];

    const int n_side = kSingle ? 1 : a.n_ds;
    // one round of kernel-argument loads for both paths
    if (kSingle) asm volatile("" ::"s"(a.chi), "s"(a.chol), "s"(a.acc), "s"(a.dd), "s"(a.n_total));
    if (static_cast<int>(blockIdx.x) < n_side) {
        const int ds = blockIdx.x;
        const CycleState *cs = a.cs + ds;
        if (!cs->active) return;
        __shared__ Precomp sd;
        __shared__ double zred[1][kBlock];
        const int64_t qo = static_cast<int64_t>(ds) * a.nq;
        side_values<M>(*cs, a.st[ds], a.qx + qo, a.qw + qo, a.qeps + qo, a.nq, sd, zred, a.side + ds);
        return;
    }

    using T = typename M::T;
    constexpr int D = M::D, NC = M::NC;
    const int g0 = (static_cast<int>(blockIdx.x) - n_side) * TPW;     // first tile
    // A dataset's objects start on a tile boundary, so position i of tile g
    // is g * 256 + lane whatever the dataset.  The objects' state is loaded
    // before the tile's dataset is looked up, so the loads overlap the table
    // and state lookups; every position below n_total lies inside the
    // caller's buffers (positions between datasets are read, never written).
    T xs[TPW][D], Ss[TPW][NC];
    uint32_t na[TPW];
    typename M::Obj os[TPW];
    TileView<T> tv[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        // positions past the end read the last position instead (unused): no
        // branch, so the loads issue with the kernel arguments they need
        int64_t i = static_cast<int64_t>(g0 + u) * kBlock + threadIdx.x;
        i = i < a.n_total ? i : a.n_total - 1;
#pragma unroll
        for (int j = 0; j < D; ++j) xs[u][j] = a.chi[j * a.n_total + i];
#pragma unroll
        for (int e = 0; e < NC; ++e) Ss[u][e] = a.chol[e * a.n_total + i];
        na[u] = a.acc[i];
        os[u] = M::load(a.dd, i, a.n_total);
    }
    if constexpr (kSingle) {
        // the one dataset's scalars, in one round behind the object loads
        tv[0] = tile_view<M>(a, 0);
        asm volatile("" ::"s"(tv[0].k), "s"(tv[0].key0), "s"(tv[0].key1), "s"(tv[0].active), "s"(tv[0].eta));
#pragma unroll
        for (int u = 1; u < TPW; ++u) tv[u] = tv[0];
    }
    int dss[TPW];
    bool any = false;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int g = g0 + u;
        int ds;
        if constexpr (kSingle) {
            ds = (g < a.n_tiles_total) ? 0 : -1;
        } else {
            ds = (g < a.n_tiles_total) ? a.tile_ds[g] : -1;
            tv[u] = tile_view<M>(a, ds < 0 ? 0 : ds);      // slot 0 always exists
            // issue every scalar load of the view now, as one round (the
            // compiler would otherwise chain them behind the branches below)
            asm volatile("" ::"s"(tv[u].k), "s"(tv[u].obj_start), "s"(tv[u].n), "s"(tv[u].key0),
                         "s"(tv[u].key1), "s"(tv[u].active), "s"(tv[u].eta));
        }
        if (ds >= 0 && !tv[u].active) ds = -1;          // no epilogue reads this tile
        dss[u] = ds;
        any = any || ds >= 0;
    }
    double v[kCols * TPW];
    bool accepted[TPW];
    if constexpr (kSingle) {
        // no exit between the loads and the arithmetic (the compiler would
        // otherwise move the loads behind it): every lane computes, and only
        // objects of the dataset store
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int64_t i = static_cast<int64_t>(g0 + u) * kBlock + threadIdx.x;
            accepted[u] = step_object<M, kTrace, kStats>(a, 0, tv[u], i, i, xs[u], Ss[u], na[u], os[u],
                                                         v + kCols * u, dss[u] >= 0 && i < a.n_total);
        }
    } else {
        if (!any) return;
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
#pragma unroll
            for (int q = 0; q < kCols; ++q) v[kCols * u + q] = 0.0;
            accepted[u] = false;
            const int ds = dss[u];
            if (ds < 0) continue;
            const int64_t i = static_cast<int64_t>(g0 + u) * kBlock + threadIdx.x;
            const int64_t il = i - tv[u].obj_start;
            if (il >= 0 && il < tv[u].n)
                accepted[u] = step_object<M, kTrace, kStats>(a, ds, tv[u], il, i, xs[u], Ss[u], na[u], os[u],
                                                             v + kCols * u);
        }
    }
    if (!any) return;           // (kSingle) the dataset is off: nothing to publish
    // accepted moves: one ballot per wavefront and tile
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const uint32_t nw = static_cast<uint32_t>(__popcll(__ballot(accepted[u])));
        if ((threadIdx.x & (kWave - 1)) == 0) nacc_w[u][threadIdx.x / kWave] = nw;
    }
    block_sum<kCols * TPW>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            if (dss[u] < 0) continue;
            const int g = g0 + u;
#pragma unroll
            for (int q = 0; q < kCols; ++q) a.partials[q * a.n_tiles_total + g] = v[kCols * u + q];
            a.partials[kCols * a.n_tiles_total + g] =
                static_cast<double>((nacc_w[u][0] + nacc_w[u][1]) + (nacc_w[u][2] + nacc_w[u][3]));
        }
    }
}

struct EpiArgs {
    CycleState *cs;            // the chain states the sweep ran with (sums pending)
    CycleState *cs_out;        // where the epilogue leaves them (cs itself, or the other buffer of a fused run)
    const Statics *st;
    const double *partials;
    const Precomp *side;
    double *theta_trace;       // [n_ds][trace_stride][p]
    const double *qx, *qw, *qeps;   // [n_ds][nq] selection tables (theta sub-steps)
    int64_t trace_stride;
    int32_t n_tiles_total;
    int32_t nq;
};

// Epilogue of a sweep for dataset ds, by one workgroup, into its LDS copy c
// of the chain state: fixed-order reduction of the dataset's tile partials,
// bookkeeping, then (kFull) the theta step, then the proposal for the next
// sweep.  Returns false (c staged unchanged) when the dataset is off.  The
// theta trace row is written only with write_trace.  The dataset's constants
// are staged into the LDS copy sst in the same round of loads as the state,
// and the sequential theta chain reads them there: read from memory where
// the chain first needs them, each would stall lane 0 for a memory round
// trip (a scalar load after the kernel start's cache invalidation).
// In a workgroup of NT > 256 threads the first 256 do the work and the
// others pass the barriers.  While lane 0 runs the theta chain every other
// thread calls during(k) with the sweep count k the state was staged with.
struct NoChainHook {
    __device__ void operator()(int64_t) const {}
};

template <class M, bool kFull, bool kSingle, bool kStats = false, int NT = kBlock, class Hook = NoChainHook>
__device__ __forceinline__ bool epilogue_body(const EpiArgs &a, int ds, CycleState &c, Precomp &pc, Statics &sst,
                              double (*red)[kBlock], bool write_trace, const Hook &during = Hook{})
{
    static_assert(NT == kBlock || !kStats, "theta sub-steps run in 256-thread workgroups");
    const bool lane_ok = NT == kBlock || threadIdx.x < kBlock;
    constexpr int NCOL = (kStats ? 1 + M::NS : 2) + 1;     // tile sums, then the accepted count
    constexpr int G = NCOL > 3 ? 4 : 8;                     // tiles whose loads are issued together
    const Statics &st = a.st[ds];
    const int32_t ntt = a.n_tiles_total;
    const int32_t t0 = kSingle ? 0 : st.tile_start, nt = kSingle ? ntt : st.n_tiles;
    // Every load is issued before the dataset's flag is looked at (it arrives
    // with the staged state); the values of a dataset that is off are unused.
    // The state and the side values are loaded first, into registers, so
    // their latency overlaps the partials' (loads complete in issue order).
    constexpr int kCsWords = static_cast<int>(sizeof(CycleState) / 8), kPcWords = static_cast<int>(sizeof(Precomp) / 8);
    constexpr int kStWords = static_cast<int>(sizeof(Statics) / 8);
    constexpr int kCsPer = (kCsWords + kBlock - 1) / kBlock;
    static_assert(kPcWords + kStWords <= kBlock, "one side or constants word per thread");
    uint64_t csw[kCsPer], pcw = 0;
    {
        const uint64_t *src = reinterpret_cast<const uint64_t *>(a.cs + ds);
#pragma unroll
        for (int u = 0; u < kCsPer; ++u) {
            const int j = u * kBlock + static_cast<int>(threadIdx.x);
            csw[u] = (lane_ok && j < kCsWords) ? src[j] : 0;
        }
        const int t = static_cast<int>(threadIdx.x);
        if (t < kPcWords) pcw = reinterpret_cast<const uint64_t *>(a.side + ds)[t];
        else if (t < kPcWords + kStWords) pcw = reinterpret_cast<const uint64_t *>(a.st + ds)[t - kPcWords];
    }
    // tile partials of this dataset, structure of arrays [NCOL][n_tiles_total]:
    // lane t adds tiles t, t + 256, t + 512, ... in that order; the loads of
    // up to G such tiles are issued together before any is added
    double v[NCOL];
#pragma unroll
    for (int col = 0; col < NCOL; ++col) v[col] = 0.0;
    for (int base = 0; base < nt; base += G * kBlock) {
        double q[NCOL][G];
#pragma unroll
        for (int m = 0; m < G; ++m) {
            const int t = base + m * kBlock + threadIdx.x;
            const bool in = lane_ok && t < nt;
#pragma unroll
            for (int col = 0; col < NCOL; ++col) q[col][m] = in ? a.partials[col * ntt + t0 + t] : 0.0;
        }
#pragma unroll
        for (int m = 0; m < G; ++m) {
            if (lane_ok && base + m * kBlock + static_cast<int>(threadIdx.x) < nt) {
#pragma unroll
                for (int col = 0; col < NCOL; ++col) v[col] += q[col][m];
            }
        }
    }
    {
        uint64_t *dc = reinterpret_cast<uint64_t *>(&c);
#pragma unroll
        for (int u = 0; u < kCsPer; ++u) {
            const int j = u * kBlock + static_cast<int>(threadIdx.x);
            if (lane_ok && j < kCsWords) dc[j] = csw[u];
        }
        const int t = static_cast<int>(threadIdx.x);
        if (t < kPcWords) reinterpret_cast<uint64_t *>(&pc)[t] = pcw;
        else if (t < kPcWords + kStWords) reinterpret_cast<uint64_t *>(&sst)[t - kPcWords] = pcw;
    }
    __syncthreads();
    if (!c.active) return false;         // uniform: read from LDS after the barrier
    const int64_t k_staged = c.k;        // (lane 0 changes c.k only after the barrier below)
    (void)k_staged;
    block_sum_at<NCOL>(v, red, static_cast<int>(threadIdx.x), lane_ok);
    double *trace = write_trace ? a.theta_trace + ds * a.trace_stride * M::P : nullptr;
    if constexpr (kStats) {
        if (threadIdx.x == 0) finish_sweep<M, true>(c, sst, v, pc);
        if constexpr (kFull) {
            __syncthreads();
            const int64_t qo = static_cast<int64_t>(ds) * a.nq;
            theta_substeps<M>(c, sst, trace, pc, a.qx + qo, a.qw + qo, a.qeps + qo, a.nq, red);
        }
        if (threadIdx.x == 0) prepare_next<M>(c, sst, pc);
    } else if (threadIdx.x == 0) {
        // the chain's wavefront first at the SIMD while other wavefronts
        // sweep (a fused cycle) or other workgroups run
        __builtin_amdgcn_s_setprio(3);
        finish_sweep<M>(c, sst, v, pc);
        if (kFull) theta_mh<M>(c, sst, trace, pc.ln_u);
        prepare_next<M>(c, sst, pc);
        __builtin_amdgcn_s_setprio(0);
    } else {
        during(k_staged);
    }
    return true;
}

// Epilogue of a sweep, one workgroup per dataset (epilogue_body); the state
// goes to cs_out (a dataset that is off is copied there unchanged when
// cs_out is not cs).
template <class M, bool kFull, bool kSingle, bool kStats = false>
__global__ __launch_bounds__(kBlock) void epilogue_kernel(EpiArgs a)
{
    __shared__ CycleState c;
    __shared__ Precomp pc;
    __shared__ Statics sst;
    __shared__ double red[(kStats ? 1 + M::NS : 2) + 1][kBlock];
    const int ds = kSingle ? 0 : static_cast<int>(blockIdx.x);
    if (!epilogue_body<M, kFull, kSingle, kStats>(a, ds, c, pc, sst, red, true) && a.cs_out == a.cs) return;
    stage_out(a.cs_out + ds, c);
}

constexpr int kKc = 16;              // per-sweep constants the models read (kc[0..15])

// A value read in one lane made uniform (scalar registers).
__device__ __forceinline__ float uniform_of(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform_of(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<int>(b & 0xffffffffu));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<int>(b >> 32));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// The chain state c of a fused launch written to the other buffer by the
// NT threads of a side workgroup: every word but the flags, which this
// launch's tiles may raise meanwhile (atomicOr in step_object), then c's
// flags OR-ed in (flags only accumulate, so the word ends as c's flags plus
// any the tiles raise).
template <int NT>
__device__ __forceinline__ void publish_state(CycleState *dst, const CycleState &c)
{
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&c);
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
    constexpr int kWords = static_cast<int>(sizeof(CycleState) / 4);
    constexpr int kFlagsWord = static_cast<int>(offsetof(CycleState, flags) / 4);
    for (int q = threadIdx.x; q < kWords; q += NT)
        if (q != kFlagsWord) d[q] = src[q];
    if (threadIdx.x == 0 && c.flags != 0) atomicOr(&dst->flags, c.flags);
}

// ---------------------------------------------------------------------------
// One full cycle in one launch, for a context that holds one dataset: the
// theta step of the previous sweep, then this sweep.  Every workgroup takes
// the theta step itself -- the previous sweep's partials reduced in the
// epilogue's fixed order, so every copy of the chain is bit for bit the
// same -- and then, with the new state in its LDS, steps its tiles (the
// tiles' object loads are issued first, so their latency overlaps the theta
// step).  Workgroup 0 writes the chain state, the trace row and the side
// values of the new proposal.  A fused run reads the previous sweep's state,
// partials and side values from one set of buffers and writes this sweep's
// to the other, so no workgroup reads what another writes in the same launch
// and none waits for another; the kernel boundary orders consecutive cycles.
// ---------------------------------------------------------------------------
template <typename T>
struct FusedArgs {
    SweepArgs<T> sw;           // this sweep: objects, and the buffers it writes (cs, partials, side)
    EpiArgs epi;               // the previous sweep's state, partials and side values; the trace
};

template <class M, int TPW, bool kStats>
__global__ __launch_bounds__(kBlock) void fused_kernel(FusedArgs<typename M::T> a)
{
    using T = typename M::T;
    constexpr int D = M::D, NC = M::NC;
    constexpr int kCols = kStats ? 1 + M::NS : 2;     // FP64 sums per tile besides the accepted count
    constexpr int NCOL = kCols + 1;
    constexpr int kRed = kCols * TPW > NCOL ? kCols * TPW : NCOL;
    __shared__ CycleState c;
    __shared__ Precomp pc;
    __shared__ Statics st;
    __shared__ double red[kRed][kBlock];
    __shared__ uint32_t nacc_w[TPW][kWavesPerBlock];
    __shared__ Precomp sd;
    const SweepArgs<T> &sw = a.sw;
    const bool side = blockIdx.x == 0;                 // uniform
    const int64_t n = sw.n_total;
    const int g0 = (static_cast<int>(blockIdx.x) - 1) * TPW;     // first tile of a tile workgroup
    // this workgroup's objects first (positions past the end read the last one, unused)
    T xs[TPW][D], Ss[TPW][NC];
    uint32_t na[TPW];
    typename M::Obj os[TPW];
    if (!side) {
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            int64_t i = static_cast<int64_t>(g0 + u) * kBlock + threadIdx.x;
            i = i < n ? i : n - 1;
#pragma unroll
            for (int j = 0; j < D; ++j) xs[u][j] = sw.chi[j * n + i];
#pragma unroll
            for (int e = 0; e < NC; ++e) Ss[u][e] = sw.chol[e * n + i];
            na[u] = sw.acc[i];
            os[u] = M::load(sw.dd, i, n);
        }
    }
    // the previous sweep's theta step, in every workgroup; the side
    // workgroup's wavefronts 1-3 take the next side values' draws (for sweep
    // staged count + 2) while lane 0 runs the chain
    const auto during_chain = [&](int64_t k) {
        if (side) precompute_draws<M>(sd, k + 2, st);
    };
    epilogue_body<M, true, true, kStats>(a.epi, 0, c, pc, st, red, side, during_chain);
    __syncthreads();
    if (side) {
        // the chain state, then the new proposal's side values
        publish_state<kBlock>(sw.cs, c);
        if (!c.active) return;                         // uniform: LDS after a barrier
        __shared__ double zred[1][kBlock];
        side_values<M>(c, st, sw.qx, sw.qw, sw.qeps, sw.nq, sd, zred, sw.side, !kStats);
        return;
    }
    if (!c.active) return;
    const TileView<T> tv{c.k + 1, st.obj_start, st.n, st.snap_cap, st.key0, st.key1, st.thin, c.active,
                         st.snap_ring, static_cast<T>(c.eta_next), static_cast<T>(st.alpha_star)};
    T kc[kKc];
#pragma unroll
    for (int q = 0; q < kKc; ++q) kc[q] = uniform_of(kc_of<T>(&c)[q]);
    double v[kCols * TPW];
    bool accepted[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int64_t i = static_cast<int64_t>(g0 + u) * kBlock + threadIdx.x;
        accepted[u] = step_object<M, false, kStats>(sw, 0, tv, i, i, xs[u], Ss[u], na[u], os[u], v + kCols * u,
                                                    g0 + u < sw.n_tiles_total && i < n, kc);
    }
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const uint32_t nw = static_cast<uint32_t>(__popcll(__ballot(accepted[u])));
        if ((threadIdx.x & (kWave - 1)) == 0) nacc_w[u][threadIdx.x / kWave] = nw;
    }
    block_sum<kCols * TPW>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int g = g0 + u;
            if (g >= sw.n_tiles_total) continue;
#pragma unroll
            for (int q = 0; q < kCols; ++q) sw.partials[q * sw.n_tiles_total + g] = v[kCols * u + q];
            sw.partials[kCols * sw.n_tiles_total + g] =
                static_cast<double>((nacc_w[u][0] + nacc_w[u][1]) + (nacc_w[u][2] + nacc_w[u][3]));
        }
    }
}

// ---------------------------------------------------------------------------
// The fused cycle in workgroups of TPW x 256 threads, one object per thread:
// the 256-thread slice u steps tile TPW (w - 1) + u.  A workgroup holds TPW
// tiles without stepping several objects per thread, and the redundant
// theta step -- its reads of every tile partial, and its serial chain on
// lane 0 -- is taken once per TPW tiles.  The first 256 threads take it
// exactly as fused_kernel does; the tile sums are the same block sums per
// tile, so the chain is bit for bit the two-kernel cycle's.  The side
// workgroup (0) uses its extra wavefronts for the selection quadrature of
// the new proposal while wavefronts 0 and 2 evaluate the proposal's
// per-theta scalars, and takes the draws that depend only on the sweep
// count while lane 0 runs the chain.
// ---------------------------------------------------------------------------
// The side values of side_values() in a workgroup of NT = 256 m threads
// (m >= 2), the draws already in sd: the judged proposal's scalars by
// wavefronts 0 and 2 while the threads from 256 on evaluate the quadrature
// terms, NT - 256 at a time into zt; the first 256 threads add them in
// block_log_z's order (lane t: nodes t, t + 256, ...), so ln Z has the same
// bits as there.
template <class M, int NT>
__device__ __forceinline__ void side_values_wide(const CycleState &cs, const Statics &st, const double *qx,
                                                 const double *qw, const double *qeps, int32_t nq, Precomp &sd,
                                                 double (*zred)[kBlock], double *zt, Precomp *out)
{
    static_assert(NT > kBlock && NT % kBlock == 0, "a workgroup of several 256-thread slices");
    constexpr int NQT = NT - kBlock;
    const int tid = static_cast<int>(threadIdx.x);
    const bool valid = cs.prop_valid != 0;
    double judged[kMaxP];
    for (int r = 0; r < M::P; ++r) judged[r] = cs.prop[r];
    precompute_judged<M>(sd, judged, valid);
    double zraw = 0.0;
    if constexpr (M::kSelection) {
        if (valid) {                   // uniform
            const double zc[4] = {cs.zc_prop[0], cs.zc_prop[1], cs.zc_prop[2], cs.zc_prop[3]};
            double v[1] = {0.0};
            for (int c0 = 0; c0 < nq; c0 += NQT) {
                if (tid >= kBlock) {
                    const int j = c0 + tid - kBlock;
                    if (j < nq) zt[tid - kBlock] = quad_term<M>(zc, qx, qw, qeps, j);
                }
                __syncthreads();
                if (tid < kBlock) {
#pragma unroll
                    for (int m = 0; m < NQT / kBlock; ++m) {
                        const int j = c0 + m * kBlock + tid;
                        if (j < nq) v[0] = v[0] + zt[m * kBlock + tid];
                    }
                }
                __syncthreads();
            }
            block_sum_at<1>(v, zred, tid, tid < kBlock);
            zraw = log(v[0]);
        }
    }
    if (tid == 0) sd.zraw = zraw;
    __syncthreads();
    if (tid == 0) {
        sd.logz_used = (valid && M::kSelection) ? zraw - M::logz_shift(sd.aux_used) : 0.0;
        sd.dconst = valid ? static_cast<double>(st.n) * M::dlf_const(cs.theta, judged, cs.aux_cur, sd.aux_used) : 0.0;
    }
    __syncthreads();
    const uint64_t *src = reinterpret_cast<const uint64_t *>(&sd);
    uint64_t *dst = reinterpret_cast<uint64_t *>(out);
    for (int j = tid; j < static_cast<int>(sizeof(Precomp) / 8); j += NT) dst[j] = src[j];
}

template <class M, int TPW>
__global__ __launch_bounds__(kBlock * TPW) void fused_wide_kernel(FusedArgs<typename M::T> a)
{
    static_assert(TPW >= 2, "one tile per workgroup is fused_kernel");
    using T = typename M::T;
    constexpr int NT = kBlock * TPW;
    constexpr int D = M::D, NC = M::NC;
    constexpr int kCols = 2;                          // sum log f, sum of log f changes
    constexpr int NCOL = kCols + 1;
    __shared__ CycleState c;
    __shared__ Precomp pc;
    __shared__ Statics st;
    __shared__ double red[NCOL][kBlock];
    __shared__ double tred[TPW][kCols][kBlock];
    __shared__ uint32_t nacc_w[TPW][kWavesPerBlock];
    __shared__ Precomp sd;
    __shared__ double zt[NT - kBlock];
    const SweepArgs<T> &sw = a.sw;
    const bool side = blockIdx.x == 0;                 // uniform
    const int64_t n = sw.n_total;
    const int u = static_cast<int>(threadIdx.x) / kBlock, lane = static_cast<int>(threadIdx.x) % kBlock;
    const int g = (static_cast<int>(blockIdx.x) - 1) * TPW + u;     // this slice's tile
    const int64_t i = static_cast<int64_t>(g) * kBlock + lane;
    // this thread's object first (positions past the end read the last one, unused)
    T xs[D], Ss[NC];
    uint32_t na = 0;
    typename M::Obj os{};
    if (!side) {
        const int64_t ic = i < n ? i : n - 1;
#pragma unroll
        for (int j = 0; j < D; ++j) xs[j] = sw.chi[j * n + ic];
#pragma unroll
        for (int e = 0; e < NC; ++e) Ss[e] = sw.chol[e * n + ic];
        na = sw.acc[ic];
        os = M::load(sw.dd, ic, n);
    }
    // the previous sweep's theta step, in every workgroup; the side
    // workgroup's wavefronts 1-3 take the next side values' draws (for sweep
    // staged count + 2) while lane 0 runs the chain
    const auto during_chain = [&](int64_t k) {
        if (side) precompute_draws<M>(sd, k + 2, st);
    };
    epilogue_body<M, true, true, false, NT>(a.epi, 0, c, pc, st, red, side, during_chain);
    __syncthreads();
    if (side) {
        publish_state<NT>(sw.cs, c);
        if (!c.active) return;                         // uniform: LDS after a barrier
        side_values_wide<M, NT>(c, st, sw.qx, sw.qw, sw.qeps, sw.nq, sd, red, zt, sw.side);
        return;
    }
    if (!c.active) return;
    const TileView<T> tv{c.k + 1, st.obj_start, st.n, st.snap_cap, st.key0, st.key1, st.thin, c.active,
                         st.snap_ring, static_cast<T>(c.eta_next), static_cast<T>(st.alpha_star)};
    T kc[kKc];
#pragma unroll
    for (int q = 0; q < kKc; ++q) kc[q] = uniform_of(kc_of<T>(&c)[q]);
    double v[kCols];
    const bool accepted = step_object<M, false, false>(sw, 0, tv, i, i, xs, Ss, na, os, v,
                                                       g < sw.n_tiles_total && i < n, kc);
    const uint32_t nw = static_cast<uint32_t>(__popcll(__ballot(accepted)));
    if ((lane & (kWave - 1)) == 0) nacc_w[u][lane / kWave] = nw;
    block_sum_at<kCols>(v, tred[u], lane, true);
    if (lane == 0 && g < sw.n_tiles_total) {
#pragma unroll
        for (int q = 0; q < kCols; ++q) sw.partials[q * sw.n_tiles_total + g] = v[q];
        sw.partials[kCols * sw.n_tiles_total + g] =
            static_cast<double>((nacc_w[u][0] + nacc_w[u][1]) + (nacc_w[u][2] + nacc_w[u][3]));
    }
}

// ---------------------------------------------------------------------------
// The fused cycle of a context with several datasets (a batch or a pool),
// one tile per workgroup: workgroup ds < n_ds is dataset ds's side
// workgroup (it takes the dataset's theta step, writes its state, trace row
// and the new proposal's side values), every other workgroup a tile, which
// takes the theta step of its own dataset -- the reduction of that
// dataset's tile partials only -- and steps its objects.  A dataset that is
// off keeps its state (copied to the other buffer) and its tiles do
// nothing, as in the two-kernel cycle.
// ---------------------------------------------------------------------------
template <class M, bool kStats>
__global__ __launch_bounds__(kBlock) void fused_pool_kernel(FusedArgs<typename M::T> a)
{
    using T = typename M::T;
    constexpr int D = M::D, NC = M::NC;
    constexpr int kCols = kStats ? 1 + M::NS : 2;     // FP64 sums per tile besides the accepted count
    constexpr int NCOL = kCols + 1;
    __shared__ CycleState c;
    __shared__ Precomp pc;
    __shared__ Statics st;
    __shared__ double red[NCOL][kBlock];
    __shared__ uint32_t nacc_w[kWavesPerBlock];
    __shared__ Precomp sd;
    const SweepArgs<T> &sw = a.sw;
    const int n_side = sw.n_ds;
    const bool side = static_cast<int>(blockIdx.x) < n_side;      // uniform
    const int g = static_cast<int>(blockIdx.x) - n_side;          // tile of a tile workgroup
    const int ds = side ? static_cast<int>(blockIdx.x) : (g < sw.n_tiles_total ? sw.tile_ds[g] : -1);
    if (ds < 0) return;                                           // an unused tile
    const int64_t n = sw.n_total;
    const int64_t i = static_cast<int64_t>(g) * kBlock + threadIdx.x;
    // the object first (tile workgroups; every position below n_total lies
    // inside the caller's buffers)
    T xs[D], Ss[NC];
    uint32_t na = 0;
    typename M::Obj os{};
    if (!side) {
        const int64_t ic = i < n ? i : n - 1;
#pragma unroll
        for (int j = 0; j < D; ++j) xs[j] = sw.chi[j * n + ic];
#pragma unroll
        for (int e = 0; e < NC; ++e) Ss[e] = sw.chol[e * n + ic];
        na = sw.acc[ic];
        os = M::load(sw.dd, ic, n);
    }
    // the dataset's previous theta step; the side workgroup's wavefronts 1-3
    // take the next side values' draws (sweep staged count + 2) meanwhile
    const auto during_chain = [&](int64_t k) {
        if (side) precompute_draws<M>(sd, k + 2, st);
    };
    epilogue_body<M, true, false, kStats>(a.epi, ds, c, pc, st, red, side, during_chain);
    __syncthreads();
    if (side) {
        publish_state<kBlock>(sw.cs + ds, c);
        if (!c.active) return;                         // uniform: LDS after a barrier
        __shared__ double zred[1][kBlock];
        const int64_t qo = static_cast<int64_t>(ds) * sw.nq;
        side_values<M>(c, st, sw.qx + qo, sw.qw + qo, sw.qeps + qo, sw.nq, sd, zred, sw.side + ds, !kStats);
        return;
    }
    if (!c.active) return;
    const TileView<T> tv{c.k + 1, st.obj_start, st.n, st.snap_cap, st.key0, st.key1, st.thin, c.active,
                         st.snap_ring, static_cast<T>(c.eta_next), static_cast<T>(st.alpha_star)};
    T kc[kKc];
#pragma unroll
    for (int q = 0; q < kKc; ++q) kc[q] = uniform_of(kc_of<T>(&c)[q]);
    const int64_t il = i - st.obj_start;
    double v[kCols];
    const bool accepted =
        step_object<M, false, kStats>(sw, ds, tv, il, i, xs, Ss, na, os, v, il >= 0 && il < st.n, kc);
    const uint32_t nw = static_cast<uint32_t>(__popcll(__ballot(accepted)));
    if ((threadIdx.x & (kWave - 1)) == 0) nacc_w[threadIdx.x / kWave] = nw;
    block_sum<kCols>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < kCols; ++q) sw.partials[q * sw.n_tiles_total + g] = v[q];
        sw.partials[kCols * sw.n_tiles_total + g] =
            static_cast<double>((nacc_w[0] + nacc_w[1]) + (nacc_w[2] + nacc_w[3]));
    }
}

// Theta step on its own, after a ram_sweep (plain cycle), one workgroup per dataset.
template <class M, bool kStats = false>
__global__ __launch_bounds__(kBlock) void theta_kernel(EpiArgs a)
{
    __shared__ CycleState c;
    __shared__ Precomp pc;
    __shared__ double red[1][kBlock];
    const int ds = blockIdx.x;
    if (!a.cs[ds].active) return;
    {
        const uint64_t *src = reinterpret_cast<const uint64_t *>(a.side + ds);
        uint64_t *dst = reinterpret_cast<uint64_t *>(&pc);
        for (int j = threadIdx.x; j < static_cast<int>(sizeof(Precomp) / 8); j += kBlock) dst[j] = src[j];
    }
    stage_in(c, a.cs + ds);
    const bool ready = c.sums_ready != 0;       // uniform: read from LDS after the barrier
    if constexpr (kStats) {
        if (ready) {
            const int64_t qo = static_cast<int64_t>(ds) * a.nq;
            theta_substeps<M>(c, a.st[ds], a.theta_trace + ds * a.trace_stride * M::P, pc, a.qx + qo, a.qw + qo,
                              a.qeps + qo, a.nq, red);
        }
        if (threadIdx.x == 0) {
            if (ready) prepare_next<M>(c, a.st[ds], pc);
            else c.flags |= kFlagNoSums;
        }
    } else if (threadIdx.x == 0) {
        if (ready) {
            theta_mh<M>(c, a.st[ds], a.theta_trace + ds * a.trace_stride * M::P, pc.ln_u);
            prepare_next<M>(c, a.st[ds], pc);
        } else {
            c.flags |= kFlagNoSums;
        }
    }
    (void)red;
    stage_out(a.cs + ds, c);
}

// Recompute everything that depends on theta after it is set from the host,
// for the datasets whose flag in `which` is set (one workgroup each).
template <class M>
__global__ __launch_bounds__(kBlock) void set_theta_kernel(CycleState *cs_all, const Statics *st_all,
                                                           const double *qx, const double *qw, const double *qeps,
                                                           int32_t nq, const int32_t *which)
{
    __shared__ CycleState c;
    __shared__ Precomp pc;
    __shared__ double red[1][kBlock];
    const int ds = blockIdx.x;
    if (!which[ds]) return;
    CycleState *cs = cs_all + ds;
    const Statics &st = st_all[ds];
    stage_in(c, cs);
    const bool ok = M::in_support(c.theta);
    // the judged-proposal slots of pc carry theta itself here
    precompute<M>(pc, c.k, c.theta, ok, st);
    double lz = 0.0;
    if constexpr (M::kSelection) {
        if (ok) {
            double zc[4];
            M::z_consts(c.theta, zc);
            const int64_t qo = static_cast<int64_t>(ds) * nq;
            lz = block_log_z<M>(zc, qx + qo, qw + qo, qeps + qo, nq, red);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        c.lprior_cur = pc.lprior_used;
        c.aux_cur[0] = pc.aux_used[0];
        c.aux_cur[1] = pc.aux_used[1];
        c.logZ_cur = (M::kSelection && ok) ? lz - M::logz_shift(c.aux_cur) : 0.0;
        if (M::kSelection && ok && !(c.logZ_cur > -HUGE_VAL && c.logZ_cur < HUGE_VAL)) c.flags |= kFlagBadZ;
        c.sums_ready = 0;
        prepare_next<M>(c, st, pc);
    }
    stage_out(cs, c);
}

template <class M>
__global__ void statics_kernel(Statics *st, const int32_t *which)
{
    if (threadIdx.x == 0 && which[blockIdx.x]) M::derive_statics(st[blockIdx.x]);
}

// Per-tile kernels of the initialisation: each workgroup takes one tile of
// one dataset (tiles of unloaded or unselected datasets are skipped).
template <class M>
__global__ __launch_bounds__(kBlock) void derive_data_kernel(const typename M::T *data, typename M::T *dd,
                                                             const Statics *st, const int32_t *tile_ds,
                                                             const int32_t *which, int64_t n_total)
{
    const int ds = tile_ds[blockIdx.x];
    if (ds < 0 || !which[ds]) return;
    const Statics &s = st[ds];
    const int64_t il = static_cast<int64_t>(blockIdx.x - s.tile_start) * kBlock + threadIdx.x;
    if (il < s.n) M::derive_obj(data, dd, s.obj_start + il, n_total, s);
}

template <class M>
__global__ __launch_bounds__(kBlock) void init_chain_kernel(typename M::T *chol, uint32_t *acc, const Statics *st, const int32_t *tile_ds,
                                                            const int32_t *which, int64_t n_total)
{
    using T = typename M::T;
    const int ds = tile_ds[blockIdx.x];
    if (ds < 0 || !which[ds]) return;
    const Statics &s = st[ds];
    const int64_t il = static_cast<int64_t>(blockIdx.x - s.tile_start) * kBlock + threadIdx.x;
    if (il >= s.n) return;
    const int64_t i = s.obj_start + il;
    for (int r = 0, e = 0; r < M::D; ++r)
        for (int q = 0; q <= r; ++q, ++e) chol[e * n_total + i] = (r == q) ? static_cast<T>(s.s0) : static_cast<T>(0);
    acc[i] = 0u;
}

// Flags objects whose starting log density is not finite (pi(X_1) > 0 is required).
template <class M>
__global__ __launch_bounds__(kBlock) void check_init_kernel(const typename M::T *chi, const typename M::T *dd,
                                                            CycleState *cs, const Statics *st, const int32_t *tile_ds,
                                                            const int32_t *which, int64_t n_total)
{
    using T = typename M::T;
    const int ds = tile_ds[blockIdx.x];
    if (ds < 0 || !which[ds]) return;
    const Statics &s = st[ds];
    const int64_t il = static_cast<int64_t>(blockIdx.x - s.tile_start) * kBlock + threadIdx.x;
    if (il >= s.n) return;
    const int64_t i = s.obj_start + il;
    T x[M::D];
    for (int j = 0; j < M::D; ++j) x[j] = chi[j * n_total + i];
    const Eval<T> e = M::eval(M::load(dd, i, n_total), x, kc_of<T>(cs + ds), s);
    if (!(e.lpv > -static_cast<T>(HUGE_VAL) && e.lpv < static_cast<T>(HUGE_VAL))) {
        atomicMin(&cs[ds].first_bad, static_cast<int32_t>(il));
        atomicOr(&cs[ds].flags, kFlagNonFiniteState);
    }
}

template <typename T>
struct PopArgs {
    const T *chi;
    const T *dd;
    double *partials;
    double *pout;              // [n_ds][2]: ln Z(theta), sum log f - N ln Z
    const double *theta;       // [n_ds][p]
    const Statics *st;
    const double *qx, *qw, *qeps;
    const int32_t *tile_ds;
    int64_t n_total;
    int32_t n_tiles_total;
    int32_t n_ds;
    int32_t nq;
};

// Partial sums of log f(chi_i; theta_ds) per tile; side workgroups evaluate ln Z(theta_ds).
template <class M>
__global__ __launch_bounds__(kBlock) void poplik_kernel(PopArgs<typename M::T> a)
{
    using T = typename M::T;
    __shared__ double red[1][kBlock];
    __shared__ T kc[32];
    if (static_cast<int>(blockIdx.x) < a.n_ds) {
        const int ds = blockIdx.x;
        if (a.st[ds].n == 0) {                    // empty slot
            if (threadIdx.x == 0) a.pout[2 * ds] = a.pout[2 * ds + 1] = static_cast<double>(NAN);
            return;
        }
        const double *th = a.theta + ds * M::P;
        double ag[2];
        M::aux(th, ag);
        double lz = 0.0;
        if constexpr (M::kSelection) {
            double zc[4];
            M::z_consts(th, zc);
            const int64_t qo = static_cast<int64_t>(ds) * a.nq;
            lz = block_log_z<M>(zc, a.qx + qo, a.qw + qo, a.qeps + qo, a.nq, red) - M::logz_shift(ag);
        }
        if (threadIdx.x == 0) a.pout[2 * ds] = lz;
        return;
    }
    const int g = blockIdx.x - a.n_ds;
    const int ds = a.tile_ds[g];
    if (ds < 0) return;
    const Statics &st = a.st[ds];
    const double *th = a.theta + ds * M::P;
    if (threadIdx.x == 0) {
        double ag[2];
        M::aux(th, ag);
        M::derive_kc(th, th, ag, st, kc);
    }
    __syncthreads();
    const int64_t il = static_cast<int64_t>(g - st.tile_start) * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (il < st.n) {
        const int64_t i = st.obj_start + il;
        T x[M::D];
        for (int j = 0; j < M::D; ++j) x[j] = a.chi[j * a.n_total + i];
        v[0] = static_cast<double>(M::eval(M::load(a.dd, i, a.n_total), x, kc, st).lf);
    }
    block_sum<1>(v, red);
    if (threadIdx.x == 0) a.partials[g] = v[0];
}

__global__ __launch_bounds__(kBlock) void poplik_finish_kernel(const Statics *st, const double *partials, double *pout)
{
    __shared__ double red[1][kBlock];
    const int ds = blockIdx.x;
    const Statics &s = st[ds];
    if (s.n == 0) return;
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < s.n_tiles; t += kBlock) v[0] += partials[s.tile_start + t];
    block_sum<1>(v, red);
    if (threadIdx.x == 0) pout[2 * ds + 1] = v[0] - static_cast<double>(s.n) * pout[2 * ds];
}

// ---------------------------------------------------------------------------
// Selection tables.  Gauss-Legendre nodes on [-1, 1]: node j is the root of
// P_n near cos(pi (4j + 3) / (4n + 2)) (Tricomi's first term), polished by
// Newton steps on the three-term recurrence; weight 2 / ((1 - t^2) P_n'(t)^2).
// ---------------------------------------------------------------------------
__global__ void gauss_legendre_kernel(double *t_out, double *w_out, int nq)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nq) return;
    const double pi = 3.14159265358979323846;
    const double theta = pi * (4.0 * j + 3.0) / (4.0 * nq + 2.0);
    double t = cos(theta) * (1.0 - (nq - 1.0) / (8.0 * nq * nq * nq));
    double dp = 1.0;
    for (int it = 0; it < 60; ++it) {
        double pm1 = 1.0, p = t;
        for (int l = 1; l < nq; ++l) {
            const double pn = ((2.0 * l + 1.0) * t * p - l * pm1) / (l + 1.0);
            pm1 = p;
            p = pn;
        }
        dp = nq * (pm1 - t * p) / (1.0 - t * t);
        const double step = p / dp;
        t -= step;
        if (fabs(step) <= 1e-17) break;
    }
    {
        double pm1 = 1.0, p = t;
        for (int l = 1; l < nq; ++l) {
            const double pn = ((2.0 * l + 1.0) * t * p - l * pm1) / (l + 1.0);
            pm1 = p;
            p = pn;
        }
        dp = nq * (pm1 - t * p) / (1.0 - t * t);
    }
    t_out[j] = t;
    w_out[j] = 2.0 / ((1.0 - t * t) * dp * dp);
}

// Outer rule in x = ln L on [ln L0 - 30, ln L0 + ln 40] and, per node, the
// detection efficiency eps(x) = int_0^rmax dr h(r) eta(L / 4 pi r^2) with
// h(r) = 3 r^2 / rmax^3 and eta(F) = Phi((F - F_th) / sigma_F) (eq 5.10),
// written in s = ln u, u = (r / rmax)^3, so that h dr = e^s ds, over
// s in [-60, 0] with the same n-point rule (the part below e^-60 is dropped).
template <class M>
__global__ void eps_table_kernel(const double *t, const double *w, double *qx_all, double *qw_all, double *qeps_all,
                                 const Statics *st_all, const int32_t *which)
{
    const int ds = blockIdx.y;
    if (!which[ds]) return;
    const Statics *st = st_all + ds;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int nq = st->nq;
    if (j >= nq) return;
    double *qx = qx_all + static_cast<int64_t>(ds) * nq, *qw = qw_all + static_cast<int64_t>(ds) * nq;
    double *qeps = qeps_all + static_cast<int64_t>(ds) * nq;
    double lo, hi;
    M::quad_interval(*st, &lo, &hi);
    // nodes ascend in x: t descends with the node index
    const double x = 0.5 * (lo + hi) - 0.5 * (hi - lo) * t[j];
    qx[j] = x;
    qw[j] = 0.5 * (hi - lo) * w[j];
    // flux of luminosity e^x at the survey edge; at u = (r / rmax)^3 = e^s it is u^(-2/3) times that
    const double edge_flux = exp(x) / M::edge_area(*st);
    double acc = 0.0;
    for (int l = 0; l < nq; ++l) {
        const double s = -30.0 - 30.0 * t[l];
        acc += 30.0 * w[l] * exp(s) * M::detect(edge_flux * exp(-2.0 * s / 3.0), *st);
    }
    qeps[j] = acc;
}

}  // namespace hbm
