// Kernels of the sampler.
//
//  sweep_kernel     one RAM sweep of every object (Sec. 2.2) fused with the
//                   per-tile FP64 partial sums the theta step consumes, and
//                   the selection quadrature for the pending theta'
//                   (workgroup 0).
//  epilogue_kernel  one workgroup: fixed-order reduction of the partials,
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
};
static_assert(sizeof(Precomp) % 8 == 0, "Precomp is copied in 8-byte words");

template <typename T>
struct SweepArgs {
    T *chi;
    T *chol;
    uint32_t *acc;
    const T *dd;               // derived per-object data [MD][N]
    T *snaps;                  // latent snapshots or nullptr
    T *trace;                  // [3 + D][N] or nullptr
    double *partials;          // [3][n_tiles]: sum log f, sum of log f changes, accepted moves
    Precomp *side;             // values for the epilogue, written by workgroup 0
    CycleState *cs;
    const Statics *st;
    const double *qx, *qw, *qeps;
    int64_t n;
    int32_t n_tiles;
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
// sums refer to (nullptr when there is none to judge).
template <class M>
__device__ __forceinline__ void precompute(Precomp &pc, int64_t k, const double *judged, bool judged_valid,
                                           const Statics &s)
{
    constexpr int NB = (M::P + 3) / 4;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    if (wave == 0 && lane == 0 && judged != nullptr) {
        if (judged_valid) M::aux(judged, pc.aux_used);
        else pc.aux_used[0] = pc.aux_used[1] = 0.0;
    }
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
        if (judged != nullptr) pc.lprior_used = judged_valid ? M::log_prior(judged) : -HUGE_VAL;
    }
    if (wave == 3 && lane == 0) pc.eta_next = pow(static_cast<double>(k + 2), -s.gamma);
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
template <class M>
__device__ void finish_sweep(CycleState &c, const Statics &s, const double *v, double zraw, const Precomp &pc)
{
    c.k += 1;
    c.sum_lf = v[0];
    c.sum_dlf_raw = v[1];
    c.n_acc_last = v[2];
    for (int r = 0; r < M::P; ++r) {
        c.used_prop[r] = c.prop[r];
        c.used_z[r] = c.zprop[r];
    }
    c.used_valid = c.prop_valid;
    c.aux_used[0] = pc.aux_used[0];
    c.aux_used[1] = pc.aux_used[1];
    c.lprior_used = pc.lprior_used;
    c.logZ_used = 0.0;
    c.sum_dlf = v[1];
    if (c.used_valid) {
        if (M::kSelection) {
            c.logZ_used = zraw - M::logz_shift(c.aux_used);
            if (!(c.logZ_used > -HUGE_VAL && c.logZ_used < HUGE_VAL)) c.flags |= kFlagBadZ;
        }
        c.sum_dlf = v[1] - static_cast<double>(s.n) * M::dlf_const(c.theta, c.used_prop, c.aux_cur, c.aux_used);
    }
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
        for (int r = 0; r < P; ++r) theta_trace[c.n_theta * P + r] = c.theta[r];
        c.n_theta += 1;
    } else {
        c.flags |= kFlagTraceFull;
    }
    c.sums_ready = 0;
    c.delta_last = delta;
    c.alpha_last = alpha;
    c.accepted_last = accepted;
}

// ln Z(theta) + lnGamma(beta + 1) = ln sum_j w_j f_x(x_j; theta) Gamma(beta + 1) eps_j
// over the fixed ln L rule (the normaliser of the gamma law is applied by
// the caller); every lane of one workgroup takes nodes tid, tid + 256, ...
// Valid in thread 0.
__device__ __forceinline__ double block_log_z(const double *zc, const double *qx, const double *qw,
                                              const double *qeps, int nq, double (*red)[kWavesPerBlock])
{
    double v[1] = {0.0};
    for (int j = threadIdx.x; j < nq; j += kBlock) {
        const double t = qx[j] - zc[1];
        v[0] += qw[j] * exp(zc[0] * t - exp(t)) * qeps[j];
    }
    block_sum<1>(v, red);
    return log(v[0]);
}

// ---------------------------------------------------------------------------
// The sweep: workgroup 0 evaluates ln Z at the pending proposal; every
// other workgroup updates one tile of 256 objects and writes the tile's
// FP64 partial sums.  No workgroup waits on another: the epilogue kernel
// that follows on the stream reduces the partials.
// ---------------------------------------------------------------------------
template <class M, bool kTrace>
__global__ __launch_bounds__(kBlock) void sweep_kernel(SweepArgs<typename M::T> a)
{
    using T = typename M::T;
    constexpr int D = M::D, NC = M::NC;
    __shared__ double red[3][kWavesPerBlock];
    CycleState *cs = a.cs;
    const Statics &st = *a.st;

    if (blockIdx.x == 0) {
        // everything the epilogue needs that the objects do not decide
        __shared__ Precomp sd;
        const bool valid = cs->prop_valid != 0;
        double judged[kMaxP];
        for (int r = 0; r < M::P; ++r) judged[r] = cs->prop[r];
        double zraw = 0.0;
        if (M::kSelection && valid) {
            double zc[2] = {cs->zc_prop[0], cs->zc_prop[1]};
            zraw = block_log_z(zc, a.qx, a.qw, a.qeps, st.nq, red);
        }
        precompute<M>(sd, cs->k + 1, judged, valid, st);
        if (threadIdx.x == 0) sd.zraw = zraw;
        __syncthreads();
        const uint64_t *src = reinterpret_cast<const uint64_t *>(&sd);
        uint64_t *dst = reinterpret_cast<uint64_t *>(a.side);
        for (int j = threadIdx.x; j < static_cast<int>(sizeof(Precomp) / 8); j += kBlock) dst[j] = src[j];
        return;
    }
    const int tile = blockIdx.x - 1;
    const int64_t i = static_cast<int64_t>(tile) * kBlock + threadIdx.x;
    const int64_t n = a.n;
    const int64_t k = cs->k + 1;
    const T *kc = kc_of<T>(cs);
    const T eta = static_cast<T>(cs->eta_next);
    const T astar = static_cast<T>(st.alpha_star);
    double v[2] = {0.0, 0.0};
    bool accept = false;
    if (i < n) {
        T x[D], S[NC], U[D], y[D];
#pragma unroll
        for (int j = 0; j < D; ++j) x[j] = a.chi[j * n + i];
#pragma unroll
        for (int e = 0; e < NC; ++e) S[e] = a.chol[e * n + i];
        uint32_t nacc = a.acc[i];
        const typename M::Obj o = M::load(a.dd, i, n);
        const Block4 b = philox(static_cast<uint32_t>(i), static_cast<uint32_t>(k), 0u, 0u, st.key0, st.key1);
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
        accept = ln_uniform(b, T(0)) < delta;
        const T alpha = accept_prob(delta);
        if (accept) {
#pragma unroll
            for (int j = 0; j < D; ++j) x[j] = y[j];
            nacc += 1u;
        }
        const Eval<T> en = accept ? ey : ex;
        ram_adapt<T, D>(S, U, eta * (alpha - astar));
#pragma unroll
        for (int j = 0; j < D; ++j) a.chi[j * n + i] = x[j];
#pragma unroll
        for (int e = 0; e < NC; ++e) a.chol[e * n + i] = S[e];
        a.acc[i] = nacc;
        v[0] = static_cast<double>(en.lf);
        v[1] = static_cast<double>(M::dlf(o, x, en, kc, st));
        if (!(ex.lpv > neg_inf)) atomicOr(&cs->flags, kFlagNonFiniteState);
        if (kTrace) {
            a.trace[i] = ex.lp;
            a.trace[n + i] = ey.lp;
            a.trace[2 * n + i] = accept ? static_cast<T>(1) : static_cast<T>(0);
#pragma unroll
            for (int j = 0; j < D; ++j) a.trace[(3 + j) * n + i] = y[j];
        }
        if (a.snaps != nullptr && st.thin > 0 && k % st.thin == 0) {
            const int64_t snap = k / st.thin - 1;
            if (snap < st.snap_cap) {
#pragma unroll
                for (int j = 0; j < D; ++j) a.snaps[(snap * D + j) * n + i] = x[j];
            }
        }
    }
    // accepted moves: one ballot per wavefront
    __shared__ uint32_t nacc_w[kWavesPerBlock];
    const uint32_t nw = static_cast<uint32_t>(__popcll(__ballot(accept)));
    if ((threadIdx.x & (kWave - 1)) == 0) nacc_w[threadIdx.x / kWave] = nw;
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
        a.partials[tile] = v[0];
        a.partials[a.n_tiles + tile] = v[1];
        a.partials[2 * a.n_tiles + tile] = static_cast<double>((nacc_w[0] + nacc_w[1]) + (nacc_w[2] + nacc_w[3]));
    }
}

// Epilogue of a sweep (one workgroup): fixed-order reduction of the tile
// partials, bookkeeping, then (kFull) the theta step, then the proposal
// for the next sweep.
template <class M, bool kFull>
__global__ __launch_bounds__(kBlock) void epilogue_kernel(CycleState *cs, const Statics *stp, const double *partials,
                                                          const Precomp *side, double *theta_trace, int32_t n_tiles)
{
    __shared__ CycleState c;
    __shared__ Precomp pc;
    __shared__ double red[3][kWavesPerBlock];
    const Statics &st = *stp;
    // tile partials, structure of arrays [3][n_tiles]
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll 4
    for (int t = threadIdx.x; t < n_tiles; t += kBlock) {
        v[0] += partials[t];
        v[1] += partials[n_tiles + t];
        v[2] += partials[2 * n_tiles + t];
    }
    {
        const uint64_t *src = reinterpret_cast<const uint64_t *>(side);
        uint64_t *dst = reinterpret_cast<uint64_t *>(&pc);
        for (int j = threadIdx.x; j < static_cast<int>(sizeof(Precomp) / 8); j += kBlock) dst[j] = src[j];
    }
    stage_in(c, cs);                     // its barrier also publishes pc
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
        finish_sweep<M>(c, st, v, pc.zraw, pc);
        if (kFull) theta_mh<M>(c, st, theta_trace, pc.ln_u);
        prepare_next<M>(c, st, pc);
    }
    stage_out(cs, c);
}

// Theta step on its own, after a ram_sweep (plain cycle).
template <class M>
__global__ __launch_bounds__(kBlock) void theta_kernel(CycleState *cs, const Statics *st, const Precomp *side,
                                                       double *theta_trace)
{
    __shared__ CycleState c;
    __shared__ Precomp pc;
    {
        const uint64_t *src = reinterpret_cast<const uint64_t *>(side);
        uint64_t *dst = reinterpret_cast<uint64_t *>(&pc);
        for (int j = threadIdx.x; j < static_cast<int>(sizeof(Precomp) / 8); j += kBlock) dst[j] = src[j];
    }
    stage_in(c, cs);
    const bool ready = c.sums_ready != 0;
    if (threadIdx.x == 0) {
        if (ready) {
            theta_mh<M>(c, *st, theta_trace, pc.ln_u);
            prepare_next<M>(c, *st, pc);
        } else {
            c.flags |= kFlagNoSums;
        }
    }
    stage_out(cs, c);
}

// Recompute everything that depends on theta after it is set from the host.
template <class M>
__global__ __launch_bounds__(kBlock) void set_theta_kernel(CycleState *cs, const Statics *st, const double *qx,
                                                           const double *qw, const double *qeps)
{
    __shared__ CycleState c;
    __shared__ Precomp pc;
    __shared__ double red[1][kWavesPerBlock];
    stage_in(c, cs);
    const bool ok = M::in_support(c.theta);
    // the judged-proposal slots of pc carry theta itself here
    precompute<M>(pc, c.k, c.theta, ok, *st);
    double lz = 0.0;
    if (M::kSelection && ok) {
        double zc[2];
        M::z_consts(c.theta, zc);
        lz = block_log_z(zc, qx, qw, qeps, st->nq, red);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        c.lprior_cur = pc.lprior_used;
        c.aux_cur[0] = pc.aux_used[0];
        c.aux_cur[1] = pc.aux_used[1];
        c.logZ_cur = (M::kSelection && ok) ? lz - M::logz_shift(c.aux_cur) : 0.0;
        if (M::kSelection && ok && !(c.logZ_cur > -HUGE_VAL && c.logZ_cur < HUGE_VAL)) c.flags |= kFlagBadZ;
        c.sums_ready = 0;
        prepare_next<M>(c, *st, pc);
    }
    stage_out(cs, c);
}

template <class M>
__global__ void statics_kernel(Statics *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) M::derive_statics(*st);
}

template <class M>
__global__ __launch_bounds__(kBlock) void derive_data_kernel(const typename M::T *data, typename M::T *dd,
                                                             const Statics *st)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < st->n) M::derive_obj(data, dd, i, st->n, *st);
}

template <class M>
__global__ __launch_bounds__(kBlock) void init_chain_kernel(typename M::T *chol, uint32_t *acc, double s0,
                                                            const Statics *st)
{
    using T = typename M::T;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t n = st->n;
    if (i >= n) return;
    for (int r = 0, e = 0; r < M::D; ++r)
        for (int q = 0; q <= r; ++q, ++e) chol[e * n + i] = (r == q) ? static_cast<T>(s0) : static_cast<T>(0);
    acc[i] = 0u;
}

// Flags objects whose starting log density is not finite (pi(X_1) > 0 is required).
template <class M>
__global__ __launch_bounds__(kBlock) void check_init_kernel(const typename M::T *chi, const typename M::T *dd,
                                                            CycleState *cs, const Statics *st)
{
    using T = typename M::T;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t n = st->n;
    if (i >= n) return;
    T x[M::D];
    for (int j = 0; j < M::D; ++j) x[j] = chi[j * n + i];
    const Eval<T> e = M::eval(M::load(dd, i, n), x, kc_of<T>(cs), *st);
    if (!(e.lpv > -static_cast<T>(HUGE_VAL) && e.lpv < static_cast<T>(HUGE_VAL))) {
        atomicMin(&cs->first_bad, static_cast<int32_t>(i));
        atomicOr(&cs->flags, kFlagNonFiniteState);
    }
}

template <typename T>
struct PopArgs {
    const T *chi;
    const T *dd;
    double *partials;
    double *zout;
    const Statics *st;
    const double *qx, *qw, *qeps;
    int64_t n;
    double theta[kMaxP];
};

// Partial sums of log f(chi_i; theta) per tile; workgroup 0 evaluates ln Z(theta).
template <class M>
__global__ __launch_bounds__(kBlock) void poplik_kernel(PopArgs<typename M::T> a)
{
    using T = typename M::T;
    __shared__ double red[1][kWavesPerBlock];
    __shared__ T kc[32];
    const Statics &st = *a.st;
    double ag[2];
    M::aux(a.theta, ag);
    if (blockIdx.x == 0) {
        if (M::kSelection) {
            double zc[2];
            M::z_consts(a.theta, zc);
            const double lz = block_log_z(zc, a.qx, a.qw, a.qeps, st.nq, red);
            if (threadIdx.x == 0) a.zout[1] = lz - M::logz_shift(ag);
        } else if (threadIdx.x == 0) {
            a.zout[1] = 0.0;
        }
        return;
    }
    if (threadIdx.x == 0) M::derive_kc(a.theta, a.theta, ag, st, kc);
    __syncthreads();
    const int tile = blockIdx.x - 1;
    const int64_t i = static_cast<int64_t>(tile) * kBlock + threadIdx.x;
    double v[1] = {0.0};
    if (i < a.n) {
        T x[M::D];
        for (int j = 0; j < M::D; ++j) x[j] = a.chi[j * a.n + i];
        v[0] = static_cast<double>(M::eval(M::load(a.dd, i, a.n), x, kc, st).lf);
    }
    block_sum<1>(v, red);
    if (threadIdx.x == 0) a.partials[tile] = v[0];
}

__global__ __launch_bounds__(kBlock) void poplik_finish_kernel(CycleState *cs, const double *partials,
                                                               const double *zout, int64_t n, int32_t n_tiles)
{
    __shared__ double red[1][kWavesPerBlock];
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < n_tiles; t += kBlock) v[0] += partials[t];
    block_sum<1>(v, red);
    if (threadIdx.x == 0) {
        cs->poplik_logz = zout[1];
        cs->poplik_out = v[0] - static_cast<double>(n) * zout[1];
    }
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
__global__ void eps_table_kernel(const double *t, const double *w, double *qx, double *qw, double *qeps,
                                 const Statics *st)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int nq = st->nq;
    if (j >= nq) return;
    const double fth = st->mc[0], sigf = st->mc[1], rmax = st->mc[2], lnl0 = st->mc[3];
    const double lo = lnl0 - 30.0, hi = lnl0 + log(40.0);
    // nodes ascend in x: t descends with the node index
    const double x = 0.5 * (lo + hi) - 0.5 * (hi - lo) * t[j];
    qx[j] = x;
    qw[j] = 0.5 * (hi - lo) * w[j];
    const double lum_scaled = exp(x) / (4.0 * 3.14159265358979323846 * rmax * rmax);
    double acc = 0.0;
    for (int l = 0; l < nq; ++l) {
        const double s = -30.0 - 30.0 * t[l];
        const double flux = lum_scaled * exp(-2.0 * s / 3.0);
        const double eta = 0.5 * erfc(-(flux - fth) / (sigf * 1.4142135623730950488));
        acc += 30.0 * w[l] * exp(s) * eta;
    }
    qeps[j] = acc;
}

}  // namespace hbm
