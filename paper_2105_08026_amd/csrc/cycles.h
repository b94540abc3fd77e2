// Persistent cycle kernel: many Metropolis-within-Gibbs cycles (Sec. 2.1,
// eqs 2.4/2.5) of one dataset in a single cooperative launch.
//
// The two-kernel cycle (sweep_kernel, then the one-workgroup
// epilogue_kernel) pays, per cycle, two kernel launches and a round of loads
// of the tile partials from memory.  Here W co-resident workgroups (W
// divides 256; one per compute unit) stay on the device for all the
// cycles of a call:
//
//   1. each workgroup sweeps its own tiles (the same per-object step and the
//      same per-tile FP64 reduction as sweep_kernel) -- its tiles do not
//      change from cycle to cycle, so their latents and factors come back
//      from the compute unit's own L2;
//   2. it publishes its share of the 256 lane sums that the epilogue's fixed
//      reduction order defines: lane t sums tiles t, t + 256, t + 512, ...
//      in that order, and workgroup w owns lanes t = w mod W, so these sums
//      are bit for bit the epilogue's;
//   3. it computes the theta step's object-independent values (the side
//      workgroup's work in the two-kernel cycle) while the others finish;
//   4. it waits until all 256 lane sums of the cycle are visible, reduces
//      them exactly as the epilogue does, and takes the theta step itself.
//
// Every workgroup thus holds an identical copy of the theta chain; no second
// exchange is needed before the next sweep, and workgroup 0 writes the trace
// and, at the end, the state.  The chain is bit-identical to the two-kernel
// cycle's.
//
// Exchange without fences: each lane sum travels as two 64-bit words, each
// holding one 32-bit half of the double under a 32-bit tag unique to the
// cycle; words are written and read with device-scope atomic stores and
// loads, so a reader accepts a word only when its tag is the cycle's and
// never needs an ordering between words.  Two buffers alternate by cycle: a
// workgroup can only overwrite a buffer two cycles later, after every
// workgroup has read it.  Each wait is bounded (s_memrealtime, 100 MHz
// ticks): past the bound the workgroup raises a flag and leaves, and the
// others then time out in turn, so the grid always drains.
#pragma once

#include "kernels.h"

namespace hbm {

constexpr int kXchCols = 2 + kMaxStats;   // most columns of lane sums (statistics path)
constexpr int kMaxLanesPerGroup = 4;       // W >= 64

enum : int32_t { kFlagBarrierTimeout = 16 };

template <typename T>
struct CyclesArgs {
    SweepArgs<T> sw;           // the one dataset's arrays, state, statics and tables
    double *theta_trace;       // its theta trace
    uint64_t *xch;             // [2][kXchCols][2][256] tagged words
    int64_t n_cycles;
    int64_t spin_ticks;        // bound on one wait, in s_memrealtime ticks
    uint32_t tag0;             // tag of the launch's first cycle (then +1 per cycle)
    int32_t n_groups;          // W
};

__device__ __forceinline__ uint64_t *xch_word(uint64_t *x, int buf, int col, int half, int lane)
{
    return x + ((static_cast<int64_t>(buf) * kXchCols + col) * 2 + half) * kBlock + lane;
}

// B: tiles whose loads and steps are issued together.
template <class M, int B, bool kStats>
__global__ __launch_bounds__(kBlock) void cycles_kernel(CyclesArgs<typename M::T> a)
{
    using T = typename M::T;
    constexpr int D = M::D, NC = M::NC;
    constexpr int kCols = kStats ? 1 + M::NS : 2;      // FP64 sums per tile besides the accepted count
    constexpr int NCOL = kCols + 1;
    static_assert(NCOL <= kXchCols, "exchange columns");
    constexpr int kRed = kCols * B > NCOL ? kCols * B : NCOL;
    __shared__ CycleState c;
    __shared__ Precomp pc;
    __shared__ double red[kRed][kBlock];
    __shared__ double zred[1][kBlock];
    __shared__ uint32_t nacc_w[B][kWavesPerBlock];
    __shared__ double lsum[kMaxLanesPerGroup][NCOL];     // this workgroup's lane sums (thread 0)

    const SweepArgs<T> &sa = a.sw;
    const Statics &st = sa.st[0];
    const int W = a.n_groups, w = static_cast<int>(blockIdx.x);
    const int n_lanes = kBlock / W;                    // lane sums this workgroup owns
    const int32_t nt = sa.n_tiles_total;
    const int64_t n = sa.n_total;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;

    stage_in(c, sa.cs);
    bool stepped = false;
    for (int64_t j = 0; j < a.n_cycles; ++j) {
        if (!c.active) break;                          // uniform: LDS after a barrier
        stepped = true;
        const uint32_t tag = a.tag0 + static_cast<uint32_t>(j);
        const int buf = static_cast<int>(tag & 1u);
        // ---- 1. the sweep of this workgroup's tiles ------------------------
        const TileView<T> tv{c.k + 1, 0, st.n, st.snap_cap, st.key0, st.key1, st.thin, 1, st.snap_ring,
                             static_cast<T>(c.eta_next), static_cast<T>(st.alpha_star)};
        T kc[kKc];
#pragma unroll
        for (int q = 0; q < kKc; ++q) kc[q] = uniform_of(kc_of<T>(&c)[q]);
        for (int l = 0; l < n_lanes; ++l) {
            const int t = w + l * W;
            if (threadIdx.x == 0)
#pragma unroll
                for (int q = 0; q < NCOL; ++q) lsum[l][q] = 0.0;
            for (int m0 = 0; t + kBlock * m0 < nt; m0 += B) {
                T xs[B][D], Ss[B][NC];
                uint32_t na[B];
                typename M::Obj os[B];
                int64_t pos[B];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int64_t g = static_cast<int64_t>(t) + static_cast<int64_t>(kBlock) * (m0 + b);
                    pos[b] = g * kBlock + threadIdx.x;
                    // positions past the end read the last object instead (unused)
                    const int64_t i = pos[b] < n ? pos[b] : n - 1;
#pragma unroll
                    for (int r = 0; r < D; ++r) xs[b][r] = sa.chi[r * n + i];
#pragma unroll
                    for (int e = 0; e < NC; ++e) Ss[b][e] = sa.chol[e * n + i];
                    na[b] = sa.acc[i];
                    os[b] = M::load(sa.dd, i, n);
                }
                double v[kCols * B];
                bool accepted[B];
#pragma unroll
                for (int b = 0; b < B; ++b)
                    accepted[b] = step_object<M, false, kStats>(sa, 0, tv, pos[b], pos[b], xs[b], Ss[b], na[b], os[b],
                                                                v + kCols * b, pos[b] < n, kc);
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const uint32_t nw = static_cast<uint32_t>(__popcll(__ballot(accepted[b])));
                    if (lane == 0) nacc_w[b][wave] = nw;
                }
                block_sum<kCols * B>(v, red);
                if (threadIdx.x == 0) {
                    // tiles of the batch in ascending order, as the epilogue adds them
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        if (t + kBlock * (m0 + b) >= nt) continue;
#pragma unroll
                        for (int q = 0; q < kCols; ++q) lsum[l][q] += v[kCols * b + q];
                        lsum[l][kCols] +=
                            static_cast<double>((nacc_w[b][0] + nacc_w[b][1]) + (nacc_w[b][2] + nacc_w[b][3]));
                    }
                }
                __syncthreads();                       // red and nacc_w are reused
            }
        }
        // ---- 2. publish the lane sums --------------------------------------
        if (threadIdx.x == 0) {
            for (int l = 0; l < n_lanes; ++l) {
                const int t = w + l * W;
#pragma unroll
                for (int q = 0; q < NCOL; ++q) {
                    const uint64_t bits = __builtin_bit_cast(uint64_t, lsum[l][q]);
                    const uint64_t hi_tag = static_cast<uint64_t>(tag) << 32;
                    __hip_atomic_store(xch_word(a.xch, buf, q, 0, t), hi_tag | (bits & 0xffffffffu), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(xch_word(a.xch, buf, q, 1, t), hi_tag | (bits >> 32), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        // ---- 3. the theta step's values that the objects do not decide ------
        {
            const bool valid = c.prop_valid != 0;
            double judged[kMaxP];
            for (int r = 0; r < M::P; ++r) judged[r] = c.prop[r];
            double zraw = 0.0;
            if constexpr (M::kSelection) {
                if (valid) {
                    double zc[4] = {c.zc_prop[0], c.zc_prop[1], c.zc_prop[2], c.zc_prop[3]};
                    zraw = block_log_z<M>(zc, sa.qx, sa.qw, sa.qeps, sa.nq, zred);
                }
            }
            precompute<M>(pc, c.k + 1, judged, valid, st);
            if (threadIdx.x == 0) pc.zraw = zraw;
            __syncthreads();
            if (threadIdx.x == 0) {
                pc.logz_used = (valid && M::kSelection) ? zraw - M::logz_shift(pc.aux_used) : 0.0;
                pc.dconst = valid ? static_cast<double>(st.n) * M::dlf_const(c.theta, judged, c.aux_cur, pc.aux_used)
                                  : 0.0;
            }
        }
        // ---- 4. wait for every lane sum of this cycle ------------------------
        double v[NCOL];
        bool timed_out = false;
        {
            uint64_t wv[NCOL][2];
            uint32_t have = 0;                         // bit 2q + h: word (q, h) arrived
            constexpr uint32_t kAll = (1u << (2 * NCOL)) - 1u;
            const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
            for (;;) {
#pragma unroll
                for (int q = 0; q < NCOL; ++q)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t bit = 1u << (2 * q + h);
                        if (have & bit) continue;
                        wv[q][h] = __hip_atomic_load(xch_word(a.xch, buf, q, h, threadIdx.x), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                        if (static_cast<uint32_t>(wv[q][h] >> 32) == tag) have |= bit;
                    }
                if (have == kAll) break;
                if (__builtin_amdgcn_s_memrealtime() - t_start > static_cast<uint64_t>(a.spin_ticks)) {
                    timed_out = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
#pragma unroll
            for (int q = 0; q < NCOL; ++q)
                v[q] = __builtin_bit_cast(double, (wv[q][1] << 32) | (wv[q][0] & 0xffffffffu));
        }
        if (__syncthreads_or(timed_out)) {
            if (threadIdx.x == 0) atomicOr(&sa.cs[0].flags, kFlagBarrierTimeout);
            return;                                    // the state stays as it was; the host poisons the context
        }
        // ---- 5. the fixed-order reduction and the theta step -----------------
        block_sum<NCOL>(v, red);
        double *trace = w == 0 ? a.theta_trace : nullptr;
        if constexpr (kStats) {
            if (threadIdx.x == 0) finish_sweep<M, true>(c, st, v, pc);
            __syncthreads();
            theta_substeps<M>(c, st, trace, pc, sa.qx, sa.qw, sa.qeps, sa.nq, zred);
            if (threadIdx.x == 0) prepare_next<M>(c, st, pc);
        } else if (threadIdx.x == 0) {
            finish_sweep<M>(c, st, v, pc);
            theta_mh<M>(c, st, trace, pc.ln_u);
            prepare_next<M>(c, st, pc);
        }
        __syncthreads();
    }
    // ---- the state back to memory (workgroup 0): every word but the flags,
    // which the tiles may have raised meanwhile, then this copy's flags ------
    if (w == 0 && stepped) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&c);
        uint32_t *dst = reinterpret_cast<uint32_t *>(sa.cs);
        constexpr int kWords = static_cast<int>(sizeof(CycleState) / 4);
        constexpr int kFlagsWord = static_cast<int>(offsetof(CycleState, flags) / 4);
        for (int q = threadIdx.x; q < kWords; q += kBlock)
            if (q != kFlagsWord) dst[q] = src[q];
        if (threadIdx.x == 0 && c.flags != 0) atomicOr(&sa.cs[0].flags, c.flags);
    }
}

}  // namespace hbm
