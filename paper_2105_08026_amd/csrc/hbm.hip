// Host runtime and C ABI of the sampler (declared in include/hbm.h).
//
// The host only validates arguments, allocates the library's scratch,
// keeps the slot table of a pool, enqueues kernels and copies results; all
// sampler arithmetic runs in the kernels of kernels.h.
//
// A context is a pool of slots.  Each loaded slot holds one dataset whose
// objects occupy a contiguous, tile-aligned range of the caller's packed
// [component][capacity] buffers.  Every launch covers all slots at once
// (one side workgroup per slot, one workgroup per 256-object tile); a
// device-side flag per slot switches a dataset off when it is unloaded or
// its theta-step budget is spent, so a captured graph stays valid while
// datasets come and go.
#include "hbm.h"
#include "cycles.h"
#include "kernels.h"
#include "marginal.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <climits>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace hbm;

// Device memory of marginal_loglik_noalloc, for callers that cannot allocate:
// the marginal likelihood's node rule, then one call's theta rows, results,
// workgroup partial sums and per-row scalars.  Each device the library runs
// on holds its own copy until the process ends.  Host code never passes this
// name to a kernel or a copy (on the host it is only a stand-in): it uses the
// per-device address that hipGetSymbolAddress returns.
constexpr size_t kNoAllocScratchBytes = size_t(HBM_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_init_error;

// exchange words of the persistent cycle kernel: [2][kXchCols][2][256]
constexpr size_t kXchBytes = sizeof(uint64_t) * 2 * kXchCols * 2 * kBlock;
// bound on one wait inside the persistent kernel: 2 s of s_memrealtime (100 MHz)
constexpr int64_t kSpinTicks = 200000000;
// warm-up cycles of each autotuner candidate before its timed cycles
constexpr int64_t kTuneWarm = 8;

struct CtxImpl;

struct Launch {
    hbm_status (*sweep)(CtxImpl *, bool full, void *trace);
    hbm_status (*theta)(CtxImpl *);
    hbm_status (*set_theta)(CtxImpl *);       // slots flagged in c->which
    hbm_status (*poplik)(CtxImpl *);          // theta of every slot in c->theta_in
    hbm_status (*prepare)(CtxImpl *);         // slots flagged in c->which
    hbm_status (*check_init)(CtxImpl *);      // slots flagged in c->which
    hbm_status (*quadrature)(CtxImpl *);      // reference Gauss-Legendre rule
    hbm_status (*marginal)(CtxImpl *, int32_t slot, int32_t n_theta, const double *theta, double *out,
                           double *partials, double *th, double *terms, const MargNode *rule);   // device arguments
    // n full cycles as one persistent cooperative launch; *launched = false
    // (and nothing enqueued) when the context or device cannot take it
    hbm_status (*cycles)(CtxImpl *, int64_t n, bool *launched);
    hbm_status (*fused)(CtxImpl *, int64_t len);  // len >= 2 fused cycles
};

// Host mirror of one slot.  Every field follows from the calls made, so the
// host never has to read the device to know a slot's progress.
struct Slot {
    bool loaded = false;
    bool active = false;       // loaded and budget not spent
    bool sums_ready = false;   // a plain sweep waits for its theta step
    int64_t n = 0, obj_start = 0;
    int32_t tile_start = 0, n_tiles = 0;
    int64_t k = 0, n_theta = 0, budget = 0, trace_cap = 0, snap_cap = 0;
    int32_t thin = 0;
};

struct CtxImpl {
    hbm_pool_config pool{};
    hbm_buffers buf{};
    int d = 0, p = 0, m = 0, md = 0, nc = 0;
    size_t esize = 0;
    int64_t cap = 0;                // object positions (array stride)
    int32_t n_tiles = 0;            // ceil(cap / 256)
    int32_t n_slots = 0;
    int32_t nq = 1;
    int32_t tpw = 1;                // tiles per sweep workgroup (1, 2 or 4)
    int32_t occ_cap = 0;            // most sweep workgroups per compute unit (0: as many as fit)
    // dynamic LDS that holds a sweep kernel to occ_cap workgroups per CU, per (kernel, cap)
    std::vector<std::pair<std::pair<const void *, int32_t>, size_t>> occ_lds;
    bool stats_mode = false;        // theta steps from sufficient statistics
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    int device = -1;                // ordinal of the device holding the buffers
    void *dd = nullptr;             // [md][cap] derived per-object data
    double *partials = nullptr;     // [2 + kMaxStats][n_tiles]: tile sums, then accepted counts
    double *pout = nullptr;         // [n_slots][2] results of pop_loglik
    double *theta_in = nullptr;     // [n_slots][p] arguments of pop_loglik
    Precomp *side = nullptr;        // [n_slots] values the side workgroups leave for the epilogue
    // the other buffers of a fused run: chain states, tile partials, side values
    CycleState *cs_alt = nullptr;
    double *partials_alt = nullptr;
    Precomp *side_alt = nullptr;
    double *ref_t = nullptr, *ref_w = nullptr;       // [nq]
    double *qx = nullptr, *qw = nullptr, *qeps = nullptr;   // [n_slots][nq]
    CycleState *cs = nullptr;       // [n_slots]
    Statics *st = nullptr;          // [n_slots]
    double *theta_trace = nullptr;  // [n_slots][max_cycles][p]
    int32_t *tile_ds = nullptr;     // [n_tiles] slot of each tile or -1
    int32_t *which = nullptr;       // [n_slots] slots an initialisation kernel acts on
    std::vector<Slot> slots;
    std::vector<int32_t> h_tile_ds, h_which;
    std::vector<CycleState> h_cs;   // staging of state reads
    bool poisoned = false;
    std::string err;
    const Launch *ops = nullptr;
    // graphs of consecutive full cycles: kGraphCycles of them, and one of
    // the remainder a run_cycles call last needed
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t graph_len = 0;
    hipGraphExec_t tail_exec = nullptr;
    hipGraph_t tail = nullptr;
    int64_t tail_len = 0;
    // cycles issued by run_cycles: graph replays, cycles inside them, plain cycles, graph captures,
    // persistent launches and the cycles inside them
    int64_t n_replays = 0, n_replayed_cycles = 0, n_plain_cycles = 0, n_captures = 0;
    int64_t n_persistent = 0, n_persistent_cycles = 0;
    // persistent cycle kernel: exchange words, the next cycle's tag, its
    // grid (0: not yet decided, -1: unavailable) and whether it may be used
    uint64_t *xch = nullptr;
    uint32_t xch_tag = 1;
    int32_t persist_groups = 0;
    int32_t cycle_mode = HBM_CYCLES_AUTO;
    // launch extent of the cycle kernels in a multi-slot context: side and
    // epilogue workgroups for slots [0, ext_slots), tile workgroups for tiles
    // [0, ext_tiles), up to the last loaded slot and occupied tile
    int32_t ext_slots = 1, ext_tiles = 0;
    // latent snapshots: the pointer kernels write through (chi_samples, or its
    // device mapping when the caller gave pinned host memory)
    void *snaps_dev = nullptr;
    bool snaps_host = false;
    // streamed runs: the copy stream and its events
    hipStream_t copy_stream = nullptr;
    hipEvent_t swept[2] = {nullptr, nullptr}, copied[2] = {nullptr, nullptr};
    // marginal likelihood: node tables (datum rule, then product rule) and a
    // scratch area grown on demand for theta, results and partial sums
    MargNode *marg_rule = nullptr;
    double *marg_buf = nullptr;
    size_t marg_bytes = 0;
    // per-launch timing of the sweep and marginal kernels
    bool timing = false;
    std::vector<hipEvent_t> ev_free, ev_pending;
    int64_t timed_launches = 0;
    double timed_ms = 0.0;
};

}  // namespace

// The opaque handle of the C ABI.
struct hbm_ctx : CtxImpl {};

namespace {

hbm_status fail(CtxImpl *c, hbm_status code, const std::string &msg)
{
    if (c) c->err = msg; else g_init_error = msg;
    return code;
}

hbm_status hip_fail(CtxImpl *c, hipError_t e, const char *what)
{
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    if (c) {
        c->poisoned = true;
        c->err = msg;
    } else {
        g_init_error = msg;
    }
    return HBM_EHIP;
}

#define HIPCHK(c, call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail((c), e_, #call); \
    } while (0)

#define LAUNCHCHK(c, what)                                \
    do {                                                  \
        hipError_t e_ = hipGetLastError();                \
        if (e_ != hipSuccess) return hip_fail((c), e_, what); \
    } while (0)

int32_t tiles_for(int64_t n) { return static_cast<int32_t>((n + kBlock - 1) / kBlock); }

bool single(const CtxImpl *c);
void setup_noalloc_scratch(CtxImpl *c);

// Events that time one sweep-kernel launch.
hipEvent_t take_event(CtxImpl *c)
{
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Workgroups of the marginal kernel for n objects (kMargLanes lanes each).
int32_t marg_blocks(int64_t n)
{
    constexpr int64_t per = kBlock / kMargLanes;
    return static_cast<int32_t>((n + per - 1) / per);
}

constexpr int kMargShapeNodes = 2 * MargRuleShape::kCore + MargRuleShape::kGraded + MargRuleShape::kTail;
constexpr int kMargProductNodes = 2 * MargRuleProduct::kCore;

// Dynamic LDS (unused by the kernel) that limits fn, launched with threads
// per workgroup, to c->occ_cap resident workgroups per compute unit: the
// smallest multiple of 256 bytes at which the occupancy calculator reports
// no more than the cap (the largest the device allows, if even that leaves
// more).  Cached per kernel and cap.
size_t occupancy_lds(CtxImpl *c, const void *fn, int threads = kBlock)
{
    const auto key = std::make_pair(fn, c->occ_cap);
    for (const auto &e : c->occ_lds)
        if (e.first == key) return e.second;
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
        max_lds = 65536;
    auto fits = [&](size_t lds) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return nb <= c->occ_cap;
    };
    size_t lo = 0, hi = static_cast<size_t>(max_lds) / 256;   // in units of 256 bytes
    size_t pick = 0;
    if (!fits(0)) {
        if (!fits(hi * 256)) {
            pick = hi * 256;
        } else {
            while (hi - lo > 1) {
                const size_t mid = (lo + hi) / 2;
                if (fits(mid * 256)) hi = mid;
                else lo = mid;
            }
            pick = hi * 256;
        }
    }
    (void)hipGetLastError();
    c->occ_lds.push_back(std::make_pair(key, pick));
    return pick;
}

// Workgroups of the persistent cycle kernel: the largest of 256, 128 and 64
// that the device holds at once (cooperative launch), or -1.
int32_t persistent_groups(CtxImpl *c, const void *fn)
{
    int coop = 0, cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device) != hipSuccess || !coop ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    const int64_t fit = static_cast<int64_t>(cus) * per_cu;
    for (int32_t w : {256, 128, 64})
        if (w <= fit) return w;
    return -1;
}

template <class M>
struct Ops {
    using T = typename M::T;

    static SweepArgs<T> sweep_args(CtxImpl *c, void *trace)
    {
        SweepArgs<T> a;
        a.chi = static_cast<T *>(c->buf.chi);
        a.chol = static_cast<T *>(c->buf.chol);
        a.acc = c->buf.acc;
        a.dd = static_cast<const T *>(c->dd);
        a.snaps = static_cast<T *>(c->snaps_dev);
        a.trace = static_cast<T *>(trace);
        a.partials = c->partials;
        a.side = c->side;
        a.cs = c->cs;
        a.st = c->st;
        a.qx = c->qx;
        a.qw = c->qw;
        a.qeps = c->qeps;
        a.tile_ds = c->tile_ds;
        a.n_total = c->cap;
        a.n_tiles_total = c->n_tiles;
        // a multi-slot context launches only up to its last loaded slot and
        // occupied tile: the workgroups beyond would find nothing to do
        a.n_ds = single(c) ? c->n_slots : c->ext_slots;
        a.nq = c->nq;
        return a;
    }

    static hbm_status sweep(CtxImpl *c, bool full, void *trace)
    {
        const SweepArgs<T> a = sweep_args(c, trace);
        const bool whole = single(c);
        const int32_t n_t = whole ? c->n_tiles : c->ext_tiles;
        // traced sweeps (a checking aid) always take one tile per workgroup
        const int tpw = trace ? 1 : c->tpw;
        const dim3 grid(static_cast<unsigned>(a.n_ds + (n_t + tpw - 1) / tpw));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            // the runtime takes both timestamps from the dispatch itself
            e0 = take_event(c);
            e1 = take_event(c);
            if (!e0 || !e1) return fail(c, HBM_ENOMEM, "hipEventCreate failed");
            c->ev_pending.push_back(e0);
            c->ev_pending.push_back(e1);
        }
        if constexpr (M::NS > 0) {
            if (c->stats_mode) return sweep_as<true>(c, full, trace, grid, tpw, a, e0, e1);
        }
        return sweep_as<false>(c, full, trace, grid, tpw, a, e0, e1);
    }

    template <bool kStats>
    static hbm_status sweep_as(CtxImpl *c, bool full, void *trace, dim3 grid, int tpw, const SweepArgs<T> &a,
                               hipEvent_t e0, hipEvent_t e1)
    {
        const bool one = single(c);
        if (trace) launch_sweep<true, 1, false, kStats>(c, grid, a, e0, e1);
        else if (one && tpw == 4) launch_sweep<false, 4, true, kStats>(c, grid, a, e0, e1);
        else if (one && tpw == 2) launch_sweep<false, 2, true, kStats>(c, grid, a, e0, e1);
        else if (one) launch_sweep<false, 1, true, kStats>(c, grid, a, e0, e1);
        else if (tpw == 4) launch_sweep<false, 4, false, kStats>(c, grid, a, e0, e1);
        else if (tpw == 2) launch_sweep<false, 2, false, kStats>(c, grid, a, e0, e1);
        else launch_sweep<false, 1, false, kStats>(c, grid, a, e0, e1);
        LAUNCHCHK(c, "sweep_kernel");
        const EpiArgs e = epi_args(c);
        if (full && one)
            hipLaunchKernelGGL((epilogue_kernel<M, true, true, kStats>), dim3(1), dim3(kBlock), 0, c->stream, e);
        else if (full)
            hipLaunchKernelGGL((epilogue_kernel<M, true, false, kStats>), dim3(c->ext_slots), dim3(kBlock), 0,
                               c->stream, e);
        else if (one)
            hipLaunchKernelGGL((epilogue_kernel<M, false, true, kStats>), dim3(1), dim3(kBlock), 0, c->stream, e);
        else
            hipLaunchKernelGGL((epilogue_kernel<M, false, false, kStats>), dim3(c->ext_slots), dim3(kBlock), 0,
                               c->stream, e);
        LAUNCHCHK(c, "epilogue_kernel");
        return HBM_OK;
    }

    template <bool kTrace, int TPW, bool kSingle, bool kStats>
    static void launch_sweep(CtxImpl *c, dim3 grid, const SweepArgs<T> &a, hipEvent_t e0, hipEvent_t e1)
    {
        const size_t lds = c->occ_cap > 0 ? occupancy_lds(c, reinterpret_cast<const void *>(
                                                                 &sweep_kernel<M, kTrace, TPW, kSingle, kStats>))
                                          : 0;
        if (e0)
            hipExtLaunchKernelGGL((sweep_kernel<M, kTrace, TPW, kSingle, kStats>), grid, dim3(kBlock), lds,
                                  c->stream, e0, e1, 0, a);
        else
            hipLaunchKernelGGL((sweep_kernel<M, kTrace, TPW, kSingle, kStats>), grid, dim3(kBlock), lds, c->stream,
                               a);
    }

    // len >= 2 full cycles with one launch per cycle after the first: the
    // sweep kernel (its state, partials and side values in the primary
    // buffers), len - 1 fused kernels, each taking the previous sweep's theta
    // step and running the next sweep with the buffers alternating, then the
    // last sweep's epilogue, which leaves the state in the primary buffer.
    // A context with several datasets runs one tile per workgroup
    // (fused_pool_kernel) whatever its launch shape.
    static hbm_status fused(CtxImpl *c, int64_t len)
    {
        if constexpr (M::NS > 0) {
            if (c->stats_mode) return fused_as<true>(c, len);
        }
        return fused_as<false>(c, len);
    }

    template <bool kStats>
    static hbm_status fused_as(CtxImpl *c, int64_t len)
    {
        const SweepArgs<T> a = sweep_args(c, nullptr);
        const bool one = single(c);
        const int tpw = one ? c->tpw : 1;
        const int32_t n_t = one ? c->n_tiles : c->ext_tiles;
        const dim3 grid(static_cast<unsigned>(a.n_ds + (n_t + tpw - 1) / tpw));
        if (!one) launch_sweep<false, 1, false, kStats>(c, grid, a, nullptr, nullptr);
        else if (tpw == 4) launch_sweep<false, 4, true, kStats>(c, grid, a, nullptr, nullptr);
        else if (tpw == 2) launch_sweep<false, 2, true, kStats>(c, grid, a, nullptr, nullptr);
        else launch_sweep<false, 1, true, kStats>(c, grid, a, nullptr, nullptr);
        LAUNCHCHK(c, "sweep_kernel");
        CycleState *csb[2] = {c->cs, c->cs_alt};
        double *pb[2] = {c->partials, c->partials_alt};
        Precomp *sb[2] = {c->side, c->side_alt};
        int cur = 0;
        for (int64_t j = 1; j < len; ++j) {
            FusedArgs<T> f;
            f.sw = a;
            f.sw.cs = csb[1 - cur];
            f.sw.partials = pb[1 - cur];
            f.sw.side = sb[1 - cur];
            f.epi = epi_args(c);
            f.epi.cs = f.epi.cs_out = csb[cur];
            f.epi.partials = pb[cur];
            f.epi.side = sb[cur];
            const hbm_status st = !one       ? launch_fused_pool<kStats>(c, grid, f)
                                  : tpw == 4 ? launch_fused<4, kStats>(c, grid, f)
                                  : tpw == 2 ? launch_fused<2, kStats>(c, grid, f)
                                             : launch_fused<1, kStats>(c, grid, f);
            if (st != HBM_OK) return st;
            LAUNCHCHK(c, "fused_kernel");
            cur = 1 - cur;
        }
        EpiArgs e = epi_args(c);
        e.cs = csb[cur];
        e.cs_out = c->cs;
        e.partials = pb[cur];
        e.side = sb[cur];
        if (one)
            hipLaunchKernelGGL((epilogue_kernel<M, true, true, kStats>), dim3(1), dim3(kBlock), 0, c->stream, e);
        else
            hipLaunchKernelGGL((epilogue_kernel<M, true, false, kStats>), dim3(c->ext_slots), dim3(kBlock), 0,
                               c->stream, e);
        LAUNCHCHK(c, "epilogue_kernel");
        return HBM_OK;
    }

    template <bool kStats>
    static hbm_status launch_fused_pool(CtxImpl *c, dim3 grid, const FusedArgs<T> &f)
    {
        void (*fn)(FusedArgs<T>) = &fused_pool_kernel<M, kStats>;
        const size_t lds = c->occ_cap > 0 ? occupancy_lds(c, reinterpret_cast<const void *>(fn)) : 0;
        if (c->timing) {
            hipEvent_t e0 = take_event(c), e1 = take_event(c);
            if (!e0 || !e1) return fail(c, HBM_ENOMEM, "hipEventCreate failed");
            c->ev_pending.push_back(e0);
            c->ev_pending.push_back(e1);
            hipExtLaunchKernelGGL(fn, grid, dim3(kBlock), lds, c->stream, e0, e1, 0, f);
        } else {
            hipLaunchKernelGGL(fn, grid, dim3(kBlock), lds, c->stream, f);
        }
        return HBM_OK;
    }

    // TPW tiles per workgroup: one object per thread in TPW x 256 threads
    // (fused_wide_kernel), or TPW objects per thread in 256 threads with
    // theta sub-steps (fused_kernel, whose sub-steps use 256-thread reductions)
    template <int TPW, bool kStats>
    static hbm_status launch_fused(CtxImpl *c, dim3 grid, const FusedArgs<T> &f)
    {
        constexpr bool kWide = TPW > 1 && !kStats;
        constexpr int kThreads = kWide ? kBlock * TPW : kBlock;
        void (*fn)(FusedArgs<T>);
        if constexpr (kWide) fn = &fused_wide_kernel<M, TPW>;
        else fn = &fused_kernel<M, TPW, kStats>;
        const size_t lds = c->occ_cap > 0 ? occupancy_lds(c, reinterpret_cast<const void *>(fn), kThreads) : 0;
        if (c->timing) {
            // the runtime takes both timestamps from the dispatch itself
            hipEvent_t e0 = take_event(c), e1 = take_event(c);
            if (!e0 || !e1) return fail(c, HBM_ENOMEM, "hipEventCreate failed");
            c->ev_pending.push_back(e0);
            c->ev_pending.push_back(e1);
            hipExtLaunchKernelGGL(fn, grid, dim3(kThreads), lds, c->stream, e0, e1, 0, f);
        } else {
            hipLaunchKernelGGL(fn, grid, dim3(kThreads), lds, c->stream, f);
        }
        return HBM_OK;
    }

    static EpiArgs epi_args(CtxImpl *c)
    {
        EpiArgs e;
        e.cs = c->cs;
        e.cs_out = c->cs;
        e.st = c->st;
        e.partials = c->partials;
        e.side = c->side;
        e.theta_trace = c->theta_trace;
        e.qx = c->qx;
        e.qw = c->qw;
        e.qeps = c->qeps;
        e.trace_stride = c->pool.max_cycles;
        e.n_tiles_total = c->n_tiles;
        e.nq = c->nq;
        return e;
    }

    static hbm_status theta(CtxImpl *c)
    {
        bool launched = false;
        if constexpr (M::NS > 0) {
            if (c->stats_mode) {
                hipLaunchKernelGGL((theta_kernel<M, true>), dim3(c->n_slots), dim3(kBlock), 0, c->stream, epi_args(c));
                launched = true;
            }
        }
        if (!launched) hipLaunchKernelGGL((theta_kernel<M>), dim3(c->n_slots), dim3(kBlock), 0, c->stream, epi_args(c));
        LAUNCHCHK(c, "theta_kernel");
        return HBM_OK;
    }

    static hbm_status set_theta(CtxImpl *c)
    {
        hipLaunchKernelGGL((set_theta_kernel<M>), dim3(c->n_slots), dim3(kBlock), 0, c->stream, c->cs, c->st, c->qx,
                           c->qw, c->qeps, c->nq, c->which);
        LAUNCHCHK(c, "set_theta_kernel");
        return HBM_OK;
    }

    static hbm_status poplik(CtxImpl *c)
    {
        PopArgs<T> a;
        a.chi = static_cast<const T *>(c->buf.chi);
        a.dd = static_cast<const T *>(c->dd);
        a.partials = c->partials;
        a.pout = c->pout;
        a.theta = c->theta_in;
        a.st = c->st;
        a.qx = c->qx;
        a.qw = c->qw;
        a.qeps = c->qeps;
        a.tile_ds = c->tile_ds;
        a.n_total = c->cap;
        a.n_tiles_total = c->n_tiles;
        a.n_ds = c->n_slots;
        a.nq = c->nq;
        hipLaunchKernelGGL((poplik_kernel<M>), dim3(c->n_slots + c->n_tiles), dim3(kBlock), 0, c->stream, a);
        LAUNCHCHK(c, "poplik_kernel");
        hipLaunchKernelGGL(poplik_finish_kernel, dim3(c->n_slots), dim3(kBlock), 0, c->stream, c->st, c->partials,
                           c->pout);
        LAUNCHCHK(c, "poplik_finish_kernel");
        return HBM_OK;
    }

    static hbm_status prepare(CtxImpl *c)
    {
        hipLaunchKernelGGL((statics_kernel<M>), dim3(c->n_slots), dim3(1), 0, c->stream, c->st, c->which);
        LAUNCHCHK(c, "statics_kernel");
        hipLaunchKernelGGL((derive_data_kernel<M>), dim3(c->n_tiles), dim3(kBlock), 0, c->stream,
                           static_cast<const T *>(c->buf.data), static_cast<T *>(c->dd), c->st, c->tile_ds, c->which,
                           c->cap);
        LAUNCHCHK(c, "derive_data_kernel");
        hipLaunchKernelGGL((init_chain_kernel<M>), dim3(c->n_tiles), dim3(kBlock), 0, c->stream,
                           static_cast<T *>(c->buf.chol), c->buf.acc, c->st, c->tile_ds, c->which, c->cap);
        LAUNCHCHK(c, "init_chain_kernel");
        if constexpr (M::kSelection) {
            hipLaunchKernelGGL((eps_table_kernel<M>), dim3((c->nq + 63) / 64, c->n_slots), dim3(64), 0, c->stream, c->ref_t,
                               c->ref_w, c->qx, c->qw, c->qeps, c->st, c->which);
            LAUNCHCHK(c, "eps_table_kernel");
        }
        return HBM_OK;
    }

    static hbm_status check_init(CtxImpl *c)
    {
        hipLaunchKernelGGL((check_init_kernel<M>), dim3(c->n_tiles), dim3(kBlock), 0, c->stream,
                           static_cast<const T *>(c->buf.chi), static_cast<const T *>(c->dd), c->cs, c->st,
                           c->tile_ds, c->which, c->cap);
        LAUNCHCHK(c, "check_init_kernel");
        return HBM_OK;
    }

    static hbm_status quadrature(CtxImpl *c)
    {
        if (!M::kSelection) return HBM_OK;
        hipLaunchKernelGGL(gauss_legendre_kernel, dim3((c->nq + 127) / 128), dim3(128), 0, c->stream, c->ref_t,
                           c->ref_w, c->nq);
        LAUNCHCHK(c, "gauss_legendre_kernel");
        return HBM_OK;
    }

    static hbm_status marginal(CtxImpl *c, int32_t slot, int32_t n_theta, const double *theta, double *out,
                               double *partials, double *th, double *terms, const MargNode *rule)
    {
        if constexpr (HasMarg<M>::value) {
            using R = typename Marg<M>::R;
            hipLaunchKernelGGL((marginal_prep_kernel<M>), dim3((n_theta + 63) / 64), dim3(64), 0, c->stream, theta,
                               th, n_theta);
            LAUNCHCHK(c, "marginal_prep_kernel");
            MargArgs a;
            a.data = c->buf.data;
            a.rule = rule + (R::kGraded > 0 ? 0 : kMargShapeNodes);
            a.theta = theta;
            a.th = th;
            a.partials = partials;
            a.terms = terms;
            a.st = c->st + slot;
            a.cap = c->cap;
            a.n_blocks = marg_blocks(c->slots[slot].n);
            const dim3 grid(static_cast<unsigned>(a.n_blocks), static_cast<unsigned>(n_theta));
            if (c->timing) {
                hipEvent_t e0 = take_event(c), e1 = take_event(c);
                if (!e0 || !e1) return fail(c, HBM_ENOMEM, "hipEventCreate failed");
                c->ev_pending.push_back(e0);
                c->ev_pending.push_back(e1);
                hipExtLaunchKernelGGL((marginal_kernel<M>), grid, dim3(kBlock), 0, c->stream, e0, e1, 0, a);
            } else {
                hipLaunchKernelGGL((marginal_kernel<M>), grid, dim3(kBlock), 0, c->stream, a);
            }
            LAUNCHCHK(c, "marginal_kernel");
            const int64_t qo = static_cast<int64_t>(slot) * c->nq;
            hipLaunchKernelGGL((marginal_finish_kernel<M>), dim3(static_cast<unsigned>(n_theta)), dim3(kBlock), 0,
                               c->stream, theta, partials, a.n_blocks, c->st + slot, c->qx + qo, c->qw + qo,
                               c->qeps + qo, c->nq, out);
            LAUNCHCHK(c, "marginal_finish_kernel");
            return HBM_OK;
        } else {
            (void)slot; (void)n_theta; (void)theta; (void)out; (void)partials; (void)th; (void)terms; (void)rule;
            return fail(c, HBM_EINVAL, "the marginal likelihood needs a model with a 1-D latent");
        }
    }

    static hbm_status cycles(CtxImpl *c, int64_t n, bool *launched)
    {
        *launched = false;
        if (c->cycle_mode != HBM_CYCLES_AUTO || !single(c)) return HBM_OK;
        if constexpr (M::NS > 0) {
            if (c->stats_mode) return cycles_as<true>(c, n, launched);
        }
        if (c->stats_mode) return HBM_OK;
        return cycles_as<false>(c, n, launched);
    }

    template <bool kStats>
    static hbm_status cycles_as(CtxImpl *c, int64_t n, bool *launched)
    {
        // tiles per register batch: four single-precision 1-D objects, else two
        constexpr int B = (M::D == 1 && sizeof(T) == 4) ? 4 : 2;
        const void *fn = reinterpret_cast<const void *>(&cycles_kernel<M, B, kStats>);
        if (c->persist_groups == 0) c->persist_groups = persistent_groups(c, fn);
        if (c->persist_groups < 0) return HBM_OK;
        CyclesArgs<T> a;
        a.sw = sweep_args(c, nullptr);
        a.theta_trace = c->theta_trace;
        a.xch = c->xch;
        a.n_cycles = n;
        a.spin_ticks = kSpinTicks;
        a.tag0 = c->xch_tag;
        a.n_groups = c->persist_groups;
        void *args[] = {&a};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            e0 = take_event(c);
            e1 = take_event(c);
            if (!e0 || !e1) return fail(c, HBM_ENOMEM, "hipEventCreate failed");
            HIPCHK(c, hipEventRecord(e0, c->stream));
        }
        const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(static_cast<unsigned>(a.n_groups)), dim3(kBlock), args,
                                                        0, c->stream);
        if (e != hipSuccess) {
            // the device would not take the grid: graphs from now on
            (void)hipGetLastError();
            c->persist_groups = -1;
            if (e0) c->ev_free.push_back(e0);
            if (e1) c->ev_free.push_back(e1);
            return HBM_OK;
        }
        if (c->timing) {
            HIPCHK(c, hipEventRecord(e1, c->stream));
            c->ev_pending.push_back(e0);
            c->ev_pending.push_back(e1);
        }
        // tags never repeat within 2^32 cycles; 0 (the buffer's initial words) is skipped
        const uint32_t next = c->xch_tag + static_cast<uint32_t>(n);
        c->xch_tag = next < c->xch_tag || next == 0 ? 1u : next;
        c->n_persistent += 1;
        c->n_persistent_cycles += n;
        *launched = true;
        return HBM_OK;
    }

    static const Launch *table()
    {
        static const Launch t{&sweep, &theta, &set_theta, &poplik, &prepare, &check_init, &quadrature, &marginal,
                              &cycles, &fused};
        return &t;
    }
};

struct ModelInfo {
    int d, p, m, md, precision;
    const Launch *ops;
    int ns;                    // sufficient statistics (0: none)
};

bool model_info(int model, ModelInfo *mi)
{
    switch (model) {
    case HBM_NORMAL_NORMAL_1D: *mi = {NN1D::D, NN1D::P, NN1D::M, NN1D::MD, HBM_FP64, Ops<NN1D>::table(), NN1D::NS}; return true;
    case HBM_GAMMA_LF_1D: *mi = {LF1D::D, LF1D::P, LF1D::M, LF1D::MD, HBM_FP32, Ops<LF1D>::table(), LF1D::NS}; return true;
    case HBM_GAMMA_LF_COLOR_3D: *mi = {LF3D::D, LF3D::P, LF3D::M, LF3D::MD, HBM_FP32, Ops<LF3D>::table(), LF3D::NS}; return true;
    case HBM_NORMAL_NORMAL_3D: *mi = {NN3D::D, NN3D::P, NN3D::M, NN3D::MD, HBM_FP64, Ops<NN3D>::table(), NN3D::NS}; return true;
    case HBM_BB1_LF: *mi = {BB1::D, BB1::P, BB1::M, BB1::MD, HBM_FP32, Ops<BB1>::table(), BB1::NS}; return true;
    default: return false;
    }
}

bool has_selection(int model)
{
    return model == HBM_GAMMA_LF_1D || model == HBM_GAMMA_LF_COLOR_3D || model == HBM_BB1_LF;
}

hbm_status usable(CtxImpl *c)
{
    if (!c) return HBM_EINVAL;
    if (c->poisoned) return fail(c, HBM_ESTATE, "context poisoned by an earlier HIP error: " + c->err);
    return HBM_OK;
}

hbm_status check_slot(CtxImpl *c, int32_t slot, bool need_loaded)
{
    if (slot < 0 || slot >= c->n_slots) return fail(c, HBM_EINVAL, "slot out of range");
    if (need_loaded && !c->slots[slot].loaded) return fail(c, HBM_EINVAL, "slot holds no dataset");
    return HBM_OK;
}

hbm_status read_slot(CtxImpl *c, int32_t slot, CycleState *h)
{
    HIPCHK(c, hipMemcpyAsync(h, c->cs + slot, sizeof(CycleState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HBM_OK;
}

hbm_status read_all(CtxImpl *c)
{
    HIPCHK(c, hipMemcpyAsync(c->h_cs.data(), c->cs, sizeof(CycleState) * c->n_slots, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HBM_OK;
}

template <typename V>
hbm_status put_field(CtxImpl *c, int32_t slot, size_t offset, V value)
{
    HIPCHK(c, hipMemcpyAsync(reinterpret_cast<char *>(c->cs + slot) + offset, &value, sizeof(V),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HBM_OK;
}

// Turns the sticky device flags of every slot (read into c->h_cs) into a
// status, and clears them.
hbm_status check_flags(CtxImpl *c)
{
    int32_t all = 0;
    std::string msg;
    for (int32_t j = 0; j < c->n_slots; ++j) {
        const int32_t f = c->h_cs[j].flags;
        if (f == 0) continue;
        all |= f;
        std::string m;
        if (f & kFlagNonFiniteState) m += "non-finite latent log density; ";
        if (f & kFlagBadZ) m += "selection normaliser not positive and finite; ";
        if (f & kFlagTraceFull) m += "theta trace full; ";
        if (f & kFlagNoSums) m += "theta step without a sweep; ";
        if (msg.size() < 512) msg += (c->n_slots > 1 ? "slot " + std::to_string(j) + ": " : std::string()) + m;
        hbm_status s = put_field<int32_t>(c, j, offsetof(CycleState, flags), 0);
        if (s != HBM_OK) return s;
    }
    if (all == 0) return HBM_OK;
    if (all & (kFlagNonFiniteState | kFlagBadZ)) return fail(c, HBM_EDOMAIN, msg);
    if (all & kFlagTraceFull) return fail(c, HBM_ENOSPACE, msg);
    return fail(c, HBM_ESTATE, msg);
}

void release(CtxImpl *c)
{
    if (!c) return;
    if (c->stream || c->cs) (void)hipStreamSynchronize(c->stream);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->tail_exec) (void)hipGraphExecDestroy(c->tail_exec);
    if (c->tail) (void)hipGraphDestroy(c->tail);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->copy_stream) {
        (void)hipStreamSynchronize(c->copy_stream);
        (void)hipStreamDestroy(c->copy_stream);
    }
    for (hipEvent_t e : {c->swept[0], c->swept[1], c->copied[0], c->copied[1]})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_pending) (void)hipEventDestroy(e);
    void *ptrs[] = {c->dd, c->partials, c->pout, c->theta_in, c->side, c->ref_t, c->ref_w, c->qx, c->qw, c->qeps,
                    c->cs, c->st, c->theta_trace, c->tile_ds, c->which, c->marg_rule, c->marg_buf, c->xch,
                    c->cs_alt, c->partials_alt, c->side_alt};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete static_cast<hbm_ctx *>(c);
}

// Checks one dataset's configuration (everything but its placement).
// stats_mode: whether the context takes its theta steps from sufficient
// statistics (c may be null: the check then runs before the context exists).
hbm_status validate_dataset(CtxImpl *c, const hbm_config *cfg, const double *theta0, const ModelInfo &mi,
                            bool stats_mode)
{
    if (!cfg || !theta0) return fail(c, HBM_EINVAL, "config and theta0 must be non-NULL");
    if (cfg->precision != mi.precision)
        return fail(c, HBM_EINVAL, "precision does not match the model (NN: FP64, LF: FP32)");
    if (cfg->n_objects < 1 || cfg->n_objects > (int64_t)INT32_MAX - kBlock)
        return fail(c, HBM_EINVAL, "n_objects must be in [1, 2^31 - 257]");
    if (!(cfg->target_accept > 0.0 && cfg->target_accept < 1.0) ||
        !(cfg->theta_target_accept > 0.0 && cfg->theta_target_accept < 1.0))
        return fail(c, HBM_EINVAL, "target acceptance rates must lie in (0, 1)");
    if (!(cfg->eta_exponent > 0.5 && cfg->eta_exponent <= 1.0))
        return fail(c, HBM_EINVAL, "eta_exponent must lie in (1/2, 1]");
    if (!(cfg->s0 > 0.0) || !std::isfinite(cfg->s0)) return fail(c, HBM_EINVAL, "s0 must be positive");
    if (cfg->thin_chi < 0 || cfg->max_cycles < 0) return fail(c, HBM_EINVAL, "thin_chi and max_cycles must be >= 0");
    if (cfg->snap_rows < 0) return fail(c, HBM_EINVAL, "snap_rows must be >= 0");
    if (stats_mode ? (cfg->theta_substeps < 1 || cfg->theta_substeps > 64) : cfg->theta_substeps != 0)
        return fail(c, HBM_EINVAL,
                    stats_mode ? "theta_substeps must be in [1, 64] in a context whose theta steps use sufficient "
                                 "statistics"
                               : "theta_substeps must be 0 in a context whose theta steps use the N-term sums");
    if (stats_mode && mi.ns == 0)
        return fail(c, HBM_EINVAL, "this model has no sufficient statistics (theta steps need the N-term sums)");
    if (cfg->model == HBM_BB1_LF) {
        const double *mc = cfg->model_consts;
        if (!(mc[0] > 0.0) || !(mc[1] > 0.0) || !(mc[2] >= 0.0) || !std::isfinite(mc[3]) || !std::isfinite(mc[4]) ||
            !(mc[3] < mc[4]))
            return fail(c, HBM_EINVAL, "BB1 model constants need F_th, sigma0 > 0, alpha >= 0 and finite ln l < ln u");
    } else if (has_selection(cfg->model)) {
        const double *mc = cfg->model_consts;
        if (!(mc[0] > 0.0) || !(mc[1] > 0.0) || !(mc[2] > 0.0) || !std::isfinite(mc[3]))
            return fail(c, HBM_EINVAL, "LF model constants need F_th, sigma_F, rmax > 0 and a finite ln L0");
        if (cfg->model == HBM_GAMMA_LF_COLOR_3D && (!(mc[4] > 0.0) || !(mc[5] > 0.0)))
            return fail(c, HBM_EINVAL, "LF colour model needs f_r > 0 and sigma_c > 0");
    }
    if (cfg->model == HBM_NORMAL_NORMAL_3D) {
        const double *mc = cfg->model_consts;
        const double a = mc[0], b2 = mc[1], c2 = mc[2], d2 = mc[3], e2 = mc[4], f2 = mc[5];
        const double det = a * (c2 * f2 - e2 * e2) - b2 * (b2 * f2 - e2 * d2) + d2 * (b2 * e2 - c2 * d2);
        if (!(a > 0.0) || !(a * c2 - b2 * b2 > 0.0) || !(det > 0.0) || !(mc[6] > 0) || !(mc[7] > 0) || !(mc[8] > 0))
            return fail(c, HBM_EINVAL, "C_pop must be positive definite and sigma_j > 0");
    }
    for (int r = 0; r < mi.p; ++r) {
        if (!std::isfinite(theta0[r])) return fail(c, HBM_EINVAL, "theta0 must be finite");
        if (!(cfg->theta_chol0[r * mi.p + r] > 0.0))
            return fail(c, HBM_EINVAL, "theta_chol0 must have a positive diagonal");
        for (int q = 0; q <= r; ++q)
            if (!std::isfinite(cfg->theta_chol0[r * mi.p + q])) return fail(c, HBM_EINVAL, "theta_chol0 not finite");
    }
    return HBM_OK;
}

hbm_status validate_pool(const hbm_pool_config *pool, const hbm_buffers *b, ModelInfo *mi)
{
    if (!pool || !b) return fail(nullptr, HBM_EINVAL, "pool config and buffers must be non-NULL");
    if (!model_info(pool->model, mi)) return fail(nullptr, HBM_EINVAL, "unknown model id");
    if (pool->precision != mi->precision)
        return fail(nullptr, HBM_EINVAL, "precision does not match the model (NN: FP64, LF: FP32)");
    if (pool->n_slots < 1 || pool->n_slots > 65535) return fail(nullptr, HBM_EINVAL, "n_slots must be in [1, 65535]");
    if (pool->capacity < 1 || pool->capacity > (int64_t)INT32_MAX - kBlock)
        return fail(nullptr, HBM_EINVAL, "capacity must be in [1, 2^31 - 257]");
    if (pool->max_cycles < 0 || pool->snap_rows < 0) return fail(nullptr, HBM_EINVAL, "max_cycles and snap_rows >= 0");
    if (has_selection(pool->model) && (pool->n_quad < 16 || pool->n_quad > 4096))
        return fail(nullptr, HBM_EINVAL, "n_quad must be in [16, 4096]");
    if (!b->data || !b->chi || !b->chol || !b->acc)
        return fail(nullptr, HBM_EINVAL, "data, chi, chol and acc buffers must be non-NULL");
    if (pool->tiles_per_group != 0 && pool->tiles_per_group != 1 && pool->tiles_per_group != 2 &&
        pool->tiles_per_group != 4)
        return fail(nullptr, HBM_EINVAL, "tiles_per_group must be 0 (default), 1, 2 or 4");
    if (pool->snap_rows > 0 && !b->chi_samples)
        return fail(nullptr, HBM_EINVAL, "snap_rows > 0 needs a chi_samples buffer");
    if (pool->stats_theta != 0 && pool->stats_theta != 1) return fail(nullptr, HBM_EINVAL, "stats_theta must be 0 or 1");
    if (pool->stats_theta && mi->ns == 0)
        return fail(nullptr, HBM_EINVAL, "this model has no sufficient statistics (theta steps need the N-term sums)");
    return HBM_OK;
}

template <typename F>
hbm_status with_ctx(hbm_ctx *ctx, F &&f)
{
    CtxImpl *c = reinterpret_cast<CtxImpl *>(ctx);
    hbm_status s = usable(c);
    if (s != HBM_OK) return s;
    return f(c);
}

hbm_status drain_timing(CtxImpl *c)
{
    for (size_t j = 0; j + 1 < c->ev_pending.size(); j += 2) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pending[j], c->ev_pending[j + 1]));
        c->timed_ms += ms;
        c->timed_launches += 1;
    }
    for (hipEvent_t e : c->ev_pending) c->ev_free.push_back(e);
    c->ev_pending.clear();
    return HBM_OK;
}

// One dataset covering every position of a one-slot context (the
// init_chains case): the launches take the table-free kernel variants.
bool single(const CtxImpl *c)
{
    return c->n_slots == 1 && c->slots[0].loaded && c->slots[0].obj_start == 0 && c->slots[0].n == c->cap;
}

// A one-slot context picks its kernel variants from its slot's placement;
// a captured graph is dropped when that changes.
hbm_status drop_graph(CtxImpl *c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->graph_exec) HIPCHK(c, hipGraphExecDestroy(c->graph_exec));
    if (c->graph) HIPCHK(c, hipGraphDestroy(c->graph));
    if (c->tail_exec) HIPCHK(c, hipGraphExecDestroy(c->tail_exec));
    if (c->tail) HIPCHK(c, hipGraphDestroy(c->tail));
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_len = 0;
    c->tail_exec = nullptr;
    c->tail = nullptr;
    c->tail_len = 0;
    return HBM_OK;
}

// Recomputes the launch extent of a multi-slot context from its loaded
// slots; a captured graph holds the extent, so it is dropped on a change.
hbm_status update_extent(CtxImpl *c)
{
    int32_t es = 1, et = 0;
    for (int32_t j = 0; j < c->n_slots; ++j) {
        const Slot &sl = c->slots[j];
        if (!sl.loaded) continue;
        es = j + 1;
        et = std::max(et, sl.tile_start + sl.n_tiles);
    }
    if (es == c->ext_slots && et == c->ext_tiles) return HBM_OK;
    c->ext_slots = es;
    c->ext_tiles = et;
    return drop_graph(c);
}

hbm_status create_ctx(const hbm_pool_config *pool, const hbm_buffers *buffers, void *hip_stream, CtxImpl **out)
{
    ModelInfo mi;
    hbm_status s = validate_pool(pool, buffers, &mi);
    if (s != HBM_OK) return s;
    CtxImpl *c = new (std::nothrow) hbm_ctx();
    if (!c) return fail(nullptr, HBM_ENOMEM, "host allocation failed");
    c->pool = *pool;
    c->buf = *buffers;
    c->snaps_dev = buffers->chi_samples;
    if (buffers->chi_samples) {
        // pinned host memory (hipHostMalloc): the sweep writes the snapshots
        // straight to the host through its device mapping
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, buffers->chi_samples) == hipSuccess && at.type == hipMemoryTypeHost) {
            void *dp = nullptr;
            if (hipHostGetDevicePointer(&dp, buffers->chi_samples, 0) != hipSuccess || !dp) {
                delete static_cast<hbm_ctx *>(c);
                return fail(nullptr, HBM_EINVAL, "chi_samples in host memory must be pinned and mapped (hipHostMalloc)");
            }
            c->snaps_dev = dp;
            c->snaps_host = true;
        }
        (void)hipGetLastError();     // a pointer HIP does not know leaves only a non-sticky error
    }
    c->d = mi.d;
    c->p = mi.p;
    c->m = mi.m;
    c->md = mi.md;
    c->nc = mi.d * (mi.d + 1) / 2;
    c->esize = mi.precision == HBM_FP64 ? 8 : 4;
    c->cap = pool->capacity;
    c->n_tiles = tiles_for(c->cap);
    c->n_slots = pool->n_slots;
    c->nq = has_selection(pool->model) ? pool->n_quad : 1;
    c->tpw = pool->tiles_per_group > 0 ? pool->tiles_per_group : 1;
    c->stats_mode = pool->stats_theta != 0;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ops = mi.ops;
    {
        // the device of the caller's buffers (else the current one)
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, buffers->data) == hipSuccess && at.type == hipMemoryTypeDevice)
            c->device = at.device;
        else if (hipGetDevice(&c->device) != hipSuccess)
            c->device = -1;
        (void)hipGetLastError();
    }
    c->slots.assign(c->n_slots, Slot{});
    c->h_tile_ds.assign(c->n_tiles, -1);
    c->h_which.assign(c->n_slots, 0);
    c->h_cs.resize(c->n_slots);

    auto bail = [&](hbm_status code) {
        g_init_error = c->err;
        release(c);
        return code;
    };
    auto alloc = [&](void **p, size_t bytes) -> hbm_status {
        hipError_t e = hipMalloc(p, bytes > 0 ? bytes : 8);
        if (e != hipSuccess) {
            c->err = std::string("hipMalloc: ") + hipGetErrorString(e);
            return HBM_ENOMEM;
        }
        return HBM_OK;
    };
    const size_t ns = static_cast<size_t>(c->n_slots), nq = static_cast<size_t>(c->nq);
    if ((s = alloc(&c->dd, c->esize * c->md * c->cap)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->partials), sizeof(double) * (2 + kMaxStats) * c->n_tiles)) !=
            HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->pout), sizeof(double) * 2 * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->theta_in), sizeof(double) * c->p * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->side), sizeof(Precomp) * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->ref_t), sizeof(double) * nq)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->ref_w), sizeof(double) * nq)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->qx), sizeof(double) * nq * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->qw), sizeof(double) * nq * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->qeps), sizeof(double) * nq * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->cs), sizeof(CycleState) * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->st), sizeof(Statics) * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->theta_trace),
                   sizeof(double) * c->p * static_cast<size_t>(pool->max_cycles) * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->tile_ds), sizeof(int32_t) * c->n_tiles)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->which), sizeof(int32_t) * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->xch), kXchBytes)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->cs_alt), sizeof(CycleState) * ns)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->partials_alt), sizeof(double) * (2 + kMaxStats) * c->n_tiles)) !=
            HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->side_alt), sizeof(Precomp) * ns)) != HBM_OK)
        return bail(s);
    // every slot starts empty: zero statics (n = 0) and inactive states
    std::vector<Statics> hs(ns);
    std::memset(hs.data(), 0, sizeof(Statics) * ns);
    std::memset(c->h_cs.data(), 0, sizeof(CycleState) * ns);
    hipError_t e;
    if ((e = hipMemcpyAsync(c->st, hs.data(), sizeof(Statics) * ns, hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c->cs, c->h_cs.data(), sizeof(CycleState) * ns, hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(c->tile_ds, c->h_tile_ds.data(), sizeof(int32_t) * c->n_tiles, hipMemcpyHostToDevice,
                            c->stream)) != hipSuccess ||
        (e = hipMemsetAsync(c->xch, 0, kXchBytes, c->stream)) != hipSuccess ||
        (e = hipMemsetAsync(c->cs_alt, 0, sizeof(CycleState) * ns, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
        hip_fail(c, e, "pool initialisation copies");
        return bail(HBM_EHIP);
    }
    if ((s = c->ops->quadrature(c)) != HBM_OK) return bail(s);
    setup_noalloc_scratch(c);
    *out = c;
    return HBM_OK;
}

// Loads datasets into free slots (the body of load_datasets).
hbm_status load(CtxImpl *c, int32_t count, const int32_t *slots, const int64_t *obj_start, const hbm_config *configs,
                const double *theta0, const int64_t *budgets)
{
    if (count < 1 || !slots || !obj_start || !configs || !theta0)
        return fail(c, HBM_EINVAL, "count >= 1 and non-NULL slots, obj_start, configs and theta0");
    ModelInfo mi;
    model_info(c->pool.model, &mi);
    std::vector<int32_t> owner(c->h_tile_ds);
    for (int32_t q = 0; q < count; ++q) {
        const hbm_config *cfg = configs + q;
        const int32_t j = slots[q];
        const std::string who = count > 1 ? "dataset " + std::to_string(q) + ": " : std::string();
        hbm_status s = check_slot(c, j, false);
        if (s != HBM_OK) return s;
        if (c->slots[j].loaded) return fail(c, HBM_EINVAL, who + "slot already holds a dataset");
        if (cfg->model != c->pool.model) return fail(c, HBM_EINVAL, who + "model differs from the pool's");
        if ((s = validate_dataset(c, cfg, theta0 + static_cast<size_t>(q) * c->p, mi, c->stats_mode)) != HBM_OK) {
            c->err = who + c->err;
            return s;
        }
        if (has_selection(cfg->model) && cfg->n_quad != c->pool.n_quad)
            return fail(c, HBM_EINVAL, who + "n_quad differs from the pool's");
        if (cfg->max_cycles > c->pool.max_cycles) return fail(c, HBM_EINVAL, who + "max_cycles exceeds the pool's");
        const int64_t b = budgets ? budgets[q] : 0;
        if (b < 0 || b > cfg->max_cycles) return fail(c, HBM_EINVAL, who + "budget must be in [0, max_cycles]");
        const int64_t o = obj_start[q];
        if (o < 0 || o % kBlock != 0 || o + cfg->n_objects > c->cap)
            return fail(c, HBM_EINVAL, who + "obj_start must be a multiple of 256 with obj_start + n <= capacity");
        const int32_t t0 = static_cast<int32_t>(o / kBlock), nt = tiles_for(cfg->n_objects);
        for (int32_t t = t0; t < t0 + nt; ++t) {
            if (owner[t] >= 0) return fail(c, HBM_EINVAL, who + "object range overlaps another dataset");
            owner[t] = j;
        }
        for (int32_t r = 0; r < q; ++r)
            if (slots[r] == j) return fail(c, HBM_EINVAL, who + "slot listed twice");
    }

    // statics and states of the new slots
    std::vector<Statics> hs(count);
    std::vector<CycleState> hc(count);
    std::memset(hs.data(), 0, sizeof(Statics) * count);
    std::memset(hc.data(), 0, sizeof(CycleState) * count);
    std::fill(c->h_which.begin(), c->h_which.end(), 0);
    for (int32_t q = 0; q < count; ++q) {
        const hbm_config *cfg = configs + q;
        const int64_t o = obj_start[q];
        Statics &s = hs[q];
        s.n = cfg->n_objects;
        s.obj_start = o;
        s.tile_start = static_cast<int32_t>(o / kBlock);
        s.n_tiles = tiles_for(cfg->n_objects);
        s.trace_cap = cfg->max_cycles;
        s.snap_cap = 0;
        if (cfg->thin_chi > 0 && c->buf.chi_samples) {
            const int64_t want = cfg->max_cycles / cfg->thin_chi;
            const int64_t rows = (cfg->snap_rows > 0 && cfg->snap_rows < c->pool.snap_rows) ? cfg->snap_rows
                                                                                            : c->pool.snap_rows;
            s.snap_cap = want < rows ? want : rows;
        }
        s.thin = cfg->thin_chi;
        s.nq = c->nq;
        s.adapt_theta = cfg->adapt_theta;
        s.p = c->p;
        s.substeps = cfg->theta_substeps;
        s.key0 = static_cast<uint32_t>(cfg->seed & 0xffffffffu);
        s.key1 = static_cast<uint32_t>(cfg->seed >> 32);
        s.gamma = cfg->eta_exponent;
        s.alpha_star = cfg->target_accept;
        s.alpha_star_theta = cfg->theta_target_accept;
        s.s0 = cfg->s0;
        std::memcpy(s.mc, cfg->model_consts, sizeof(s.mc));
        CycleState &h = hc[q];
        const double *t0 = theta0 + static_cast<size_t>(q) * c->p;
        for (int r = 0; r < c->p; ++r) {
            h.theta[r] = t0[r];
            for (int qq = 0; qq < c->p; ++qq)
                h.chol_theta[r * c->p + qq] = qq <= r ? cfg->theta_chol0[r * c->p + qq] : 0.0;
        }
        h.first_bad = INT32_MAX;
        h.budget = budgets ? budgets[q] : 0;
        h.active = 1;
        c->h_which[slots[q]] = 1;
    }
    for (int32_t q = 0; q < count; ++q) {
        HIPCHK(c, hipMemcpyAsync(c->st + slots[q], &hs[q], sizeof(Statics), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->cs + slots[q], &hc[q], sizeof(CycleState), hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->tile_ds, owner.data(), sizeof(int32_t) * c->n_tiles, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->which, c->h_which.data(), sizeof(int32_t) * c->n_slots, hipMemcpyHostToDevice,
                             c->stream));
    hbm_status s;
    if ((s = c->ops->prepare(c)) != HBM_OK) return s;
    if ((s = c->ops->set_theta(c)) != HBM_OK) return s;
    if ((s = c->ops->check_init(c)) != HBM_OK) return s;
    if ((s = read_all(c)) != HBM_OK) return s;

    // the first failing dataset, if any, fails the whole call
    std::string msg;
    for (int32_t q = 0; q < count && msg.empty(); ++q) {
        const CycleState &b = c->h_cs[slots[q]];
        const std::string who = count > 1 ? "dataset " + std::to_string(q) + ": " : std::string();
        if (!(b.lprior_cur > -HUGE_VAL)) msg = who + "theta0 is outside the prior support";
        else if (b.flags & kFlagBadZ) msg = who + "selection normaliser Z(theta0) is not positive and finite";
        else if (b.flags & kFlagNonFiniteState)
            msg = who + "non-finite initial log density at object " + std::to_string(b.first_bad);
    }
    if (!msg.empty()) {
        // leave the failed slots empty again
        std::vector<CycleState> zero(1);
        std::memset(zero.data(), 0, sizeof(CycleState));
        Statics zs;
        std::memset(&zs, 0, sizeof(zs));
        for (int32_t q = 0; q < count; ++q) {
            HIPCHK(c, hipMemcpyAsync(c->cs + slots[q], zero.data(), sizeof(CycleState), hipMemcpyHostToDevice,
                                     c->stream));
            HIPCHK(c, hipMemcpyAsync(c->st + slots[q], &zs, sizeof(Statics), hipMemcpyHostToDevice, c->stream));
        }
        HIPCHK(c, hipMemcpyAsync(c->tile_ds, c->h_tile_ds.data(), sizeof(int32_t) * c->n_tiles,
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return fail(c, HBM_EDOMAIN, msg);
    }
    c->h_tile_ds.swap(owner);
    if (c->n_slots == 1 && (s = drop_graph(c)) != HBM_OK) return s;
    for (int32_t q = 0; q < count; ++q) {
        Slot &sl = c->slots[slots[q]];
        sl = Slot{};
        sl.loaded = sl.active = true;
        sl.n = hs[q].n;
        sl.obj_start = hs[q].obj_start;
        sl.tile_start = hs[q].tile_start;
        sl.n_tiles = hs[q].n_tiles;
        sl.budget = hc[q].budget;
        sl.trace_cap = hs[q].trace_cap;
        sl.snap_cap = hs[q].snap_cap;
        sl.thin = hs[q].thin;
    }
    return update_extent(c);
}

// Theta steps a slot takes in n more full cycles.
int64_t cycles_taken(const Slot &s, int64_t n)
{
    if (!s.active) return 0;
    if (s.budget > 0 && s.n_theta + n > s.budget) return s.budget - s.n_theta;
    return n;
}

void after_theta_steps(Slot &s, int64_t n)
{
    s.k += n;
    s.n_theta += n;
    if (s.budget > 0 && s.n_theta >= s.budget) s.active = false;
}

// Gauss-Legendre nodes and weights on [-1, 1] (host, FP64): Newton's method
// on P_n from the asymptotic root guesses, P_n by the three-term recurrence.
void host_gauss_legendre(int n, double *t, double *w)
{
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < n; ++j) {
        double x = std::cos(pi * (j + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int l = 1; l < n; ++l) {
                const double p2 = ((2.0 * l + 1.0) * x * p1 - l * p0) / (l + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        t[j] = x;
        w[j] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

// Node tables of the marginal likelihood (the layouts marginal.h documents),
// built once per process on the host.
constexpr int kMargRuleNodes = kMargShapeNodes + kMargProductNodes;

hbm_status build_marg_rule(CtxImpl *c, MargNode *r)
{
    double t[64], w[64];
    using S = MargRuleShape;
    host_gauss_legendre(S::kCore, t, w);
    for (int q = 0; q < 2 * S::kCore; ++q) r[q] = MargNode{t[q % S::kCore], w[q % S::kCore], 0.0, 0.0};
    // graded panels from the top: 4 of width 0.25, 8 of 0.5, 8 of 1
    constexpr int kPerPanel = 8;
    host_gauss_legendre(kPerPanel, t, w);
    double top = 0.0;
    int q = 2 * S::kCore;
    for (int panel = 0; panel < S::kGraded / kPerPanel; ++panel) {
        const double width = panel < 4 ? 0.25 : panel < 12 ? 0.5 : 1.0;
        for (int j = 0; j < kPerPanel; ++j) {
            const double depth = top + 0.5 * width * (1.0 - t[j]);
            r[q++] = MargNode{depth, 0.5 * width * w[j], std::exp(-depth), 0.0};
        }
        top += width;
    }
    if (std::fabs(top - S::kDepth) > 1e-12) return fail(c, HBM_EINVAL, "marginal rule: graded panels miss the depth");
    host_gauss_legendre(S::kTail, t, w);
    for (int j = 0; j < S::kTail; ++j) r[q++] = MargNode{std::log(0.5 * (1.0 + t[j])), 0.5 * w[j], 0.0, 0.0};
    host_gauss_legendre(MargRuleProduct::kCore, t, w);
    for (int j = 0; j < kMargProductNodes; ++j)
        r[q++] = MargNode{t[j % MargRuleProduct::kCore], w[j % MargRuleProduct::kCore], 0.0, 0.0};
    return HBM_OK;
}

std::mutex g_rule_mu;
MargNode g_host_rule[kMargRuleNodes];
bool g_host_rule_ready = false;

// The host table, built on first use (no heap allocation).
hbm_status host_marg_rule(CtxImpl *c, const MargNode **out)
{
    std::lock_guard<std::mutex> lk(g_rule_mu);
    if (!g_host_rule_ready) {
        hbm_status st = build_marg_rule(c, g_host_rule);
        if (st != HBM_OK) return st;
        g_host_rule_ready = true;
    }
    *out = g_host_rule;
    return HBM_OK;
}

// The context's own device copy of the rule (marginal_loglik).
hbm_status ensure_marg_rule(CtxImpl *c)
{
    if (c->marg_rule) return HBM_OK;
    const MargNode *hr = nullptr;
    hbm_status st = host_marg_rule(c, &hr);
    if (st != HBM_OK) return st;
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(MargNode) * kMargRuleNodes) != hipSuccess)
        return fail(c, HBM_ENOMEM, "hipMalloc: marginal rule");
    c->marg_rule = static_cast<MargNode *>(p);
    HIPCHK(c, hipMemcpyAsync(c->marg_rule, hr, sizeof(MargNode) * kMargRuleNodes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HBM_OK;
}

// Per device: the address of `scratch` (from hipGetSymbolAddress, taken
// with that device current) once the node rule sits at its start, or the
// error that prevented it.
constexpr int kMaxDevices = 64;
constexpr size_t kNoAllocRuleBytes = (sizeof(MargNode) * kMargRuleNodes + 255) / 256 * 256;
static_assert(kNoAllocRuleBytes < kNoAllocScratchBytes, "the static scratch must hold the node rule");
struct NoAllocScratch {
    unsigned char *ptr = nullptr;
    bool tried = false;
    std::string err;
};
std::mutex g_noalloc_mu;
NoAllocScratch g_noalloc[kMaxDevices];

// Set-up of the static scratch on c's device, once per device (called when a
// context is created): resolve its address and copy the node rule there.  A
// failure is kept for marginal_loglik_noalloc to report; it does not stop the
// context.
void setup_noalloc_scratch(CtxImpl *c)
{
    const int dev = c->device;
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    NoAllocScratch &ns = g_noalloc[dev];
    if (ns.tried) return;
    ns.tried = true;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const MargNode *hr = nullptr;
    const std::string saved = c->err;
    const bool rule_ok = e == hipSuccess && host_marg_rule(c, &hr) == HBM_OK;
    if (rule_ok) e = hipMemcpy(p, hr, sizeof(MargNode) * kMargRuleNodes, hipMemcpyHostToDevice);
    if (e != hipSuccess)
        ns.err = std::string("static scratch set-up: ") + hipGetErrorString(e);
    else if (!rule_ok)
        ns.err = "static scratch set-up: " + c->err;
    else
        ns.ptr = static_cast<unsigned char *>(p);
    c->err = saved;
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    (void)hipGetLastError();
}

// The static scratch of c's device (nullptr and a message if unavailable).
unsigned char *noalloc_scratch(CtxImpl *c, std::string *why)
{
    if (c->device < 0 || c->device >= kMaxDevices) {
        *why = "static scratch: device ordinal out of range";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    const NoAllocScratch &ns = g_noalloc[c->device];
    if (!ns.ptr) *why = ns.tried ? ns.err : std::string("static scratch: not set up on this device");
    return ns.ptr;
}

// Values of theta at which the population density exists: the gamma law
// needs beta + 1 > 0 and BB1 beta + 2 > 0 (its lower tail integrable).
bool marg_density_ok(int model, const double *th)
{
    switch (model) {
    case HBM_GAMMA_LF_1D: return th[0] > -1.0;
    case HBM_BB1_LF: return th[0] > -2.0;
    default: return true;
    }
}

// Argument checks shared by the marginal-likelihood entry points.
hbm_status check_marginal_args(CtxImpl *c, int32_t slot, int32_t n_theta, const double *theta, const double *out)
{
    hbm_status st = check_slot(c, slot, true);
    if (st != HBM_OK) return st;
    if (c->d != 1) return fail(c, HBM_EINVAL, "the marginal likelihood needs a model with a 1-D latent");
    if (n_theta < 1 || n_theta > 65535) return fail(c, HBM_EINVAL, "n_theta must be in [1, 65535]");
    if (!theta || !out) return fail(c, HBM_EINVAL, "theta and out must be non-NULL");
    for (int64_t j = 0; j < static_cast<int64_t>(n_theta) * c->p; ++j)
        if (!std::isfinite(theta[j])) return fail(c, HBM_EINVAL, "theta must be finite");
    for (int32_t j = 0; j < n_theta; ++j)
        if (!marg_density_ok(c->pool.model, theta + static_cast<size_t>(j) * c->p))
            return fail(c, HBM_EDOMAIN, "theta outside the domain of the population density");
    return HBM_OK;
}

// Device scratch of one marginal-likelihood call, in doubles: theta rows,
// results, per-workgroup partial sums, per-row scalars.
size_t marginal_scratch_bytes(const CtxImpl *c, int32_t slot, int32_t n_theta)
{
    const size_t nb = static_cast<size_t>(marg_blocks(c->slots[slot].n)), nt = static_cast<size_t>(n_theta);
    return sizeof(double) * (nt * c->p + nt + nt * nb + nt * kMargThWords);
}

// One marginal-likelihood evaluation with its scratch at `buf` (laid out as
// marginal_scratch_bytes counts it) and the node rule at `rule`.
hbm_status run_marginal(CtxImpl *c, int32_t slot, int32_t n_theta, const double *theta, double *out, double *terms,
                        double *buf, const MargNode *rule)
{
    const size_t nb = static_cast<size_t>(marg_blocks(c->slots[slot].n));
    const size_t n_th = static_cast<size_t>(n_theta) * c->p, n_part = static_cast<size_t>(n_theta) * nb;
    double *d_theta = buf, *d_out = d_theta + n_th, *d_part = d_out + n_theta, *d_pre = d_part + n_part;
    HIPCHK(c, hipMemcpyAsync(d_theta, theta, sizeof(double) * n_th, hipMemcpyHostToDevice, c->stream));
    hbm_status st = c->ops->marginal(c, slot, n_theta, d_theta, d_out, d_part, d_pre, terms, rule);
    if (st != HBM_OK) return st;
    HIPCHK(c, hipMemcpyAsync(out, d_out, sizeof(double) * n_theta, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HBM_OK;
}

// Checks that n_cycles full cycles can run now.
hbm_status check_cycles(CtxImpl *c, int64_t n_cycles)
{
    if (n_cycles < 0) return fail(c, HBM_EINVAL, "n_cycles must be >= 0");
    for (const Slot &sl : c->slots) {
        if (!sl.active) continue;
        if (sl.sums_ready) return fail(c, HBM_ESTATE, "a ram_sweep is waiting for its theta_step");
        if (sl.n_theta + cycles_taken(sl, n_cycles) > sl.trace_cap)
            return fail(c, HBM_ENOSPACE, "theta trace would overflow (max_cycles)");
    }
    return HBM_OK;
}

constexpr int64_t kGraphCycles = 32;

// Captures len consecutive full cycles into an executable graph (nothing runs).
hbm_status capture_cycles(CtxImpl *c, int64_t len, hipGraph_t *g_out, hipGraphExec_t *ge_out)
{
    if (!c->capture_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    hipStream_t saved = c->stream;
    c->stream = c->capture_stream;
    HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    hbm_status st = HBM_OK;
    if (c->cycle_mode == HBM_CYCLES_FUSED && len >= 2)
        st = c->ops->fused(c, len);
    else
        for (int64_t j = 0; j < len && st == HBM_OK; ++j) st = c->ops->sweep(c, true, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
    c->stream = saved;
    if (st != HBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(c, e, "hipGraphInstantiate");
    }
    // upload now, so that the first replay does not pay for it
    e = hipGraphUpload(ge, c->stream);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(ge);
        (void)hipGraphDestroy(g);
        return hip_fail(c, e, "hipGraphUpload");
    }
    *g_out = g;
    *ge_out = ge;
    c->n_captures += 1;
    return HBM_OK;
}

// Makes sure the graphs that n_cycles graph-issued cycles use exist: the
// kGraphCycles-cycle graph when n_cycles reaches it, and the graph of the
// remainder n_cycles mod kGraphCycles (recaptured when the remainder changes).
hbm_status ensure_graphs(CtxImpl *c, int64_t n_cycles)
{
    if (n_cycles >= kGraphCycles && !c->graph_exec) {
        hbm_status st = capture_cycles(c, kGraphCycles, &c->graph, &c->graph_exec);
        if (st != HBM_OK) return st;
        c->graph_len = kGraphCycles;
    }
    const int64_t rem = n_cycles % kGraphCycles;
    if (rem > 0 && c->tail_len != rem) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->tail_exec) HIPCHK(c, hipGraphExecDestroy(c->tail_exec));
        if (c->tail) HIPCHK(c, hipGraphDestroy(c->tail));
        c->tail_exec = nullptr;
        c->tail = nullptr;
        c->tail_len = 0;
        hbm_status st = capture_cycles(c, rem, &c->tail, &c->tail_exec);
        if (st != HBM_OK) return st;
        c->tail_len = rem;
    }
    return HBM_OK;
}

// Issues n full cycles on the context's stream: with use_graph (and no
// per-launch timing) as replays of the kGraphCycles-cycle graph and one
// replay of the remainder's graph, else as plain launches.  Host mirrors
// unchanged.
hbm_status issue_cycles(CtxImpl *c, int64_t n_cycles, bool use_graph)
{
    if (n_cycles <= 0) return HBM_OK;
    if (use_graph) {
        bool launched = false;
        hbm_status st = c->ops->cycles(c, n_cycles, &launched);
        if (st != HBM_OK || launched) return st;
    }
    if (use_graph && c->timing && c->cycle_mode == HBM_CYCLES_FUSED && n_cycles >= 2) {
        // fused cycles as plain launches, each fused kernel timed
        hbm_status st = c->ops->fused(c, n_cycles);
        if (st != HBM_OK) return st;
        c->n_plain_cycles += n_cycles;
        return HBM_OK;
    }
    if (use_graph && !c->timing) {
        hbm_status st = ensure_graphs(c, n_cycles);
        if (st != HBM_OK) return st;
        for (int64_t left = n_cycles; left > 0;) {
            const bool whole = left >= kGraphCycles;
            HIPCHK(c, hipGraphLaunch(whole ? c->graph_exec : c->tail_exec, c->stream));
            const int64_t len = whole ? kGraphCycles : left;
            c->n_replays += 1;
            c->n_replayed_cycles += len;
            left -= len;
        }
        return HBM_OK;
    }
    for (int64_t j = 0; j < n_cycles; ++j) {
        hbm_status st = c->ops->sweep(c, true, nullptr);
        if (st != HBM_OK) return st;
    }
    c->n_plain_cycles += n_cycles;
    return HBM_OK;
}

// Sets every streaming slot's ring flag in its device statics.
hbm_status set_snap_ring(CtxImpl *c, int32_t on)
{
    for (int32_t j = 0; j < c->n_slots; ++j) {
        const Slot &sl = c->slots[j];
        if (!sl.loaded || sl.thin <= 0) continue;
        HIPCHK(c, hipMemcpyAsync(reinterpret_cast<char *>(c->st + j) + offsetof(Statics, snap_ring), &on,
                                 sizeof(on), hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HBM_OK;
}

// Rows of one slot copied in one chunk: snapshots [first, first + count).
struct ChunkPiece {
    int32_t slot;
    int64_t first, count;
    size_t offset, bytes;      // into the chunk's staging
};

// The body of run_cycles_streamed (arguments checked).  Device ring: each
// chunk's rows are copied on the copy stream into pinned staging.  Host ring
// (chi_samples in pinned host memory): the sweeps already wrote the rows to
// the host; a slot whose rows are back to back is handed to the sink in
// place, any other is packed on the host first.
hbm_status stream_cycles(CtxImpl *c, int64_t n_cycles, int32_t chunk_cycles, size_t chunk_bytes,
                         hbm_snapshot_sink sink, void *user)
{
    const bool host = c->snaps_host;
    if (!host && !c->copy_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
        if (!c->swept[b]) HIPCHK(c, hipEventCreateWithFlags(&c->swept[b], hipEventDisableTiming));
        if (!host && !c->copied[b]) HIPCHK(c, hipEventCreateWithFlags(&c->copied[b], hipEventDisableTiming));
    }
    void *staging[2] = {nullptr, nullptr};
    std::vector<char> packed;               // host ring: rows of a slot that are not back to back
    if (!host)
        for (int b = 0; b < 2; ++b)
            if (chunk_bytes > 0 && hipHostMalloc(&staging[b], chunk_bytes, hipHostMallocDefault) != hipSuccess) {
                if (staging[0]) (void)hipHostFree(staging[0]);
                return fail(c, HBM_ENOMEM, "hipHostMalloc: snapshot staging");
            }
    std::vector<ChunkPiece> pieces[2];
    hbm_status st = set_snap_ring(c, 1);
    bool stop = false;
    const int64_t n_chunks = (n_cycles + chunk_cycles - 1) / chunk_cycles;
    // hands chunk q's rows to the sink once they have landed
    auto deliver = [&](int64_t q) -> hbm_status {
        const int b = static_cast<int>(q & 1);
        HIPCHK(c, hipEventSynchronize(host ? c->swept[b] : c->copied[b]));
        for (const ChunkPiece &pc : pieces[b]) {
            if (stop) break;
            const void *rows = nullptr;
            if (!host) {
                rows = static_cast<char *>(staging[b]) + pc.offset;
            } else {
                const Slot &sl = c->slots[pc.slot];
                const int64_t ring = pc.first % sl.snap_cap;
                const size_t row_bytes = static_cast<size_t>(c->d) * sl.n * c->esize;
                const char *base = static_cast<const char *>(c->buf.chi_samples);
                if (sl.n == c->cap && ring + pc.count <= sl.snap_cap) {
                    rows = base + static_cast<size_t>(ring) * row_bytes;
                } else {
                    packed.resize(pc.bytes);
                    for (int64_t r = 0; r < pc.count; ++r)
                        for (int j = 0; j < c->d; ++j) {
                            const int64_t rr = (pc.first + r) % sl.snap_cap;
                            std::memcpy(packed.data() + (static_cast<size_t>(r) * c->d + j) * sl.n * c->esize,
                                        base + ((static_cast<size_t>(rr) * c->d + j) * c->cap + sl.obj_start) *
                                                   c->esize,
                                        sl.n * c->esize);
                        }
                    rows = packed.data();
                }
            }
            if (sink(user, pc.slot, pc.first, pc.count, rows, static_cast<int64_t>(pc.bytes)) != 0) stop = true;
        }
        pieces[b].clear();
        return HBM_OK;
    };
    for (int64_t q = 0; q < n_chunks && st == HBM_OK && !stop; ++q) {
        const int b = static_cast<int>(q & 1);
        const int64_t len = std::min<int64_t>(chunk_cycles, n_cycles - q * chunk_cycles);
        // device ring: the rows chunk q - 2 left must be copied before this chunk
        // overwrites them (host ring: they were delivered before this chunk was issued)
        if (!host && q >= 2) HIPCHK(c, hipStreamWaitEvent(c->stream, c->copied[b], 0));
        std::vector<int64_t> k0(c->n_slots);
        for (int32_t j = 0; j < c->n_slots; ++j) k0[j] = c->slots[j].k;
        if ((st = issue_cycles(c, len, true)) != HBM_OK) break;
        for (Slot &sl : c->slots) after_theta_steps(sl, cycles_taken(sl, len));
        HIPCHK(c, hipEventRecord(c->swept[b], c->stream));
        if (q >= 1 && (st = deliver(q - 1)) != HBM_OK) break;
        // this chunk's snapshots, slot by slot
        if (!host) HIPCHK(c, hipStreamWaitEvent(c->copy_stream, c->swept[b], 0));
        size_t off = 0;
        for (int32_t j = 0; j < c->n_slots; ++j) {
            const Slot &sl = c->slots[j];
            if (!sl.loaded || sl.thin <= 0) continue;
            const int64_t first = k0[j] / sl.thin, end = sl.k / sl.thin;
            if (end <= first) continue;
            const size_t row_bytes = static_cast<size_t>(c->d) * sl.n * c->esize;
            pieces[b].push_back(ChunkPiece{j, first, end - first, off, static_cast<size_t>(end - first) * row_bytes});
            if (host) continue;
            for (int64_t r = first; r < end;) {
                // a run of consecutive ring rows: one copy of its d x N blocks
                const int64_t ring = r % sl.snap_cap;
                const int64_t run = std::min<int64_t>(end - r, sl.snap_cap - ring);
                const char *src = static_cast<const char *>(c->buf.chi_samples) +
                                  (static_cast<size_t>(ring) * c->d * c->cap + sl.obj_start) * c->esize;
                if (sl.n == c->cap)         // rows back to back: one linear copy
                    HIPCHK(c, hipMemcpyAsync(static_cast<char *>(staging[b]) + off, src,
                                             static_cast<size_t>(run) * row_bytes, hipMemcpyDeviceToHost,
                                             c->copy_stream));
                else
                    HIPCHK(c, hipMemcpy2DAsync(static_cast<char *>(staging[b]) + off, sl.n * c->esize, src,
                                               c->cap * c->esize, sl.n * c->esize, run * c->d,
                                               hipMemcpyDeviceToHost, c->copy_stream));
                off += static_cast<size_t>(run) * row_bytes;
                r += run;
            }
        }
        if (!host) HIPCHK(c, hipEventRecord(c->copied[b], c->copy_stream));
        if (q == n_chunks - 1 || stop) st = deliver(q);
    }
    hbm_status st2 = HBM_OK;
    {
        hipError_t e1 = host ? hipSuccess : hipStreamSynchronize(c->copy_stream);
        hipError_t e2 = hipStreamSynchronize(c->stream);
        if (e1 != hipSuccess) st2 = hip_fail(c, e1, "copy stream");
        else if (e2 != hipSuccess) st2 = hip_fail(c, e2, "stream");
    }
    if (st2 == HBM_OK) st2 = set_snap_ring(c, 0);
    for (void *p : staging)
        if (p) (void)hipHostFree(p);
    if (st != HBM_OK) return st;
    if (st2 != HBM_OK) return st2;
    if (stop) return fail(c, HBM_ESTATE, "the snapshot sink stopped the run");
    return HBM_OK;
}

}  // namespace

extern "C" {

hbm_status create_pool(const hbm_pool_config *pool, const hbm_buffers *buffers, void *hip_stream, hbm_ctx **out)
{
    if (!out) return fail(nullptr, HBM_EINVAL, "out must be non-NULL");
    *out = nullptr;
    CtxImpl *c = nullptr;
    hbm_status s = create_ctx(pool, buffers, hip_stream, &c);
    if (s == HBM_OK) *out = static_cast<hbm_ctx *>(c);
    return s;
}

hbm_status load_datasets(hbm_ctx *ctx, int32_t count, const int32_t *slots, const int64_t *obj_start,
                         const hbm_config *configs, const double *theta0, const int64_t *budgets)
{
    return with_ctx(ctx, [&](CtxImpl *c) { return load(c, count, slots, obj_start, configs, theta0, budgets); });
}

hbm_status unload_dataset(hbm_ctx *ctx, int32_t slot)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        hbm_status s = check_slot(c, slot, true);
        if (s != HBM_OK) return s;
        Slot &sl = c->slots[slot];
        for (int32_t t = sl.tile_start; t < sl.tile_start + sl.n_tiles; ++t) c->h_tile_ds[t] = -1;
        HIPCHK(c, hipMemcpyAsync(c->tile_ds + sl.tile_start, c->h_tile_ds.data() + sl.tile_start,
                                 sizeof(int32_t) * sl.n_tiles, hipMemcpyHostToDevice, c->stream));
        const int64_t zero_n = 0;
        HIPCHK(c, hipMemcpyAsync(reinterpret_cast<char *>(c->st + slot) + offsetof(Statics, n), &zero_n,
                                 sizeof(zero_n), hipMemcpyHostToDevice, c->stream));
        if ((s = put_field<int32_t>(c, slot, offsetof(CycleState, active), 0)) != HBM_OK) return s;
        sl = Slot{};
        if (c->n_slots == 1 && (s = drop_graph(c)) != HBM_OK) return s;
        return update_extent(c);
    });
}

hbm_status slot_info(hbm_ctx *ctx, int32_t slot, int64_t out[6])
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!out) return fail(c, HBM_EINVAL, "out must be non-NULL");
        hbm_status s = check_slot(c, slot, false);
        if (s != HBM_OK) return s;
        const Slot &sl = c->slots[slot];
        out[0] = sl.loaded;
        out[1] = sl.active;
        out[2] = sl.k;
        out[3] = sl.n_theta;
        out[4] = sl.obj_start;
        out[5] = sl.n;
        return HBM_OK;
    });
}

hbm_status init_chains(const hbm_config *config, const hbm_buffers *buffers, const double *chi0_host,
                       const double *theta0, void *hip_stream, hbm_ctx **out)
{
    if (!out) return fail(nullptr, HBM_EINVAL, "out must be non-NULL");
    *out = nullptr;
    if (!config || !buffers || !theta0) return fail(nullptr, HBM_EINVAL, "config, buffers and theta0 must be non-NULL");
    hbm_pool_config pool;
    std::memset(&pool, 0, sizeof(pool));
    pool.model = config->model;
    pool.precision = config->precision;
    pool.n_slots = 1;
    pool.n_quad = config->n_quad;
    pool.capacity = config->n_objects;
    pool.max_cycles = config->max_cycles;
    pool.snap_rows = (config->thin_chi > 0 && buffers->chi_samples)
                         ? (config->snap_rows > 0 ? config->snap_rows : config->max_cycles / config->thin_chi)
                         : 0;
    pool.tiles_per_group = config->tiles_per_group;
    pool.stats_theta = config->theta_substeps > 0 ? 1 : 0;
    // dataset checks first, so a bad dataset reports its own reason
    ModelInfo mi;
    if (!model_info(config->model, &mi)) return fail(nullptr, HBM_EINVAL, "unknown model id");
    hbm_status s = validate_dataset(nullptr, config, theta0, mi, config->theta_substeps > 0);
    if (s != HBM_OK) return s;
    if (has_selection(config->model) && (config->n_quad < 16 || config->n_quad > 4096))
        return fail(nullptr, HBM_EINVAL, "n_quad must be in [16, 4096]");
    CtxImpl *c = nullptr;
    if ((s = create_ctx(&pool, buffers, hip_stream, &c)) != HBM_OK) return s;
    if (chi0_host) {
        std::vector<char> tmp(c->esize * c->d * c->cap);
        for (int64_t j = 0; j < c->d * c->cap; ++j) {
            if (c->esize == 4) reinterpret_cast<float *>(tmp.data())[j] = static_cast<float>(chi0_host[j]);
            else reinterpret_cast<double *>(tmp.data())[j] = chi0_host[j];
        }
        hipError_t e;
        if ((e = hipMemcpyAsync(c->buf.chi, tmp.data(), tmp.size(), hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
            hip_fail(c, e, "chi0 copy");
            g_init_error = c->err;
            release(c);
            return HBM_EHIP;
        }
    }
    const int32_t slot = 0;
    const int64_t o = 0;
    if ((s = load(c, 1, &slot, &o, config, theta0, nullptr)) != HBM_OK) {
        g_init_error = c->err;
        release(c);
        return s;
    }
    *out = static_cast<hbm_ctx *>(c);
    return HBM_OK;
}

hbm_status init_batch(int32_t n_datasets, const hbm_config *configs, const hbm_buffers *buffers, const double *theta0,
                      void *hip_stream, hbm_ctx **out)
{
    if (!out) return fail(nullptr, HBM_EINVAL, "out must be non-NULL");
    *out = nullptr;
    if (n_datasets < 1 || n_datasets > 65535 || !configs || !buffers || !theta0)
        return fail(nullptr, HBM_EINVAL, "1 <= n_datasets <= 65535 and non-NULL configs, buffers, theta0");
    std::vector<int32_t> slots(n_datasets);
    std::vector<int64_t> starts(n_datasets);
    hbm_pool_config pool;
    std::memset(&pool, 0, sizeof(pool));
    pool.model = configs[0].model;
    pool.precision = configs[0].precision;
    pool.n_slots = n_datasets;
    pool.n_quad = configs[0].n_quad;
    pool.tiles_per_group = configs[0].tiles_per_group;
    pool.stats_theta = configs[0].theta_substeps > 0 ? 1 : 0;
    int64_t o = 0;
    for (int32_t q = 0; q < n_datasets; ++q) {
        const hbm_config &cf = configs[q];
        if (cf.n_objects < 1 || cf.n_objects > (int64_t)INT32_MAX - kBlock)
            return fail(nullptr, HBM_EINVAL, "n_objects must be in [1, 2^31 - 257]");
        slots[q] = q;
        starts[q] = o;
        pool.capacity = o + cf.n_objects;
        o += static_cast<int64_t>(tiles_for(cf.n_objects)) * kBlock;
        if (cf.max_cycles > pool.max_cycles) pool.max_cycles = cf.max_cycles;
        const int64_t rows = cf.snap_rows > 0 ? cf.snap_rows : (cf.thin_chi > 0 ? cf.max_cycles / cf.thin_chi : 0);
        if (cf.thin_chi > 0 && buffers->chi_samples && rows > pool.snap_rows) pool.snap_rows = rows;
    }
    CtxImpl *c = nullptr;
    hbm_status s = create_ctx(&pool, buffers, hip_stream, &c);
    if (s != HBM_OK) return s;
    if ((s = load(c, n_datasets, slots.data(), starts.data(), configs, theta0, nullptr)) != HBM_OK) {
        g_init_error = c->err;
        release(c);
        return s;
    }
    *out = static_cast<hbm_ctx *>(c);
    return HBM_OK;
}

hbm_status ram_sweep(hbm_ctx *ctx, int32_t n_sweeps, double *out_accept_rate)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (n_sweeps < 0) return fail(c, HBM_EINVAL, "n_sweeps must be >= 0");
        for (int32_t s = 0; s < n_sweeps; ++s) {
            hbm_status st = c->ops->sweep(c, false, nullptr);
            if (st != HBM_OK) return st;
            for (Slot &sl : c->slots)
                if (sl.active) {
                    sl.k += 1;
                    sl.sums_ready = true;
                }
        }
        if (out_accept_rate) {
            hbm_status st = read_all(c);
            if (st != HBM_OK) return st;
            for (int32_t j = 0; j < c->n_slots; ++j)
                out_accept_rate[j] = c->slots[j].active ? c->h_cs[j].n_acc_last / static_cast<double>(c->slots[j].n)
                                                        : static_cast<double>(NAN);
            return check_flags(c);
        }
        return HBM_OK;
    });
}

hbm_status pop_loglik(hbm_ctx *ctx, const double *theta, double *out)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!theta || !out) return fail(c, HBM_EINVAL, "theta and out must be non-NULL");
        std::vector<double> th(static_cast<size_t>(c->n_slots) * c->p, 0.0);
        for (int32_t j = 0; j < c->n_slots; ++j) {
            if (!c->slots[j].loaded) continue;
            for (int r = 0; r < c->p; ++r) {
                const double v = theta[static_cast<size_t>(j) * c->p + r];
                if (!std::isfinite(v)) return fail(c, HBM_EINVAL, "theta must be finite");
                th[static_cast<size_t>(j) * c->p + r] = v;
            }
        }
        HIPCHK(c, hipMemcpyAsync(c->theta_in, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice, c->stream));
        hbm_status st = c->ops->poplik(c);
        if (st != HBM_OK) return st;
        std::vector<double> po(2 * static_cast<size_t>(c->n_slots));
        HIPCHK(c, hipMemcpyAsync(po.data(), c->pout, sizeof(double) * po.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int32_t j = 0; j < c->n_slots; ++j) out[j] = c->slots[j].loaded ? po[2 * j + 1] : static_cast<double>(NAN);
        return HBM_OK;
    });
}

hbm_status marginal_loglik(hbm_ctx *ctx, int32_t slot, int32_t n_theta, const double *theta, double *out,
                           double *terms)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        hbm_status st = check_marginal_args(c, slot, n_theta, theta, out);
        if (st != HBM_OK) return st;
        if ((st = ensure_marg_rule(c)) != HBM_OK) return st;
        const size_t need = marginal_scratch_bytes(c, slot, n_theta);
        if (need > c->marg_bytes) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (c->marg_buf) HIPCHK(c, hipFree(c->marg_buf));
            c->marg_buf = nullptr;
            c->marg_bytes = 0;
            void *p = nullptr;
            if (hipMalloc(&p, need) != hipSuccess) return fail(c, HBM_ENOMEM, "hipMalloc: marginal scratch");
            c->marg_buf = static_cast<double *>(p);
            c->marg_bytes = need;
        }
        return run_marginal(c, slot, n_theta, theta, out, terms, c->marg_buf, c->marg_rule);
    });
}

hbm_status marginal_loglik_noalloc(hbm_ctx *ctx, int32_t slot, int32_t n_theta, const double *theta, double *out,
                                   double *terms)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        hbm_status st = check_marginal_args(c, slot, n_theta, theta, out);
        if (st != HBM_OK) return st;
        const size_t need = marginal_scratch_bytes(c, slot, n_theta);
        if (need > kNoAllocScratchBytes - kNoAllocRuleBytes)
            return fail(c, HBM_EINVAL,
                        "marginal_loglik_noalloc: " + std::to_string(n_theta) + " theta rows over " +
                            std::to_string(c->slots[slot].n) + " objects need " + std::to_string(need) +
                            " bytes of scratch; the static scratch holds " +
                            std::to_string(kNoAllocScratchBytes - kNoAllocRuleBytes));
        std::string why;
        unsigned char *base = noalloc_scratch(c, &why);
        if (!base) return fail(c, HBM_ENOMEM, why);
        // no events either: kernel timing would create them
        const bool timing = c->timing;
        c->timing = false;
        st = run_marginal(c, slot, n_theta, theta, out, terms, reinterpret_cast<double *>(base + kNoAllocRuleBytes),
                          reinterpret_cast<const MargNode *>(base));
        c->timing = timing;
        return st;
    });
}

hbm_status theta_step(hbm_ctx *ctx, int32_t *out_accepted)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        for (const Slot &sl : c->slots) {
            if (!sl.active) continue;
            if (!sl.sums_ready) return fail(c, HBM_ESTATE, "theta_step needs a ram_sweep since the last theta step");
            if (sl.n_theta >= sl.trace_cap) return fail(c, HBM_ENOSPACE, "theta trace full (max_cycles)");
        }
        hbm_status st = c->ops->theta(c);
        if (st != HBM_OK) return st;
        std::vector<char> stepped(c->n_slots, 0);
        for (int32_t j = 0; j < c->n_slots; ++j) {
            Slot &sl = c->slots[j];
            if (!sl.active) continue;
            stepped[j] = 1;
            sl.sums_ready = false;
            sl.n_theta += 1;
            if (sl.budget > 0 && sl.n_theta >= sl.budget) sl.active = false;
        }
        if ((st = read_all(c)) != HBM_OK) return st;
        if (out_accepted)
            for (int32_t j = 0; j < c->n_slots; ++j) out_accepted[j] = stepped[j] ? c->h_cs[j].accepted_last : -1;
        return check_flags(c);
    });
}

hbm_status run_cycles(hbm_ctx *ctx, int64_t n_cycles, int32_t use_graph)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        hbm_status st = check_cycles(c, n_cycles);
        if (st != HBM_OK) return st;
        if ((st = issue_cycles(c, n_cycles, use_graph != 0)) != HBM_OK) return st;
        for (Slot &sl : c->slots) after_theta_steps(sl, cycles_taken(sl, n_cycles));
        return HBM_OK;
    });
}

hbm_status prepare_cycles(hbm_ctx *ctx, int64_t n_cycles)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (n_cycles < 0) return fail(c, HBM_EINVAL, "n_cycles must be >= 0");
        return ensure_graphs(c, n_cycles);
    });
}

hbm_status launch_counts(hbm_ctx *ctx, int64_t out[6])
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!out) return fail(c, HBM_EINVAL, "out must be non-NULL");
        out[0] = c->n_replays;
        out[1] = c->n_replayed_cycles;
        out[2] = c->n_plain_cycles;
        out[3] = c->n_captures;
        out[4] = c->n_persistent;
        out[5] = c->n_persistent_cycles;
        return HBM_OK;
    });
}

hbm_status set_cycle_mode(hbm_ctx *ctx, int32_t mode)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (mode != HBM_CYCLES_AUTO && mode != HBM_CYCLES_GRAPH && mode != HBM_CYCLES_FUSED)
            return fail(c, HBM_EINVAL, "mode must be HBM_CYCLES_AUTO, HBM_CYCLES_GRAPH or HBM_CYCLES_FUSED");
        // the captured graphs hold fused cycles or not
        if ((mode == HBM_CYCLES_FUSED) != (c->cycle_mode == HBM_CYCLES_FUSED)) {
            hbm_status st = drop_graph(c);
            if (st != HBM_OK) return st;
        }
        c->cycle_mode = mode;
        return HBM_OK;
    });
}

hbm_status run_cycles_streamed(hbm_ctx *ctx, int64_t n_cycles, int32_t chunk_cycles, hbm_snapshot_sink sink,
                               void *user)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        hbm_status st = check_cycles(c, n_cycles);
        if (st != HBM_OK) return st;
        if (!sink) return fail(c, HBM_EINVAL, "sink must be non-NULL");
        if (chunk_cycles < 1) return fail(c, HBM_EINVAL, "chunk_cycles must be >= 1");
        // every streaming slot needs two chunks of ring rows
        size_t chunk_bytes = 0;
        for (const Slot &sl : c->slots) {
            if (!sl.active || sl.thin <= 0) continue;
            const int64_t per_chunk = (chunk_cycles + sl.thin - 1) / sl.thin;
            if (sl.snap_cap < 2 * per_chunk)
                return fail(c, HBM_EINVAL, "a streaming slot needs snap_rows >= 2 * ceil(chunk_cycles / thin_chi)");
            chunk_bytes += static_cast<size_t>(per_chunk) * c->d * sl.n * c->esize;
        }
        return stream_cycles(c, n_cycles, chunk_cycles, chunk_bytes, sink, user);
    });
}

int32_t fd_sink(void *user, int32_t, int64_t, int64_t, const void *rows, int64_t bytes)
{
    const int fd = static_cast<int>(reinterpret_cast<intptr_t>(user));
    const char *p = static_cast<const char *>(rows);
    while (bytes > 0) {
        const ssize_t w = ::write(fd, p, static_cast<size_t>(bytes));
        if (w < 0 && errno == EINTR) continue;
        if (w <= 0) return 1;
        p += w;
        bytes -= w;
    }
    return 0;
}

hbm_status get_samples(hbm_ctx *ctx, int32_t slot, int64_t first, int64_t count, double *theta_out, void *chi_out,
                       int64_t *n_written)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        hbm_status s = check_slot(c, slot, true);
        if (s != HBM_OK) return s;
        if (first < 0 || count < 0) return fail(c, HBM_EINVAL, "first and count must be >= 0");
        const Slot &sl = c->slots[slot];
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (!theta_out && !chi_out) {
            if (n_written) *n_written = sl.n_theta;
            return HBM_OK;
        }
        if (theta_out) {
            if (first + count > sl.n_theta) return fail(c, HBM_EINVAL, "theta rows requested beyond the trace");
            const double *src = c->theta_trace + (static_cast<size_t>(slot) * c->pool.max_cycles + first) * c->p;
            HIPCHK(c, hipMemcpy(theta_out, src, sizeof(double) * c->p * count, hipMemcpyDeviceToHost));
        }
        if (chi_out) {
            const int64_t taken = sl.thin > 0 ? sl.k / sl.thin : 0;
            const int64_t have = taken < sl.snap_cap ? taken : sl.snap_cap;
            if (first + count > have) return fail(c, HBM_EINVAL, "latent snapshots requested beyond those taken");
            if (count > 0) {
                // rows (snapshot, component) of the slot's object range
                const size_t w = c->esize * sl.n, pitch = c->esize * c->cap;
                const char *src = static_cast<const char *>(c->buf.chi_samples) +
                                  pitch * static_cast<size_t>(first * c->d) + c->esize * sl.obj_start;
                HIPCHK(c, hipMemcpy2D(chi_out, w, src, pitch, w, static_cast<size_t>(count * c->d),
                                      hipMemcpyDefault));
            }
        }
        if (n_written) *n_written = count;
        return HBM_OK;
    });
}

hbm_status get_theta(hbm_ctx *ctx, int32_t slot, double *theta, double *chol_theta, int64_t *k)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        hbm_status st = check_slot(c, slot, true);
        if (st != HBM_OK) return st;
        CycleState &h = c->h_cs[slot];
        if ((st = read_slot(c, slot, &h)) != HBM_OK) return st;
        if (theta) std::memcpy(theta, h.theta, sizeof(double) * c->p);
        if (chol_theta) std::memcpy(chol_theta, h.chol_theta, sizeof(double) * c->p * c->p);
        if (k) *k = h.k;
        return HBM_OK;
    });
}

hbm_status set_theta(hbm_ctx *ctx, int32_t slot, const double *theta, const double *chol_theta, int64_t k)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        hbm_status st = check_slot(c, slot, true);
        if (st != HBM_OK) return st;
        if (!theta || !chol_theta || k < 0) return fail(c, HBM_EINVAL, "theta, chol_theta non-NULL and k >= 0");
        for (int r = 0; r < c->p; ++r) {
            if (!std::isfinite(theta[r]) || !(chol_theta[r * c->p + r] > 0.0))
                return fail(c, HBM_EINVAL, "theta finite and chol_theta with a positive diagonal");
        }
        CycleState h;
        if ((st = read_slot(c, slot, &h)) != HBM_OK) return st;
        const CycleState keep = h;
        for (int r = 0; r < c->p; ++r) {
            h.theta[r] = theta[r];
            for (int q = 0; q < c->p; ++q) h.chol_theta[r * c->p + q] = q <= r ? chol_theta[r * c->p + q] : 0.0;
        }
        h.k = k;
        std::fill(c->h_which.begin(), c->h_which.end(), 0);
        c->h_which[slot] = 1;
        HIPCHK(c, hipMemcpyAsync(c->cs + slot, &h, sizeof(h), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->which, c->h_which.data(), sizeof(int32_t) * c->n_slots, hipMemcpyHostToDevice,
                                 c->stream));
        if ((st = c->ops->set_theta(c)) != HBM_OK) return st;
        CycleState back;
        if ((st = read_slot(c, slot, &back)) != HBM_OK) return st;
        if (!(back.lprior_cur > -HUGE_VAL) || (back.flags & kFlagBadZ)) {
            HIPCHK(c, hipMemcpyAsync(c->cs + slot, &keep, sizeof(keep), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            return fail(c, HBM_EDOMAIN, "theta outside the prior support or Z(theta) not positive");
        }
        c->slots[slot].k = k;
        c->slots[slot].sums_ready = false;
        return HBM_OK;
    });
}

hbm_status ram_sweep_trace(hbm_ctx *ctx, void *trace)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!trace) return fail(c, HBM_EINVAL, "trace must be non-NULL");
        hbm_status st = c->ops->sweep(c, false, trace);
        if (st != HBM_OK) return st;
        for (Slot &sl : c->slots)
            if (sl.active) {
                sl.k += 1;
                sl.sums_ready = true;
            }
        if ((st = read_all(c)) != HBM_OK) return st;
        return check_flags(c);
    });
}

namespace {

// Checkpoint blob: header, one record per slot, every slot's device
// theta-chain state, then every slot's theta trace rows.
constexpr uint64_t kStateMagic = 0x4554415453424d48ull;   // "HBMSTATE"

struct StateHeader {
    uint64_t magic;
    uint32_t version;
    int32_t model;
    int32_t n_slots;
    int32_t p;
    int64_t cap;
    int64_t max_cycles;
    int64_t state_size;        // sizeof(CycleState)
    int64_t bytes;             // whole blob
};

struct SlotRecord {
    int32_t loaded, active, sums_ready, thin;
    int64_t n, obj_start, k, n_theta, budget, trace_cap, snap_cap;
};

size_t state_bytes(const CtxImpl *c)
{
    size_t b = sizeof(StateHeader) + (sizeof(SlotRecord) + sizeof(CycleState)) * c->n_slots;
    for (const Slot &sl : c->slots) b += sizeof(double) * c->p * (sl.loaded ? sl.n_theta : 0);
    return b;
}

}  // namespace

hbm_status get_state(hbm_ctx *ctx, void *blob, size_t *size)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!size) return fail(c, HBM_EINVAL, "size must be non-NULL");
        for (const Slot &sl : c->slots)
            if (sl.sums_ready) return fail(c, HBM_ESTATE, "a ram_sweep is waiting for its theta_step");
        const size_t need = state_bytes(c);
        if (!blob) {
            *size = need;
            return HBM_OK;
        }
        if (*size < need) {
            *size = need;
            return fail(c, HBM_ENOSPACE, "state buffer too small");
        }
        hbm_status st = read_all(c);
        if (st != HBM_OK) return st;
        char *out = static_cast<char *>(blob);
        StateHeader h{kStateMagic, 1u, c->pool.model, c->n_slots, c->p, c->cap, c->pool.max_cycles,
                      static_cast<int64_t>(sizeof(CycleState)), static_cast<int64_t>(need)};
        std::memcpy(out, &h, sizeof(h));
        out += sizeof(h);
        for (const Slot &sl : c->slots) {
            SlotRecord r{sl.loaded, sl.active, sl.sums_ready, sl.thin, sl.n, sl.obj_start, sl.k, sl.n_theta,
                         sl.budget, sl.trace_cap, sl.snap_cap};
            std::memcpy(out, &r, sizeof(r));
            out += sizeof(r);
        }
        std::memcpy(out, c->h_cs.data(), sizeof(CycleState) * c->n_slots);
        out += sizeof(CycleState) * c->n_slots;
        for (int32_t j = 0; j < c->n_slots; ++j) {
            const Slot &sl = c->slots[j];
            if (!sl.loaded || sl.n_theta == 0) continue;
            const size_t bytes = sizeof(double) * c->p * sl.n_theta;
            HIPCHK(c, hipMemcpy(out, c->theta_trace + static_cast<size_t>(j) * c->pool.max_cycles * c->p, bytes,
                                hipMemcpyDeviceToHost));
            out += bytes;
        }
        *size = need;
        return HBM_OK;
    });
}

hbm_status set_state(hbm_ctx *ctx, const void *blob, size_t size)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!blob || size < sizeof(StateHeader)) return fail(c, HBM_EINVAL, "state blob missing or truncated");
        StateHeader h;
        std::memcpy(&h, blob, sizeof(h));
        if (h.magic != kStateMagic || h.version != 1u) return fail(c, HBM_EINVAL, "not a state blob of this library");
        if (h.model != c->pool.model || h.n_slots != c->n_slots || h.p != c->p || h.cap != c->cap ||
            h.max_cycles != c->pool.max_cycles || h.state_size != static_cast<int64_t>(sizeof(CycleState)) ||
            h.bytes != static_cast<int64_t>(size))
            return fail(c, HBM_EINVAL, "state blob is for a differently shaped context");
        const char *in = static_cast<const char *>(blob) + sizeof(h);
        std::vector<SlotRecord> recs(c->n_slots);
        std::memcpy(recs.data(), in, sizeof(SlotRecord) * c->n_slots);
        in += sizeof(SlotRecord) * c->n_slots;
        size_t need = sizeof(StateHeader) + (sizeof(SlotRecord) + sizeof(CycleState)) * c->n_slots;
        for (int32_t j = 0; j < c->n_slots; ++j) {
            const SlotRecord &r = recs[j];
            const Slot &sl = c->slots[j];
            if (r.loaded != static_cast<int32_t>(sl.loaded) || (r.loaded && (r.n != sl.n || r.obj_start != sl.obj_start)))
                return fail(c, HBM_EINVAL, "slot " + std::to_string(j) + " holds a different dataset placement");
            if (r.loaded && (r.n_theta < 0 || r.n_theta > sl.trace_cap || r.k < 0))
                return fail(c, HBM_EINVAL, "slot " + std::to_string(j) + ": counters out of range");
            need += r.loaded ? sizeof(double) * c->p * r.n_theta : 0;
        }
        if (need != size) return fail(c, HBM_EINVAL, "state blob size does not match its contents");
        std::vector<CycleState> cs(c->n_slots);
        std::memcpy(cs.data(), in, sizeof(CycleState) * c->n_slots);
        in += sizeof(CycleState) * c->n_slots;
        HIPCHK(c, hipMemcpyAsync(c->cs, cs.data(), sizeof(CycleState) * c->n_slots, hipMemcpyHostToDevice, c->stream));
        for (int32_t j = 0; j < c->n_slots; ++j) {
            const SlotRecord &r = recs[j];
            if (!r.loaded || r.n_theta == 0) continue;
            const size_t bytes = sizeof(double) * c->p * r.n_theta;
            HIPCHK(c, hipMemcpyAsync(c->theta_trace + static_cast<size_t>(j) * c->pool.max_cycles * c->p, in, bytes,
                                     hipMemcpyHostToDevice, c->stream));
            in += bytes;
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int32_t j = 0; j < c->n_slots; ++j) {
            Slot &sl = c->slots[j];
            const SlotRecord &r = recs[j];
            if (!r.loaded) continue;
            sl.active = r.active != 0;
            sl.sums_ready = r.sums_ready != 0;
            sl.k = r.k;
            sl.n_theta = r.n_theta;
            sl.budget = r.budget;
        }
        return HBM_OK;
    });
}

hbm_status get_stats(hbm_ctx *ctx, int32_t slot, double out[8])
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        hbm_status st = check_slot(c, slot, true);
        if (st != HBM_OK) return st;
        if (!out) return fail(c, HBM_EINVAL, "out must be non-NULL");
        CycleState &h = c->h_cs[slot];
        if ((st = read_slot(c, slot, &h)) != HBM_OK) return st;
        out[0] = h.sum_lf;
        out[1] = h.sum_dlf;
        out[2] = h.logZ_cur;
        out[3] = h.logZ_used;
        out[4] = h.delta_last;
        out[5] = h.alpha_last;
        out[6] = h.n_acc_last;
        out[7] = h.accepted_last;
        return HBM_OK;
    });
}

hbm_status set_launch(hbm_ctx *ctx, int32_t tiles_per_group)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (tiles_per_group != 1 && tiles_per_group != 2 && tiles_per_group != 4)
            return fail(c, HBM_EINVAL, "tiles_per_group must be 1, 2 or 4");
        if (tiles_per_group == c->tpw) return HBM_OK;
        hbm_status st = drop_graph(c);
        if (st != HBM_OK) return st;
        c->tpw = tiles_per_group;
        return HBM_OK;
    });
}

hbm_status set_occupancy(hbm_ctx *ctx, int32_t groups_per_cu)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (groups_per_cu < 0 || groups_per_cu > 64)
            return fail(c, HBM_EINVAL, "groups_per_cu must be 0 (no cap) or in [1, 64]");
        if (groups_per_cu == c->occ_cap) return HBM_OK;
        hbm_status st = drop_graph(c);
        if (st != HBM_OK) return st;
        c->occ_cap = groups_per_cu;
        return HBM_OK;
    });
}

hbm_status autotune(hbm_ctx *ctx, int32_t trial_cycles, int32_t out_choice[3], double out_us[HBM_TUNE_CANDIDATES])
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (trial_cycles < 1) return fail(c, HBM_EINVAL, "trial_cycles must be >= 1");
        const int64_t per = kTuneWarm + trial_cycles, total = HBM_TUNE_CANDIDATES * per;
        for (const Slot &sl : c->slots) {
            if (!sl.active) continue;
            if (sl.sums_ready) return fail(c, HBM_ESTATE, "a ram_sweep is waiting for its theta_step");
            if (sl.n_theta + cycles_taken(sl, total) > sl.trace_cap)
                return fail(c, HBM_ENOSPACE, "theta trace too small for the autotuner's cycles");
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCHK(c, hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(c, HBM_ENOMEM, "hipEventCreate failed");
        }
        // candidates: the two-kernel cycle with tiles per workgroup {1, 2, 4}
        // under a cap of {none, 4, 2} workgroups per compute unit, then the
        // persistent launch (one-dataset contexts in mode HBM_CYCLES_AUTO),
        // then fused cycles with tiles per workgroup {1, 2, 4} (one tile per
        // workgroup for contexts with several datasets).  how: 0 two-kernel
        // graphs, 1 persistent, 2 fused graphs.
        struct Cand { int32_t tpw, cap, how; };
        Cand cand[HBM_TUNE_CANDIDATES];
        int q = 0;
        for (int32_t cap : {0, 4, 2})
            for (int32_t tpw : {1, 2, 4}) cand[q++] = Cand{tpw, cap, 0};
        cand[q++] = Cand{c->tpw, c->occ_cap, 1};
        for (int32_t tpw : {1, 2, 4}) cand[q++] = Cand{tpw, 0, 2};
        const int32_t mode = c->cycle_mode;
        const int32_t keep_tpw = c->tpw, keep_cap = c->occ_cap;
        double best = HUGE_VAL;
        Cand pick{keep_tpw, keep_cap,
                  mode == HBM_CYCLES_AUTO && single(c) ? 1 : (mode == HBM_CYCLES_FUSED ? 2 : 0)};
        hbm_status st = HBM_OK;
        for (int j = 0; j < HBM_TUNE_CANDIDATES && st == HBM_OK; ++j) {
            const Cand &cd = cand[j];
            if (out_us) out_us[j] = static_cast<double>(NAN);
            // every candidate runs its cycles (the trace counts them), timed or not
            const bool usable = cd.how == 0 || (cd.how == 1 && mode == HBM_CYCLES_AUTO && single(c) && !c->stats_mode) ||
                                (cd.how == 2 && (single(c) || cd.tpw == 1));
            const int32_t cm = cd.how == 1 ? HBM_CYCLES_AUTO : cd.how == 2 ? HBM_CYCLES_FUSED : HBM_CYCLES_GRAPH;
            if ((st = set_cycle_mode(ctx, cm)) != HBM_OK) break;
            if (cd.how != 1) {
                if ((st = set_launch(ctx, cd.tpw)) != HBM_OK || (st = set_occupancy(ctx, cd.cap)) != HBM_OK) break;
                if ((st = ensure_graphs(c, kTuneWarm)) != HBM_OK || (st = ensure_graphs(c, trial_cycles)) != HBM_OK)
                    break;
            }
            if ((st = run_cycles(ctx, kTuneWarm, 1)) != HBM_OK) break;
            const int64_t p0 = c->n_persistent_cycles;
            float ms = 0.0f;
            hipError_t e = hipSuccess;
            if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) { st = hip_fail(c, e, "hipEventRecord"); break; }
            if ((st = run_cycles(ctx, trial_cycles, 1)) != HBM_OK) break;
            if ((e = hipEventRecord(e1, c->stream)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
                st = hip_fail(c, e, "autotune timing");
                break;
            }
            // a persistent candidate counts only when the launch really happened
            if (!usable || (cd.how == 1 && c->n_persistent_cycles - p0 != trial_cycles)) continue;
            const double us = 1e3 * ms / trial_cycles;
            if (out_us) out_us[j] = us;
            if (us < best) {
                best = us;
                pick = cd;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != HBM_OK) {
            c->cycle_mode = mode;
            return st;
        }
        if (pick.how == 1) {
            if ((st = set_cycle_mode(ctx, HBM_CYCLES_AUTO)) != HBM_OK || (st = set_launch(ctx, keep_tpw)) != HBM_OK ||
                (st = set_occupancy(ctx, keep_cap)) != HBM_OK)
                return st;
        } else {
            if ((st = set_cycle_mode(ctx, pick.how == 2 ? HBM_CYCLES_FUSED : HBM_CYCLES_GRAPH)) != HBM_OK ||
                (st = set_launch(ctx, pick.tpw)) != HBM_OK || (st = set_occupancy(ctx, pick.cap)) != HBM_OK)
                return st;
        }
        if (out_choice) {
            out_choice[0] = c->tpw;
            out_choice[1] = c->occ_cap;
            out_choice[2] = pick.how;
        }
        return HBM_OK;
    });
}

hbm_status kernel_timing(hbm_ctx *ctx, int32_t enable)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        c->timing = enable != 0;
        return HBM_OK;
    });
}

hbm_status read_kernel_timing(hbm_ctx *ctx, int64_t *n_launches, double *mean_ms)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        hbm_status st = drain_timing(c);
        if (st != HBM_OK) return st;
        if (n_launches) *n_launches = c->timed_launches;
        if (mean_ms) *mean_ms = c->timed_launches > 0 ? c->timed_ms / c->timed_launches : 0.0;
        c->timed_launches = 0;
        c->timed_ms = 0.0;
        return HBM_OK;
    });
}

const char *last_error(const hbm_ctx *ctx)
{
    if (!ctx) return g_init_error.c_str();
    return static_cast<const CtxImpl *>(ctx)->err.c_str();
}

void destroy_chains(hbm_ctx *ctx) { release(static_cast<CtxImpl *>(ctx)); }

}  // extern "C"
