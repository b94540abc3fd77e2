// Host runtime and C ABI of the sampler (declared in include/hbm.h).
//
// The host only validates arguments, allocates the library's scratch,
// enqueues kernels and copies results; all sampler arithmetic runs in the
// kernels of kernels.h.
#include "hbm.h"
#include "kernels.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace hbm;

namespace {

thread_local std::string g_init_error;

struct CtxImpl;

struct Launch {
    hbm_status (*sweep)(CtxImpl *, bool full, void *trace);
    hbm_status (*theta)(CtxImpl *);
    hbm_status (*set_theta)(CtxImpl *);
    hbm_status (*poplik)(CtxImpl *, const double *theta);
    hbm_status (*prepare)(CtxImpl *);
    hbm_status (*check_init)(CtxImpl *);
};

struct CtxImpl {
    hbm_config cfg{};
    hbm_buffers buf{};
    int d = 0, p = 0, m = 0, md = 0, nc = 0;
    size_t esize = 0;
    int64_t n = 0;
    int32_t n_tiles = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    void *dd = nullptr;
    double *partials = nullptr;     // [n_tiles][3]
    double *zout = nullptr;         // [2]: ln Z of pop_loglik
    Precomp *side = nullptr;        // values the sweep's workgroup 0 leaves for the epilogue
    double *ref_t = nullptr, *ref_w = nullptr, *qx = nullptr, *qw = nullptr, *qeps = nullptr;
    CycleState *cs = nullptr;
    Statics *st = nullptr;
    double *theta_trace = nullptr;
    int64_t trace_cap = 0, snap_cap = 0;
    // host bookkeeping that mirrors the device state
    int64_t k = 0, n_theta = 0;
    bool sums_ready = false;
    bool poisoned = false;
    std::string err;
    const Launch *ops = nullptr;
    // graph of consecutive full cycles
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t graph_len = 0;
    // per-launch timing of the sweep kernel
    bool timing = false;
    std::vector<hipEvent_t> ev_free, ev_pending;
    int64_t timed_launches = 0;
    double timed_ms = 0.0;
};

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

int blocks_for(int64_t n) { return static_cast<int>((n + kBlock - 1) / kBlock); }

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
        a.snaps = static_cast<T *>(c->buf.chi_samples);
        a.trace = static_cast<T *>(trace);
        a.partials = c->partials;
        a.side = c->side;
        a.cs = c->cs;
        a.st = c->st;
        a.qx = c->qx;
        a.qw = c->qw;
        a.qeps = c->qeps;
        a.n = c->n;
        a.n_tiles = c->n_tiles;
        return a;
    }

    static hbm_status sweep(CtxImpl *c, bool full, void *trace)
    {
        const SweepArgs<T> a = sweep_args(c, trace);
        const dim3 grid(static_cast<unsigned>(c->n_tiles + 1));
        if (c->timing) {
            // the runtime takes both timestamps from the dispatch itself
            hipEvent_t e0 = take_event(c), e1 = take_event(c);
            if (!e0 || !e1) return fail(c, HBM_ENOMEM, "hipEventCreate failed");
            if (trace)
                hipExtLaunchKernelGGL((sweep_kernel<M, true>), grid, dim3(kBlock), 0, c->stream, e0, e1, 0, a);
            else
                hipExtLaunchKernelGGL((sweep_kernel<M, false>), grid, dim3(kBlock), 0, c->stream, e0, e1, 0, a);
            c->ev_pending.push_back(e0);
            c->ev_pending.push_back(e1);
        } else if (trace) {
            hipLaunchKernelGGL((sweep_kernel<M, true>), grid, dim3(kBlock), 0, c->stream, a);
        } else {
            hipLaunchKernelGGL((sweep_kernel<M, false>), grid, dim3(kBlock), 0, c->stream, a);
        }
        LAUNCHCHK(c, "sweep_kernel");
        if (full)
            hipLaunchKernelGGL((epilogue_kernel<M, true>), dim3(1), dim3(kBlock), 0, c->stream, c->cs, c->st,
                               c->partials, c->side, c->theta_trace, c->n_tiles);
        else
            hipLaunchKernelGGL((epilogue_kernel<M, false>), dim3(1), dim3(kBlock), 0, c->stream, c->cs, c->st,
                               c->partials, c->side, c->theta_trace, c->n_tiles);
        LAUNCHCHK(c, "epilogue_kernel");
        return HBM_OK;
    }

    static hbm_status theta(CtxImpl *c)
    {
        hipLaunchKernelGGL((theta_kernel<M>), dim3(1), dim3(kBlock), 0, c->stream, c->cs, c->st, c->side,
                           c->theta_trace);
        LAUNCHCHK(c, "theta_kernel");
        return HBM_OK;
    }

    static hbm_status set_theta(CtxImpl *c)
    {
        hipLaunchKernelGGL((set_theta_kernel<M>), dim3(1), dim3(kBlock), 0, c->stream, c->cs, c->st, c->qx, c->qw,
                           c->qeps);
        LAUNCHCHK(c, "set_theta_kernel");
        return HBM_OK;
    }

    static hbm_status poplik(CtxImpl *c, const double *theta)
    {
        PopArgs<T> a;
        a.chi = static_cast<const T *>(c->buf.chi);
        a.dd = static_cast<const T *>(c->dd);
        a.partials = c->partials;
        a.zout = c->zout;
        a.st = c->st;
        a.qx = c->qx;
        a.qw = c->qw;
        a.qeps = c->qeps;
        a.n = c->n;
        for (int r = 0; r < kMaxP; ++r) a.theta[r] = r < M::P ? theta[r] : 0.0;
        hipLaunchKernelGGL((poplik_kernel<M>), dim3(c->n_tiles + 1), dim3(kBlock), 0, c->stream, a);
        LAUNCHCHK(c, "poplik_kernel");
        hipLaunchKernelGGL(poplik_finish_kernel, dim3(1), dim3(kBlock), 0, c->stream, c->cs, c->partials, c->zout,
                           c->n, c->n_tiles);
        LAUNCHCHK(c, "poplik_finish_kernel");
        return HBM_OK;
    }

    static hbm_status prepare(CtxImpl *c)
    {
        hipLaunchKernelGGL((statics_kernel<M>), dim3(1), dim3(1), 0, c->stream, c->st);
        LAUNCHCHK(c, "statics_kernel");
        hipLaunchKernelGGL((derive_data_kernel<M>), dim3(blocks_for(c->n)), dim3(kBlock), 0, c->stream,
                           static_cast<const T *>(c->buf.data), static_cast<T *>(c->dd), c->st);
        LAUNCHCHK(c, "derive_data_kernel");
        hipLaunchKernelGGL((init_chain_kernel<M>), dim3(blocks_for(c->n)), dim3(kBlock), 0, c->stream,
                           static_cast<T *>(c->buf.chol), c->buf.acc, c->cfg.s0, c->st);
        LAUNCHCHK(c, "init_chain_kernel");
        if (M::kSelection) {
            const int nq = c->cfg.n_quad;
            hipLaunchKernelGGL(gauss_legendre_kernel, dim3((nq + 127) / 128), dim3(128), 0, c->stream, c->ref_t,
                               c->ref_w, nq);
            LAUNCHCHK(c, "gauss_legendre_kernel");
            hipLaunchKernelGGL(eps_table_kernel, dim3((nq + 63) / 64), dim3(64), 0, c->stream, c->ref_t, c->ref_w,
                               c->qx, c->qw, c->qeps, c->st);
            LAUNCHCHK(c, "eps_table_kernel");
        }
        return HBM_OK;
    }

    static hbm_status check_init(CtxImpl *c)
    {
        hipLaunchKernelGGL((check_init_kernel<M>), dim3(blocks_for(c->n)), dim3(kBlock), 0, c->stream,
                           static_cast<const T *>(c->buf.chi), static_cast<const T *>(c->dd), c->cs, c->st);
        LAUNCHCHK(c, "check_init_kernel");
        return HBM_OK;
    }

    static const Launch *table()
    {
        static const Launch t{&sweep, &theta, &set_theta, &poplik, &prepare, &check_init};
        return &t;
    }
};

struct ModelInfo {
    int d, p, m, md, precision;
    const Launch *ops;
};

bool model_info(int model, ModelInfo *mi)
{
    switch (model) {
    case HBM_NORMAL_NORMAL_1D: *mi = {NN1D::D, NN1D::P, NN1D::M, NN1D::MD, HBM_FP64, Ops<NN1D>::table()}; return true;
    case HBM_GAMMA_LF_1D: *mi = {LF1D::D, LF1D::P, LF1D::M, LF1D::MD, HBM_FP32, Ops<LF1D>::table()}; return true;
    case HBM_GAMMA_LF_COLOR_3D: *mi = {LF3D::D, LF3D::P, LF3D::M, LF3D::MD, HBM_FP32, Ops<LF3D>::table()}; return true;
    case HBM_NORMAL_NORMAL_3D: *mi = {NN3D::D, NN3D::P, NN3D::M, NN3D::MD, HBM_FP64, Ops<NN3D>::table()}; return true;
    default: return false;
    }
}

bool has_selection(int model) { return model == HBM_GAMMA_LF_1D || model == HBM_GAMMA_LF_COLOR_3D; }

hbm_status usable(CtxImpl *c)
{
    if (!c) return HBM_EINVAL;
    if (c->poisoned) return fail(c, HBM_ESTATE, "context poisoned by an earlier HIP error: " + c->err);
    return HBM_OK;
}

hbm_status read_state(CtxImpl *c, CycleState *h)
{
    HIPCHK(c, hipMemcpyAsync(h, c->cs, sizeof(CycleState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HBM_OK;
}

hbm_status clear_flags(CtxImpl *c)
{
    const int32_t zero = 0;
    HIPCHK(c, hipMemcpyAsync(reinterpret_cast<char *>(c->cs) + offsetof(CycleState, flags), &zero, sizeof(zero),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HBM_OK;
}

// Turns sticky device flags into a status after a synchronising call.
hbm_status check_flags(CtxImpl *c, const CycleState &h)
{
    if (h.flags == 0) return HBM_OK;
    std::string msg;
    if (h.flags & kFlagNonFiniteState) msg += "non-finite latent log density; ";
    if (h.flags & kFlagBadZ) msg += "selection normaliser not positive and finite; ";
    if (h.flags & kFlagTraceFull) msg += "theta trace full; ";
    if (h.flags & kFlagNoSums) msg += "theta step without a sweep; ";
    hbm_status st = clear_flags(c);
    if (st != HBM_OK) return st;
    if (h.flags & (kFlagNonFiniteState | kFlagBadZ)) return fail(c, HBM_EDOMAIN, msg);
    if (h.flags & kFlagTraceFull) return fail(c, HBM_ENOSPACE, msg);
    return fail(c, HBM_ESTATE, msg);
}

void release(CtxImpl *c)
{
    if (!c) return;
    if (c->stream || c->cs) (void)hipStreamSynchronize(c->stream);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_pending) (void)hipEventDestroy(e);
    void *ptrs[] = {c->dd, c->partials, c->zout, c->side, c->ref_t, c->ref_w, c->qx, c->qw, c->qeps,
                    c->cs, c->st, c->theta_trace};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete c;
}

hbm_status validate_config(const hbm_config *cfg, const hbm_buffers *b, const double *theta0, ModelInfo *mi)
{
    if (!cfg || !b || !theta0) return fail(nullptr, HBM_EINVAL, "config, buffers and theta0 must be non-NULL");
    if (!model_info(cfg->model, mi)) return fail(nullptr, HBM_EINVAL, "unknown model id");
    if (cfg->precision != mi->precision)
        return fail(nullptr, HBM_EINVAL, "precision does not match the model (NN: FP64, LF: FP32)");
    if (cfg->n_objects < 1 || cfg->n_objects > (int64_t)INT32_MAX - kBlock)
        return fail(nullptr, HBM_EINVAL, "n_objects must be in [1, 2^31 - 257]");
    if (!b->data || !b->chi || !b->chol || !b->acc)
        return fail(nullptr, HBM_EINVAL, "data, chi, chol and acc buffers must be non-NULL");
    if (!(cfg->target_accept > 0.0 && cfg->target_accept < 1.0) ||
        !(cfg->theta_target_accept > 0.0 && cfg->theta_target_accept < 1.0))
        return fail(nullptr, HBM_EINVAL, "target acceptance rates must lie in (0, 1)");
    if (!(cfg->eta_exponent > 0.5 && cfg->eta_exponent <= 1.0))
        return fail(nullptr, HBM_EINVAL, "eta_exponent must lie in (1/2, 1]");
    if (!(cfg->s0 > 0.0) || !std::isfinite(cfg->s0)) return fail(nullptr, HBM_EINVAL, "s0 must be positive");
    if (cfg->thin_chi < 0 || cfg->max_cycles < 0) return fail(nullptr, HBM_EINVAL, "thin_chi and max_cycles must be >= 0");
    if (has_selection(cfg->model)) {
        if (cfg->n_quad < 16 || cfg->n_quad > 4096) return fail(nullptr, HBM_EINVAL, "n_quad must be in [16, 4096]");
        const double *mc = cfg->model_consts;
        if (!(mc[0] > 0.0) || !(mc[1] > 0.0) || !(mc[2] > 0.0) || !std::isfinite(mc[3]))
            return fail(nullptr, HBM_EINVAL, "LF model constants need F_th, sigma_F, rmax > 0 and a finite ln L0");
        if (cfg->model == HBM_GAMMA_LF_COLOR_3D && (!(mc[4] > 0.0) || !(mc[5] > 0.0)))
            return fail(nullptr, HBM_EINVAL, "LF colour model needs f_r > 0 and sigma_c > 0");
    }
    if (cfg->model == HBM_NORMAL_NORMAL_3D) {
        const double *mc = cfg->model_consts;
        const double a = mc[0], b2 = mc[1], c2 = mc[2], d2 = mc[3], e2 = mc[4], f2 = mc[5];
        const double det = a * (c2 * f2 - e2 * e2) - b2 * (b2 * f2 - e2 * d2) + d2 * (b2 * e2 - c2 * d2);
        if (!(a > 0.0) || !(a * c2 - b2 * b2 > 0.0) || !(det > 0.0) || !(mc[6] > 0) || !(mc[7] > 0) || !(mc[8] > 0))
            return fail(nullptr, HBM_EINVAL, "C_pop must be positive definite and sigma_j > 0");
    }
    for (int r = 0; r < mi->p; ++r) {
        if (!std::isfinite(theta0[r])) return fail(nullptr, HBM_EINVAL, "theta0 must be finite");
        if (!(cfg->theta_chol0[r * mi->p + r] > 0.0))
            return fail(nullptr, HBM_EINVAL, "theta_chol0 must have a positive diagonal");
        for (int q = 0; q <= r; ++q)
            if (!std::isfinite(cfg->theta_chol0[r * mi->p + q])) return fail(nullptr, HBM_EINVAL, "theta_chol0 not finite");
    }
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

}  // namespace

struct hbm_ctx : CtxImpl {};

extern "C" {

hbm_status init_chains(const hbm_config *config, const hbm_buffers *buffers, const double *chi0_host,
                       const double *theta0, void *hip_stream, hbm_ctx **out)
{
    if (!out) return fail(nullptr, HBM_EINVAL, "out must be non-NULL");
    *out = nullptr;
    ModelInfo mi;
    hbm_status s = validate_config(config, buffers, theta0, &mi);
    if (s != HBM_OK) return s;

    CtxImpl *c = new (std::nothrow) hbm_ctx();
    if (!c) return fail(nullptr, HBM_ENOMEM, "host allocation failed");
    c->cfg = *config;
    c->buf = *buffers;
    c->d = mi.d;
    c->p = mi.p;
    c->m = mi.m;
    c->md = mi.md;
    c->nc = mi.d * (mi.d + 1) / 2;
    c->esize = mi.precision == HBM_FP64 ? 8 : 4;
    c->n = config->n_objects;
    c->n_tiles = blocks_for(c->n);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ops = mi.ops;
    c->trace_cap = config->max_cycles;
    c->snap_cap = (config->thin_chi > 0 && buffers->chi_samples) ? config->max_cycles / config->thin_chi : 0;

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
    const bool sel = has_selection(config->model);
    const int nq = sel ? config->n_quad : 1;
    if ((s = alloc(&c->dd, c->esize * c->md * c->n)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->partials), sizeof(double) * 3 * c->n_tiles)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->zout), sizeof(double) * 2)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->side), sizeof(Precomp))) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->ref_t), sizeof(double) * nq)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->ref_w), sizeof(double) * nq)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->qx), sizeof(double) * nq)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->qw), sizeof(double) * nq)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->qeps), sizeof(double) * nq)) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->cs), sizeof(CycleState))) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->st), sizeof(Statics))) != HBM_OK ||
        (s = alloc(reinterpret_cast<void **>(&c->theta_trace), sizeof(double) * c->p * c->trace_cap)) != HBM_OK)
        return bail(s);

    Statics hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.n = c->n;
    hs.trace_cap = c->trace_cap;
    hs.snap_cap = c->snap_cap;
    hs.thin = config->thin_chi;
    hs.nq = nq;
    hs.adapt_theta = config->adapt_theta;
    hs.p = c->p;
    hs.key0 = static_cast<uint32_t>(config->seed & 0xffffffffu);
    hs.key1 = static_cast<uint32_t>(config->seed >> 32);
    hs.gamma = config->eta_exponent;
    hs.alpha_star = config->target_accept;
    hs.alpha_star_theta = config->theta_target_accept;
    std::memcpy(hs.mc, config->model_consts, sizeof(hs.mc));

    CycleState hc;
    std::memset(&hc, 0, sizeof(hc));
    for (int r = 0; r < c->p; ++r) {
        hc.theta[r] = theta0[r];
        for (int q = 0; q < c->p; ++q) hc.chol_theta[r * c->p + q] = q <= r ? config->theta_chol0[r * c->p + q] : 0.0;
    }
    hc.first_bad = INT32_MAX;

    hipError_t e;
    if ((e = hipMemcpyAsync(c->st, &hs, sizeof(hs), hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c->cs, &hc, sizeof(hc), hipMemcpyHostToDevice, c->stream)) != hipSuccess) {
        hip_fail(c, e, "init copies");
        return bail(HBM_EHIP);
    }
    if (chi0_host) {
        std::vector<char> tmp(c->esize * c->d * c->n);
        for (int64_t j = 0; j < c->d * c->n; ++j) {
            if (c->esize == 4) reinterpret_cast<float *>(tmp.data())[j] = static_cast<float>(chi0_host[j]);
            else reinterpret_cast<double *>(tmp.data())[j] = chi0_host[j];
        }
        if ((e = hipMemcpyAsync(c->buf.chi, tmp.data(), tmp.size(), hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
            hip_fail(c, e, "chi0 copy");
            return bail(HBM_EHIP);
        }
    }
    if ((s = c->ops->prepare(c)) != HBM_OK) return bail(s);
    if ((s = c->ops->set_theta(c)) != HBM_OK) return bail(s);
    if ((s = c->ops->check_init(c)) != HBM_OK) return bail(s);
    CycleState back;
    if ((s = read_state(c, &back)) != HBM_OK) return bail(s);
    if (!(back.lprior_cur > -HUGE_VAL)) {
        c->err = "theta0 is outside the prior support";
        return bail(HBM_EDOMAIN);
    }
    if (back.flags & kFlagBadZ) {
        c->err = "selection normaliser Z(theta0) is not positive and finite";
        return bail(HBM_EDOMAIN);
    }
    if (back.flags & kFlagNonFiniteState) {
        c->err = "non-finite initial log density at object " + std::to_string(back.first_bad);
        return bail(HBM_EDOMAIN);
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
            c->k += 1;
            c->sums_ready = true;
        }
        if (out_accept_rate) {
            CycleState h;
            hbm_status st = read_state(c, &h);
            if (st != HBM_OK) return st;
            *out_accept_rate = h.n_acc_last / static_cast<double>(c->n);
            return check_flags(c, h);
        }
        return HBM_OK;
    });
}

hbm_status pop_loglik(hbm_ctx *ctx, const double *theta, double *out)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!theta || !out) return fail(c, HBM_EINVAL, "theta and out must be non-NULL");
        for (int r = 0; r < c->p; ++r)
            if (!std::isfinite(theta[r])) return fail(c, HBM_EINVAL, "theta must be finite");
        hbm_status st = c->ops->poplik(c, theta);
        if (st != HBM_OK) return st;
        CycleState h;
        if ((st = read_state(c, &h)) != HBM_OK) return st;
        *out = h.poplik_out;
        return HBM_OK;
    });
}

hbm_status theta_step(hbm_ctx *ctx, int32_t *out_accepted)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!c->sums_ready) return fail(c, HBM_ESTATE, "theta_step needs a ram_sweep since the last theta step");
        if (c->n_theta >= c->trace_cap) return fail(c, HBM_ENOSPACE, "theta trace full (max_cycles)");
        hbm_status st = c->ops->theta(c);
        if (st != HBM_OK) return st;
        c->sums_ready = false;
        c->n_theta += 1;
        CycleState h;
        if ((st = read_state(c, &h)) != HBM_OK) return st;
        if (out_accepted) *out_accepted = h.accepted_last;
        return check_flags(c, h);
    });
}

hbm_status run_cycles(hbm_ctx *ctx, int64_t n_cycles, int32_t use_graph)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (n_cycles < 0) return fail(c, HBM_EINVAL, "n_cycles must be >= 0");
        if (c->n_theta + n_cycles > c->trace_cap) return fail(c, HBM_ENOSPACE, "theta trace would overflow (max_cycles)");
        if (c->sums_ready) return fail(c, HBM_ESTATE, "a ram_sweep is waiting for its theta_step");
        int64_t left = n_cycles;
        if (use_graph && !c->timing && n_cycles > 0) {
            const int64_t glen = 32;
            if (!c->graph_exec) {
                if (!c->capture_stream)
                    HIPCHK(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
                hipStream_t saved = c->stream;
                c->stream = c->capture_stream;
                HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
                hbm_status st = HBM_OK;
                for (int64_t j = 0; j < glen && st == HBM_OK; ++j) st = c->ops->sweep(c, true, nullptr);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
                c->stream = saved;
                if (st != HBM_OK) return st;
                if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
                c->graph = g;
                HIPCHK(c, hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
                c->graph_len = glen;
            }
            while (left >= c->graph_len) {
                HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
                left -= c->graph_len;
            }
        }
        for (int64_t j = 0; j < left; ++j) {
            hbm_status st = c->ops->sweep(c, true, nullptr);
            if (st != HBM_OK) return st;
        }
        c->k += n_cycles;
        c->n_theta += n_cycles;
        return HBM_OK;
    });
}

hbm_status get_samples(hbm_ctx *ctx, int64_t first, int64_t count, double *theta_out, void *chi_out,
                       int64_t *n_written)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (first < 0 || count < 0) return fail(c, HBM_EINVAL, "first and count must be >= 0");
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (!theta_out && !chi_out) {
            if (n_written) *n_written = c->n_theta;
            return HBM_OK;
        }
        if (theta_out) {
            if (first + count > c->n_theta) return fail(c, HBM_EINVAL, "theta rows requested beyond the trace");
            HIPCHK(c, hipMemcpy(theta_out, c->theta_trace + first * c->p, sizeof(double) * c->p * count,
                                hipMemcpyDeviceToHost));
        }
        if (chi_out) {
            const int64_t taken = c->cfg.thin_chi > 0 ? c->k / c->cfg.thin_chi : 0;
            const int64_t have = taken < c->snap_cap ? taken : c->snap_cap;
            if (first + count > have) return fail(c, HBM_EINVAL, "latent snapshots requested beyond those taken");
            const size_t row = c->esize * c->d * c->n;
            HIPCHK(c, hipMemcpy(chi_out, static_cast<char *>(c->buf.chi_samples) + row * first, row * count,
                                hipMemcpyDeviceToHost));
        }
        if (n_written) *n_written = count;
        return HBM_OK;
    });
}

hbm_status get_theta(hbm_ctx *ctx, double *theta, double *chol_theta, int64_t *k)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        CycleState h;
        hbm_status st = read_state(c, &h);
        if (st != HBM_OK) return st;
        if (theta) std::memcpy(theta, h.theta, sizeof(double) * c->p);
        if (chol_theta) std::memcpy(chol_theta, h.chol_theta, sizeof(double) * c->p * c->p);
        if (k) *k = h.k;
        return HBM_OK;
    });
}

hbm_status set_theta(hbm_ctx *ctx, const double *theta, const double *chol_theta, int64_t k)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!theta || !chol_theta || k < 0) return fail(c, HBM_EINVAL, "theta, chol_theta non-NULL and k >= 0");
        for (int r = 0; r < c->p; ++r) {
            if (!std::isfinite(theta[r]) || !(chol_theta[r * c->p + r] > 0.0))
                return fail(c, HBM_EINVAL, "theta finite and chol_theta with a positive diagonal");
        }
        CycleState h;
        hbm_status st = read_state(c, &h);
        if (st != HBM_OK) return st;
        CycleState keep = h;
        for (int r = 0; r < c->p; ++r) {
            h.theta[r] = theta[r];
            for (int q = 0; q < c->p; ++q) h.chol_theta[r * c->p + q] = q <= r ? chol_theta[r * c->p + q] : 0.0;
        }
        h.k = k;
        HIPCHK(c, hipMemcpyAsync(c->cs, &h, sizeof(h), hipMemcpyHostToDevice, c->stream));
        if ((st = c->ops->set_theta(c)) != HBM_OK) return st;
        CycleState back;
        if ((st = read_state(c, &back)) != HBM_OK) return st;
        if (!(back.lprior_cur > -HUGE_VAL) || (back.flags & kFlagBadZ)) {
            HIPCHK(c, hipMemcpyAsync(c->cs, &keep, sizeof(keep), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            return fail(c, HBM_EDOMAIN, "theta outside the prior support or Z(theta) not positive");
        }
        c->k = k;
        c->sums_ready = false;
        return HBM_OK;
    });
}

hbm_status ram_sweep_trace(hbm_ctx *ctx, void *trace)
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!trace) return fail(c, HBM_EINVAL, "trace must be non-NULL");
        hbm_status st = c->ops->sweep(c, false, trace);
        if (st != HBM_OK) return st;
        c->k += 1;
        c->sums_ready = true;
        CycleState h;
        if ((st = read_state(c, &h)) != HBM_OK) return st;
        return check_flags(c, h);
    });
}

hbm_status get_stats(hbm_ctx *ctx, double out[8])
{
    return with_ctx(ctx, [&](CtxImpl *c) -> hbm_status {
        if (!out) return fail(c, HBM_EINVAL, "out must be non-NULL");
        CycleState h;
        hbm_status st = read_state(c, &h);
        if (st != HBM_OK) return st;
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
