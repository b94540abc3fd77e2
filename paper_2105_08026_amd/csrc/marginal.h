// Marginal likelihood of theta with each object's 1-D latent integrated out
// by quadrature (Sec. 6 proposes this for low-dimensional latents; the
// objects are conditionally independent given theta, so the integrals are
// independent):
//   ln L(theta) = sum_i ln int l_i(chi) f(chi; theta) dchi - N ln Z(theta).
// Everything here is FP64.
//
// One object is shared by kMargLanes lanes; lane s of the group takes nodes
// s, s + 8, s + 16, ... of the object's rule, keeps their log integrands in
// registers, and the group combines them as max + log-sum-exp, so no scale
// has to be guessed before the integrand is seen.
//
// The rule for a datum-centred model (flux-limited luminosity functions):
//   core     F in [F_A, Fhat] and [Fhat, F_B], kCore Gauss-Legendre nodes
//            each, integrated in the flux F (chi = ln F + k, dchi = dF / F),
//            where the member likelihood is close to a normal in F:
//            F_A = max(Fhat - K sigma(Fhat), Fhat / 4),
//            F_B = Fhat + K sigma(Fhat) / (1 - K alpha)  (so the error at F_B,
//            which grows at most by alpha per unit flux, still leaves F_B K
//            standard errors above Fhat);
//   graded   chi in [chi_A - 13, chi_A], chi_A = ln F_A + k, in 20 panels of
//            widths 0.25 (4), 0.5 (8) and 1 (8) from the top, 8 nodes each:
//            this is where the population can outweigh the member
//            likelihood (a faint detection whose plateau meets a steep
//            population, or the population's own bulk below the datum);
//   tail     chi < chi_T = chi_A - 13.  Below the datum and the population's
//            features the luminosity PDF falls as a power of L: f = e^(g chi)
//            psi(chi) with psi bounded (g = beta + 1 for the gamma law,
//            beta + 2 for BB1).  With chi = chi_T + ln(v) / g the tail is
//            e^(g chi_T) / g times the integral over v in (0, 1] of l psi,
//            a finite interval: kTail Gauss-Legendre nodes.
// The normal-normal model's product l_i f is a normal in chi with a known
// centre m and width s: two panels [m - 12 s, m] and [m, m + 12 s].
#pragma once

#include <utility>

#include "kernels.h"

namespace hbm {

constexpr int kMargLanes = 8;

// Geometry of one object's rule: the core panels as centre and half-width in
// the core variable (F, or chi for the normal-normal model), k = ln of the
// flux-to-luminosity factor, and the tops of the graded and tail regions.
struct MargGeo {
    double c0, h0, c1, h1;
    double k;
    double xa, xt;
    double fa, ft;     // flux at chi_A and at chi_T
};

// Rules, laid out per node q (the host fills the tables):
//   core nodes    a = t, w of Gauss-Legendre on [-1, 1];
//   graded nodes  a = depth below chi_A, w = weight, e = e^-depth;
//   tail nodes    a = ln v, w = weight, on v in (0, 1].
struct MargNode {
    double a, w, e, pad;
};
struct MargRuleShape {
    static constexpr int kCore = 20, kGraded = 160, kTail = 16;
    static constexpr double kSigmas = 9.0, kClip = 0.25, kDepth = 13.0;
};
struct MargRuleProduct {
    static constexpr int kCore = 24, kGraded = 0, kTail = 0;
    static constexpr double kSigmas = 12.0;
};

template <class M>
struct Marg;

// Value of lane `lane` in every lane (lane is wave-uniform).
__device__ __forceinline__ double bcast(double v, int lane) { return lane_f64(v, lane); }

template <class M>
struct HasMarg {
    static constexpr bool value = false;
};
template <> struct HasMarg<NN1D> { static constexpr bool value = true; };
template <> struct HasMarg<LF1D> { static constexpr bool value = true; };
template <> struct HasMarg<BB1> { static constexpr bool value = true; };

// ---------------------------------------------------------------------------
// Normal-normal (Sec. 3): log l = -((y - x)/sigma)^2 / 2,
// log f = -((x - mu)/tau)^2 / 2 - ln tau - ln(2 pi)/2.
// ---------------------------------------------------------------------------
template <>
struct Marg<NN1D> {
    using R = MargRuleProduct;
    static constexpr bool kFlux = false;
    struct Th {
        double mu, itau2, lnorm, g, lng;
    };
    struct Obj {
        double y, is2;
    };
    __device__ static Th prep(const double *th)
    {
        return Th{th[0], exp(-2.0 * th[1]), th[1] + 0.5 * kLn2Pi, 0.0, 0.0};
    }
    __device__ static Obj load(const void *data, int64_t i, int64_t cap)
    {
        const double *d = static_cast<const double *>(data);
        const double s = d[cap + i];
        return Obj{d[i], 1.0 / (s * s)};
    }
    __device__ static MargGeo geo(const Obj &o, const Th &t, const Statics &)
    {
        const double prec = o.is2 + t.itau2;
        const double m = (o.y * o.is2 + t.mu * t.itau2) / prec;
        const double half = 0.5 * R::kSigmas / sqrt(prec);
        return MargGeo{m - half, half, m + half, half, 0.0, 0.0, 0.0, 0.0, 0.0};
    }
    struct Pre {};
    __device__ static Pre pre(const Obj &, const Th &, const Statics &) { return Pre{}; }
    __device__ static double logh(const Obj &o, const Pre &, double, double x, const Th &t)
    {
        const double r = o.y - x, v = x - t.mu;
        return -0.5 * (r * r) * o.is2 - 0.5 * (v * v) * t.itau2 - t.lnorm;
    }
    __device__ static double log_tail(const Obj &, const Pre &, double, double, const Th &) { return 0.0; }
    __device__ static double log_l_below(const Obj &, double, const Statics &) { return 0.0; }
    __device__ static void bcast(const Obj &o, const Pre &, Obj &oj, Pre &, int src)
    {
        oj = Obj{hbm::bcast(o.y, src), hbm::bcast(o.is2, src)};
    }
};

// ---------------------------------------------------------------------------
// Gamma luminosity function, constant flux error (Sec. 4-5):
// log l = -((Fhat - F) / sigma_F)^2 / 2, F = e^(x - k),
// log f = (beta + 1)(x - ln L*) - e^(x - ln L*) - lnGamma(beta + 1).
// The nodes know the flux F (in the core it is the variable itself), so
// e^(x - ln L*) = F e^(k - ln L*) with one exponential per object.
// ---------------------------------------------------------------------------
template <>
struct Marg<LF1D> {
    using R = MargRuleShape;
    static constexpr bool kFlux = true;
    struct Th {
        double a, lnls, lga, g, lng;
    };
    struct Obj {
        double fh, k;
    };
    struct Pre {
        double ekl;      // e^(k - ln L*)
        double isig;
    };
    __device__ static Th prep(const double *th)
    {
        const double a = th[0] + 1.0;
        return Th{a, th[1], lgamma(a), a, log(a)};
    }
    __device__ static Obj load(const void *data, int64_t i, int64_t cap)
    {
        const float *d = static_cast<const float *>(data);
        return Obj{static_cast<double>(d[i]), static_cast<double>(d[cap + i])};
    }
    __device__ static Pre pre(const Obj &o, const Th &t, const Statics &s)
    {
        return Pre{exp(o.k - t.lnls), 1.0 / s.mc[1]};
    }
    __device__ static double sigma(const Obj &, const Statics &s) { return s.mc[1]; }
    __device__ static double alpha(const Statics &) { return 0.0; }
    // ln of sup l over F <= fa (l rises with F below the datum)
    __device__ static double log_l_below(const Obj &o, double fa, const Statics &s)
    {
        const double z = (o.fh - fa) / s.mc[1];
        return -0.5 * z * z;
    }
    // log l + log f - g x at flux F and x = ln F + k
    __device__ static double log_tail(const Obj &o, const Pre &p, double flux, double, const Th &t)
    {
        const double z = (o.fh - flux) * p.isig;
        return -0.5 * z * z - t.a * t.lnls - flux * p.ekl - t.lga;
    }
    __device__ static double logh(const Obj &o, const Pre &p, double flux, double x, const Th &t)
    {
        return t.a * x + log_tail(o, p, flux, x, t);
    }
    __device__ static void bcast(const Obj &o, const Pre &p, Obj &oj, Pre &pj, int src)
    {
        oj = Obj{hbm::bcast(o.fh, src), hbm::bcast(o.k, src)};
        pj = Pre{hbm::bcast(p.ekl, src), p.isig};
    }
};

// ---------------------------------------------------------------------------
// Break-by-one luminosity function (Sec. 5, Appendix C), sigma(F) of eq 5.8:
// log l = -(Fhat - F)^2 / (2 sigma(F)^2) - ln sigma(F), F = e^(x - k),
// log f = ln C + (beta + 1)(x - ln u) + ln(1 - e^(-L/l)) - L/u.
// The break factor is written as ln(L/l) + ln phi(L/l), phi(y) = (1 - e^-y)/y,
// which stays finite however far below l the node lies; L/l and L/u are the
// flux times per-object factors.
// ---------------------------------------------------------------------------
template <>
struct Marg<BB1> {
    using R = MargRuleShape;
    static constexpr bool kFlux = true;
    struct Th {
        double b1, lnl, lnu, lnc, g, lng;
    };
    struct Obj {
        double fh, k;
    };
    struct Pre {
        double ekl, eku;     // e^(k - ln l), e^(k - ln u)
        double c0;           // ln C - (beta + 1) ln u - ln l
        double s2, a2;       // sigma0^2, alpha^2
    };
    __device__ static Th prep(const double *th)
    {
        const double g = th[0] + 2.0;
        return Th{th[0] + 1.0, th[1], th[2], bb1_ln_norm(th[0], th[1], th[2]), g, log(g)};
    }
    __device__ static Obj load(const void *data, int64_t i, int64_t cap)
    {
        const float *d = static_cast<const float *>(data);
        return Obj{static_cast<double>(d[i]), static_cast<double>(d[cap + i])};
    }
    __device__ static Pre pre(const Obj &o, const Th &t, const Statics &s)
    {
        return Pre{exp(o.k - t.lnl), exp(o.k - t.lnu), t.lnc - t.b1 * t.lnu - t.lnl, s.mc[1] * s.mc[1],
                   s.mc[2] * s.mc[2]};
    }
    __device__ static double sigma(const Obj &o, const Statics &s)
    {
        return sqrt(s.mc[1] * s.mc[1] + s.mc[2] * s.mc[2] * o.fh * o.fh);
    }
    __device__ static double alpha(const Statics &s) { return s.mc[2]; }
    // sup of l over F <= fa: the normal factor rises with F below the datum
    // and 1 / sigma(F) is at most 1 / sigma0
    __device__ static double log_l_below(const Obj &o, double fa, const Statics &s)
    {
        const double r = o.fh - fa;
        return -0.5 * (r * r) / (s.mc[1] * s.mc[1] + s.mc[2] * s.mc[2] * fa * fa) - log(s.mc[1]);
    }
    // log l + log f - (beta + 2) x; -ln sigma(F) and ln phi share one log
    // (phi lies in [e^-y, 1], far from the ends of the double range here)
    __device__ static double log_tail(const Obj &o, const Pre &p, double flux, double, const Th &)
    {
        const double var = p.s2 + p.a2 * flux * flux;
        const double r = o.fh - flux;
        const double y = flux * p.ekl;
        const double phi = y > 1e-300 ? -expm1(-y) / y : 1.0;
        return -0.5 * (r * r) / var + 0.5 * log(phi * phi / var) + p.c0 - flux * p.eku;
    }
    __device__ static double logh(const Obj &o, const Pre &p, double flux, double x, const Th &t)
    {
        return t.g * x + log_tail(o, p, flux, x, t);
    }
    __device__ static void bcast(const Obj &o, const Pre &p, Obj &oj, Pre &pj, int src)
    {
        oj = Obj{hbm::bcast(o.fh, src), hbm::bcast(o.k, src)};
        pj = Pre{hbm::bcast(p.ekl, src), hbm::bcast(p.eku, src), p.c0, p.s2, p.a2};
    }
};

// Shared geometry of the datum-centred rule.
template <class G>
__device__ __forceinline__ MargGeo datum_geo(const typename G::Obj &o, const Statics &s)
{
    using R = MargRuleShape;
    const double sig = G::sigma(o, s);
    const double fa = fmax(o.fh - R::kSigmas * sig, R::kClip * o.fh);
    const double fb = o.fh + R::kSigmas * sig / (1.0 - R::kSigmas * G::alpha(s));
    const double xa = o.k + log(fa);
    return MargGeo{0.5 * (fa + o.fh), 0.5 * (o.fh - fa), 0.5 * (o.fh + fb), 0.5 * (fb - o.fh), o.k, xa,
                   xa - R::kDepth, fa, fa * exp(-R::kDepth)};
}

template <class G>
__device__ __forceinline__ MargGeo marg_geo(const typename G::Obj &o, const typename G::Th &t, const Statics &s)
{
    if constexpr (G::kFlux) return datum_geo<G>(o, s);
    else return G::geo(o, t, s);
}

// Doubles reserved per theta row for the model's per-theta scalars (Th).
constexpr int kMargThWords = 8;

// Per-theta scalars (lnGamma, ln C ...) once per row, ahead of the main kernel.
template <class M>
__global__ void marginal_prep_kernel(const double *theta, double *th, int32_t n_theta)
{
    using G = Marg<M>;
    static_assert(sizeof(typename G::Th) <= kMargThWords * sizeof(double), "Th must fit its slot");
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_theta) return;
    *reinterpret_cast<typename G::Th *>(th + static_cast<int64_t>(j) * kMargThWords) =
        G::prep(theta + static_cast<int64_t>(j) * M::P);
}

struct MargArgs {
    const void *data;          // the context's packed data [components][cap]
    const MargNode *rule;      // per node q: see MargRuleShape / MargRuleProduct
    const double *theta;       // [n_theta][p]
    const double *th;          // [n_theta][kMargThWords]: each row's Th, from marginal_prep_kernel
    double *partials;          // [n_theta][n_blocks]
    double *terms;             // [n_theta][n] or nullptr
    const Statics *st;         // the slot's statics
    int64_t cap;
    int32_t n_blocks;
};

// Core node: log of (integrand x Jacobian) at node q of the object's core
// and its weight; the core variable is the flux for datum-centred models.
template <class G, int kRow>
__device__ __forceinline__ double core_node(const typename G::Obj &o, const typename G::Pre &p,
                                            const typename G::Th &t, const MargGeo &g, const MargNode &rq, int q,
                                            double &w)
{
    using R = typename G::R;
    const bool up = q >= R::kCore;
    const double c = up ? g.c1 : g.c0, h = up ? g.h1 : g.h0;
    w = h * rq.w;
    const double u = c + h * rq.a;
    if constexpr (G::kFlux) {
        const double lu = log(u);
        return G::logh(o, p, u, g.k + lu, t) - lu;      // dchi = dF / F
    } else {
        return G::logh(o, p, 0.0, u, t);
    }
}

template <class G, int... r>
__device__ __forceinline__ void core_rows(const typename G::Obj &o, const typename G::Pre &p, const typename G::Th &t,
                                          const MargGeo &g, const MargNode *rule, int sub, double *hv, double *wv,
                                          std::integer_sequence<int, r...>)
{
    ((hv[r] = core_node<G, r>(o, p, t, g, rule[r * kMargLanes + sub], r * kMargLanes + sub, wv[r])), ...);
}

// Node q (0-based) of the region below chi_A: graded panels, then the tail.
// On the graded panels F = F_A e^-(depth), the factor held by the table.
template <class G>
__device__ __forceinline__ double below_node(const typename G::Obj &o, const typename G::Pre &p,
                                             const typename G::Th &t, const MargGeo &g, const MargNode &rq, int q,
                                             double &w)
{
    using R = typename G::R;
    if (q < R::kGraded) {
        w = rq.w;
        return G::logh(o, p, g.fa * rq.e, g.xa - rq.a, t);
    }
    if (q < R::kGraded + R::kTail) {
        w = rq.w;
        const double d = rq.a / t.g;                    // chi - chi_T
        return G::log_tail(o, p, g.ft * exp(d), g.xt + d, t) + t.g * g.xt - t.lng;
    }
    w = 0.0;
    return -HUGE_VAL;
}

// max and sum over the kMargLanes lanes of one object (every lane gets the
// same bits: each butterfly step combines the same two values in either order)
__device__ __forceinline__ double group_max(double v)
{
#pragma unroll
    for (int d = 1; d < kMargLanes; d <<= 1) v = fmax(v, __shfl_xor(v, d, kMargLanes));
    return v;
}
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int d = 1; d < kMargLanes; d <<= 1) v += __shfl_xor(v, d, kMargLanes);
    return v;
}

// Wavefront max with the fixed DPP pattern of wave_sum; uniform result.
__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x124>(v));
    v = fmax(v, dpp_f64<0x128>(v));
    return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}

// Below chi_A the member likelihood is at most its value at F_A (times
// sigma(F_A) / sigma0 for BB1) and the population density integrates to at
// most 1 there, so that region adds at most e^(log_l_below) to the
// integral.  An object skips it when this bound is below e^-30 of its core
// integral: the log integral then changes by less than 1e-13.
constexpr double kSkipBelow = -30.0;

// grid (n_blocks, n_theta); each workgroup covers kBlock / kMargLanes objects
// of the slot for one theta and writes one FP64 partial sum of their terms.
// Core: eight lanes per object.  Region below chi_A: the objects of a
// wavefront that need it are taken one at a time by all 64 lanes, so a
// wavefront pays for the objects that need it, not for its slowest group.
template <class M>
__global__ __launch_bounds__(kBlock) void marginal_kernel(MargArgs a)
{
    using G = Marg<M>;
    using R = typename G::R;
    static_assert((2 * R::kCore) % kMargLanes == 0, "core rows must be whole");
    constexpr int kCoreRows = 2 * R::kCore / kMargLanes;
    constexpr int kBelow = R::kGraded + R::kTail, kBelowRows = (kBelow + kWave - 1) / kWave;
    __shared__ double red[1][kBlock];
    const Statics &s = *a.st;
    const int it = blockIdx.y;
    const typename G::Th t = *reinterpret_cast<const typename G::Th *>(a.th + static_cast<int64_t>(it) * kMargThWords);
    const int64_t il = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kMargLanes;
    const int sub = threadIdx.x % kMargLanes, lane = threadIdx.x % kWave;
    const bool valid = il < s.n;
    const typename G::Obj o = G::load(a.data, s.obj_start + (valid ? il : s.n - 1), a.cap);
    const MargGeo g = marg_geo<G>(o, t, s);
    const typename G::Pre p = G::pre(o, t, s);
    double m, sum;
    {
        double hv[kCoreRows], wv[kCoreRows];
        core_rows<G>(o, p, t, g, a.rule, sub, hv, wv, std::make_integer_sequence<int, kCoreRows>{});
        m = hv[0];
#pragma unroll
        for (int r = 1; r < kCoreRows; ++r) m = fmax(m, hv[r]);
        m = group_max(m);
        sum = 0.0;
        if (m > -HUGE_VAL) {
#pragma unroll
            for (int r = 0; r < kCoreRows; ++r) sum += wv[r] * exp(hv[r] - m);
        }
        sum = group_sum(sum);
    }
    if constexpr (kBelow > 0) {
        const bool need = valid && sub == 0 && !(G::log_l_below(o, g.fa, s) < m + log(sum) + kSkipBelow);
        uint64_t todo = __ballot(need);
        const MargNode *rule = a.rule + 2 * R::kCore;
        while (todo) {
            const int src = __ffsll(static_cast<unsigned long long>(todo)) - 1;
            todo &= todo - 1;
            typename G::Obj oj;
            typename G::Pre pj;
            MargGeo gj;
            G::bcast(o, p, oj, pj, src);
            gj.k = bcast(g.k, src);
            gj.xa = bcast(g.xa, src);
            gj.xt = bcast(g.xt, src);
            gj.fa = bcast(g.fa, src);
            gj.ft = bcast(g.ft, src);
            double hb[kBelowRows], wb[kBelowRows];
#pragma unroll
            for (int r = 0; r < kBelowRows; ++r) {
                const int q = r * kWave + lane;
                hb[r] = below_node<G>(oj, pj, t, gj, rule[q < kBelow ? q : 0], q, wb[r]);
            }
            double mb = hb[0];
#pragma unroll
            for (int r = 1; r < kBelowRows; ++r) mb = fmax(mb, hb[r]);
            mb = wave_max(mb);
            double sb = 0.0;
            if (mb > -HUGE_VAL) {
#pragma unroll
                for (int r = 0; r < kBelowRows; ++r) sb += wb[r] * exp(hb[r] - mb);
            }
            sb = wave_sum(sb);
            if (lane / kMargLanes == src / kMargLanes && mb > -HUGE_VAL) {
                const double mm = fmax(m, mb);
                sum = (m > -HUGE_VAL ? sum * exp(m - mm) : 0.0) + sb * exp(mb - mm);
                m = mm;
            }
        }
    }
    const double term = (m > -HUGE_VAL) ? m + log(sum) : -HUGE_VAL;
    const bool writer = valid && sub == 0;
    if (writer && a.terms) a.terms[static_cast<int64_t>(it) * s.n + il] = term;
    double v[1] = {writer ? term : 0.0};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) a.partials[static_cast<int64_t>(it) * a.n_blocks + blockIdx.x] = v[0];
}

// One workgroup per theta: the fixed-order sum of the partials, less
// N ln Z(theta) for a flux-selected catalog (the slot's selection tables).
template <class M>
__global__ __launch_bounds__(kBlock) void marginal_finish_kernel(const double *theta, const double *partials,
                                                                 int32_t n_blocks, const Statics *st, const double *qx,
                                                                 const double *qw, const double *qeps, int32_t nq,
                                                                 double *out)
{
    __shared__ double red[1][kBlock];
    const int it = blockIdx.x;
    double lz = 0.0;
    if constexpr (M::kSelection) {
        const double *th = theta + static_cast<int64_t>(it) * M::P;
        double ag[2], zc[4];
        M::aux(th, ag);
        M::z_consts(th, zc);
        lz = block_log_z<M>(zc, qx, qw, qeps, nq, red) - M::logz_shift(ag);
        __syncthreads();
    }
    double v[1] = {0.0};
    const double *p = partials + static_cast<int64_t>(it) * n_blocks;
    for (int j = threadIdx.x; j < n_blocks; j += kBlock) v[0] += p[j];
    block_sum<1>(v, red);
    if (threadIdx.x == 0) out[it] = v[0] - static_cast<double>(st->n) * lz;
}

}  // namespace hbm
