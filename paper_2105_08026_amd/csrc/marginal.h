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
};

// Rules, laid out per node q (the host fills the tables):
//   core nodes    (t, w) of Gauss-Legendre on [-1, 1];
//   graded nodes  (depth below chi_A, weight);
//   tail nodes    (ln v, weight) on v in (0, 1].
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
        return MargGeo{m - half, half, m + half, half, 0.0, 0.0, 0.0};
    }
    __device__ static double logh(const Obj &o, double x, const Th &t, const Statics &)
    {
        const double r = o.y - x, v = x - t.mu;
        return -0.5 * (r * r) * o.is2 - 0.5 * (v * v) * t.itau2 - t.lnorm;
    }
    __device__ static double log_tail(const Obj &, double, const Th &, const Statics &) { return 0.0; }
};

// ---------------------------------------------------------------------------
// Gamma luminosity function, constant flux error (Sec. 4-5):
// log l = -((Fhat - e^(x - k)) / sigma_F)^2 / 2,
// log f = (beta + 1)(x - ln L*) - e^(x - ln L*) - lnGamma(beta + 1).
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
    __device__ static double sigma(const Obj &, const Statics &s) { return s.mc[1]; }
    __device__ static double alpha(const Statics &) { return 0.0; }
    __device__ static double log_meas(const Obj &o, double x, const Statics &s)
    {
        const double z = (o.fh - exp(x - o.k)) / s.mc[1];
        return -0.5 * z * z;
    }
    __device__ static double logh(const Obj &o, double x, const Th &t, const Statics &s)
    {
        const double q = x - t.lnls;
        return log_meas(o, x, s) + t.a * q - exp(q) - t.lga;
    }
    // log l + log f - g x
    __device__ static double log_tail(const Obj &o, double x, const Th &t, const Statics &s)
    {
        return log_meas(o, x, s) - t.a * t.lnls - exp(x - t.lnls) - t.lga;
    }
};

// ---------------------------------------------------------------------------
// Break-by-one luminosity function (Sec. 5, Appendix C), sigma(F) of eq 5.8:
// log l = -(Fhat - F)^2 / (2 sigma(F)^2) - ln sigma(F), F = e^(x - k),
// log f = ln C + (beta + 1)(x - ln u) + ln(1 - e^(-L/l)) - L/u.
// The break factor is written as ln(L/l) + ln phi(L/l), phi(y) = (1 - e^-y)/y,
// which stays finite however far below l the node lies.
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
    __device__ static double sigma(const Obj &o, const Statics &s)
    {
        return sqrt(s.mc[1] * s.mc[1] + s.mc[2] * s.mc[2] * o.fh * o.fh);
    }
    __device__ static double alpha(const Statics &s) { return s.mc[2]; }
    __device__ static double log_meas(const Obj &o, double x, const Statics &s)
    {
        const double flux = exp(x - o.k);
        const double var = s.mc[1] * s.mc[1] + s.mc[2] * s.mc[2] * flux * flux;
        const double r = o.fh - flux;
        return -0.5 * (r * r) / var - 0.5 * log(var);
    }
    __device__ static double log_phi(double y)
    {
        return y > 1e-300 ? log(-expm1(-y) / y) : 0.0;
    }
    // log f - (beta + 2) x
    __device__ static double log_psi(double x, const Th &t)
    {
        return t.lnc - t.b1 * t.lnu - t.lnl + log_phi(exp(x - t.lnl)) - exp(x - t.lnu);
    }
    __device__ static double logh(const Obj &o, double x, const Th &t, const Statics &s)
    {
        return log_meas(o, x, s) + t.g * x + log_psi(x, t);
    }
    __device__ static double log_tail(const Obj &o, double x, const Th &t, const Statics &s)
    {
        return log_meas(o, x, s) + log_psi(x, t);
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
                   xa - R::kDepth};
}

template <class G>
__device__ __forceinline__ MargGeo marg_geo(const typename G::Obj &o, const typename G::Th &t, const Statics &s)
{
    if constexpr (G::kFlux) return datum_geo<G>(o, s);
    else return G::geo(o, t, s);
}

struct MargArgs {
    const void *data;          // the context's packed data [components][cap]
    const double2 *rule;       // per node q: see MargRuleShape / MargRuleProduct
    const double *theta;       // [n_theta][p]
    double *partials;          // [n_theta][n_blocks]
    double *terms;             // [n_theta][n] or nullptr
    const Statics *st;         // the slot's statics
    int64_t cap;
    int32_t n_blocks;
};

// Node value: log of (integrand x Jacobian) at node q, and its weight.
template <class G, int kRow>
__device__ __forceinline__ double marg_node(const typename G::Obj &o, const typename G::Th &t, const Statics &s,
                                            const MargGeo &g, double2 rq, int q, double &w)
{
    using R = typename G::R;
    constexpr int q0 = kRow * kMargLanes;
    if constexpr (q0 < 2 * R::kCore) {
        const bool up = q >= R::kCore;
        const double c = up ? g.c1 : g.c0, h = up ? g.h1 : g.h0;
        w = h * rq.y;
        const double u = c + h * rq.x;
        if constexpr (G::kFlux) {
            const double lu = log(u);
            return G::logh(o, g.k + lu, t, s) - lu;      // dchi = dF / F
        } else {
            return G::logh(o, u, t, s);
        }
    } else if constexpr (q0 < 2 * R::kCore + R::kGraded) {
        w = rq.y;
        return G::logh(o, g.xa - rq.x, t, s);
    } else {
        w = rq.y;
        return G::log_tail(o, g.xt + rq.x / t.g, t, s) + t.g * g.xt - t.lng;
    }
}

template <class G, int... r>
__device__ __forceinline__ void marg_rows(const typename G::Obj &o, const typename G::Th &t, const Statics &s,
                                          const MargGeo &g, const double2 *rule, int sub, double *hv, double *wv,
                                          std::integer_sequence<int, r...>)
{
    ((hv[r] = marg_node<G, r>(o, t, s, g, rule[r * kMargLanes + sub], r * kMargLanes + sub, wv[r])), ...);
}

// grid (n_blocks, n_theta); each workgroup covers kBlock / kMargLanes objects
// of the slot for one theta and writes one FP64 partial sum of their terms.
template <class M>
__global__ __launch_bounds__(kBlock) void marginal_kernel(MargArgs a)
{
    using G = Marg<M>;
    using R = typename G::R;
    constexpr int kNodes = 2 * R::kCore + R::kGraded + R::kTail;
    static_assert(kNodes % kMargLanes == 0 && (2 * R::kCore) % kMargLanes == 0 && R::kGraded % kMargLanes == 0,
                  "every row of nodes must lie in one region");
    constexpr int kRows = kNodes / kMargLanes;
    __shared__ double red[1][kWavesPerBlock];
    const Statics &s = *a.st;
    const int it = blockIdx.y;
    const typename G::Th t = G::prep(a.theta + static_cast<int64_t>(it) * M::P);
    const int64_t il = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kMargLanes;
    const int sub = threadIdx.x % kMargLanes;
    const bool valid = il < s.n;
    const typename G::Obj o = G::load(a.data, s.obj_start + (valid ? il : s.n - 1), a.cap);
    const MargGeo g = marg_geo<G>(o, t, s);
    double hv[kRows], wv[kRows];
    marg_rows<G>(o, t, s, g, a.rule, sub, hv, wv, std::make_integer_sequence<int, kRows>{});
    double m = hv[0];
#pragma unroll
    for (int r = 1; r < kRows; ++r) m = fmax(m, hv[r]);
#pragma unroll
    for (int d = 1; d < kMargLanes; d <<= 1) m = fmax(m, __shfl_xor(m, d, kMargLanes));
    double sum = 0.0;
    if (m > -HUGE_VAL) {
#pragma unroll
        for (int r = 0; r < kRows; ++r) sum += wv[r] * exp(hv[r] - m);
    }
#pragma unroll
    for (int d = 1; d < kMargLanes; d <<= 1) sum += __shfl_xor(sum, d, kMargLanes);
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
    __shared__ double red[1][kWavesPerBlock];
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
