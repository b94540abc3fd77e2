// Per-model arithmetic of the sampler: the member likelihood l_i (Sec. 2.1)
// and the population density f(chi; theta) in latent coordinates, the prior
// on theta, and the constants each sweep derives from (theta, theta').
//
// Single-precision models are written around per-object centres so that the
// float arithmetic keeps ~1e-7 relative accuracy in the log densities even
// for bright objects whose likelihood is a thousandth wide in ln L:
//   * the data are re-expressed once (in FP64) as a centre c_i in float plus
//     its rounding residual e_i, so ln(F / Fhat) = (chi - c_i) - e_i is formed
//     from an exact float difference and a tiny correction, and the flux
//     residual is -(Fhat / sigma) expm1(...);
//   * ln L* is split into a float head and tail, so chi - ln L* is accurate;
//   * the change of log f between theta and theta' is formed from parameter
//     differences, never as a difference of two sums; the part of it that is
//     the same for every object is added once, N times, in FP64.
//
// Hooks every model provides (all FP64 unless noted):
//   aux(th, a)          the expensive per-theta scalars (lnGamma, ln s), NAUX of them
//   in_support(th)      prior support
//   log_prior(th)       log prior density in the theta coordinates
//   derive_kc(th, tp, a, s, kc)  per-sweep constants in the per-object precision
//                       from the current theta (with its aux a) and the proposal tp
//   dlf_const(th, tp, a, ap)     minus the object-independent part of
//                       log f(chi; tp) - log f(chi; th), subtracted N times
//   z_consts(tp, zc), logz_shift(ap)  quadrature constants of ln Z; the
//                       quadrature sum omits exp(-shift) and the shift is
//                       subtracted afterwards
//   zlog(zc, x)         (selection models) log of the luminosity PDF in
//                       x = ln L without its normaliser, from z_consts
//   quad_interval, edge_area, detect  (selection models) the ln L range of
//                       the selection quadrature, 4 pi rmax^2 in the data's
//                       units, and the detection efficiency of a flux
//   eval, dlf           per-object log densities and the per-object part of
//                       the log f change, in the per-object precision
//   NS, stats, stats_dlf (exponential-family models) NS per-object
//                       sufficient statistics at the current theta theta0,
//                       and sum_i log f(chi_i; tp) - sum_i log f(chi_i; theta0)
//                       from their FP64 sums (NS = 0: no such statistics)
#pragma once

#include "device.h"

namespace hbm {

constexpr double kLn2Pi = 1.8378770664093454836;
constexpr double kLn4Pi = 2.5310242469692907930;

template <typename T> __device__ __forceinline__ T *kc_of(CycleState *c);
template <> __device__ __forceinline__ float *kc_of<float>(CycleState *c) { return c->kc_f; }
template <> __device__ __forceinline__ double *kc_of<double>(CycleState *c) { return c->kc_d; }

template <typename T>
struct Eval {
    T lpv;   // log pi up to terms shared by X and Y (used for the accept ratio)
    T lp;    // log l_i + log f with the constants of the documented densities
    T lf;    // log f(chi; theta)
    T q;     // model scratch reused by dlf
    T eq;
    T res;
    T u;
};

// ===========================================================================
// Heteroscedastic 1-D normal-normal (Sec. 3), FP64.
//   log l_i(x) = -((y_i - x) / sigma_i)^2 / 2
//   log f(x)   = -((x - mu) / tau)^2 / 2 - ln tau - ln(2 pi) / 2
//   theta = (mu, ln tau); prior density in (mu, ln tau) is tau.
// ===========================================================================
struct NN1D {
    using T = double;
    static constexpr int D = 1, NC = 1, M = 2, MD = 2, P = 2, MODEL = 1;
    static constexpr bool kSelection = false;
    struct Obj {
        double y, is;
    };

    __device__ static void derive_statics(Statics &) {}
    __device__ static void derive_obj(const T *data, T *dd, int64_t i, int64_t n, const Statics &)
    {
        dd[i] = data[i];
        dd[n + i] = 1.0 / data[n + i];
    }
    __device__ static Obj load(const T *dd, int64_t i, int64_t n) { return Obj{dd[i], dd[n + i]}; }
    __device__ static void aux(const double *, double *a) { a[0] = a[1] = 0.0; }
    __device__ static bool in_support(const double *) { return true; }
    __device__ static double log_prior(const double *th) { return th[1]; }
    __device__ static void z_consts(const double *, double *zc) { zc[0] = zc[1] = 0.0; }
    __device__ static double logz_shift(const double *) { return 0.0; }
    __device__ static double dlf_const(const double *, const double *, const double *, const double *) { return 0.0; }
    // kc: [0] mu, [1] 1/tau, [2] ln tau + ln(2 pi)/2, [3..5] the same for theta'
    __device__ static void derive_kc(const double *th, const double *tp, const double *, const Statics &, T *kc)
    {
        kc[0] = th[0];
        kc[1] = exp(-th[1]);
        kc[2] = th[1] + 0.5 * kLn2Pi;
        kc[3] = tp[0];
        kc[4] = exp(-tp[1]);
        kc[5] = tp[1] + 0.5 * kLn2Pi;
    }
    __device__ static Eval<T> eval(const Obj &o, const T *x, const T *kc, const Statics &)
    {
        Eval<T> e;
        const T rm = (o.y - x[0]) * o.is;
        const T dv = (x[0] - kc[0]) * kc[1];
        e.lf = -0.5 * dv * dv - kc[2];
        e.lp = -0.5 * rm * rm + e.lf;
        e.lpv = e.lp;
        e.q = e.eq = e.res = e.u = 0;
        return e;
    }
    __device__ static T dlf(const Obj &, const T *x, const Eval<T> &e, const T *kc, const Statics &)
    {
        const T dv = (x[0] - kc[3]) * kc[4];
        return (-0.5 * dv * dv - kc[5]) - e.lf;
    }
    // d = chi - mu0: sum d, sum d^2; sum (chi - mu)^2 = S2 + 2 (mu0 - mu) S1 + N (mu0 - mu)^2
    static constexpr int NS = 2;
    __device__ static void stats(const Obj &, const T *x, const Eval<T> &, const T *kc, const Statics &, T *out)
    {
        const T d = x[0] - kc[0];
        out[0] = d;
        out[1] = d * d;
    }
    __device__ static double stats_dlf(const double *t0, const double *tp, const double *, const double *,
                                       const double *sv, double n, const Statics &)
    {
        const double dm = t0[0] - tp[0];
        const double ssp = sv[1] + 2.0 * dm * sv[0] + n * dm * dm;
        return -0.5 * ssp * exp(-2.0 * tp[1]) + 0.5 * sv[1] * exp(-2.0 * t0[1]) - n * (tp[1] - t0[1]);
    }
};

// ===========================================================================
// The paper's correlated 3-D normal-normal (Sec. 3), FP64.
//   log l_i(x) = -sum_j ((y_ij - x_j) / sigma_j)^2 / 2
//   log f(x)   = log MVN(x; mu, C_pop);  theta = mu, flat prior.
// Statics md: [0..5] packed C_pop^-1, [6] log normaliser, [7..9] 1/sigma_j.
// ===========================================================================
struct NN3D {
    using T = double;
    static constexpr int D = 3, NC = 6, M = 3, MD = 3, P = 3, MODEL = 4;
    static constexpr bool kSelection = false;
    struct Obj {
        double y[3];
    };

    __device__ static void derive_statics(Statics &s)
    {
        // Cholesky C = G G^T of the packed covariance, then C^-1 = G^-T G^-1.
        const double *c = s.mc;
        double g00 = sqrt(c[0]);
        double g10 = c[1] / g00, g11 = sqrt(c[2] - g10 * g10);
        double g20 = c[3] / g00, g21 = (c[4] - g20 * g10) / g11;
        double g22 = sqrt(c[5] - g20 * g20 - g21 * g21);
        // H = G^-1 (lower)
        double h00 = 1.0 / g00, h11 = 1.0 / g11, h22 = 1.0 / g22;
        double h10 = -g10 * h00 * h11;
        double h21 = -g21 * h11 * h22;
        double h20 = -(g20 * h00 + g21 * h10) * h22;
        // C^-1 = H^T H, packed lower
        s.md[0] = h00 * h00 + h10 * h10 + h20 * h20;
        s.md[1] = h11 * h10 + h21 * h20;
        s.md[2] = h11 * h11 + h21 * h21;
        s.md[3] = h22 * h20;
        s.md[4] = h22 * h21;
        s.md[5] = h22 * h22;
        s.md[6] = 1.5 * kLn2Pi + log(g00) + log(g11) + log(g22);
        for (int j = 0; j < 3; ++j) s.md[7 + j] = 1.0 / c[6 + j];
    }
    __device__ static void derive_obj(const T *data, T *dd, int64_t i, int64_t n, const Statics &)
    {
        for (int j = 0; j < 3; ++j) dd[j * n + i] = data[j * n + i];
    }
    __device__ static Obj load(const T *dd, int64_t i, int64_t n) { return Obj{{dd[i], dd[n + i], dd[2 * n + i]}}; }
    __device__ static void aux(const double *, double *a) { a[0] = a[1] = 0.0; }
    __device__ static bool in_support(const double *) { return true; }
    __device__ static double log_prior(const double *) { return 0.0; }
    __device__ static void z_consts(const double *, double *zc) { zc[0] = zc[1] = 0.0; }
    __device__ static double logz_shift(const double *) { return 0.0; }
    __device__ static double dlf_const(const double *, const double *, const double *, const double *) { return 0.0; }
    __device__ static void derive_kc(const double *th, const double *tp, const double *, const Statics &, T *kc)
    {
        for (int j = 0; j < 3; ++j) {
            kc[j] = th[j];
            kc[3 + j] = tp[j];
        }
    }
    __device__ static double quad(const Statics &s, double d0, double d1, double d2)
    {
        const double *w = s.md;
        return w[0] * d0 * d0 + w[2] * d1 * d1 + w[5] * d2 * d2 + 2.0 * (w[1] * d1 * d0 + w[3] * d2 * d0 + w[4] * d2 * d1);
    }
    __device__ static Eval<T> eval(const Obj &o, const T *x, const T *kc, const Statics &s)
    {
        Eval<T> e;
        double lm = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double r = (o.y[j] - x[j]) * s.md[7 + j];
            lm += -0.5 * r * r;
        }
        e.lf = -0.5 * quad(s, x[0] - kc[0], x[1] - kc[1], x[2] - kc[2]) - s.md[6];
        e.lp = lm + e.lf;
        e.lpv = e.lp;
        e.q = e.eq = e.res = e.u = 0;
        return e;
    }
    __device__ static T dlf(const Obj &, const T *x, const Eval<T> &e, const T *kc, const Statics &s)
    {
        return (-0.5 * quad(s, x[0] - kc[3], x[1] - kc[4], x[2] - kc[5]) - s.md[6]) - e.lf;
    }
    // d = chi - mu0 (3 sums); with delta = mu0 - mu the change of sum log f is
    // -delta^T C^-1 sum d - N delta^T C^-1 delta / 2
    static constexpr int NS = 3;
    __device__ static void stats(const Obj &, const T *x, const Eval<T> &, const T *kc, const Statics &, T *out)
    {
        for (int j = 0; j < 3; ++j) out[j] = x[j] - kc[j];
    }
    __device__ static double stats_dlf(const double *t0, const double *tp, const double *, const double *,
                                       const double *sv, double n, const Statics &s)
    {
        const double d0 = t0[0] - tp[0], d1 = t0[1] - tp[1], d2 = t0[2] - tp[2];
        const double *w = s.md;
        const double g0 = w[0] * d0 + w[1] * d1 + w[3] * d2;      // C^-1 delta
        const double g1 = w[1] * d0 + w[2] * d1 + w[4] * d2;
        const double g2 = w[3] * d0 + w[4] * d1 + w[5] * d2;
        return -(g0 * sv[0] + g1 * sv[1] + g2 * sv[2]) - 0.5 * n * (g0 * d0 + g1 * d1 + g2 * d2);
    }
};

// ---------------------------------------------------------------------------
// Shared pieces of the luminosity-function models (Sec. 4-5, Appendix B).
// The luminosity PDF is the gamma law of shape beta + 1 and scale L* (the
// BB1 model as l -> 0); in chi = ln L it reads
//   log f(chi) = (beta + 1)(chi - ln L*) - exp(chi - ln L*) - lnGamma(beta + 1).
// kc: [0] beta + 1, [1] float head of ln L*, [2] its tail, [3] lnGamma(beta+1),
//     [4] beta' - beta, [5] expm1(ln L* - ln L*').
// With q = chi - ln L*, log f' - log f = (beta' - beta) q - e^q [5] - C where
// C = (beta' + 1)(ln L*' - ln L*) + lnGamma(beta'+1) - lnGamma(beta+1) is the
// object-independent part.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gamma_kc(const double *th, const double *tp, double lg, float *kc)
{
    const float head = static_cast<float>(th[1]);
    kc[0] = static_cast<float>(th[0] + 1.0);
    kc[1] = head;
    kc[2] = static_cast<float>(th[1] - static_cast<double>(head));
    kc[3] = static_cast<float>(lg);
    kc[4] = static_cast<float>(tp[0] - th[0]);
    // single precision suffices: the factor multiplies a float per-object term
    kc[5] = expm1f(static_cast<float>(th[1] - tp[1]));
}

__device__ __forceinline__ double gamma_dconst(const double *th, const double *tp, const double *a, const double *ap)
{
    return (tp[0] + 1.0) * (tp[1] - th[1]) + (ap[0] - a[0]);
}

__device__ __forceinline__ bool lf_beta_ok(double beta) { return beta > -1.0 && beta < 0.0; }

// Change of sum_i log f of the gamma law from theta0 to tp, from the sums
// Sq = sum (chi - ln L*0) and Se = sum e^(chi - ln L*0) (lnGamma in a0, ap):
// (beta' - beta0) Sq + (beta' + 1) N (ln L*0 - ln L*') - expm1(ln L*0 - ln L*') Se
// - N (lnGamma(beta' + 1) - lnGamma(beta0 + 1)).
__device__ __forceinline__ double gamma_stats_dlf(const double *t0, const double *tp, const double *a0,
                                                  const double *ap, double sq, double se, double n)
{
    const double dl = t0[1] - tp[1];
    return (tp[0] - t0[0]) * sq + (tp[0] + 1.0) * n * dl - expm1(dl) * se - n * (ap[0] - a0[0]);
}

// ===========================================================================
// Gamma luminosity function, flux-limited, known distances; chi = ln L.
//   log l_i(chi) = -((Fhat_i - exp(chi - k_i)) / sigma_F)^2 / 2,  k_i = ln 4 pi r_i^2.
// Derived data per object: a = Fhat / sigma_F, centre c = ln(4 pi r^2 Fhat)
// rounded to float, and e = (exact centre) - c.
// aux: [0] lnGamma(beta + 1).
// ===========================================================================
struct LF1D {
    using T = float;
    static constexpr int D = 1, NC = 1, M = 2, MD = 3, P = 2, MODEL = 2;
    static constexpr bool kSelection = true;
    struct Obj {
        float a, c, e;
    };

    __device__ static void derive_statics(Statics &) {}
    __device__ static void derive_obj(const T *data, T *dd, int64_t i, int64_t n, const Statics &s)
    {
        const double fhat = data[i], k = data[n + i];
        const double centre = k + log(fhat);
        const float c = static_cast<float>(centre);
        dd[i] = static_cast<float>(fhat / s.mc[1]);
        dd[n + i] = c;
        dd[2 * n + i] = static_cast<float>(centre - static_cast<double>(c));
    }
    __device__ static Obj load(const T *dd, int64_t i, int64_t n) { return Obj{dd[i], dd[n + i], dd[2 * n + i]}; }
    __device__ static void aux(const double *th, double *a)
    {
        a[0] = lgamma(th[0] + 1.0);
        a[1] = 0.0;
    }
    __device__ static bool in_support(const double *th) { return lf_beta_ok(th[0]); }
    // truncated Cauchy on the slope, flat in ln L*
    __device__ static double log_prior(const double *th) { return in_support(th) ? -log1p(th[0] * th[0]) : -HUGE_VAL; }
    __device__ static void z_consts(const double *tp, double *zc)
    {
        zc[0] = tp[0] + 1.0;
        zc[1] = tp[1];
    }
    __device__ static double logz_shift(const double *ap) { return ap[0]; }
    __device__ static double zlog(const double *zc, double x)
    {
        const double t = x - zc[1];
        return zc[0] * t - exp(t);
    }
    // ln L from 30 e-folds below the reference ln L0 to 40 L0
    __device__ static void quad_interval(const Statics &s, double *lo, double *hi)
    {
        *lo = s.mc[3] - 30.0;
        *hi = s.mc[3] + log(40.0);
    }
    __device__ static double edge_area(const Statics &s) { return 4.0 * 3.14159265358979323846 * s.mc[2] * s.mc[2]; }
    // eta(F) = Phi((F - F_th) / sigma_F)
    __device__ static double detect(double flux, const Statics &s)
    {
        return 0.5 * erfc(-(flux - s.mc[0]) / (s.mc[1] * 1.4142135623730950488));
    }
    __device__ static double dlf_const(const double *th, const double *tp, const double *a, const double *ap)
    {
        return gamma_dconst(th, tp, a, ap);
    }
    __device__ static void derive_kc(const double *th, const double *tp, const double *a, const Statics &, T *kc)
    {
        gamma_kc(th, tp, a[0], kc);
    }
    __device__ static Eval<T> eval(const Obj &o, const T *x, const T *kc, const Statics &)
    {
        Eval<T> e;
        e.q = (x[0] - kc[1]) - kc[2];
        e.eq = exp_fin(e.q);
        const float z = -o.a * expm1_fin((x[0] - o.c) - o.e);
        const float lm = -0.5f * z * z;
        const float g = kc[0] * e.q - e.eq;
        e.lpv = lm + g;
        e.lf = g - kc[3];
        e.lp = lm + e.lf;
        e.res = e.u = 0.0f;
        return e;
    }
    __device__ static T dlf(const Obj &, const T *, const Eval<T> &e, const T *kc, const Statics &)
    {
        return kc[4] * e.q - e.eq * kc[5];
    }
    // q = chi - ln L*0 and e^q, as the density evaluation has them
    static constexpr int NS = 2;
    __device__ static void stats(const Obj &, const T *, const Eval<T> &e, const T *, const Statics &, T *out)
    {
        out[0] = e.q;
        out[1] = e.eq;
    }
    __device__ static double stats_dlf(const double *t0, const double *tp, const double *a0, const double *ap,
                                       const double *sv, double n, const Statics &)
    {
        return gamma_stats_dlf(t0, tp, a0, ap, sv[0], sv[1], n);
    }
};

// ===========================================================================
// Gamma luminosity function with measured distance and colour; chi = (ln L, ln r, c).
//   log l_i = -(zF^2 + zr^2 + zc^2) / 2 with
//     zF = (Fhat - L / 4 pi r^2) / sigma_F, zr = (rhat - r) / (f_r rhat), zc = (chat - c) / sigma_c
//   log f = gamma term + ln(3 r^3 / rmax^3) [ln r <= ln rmax, else -inf]
//           - ((c - a - b ln L) / s)^2 / 2 - ln s - ln(2 pi) / 2
// Derived data: a = Fhat / sigma_F, c1 = centre of ln L, e1 its residual
// against ln 4 pi + 2 c2 + ln Fhat, c2 = ln rhat in float, e2 its residual, chat.
// Statics mf: [0] 1/f_r, [1] 1/sigma_c, [2] ln rmax, [3] ln 3 - 3 ln rmax.
// aux: [0] lnGamma(beta + 1), [1] ln s.
// kc beyond the gamma part: [7] a, [8] b, [9] 1/s, [10] ln s + ln(2 pi)/2,
//   [11] a' - a, [12] b' - b, [13] 1/s' - 1/s, [14] 1/s'.
// The colour term's object-independent change is -ln(s'/s).
// ===========================================================================
struct LF3D {
    using T = float;
    static constexpr int D = 3, NC = 6, M = 3, MD = 6, P = 5, MODEL = 3;
    static constexpr bool kSelection = true;
    struct Obj {
        float a, c1, e1, c2, e2, ch;
    };

    __device__ static void derive_statics(Statics &s)
    {
        s.mf[0] = static_cast<float>(1.0 / s.mc[4]);
        s.mf[1] = static_cast<float>(1.0 / s.mc[5]);
        s.mf[2] = static_cast<float>(log(s.mc[2]));
        s.mf[3] = static_cast<float>(log(3.0) - 3.0 * log(s.mc[2]));
    }
    __device__ static void derive_obj(const T *data, T *dd, int64_t i, int64_t n, const Statics &s)
    {
        const double fhat = data[i], rhat = data[n + i], chat = data[2 * n + i];
        const double lr = log(rhat);
        const float c2 = static_cast<float>(lr);
        const double centre = kLn4Pi + 2.0 * lr + log(fhat);
        const float c1 = static_cast<float>(centre);
        dd[i] = static_cast<float>(fhat / s.mc[1]);
        dd[n + i] = c1;
        dd[2 * n + i] = static_cast<float>(kLn4Pi + 2.0 * static_cast<double>(c2) + log(fhat) - static_cast<double>(c1));
        dd[3 * n + i] = c2;
        dd[4 * n + i] = static_cast<float>(lr - static_cast<double>(c2));
        dd[5 * n + i] = static_cast<float>(chat);
    }
    __device__ static Obj load(const T *dd, int64_t i, int64_t n)
    {
        return Obj{dd[i], dd[n + i], dd[2 * n + i], dd[3 * n + i], dd[4 * n + i], dd[5 * n + i]};
    }
    __device__ static void aux(const double *th, double *a)
    {
        a[0] = lgamma(th[0] + 1.0);
        a[1] = log(th[4]);
    }
    __device__ static bool in_support(const double *th) { return lf_beta_ok(th[0]) && th[4] > 0.0; }
    // as 1-D, plus flat a and b and a uniform s > 0
    __device__ static double log_prior(const double *th) { return in_support(th) ? -log1p(th[0] * th[0]) : -HUGE_VAL; }
    __device__ static void z_consts(const double *tp, double *zc) { LF1D::z_consts(tp, zc); }
    __device__ static double logz_shift(const double *ap) { return ap[0]; }
    __device__ static double zlog(const double *zc, double x) { return LF1D::zlog(zc, x); }
    __device__ static void quad_interval(const Statics &s, double *lo, double *hi) { LF1D::quad_interval(s, lo, hi); }
    __device__ static double edge_area(const Statics &s) { return LF1D::edge_area(s); }
    __device__ static double detect(double flux, const Statics &s) { return LF1D::detect(flux, s); }
    __device__ static double dlf_const(const double *th, const double *tp, const double *a, const double *ap)
    {
        return gamma_dconst(th, tp, a, ap) + (ap[1] - a[1]);
    }
    __device__ static void derive_kc(const double *th, const double *tp, const double *a, const Statics &, T *kc)
    {
        gamma_kc(th, tp, a[0], kc);
        kc[7] = static_cast<float>(th[2]);
        kc[8] = static_cast<float>(th[3]);
        kc[9] = static_cast<float>(1.0 / th[4]);
        kc[10] = static_cast<float>(a[1] + 0.5 * kLn2Pi);
        kc[11] = static_cast<float>(tp[2] - th[2]);
        kc[12] = static_cast<float>(tp[3] - th[3]);
        kc[13] = static_cast<float>(1.0 / tp[4] - 1.0 / th[4]);
        kc[14] = static_cast<float>(1.0 / tp[4]);
    }
    __device__ static Eval<T> eval(const Obj &o, const T *x, const T *kc, const Statics &s)
    {
        Eval<T> e;
        e.q = (x[0] - kc[1]) - kc[2];
        e.eq = exp_fin(e.q);
        const float d0 = x[0] - o.c1, d1 = x[1] - o.c2;
        const float zF = -o.a * expm1_fin((d0 - 2.0f * d1) - o.e1);
        const float zr = -s.mf[0] * expm1_fin(d1 - o.e2);
        const float zc = (x[2] - o.ch) * s.mf[1];
        const float lm = -0.5f * (zF * zF + zr * zr + zc * zc);
        // colour residual c - a - b ln L around the object's centre: the
        // rounding of the per-object constant is shared by X and Y.
        const float kres = (o.ch - kc[7]) - kc[8] * o.c1;
        e.res = ((x[2] - o.ch) + kres) - kc[8] * d0;
        e.u = e.res * kc[9];
        const float g = kc[0] * e.q - e.eq;
        const float col = -0.5f * e.u * e.u;
        const bool inside = x[1] <= s.mf[2];
        e.lpv = inside ? lm + g + 3.0f * d1 + col : -HUGE_VALF;
        e.lf = inside ? g - kc[3] + (3.0f * x[1] + s.mf[3]) + col - kc[10] : -HUGE_VALF;
        e.lp = lm + e.lf;
        return e;
    }
    __device__ static T dlf(const Obj &, const T *x, const Eval<T> &e, const T *kc, const Statics &)
    {
        const float dg = kc[4] * e.q - e.eq * kc[5];
        const float du = e.res * kc[13] - (kc[11] + kc[12] * x[0]) * kc[14];
        return dg - 0.5f * du * (2.0f * e.u + du);
    }
    // gamma part: q = chi_1 - ln L*0, e^q; colour part: r = c - a0 - b0 chi_1,
    // r^2, r q, q^2.  With A = (a0 - a') + (b0 - b') ln L*0, B = b0 - b':
    // sum (c - a' - b' chi_1)^2 = Sr2 + 2A Sr + 2B Srq + N A^2 + 2AB Sq + B^2 Sq2.
    // a0 and b0 are the single-precision values the sweep formed r with
    // (their rounding would otherwise enter N times).
    static constexpr int NS = 6;
    __device__ static void stats(const Obj &, const T *, const Eval<T> &e, const T *, const Statics &, T *out)
    {
        out[0] = e.q;
        out[1] = e.eq;
        out[2] = e.res;
        out[3] = e.res * e.res;
        out[4] = e.res * e.q;
        out[5] = e.q * e.q;
    }
    __device__ static double stats_dlf(const double *t0, const double *tp, const double *a0, const double *ap,
                                       const double *sv, double n, const Statics &)
    {
        const double af = static_cast<float>(t0[2]), bf = static_cast<float>(t0[3]);
        const double A = (af - tp[2]) + (bf - tp[3]) * t0[1], B = bf - tp[3];
        const double ssp = sv[3] + 2.0 * A * sv[2] + 2.0 * B * sv[4] + n * A * A + 2.0 * A * B * sv[0] + B * B * sv[5];
        const double dcol = -0.5 * ssp / (tp[4] * tp[4]) + 0.5 * sv[3] / (t0[4] * t0[4]) - n * (ap[1] - a0[1]);
        return gamma_stats_dlf(t0, tp, a0, ap, sv[0], sv[1], n) + dcol;
    }
};

// ===========================================================================
// Break-by-one luminosity function (Sec. 5, Appendix C), flux-limited, known
// distances; chi = ln L; theta = (beta, ln l, ln u).  Units: L in units of a
// reference scale, distances in units of rmax, F = L / r^2, so k_i = ln r_i^2.
//   f(L) = C / u (1 - e^{-L/l}) (L/u)^beta e^{-L/u},
//   C = 1 / (Gamma(beta + 1) (1 - (1 + u/l)^-(beta+1))), or 1 / ln(1 + u/l) at beta = -1;
//   log f in chi: ln C + (beta + 1)(chi - ln u) + ln(1 - e^{-L/l}) - e^{chi - ln u}.
//   log l_i(chi) = -z^2 / 2 - ln sigma(F), z = (Fhat - F) / sigma(F),
//   sigma(F) = sqrt(sigma0^2 + (alpha F)^2)  (the sampling density of Fhat, eq 5.8).
// Prior: -2 < beta < 0 truncated Cauchy, flat in l, flat in ln u, l < u; as
// a density in (beta, ln l, ln u) that is l / (1 + beta^2) (eq 5.5).
// Derived data per object: Fhat, centre c = ln(r^2 Fhat) in float and its
// residual e.  Statics mc: [0] F_th, [1] sigma0, [2] alpha, [3] ln l and
// [4] ln u of the reference PDF (they fix the quadrature range); mf:
// [0] sigma0^2, [1] alpha^2.  aux: [0] ln C.
// kc: [0] beta + 1, [1] ln u head, [2] its tail, [3] ln l head, [4] its tail,
//     [5] ln C, [6] expm1(ln u - ln u'), [7] expm1(ln l - ln l'), [8] beta' - beta.
// The object-dependent part of log f' - log f is
//   (beta' - beta) q - e^q [6] + ln((1 - e^{-x'}) / (1 - e^{-x})),  q = chi - ln u,
// x = L / l, x' = x (1 + [7]); the rest, (beta' + 1)(ln u - ln u') + ln C' - ln C,
// is object-independent (dlf_const returns its negative).
// ===========================================================================
__device__ __forceinline__ double bb1_ln_norm(double beta, double ln_l, double ln_u)
{
    const double ln_q = log1p(exp(ln_u - ln_l));
    const double a = beta + 1.0;
    if (a == 0.0) return -log(ln_q);
    // Gamma(a) and 1 - q^-a = -expm1(-a ln q) share their sign
    return -(log(fabs(tgamma(a))) + log(fabs(expm1(-a * ln_q))));
}

struct BB1 {
    using T = float;
    static constexpr int D = 1, NC = 1, M = 2, MD = 3, P = 3, MODEL = 5;
    static constexpr bool kSelection = true;
    struct Obj {
        float fh, c, e;
    };

    __device__ static void derive_statics(Statics &s)
    {
        s.mf[0] = static_cast<float>(s.mc[1] * s.mc[1]);
        s.mf[1] = static_cast<float>(s.mc[2] * s.mc[2]);
    }
    __device__ static void derive_obj(const T *data, T *dd, int64_t i, int64_t n, const Statics &)
    {
        const double fhat = data[i], k = data[n + i];
        const double centre = k + log(fhat);
        const float c = static_cast<float>(centre);
        dd[i] = static_cast<float>(fhat);
        dd[n + i] = c;
        dd[2 * n + i] = static_cast<float>(centre - static_cast<double>(c));
    }
    __device__ static Obj load(const T *dd, int64_t i, int64_t n) { return Obj{dd[i], dd[n + i], dd[2 * n + i]}; }
    __device__ static void aux(const double *th, double *a)
    {
        a[0] = bb1_ln_norm(th[0], th[1], th[2]);
        a[1] = 0.0;
    }
    __device__ static bool in_support(const double *th) { return th[0] > -2.0 && th[0] < 0.0 && th[1] < th[2]; }
    __device__ static double log_prior(const double *th) { return in_support(th) ? th[1] - log1p(th[0] * th[0]) : -HUGE_VAL; }
    __device__ static void z_consts(const double *tp, double *zc)
    {
        zc[0] = tp[0] + 1.0;
        zc[1] = tp[2];
        zc[2] = tp[1];
        zc[3] = 0.0;
    }
    // the quadrature sum carries no ln C: ln Z = ln sum + ln C
    __device__ static double logz_shift(const double *ap) { return -ap[0]; }
    __device__ static double zlog(const double *zc, double x)
    {
        return zc[0] * (x - zc[1]) + log(-expm1(-exp(x - zc[2]))) - exp(x - zc[1]);
    }
    // ln L from 80 e-folds below the reference l (the PDF falls only as
    // L^(beta+2) there) to 40 times the reference u
    __device__ static void quad_interval(const Statics &s, double *lo, double *hi)
    {
        *lo = s.mc[3] - 80.0;
        *hi = s.mc[4] + log(40.0);
    }
    __device__ static double edge_area(const Statics &) { return 1.0; }
    // eta(F) = Phi((F - F_th) / sigma(F))
    __device__ static double detect(double flux, const Statics &s)
    {
        const double sig = sqrt(s.mc[1] * s.mc[1] + s.mc[2] * s.mc[2] * flux * flux);
        return 0.5 * erfc(-(flux - s.mc[0]) / (sig * 1.4142135623730950488));
    }
    __device__ static double dlf_const(const double *th, const double *tp, const double *a, const double *ap)
    {
        return (tp[0] + 1.0) * (tp[2] - th[2]) + (a[0] - ap[0]);
    }
    __device__ static void derive_kc(const double *th, const double *tp, const double *a, const Statics &, T *kc)
    {
        const float uh = static_cast<float>(th[2]), lh = static_cast<float>(th[1]);
        kc[0] = static_cast<float>(th[0] + 1.0);
        kc[1] = uh;
        kc[2] = static_cast<float>(th[2] - static_cast<double>(uh));
        kc[3] = lh;
        kc[4] = static_cast<float>(th[1] - static_cast<double>(lh));
        kc[5] = static_cast<float>(a[0]);
        kc[6] = static_cast<float>(expm1(th[2] - tp[2]));
        kc[7] = static_cast<float>(expm1(th[1] - tp[1]));
        kc[8] = static_cast<float>(tp[0] - th[0]);
    }
    __device__ static Eval<T> eval(const Obj &o, const T *x, const T *kc, const Statics &s)
    {
        Eval<T> e;
        // member likelihood around the object's centre: F = Fhat e^d
        const float d = (x[0] - o.c) - o.e;
        const float em = expm1f(d);
        const float flux = o.fh + o.fh * em;
        const float var = s.mf[0] + s.mf[1] * flux * flux;
        const float z = o.fh * em;
        const float lm = -0.5f * (z * z) / var - 0.5f * logf(var);
        // population term
        e.q = (x[0] - kc[1]) - kc[2];
        e.eq = expf(e.q);
        e.res = expf((x[0] - kc[3]) - kc[4]);          // x = L / l
        const float brk = logf(-expm1f(-e.res));
        const float g = kc[0] * e.q + brk - e.eq;
        e.lpv = lm + g;
        e.lf = g + kc[5];
        e.lp = lm + e.lf;
        e.u = 0.0f;
        return e;
    }
    __device__ static T dlf(const Obj &, const T *, const Eval<T> &e, const T *kc, const Statics &)
    {
        // ln((1 - e^{-x'}) / (1 - e^{-x})) = log1p((e^{-x} - e^{-x'}) / (1 - e^{-x}))
        const float x = e.res, dx = x * kc[7];                 // x' - x
        const float den = -expm1f(-x);
        const float num = (dx > -60.0f) ? expf(-x) * -expm1f(-dx) : expf(-x) - expf(-(x + dx));
        const float brk = (den > 0.0f) ? log1pf(num / den) : log1pf(kc[7]);
        return kc[8] * e.q - e.eq * kc[6] + brk;
    }
    // the break factor ties l to every object: no finite sufficient statistics
    static constexpr int NS = 0;
    __device__ static void stats(const Obj &, const T *, const Eval<T> &, const T *, const Statics &, T *) {}
    __device__ static double stats_dlf(const double *, const double *, const double *, const double *, const double *,
                                       double, const Statics &)
    {
        return 0.0;
    }
};

}  // namespace hbm
