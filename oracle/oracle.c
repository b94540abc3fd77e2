/*
 * Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written for clarity, not speed.  Nothing here is blocked, fused or
 * reordered beyond what the definitions state; the only parallelism is an
 * OpenMP loop over objects in the latent sweep, whose updates are
 * independent given theta (Sec. 2.1: the psi_i are conditionally
 * independent in eq 2.4).  Sums over objects run serially in object order.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

struct orc_ctx {
    int model, d, p, m;
    int64_t n;
    double *data;            /* [m][n] */
    double consts[16];
    uint64_t seed;
    double alpha_star, gamma, alpha_star_theta;
    int adapt_theta;
    int theta_substeps;      /* Metropolis steps on theta per cycle (>= 1) */
    /* selection normaliser: nodes in x = ln L, weights, efficiency per node */
    int nq;
    double *qx, *qw, *qeps;
    double *qt, *qv;         /* inner rule in t = ln u on [-60, 0] */
    /* normal-normal 3-D: inverse population covariance and log normaliser */
    double cinv[9];
    double log_norm3;
};

/* ===================================================================== */
/* Philox4x32-10 (Salmon et al. 2011): 10 rounds of two 32x32->64-bit     */
/* multiplies with the published multipliers, key bumped by the Weyl      */
/* constants between rounds.                                              */
/* ===================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t prod0 = (uint64_t)mult0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)mult1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)prod1;
        uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)prod0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The four output words, read as one 128-bit little-endian integer, are cut
 * into five 24-bit fields; field j maps to u_j = (field_j + 1) 2^-24 in
 * (0, 1].  Box-Muller turns (u0, u1) and (u2, u3) into four standard
 * normals; u4 is left for the accept test. */
void orc_variates(uint64_t seed, const uint32_t ctr[4], double u[5], double z[4])
{
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    unsigned __int128 v = 0;
    for (int w = 3; w >= 0; w--)
        v = (v << 32) | (unsigned __int128)x[w];
    for (int j = 0; j < 5; j++) {
        uint32_t field = (uint32_t)((v >> (24 * j)) & 0xffffffu);
        u[j] = ((double)field + 1.0) / 16777216.0;
    }
    double r0 = sqrt(-2.0 * log(u[0]));
    double r1 = sqrt(-2.0 * log(u[2]));
    z[0] = r0 * cos(2.0 * M_PI * u[1]);
    z[1] = r0 * sin(2.0 * M_PI * u[1]);
    z[2] = r1 * cos(2.0 * M_PI * u[3]);
    z[3] = r1 * sin(2.0 * M_PI * u[3]);
}

/* ===================================================================== */
/* Gauss-Legendre rule on [a, b]: roots of P_n by Newton's method from    */
/* the usual cosine first guess, weights 2 / ((1 - t^2) P_n'(t)^2).       */
/* Nodes are returned in ascending order.                                 */
/* ===================================================================== */
static void legendre_pair(int n, double t, double *pn, double *dpn)
{
    double p_prev = 1.0, p = t;
    for (int j = 2; j <= n; j++) {
        double p_next = ((2.0 * j - 1.0) * t * p - (j - 1.0) * p_prev) / j;
        p_prev = p;
        p = p_next;
    }
    *pn = p;
    *dpn = n * (t * p - p_prev) / (t * t - 1.0);
}

void orc_gauss_legendre(int n, double a, double b, double *x, double *w)
{
    double mid = 0.5 * (a + b), half = 0.5 * (b - a);
    for (int i = 0; i < n; i++) {
        double t = cos(M_PI * (i + 0.75) / (n + 0.5));
        double pn, dpn;
        for (int it = 0; it < 100; it++) {
            legendre_pair(n, t, &pn, &dpn);
            double step = pn / dpn;
            t -= step;
            if (fabs(step) < 1e-16)
                break;
        }
        legendre_pair(n, t, &pn, &dpn);
        x[i] = mid - half * t;           /* t descends with i, so x ascends */
        w[i] = half * 2.0 / ((1.0 - t * t) * dpn * dpn);
    }
}

/* ===================================================================== */
/* Models: log member likelihood log l_i(x) (Sec. 2.1, up to a constant)  */
/* and log population density log f(x; theta) in the latent coordinates.  */
/* ===================================================================== */
static const double LOG_2PI = 1.8378770664093454836;

/* Gamma luminosity PDF (the l -> 0 limit of BB1, shape beta + 1, scale L*)
 * expressed in x = ln L, i.e. including the Jacobian dL/dx = L. */
static double log_gamma_lum(double x, double beta, double ln_lstar)
{
    double a = beta + 1.0;
    return a * (x - ln_lstar) - exp(x - ln_lstar) - lgamma(a);
}

/* Normaliser C(beta, u, l) of the break-by-one PDF (Appendix C):
 * 1 / (Gamma(beta + 1) (1 - (1 + u/l)^-(beta+1))) for beta != -1 and
 * 1 / ln(1 + u/l) at beta = -1.  For -2 < beta < -1 both factors of the
 * first form are negative.  Returned as ln C. */
double orc_bb1_log_norm(double beta, double ln_l, double ln_u)
{
    double q = 1.0 + exp(ln_u - ln_l);
    double a = beta + 1.0;
    if (a == 0.0)
        return -log(log(q));
    double g = tgamma(a);
    double f = -expm1(-a * log(q));   /* 1 - q^-a */
    return -log(g * f);
}

/* Break-by-one luminosity PDF (Sec. 5.1 and Appendix C),
 * f(L) = C / u (1 - e^{-L/l}) (L/u)^beta e^{-L/u}, expressed in x = ln L
 * (times the Jacobian L). */
static double log_bb1_lum(double x, double beta, double ln_l, double ln_u)
{
    return orc_bb1_log_norm(beta, ln_l, ln_u) + (beta + 1.0) * (x - ln_u) + log(-expm1(-exp(x - ln_l)))
           - exp(x - ln_u);
}

/* Flux-dependent measurement error sigma(F) = sqrt(sigma0^2 + (alpha F)^2) (eq 5.8). */
static double bb1_sigma(const orc_ctx *c, double flux)
{
    return sqrt(c->consts[1] * c->consts[1] + c->consts[2] * flux * c->consts[2] * flux);
}

void orc_log_terms(const orc_ctx *c, int64_t i, const double *x, const double *theta,
                   double *log_meas, double *log_pop)
{
    const double *col0 = c->data, *col1 = c->data + c->n, *col2 = c->data + 2 * c->n;
    switch (c->model) {
    case ORC_NN1D: {
        /* y_i ~ N(chi_i, sigma_i^2), chi_i ~ N(mu, tau^2); theta = (mu, ln tau). */
        double y = col0[i], sig = col1[i];
        double tau = exp(theta[1]);
        *log_meas = -0.5 * ((y - x[0]) / sig) * ((y - x[0]) / sig);
        *log_pop = -0.5 * ((x[0] - theta[0]) / tau) * ((x[0] - theta[0]) / tau) - theta[1] - 0.5 * LOG_2PI;
        break;
    }
    case ORC_LF1D: {
        /* Fhat_i ~ N(F, sigma_F^2) with F = L / (4 pi r_i^2) = exp(x - k_i). */
        double fhat = col0[i], k = col1[i], sigf = c->consts[1];
        double flux = exp(x[0] - k);
        *log_meas = -0.5 * ((fhat - flux) / sigf) * ((fhat - flux) / sigf);
        *log_pop = log_gamma_lum(x[0], theta[0], theta[1]);
        break;
    }
    case ORC_LF3D: {
        /* latent (ln L, ln r, c); data Fhat, rhat, chat. */
        double fhat = col0[i], rhat = col1[i], chat = col2[i];
        double sigf = c->consts[1], rmax = c->consts[2], sigr = c->consts[4] * rhat, sigc = c->consts[5];
        double flux = exp(x[0] - log(4.0 * M_PI) - 2.0 * x[1]);
        double r = exp(x[1]);
        *log_meas = -0.5 * ((fhat - flux) / sigf) * ((fhat - flux) / sigf)
                    - 0.5 * ((rhat - r) / sigr) * ((rhat - r) / sigr)
                    - 0.5 * ((chat - x[2]) / sigc) * ((chat - x[2]) / sigc);
        /* h(r) = 3 r^2 / rmax^3 on (0, rmax], as a density in ln r. */
        double log_h = (x[1] <= log(rmax)) ? log(3.0) + 3.0 * x[1] - 3.0 * log(rmax) : -INFINITY;
        double s = theta[4];
        double resid = (x[2] - theta[2] - theta[3] * x[0]) / s;
        *log_pop = log_gamma_lum(x[0], theta[0], theta[1]) + log_h
                   - 0.5 * resid * resid - log(s) - 0.5 * LOG_2PI;
        break;
    }
    case ORC_BB1: {
        /* Fhat_i ~ N(F, sigma(F)^2), F = exp(x - k_i) (the member likelihood is
         * the sampling density of Fhat, with its 1/sigma(F)); theta = (beta, ln l, ln u). */
        double fhat = col0[i], k = col1[i];
        double flux = exp(x[0] - k), sig = bb1_sigma(c, flux);
        *log_meas = -0.5 * ((fhat - flux) / sig) * ((fhat - flux) / sig) - log(sig);
        *log_pop = log_bb1_lum(x[0], theta[0], theta[1], theta[2]);
        break;
    }
    case ORC_NN3D: {
        /* y_ij ~ N(chi_ij, sigma_j^2), chi_i ~ MVN(mu, C_pop); theta = mu. */
        double dev[3], q = 0.0, lm = 0.0;
        for (int j = 0; j < 3; j++) {
            double y = c->data[j * c->n + i], sig = c->consts[6 + j];
            lm += -0.5 * ((y - x[j]) / sig) * ((y - x[j]) / sig);
            dev[j] = x[j] - theta[j];
        }
        for (int r = 0; r < 3; r++)
            for (int s = 0; s < 3; s++)
                q += dev[r] * c->cinv[3 * r + s] * dev[s];
        *log_meas = lm;
        *log_pop = -0.5 * q - c->log_norm3;
        break;
    }
    default:
        *log_meas = NAN;
        *log_pop = NAN;
    }
}

double orc_log_prior(const orc_ctx *c, const double *theta)
{
    switch (c->model) {
    case ORC_NN1D:
        /* flat in mu, uniform in tau > 0: density in ln tau is tau. */
        return theta[1];
    case ORC_LF1D:
        /* truncated Cauchy slope prior on (-1, 0) (gamma shape beta+1 > 0,
         * decreasing PDF), flat in ln L*. */
        if (!(theta[0] > -1.0 && theta[0] < 0.0))
            return -INFINITY;
        return -log(1.0 + theta[0] * theta[0]);
    case ORC_LF3D:
        if (!(theta[0] > -1.0 && theta[0] < 0.0) || !(theta[4] > 0.0))
            return -INFINITY;
        return -log(1.0 + theta[0] * theta[0]);
    case ORC_NN3D:
        return 0.0;
    case ORC_BB1:
        /* truncated Cauchy on -2 < beta < 0, flat in l, flat in ln u, l < u
         * (eq 5.5); as a density in (beta, ln l, ln u) that is l / (1 + beta^2). */
        if (!(theta[0] > -2.0 && theta[0] < 0.0) || !(theta[1] < theta[2]))
            return -INFINITY;
        return theta[1] - log(1.0 + theta[0] * theta[0]);
    }
    return NAN;
}

/* Detection efficiency eta(F) = Phi((F - F_th) / sigma) (eq 5.10), with
 * sigma = sigma_F for the gamma models and sigma(F) for the BB1 model. */
static double detect_eff(const orc_ctx *c, double flux)
{
    double sig = c->model == ORC_BB1 ? bb1_sigma(c, flux) : c->consts[1];
    double zz = (flux - c->consts[0]) / sig;
    return 0.5 * erfc(-zz / sqrt(2.0));
}

/* eps(ln L) = int_0^rmax dr h(r) eta(L / 4 pi r^2), h(r) = 3 r^2 / rmax^3.
 * With u = (r/rmax)^3 (so h dr = du) and t = ln u this is
 * int_{-inf}^0 e^t eta(L / (4 pi rmax^2 e^{2t/3})) dt; the part below t = -60
 * is below e^-60 and dropped. */
double orc_eps(const orc_ctx *c, double x)
{
    if (c->nq <= 0)
        return NAN;
    /* BB1 catalogs measure distance in units of rmax and flux in units of
     * L / rmax^2: the flux at u is L u^(-2/3). */
    double scale = c->model == ORC_BB1 ? 1.0 : 4.0 * M_PI * c->consts[2] * c->consts[2];
    double lum = exp(x), sum = 0.0;
    for (int l = 0; l < c->nq; l++) {
        double flux = lum / (scale * exp(2.0 * c->qt[l] / 3.0));
        sum += c->qv[l] * exp(c->qt[l]) * detect_eff(c, flux);
    }
    return sum;
}

/* Selection normaliser Z(theta) = int dr h(r) int dL f(L; theta) eta(L/4 pi r^2)
 * (denominator of eq 4.4), as a Gauss-Legendre sum over x = ln L on
 * [ln L0 - 30, ln L0 + ln 40] of f_x(x; theta) eps(x). */
double orc_log_Z(const orc_ctx *c, const double *theta)
{
    if (c->nq <= 0)
        return 0.0;
    double z = 0.0;
    for (int j = 0; j < c->nq; j++) {
        double lf = c->model == ORC_BB1 ? log_bb1_lum(c->qx[j], theta[0], theta[1], theta[2])
                                        : log_gamma_lum(c->qx[j], theta[0], theta[1]);
        z += c->qw[j] * exp(lf) * c->qeps[j];
    }
    return log(z);
}

double orc_pop_sum(const orc_ctx *c, const double *theta, const double *chi)
{
    double sum = 0.0, x[3], lm, lp;
    for (int64_t i = 0; i < c->n; i++) {
        for (int j = 0; j < c->d; j++)
            x[j] = chi[j * c->n + i];
        orc_log_terms(c, i, x, theta, &lm, &lp);
        sum += lp;
    }
    return sum;
}

void orc_log_post(const orc_ctx *c, const double *theta, const double *pts, double *out)
{
    double x[3], lm, lp;
    for (int64_t i = 0; i < c->n; i++) {
        for (int j = 0; j < c->d; j++)
            x[j] = pts[j * c->n + i];
        orc_log_terms(c, i, x, theta, &lm, &lp);
        out[i] = lm + lp;
    }
}

void orc_pop_terms(const orc_ctx *c, const double *theta, const double *chi, double *out)
{
    double x[3], lm;
    for (int64_t i = 0; i < c->n; i++) {
        for (int j = 0; j < c->d; j++)
            x[j] = chi[j * c->n + i];
        orc_log_terms(c, i, x, theta, &lm, &out[i]);
    }
}

/* ===================================================================== */
/* Marginal likelihood of a 1-D latent by composite Gauss-Legendre panels */
/* ===================================================================== */
static double log_joint(const orc_ctx *c, int64_t i, double x, const double *theta)
{
    double lm, lp;
    orc_log_terms(c, i, &x, theta, &lm, &lp);
    return lm + lp;
}

/* Composite 20-point Gauss-Legendre rule of exp(g - shift) over [a, b] cut
 * into panels no wider than h. */
static double gl_composite(const orc_ctx *c, int64_t i, const double *theta, double shift, double a, double b,
                           double h, const double *t20, const double *w20)
{
    if (!(b > a))
        return 0.0;
    int np = (int)ceil((b - a) / h);
    double width = (b - a) / np, sum = 0.0;
    for (int q = 0; q < np; q++) {
        double lo = a + q * width, mid = lo + 0.5 * width;
        for (int j = 0; j < 20; j++)
            sum += 0.5 * width * w20[j] * exp(log_joint(c, i, mid + 0.5 * width * t20[j], theta) - shift);
    }
    return sum;
}

int orc_marginal_terms(const orc_ctx *c, const double *theta, double *out)
{
    if (c->d != 1)
        return -1;
    const double *col0 = c->data, *col1 = c->data + c->n;
    double t20[20], w20[20];
    orc_gauss_legendre(20, -1.0, 1.0, t20, w20);
    for (int64_t i = 0; i < c->n; i++) {
        /* where the integrand lives: the peak of the member likelihood (the
         * datum) with its width in chi, or for the normal-normal model the
         * exact peak and width of the product */
        double centre, width;
        if (c->model == ORC_NN1D) {
            double y = col0[i], sig = col1[i], tau = exp(theta[1]);
            double prec = 1.0 / (sig * sig) + 1.0 / (tau * tau);
            centre = (y / (sig * sig) + theta[0] / (tau * tau)) / prec;
            width = 1.0 / sqrt(prec);
        } else {
            double fhat = col0[i];
            double sig = c->model == ORC_BB1 ? bb1_sigma(c, fhat) : c->consts[1];
            centre = log(fhat) + col1[i];
            width = fmin(sig / fhat, 1.0);
        }
        double shift = log_joint(c, i, centre, theta);
        /* fine panels (a quarter width) within 40 widths of the peak, panels
         * of 0.25 in chi out to 200 below and 15 above it (above the datum
         * the member likelihood falls faster than any normal in chi) */
        double lo = centre - 40.0 * width, hi = centre + 40.0 * width;
        double h_fine = fmin(0.25 * width, 0.25);
        double total = gl_composite(c, i, theta, shift, centre - 200.0, lo, 0.25, t20, w20)
                       + gl_composite(c, i, theta, shift, lo, hi, h_fine, t20, w20)
                       + gl_composite(c, i, theta, shift, hi, centre + 15.0, 0.25, t20, w20);
        /* further down in unit panels: far below the datum and below the
         * population's own features (ln L*, ln l, ln u, mu) the integrand
         * only falls, as a power of L, which for BB1 near beta = -2 is
         * slow; stop at the first panel there that adds < 1e-17 of the total */
        double feature = centre;
        if (c->model == ORC_NN1D)
            feature = fmin(feature, theta[0]);
        else
            feature = fmin(feature, theta[1]);
        if (c->model == ORC_BB1)
            feature = fmin(feature, theta[2]);
        for (double top = centre - 200.0; top > -1e6; top -= 1.0) {
            double add = gl_composite(c, i, theta, shift, top - 1.0, top, 1.0, t20, w20);
            total += add;
            if (top < feature - 40.0 && !(add > 1e-17 * total))
                break;
        }
        out[i] = shift + log(total);
    }
    return 0;
}

/* ===================================================================== */
/* Construction                                                           */
/* ===================================================================== */
orc_ctx *orc_new(int model, int64_t n, const double *data, const double *consts,
                 uint64_t seed, double alpha_star, double gamma,
                 double alpha_star_theta, int adapt_theta, int nq)
{
    orc_ctx *c = calloc(1, sizeof(orc_ctx));
    c->model = model;
    c->n = n;
    switch (model) {
    case ORC_NN1D: c->d = 1; c->p = 2; c->m = 2; break;
    case ORC_LF1D: c->d = 1; c->p = 2; c->m = 2; break;
    case ORC_LF3D: c->d = 3; c->p = 5; c->m = 3; break;
    case ORC_NN3D: c->d = 3; c->p = 3; c->m = 3; break;
    case ORC_BB1: c->d = 1; c->p = 3; c->m = 2; break;
    default: free(c); return NULL;
    }
    c->data = malloc(sizeof(double) * (size_t)c->m * (size_t)n);
    memcpy(c->data, data, sizeof(double) * (size_t)c->m * (size_t)n);
    memcpy(c->consts, consts, sizeof(c->consts));
    c->seed = seed;
    c->alpha_star = alpha_star;
    c->gamma = gamma;
    c->alpha_star_theta = alpha_star_theta;
    c->adapt_theta = adapt_theta;
    c->theta_substeps = 1;
    c->nq = (model == ORC_LF1D || model == ORC_LF3D || model == ORC_BB1) ? nq : 0;
    if (c->nq > 0) {
        c->qx = malloc(sizeof(double) * c->nq);
        c->qw = malloc(sizeof(double) * c->nq);
        c->qeps = malloc(sizeof(double) * c->nq);
        c->qt = malloc(sizeof(double) * c->nq);
        c->qv = malloc(sizeof(double) * c->nq);
        orc_gauss_legendre(c->nq, -60.0, 0.0, c->qt, c->qv);
        if (model == ORC_BB1) {
            /* from 80 e-folds below the break l (the PDF falls only as
             * L^(beta+2) there) to 40 u, at the reference l and u */
            orc_gauss_legendre(c->nq, c->consts[3] - 80.0, c->consts[4] + log(40.0), c->qx, c->qw);
        } else {
            double lnl0 = c->consts[3];
            orc_gauss_legendre(c->nq, lnl0 - 30.0, lnl0 + log(40.0), c->qx, c->qw);
        }
        for (int j = 0; j < c->nq; j++)
            c->qeps[j] = orc_eps(c, c->qx[j]);
    }
    if (model == ORC_NN3D) {
        /* C_pop from its packed lower triangle; inverse by the adjugate. */
        double a[9];
        const double *t = c->consts;
        a[0] = t[0]; a[1] = t[1]; a[2] = t[3];
        a[3] = t[1]; a[4] = t[2]; a[5] = t[4];
        a[6] = t[3]; a[7] = t[4]; a[8] = t[5];
        double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6])
                     + a[2] * (a[3] * a[7] - a[4] * a[6]);
        c->cinv[0] = (a[4] * a[8] - a[5] * a[7]) / det;
        c->cinv[1] = -(a[1] * a[8] - a[2] * a[7]) / det;
        c->cinv[2] = (a[1] * a[5] - a[2] * a[4]) / det;
        c->cinv[3] = -(a[3] * a[8] - a[5] * a[6]) / det;
        c->cinv[4] = (a[0] * a[8] - a[2] * a[6]) / det;
        c->cinv[5] = -(a[0] * a[5] - a[2] * a[3]) / det;
        c->cinv[6] = (a[3] * a[7] - a[4] * a[6]) / det;
        c->cinv[7] = -(a[0] * a[7] - a[1] * a[6]) / det;
        c->cinv[8] = (a[0] * a[4] - a[1] * a[3]) / det;
        c->log_norm3 = 0.5 * (3.0 * LOG_2PI + log(det));
    }
    return c;
}

void orc_free(orc_ctx *c)
{
    if (!c)
        return;
    free(c->data);
    free(c->qx);
    free(c->qw);
    free(c->qeps);
    free(c->qt);
    free(c->qv);
    free(c);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_dims(const orc_ctx *c, int *d, int *p, int *m)
{
    *d = c->d;
    *p = c->p;
    *m = c->m;
    return 0;
}

/* ===================================================================== */
/* RAM (Sec. 2.2, eq 2.6)                                                 */
/* ===================================================================== */

/* Textbook Cholesky-Banachiewicz of a dense symmetric q x q matrix (lower
 * triangle read).  Returns 0 on success, -1 if not positive definite. */
static int cholesky_dense(int q, const double *mat, double *low)
{
    memset(low, 0, sizeof(double) * q * q);
    for (int i = 0; i < q; i++) {
        for (int j = 0; j <= i; j++) {
            double s = mat[i * q + j];
            for (int k = 0; k < j; k++)
                s -= low[i * q + k] * low[j * q + k];
            if (i == j) {
                if (!(s > 0.0))
                    return -1;
                low[i * q + i] = sqrt(s);
            } else {
                low[i * q + j] = s / low[j * q + j];
            }
        }
    }
    return 0;
}

/* S_n = chol(S (I + c U U^T / |U|^2) S^T), S dense lower q x q, in place.
 * For q = 1 the matrix U U^T / |U|^2 is 1 whatever the nonzero U, so
 * S_n = S sqrt(1 + c); U = 0 (the variate map reaches it when u0 = 1) takes
 * that same value, the limit of eq 2.6 as U -> 0.  For q > 1 the direction
 * U / |U| has no limit at U = 0, and a zero |U| leaves S unchanged. */
static void ram_adapt(int q, double *s_mat, const double *u, double cadapt)
{
    if (q == 1) {
        s_mat[0] *= sqrt(1.0 + cadapt);
        return;
    }
    double nrm2 = 0.0;
    for (int j = 0; j < q; j++)
        nrm2 += u[j] * u[j];
    if (!(nrm2 > 0.0))
        return;
    double amat[25], tmat[25], mmat[25], low[25];
    for (int r = 0; r < q; r++)
        for (int s = 0; s < q; s++)
            amat[r * q + s] = (r == s ? 1.0 : 0.0) + cadapt * u[r] * u[s] / nrm2;
    for (int r = 0; r < q; r++)
        for (int s = 0; s < q; s++) {
            double acc = 0.0;
            for (int k = 0; k < q; k++)
                acc += s_mat[r * q + k] * amat[k * q + s];
            tmat[r * q + s] = acc;
        }
    for (int r = 0; r < q; r++)
        for (int s = 0; s < q; s++) {
            double acc = 0.0;
            for (int k = 0; k < q; k++)
                acc += tmat[r * q + k] * s_mat[s * q + k];
            mmat[r * q + s] = acc;
        }
    if (cholesky_dense(q, mmat, low) == 0)
        memcpy(s_mat, low, sizeof(double) * q * q);
}

static double eta_of(const orc_ctx *c, int64_t k)
{
    /* eta_n = n^-gamma with n = k + 1: sweep k turns X_k into X_{k+1}. */
    return pow((double)(k + 1), -c->gamma);
}

void orc_sweep(const orc_ctx *c, int64_t k, const double *theta,
               double *chi, double *chol, uint32_t *acc, double *trace)
{
    const int d = c->d;
    const int64_t n = c->n;
    const double eta = eta_of(c, k);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double x[3], y[3], s_mat[9] = {0}, uvec[3], u[5], z[4];
        for (int j = 0; j < d; j++)
            x[j] = chi[j * n + i];
        /* packed lower triangle, row-major: (0,0) (1,0) (1,1) (2,0) (2,1) (2,2) */
        for (int r = 0, e = 0; r < d; r++)
            for (int s = 0; s <= r; s++, e++)
                s_mat[r * d + s] = chol[e * n + i];
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)k, 0u, 0u};
        orc_variates(c->seed, ctr, u, z);
        for (int j = 0; j < d; j++)
            uvec[j] = z[j];
        /* Y = X + S U */
        for (int r = 0; r < d; r++) {
            y[r] = x[r];
            for (int s = 0; s <= r; s++)
                y[r] += s_mat[r * d + s] * uvec[s];
        }
        double lm_x, lp_x, lm_y, lp_y;
        orc_log_terms(c, i, x, theta, &lm_x, &lp_x);
        orc_log_terms(c, i, y, theta, &lm_y, &lp_y);
        double post_x = lm_x + lp_x, post_y = lm_y + lp_y;
        double delta = isfinite(post_y) ? post_y - post_x : -INFINITY;
        double alpha = delta >= 0.0 ? 1.0 : exp(delta);
        double ln_u = log(u[4]);
        int accepted = ln_u < delta;
        if (accepted) {
            for (int j = 0; j < d; j++)
                chi[j * n + i] = y[j];
            acc[i] += 1u;
        }
        ram_adapt(d, s_mat, uvec, eta * (alpha - c->alpha_star));
        for (int r = 0, e = 0; r < d; r++)
            for (int s = 0; s <= r; s++, e++)
                chol[e * n + i] = s_mat[r * d + s];
        if (trace) {
            trace[5 * i + 0] = post_x;
            trace[5 * i + 1] = post_y;
            trace[5 * i + 2] = ln_u;
            trace[5 * i + 3] = accepted;
            trace[5 * i + 4] = alpha;
        }
    }
}

/* ===================================================================== */
/* Theta step: Gaussian random walk with a RAM-adapted factor, accepted   */
/* on  log pi(theta) + sum_i log f(chi_i; theta) - N log Z(theta).        */
/* ===================================================================== */
/* Sub-step j (0-based) of cycle k draws its proposal normals from blocks
 * (j, k, 1, b) and its accept uniform from block (j, k, 2, 0). */
static void theta_normals(const orc_ctx *c, int64_t k, int j, double *zv)
{
    for (int r = 0; r < c->p; r++) {
        double u[5], z[4];
        uint32_t ctr[4] = {(uint32_t)j, (uint32_t)k, 1u, (uint32_t)(r / 4)};
        orc_variates(c->seed, ctr, u, z);
        zv[r] = z[r % 4];
    }
}

static void proposal_from(const orc_ctx *c, const double *zv, const double *theta, const double *chol_theta,
                          double *theta_prop)
{
    for (int r = 0; r < c->p; r++) {
        theta_prop[r] = theta[r];
        for (int s = 0; s <= r; s++)
            theta_prop[r] += chol_theta[r * c->p + s] * zv[s];
    }
}

void orc_theta_proposal(const orc_ctx *c, int64_t k, const double *theta,
                        const double *chol_theta, double *theta_prop)
{
    double zv[8];
    theta_normals(c, k, 0, zv);
    proposal_from(c, zv, theta, chol_theta, theta_prop);
}

void orc_set_theta_substeps(orc_ctx *c, int substeps)
{
    c->theta_substeps = substeps > 1 ? substeps : 1;
}

/* One Metropolis step on theta given chi: sub-step j of cycle k.  The RAM
 * factor adapts with eta_n, n counting theta steps: n = (k - 1) K + j + 1
 * for K steps per cycle (n = k when K = 1, the latent sweeps' count). */
static int theta_substep(const orc_ctx *c, int64_t k, int j, double *theta, double *chol_theta,
                         const double *chi, double *info)
{
    const int p = c->p;
    double zv[8], prop[8];
    theta_normals(c, k, j, zv);
    proposal_from(c, zv, theta, chol_theta, prop);
    double lprior_prop = orc_log_prior(c, prop);
    double sum_prop = NAN, sum_cur = NAN, delta = -INFINITY;
    if (isfinite(lprior_prop)) {
        sum_prop = orc_pop_sum(c, prop, chi);
        sum_cur = orc_pop_sum(c, theta, chi);
        double post_prop = lprior_prop + sum_prop - (double)c->n * orc_log_Z(c, prop);
        double post_cur = orc_log_prior(c, theta) + sum_cur - (double)c->n * orc_log_Z(c, theta);
        delta = post_prop - post_cur;
        if (isnan(delta))
            delta = -INFINITY;
    }
    double alpha = delta >= 0.0 ? 1.0 : exp(delta);
    double u[5], z[4];
    uint32_t ctr[4] = {(uint32_t)j, (uint32_t)k, 2u, 0u};
    orc_variates(c->seed, ctr, u, z);
    double ln_u = log(u[4]);
    int accepted = ln_u < delta;
    if (accepted)
        memcpy(theta, prop, sizeof(double) * p);
    if (c->adapt_theta) {
        int64_t n = (k - 1) * (int64_t)c->theta_substeps + j + 1;
        ram_adapt(p, chol_theta, zv, pow((double)(n + 1), -c->gamma) * (alpha - c->alpha_star_theta));
    }
    if (info) {
        info[0] = delta;
        info[1] = ln_u;
        info[2] = accepted;
        info[3] = alpha;
        info[4] = sum_prop;
        info[5] = sum_cur;
        memcpy(info + 6, prop, sizeof(double) * p);
    }
    return accepted;
}

int orc_theta_step(const orc_ctx *c, int64_t k, double *theta, double *chol_theta,
                   const double *chi, double *info)
{
    int n_acc = 0;
    for (int j = 0; j < c->theta_substeps; j++) {
        if (info)
            memcpy(info + 6 + c->p, theta, sizeof(double) * c->p);
        n_acc += theta_substep(c, k, j, theta, chol_theta, chi, info);
    }
    if (info)
        info[2] = n_acc;
    return n_acc;
}

void orc_run(const orc_ctx *c, int64_t k0, int64_t n_cycles, double *theta, double *chol_theta,
             double *chi, double *chol, uint32_t *acc, double *theta_trace,
             double *chi_trace, int64_t thin, int fix_theta, int fix_chi)
{
    int64_t snap = 0;
    for (int64_t k = k0 + 1; k <= k0 + n_cycles; k++) {
        if (!fix_chi)
            orc_sweep(c, k, theta, chi, chol, acc, NULL);
        if (!fix_theta)
            orc_theta_step(c, k, theta, chol_theta, chi, NULL);
        if (theta_trace)
            memcpy(theta_trace + (k - k0 - 1) * c->p, theta, sizeof(double) * c->p);
        if (chi_trace && thin > 0 && k % thin == 0) {
            memcpy(chi_trace + snap * c->d * c->n, chi, sizeof(double) * c->d * c->n);
            snap++;
        }
    }
}
