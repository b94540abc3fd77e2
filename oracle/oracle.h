/*
 * Plain FP64 CPU oracle for the Metropolis-within-Gibbs sampler of
 * single-plate hierarchical models (robust adaptive Metropolis per object,
 * Metropolis-Hastings on the population parameters).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.
 * It is deliberately slow and literal: every density is written out from
 * its definition, the RAM factor is obtained by forming the matrix of the
 * RAM update equation and Cholesky-factoring it, and per-object terms are
 * summed serially in object order.  It shares no source with the GPU
 * library and must never be linked into it.
 *
 * Paper map (Szalai-Gindl et al., CUDAHM):
 *   MWG cycle ............................. Sec. 2.1, eqs (2.4)/(2.5)
 *   RAM proposal / accept / adaptation .... Sec. 2.2, eq (2.6)
 *   theta step on the population posterior  Sec. 2.2 (host-side MH)
 *   normal-normal models .................. Sec. 3, eqs (3.1)-(3.4)
 *   thinned point-process likelihood ...... Sec. 4.3, eqs (4.2)-(4.4)
 *   detection efficiency .................. Sec. 5.2, eq (5.10)
 *   gamma luminosity PDF (BB1, l -> 0) .... Appendix B, eqs (C.2)/(C.3)
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the
 * Box-Muller transform (1958).
 *
 * Parity status: every function here is pinned by tests under tests/ that
 * check it against closed forms, library routines or brute force.
 */
#ifndef ORACLE_H
#define ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_NN1D = 1, ORC_LF1D = 2, ORC_LF3D = 3, ORC_NN3D = 4, ORC_BB1 = 5 };

typedef struct orc_ctx orc_ctx;

/* Random numbers -------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Uniforms u[0..4] in (0,1] and normals z[0..3] of one block. */
void orc_variates(uint64_t seed, const uint32_t ctr[4], double u[5], double z[4]);

/* Quadrature ------------------------------------------------------------ */
void orc_gauss_legendre(int n, double a, double b, double *x, double *w);

/* Problem --------------------------------------------------------------- */
/* data: [m][n] row-major doubles, copied.  consts: 16 model constants.
 * nq: quadrature nodes for the selection normaliser (0 = no selection). */
orc_ctx *orc_new(int model, int64_t n, const double *data, const double *consts,
                 uint64_t seed, double alpha_star, double gamma,
                 double alpha_star_theta, int adapt_theta, int nq);
void orc_free(orc_ctx *c);
int orc_dims(const orc_ctx *c, int *d, int *p, int *m);
int orc_num_threads(void);   /* threads the latent sweep uses */
void orc_set_num_threads(int n);   /* sets it (timing on one core) */

/* log member likelihood and log population density of object i at x[d]. */
void orc_log_terms(const orc_ctx *c, int64_t i, const double *x, const double *theta,
                   double *log_meas, double *log_pop);
double orc_log_prior(const orc_ctx *c, const double *theta);
double orc_log_Z(const orc_ctx *c, const double *theta);
double orc_eps(const orc_ctx *c, double x);   /* detection efficiency of ln L = x */
double orc_bb1_log_norm(double beta, double ln_l, double ln_u);   /* ln C of the break-by-one PDF */
/* sum_i log f(chi_i; theta), serial in object order.  chi: [d][n]. */
double orc_pop_sum(const orc_ctx *c, const double *theta, const double *chi);
/* out[i] = log l_i(pts_i) + log f(pts_i; theta), pts [d][n]. */
void orc_log_post(const orc_ctx *c, const double *theta, const double *pts, double *out);
/* out[i] = log f(chi_i; theta). */
void orc_pop_terms(const orc_ctx *c, const double *theta, const double *chi, double *out);

/* Per-object marginal likelihood of 1-D latents (models with d = 1):
 * out[i] = ln of the integral over chi of exp(log l_i(chi) + log f(chi; theta)),
 * with log l_i as in orc_log_terms (its constants included), by composite
 * 20-point Gauss-Legendre panels, fine near the member likelihood's peak
 * (Sec. 6 proposes marginalising low-dimensional latents by quadrature).
 * The marginal log-likelihood of theta is sum_i out[i] - n ln Z(theta).
 * Returns -1 for d > 1. */
int orc_marginal_terms(const orc_ctx *c, const double *theta, double *out);

/* One RAM sweep k (1-based) of every object at fixed theta.
 * chi [d][n], chol [d(d+1)/2][n] (packed lower, row-major), acc [n].
 * trace (nullable) [n][5]: lp_x, lp_y, ln_u, accepted, alpha. */
void orc_sweep(const orc_ctx *c, int64_t k, const double *theta,
               double *chi, double *chol, uint32_t *acc, double *trace);

/* Proposal of the theta step of cycle k: theta' = theta + S_theta z. */
void orc_theta_proposal(const orc_ctx *c, int64_t k, const double *theta,
                        const double *chol_theta, double *theta_prop);
/* Theta step of cycle k at latent state chi: K Metropolis steps on theta
 * given chi (K = 1 unless set below), each from the full N-term sums.
 * Updates theta and chol_theta (p x p lower, row-major).  info (nullable)
 * [6 + 2p]: delta, ln_u, accepted, alpha, sum lf(theta'), sum lf(theta) of
 * the last step, with info[2] the number of steps accepted, then that
 * step's proposal and the theta it started from.  Returns the number. */
int orc_theta_step(const orc_ctx *c, int64_t k, double *theta, double *chol_theta,
                   const double *chi, double *info);

/* Metropolis steps on theta per cycle (values below 1 mean 1). */
void orc_set_theta_substeps(orc_ctx *c, int substeps);

/* n_cycles MWG cycles starting after sweep k0.
 * theta_trace [n_cycles][p] (nullable); chi_trace [n_cycles/thin][d][n]
 * (nullable, snapshot after cycles k with k % thin == 0).
 * fix_theta: skip theta steps; fix_chi: skip the latent sweeps. */
void orc_run(const orc_ctx *c, int64_t k0, int64_t n_cycles, double *theta, double *chol_theta,
             double *chi, double *chol, uint32_t *acc, double *theta_trace,
             double *chi_trace, int64_t thin, int fix_theta, int fix_chi);

#ifdef __cplusplus
}
#endif
#endif
