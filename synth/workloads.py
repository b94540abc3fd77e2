"""Simulated catalogs for the single-plate models the sampler handles.

Every generator is seeded (numpy PCG64 via ``default_rng``) and returns a
:class:`Workload`: the per-object data arrays exactly as both the oracle and
the GPU library receive them, the model constants, the true population
parameters and the chain's starting point.

Data follow the simulation designs of the paper: the heteroscedastic
normal-normal benchmark (Sec. 3, eqs 3.1-3.4) and the luminosity-function
study with a thinned (flux-selected) population (Sec. 4-5, eqs 4.2-4.4 and
5.10), with the gamma luminosity PDF that the BB1 model reduces to as l -> 0
(Appendix B), and the paper's own break-by-one (BB1) case study (Sec. 5).  Quantities are dimensionless.  Where an array feeds a
single-precision sampler it is stored already rounded to float32, so both
sides see bit-identical inputs.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

# Model identifiers; the C ABI uses the same integers.
NORMAL_NORMAL_1D = 1
GAMMA_LF_1D = 2
GAMMA_LF_COLOR_3D = 3
NORMAL_NORMAL_3D = 4
BB1_LF = 5

MODEL_NAMES = {
    NORMAL_NORMAL_1D: "normal_normal_1d",
    GAMMA_LF_1D: "gamma_lf_1d",
    GAMMA_LF_COLOR_3D: "gamma_lf_color_3d",
    NORMAL_NORMAL_3D: "normal_normal_3d",
    BB1_LF: "bb1_lf",
}

# Index of each model constant inside the 16-slot constant vector.
C_FTH, C_SIGF, C_RMAX, C_LNL0, C_SIGR, C_SIGC = 0, 1, 2, 3, 4, 5


@dataclasses.dataclass
class Workload:
    model: int
    n: int
    d: int                    # latent dimension per object
    p: int                    # population-parameter dimension
    precision: str            # "f64" or "f32": per-object arithmetic
    data: np.ndarray          # [m][n], dtype float64 or float32
    consts: np.ndarray        # [16] float64 model constants
    theta_true: np.ndarray    # [p]
    theta0: np.ndarray        # [p] chain start
    theta_chol0: np.ndarray   # [p][p] lower-triangular start of the theta proposal factor
    chi0: np.ndarray          # [d][n] float64 (float32-representable when precision == f32)
    seed: int
    alpha_star: float         # target acceptance of the per-object RAM
    truth: Dict[str, np.ndarray] = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.data.shape[0])

    @property
    def name(self) -> str:
        return MODEL_NAMES[self.model]


NormalNormal1D = NORMAL_NORMAL_1D
GammaLF1D = GAMMA_LF_1D
GammaLF3D = GAMMA_LF_COLOR_3D


def _consts(**kw) -> np.ndarray:
    c = np.zeros(16, dtype=np.float64)
    for k, v in kw.items():
        c[int(k[1:])] = v
    return c


def normal_normal_1d(n: int = 1000, seed: int = 0, mu: float = 0.0, tau: float = 1.0) -> Workload:
    """Heteroscedastic 1-D normal-normal population.

    chi_i ~ N(mu, tau^2), sigma_i ~ U[0.5, 1.5], y_i ~ N(chi_i, sigma_i^2).
    theta = (mu, ln tau).  The chain starts at chi_i = y_i and theta at the truth.
    """
    rng = np.random.default_rng(seed)
    chi = rng.normal(mu, tau, n)
    sig = rng.uniform(0.5, 1.5, n)
    y = rng.normal(chi, sig)
    data = np.stack([y, sig]).astype(np.float64)
    theta = np.array([mu, math.log(tau)])
    return Workload(
        model=NORMAL_NORMAL_1D, n=n, d=1, p=2, precision="f64",
        data=data, consts=_consts(), theta_true=theta.copy(), theta0=theta.copy(),
        theta_chol0=np.diag([0.05, 0.05]), chi0=y[None, :].copy(), seed=seed,
        alpha_star=0.44, truth={"chi": chi},
    )


# The paper's 3-D normal-normal instance (Sec. 3): population mean, marginal
# standard deviations, correlation matrix and per-component noise.
NN3D_MU = np.array([1.2, -0.4, 3.4])
NN3D_D = np.array([2.3, 0.45, 13.4])
NN3D_R = np.array([[1.0, 0.3, -0.5], [0.3, 1.0, 0.54], [-0.5, 0.54, 1.0]])
NN3D_SIGMA = np.array([1.2, 0.4, 0.24])


def normal_normal_3d(n: int = 1000, seed: int = 5) -> Workload:
    """The paper's correlated 3-D normal-normal benchmark (Sec. 3).

    chi_i ~ MVN(mu, D R D), y_ij ~ N(chi_ij, sigma_j^2); C_pop and sigma are
    known, theta = mu with a flat prior.  Constants: the six lower-triangle
    entries of C_pop (row-major) then sigma_1..3.
    """
    rng = np.random.default_rng(seed)
    cpop = np.diag(NN3D_D) @ NN3D_R @ np.diag(NN3D_D)
    chi = rng.multivariate_normal(NN3D_MU, cpop, size=n).T
    y = chi + NN3D_SIGMA[:, None] * rng.standard_normal((3, n))
    c = np.zeros(16)
    c[0:6] = [cpop[0, 0], cpop[1, 0], cpop[1, 1], cpop[2, 0], cpop[2, 1], cpop[2, 2]]
    c[6:9] = NN3D_SIGMA
    return Workload(
        model=NORMAL_NORMAL_3D, n=n, d=3, p=3, precision="f64",
        data=y.astype(np.float64), consts=c, theta_true=NN3D_MU.copy(), theta0=NN3D_MU.copy(),
        theta_chol0=np.diag([0.1, 0.02, 0.4]), chi0=y.copy(), seed=seed,
        alpha_star=0.4, truth={"chi": chi},
    )


def _draw_population(rng, count: int, shape: float, lstar: float, rmax: float):
    lum = rng.gamma(shape, lstar, count)
    r = rmax * rng.random(count) ** (1.0 / 3.0)
    return lum, r


def calibrate_threshold(rng, shape: float, lstar: float, rmax: float, det_frac: float,
                        sigma_frac: float = 0.1, n_mc: int = 2_000_000) -> float:
    """Flux threshold giving the requested detected fraction, by Monte Carlo.

    Draws a population sample (L ~ Gamma(shape, lstar), r with density
    proportional to r^2 on [0, rmax]) and one noise draw per object, and
    bisects for the threshold T at which the fraction with
    F + sigma_frac*T*eps > T equals ``det_frac``.  The fraction is monotone
    in T, so the bisection converges to the empirical root.
    """
    lum, r = _draw_population(rng, n_mc, shape, lstar, rmax)
    flux = lum / (4.0 * math.pi * r * r)
    eps = rng.standard_normal(n_mc)
    lo, hi = math.log(np.quantile(flux, 0.01)), math.log(np.quantile(flux, 0.999))
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        t = math.exp(mid)
        frac = np.count_nonzero(flux + sigma_frac * t * eps > t) / n_mc
        if frac > det_frac:
            lo = mid
        else:
            hi = mid
    return math.exp(0.5 * (lo + hi))


def _detected_catalog(rng, n: int, shape: float, lstar: float, rmax: float, fth: float,
                      sigma_frac: float = 0.1, det_frac_guess: float = 0.3):
    """Draw objects until exactly ``n`` pass the flux cut; keep draw order."""
    keep_l, keep_r, keep_fh = [], [], []
    have = 0
    chunk = max(4096, int(1.15 * n / det_frac_guess))
    while have < n:
        lum, r = _draw_population(rng, chunk, shape, lstar, rmax)
        flux = lum / (4.0 * math.pi * r * r)
        fhat = flux + sigma_frac * fth * rng.standard_normal(chunk)
        sel = fhat > fth
        keep_l.append(lum[sel]); keep_r.append(r[sel]); keep_fh.append(fhat[sel])
        have += int(sel.sum())
    lum = np.concatenate(keep_l)[:n]
    r = np.concatenate(keep_r)[:n]
    fhat = np.concatenate(keep_fh)[:n]
    return lum, r, fhat


def gamma_lf_1d(n: int = 300_000, seed: int = 1, beta: float = -0.3, lstar: float = 5e10,
                rmax: float = 4000.0, det_frac: float = 0.3, n_mc: int = 2_000_000,
                fth: Optional[float] = None) -> Workload:
    """Gamma luminosity function with a flux-thinned catalog, latent chi = ln L.

    L ~ Gamma(shape beta+1, scale L*), r ~ r^2 on [0, rmax], F = L/(4 pi r^2),
    Fhat ~ N(F, (0.1 F_th)^2), kept when Fhat > F_th; F_th gives ~det_frac
    detected.  Distances are known.  Data (float32): Fhat and k = ln(4 pi r^2).
    theta = (beta, ln L*).  The chain starts at chi_i = ln(4 pi r_i^2 Fhat_i).
    """
    rng = np.random.default_rng(seed)
    shape = beta + 1.0
    if fth is None:
        fth = calibrate_threshold(rng, shape, lstar, rmax, det_frac, n_mc=n_mc)
    lum, r, fhat = _detected_catalog(rng, n, shape, lstar, rmax, fth, det_frac_guess=det_frac)
    fhat32 = fhat.astype(np.float32)
    k32 = np.log(4.0 * math.pi * r * r).astype(np.float32)
    data = np.stack([fhat32, k32])
    chi0 = (k32.astype(np.float64) + np.log(fhat32.astype(np.float64))).astype(np.float32)
    c = _consts(c0=fth, c1=0.1 * fth, c2=rmax, c3=math.log(lstar))
    theta = np.array([beta, math.log(lstar)])
    return Workload(
        model=GAMMA_LF_1D, n=n, d=1, p=2, precision="f32",
        data=data, consts=c, theta_true=theta.copy(), theta0=theta.copy(),
        theta_chol0=np.diag([0.05, 0.05]), chi0=chi0.astype(np.float64)[None, :], seed=seed,
        alpha_star=0.44, truth={"lum": lum, "r": r},
    )


def gamma_lf_3d(n: int = 1_000_000, seed: int = 2, beta: float = -0.3, lstar: float = 5e10,
                rmax: float = 4000.0, det_frac: float = 0.3, a: float = -2.0, b: float = 0.1,
                s: float = 0.2, n_mc: int = 2_000_000, fth: Optional[float] = None) -> Workload:
    """Three latents per object: (ln L, ln r, colour c).

    As :func:`gamma_lf_1d`, plus colour c ~ N(a + b ln L, s^2); the distance is
    now measured with 5 % noise, rhat = r (1 + 0.05 eps), and the colour with
    absolute noise 0.05, chat = c + 0.05 eps'.  Data (float32): Fhat, rhat,
    chat.  theta = (beta, ln L*, a, b, s).
    """
    rng = np.random.default_rng(seed)
    shape = beta + 1.0
    if fth is None:
        fth = calibrate_threshold(rng, shape, lstar, rmax, det_frac, n_mc=n_mc)
    lum, r, fhat = _detected_catalog(rng, n, shape, lstar, rmax, fth, det_frac_guess=det_frac)
    col = a + b * np.log(lum) + s * rng.standard_normal(n)
    rhat = r * (1.0 + 0.05 * rng.standard_normal(n))
    chat = col + 0.05 * rng.standard_normal(n)
    fh32, rh32, ch32 = fhat.astype(np.float32), rhat.astype(np.float32), chat.astype(np.float32)
    data = np.stack([fh32, rh32, ch32])
    f64 = lambda v: v.astype(np.float64)  # noqa: E731
    chi0 = np.stack([
        (np.log(4.0 * math.pi) + 2.0 * np.log(f64(rh32)) + np.log(f64(fh32))).astype(np.float32),
        np.log(f64(rh32)).astype(np.float32),
        ch32,
    ]).astype(np.float64)
    # A start outside r <= rmax has zero population density; pull it inside.
    over = chi0[1] >= math.log(rmax)
    if np.any(over):
        chi0[1, over] = np.float32(math.log(rmax) - 1e-3)
    c = _consts(c0=fth, c1=0.1 * fth, c2=rmax, c3=math.log(lstar), c4=0.05, c5=0.05)
    theta = np.array([beta, math.log(lstar), a, b, s])
    return Workload(
        model=GAMMA_LF_COLOR_3D, n=n, d=3, p=5, precision="f32",
        data=data, consts=c, theta_true=theta.copy(), theta0=theta.copy(),
        theta_chol0=np.diag([0.02, 0.02, 0.05, 0.005, 0.02]), chi0=chi0, seed=seed,
        alpha_star=0.4, truth={"lum": lum, "r": r, "col": col},
    )


def gamma_lf_batch(n_datasets: int = 256, master_seed: int = 3, seed0: int = 1000,
                   n_lo: float = 1e3, n_hi: float = 1e5, n_mc: int = 200_000) -> List[Workload]:
    """Independent luminosity-function datasets of uneven size.

    N_j is log-uniform on [n_lo, n_hi]; each dataset has its own seed
    (seed0 + j) and true theta drawn near the reference one
    (beta ~ U[-0.35, -0.25], ln L* ~ ln 5e10 + N(0, 0.05^2)); its threshold is
    calibrated at its own theta.
    """
    master = np.random.default_rng(master_seed)
    out = []
    for j in range(n_datasets):
        nj = int(round(math.exp(master.uniform(math.log(n_lo), math.log(n_hi)))))
        beta = float(master.uniform(-0.35, -0.25))
        lstar = math.exp(math.log(5e10) + 0.05 * float(master.standard_normal()))
        out.append(gamma_lf_1d(n=nj, seed=seed0 + j, beta=beta, lstar=lstar, n_mc=n_mc))
    return out


def serving_arrivals(rate: float = 20.0, horizon_s: float = 600.0, seed: int = 4,
                     n_lo: float = 1e3, n_hi: float = 3e5, sweep_choices=(1000, 2000, 5000),
                     job_seed0: int = 10000):
    """Poisson stream of inference jobs: (arrival_time, job_seed, n_objects, n_sweeps)."""
    rng = np.random.default_rng(seed)
    t, jobs, j = 0.0, [], 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > horizon_s:
            break
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        sweeps = int(rng.choice(np.asarray(sweep_choices)))
        jobs.append((t, job_seed0 + j, n, sweeps))
        j += 1
    return jobs


def bb1_sample(rng, count: int, beta: float, l: float, u: float) -> np.ndarray:
    """Draws from the break-by-one PDF f(L) ~ (1 - e^{-L/l}) (L/u)^beta e^{-L/u}.

    Writing 1 - e^{-L/l} as the integral of L e^{-L s} over s in [0, 1/l]
    makes f a mixture of gamma laws: s has density proportional to
    (1/u + s)^-(beta+2) on [0, 1/l] (drawn by inverting its CDF) and
    L | s ~ Gamma(beta + 2, scale 1 / (1/u + s)).  Valid for -2 < beta.
    """
    g = beta + 2.0
    a, b = 1.0 / u, 1.0 / l
    q = rng.random(count)
    if abs(g - 1.0) < 1e-12:
        s = a * np.exp(q * math.log((a + b) / a)) - a
    else:
        lo, hi = a ** (1.0 - g), (a + b) ** (1.0 - g)
        s = (lo + q * (hi - lo)) ** (1.0 / (1.0 - g)) - a
    return rng.gamma(g, 1.0 / (a + s))


def bb1_lf(n: int = 100_000, seed: int = 6, beta: float = -1.5, l: float = 0.01, u: float = 1.0,
           alpha: float = 0.01, nu: float = 5.0, fth: float = 20.0, chunk: int = 4_000_000) -> Workload:
    """The paper's break-by-one luminosity-function study (Sec. 5), dimensionless.

    Luminosities in units of the reference upper scale, distances in units of
    rmax (density 3 r^2 on (0, 1]), fluxes F = L / r^2 in units of the
    fiducial flux u / (4 pi rmax^2).  Fhat ~ N(F, sigma(F)^2) with
    sigma(F) = sqrt(sigma0^2 + (alpha F)^2); an object is detected when
    Fhat > F_th, the threshold at nu times its own error,
    F_th = nu sigma0 / sqrt(1 - nu^2 alpha^2).  sigma0 is set so that F_th = fth
    (20: a source of 20 u at rmax is just detectable).  Objects are drawn
    from the whole population until n are detected.  Data (float32): Fhat
    and k = ln r^2, so F = exp(chi - k) for chi = ln L.  theta = (beta, ln l, ln u).
    """
    rng = np.random.default_rng(seed)
    sigma0 = fth * math.sqrt(1.0 - nu * nu * alpha * alpha) / nu
    keep_f, keep_r, keep_l, keep_fl = [], [], [], []
    have = 0
    while have < n:
        lum = bb1_sample(rng, chunk, beta, l, u)
        r = rng.random(chunk) ** (1.0 / 3.0)
        flux = lum / (r * r)
        fhat = flux + np.sqrt(sigma0 * sigma0 + (alpha * flux) ** 2) * rng.standard_normal(chunk)
        sel = fhat > fth
        keep_f.append(fhat[sel]); keep_r.append(r[sel]); keep_l.append(lum[sel]); keep_fl.append(flux[sel])
        have += int(sel.sum())
    fhat = np.concatenate(keep_f)[:n]
    r = np.concatenate(keep_r)[:n]
    lum = np.concatenate(keep_l)[:n]
    fhat32 = fhat.astype(np.float32)
    k32 = np.log(r * r).astype(np.float32)
    data = np.stack([fhat32, k32])
    chi0 = (k32.astype(np.float64) + np.log(fhat32.astype(np.float64))).astype(np.float32)
    c = _consts(c0=fth, c1=sigma0, c2=alpha, c3=math.log(l), c4=math.log(u))
    theta = np.array([beta, math.log(l), math.log(u)])
    return Workload(
        model=BB1_LF, n=n, d=1, p=3, precision="f32",
        data=data, consts=c, theta_true=theta.copy(), theta0=theta.copy(),
        theta_chol0=np.diag([0.02, 0.05, 0.02]), chi0=chi0.astype(np.float64)[None, :], seed=seed,
        alpha_star=0.44, truth={"lum": lum, "r": r},
    )
