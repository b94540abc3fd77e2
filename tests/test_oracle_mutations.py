"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a temporary copy of oracle/oracle.c (a wrong
constant, a dropped term, a wrong sign or index, a transposed operand),
compiles it, and runs the pin that guards that part of the oracle: the pin
must fail on the altered copy and pass on the real source.  Mistakes are
planted in the oracle only, on the CPU.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_bin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("rr") / "rocrand_philox")
    subprocess.run([hipcc, "-O1", "-o", out, os.path.join(HERE, "pins", "rocrand_philox.cpp")],
                   check=True, capture_output=True)
    return out


# -- pins, each returning True when it holds ---------------------------------

def pin_philox(path, rr):
    cases = [(0, 0, 0, 0, 0), (77, 5, 9, 1, 0), (2**40 + 3, 123456, 7, 2, 3)]
    res = subprocess.run([rr], input="".join(f"{a} {b} {c} {d} {e}\n" for a, b, c, d, e in cases),
                         capture_output=True, text=True, check=True)
    ref = [[int(v) for v in ln.split()] for ln in res.stdout.split("\n") if ln.strip()]
    for (s, a, b, c, d), r in zip(cases, ref):
        if list(oracle.philox4x32_10([a, b, c, d], [s & 0xFFFFFFFF, s >> 32], lib_path=path)) != r:
            return False
    return True


def pin_fields(path, rr):
    for seed, ctr in [(3, [1, 2, 0, 0]), (99, [40, 7, 1, 0])]:
        x = oracle.philox4x32_10(ctr, [seed & 0xFFFFFFFF, seed >> 32], lib_path=path)
        v = int(x[0]) | (int(x[1]) << 32) | (int(x[2]) << 64) | (int(x[3]) << 96)
        u, _ = oracle.variates(seed, ctr, lib_path=path)
        if any(u[j] * 16777216.0 != ((v >> (24 * j)) & 0xFFFFFF) + 1 for j in range(5)):
            return False
    return True


def pin_normals(path, rr):
    zs = np.array([oracle.variates(5, [i, 3, 0, 0], lib_path=path)[1] for i in range(20000)])
    return all(stats.kstest(zs[:, j], "norm").pvalue > 1e-4 for j in range(4))


def pin_gamma_density(path, rr):
    o = oracle.Oracle(synth.gamma_lf_1d(n=8, seed=21, fth=389.75), lib_path=path)
    th = [-0.3, math.log(5e10)]
    for x in [th[1] - 2, th[1], th[1] + 1]:
        if abs(o.log_terms(0, [x], th)[1] - (stats.gamma.logpdf(math.exp(x), 0.7, scale=5e10) + x)) > 1e-10:
            return False
    return True


def pin_mvn_density(path, rr):
    o = oracle.Oracle(synth.normal_normal_3d(n=8), lib_path=path)
    cpop = np.diag(synth.workloads.NN3D_D) @ synth.workloads.NN3D_R @ np.diag(synth.workloads.NN3D_D)
    x, mu = np.array([1.0, -2.0, 7.0]), np.array([0.3, 0.1, -1.0])
    return abs(o.log_terms(0, x, mu)[1] - stats.multivariate_normal.logpdf(x, mu, cpop)) < 1e-10


def pin_efficiency(path, rr):
    wl = synth.gamma_lf_1d(n=8, seed=11, fth=389.75)
    o = oracle.Oracle(wl, lib_path=path)
    fth, sigf, rmax = wl.consts[0], wl.consts[1], wl.consts[2]
    x = math.log(4 * math.pi * rmax**2 * fth) - 1.0
    lum = math.exp(x)
    ref = integrate.quad(lambda r: 3 * r * r / rmax**3 * stats.norm.cdf((lum / (4 * math.pi * r * r) - fth) / sigf),
                         0, rmax, points=[math.sqrt(lum / (4 * math.pi * fth))], limit=200)[0]
    return abs(o.eps(x) - ref) <= 1e-6 * ref


def pin_ram_one_step(path, rr):
    wl = synth.normal_normal_3d(n=40)
    o = oracle.Oracle(wl, lib_path=path)
    st = o.initial_state()
    o.run(st, 20)
    before = st.copy()
    tr = o.sweep(st, trace=True)
    k = st.k
    eta = (k + 1) ** (-2.0 / 3.0)
    for i in range(wl.n):
        _, z = oracle.variates(wl.seed, [i, k, 0, 0], lib_path=path)
        s_old = np.zeros((3, 3))
        e = 0
        for r in range(3):
            for c in range(r + 1):
                s_old[r, c] = before.chol[e, i]
                e += 1
        c_ad = eta * (tr[i, 4] - wl.alpha_star)
        tgt = s_old @ (np.eye(3) + c_ad * np.outer(z[:3], z[:3]) / z[:3].dot(z[:3])) @ s_old.T
        new = np.zeros((3, 3))
        e = 0
        for r in range(3):
            for c in range(r + 1):
                new[r, c] = st.chol[e, i]
                e += 1
        if not np.allclose(new, np.linalg.cholesky(tgt), rtol=1e-10, atol=1e-12):
            return False
    return True


def pin_acceptance_fixed_point(path, rr):
    wl = synth.normal_normal_1d(n=300)
    o = oracle.Oracle(wl, lib_path=path)
    st = o.initial_state()
    o.run(st, 4000, fix_theta=True)
    return abs(st.acc.mean() / 4000 - wl.alpha_star) < 0.015


def pin_theta_given_chi(path, rr):
    from conftest import batch_means
    wl = synth.normal_normal_1d(n=40, seed=0)
    o = oracle.Oracle(wl, lib_path=path)
    st = o.initial_state()
    chi = wl.truth["chi"]
    st.chi[0] = chi
    tt, _ = o.run(st, 40000, fix_chi=True)
    keep = tt[4000:, 1]
    n, ss = chi.size, np.sum((chi - chi.mean()) ** 2)
    lt = np.linspace(-2, 2, 200001)
    lp = -(n - 2) * lt - ss / (2 * np.exp(2 * lt))
    p = np.exp(lp - lp.max())
    p /= np.trapezoid(p, lt)
    m, se = batch_means(keep)
    return abs(m - np.trapezoid(lt * p, lt)) < 3 * se


def pin_selection_in_theta_step(path, rr):
    # the theta step of a flux-limited catalog includes -N ln Z: with the
    # latents held fixed its acceptance ratio must match the definition
    wl = synth.gamma_lf_1d(n=50, seed=41, fth=389.75)
    o = oracle.Oracle(wl, lib_path=path)
    st = o.initial_state()
    o.run(st, 30)
    cur = st.theta.copy()
    st.k += 1
    prop = o.theta_proposal(st, k=st.k)
    info = o.theta_step(st)
    ref = (o.log_prior(prop) + o.pop_sum(prop, st.chi) - wl.n * o.log_Z(prop)) - \
          (o.log_prior(cur) + o.pop_sum(cur, st.chi) - wl.n * o.log_Z(cur))
    return abs(info["delta"] - ref) < 1e-8 and abs(o.log_Z(wl.theta_true) - math.log(0.3)) < 0.05


def _bb1_oracle(path):
    return oracle.Oracle(synth.bb1_lf(n=20, seed=12, chunk=400_000), lib_path=path)


def pin_bb1_normalisation(path, rr):
    o = _bb1_oracle(path)
    pts = [-500, -200, -60, -20, -10, -5, -2, 0, 2, 5]
    for th in ([-1.5, math.log(0.01), 0.0], [-0.5, math.log(0.2), math.log(2.0)]):
        f = lambda x: math.exp(o.log_terms(0, [x], th)[1])
        tot = sum(integrate.quad(f, a, b, limit=400, epsabs=0, epsrel=1e-12)[0] for a, b in zip(pts, pts[1:]))
        if not abs(tot - 1.0) < 1e-8:
            return False
    return True


def pin_bb1_member_likelihood(path, rr):
    o = _bb1_oracle(path)
    wl = o.wl
    s0, alpha = wl.consts[1], wl.consts[2]
    fhat, k = float(wl.data[0][3]), float(wl.data[1][3])
    for x in (k + math.log(fhat) - 0.05, k + math.log(fhat) + 0.2):
        flux = math.exp(x - k)
        ref = stats.norm.logpdf(fhat, flux, math.sqrt(s0 ** 2 + (alpha * flux) ** 2)) + 0.5 * math.log(2 * math.pi)
        if abs(o.log_terms(3, [x], wl.theta_true)[0] - ref) > 1e-12:
            return False
    return True


def pin_bb1_efficiency(path, rr):
    o = _bb1_oracle(path)
    fth, s0, alpha = o.wl.consts[0], o.wl.consts[1], o.wl.consts[2]
    lum = 3.0
    integrand = lambda r: 3 * r * r * stats.norm.cdf((lum / (r * r) - fth) / math.sqrt(s0 ** 2 + (alpha * lum / (r * r)) ** 2))
    r_th = math.sqrt(lum / fth)
    ref = integrate.quad(integrand, 0, 1, points=[0.5 * r_th, r_th, 1.5 * r_th], limit=400, epsabs=1e-15,
                         epsrel=1e-11)[0]
    return abs(o.eps(math.log(lum)) - ref) <= 1e-7 * ref


def pin_bb1_prior(path, rr):
    o = _bb1_oracle(path)
    a, b = [-1.5, math.log(0.01), 0.0], [-0.4, math.log(0.2), math.log(3.0)]
    ref = (math.log(0.2) - math.log(1.16)) - (math.log(0.01) - math.log(3.25))
    return abs((o.log_prior(b) - o.log_prior(a)) - ref) < 1e-13 and o.log_prior([-1.0, 0.5, 0.4]) == -math.inf


def pin_marginal_nn1d(path, rr):
    o = oracle.Oracle(synth.normal_normal_1d(n=50, seed=5), lib_path=path)
    y, sig = o.wl.data
    for mu, tau in ((0.1, 0.8), (5.0, 1e-3), (-2.0, 30.0)):
        v = sig * sig + tau * tau
        ref = np.log(sig / np.sqrt(v)) - (y - mu) ** 2 / (2.0 * v)
        if np.max(np.abs(o.marginal_terms([mu, math.log(tau)]) - ref)) > 1e-12:
            return False
    return True


def pin_marginal_bb1(path, rr):
    o = _bb1_oracle(path)
    th = [-1.5, math.log(0.01), 0.0]
    i = int(np.argmin(o.wl.data[0]))
    fhat, k = float(o.wl.data[0][i]), float(o.wl.data[1][i])
    peak = math.log(fhat) + k
    shift = sum(o.log_terms(i, [peak], th))
    pts = [peak - 400, peak - 60, peak - 10, peak - 1, peak, peak + 1, peak + 15]
    ref = shift + math.log(sum(integrate.quad(lambda x: math.exp(sum(o.log_terms(i, [x], th)) - shift), a, b,
                                              limit=400, epsabs=0, epsrel=1e-13)[0] for a, b in zip(pts, pts[1:])))
    return abs(o.marginal_terms(th)[i] - ref) < 1e-10


def pin_marginal_bb1_slow_tail(path, rr):
    o = _bb1_oracle(path)
    th = [-1.95, math.log(0.01), 0.0]
    fhat, k = float(o.wl.data[0][0]), float(o.wl.data[1][0])
    peak = math.log(fhat) + k
    shift = sum(o.log_terms(0, [peak], th))
    g = lambda x: math.exp(sum(o.log_terms(0, [x], th)) - shift)
    pts = [peak - 60, peak - 10, peak - 1, peak, peak + 1, peak + 15]
    v = integrate.quad(g, -np.inf, pts[0], limit=400, epsabs=0, epsrel=1e-12)[0]
    v += sum(integrate.quad(g, a, b, limit=400, epsabs=0, epsrel=1e-13)[0] for a, b in zip(pts, pts[1:]))
    return abs(o.marginal_terms(th)[0] - (shift + math.log(v))) < 1e-9


def pin_theta_substeps(path, rr):
    wl = synth.gamma_lf_1d(n=60, seed=31, fth=389.75)
    K, gamma = 2, 2.0 / 3.0
    o = oracle.Oracle(wl, lib_path=path, theta_substeps=K)
    st = o.initial_state()
    o.run(st, 4)
    k = st.k + 1
    theta, low = st.theta.copy(), st.chol_theta.copy()
    st.k = k
    for j in range(K):
        z = np.array([oracle.variates(o.seed, [j, k, 1, r // 4], lib_path=path)[1][r % 4] for r in range(o.p)])
        prop = theta + low @ z
        delta = -math.inf
        if np.isfinite(o.log_prior(prop)):
            delta = (o.log_prior(prop) + o.pop_sum(prop, st.chi) - o.n * o.log_Z(prop)) - \
                    (o.log_prior(theta) + o.pop_sum(theta, st.chi) - o.n * o.log_Z(theta))
        ln_u = math.log(oracle.variates(o.seed, [j, k, 2, 0], lib_path=path)[0][4])
        alpha = 1.0 if delta >= 0 else math.exp(delta)
        if ln_u < delta:
            theta = prop
        c = ((k - 1) * K + j + 2) ** -gamma * (alpha - 0.4)
        low = np.linalg.cholesky(low @ (np.eye(o.p) + c * np.outer(z, z) / (z @ z)) @ low.T)
    o.theta_step(st)
    return np.allclose(st.theta, theta, rtol=0, atol=1e-12) and np.allclose(st.chol_theta, low, rtol=1e-10, atol=1e-13)


MUTATIONS = [
    ("philox multiplier", "0xD2511F53u", "0xD2511F57u", pin_philox),
    ("philox key bump", "k1 += weyl1;", "k1 += weyl0;", pin_philox),
    ("field cut offset", "(v >> (24 * j)) & 0xffffffu", "(v >> (24 * j + 1)) & 0xffffffu", pin_fields),
    ("box-muller radius", "double r0 = sqrt(-2.0 * log(u[0]));", "double r0 = sqrt(-log(u[0]));", pin_normals),
    ("gamma jacobian dropped", "return a * (x - ln_lstar) - exp(x - ln_lstar) - lgamma(a);",
     "return (a - 1.0) * (x - ln_lstar) - exp(x - ln_lstar) - lgamma(a);", pin_gamma_density),
    ("gamma normaliser sign", "return a * (x - ln_lstar) - exp(x - ln_lstar) - lgamma(a);",
     "return a * (x - ln_lstar) - exp(x - ln_lstar) + lgamma(a);", pin_gamma_density),
    ("covariance inverse cofactor sign", "c->cinv[1] = -(a[1] * a[8] - a[2] * a[7]) / det;",
     "c->cinv[1] = (a[1] * a[8] - a[2] * a[7]) / det;", pin_mvn_density),
    ("efficiency weight e^t dropped", "sum += c->qv[l] * exp(c->qt[l]) * detect_eff(c, flux);",
     "sum += c->qv[l] * detect_eff(c, flux);", pin_efficiency),
    ("cholesky transposed operand", "s -= low[i * q + k] * low[j * q + k];",
     "s -= low[k * q + i] * low[k * q + j];", pin_ram_one_step),
    ("RAM adaptation sign", "ram_adapt(d, s_mat, uvec, eta * (alpha - c->alpha_star));",
     "ram_adapt(d, s_mat, uvec, eta * (c->alpha_star - alpha));", pin_acceptance_fixed_point),
    ("accept test without log", "int accepted = ln_u < delta;", "int accepted = u[4] < delta;",
     pin_acceptance_fixed_point),
    ("tau prior dropped", "        return theta[1];", "        return 0.0;", pin_theta_given_chi),
    ("selection term dropped", "- (double)c->n * orc_log_Z(c, prop);", ";", pin_selection_in_theta_step),
    ("bb1 jacobian dropped", "return orc_bb1_log_norm(beta, ln_l, ln_u) + (beta + 1.0) * (x - ln_u)",
     "return orc_bb1_log_norm(beta, ln_l, ln_u) + beta * (x - ln_u)", pin_bb1_normalisation),
    ("bb1 break factor", "log(-expm1(-exp(x - ln_l)))", "log(-expm1(-exp(ln_l - x)))", pin_bb1_normalisation),
    ("bb1 normaliser sign", "return -log(g * f);", "return log(g * f);", pin_bb1_normalisation),
    ("bb1 normaliser ratio", "double q = 1.0 + exp(ln_u - ln_l);", "double q = 1.0 + exp(ln_l - ln_u);",
     pin_bb1_normalisation),
    ("bb1 sigma(F) normaliser dropped", "*log_meas = -0.5 * ((fhat - flux) / sig) * ((fhat - flux) / sig) - log(sig);",
     "*log_meas = -0.5 * ((fhat - flux) / sig) * ((fhat - flux) / sig);", pin_bb1_member_likelihood),
    ("bb1 constant error in the efficiency", "double sig = c->model == ORC_BB1 ? bb1_sigma(c, flux) : c->consts[1];",
     "double sig = c->consts[1];", pin_bb1_efficiency),
    ("bb1 prior l factor", "return theta[1] - log(1.0 + theta[0] * theta[0]);",
     "return -theta[1] - log(1.0 + theta[0] * theta[0]);", pin_bb1_prior),
    ("marginal scale not restored", "out[i] = shift + log(total);", "out[i] = log(total);", pin_marginal_nn1d),
    ("marginal panel half-width", "sum += 0.5 * width * w20[j]", "sum += width * w20[j]", pin_marginal_nn1d),
    ("marginal normal-normal centre", "centre = (y / (sig * sig) + theta[0] / (tau * tau)) / prec;",
     "centre = y;", pin_marginal_nn1d),
    ("marginal tail panel dropped", "double total = gl_composite(c, i, theta, shift, centre - 200.0, lo, 0.25, t20, w20)",
     "double total = 0.0 * gl_composite(c, i, theta, shift, centre - 200.0, lo, 0.25, t20, w20)", pin_marginal_bb1),
    ("theta sub-step normals reuse the first block", "uint32_t ctr[4] = {(uint32_t)j, (uint32_t)k, 1u, (uint32_t)(r / 4)};",
     "uint32_t ctr[4] = {0u, (uint32_t)k, 1u, (uint32_t)(r / 4)};", pin_theta_substeps),
    ("theta sub-step adaptation counts cycles", "int64_t n = (k - 1) * (int64_t)c->theta_substeps + j + 1;",
     "int64_t n = k;", pin_theta_substeps),
    ("marginal power tail cut at 200 e-folds", "if (top < feature - 40.0 && !(add > 1e-17 * total))",
     "if (1)", pin_marginal_bb1_slow_tail),
]


@pytest.mark.parametrize("name,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(tmp_path, rocrand_bin, name, old, new, pin):
    src = oracle.source()
    assert src.count(old) >= 1, f"mutation site not found: {old}"
    bad = oracle.build_variant(src.replace(old, new, 1), str(tmp_path / "liboracle_bad.so"))
    assert not pin(bad, rocrand_bin), f"pin did not catch: {name}"


@pytest.mark.parametrize("pin", sorted({m[3] for m in MUTATIONS}, key=lambda f: f.__name__),
                         ids=lambda f: f.__name__)
def test_pins_hold_on_the_real_oracle(rocrand_bin, pin):
    oracle.build(force=False)
    assert pin(oracle.LIB_PATH, rocrand_bin)
