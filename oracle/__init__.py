"""Python handle on the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, literal statement of the
sampler that the GPU library is checked against; it shares no code with the
library.  Only the tests, the smoke check and the bench's CPU-baseline leg
may import this package.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over objects)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_libs = {}


def lib(path: str = None):
    """The oracle library at ``path`` (default: the one built here), typed for ctypes."""
    path = path or LIB_PATH
    if path not in _libs:
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(path)
        d, i64, u64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        P = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_variates.argtypes = [u64, P, P, P]
        L.orc_gauss_legendre.argtypes = [i32, d, d, P, P]
        L.orc_new.argtypes = [i32, i64, P, P, u64, d, d, d, i32, i32]
        L.orc_new.restype = P
        L.orc_set_theta_substeps.argtypes = [P, i32]
        L.orc_set_theta_substeps.restype = None
        L.orc_free.argtypes = [P]
        L.orc_log_terms.argtypes = [P, i64, P, P, P, P]
        L.orc_log_prior.argtypes = [P, P]
        L.orc_log_prior.restype = d
        L.orc_log_Z.argtypes = [P, P]
        L.orc_log_Z.restype = d
        L.orc_eps.argtypes = [P, d]
        L.orc_eps.restype = d
        L.orc_bb1_log_norm.argtypes = [d, d, d]
        L.orc_bb1_log_norm.restype = d
        L.orc_pop_sum.argtypes = [P, P, P]
        L.orc_pop_sum.restype = d
        L.orc_pop_terms.argtypes = [P, P, P, P]
        L.orc_log_post.argtypes = [P, P, P, P]
        L.orc_marginal_terms.argtypes = [P, P, P]
        L.orc_marginal_terms.restype = i32
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.argtypes = [i32]
        L.orc_set_num_threads.restype = None
        L.orc_sweep.argtypes = [P, i64, P, P, P, P, P]
        L.orc_theta_proposal.argtypes = [P, i64, P, P, P]
        L.orc_theta_step.argtypes = [P, i64, P, P, P, P]
        L.orc_theta_step.restype = i32
        L.orc_run.argtypes = [P, i64, i64, P, P, P, P, P, P, P, i64, i32, i32]
        _libs[path] = L
    return _libs[path]


def build_variant(src_text: str, out_path: str) -> str:
    """Compile oracle source text (e.g. a deliberately altered copy) to ``out_path``."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-I", _HERE,
                    "-o", out_path, src, "-lm"], check=True)
    return out_path


def source() -> str:
    with open(_SRC) as f:
        return f.read()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key, lib_path: str = None) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib(lib_path).orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def variates(seed: int, ctr, lib_path: str = None):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    u = np.zeros(5)
    z = np.zeros(4)
    lib(lib_path).orc_variates(ctypes.c_uint64(seed), _ptr(c), _ptr(u), _ptr(z))
    return u, z


def bb1_log_norm(beta: float, ln_l: float, ln_u: float, lib_path: str = None) -> float:
    """ln C(beta, u, l) of the break-by-one luminosity PDF."""
    return float(lib(lib_path).orc_bb1_log_norm(beta, ln_l, ln_u))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int):
    lib().orc_set_num_threads(int(n))


def gauss_legendre(n: int, a: float, b: float, lib_path: str = None):
    x = np.zeros(n)
    w = np.zeros(n)
    lib(lib_path).orc_gauss_legendre(n, a, b, _ptr(x), _ptr(w))
    return x, w


@dataclasses.dataclass
class State:
    """Complete chain state: latents, RAM factors, acceptance counts, theta, theta factor, sweep index."""
    chi: np.ndarray          # [d][n] float64
    chol: np.ndarray         # [d(d+1)/2][n] float64, packed lower row-major
    acc: np.ndarray          # [n] uint32
    theta: np.ndarray        # [p]
    chol_theta: np.ndarray   # [p][p]
    k: int = 0               # sweeps completed

    def copy(self) -> "State":
        return State(self.chi.copy(), self.chol.copy(), self.acc.copy(), self.theta.copy(),
                     self.chol_theta.copy(), self.k)


class Oracle:
    """FP64 reference sampler for one dataset (a :class:`synth.workloads.Workload`)."""

    def __init__(self, wl, nq: int = 512, gamma: float = 2.0 / 3.0, alpha_star=None,
                 alpha_star_theta: float = 0.4, adapt_theta: bool = True, seed=None, lib_path: str = None,
                 theta_substeps: int = 1):
        self._L = lib(lib_path)
        self.wl = wl
        self.n, self.d, self.p = wl.n, wl.d, wl.p
        self.alpha_star = wl.alpha_star if alpha_star is None else alpha_star
        self.gamma = gamma
        data = np.ascontiguousarray(wl.data, dtype=np.float64)
        consts = np.ascontiguousarray(wl.consts, dtype=np.float64)
        self.seed = wl.seed if seed is None else seed
        self._h = self._L.orc_new(wl.model, wl.n, _ptr(data), _ptr(consts), ctypes.c_uint64(self.seed),
                                self.alpha_star, gamma, alpha_star_theta, int(adapt_theta), nq)
        if not self._h:
            raise ValueError("oracle: unknown model")
        self.theta_substeps = max(1, int(theta_substeps))
        self._L.orc_set_theta_substeps(self._h, self.theta_substeps)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_free(h)
            self._h = None

    # -- state ----------------------------------------------------------
    def initial_state(self, s0: float = 1.0) -> State:
        d, n = self.d, self.n
        chol = np.zeros((d * (d + 1) // 2, n))
        e = 0
        for r in range(d):
            for s in range(r + 1):
                if r == s:
                    chol[e] = s0
                e += 1
        return State(np.ascontiguousarray(self.wl.chi0, dtype=np.float64).copy(), chol,
                     np.zeros(n, dtype=np.uint32), self.wl.theta0.astype(np.float64).copy(),
                     np.ascontiguousarray(self.wl.theta_chol0, dtype=np.float64).copy(), 0)

    # -- densities --------------------------------------------------------
    def log_terms(self, i: int, x, theta):
        xv = np.ascontiguousarray(x, dtype=np.float64)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        lm = ctypes.c_double()
        lp = ctypes.c_double()
        self._L.orc_log_terms(self._h, i, _ptr(xv), _ptr(th), ctypes.byref(lm), ctypes.byref(lp))
        return lm.value, lp.value

    def log_prior(self, theta) -> float:
        return self._L.orc_log_prior(self._h, _ptr(np.ascontiguousarray(theta, dtype=np.float64)))

    def log_Z(self, theta) -> float:
        return self._L.orc_log_Z(self._h, _ptr(np.ascontiguousarray(theta, dtype=np.float64)))

    def eps(self, x: float) -> float:
        return self._L.orc_eps(self._h, float(x))

    def pop_sum(self, theta, chi) -> float:
        th = np.ascontiguousarray(theta, dtype=np.float64)
        c = np.ascontiguousarray(chi, dtype=np.float64)
        return self._L.orc_pop_sum(self._h, _ptr(th), _ptr(c))

    def pop_terms(self, theta, chi) -> np.ndarray:
        th = np.ascontiguousarray(theta, dtype=np.float64)
        c = np.ascontiguousarray(chi, dtype=np.float64)
        out = np.zeros(self.n)
        self._L.orc_pop_terms(self._h, _ptr(th), _ptr(c), _ptr(out))
        return out

    def log_post(self, theta, pts) -> np.ndarray:
        """log l_i(x_i) + log f(x_i; theta) for every object at points pts [d][n]."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        x = np.ascontiguousarray(pts, dtype=np.float64)
        out = np.zeros(self.n)
        self._L.orc_log_post(self._h, _ptr(th), _ptr(x), _ptr(out))
        return out

    def marginal_terms(self, theta) -> np.ndarray:
        """Per object: ln of the integral over chi of l_i(chi) f(chi; theta) (1-D latents)."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        out = np.zeros(self.n)
        if self._L.orc_marginal_terms(self._h, _ptr(th), _ptr(out)) != 0:
            raise ValueError("oracle: marginal likelihood needs a 1-D latent")
        return out

    def marginal_loglik(self, theta) -> float:
        """sum_i ln int l_i f dchi - N ln Z(theta): the latent-free log-likelihood of theta."""
        return float(np.sum(self.marginal_terms(theta))) - self.n * self.log_Z(theta)

    def pop_loglik(self, theta, chi) -> float:
        """sum_i log f(chi_i; theta) - N log Z(theta)."""
        return self.pop_sum(theta, chi) - self.n * self.log_Z(theta)

    # -- steps ------------------------------------------------------------
    def sweep(self, st: State, theta=None, trace: bool = False, k=None):
        """One RAM sweep in place; returns the [n][5] trace when asked."""
        kk = st.k + 1 if k is None else k
        th = np.ascontiguousarray(st.theta if theta is None else theta, dtype=np.float64)
        tr = np.zeros((self.n, 5)) if trace else None
        self._L.orc_sweep(self._h, kk, _ptr(th), _ptr(st.chi), _ptr(st.chol), _ptr(st.acc),
                        _ptr(tr) if trace else None)
        st.k = kk
        return tr

    def theta_proposal(self, st: State, k=None) -> np.ndarray:
        kk = st.k if k is None else k
        out = np.zeros(self.p)
        self._L.orc_theta_proposal(self._h, kk, _ptr(st.theta), _ptr(st.chol_theta), _ptr(out))
        return out

    def theta_step(self, st: State, k=None):
        """Theta step of cycle k (default: the sweep just done).  Returns info dict."""
        kk = st.k if k is None else k
        info = np.zeros(6 + 2 * self.p)
        self._L.orc_theta_step(self._h, kk, _ptr(st.theta), _ptr(st.chol_theta), _ptr(st.chi), _ptr(info))
        return {"delta": info[0], "ln_u": info[1], "accepted": bool(info[2]), "alpha": info[3],
                "sum_prop": info[4], "sum_cur": info[5], "n_accepted": int(info[2]),
                "prop_last": info[6:6 + self.p].copy(), "theta_before_last": info[6 + self.p:6 + 2 * self.p].copy()}

    def run(self, st: State, n_cycles: int, thin: int = 0, fix_theta: bool = False,
            fix_chi: bool = False, chi_trace: bool = False):
        """n_cycles MWG cycles in place; returns (theta_trace [n_cycles][p], chi_trace or None)."""
        tt = np.zeros((n_cycles, self.p))
        ct = None
        if chi_trace and thin > 0:
            n_snap = (st.k + n_cycles) // thin - st.k // thin
            ct = np.zeros((n_snap, self.d, self.n))
        self._L.orc_run(self._h, st.k, n_cycles, _ptr(st.theta), _ptr(st.chol_theta), _ptr(st.chi),
                      _ptr(st.chol), _ptr(st.acc), _ptr(tt), _ptr(ct) if ct is not None else None,
                      thin, int(fix_theta), int(fix_chi))
        st.k += n_cycles
        return tt, ct
