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


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        d, i64, u64, i32, u32 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32
        P = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_variates.argtypes = [u64, P, P, P]
        L.orc_gauss_legendre.argtypes = [i32, d, d, P, P]
        L.orc_new.argtypes = [i32, i64, P, P, u64, d, d, d, i32, i32]
        L.orc_new.restype = P
        L.orc_free.argtypes = [P]
        L.orc_log_terms.argtypes = [P, i64, P, P, P, P]
        L.orc_log_prior.argtypes = [P, P]
        L.orc_log_prior.restype = d
        L.orc_log_Z.argtypes = [P, P]
        L.orc_log_Z.restype = d
        L.orc_eps.argtypes = [P, d]
        L.orc_eps.restype = d
        L.orc_pop_sum.argtypes = [P, P, P]
        L.orc_pop_sum.restype = d
        L.orc_pop_terms.argtypes = [P, P, P, P]
        L.orc_log_post.argtypes = [P, P, P, P]
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = i32
        L.orc_sweep.argtypes = [P, i64, P, P, P, P, P]
        L.orc_theta_proposal.argtypes = [P, i64, P, P, P]
        L.orc_theta_step.argtypes = [P, i64, P, P, P, P]
        L.orc_theta_step.restype = i32
        L.orc_run.argtypes = [P, i64, i64, P, P, P, P, P, P, P, i64, i32, i32]
        _ = u32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def variates(seed: int, ctr):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    u = np.zeros(5)
    z = np.zeros(4)
    lib().orc_variates(ctypes.c_uint64(seed), _ptr(c), _ptr(u), _ptr(z))
    return u, z


def num_threads() -> int:
    return int(lib().orc_num_threads())


def gauss_legendre(n: int, a: float, b: float):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre(n, a, b, _ptr(x), _ptr(w))
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
                 alpha_star_theta: float = 0.4, adapt_theta: bool = True, seed=None):
        self.wl = wl
        self.n, self.d, self.p = wl.n, wl.d, wl.p
        self.alpha_star = wl.alpha_star if alpha_star is None else alpha_star
        data = np.ascontiguousarray(wl.data, dtype=np.float64)
        consts = np.ascontiguousarray(wl.consts, dtype=np.float64)
        self.seed = wl.seed if seed is None else seed
        self._h = lib().orc_new(wl.model, wl.n, _ptr(data), _ptr(consts), ctypes.c_uint64(self.seed),
                                self.alpha_star, gamma, alpha_star_theta, int(adapt_theta), nq)
        if not self._h:
            raise ValueError("oracle: unknown model")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
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
        lib().orc_log_terms(self._h, i, _ptr(xv), _ptr(th), ctypes.byref(lm), ctypes.byref(lp))
        return lm.value, lp.value

    def log_prior(self, theta) -> float:
        return lib().orc_log_prior(self._h, _ptr(np.ascontiguousarray(theta, dtype=np.float64)))

    def log_Z(self, theta) -> float:
        return lib().orc_log_Z(self._h, _ptr(np.ascontiguousarray(theta, dtype=np.float64)))

    def eps(self, x: float) -> float:
        return lib().orc_eps(self._h, float(x))

    def pop_sum(self, theta, chi) -> float:
        th = np.ascontiguousarray(theta, dtype=np.float64)
        c = np.ascontiguousarray(chi, dtype=np.float64)
        return lib().orc_pop_sum(self._h, _ptr(th), _ptr(c))

    def pop_terms(self, theta, chi) -> np.ndarray:
        th = np.ascontiguousarray(theta, dtype=np.float64)
        c = np.ascontiguousarray(chi, dtype=np.float64)
        out = np.zeros(self.n)
        lib().orc_pop_terms(self._h, _ptr(th), _ptr(c), _ptr(out))
        return out

    def log_post(self, theta, pts) -> np.ndarray:
        """log l_i(x_i) + log f(x_i; theta) for every object at points pts [d][n]."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        x = np.ascontiguousarray(pts, dtype=np.float64)
        out = np.zeros(self.n)
        lib().orc_log_post(self._h, _ptr(th), _ptr(x), _ptr(out))
        return out

    def pop_loglik(self, theta, chi) -> float:
        """sum_i log f(chi_i; theta) - N log Z(theta)."""
        return self.pop_sum(theta, chi) - self.n * self.log_Z(theta)

    # -- steps ------------------------------------------------------------
    def sweep(self, st: State, theta=None, trace: bool = False, k=None):
        """One RAM sweep in place; returns the [n][5] trace when asked."""
        kk = st.k + 1 if k is None else k
        th = np.ascontiguousarray(st.theta if theta is None else theta, dtype=np.float64)
        tr = np.zeros((self.n, 5)) if trace else None
        lib().orc_sweep(self._h, kk, _ptr(th), _ptr(st.chi), _ptr(st.chol), _ptr(st.acc),
                        _ptr(tr) if trace else None)
        st.k = kk
        return tr

    def theta_proposal(self, st: State, k=None) -> np.ndarray:
        kk = st.k if k is None else k
        out = np.zeros(self.p)
        lib().orc_theta_proposal(self._h, kk, _ptr(st.theta), _ptr(st.chol_theta), _ptr(out))
        return out

    def theta_step(self, st: State, k=None):
        """Theta step of cycle k (default: the sweep just done).  Returns info dict."""
        kk = st.k if k is None else k
        info = np.zeros(6)
        lib().orc_theta_step(self._h, kk, _ptr(st.theta), _ptr(st.chol_theta), _ptr(st.chi), _ptr(info))
        return {"delta": info[0], "ln_u": info[1], "accepted": bool(info[2]), "alpha": info[3],
                "sum_prop": info[4], "sum_cur": info[5]}

    def run(self, st: State, n_cycles: int, thin: int = 0, fix_theta: bool = False,
            fix_chi: bool = False, chi_trace: bool = False):
        """n_cycles MWG cycles in place; returns (theta_trace [n_cycles][p], chi_trace or None)."""
        tt = np.zeros((n_cycles, self.p))
        ct = None
        if chi_trace and thin > 0:
            n_snap = (st.k + n_cycles) // thin - st.k // thin
            ct = np.zeros((n_snap, self.d, self.n))
        lib().orc_run(self._h, st.k, n_cycles, _ptr(st.theta), _ptr(st.chol_theta), _ptr(st.chi),
                      _ptr(st.chol), _ptr(st.acc), _ptr(tt), _ptr(ct) if ct is not None else None,
                      thin, int(fix_theta), int(fix_chi))
        st.k += n_cycles
        return tt, ct
