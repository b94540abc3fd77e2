"""Python binding of the MI355X sampler library (``lib/libhbm.so``).

Argument marshalling only: every step of the sampler runs in the library's
HIP kernels.  PyTorch provides device memory and streams.  The library must
be built (``build.py``); nothing here falls back to another implementation.

Low-level functions carry the C ABI names (``init_chains``, ``ram_sweep``,
``pop_loglik``, ``theta_step``, ``get_samples`` ...).  :class:`Sampler` wraps
them for one dataset held in torch tensors.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch  # imported first so the library binds to torch's HIP runtime

from .build import LIB_PATH

HBM_OK, HBM_EINVAL, HBM_ENOMEM, HBM_EHIP, HBM_EDOMAIN, HBM_ESTATE, HBM_ENOSPACE = 0, -1, -2, -3, -4, -5, -6
HBM_NORMAL_NORMAL_1D, HBM_GAMMA_LF_1D, HBM_GAMMA_LF_COLOR_3D, HBM_NORMAL_NORMAL_3D = 1, 2, 3, 4
HBM_FP64, HBM_FP32 = 1, 2

EXPORTED = ("init_chains", "ram_sweep", "pop_loglik", "theta_step", "run_cycles", "get_samples",
            "get_theta", "set_theta", "ram_sweep_trace", "get_stats", "kernel_timing",
            "read_kernel_timing", "last_error", "destroy_chains")

_MODEL_DIMS = {  # model -> (d, p, m, precision)
    HBM_NORMAL_NORMAL_1D: (1, 2, 2, HBM_FP64),
    HBM_GAMMA_LF_1D: (1, 2, 2, HBM_FP32),
    HBM_GAMMA_LF_COLOR_3D: (3, 5, 3, HBM_FP32),
    HBM_NORMAL_NORMAL_3D: (3, 3, 3, HBM_FP64),
}


class HbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hbm status {status}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_objects", ctypes.c_int64),
        ("seed", ctypes.c_uint64), ("target_accept", ctypes.c_double), ("eta_exponent", ctypes.c_double),
        ("s0", ctypes.c_double), ("theta_target_accept", ctypes.c_double), ("adapt_theta", ctypes.c_int32),
        ("n_quad", ctypes.c_int32), ("thin_chi", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("max_cycles", ctypes.c_int64), ("theta_chol0", ctypes.c_double * 25), ("model_consts", ctypes.c_double * 16),
    ]


class Buffers(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("chi", ctypes.c_void_p), ("chol", ctypes.c_void_p),
                ("acc", ctypes.c_void_p), ("chi_samples", ctypes.c_void_p)]


_lib = None


def lib():
    """Load the built library; raises if it is missing (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run paper_2105_08026_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "init_chains": [P, P, P, P, P, P],
            "ram_sweep": [P, i32, P],
            "pop_loglik": [P, P, P],
            "theta_step": [P, P],
            "run_cycles": [P, i64, i32],
            "get_samples": [P, i64, i64, P, P, P],
            "get_theta": [P, P, P, P],
            "set_theta": [P, P, P, i64],
            "ram_sweep_trace": [P, P],
            "get_stats": [P, P],
            "kernel_timing": [P, i32],
            "read_kernel_timing": [P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.last_error.argtypes = [P]
        L.last_error.restype = ctypes.c_char_p
        L.destroy_chains.argtypes = [P]
        L.destroy_chains.restype = None
        _ = d
        _lib = L
    return _lib


def _check(status: int, ctx=None):
    if status != HBM_OK:
        msg = lib().last_error(ctx)
        raise HbmError(status, msg.decode() if msg else "")


def _arr(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# -- C ABI mirrors ------------------------------------------------------------

def init_chains(config: Config, buffers: Buffers, chi0: Optional[np.ndarray], theta0, stream: int = 0):
    ctx = ctypes.c_void_p()
    c0 = None if chi0 is None else _arr(chi0)
    t0 = _arr(theta0)
    st = lib().init_chains(ctypes.byref(config), ctypes.byref(buffers), None if c0 is None else _ptr(c0),
                           _ptr(t0), ctypes.c_void_p(stream), ctypes.byref(ctx))
    _check(st, None)
    return ctx


def ram_sweep(ctx, n_sweeps: int = 1, rate: bool = False):
    r = ctypes.c_double()
    _check(lib().ram_sweep(ctx, n_sweeps, ctypes.byref(r) if rate else None), ctx)
    return r.value if rate else None


def pop_loglik(ctx, theta) -> float:
    out = ctypes.c_double()
    _check(lib().pop_loglik(ctx, _ptr(_arr(theta)), ctypes.byref(out)), ctx)
    return out.value


def theta_step(ctx) -> bool:
    acc = ctypes.c_int32()
    _check(lib().theta_step(ctx, ctypes.byref(acc)), ctx)
    return bool(acc.value)


def run_cycles(ctx, n_cycles: int, use_graph: bool = True):
    _check(lib().run_cycles(ctx, n_cycles, int(use_graph)), ctx)


def get_samples(ctx, first: int, count: int, p: int, chi_shape=None, chi_dtype=None):
    """Returns (theta rows [count][p], latent snapshots [count][d][N] or None)."""
    th = np.zeros((count, p))
    ch = None if chi_shape is None else np.zeros((count, *chi_shape), dtype=chi_dtype)
    nw = ctypes.c_int64()
    if count > 0:
        _check(lib().get_samples(ctx, first, count, _ptr(th), None, ctypes.byref(nw)), ctx)
        if ch is not None:
            _check(lib().get_samples(ctx, first, count, None, _ptr(ch), ctypes.byref(nw)), ctx)
    return th, ch


def n_theta_samples(ctx) -> int:
    nw = ctypes.c_int64()
    _check(lib().get_samples(ctx, 0, 0, None, None, ctypes.byref(nw)), ctx)
    return nw.value


def get_theta(ctx, p: int):
    th = np.zeros(p)
    ch = np.zeros((p, p))
    k = ctypes.c_int64()
    _check(lib().get_theta(ctx, _ptr(th), _ptr(ch), ctypes.byref(k)), ctx)
    return th, ch, k.value


def set_theta(ctx, theta, chol_theta, k: int):
    _check(lib().set_theta(ctx, _ptr(_arr(theta)), _ptr(_arr(chol_theta)), k), ctx)


def ram_sweep_trace(ctx, trace_ptr: int):
    _check(lib().ram_sweep_trace(ctx, ctypes.c_void_p(trace_ptr)), ctx)


def get_stats(ctx) -> dict:
    out = np.zeros(8)
    _check(lib().get_stats(ctx, _ptr(out)), ctx)
    keys = ("sum_lf", "sum_dlf", "logZ_cur", "logZ_prop", "delta", "alpha", "n_acc", "accepted")
    return dict(zip(keys, out.tolist()))


def kernel_timing(ctx, enable: bool):
    _check(lib().kernel_timing(ctx, int(enable)), ctx)


def read_kernel_timing(ctx):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib().read_kernel_timing(ctx, ctypes.byref(n), ctypes.byref(ms)), ctx)
    return n.value, ms.value


def destroy_chains(ctx):
    if ctx:
        lib().destroy_chains(ctx)


# -- convenience wrapper -------------------------------------------------------

class Sampler:
    """One dataset's chains: torch-owned device buffers plus a library context.

    ``wl`` is a workload from :mod:`synth` (data arrays, constants, theta0,
    chi0).  Buffers: data [m][N], chi [d][N], chol [d(d+1)/2][N], acc [N]
    (int32 storage of the uint32 counters), snapshots [max_cycles/thin][d][N].
    """

    def __init__(self, wl, device: str = "cuda:0", max_cycles: int = 10000, thin: int = 0, s0: float = 1.0,
                 adapt_theta: bool = True, n_quad: int = 512, gamma: float = 2.0 / 3.0,
                 alpha_star_theta: float = 0.4, stream: Optional[torch.cuda.Stream] = None, seed=None):
        d, p, m, prec = _MODEL_DIMS[wl.model]
        self.wl, self.d, self.p, self.n = wl, d, p, wl.n
        self.dtype = torch.float64 if prec == HBM_FP64 else torch.float32
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.data = torch.as_tensor(np.ascontiguousarray(wl.data), dtype=self.dtype, device=self.device)
            self.chi = torch.empty((d, wl.n), dtype=self.dtype, device=self.device)
            self.chol = torch.empty((d * (d + 1) // 2, wl.n), dtype=self.dtype, device=self.device)
            self.acc = torch.empty((wl.n,), dtype=torch.int32, device=self.device)
            n_snap = max_cycles // thin if thin > 0 else 0
            self.snaps = torch.empty((max(n_snap, 1), d, wl.n), dtype=self.dtype, device=self.device) if n_snap else None
        cfg = Config()
        cfg.model, cfg.precision, cfg.n_objects = wl.model, prec, wl.n
        cfg.seed = int(wl.seed if seed is None else seed)
        cfg.target_accept, cfg.eta_exponent, cfg.s0 = wl.alpha_star, gamma, s0
        cfg.theta_target_accept, cfg.adapt_theta = alpha_star_theta, int(adapt_theta)
        cfg.n_quad, cfg.thin_chi, cfg.max_cycles = n_quad, thin, max_cycles
        ch0 = np.asarray(wl.theta_chol0, dtype=np.float64)
        for r in range(p):
            for q in range(p):
                cfg.theta_chol0[r * p + q] = ch0[r, q] if q <= r else 0.0
        for j in range(16):
            cfg.model_consts[j] = float(wl.consts[j])
        self.config = cfg
        bufs = Buffers(self.data.data_ptr(), self.chi.data_ptr(), self.chol.data_ptr(), self.acc.data_ptr(),
                       self.snaps.data_ptr() if self.snaps is not None else None)
        self.buffers = bufs
        torch.cuda.synchronize(self.device)
        with torch.cuda.device(self.device):
            self.ctx = init_chains(cfg, bufs, wl.chi0, wl.theta0, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "ctx", None):
            destroy_chains(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # methods mirror the ABI
    def ram_sweep(self, n: int = 1, rate: bool = False):
        return ram_sweep(self.ctx, n, rate)

    def theta_step(self) -> bool:
        return theta_step(self.ctx)

    def run_cycles(self, n: int, use_graph: bool = True):
        run_cycles(self.ctx, n, use_graph)

    def pop_loglik(self, theta) -> float:
        return pop_loglik(self.ctx, theta)

    def theta(self):
        return get_theta(self.ctx, self.p)

    def set_theta(self, theta, chol_theta, k: int):
        set_theta(self.ctx, theta, chol_theta, k)

    def stats(self) -> dict:
        return get_stats(self.ctx)

    def theta_trace(self) -> np.ndarray:
        n = n_theta_samples(self.ctx)
        return get_samples(self.ctx, 0, n, self.p)[0]

    def chi_snapshots(self, first: int, count: int) -> np.ndarray:
        npdt = np.float64 if self.dtype == torch.float64 else np.float32
        nw = ctypes.c_int64()
        out = np.zeros((count, self.d, self.n), dtype=npdt)
        _check(lib().get_samples(self.ctx, first, count, None, _ptr(out), ctypes.byref(nw)), self.ctx)
        return out

    def trace_sweep(self) -> np.ndarray:
        """One sweep returning per-object (log pi(X), log pi(Y), accepted, Y[0..d-1]) as float64 [3 + d][N]."""
        tr = torch.empty((3 + self.d, self.n), dtype=self.dtype, device=self.device)
        ram_sweep_trace(self.ctx, tr.data_ptr())
        return tr.double().cpu().numpy()

    def state(self):
        """Host copies of (chi [d][N], chol [nc][N], acc [N] uint32)."""
        torch.cuda.synchronize(self.device)
        return (self.chi.double().cpu().numpy(), self.chol.double().cpu().numpy(),
                self.acc.cpu().numpy().view(np.uint32))

    def load_state(self, chi, chol, acc):
        """Overwrite the latent buffers from host arrays (lockstep replay)."""
        with torch.no_grad():
            self.chi.copy_(torch.as_tensor(np.asarray(chi), dtype=self.dtype))
            self.chol.copy_(torch.as_tensor(np.asarray(chol), dtype=self.dtype))
            self.acc.copy_(torch.as_tensor(np.asarray(acc).astype(np.uint32).view(np.int32)))
        torch.cuda.synchronize(self.device)
