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
from .serve import TileAllocator

HBM_OK, HBM_EINVAL, HBM_ENOMEM, HBM_EHIP, HBM_EDOMAIN, HBM_ESTATE, HBM_ENOSPACE = 0, -1, -2, -3, -4, -5, -6
HBM_NORMAL_NORMAL_1D, HBM_GAMMA_LF_1D, HBM_GAMMA_LF_COLOR_3D, HBM_NORMAL_NORMAL_3D, HBM_BB1_LF = 1, 2, 3, 4, 5
HBM_FP64, HBM_FP32 = 1, 2
HBM_CYCLES_AUTO, HBM_CYCLES_GRAPH, HBM_CYCLES_FUSED = 0, 1, 2
HBM_NOALLOC_SCRATCH_BYTES = 8 << 20     # the static device array of marginal_loglik_noalloc

EXPORTED = ("init_chains", "init_batch", "create_pool", "load_datasets", "unload_dataset", "slot_info",
            "ram_sweep", "pop_loglik", "marginal_loglik", "marginal_loglik_noalloc", "theta_step", "run_cycles", "prepare_cycles", "set_cycle_mode", "launch_counts", "run_cycles_streamed",
            "fd_sink", "get_samples", "get_theta", "set_theta",
            "ram_sweep_trace", "get_state", "set_state", "get_stats", "set_launch", "set_occupancy", "autotune", "kernel_timing",
            "read_kernel_timing", "last_error", "destroy_chains")

TILE = 256   # objects per tile: datasets in a pool start on multiples of this

_MODEL_DIMS = {  # model -> (d, p, m, precision)
    HBM_NORMAL_NORMAL_1D: (1, 2, 2, HBM_FP64),
    HBM_GAMMA_LF_1D: (1, 2, 2, HBM_FP32),
    HBM_GAMMA_LF_COLOR_3D: (3, 5, 3, HBM_FP32),
    HBM_NORMAL_NORMAL_3D: (3, 3, 3, HBM_FP64),
    HBM_BB1_LF: (1, 3, 2, HBM_FP32),
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
        ("n_quad", ctypes.c_int32), ("thin_chi", ctypes.c_int32), ("tiles_per_group", ctypes.c_int32),
        ("theta_substeps", ctypes.c_int32), ("snap_rows", ctypes.c_int32), ("max_cycles", ctypes.c_int64), ("theta_chol0", ctypes.c_double * 25), ("model_consts", ctypes.c_double * 16),
    ]


class Buffers(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("chi", ctypes.c_void_p), ("chol", ctypes.c_void_p),
                ("acc", ctypes.c_void_p), ("chi_samples", ctypes.c_void_p)]


class PoolConfig(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_slots", ctypes.c_int32),
                ("n_quad", ctypes.c_int32), ("capacity", ctypes.c_int64), ("max_cycles", ctypes.c_int64),
                ("snap_rows", ctypes.c_int64), ("tiles_per_group", ctypes.c_int32), ("stats_theta", ctypes.c_int32)]


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
            "init_batch": [i32, P, P, P, P, P],
            "create_pool": [P, P, P, P],
            "load_datasets": [P, i32, P, P, P, P, P],
            "unload_dataset": [P, i32],
            "slot_info": [P, i32, P],
            "ram_sweep": [P, i32, P],
            "pop_loglik": [P, P, P],
            "marginal_loglik": [P, i32, i32, P, P, P],
            "marginal_loglik_noalloc": [P, i32, i32, P, P, P],
            "theta_step": [P, P],
            "run_cycles": [P, i64, i32],
            "prepare_cycles": [P, i64],
            "set_cycle_mode": [P, i32],
            "launch_counts": [P, P],
            "run_cycles_streamed": [P, i64, i32, SNAPSHOT_SINK, P],
            "get_samples": [P, i32, i64, i64, P, P, P],
            "get_theta": [P, i32, P, P, P],
            "set_theta": [P, i32, P, P, i64],
            "ram_sweep_trace": [P, P],
            "get_stats": [P, i32, P],
            "get_state": [P, P, P],
            "set_state": [P, P, ctypes.c_size_t],
            "set_launch": [P, i32],
            "set_occupancy": [P, i32],
            "autotune": [P, i32, P, P],
            "kernel_timing": [P, i32],
            "read_kernel_timing": [P, P, P],
        }
        L.fd_sink.argtypes = [P, i32, i64, i64, P, i64]
        L.fd_sink.restype = i32
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


def init_batch(configs, buffers: Buffers, theta0s, stream: int = 0):
    arr = (Config * len(configs))(*configs)
    t0 = _arr(theta0s)
    ctx = ctypes.c_void_p()
    _check(lib().init_batch(len(configs), arr, ctypes.byref(buffers), _ptr(t0), ctypes.c_void_p(stream),
                            ctypes.byref(ctx)), None)
    return ctx


def create_pool(pool: PoolConfig, buffers: Buffers, stream: int = 0):
    ctx = ctypes.c_void_p()
    _check(lib().create_pool(ctypes.byref(pool), ctypes.byref(buffers), ctypes.c_void_p(stream), ctypes.byref(ctx)),
           None)
    return ctx


def load_datasets(ctx, slots, obj_starts, configs, theta0s, budgets=None):
    n = len(configs)
    sl = _arr(slots, np.int32)
    os_ = _arr(obj_starts, np.int64)
    arr = (Config * n)(*configs)
    t0 = _arr(theta0s)
    bu = None if budgets is None else _arr(budgets, np.int64)
    _check(lib().load_datasets(ctx, n, _ptr(sl), _ptr(os_), arr, _ptr(t0), None if bu is None else _ptr(bu)), ctx)


def unload_dataset(ctx, slot: int):
    _check(lib().unload_dataset(ctx, slot), ctx)


def slot_info(ctx, slot: int) -> dict:
    out = np.zeros(6, dtype=np.int64)
    _check(lib().slot_info(ctx, slot, _ptr(out)), ctx)
    return dict(zip(("loaded", "active", "k", "n_theta", "obj_start", "n"), out.tolist()))


def ram_sweep(ctx, n_sweeps: int = 1, rate: bool = False, n_slots: int = 1):
    """Sweeps every active slot; with rate=True returns the [n_slots] acceptance rates."""
    r = np.zeros(n_slots)
    _check(lib().ram_sweep(ctx, n_sweeps, _ptr(r) if rate else None), ctx)
    return r if rate else None


def pop_loglik(ctx, thetas) -> np.ndarray:
    """thetas: [n_slots][p]; returns [n_slots] (NaN for free slots)."""
    th = _arr(thetas)
    out = np.zeros(th.shape[0])
    _check(lib().pop_loglik(ctx, _ptr(th), _ptr(out)), ctx)
    return out


def marginal_loglik(ctx, slot: int, thetas, n: int, terms: bool = False, device=None, noalloc: bool = False):
    """thetas: [n_theta][p]; returns [n_theta] latent-free log-likelihoods and,
    with terms=True, also the [n_theta][n] per-object log integrals.
    noalloc=True calls marginal_loglik_noalloc (the library's static scratch)."""
    th = _arr(thetas)
    if th.ndim == 1:
        th = th.reshape(1, -1)
    out = np.zeros(th.shape[0])
    tb = torch.empty((th.shape[0], n), dtype=torch.float64, device=device) if terms else None
    fn = lib().marginal_loglik_noalloc if noalloc else lib().marginal_loglik
    _check(fn(ctx, slot, th.shape[0], _ptr(th), _ptr(out), tb.data_ptr() if terms else None), ctx)
    return (out, tb.cpu().numpy()) if terms else out


def theta_step(ctx, n_slots: int = 1) -> np.ndarray:
    """Returns [n_slots]: 1 accepted, 0 rejected, -1 no step (inactive slot)."""
    acc = np.zeros(n_slots, dtype=np.int32)
    _check(lib().theta_step(ctx, _ptr(acc)), ctx)
    return acc


def run_cycles(ctx, n_cycles: int, use_graph: bool = True):
    _check(lib().run_cycles(ctx, n_cycles, int(use_graph)), ctx)


def prepare_cycles(ctx, n_cycles: int):
    _check(lib().prepare_cycles(ctx, n_cycles), ctx)


def set_cycle_mode(ctx, mode: int):
    _check(lib().set_cycle_mode(ctx, mode), ctx)


def launch_counts(ctx) -> dict:
    out = np.zeros(6, dtype=np.int64)
    _check(lib().launch_counts(ctx, _ptr(out)), ctx)
    return dict(zip(("graph_replays", "replayed_cycles", "plain_cycles", "graph_captures", "persistent_launches",
                     "persistent_cycles"), out.tolist()))


# int32 sink(void *user, int32 slot, int64 first, int64 count, const void *rows, int64 bytes)
SNAPSHOT_SINK = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_int64)


def run_cycles_streamed(ctx, n_cycles: int, chunk_cycles: int, on_rows, row_shape, dtype, copy: bool = True):
    """Runs n_cycles cycles streaming every latent snapshot: on_rows(slot, first,
    rows) receives each slot's new snapshots as a [count][d][N] array
    (row_shape(slot) gives (d, N)) -- its own copy, or with copy=False a view
    of the library's staging valid only during the call; returning True
    stops the run."""
    itemsize = np.dtype(dtype).itemsize

    def _sink(_user, slot, first, count, ptr, nbytes):
        d, n = row_shape(slot)
        assert nbytes == count * d * n * itemsize
        buf = (ctypes.c_char * nbytes).from_address(ptr)
        rows = np.frombuffer(buf, dtype=dtype).reshape(count, d, n)
        return 1 if on_rows(slot, first, rows.copy() if copy else rows) else 0
    cb = SNAPSHOT_SINK(_sink)
    _check(lib().run_cycles_streamed(ctx, n_cycles, chunk_cycles, cb, None), ctx)


def run_cycles_to_fd(ctx, n_cycles: int, chunk_cycles: int, fd: int):
    """Streams every latent snapshot, as raw rows, to an open file descriptor
    through the library's own sink (no Python on the data path)."""
    sink = ctypes.cast(lib().fd_sink, SNAPSHOT_SINK)
    _check(lib().run_cycles_streamed(ctx, n_cycles, chunk_cycles, sink, ctypes.c_void_p(fd)), ctx)


def get_samples(ctx, slot: int, first: int, count: int, p: int, chi_shape=None, chi_dtype=None):
    """Returns (theta rows [count][p], latent snapshots [count][d][N] or None)."""
    th = np.zeros((count, p))
    ch = None if chi_shape is None else np.zeros((count, *chi_shape), dtype=chi_dtype)
    nw = ctypes.c_int64()
    if count > 0:
        _check(lib().get_samples(ctx, slot, first, count, _ptr(th), None, ctypes.byref(nw)), ctx)
        if ch is not None:
            _check(lib().get_samples(ctx, slot, first, count, None, _ptr(ch), ctypes.byref(nw)), ctx)
    return th, ch


def n_theta_samples(ctx, slot: int = 0) -> int:
    nw = ctypes.c_int64()
    _check(lib().get_samples(ctx, slot, 0, 0, None, None, ctypes.byref(nw)), ctx)
    return nw.value


def get_theta(ctx, p: int, slot: int = 0):
    th = np.zeros(p)
    ch = np.zeros((p, p))
    k = ctypes.c_int64()
    _check(lib().get_theta(ctx, slot, _ptr(th), _ptr(ch), ctypes.byref(k)), ctx)
    return th, ch, k.value


def set_theta(ctx, theta, chol_theta, k: int, slot: int = 0):
    _check(lib().set_theta(ctx, slot, _ptr(_arr(theta)), _ptr(_arr(chol_theta)), k), ctx)


def ram_sweep_trace(ctx, trace_ptr: int):
    _check(lib().ram_sweep_trace(ctx, ctypes.c_void_p(trace_ptr)), ctx)


def get_state(ctx) -> bytes:
    """The library-held chain state of every slot (see set_state)."""
    n = ctypes.c_size_t()
    _check(lib().get_state(ctx, None, ctypes.byref(n)), ctx)
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().get_state(ctx, buf, ctypes.byref(n)), ctx)
    return buf.raw[: n.value]


def set_state(ctx, blob: bytes):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(lib().set_state(ctx, buf, len(blob)), ctx)


def get_stats(ctx, slot: int = 0) -> dict:
    out = np.zeros(8)
    _check(lib().get_stats(ctx, slot, _ptr(out)), ctx)
    keys = ("sum_lf", "sum_dlf", "logZ_cur", "logZ_prop", "delta", "alpha", "n_acc", "accepted")
    return dict(zip(keys, out.tolist()))


def set_launch(ctx, tiles_per_group: int):
    _check(lib().set_launch(ctx, tiles_per_group), ctx)


def set_occupancy(ctx, groups_per_cu: int):
    _check(lib().set_occupancy(ctx, groups_per_cu), ctx)


TUNE_CANDIDATES = 13      # HBM_TUNE_CANDIDATES
TUNE_WARM = 8             # warm-up cycles per candidate


def autotune_cycles(trial_cycles: int) -> int:
    """Cycles (theta-trace rows) one autotune call runs."""
    return TUNE_CANDIDATES * (TUNE_WARM + trial_cycles)


def tune_labels():
    """Names of the autotuner's candidates, in its order."""
    return ([f"tpw{t}_cap{c}" for c in (0, 4, 2) for t in (1, 2, 4)] + ["persistent"]
            + [f"fused_tpw{t}" for t in (1, 2, 4)])


def autotune(ctx, trial_cycles: int = 64):
    """Runs autotune_cycles(trial_cycles) real cycles; returns (choice dict,
    us/cycle per candidate in tune_labels() order, NaN where not timed)."""
    ch = np.zeros(3, dtype=np.int32)
    us = np.zeros(TUNE_CANDIDATES)
    _check(lib().autotune(ctx, trial_cycles, _ptr(ch), _ptr(us)), ctx)
    return {"tiles_per_group": int(ch[0]), "groups_per_cu": int(ch[1]), "persistent": int(ch[2]) == 1,
            "fused": int(ch[2]) == 2}, us


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


# -- convenience wrappers ------------------------------------------------------

def make_config(wl, max_cycles: int = 10000, thin: int = 0, s0: float = 1.0, adapt_theta: bool = True,
                n_quad: int = 512, gamma: float = 2.0 / 3.0, alpha_star_theta: float = 0.4, seed=None,
                theta_substeps: int = 0, snap_rows: int = 0) -> Config:
    """The hbm_config of a :mod:`synth` workload.  theta_substeps: 0 for one
    theta step per cycle from the N-term sums, K >= 1 for K steps per cycle
    from sufficient statistics."""
    d, p, m, prec = _MODEL_DIMS[wl.model]
    cfg = Config()
    cfg.model, cfg.precision, cfg.n_objects = wl.model, prec, wl.n
    cfg.seed = int(wl.seed if seed is None else seed)
    cfg.target_accept, cfg.eta_exponent, cfg.s0 = wl.alpha_star, gamma, s0
    cfg.theta_target_accept, cfg.adapt_theta = alpha_star_theta, int(adapt_theta)
    cfg.n_quad, cfg.thin_chi, cfg.max_cycles = n_quad, thin, max_cycles
    cfg.theta_substeps = int(theta_substeps)
    cfg.snap_rows = int(snap_rows)
    ch0 = np.asarray(wl.theta_chol0, dtype=np.float64)
    for r in range(p):
        for q in range(p):
            cfg.theta_chol0[r * p + q] = ch0[r, q] if q <= r else 0.0
    for j in range(16):
        cfg.model_consts[j] = float(wl.consts[j])
    return cfg


def packed_offsets(ns):
    """Object offsets of datasets packed back to back, each on a tile boundary, and the capacity."""
    offs, o = [], 0
    for n in ns:
        offs.append(o)
        o += -(-int(n) // TILE) * TILE
    return offs, (offs[-1] + int(ns[-1]) if ns else 0)


class _Chains:
    """Shared plumbing: torch-owned packed device buffers and a context."""

    def _alloc(self, model: int, cap: int, snap_rows: int, device, stream, snap_host: bool = False):
        d, p, m, prec = _MODEL_DIMS[model]
        self.model, self.d, self.p, self.m, self.cap = model, d, p, m, cap
        self.dtype = torch.float64 if prec == HBM_FP64 else torch.float32
        self.npdtype = np.float64 if prec == HBM_FP64 else np.float32
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.data = torch.zeros((m, cap), dtype=self.dtype, device=self.device)
            self.chi = torch.zeros((d, cap), dtype=self.dtype, device=self.device)
            self.chol = torch.empty((d * (d + 1) // 2, cap), dtype=self.dtype, device=self.device)
            self.acc = torch.empty((cap,), dtype=torch.int32, device=self.device)
            # snapshots in HBM, or in pinned host memory the sweep writes through its device mapping
            self.snaps = None
            if snap_rows > 0:
                self.snaps = (torch.empty((snap_rows, d, cap), dtype=self.dtype, pin_memory=True) if snap_host else
                              torch.empty((snap_rows, d, cap), dtype=self.dtype, device=self.device))
        self.buffers = Buffers(self.data.data_ptr(), self.chi.data_ptr(), self.chol.data_ptr(), self.acc.data_ptr(),
                               self.snaps.data_ptr() if self.snaps is not None else None)

    def close(self):
        if getattr(self, "ctx", None):
            destroy_chains(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run_cycles(self, n: int, use_graph: bool = True):
        run_cycles(self.ctx, n, use_graph)

    def prepare_cycles(self, n: int):
        prepare_cycles(self.ctx, n)

    def launch_counts(self) -> dict:
        return launch_counts(self.ctx)

    def set_cycle_mode(self, mode: int):
        set_cycle_mode(self.ctx, mode)

    def autotune(self, trial_cycles: int = 64):
        return autotune(self.ctx, trial_cycles)

    def set_launch(self, tiles_per_group: int):
        set_launch(self.ctx, tiles_per_group)

    def set_occupancy(self, groups_per_cu: int):
        set_occupancy(self.ctx, groups_per_cu)


class Sampler(_Chains):
    """One dataset's chains: torch-owned device buffers plus a library context.

    ``wl`` is a workload from :mod:`synth` (data arrays, constants, theta0,
    chi0).  Buffers: data [m][N], chi [d][N], chol [d(d+1)/2][N], acc [N]
    (int32 storage of the uint32 counters), snapshots [max_cycles/thin][d][N].
    """

    def __init__(self, wl, device: str = "cuda:0", max_cycles: int = 10000, thin: int = 0, s0: float = 1.0,
                 adapt_theta: bool = True, n_quad: int = 512, gamma: float = 2.0 / 3.0,
                 alpha_star_theta: float = 0.4, stream: Optional[torch.cuda.Stream] = None, seed=None,
                 theta_substeps: int = 0, snap_rows: int = 0, snap_host: bool = False):
        self.wl, self.n = wl, wl.n
        rows = (snap_rows if snap_rows > 0 else max_cycles // thin) if thin > 0 else 0
        self._alloc(wl.model, wl.n, rows, device, stream, snap_host)
        with torch.no_grad():
            self.data.copy_(torch.as_tensor(np.ascontiguousarray(wl.data), dtype=self.dtype))
        self.config = make_config(wl, max_cycles, thin, s0, adapt_theta, n_quad, gamma, alpha_star_theta, seed,
                                  theta_substeps, snap_rows)
        torch.cuda.synchronize(self.device)
        with torch.cuda.device(self.device):
            self.ctx = init_chains(self.config, self.buffers, wl.chi0, wl.theta0, self.stream.cuda_stream)

    # methods mirror the ABI
    def ram_sweep(self, n: int = 1, rate: bool = False):
        r = ram_sweep(self.ctx, n, rate)
        return float(r[0]) if rate else None

    def theta_step(self) -> int:
        """Steps accepted (0 or 1; up to K with K theta sub-steps)."""
        return int(theta_step(self.ctx)[0])

    def pop_loglik(self, theta) -> float:
        return float(pop_loglik(self.ctx, np.asarray(theta, dtype=np.float64).reshape(1, -1))[0])

    def marginal_loglik(self, thetas, terms: bool = False):
        """Latent-free log-likelihood at each row of thetas (1-D latents only)."""
        return marginal_loglik(self.ctx, 0, thetas, self.n, terms, self.device)

    def theta(self):
        return get_theta(self.ctx, self.p)

    def set_theta(self, theta, chol_theta, k: int):
        set_theta(self.ctx, theta, chol_theta, k)

    def stats(self) -> dict:
        return get_stats(self.ctx)

    def theta_trace(self) -> np.ndarray:
        n = n_theta_samples(self.ctx)
        return get_samples(self.ctx, 0, 0, n, self.p)[0]

    def chi_snapshots(self, first: int, count: int) -> np.ndarray:
        return get_samples(self.ctx, 0, first, count, self.p, (self.d, self.n), self.npdtype)[1]

    def run_streamed(self, n: int, chunk: int, on_rows=None, copy: bool = True):
        """n cycles with every latent snapshot streamed to the host through a
        ring of snap_rows device rows; on_rows(first, rows) receives each
        chunk's snapshots (default: collect them and return [count][d][N];
        copy=False hands on_rows a view valid only during the call)."""
        got = []
        cb = (lambda slot, first, rows: on_rows(first, rows)) if on_rows else \
            (lambda slot, first, rows: got.append((first, rows)) and False)
        run_cycles_streamed(self.ctx, n, chunk, cb, lambda slot: (self.d, self.n), self.npdtype,
                            copy=copy or on_rows is None)
        if on_rows is None:
            return np.concatenate([r for _, r in got]) if got else np.zeros((0, self.d, self.n), self.npdtype)
        return None

    def run_to_file(self, n: int, chunk: int, path: str):
        """n cycles appending every latent snapshot to the file at path as raw
        [d][N] rows of the context's precision."""
        import os
        fd = os.open(path, os.O_WRONLY | os.O_CREAT | os.O_APPEND, 0o644)
        try:
            run_cycles_to_fd(self.ctx, n, chunk, fd)
        finally:
            os.close(fd)

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

    def checkpoint(self):
        """(library state blob, chi, chol, acc) from which `restore` resumes the chain exactly."""
        blob = get_state(self.ctx)
        return (blob, *self.state())

    def restore(self, ckpt):
        blob, chi, chol, acc = ckpt
        self.load_state(chi, chol, acc)
        set_state(self.ctx, blob)

    def load_state(self, chi, chol, acc):
        """Overwrite the latent buffers from host arrays (lockstep replay)."""
        with torch.no_grad():
            self.chi.copy_(torch.as_tensor(np.asarray(chi), dtype=self.dtype))
            self.chol.copy_(torch.as_tensor(np.asarray(chol), dtype=self.dtype))
            self.acc.copy_(torch.as_tensor(np.asarray(acc).astype(np.uint32).view(np.int32)))
        torch.cuda.synchronize(self.device)


class Batch(_Chains):
    """Many datasets of one model advanced together (init_batch).

    Dataset j sits in slot j at objects [offsets[j], offsets[j] + N_j) of the
    packed buffers; every launch covers all of them.
    """

    def __init__(self, wls, device: str = "cuda:0", max_cycles: int = 10000, s0: float = 1.0,
                 adapt_theta: bool = True, n_quad: int = 512, gamma: float = 2.0 / 3.0,
                 alpha_star_theta: float = 0.4, stream: Optional[torch.cuda.Stream] = None, theta_substeps: int = 0):
        self.wls = list(wls)
        ns = [w.n for w in self.wls]
        self.offsets, cap = packed_offsets(ns)
        self.ns = ns
        self._alloc(self.wls[0].model, cap, 0, device, stream)
        data = np.zeros((self.m, cap), dtype=self.npdtype)
        chi = np.zeros((self.d, cap), dtype=self.npdtype)
        for w, o in zip(self.wls, self.offsets):
            data[:, o:o + w.n] = w.data
            chi[:, o:o + w.n] = w.chi0
        with torch.no_grad():
            self.data.copy_(torch.as_tensor(data))
            self.chi.copy_(torch.as_tensor(chi))
        self.configs = [make_config(w, max_cycles, 0, s0, adapt_theta, n_quad, gamma, alpha_star_theta,
                                    theta_substeps=theta_substeps) for w in self.wls]
        theta0 = np.array([w.theta0 for w in self.wls], dtype=np.float64)
        torch.cuda.synchronize(self.device)
        with torch.cuda.device(self.device):
            self.ctx = init_batch(self.configs, self.buffers, theta0, self.stream.cuda_stream)

    @property
    def n_datasets(self) -> int:
        return len(self.wls)

    def ram_sweep(self, n: int = 1, rate: bool = False):
        return ram_sweep(self.ctx, n, rate, self.n_datasets)

    def theta_step(self) -> np.ndarray:
        return theta_step(self.ctx, self.n_datasets)

    def pop_loglik(self, thetas) -> np.ndarray:
        return pop_loglik(self.ctx, thetas)

    def marginal_loglik(self, j: int, thetas, terms: bool = False):
        return marginal_loglik(self.ctx, j, thetas, self.wls[j].n, terms, self.device)

    def theta(self, j: int):
        return get_theta(self.ctx, self.p, j)

    def stats(self, j: int) -> dict:
        return get_stats(self.ctx, j)

    def theta_trace(self, j: int) -> np.ndarray:
        n = n_theta_samples(self.ctx, j)
        return get_samples(self.ctx, j, 0, n, self.p)[0]

    def latents(self, j: int) -> np.ndarray:
        """Host copy of dataset j's latents [d][N_j]."""
        torch.cuda.synchronize(self.device)
        o = self.offsets[j]
        return self.chi[:, o:o + self.ns[j]].double().cpu().numpy()


class Pool(_Chains):
    """A fixed pool of slots over packed buffers for continuous batching.

    Datasets are admitted into a free slot and a free run of object tiles
    (first fit), advance together with every other resident dataset, stop on
    the device when their theta-step budget is spent, and are retired to
    free their slot and tiles.
    """

    def __init__(self, model: int, capacity: int, n_slots: int, max_cycles: int, device: str = "cuda:0",
                 n_quad: int = 512, stream: Optional[torch.cuda.Stream] = None, stats_theta: bool = False,
                 snap_rows: int = 0):
        cap = -(-int(capacity) // TILE) * TILE
        self._alloc(model, cap, snap_rows, device, stream)
        pc = PoolConfig()
        pc.model, pc.precision, pc.n_slots = model, _MODEL_DIMS[model][3], n_slots
        pc.n_quad, pc.capacity, pc.max_cycles, pc.snap_rows = n_quad, cap, max_cycles, snap_rows
        pc.stats_theta = int(stats_theta)
        self.pool_config, self.n_slots, self.max_cycles = pc, n_slots, max_cycles
        self.free_slots = list(range(n_slots - 1, -1, -1))
        self.alloc = TileAllocator(cap // TILE)                     # slot owning each tile
        self.resident = {}                                          # slot -> (obj_start, n)
        self.left = {}                                              # slot -> theta steps still to run
        torch.cuda.synchronize(self.device)
        with torch.cuda.device(self.device):
            self.ctx = create_pool(pc, self.buffers, self.stream.cuda_stream)

    @property
    def tiles(self) -> np.ndarray:
        return self.alloc.owner

    def fits(self, n: int) -> bool:
        return bool(self.free_slots) and self.alloc.find(-(-n // TILE)) is not None

    def admit(self, wls, budgets, **cfg_kw):
        """Loads the workloads that fit, in order, and returns their slots (None where one did not fit)."""
        slots, starts, cfgs, th0, bud, placed = [], [], [], [], [], []
        for w, b in zip(wls, budgets):
            nt = -(-w.n // TILE)
            t0 = self.alloc.find(nt) if self.free_slots else None
            if t0 is None:
                placed.append(None)
                continue
            slot = self.free_slots.pop()
            self.alloc.take(t0, nt, slot)
            o = t0 * TILE
            slots.append(slot)
            starts.append(o)
            cfgs.append(make_config(w, max_cycles=self.max_cycles, **cfg_kw))
            th0.append(w.theta0)
            bud.append(b)
            placed.append(slot)
            self.resident[slot] = (o, w.n)
            self.left[slot] = b if b > 0 else float("inf")
        if slots:
            # data and starting latents at their positions, then one load call
            with torch.no_grad():
                for w, o in zip([w for w, s in zip(wls, placed) if s is not None], starts):
                    self.data[:, o:o + w.n].copy_(torch.as_tensor(np.asarray(w.data, dtype=self.npdtype)))
                    self.chi[:, o:o + w.n].copy_(torch.as_tensor(np.asarray(w.chi0, dtype=self.npdtype)))
            torch.cuda.current_stream(self.device).synchronize()
            try:
                load_datasets(self.ctx, slots, starts, cfgs, np.array(th0, dtype=np.float64), bud)
            except Exception:
                for sl in slots:
                    self._release(sl)
                raise
        return placed

    def _release(self, slot: int):
        self.alloc.release(slot)
        self.resident.pop(slot, None)
        self.left.pop(slot, None)
        self.free_slots.append(slot)

    def run_cycles(self, n: int, use_graph: bool = True):
        run_cycles(self.ctx, n, use_graph)
        for s in self.left:
            self.left[s] -= n

    def run_streamed(self, n: int, chunk: int, on_rows):
        """n cycles streaming every resident job's latent snapshots:
        on_rows(slot, first, rows [count][d][N_slot])."""
        run_cycles_streamed(self.ctx, n, chunk, on_rows, lambda slot: (self.d, self.resident[slot][1]),
                            self.npdtype)
        for s in self.left:
            self.left[s] -= n

    def retire(self, slot: int) -> np.ndarray:
        """Returns the slot's theta trace and frees the slot."""
        tr = self.theta_trace(slot)
        unload_dataset(self.ctx, slot)
        self._release(slot)
        return tr

    def info(self, slot: int) -> dict:
        return slot_info(self.ctx, slot)

    def finished(self):
        """Resident slots whose budget is spent (the device stops them at exactly that cycle)."""
        return [s for s, left in self.left.items() if left <= 0]

    def theta_trace(self, slot: int) -> np.ndarray:
        n = n_theta_samples(self.ctx, slot)
        return get_samples(self.ctx, slot, 0, n, self.p)[0]

    def latents(self, slot: int) -> np.ndarray:
        """Host copy of a resident dataset's latents [d][N]."""
        torch.cuda.synchronize(self.device)
        o, n = self.resident[slot]
        return self.chi[:, o:o + n].double().cpu().numpy()
