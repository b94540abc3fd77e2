"""marginal_loglik_noalloc, the marginal likelihood of 1-D latents with its
scratch in the library's static device array (no allocation in the call),
against marginal_loglik, which allocates its scratch: both run the same
kernels, so results and per-object terms must be the same bits.

Two calls in a row on one device share the static array: the second, on a
smaller catalog with fewer theta rows, must not see anything of the first.
A request larger than the array is refused with HBM_EINVAL and leaves the
context usable.
"""
import math
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FTH = 389.75
HBM_EINVAL = -1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2105_08026_amd as h
    h.lib()
    return h


def _noalloc(hbm, s, thetas):
    """One call of marginal_loglik_noalloc through the C ABI (slot 0, terms
    into a NaN-filled device buffer): returns (status, out, terms)."""
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64))
    out = np.full(th.shape[0], np.nan)
    tb = torch.full((th.shape[0], s.n), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    rc = hbm.lib().marginal_loglik_noalloc(s.ctx, 0, th.shape[0], th.ctypes.data, out.ctypes.data, tb.data_ptr())
    return rc, out, tb.cpu().numpy()


def _reference(s, thetas):
    out, terms = s.marginal_loglik(np.asarray(thetas, dtype=np.float64), terms=True)
    return out, terms


def _lf_thetas(wl, k):
    t0 = np.array(wl.theta_true, dtype=np.float64)
    rows = [t0 + [0.04 * (j % 5) - 0.08, 0.05 * (j // 5) - 0.1] for j in range(k)]
    rows.append([-0.9, t0[1] + 1.0])
    return rows


def test_noalloc_equals_allocating_entry_point_two_calls(hbm):
    big = synth.gamma_lf_1d(n=70000, seed=93, fth=FTH)        # 2,188 workgroups of 32 objects
    small = synth.gamma_lf_1d(n=3001, seed=91, fth=FTH)       # 94 workgroups, ragged tail
    nn = synth.normal_normal_1d(n=777, seed=5)
    s_big = hbm.Sampler(big, device="cuda:0", max_cycles=8)
    s_small = hbm.Sampler(small, device="cuda:0", max_cycles=8)
    s_nn = hbm.Sampler(nn, device="cuda:0", max_cycles=8)
    try:
        th_big = _lf_thetas(big, 9)
        th_small = _lf_thetas(small, 2)
        th_nn = [[0.1, math.log(0.9)], [-1.0, math.log(3.0)]]
        _say("noalloc call 1: gamma LF N=70000, 10 theta rows")
        rc, out1, terms1 = _noalloc(hbm, s_big, th_big)
        assert rc == 0, hbm.lib().last_error(s_big.ctx)
        _say("noalloc call 2: gamma LF N=3001, 3 theta rows (smaller input)")
        rc, out2, terms2 = _noalloc(hbm, s_small, th_small)
        assert rc == 0, hbm.lib().last_error(s_small.ctx)
        _say("noalloc call 3: normal-normal N=777, 2 theta rows")
        rc, out3, terms3 = _noalloc(hbm, s_nn, th_nn)
        assert rc == 0, hbm.lib().last_error(s_nn.ctx)
        _say("allocating entry point on the same inputs")
        ref1, rterms1 = _reference(s_big, th_big)
        ref2, rterms2 = _reference(s_small, th_small)
        ref3, rterms3 = _reference(s_nn, th_nn)
        for got, ref, gt, rt in ((out1, ref1, terms1, rterms1), (out2, ref2, terms2, rterms2),
                                 (out3, ref3, terms3, rterms3)):
            assert np.all(np.isfinite(got))
            assert np.array_equal(got, ref), (got, ref)
            assert np.array_equal(gt, rt)
        # the same call again after the others: the array keeps no state that matters
        _say("noalloc call 4: the first call again")
        rc, out4, terms4 = _noalloc(hbm, s_big, th_big)
        assert rc == 0
        assert np.array_equal(out4, ref1) and np.array_equal(terms4, rterms1)
    finally:
        s_big.close()
        s_small.close()
        s_nn.close()


def test_noalloc_refuses_requests_beyond_the_static_scratch(hbm):
    wl = synth.gamma_lf_1d(n=70000, seed=93, fth=FTH)
    s = hbm.Sampler(wl, device="cuda:0", max_cycles=8)
    try:
        # 8 (n_theta (p + 9 + ceil(N / 32))) bytes: 17,592 per row here, so
        # 476 rows fit in the 8 MiB array after the node rule and 477 do not
        per_row = 8 * (wl.p + 9 + (wl.n + 31) // 32)
        fit = (hbm.HBM_NOALLOC_SCRATCH_BYTES - 8448) // per_row
        assert fit == 476
        t0 = np.array(wl.theta_true, dtype=np.float64)
        _say(f"noalloc: {fit + 1} theta rows over N=70000 (refused)")
        rows = np.tile(t0, (fit + 1, 1))
        rc, out, _ = _noalloc(hbm, s, rows)
        assert rc == HBM_EINVAL
        msg = hbm.lib().last_error(s.ctx).decode()
        assert "static scratch" in msg and str(fit + 1) in msg, msg
        assert np.all(np.isnan(out))
        _say(f"noalloc: {fit} theta rows over N=70000 (accepted)")
        rc, out, terms = _noalloc(hbm, s, rows[:fit])
        assert rc == 0, hbm.lib().last_error(s.ctx)
        ref, rterms = _reference(s, rows[:1])
        assert np.all(out == ref[0]) and np.array_equal(terms[0], rterms[0]) and np.array_equal(terms[-1], rterms[0])
    finally:
        s.close()
