"""The C ABI library loads and exports every function include/hbm.h declares,
and the Python binding's struct layouts match the header's (checked with a
tiny C program compiled against hbm.h).  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hbm.h")


def declared_functions():
    text = open(HEADER).read()
    return re.findall(r"^HBM_API\s+[\w\s\*]+?\b(\w+)\s*\(", text, flags=re.M)


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("init_chains", "ram_sweep", "pop_loglik", "theta_step", "get_samples", "destroy_chains",
                 "last_error"):
        assert core in names


def test_library_exports_every_declared_symbol():
    import paper_2105_08026_amd as hbm
    if not os.path.exists(hbm.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(hbm.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(hbm.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", hbm.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert exported == set(declared_functions())


def test_struct_layout_matches_header(tmp_path):
    import paper_2105_08026_amd as hbm
    src = tmp_path / "layout.c"
    fields = [f for f, _ in hbm.Config._fields_]
    bfields = [f for f, _ in hbm.Buffers._fields_]
    pfields = [f for f, _ in hbm.PoolConfig._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hbm.h"', "int main(void){",
             'printf("%zu %zu %zu\\n", sizeof(hbm_config), sizeof(hbm_buffers), sizeof(hbm_pool_config));']
    lines += [f'printf("%zu\\n", offsetof(hbm_config, {f}));' for f in fields]
    lines += [f'printf("%zu\\n", offsetof(hbm_buffers, {f}));' for f in bfields]
    lines += [f'printf("%zu\\n", offsetof(hbm_pool_config, {f}));' for f in pfields]
    lines += ["return 0;}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(hbm.Config) and vals[1] == ctypes.sizeof(hbm.Buffers)
    assert vals[2] == ctypes.sizeof(hbm.PoolConfig)
    offs = vals[3:]
    nf, nb = len(fields), len(bfields)
    assert offs[:nf] == [getattr(hbm.Config, f).offset for f in fields]
    assert offs[nf:nf + nb] == [getattr(hbm.Buffers, f).offset for f in bfields]
    assert offs[nf + nb:] == [getattr(hbm.PoolConfig, f).offset for f in pfields]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_2105_08026_amd as hbm
    monkeypatch.setattr(hbm, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(hbm, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        hbm.lib()


def _reject(hbm, cfg, theta0):
    L = ctypes.CDLL(hbm.LIB_PATH)
    L.init_chains.argtypes = [ctypes.c_void_p] * 6
    L.init_chains.restype = ctypes.c_int32
    L.last_error.argtypes = [ctypes.c_void_p]
    L.last_error.restype = ctypes.c_char_p
    bufs = hbm.Buffers(8, 8, 8, 8, None)          # never dereferenced: the config fails first
    out = ctypes.c_void_p()
    th = (ctypes.c_double * len(theta0))(*theta0)
    st = L.init_chains(ctypes.byref(cfg), ctypes.byref(bufs), None, th, None, ctypes.byref(out))
    return st, L.last_error(None).decode(), out.value


def test_init_chains_rejects_bad_theta_modes_before_touching_the_device():
    """Dataset checks run before a context exists; they must not need one."""
    import paper_2105_08026_amd as hbm
    import synth
    if not os.path.exists(hbm.LIB_PATH):
        pytest.skip("library not built")
    lf = synth.gamma_lf_1d(n=300, seed=3, fth=389.75)
    st, msg, out = _reject(hbm, hbm.make_config(lf, max_cycles=10, theta_substeps=65), lf.theta0)
    assert st == hbm.HBM_EINVAL and "theta_substeps" in msg and not out
    cfg = hbm.make_config(lf, max_cycles=10, theta_substeps=2)
    cfg.snap_rows = -1
    st, msg, out = _reject(hbm, cfg, lf.theta0)
    assert st == hbm.HBM_EINVAL and "snap_rows" in msg and not out
    bb = synth.bb1_lf(n=50, seed=2, chunk=100_000)
    st, msg, out = _reject(hbm, hbm.make_config(bb, max_cycles=10, theta_substeps=2), bb.theta0)
    assert st == hbm.HBM_EINVAL and "sufficient statistics" in msg and not out


def test_init_chains_rejects_bad_sizes_before_touching_the_device():
    """An empty catalog and one past the index range are refused with
    HBM_EINVAL by the host checks alone."""
    import paper_2105_08026_amd as hbm
    import synth
    if not os.path.exists(hbm.LIB_PATH):
        pytest.skip("library not built")
    lf = synth.gamma_lf_1d(n=300, seed=3, fth=389.75)
    for n in (0, -5, 2 ** 31):
        cfg = hbm.make_config(lf, max_cycles=10)
        cfg.n_objects = n
        st, msg, out = _reject(hbm, cfg, lf.theta0)
        assert st == hbm.HBM_EINVAL and "n_objects" in msg and not out, (n, msg)
