"""The FP32 Box-Muller transform and accept test use the hardware
transcendentals (v_cos_f32/v_sin_f32 in revolutions, v_log_f32, v_sqrt_f32).
Over every 24-bit uniform they must stay within a few float roundings of the
FP64 functions (the per-object log densities use the library functions)."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

pytestmark = pytest.mark.gpu


def test_hardware_transcendentals_over_all_uniforms(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = str(tmp_path / "hw_transcendentals")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O3", "-o", exe, os.path.join(HERE, "pins", "hw_transcendentals.hip")],
                   check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, check=True).stdout
    print(out, flush=True)
    vals = [float(v) for v in re.findall(r"([0-9.]+e[-+][0-9]+)", out)]
    cos_err, sin_err, ln_rel, sqrt_rel = vals
    assert cos_err < 3e-7 and sin_err < 3e-7
    assert ln_rel < 4e-7 and sqrt_rel < 2.5e-7
