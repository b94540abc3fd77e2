"""Seeded synthetic inputs shared by the CPU oracle, the tests and the bench.

This package only draws data (simulated catalogs, arrival streams). It holds
none of the sampler's arithmetic: no log-densities, no RAM step, no
selection integral. Both sides of every parity test receive the arrays made
here and nothing else.
"""

from .workloads import (  # noqa: F401
    NormalNormal1D,
    GammaLF1D,
    GammaLF3D,
    normal_normal_1d,
    normal_normal_3d,
    gamma_lf_1d,
    gamma_lf_3d,
    gamma_lf_batch,
    serving_arrivals,
    calibrate_threshold,
    bb1_lf,
    bb1_sample,
)
