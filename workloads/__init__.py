"""Seeded synthetic eRTIS workloads shared by the tests, the benchmark and the oracle checks.

This package holds input generation only (array geometry, emitted sweep,
direction grids, point-reflector echoes, noise): none of the pipeline's own
arithmetic (matched filter, beamformer, envelope) lives here.
"""

from .synth import (  # noqa: F401
    CONFIGS,
    Workload,
    azimuth_grid,
    fibonacci_hemisphere,
    linear_chirp,
    make_workload,
    planar_array,
    restricted_grid,
    simulate_frame,
)
