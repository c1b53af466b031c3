"""The oracle's process-pool driver returns what the oracle returns (CPU).

The pool only distributes energyscape calls; split over direction subsets, its rows must be the
rows of the unsplit call (each direction is computed on its own), for every mode."""

import numpy as np
import pytest

import oracle as O
from oracle import pool
from workloads import synth


@pytest.mark.parametrize("mode,steps", [("td", None), ("td", 2048), ("fd", None)])
def test_pool_rows_equal_the_direct_call(mode, steps):
    w = synth.make_workload("c2", frames=2, n_samples=1200, n_dirs=37)
    jobs = [pool.Job(x=w.x[f], chirp=w.chirp, mic_pos=w.mic_pos, dirs=w.dirs, fs=w.fs, c=w.c, P=2048,
                     band=w.cfg.band, mode=mode, alpha_steps=steps) for f in range(2)]
    Es, times, wall = pool.run(jobs, workers=2, split=3)
    for f in range(2):
        Ed = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=2048,
                           band=w.cfg.band, mode=mode, alpha_steps=steps)
        assert Es[f].shape == Ed.shape
        np.testing.assert_allclose(Es[f], Ed, rtol=0, atol=1e-12 * np.abs(Ed).max())
        assert times[f]["total"] > 0 and times[f]["beamform"] > 0
    assert wall > 0


def test_stage_timings_do_not_change_the_result():
    w = synth.make_workload("c1", n_dirs=9)
    t = {}
    E1 = O.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, timings=t)
    E2 = O.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c)
    assert np.array_equal(E1, E2)
    assert set(t) == {"matched_filter", "beamform", "envelope"}
