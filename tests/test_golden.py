"""Golden fixtures: the paper's printed constants and a frozen tiny oracle result."""
import json
import os

import numpy as np

import oracle
from workloads import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_workload_constants_follow_the_paper():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        pc = json.load(f)
    assert synth.N_MICS == pc["n_mics"]["value"]
    assert synth.FS_HZ == pc["fs_hz"]["value"]
    for name in ("c1", "c2"):
        assert synth.CONFIGS[name].n_mics == pc["n_mics"]["value"]
    # the context grids match the paper's direction counts (90 -> 91 with both ends of -90..90)
    counts = pc["direction_counts"]["value"]
    assert abs(synth.azimuth_grid(91).shape[0] - counts[0]) <= 1
    assert synth.restricted_grid(counts[1]).shape[0] == counts[1]
    assert synth.fibonacci_hemisphere(counts[2]).shape[0] == counts[2]


def test_restricted_grid_respects_half_angle():
    u = synth.restricted_grid(1850)
    az = np.degrees(np.arctan2(u[:, 0], u[:, 2]))
    el = np.degrees(np.arcsin(u[:, 1]))
    assert np.all(np.abs(az) <= 45.0) and np.all(np.abs(el) <= 45.0)
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0)


def test_oracle_matches_frozen_tiny_energyscape():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    c = mg.tiny_case()
    ref = np.loadtxt(os.path.join(GOLDEN, "tiny_energyscape.txt"))
    D = c["dirs"].shape[0]
    for i, mode in enumerate(("td", "fd")):
        E = oracle.energyscape(c["x"], c["chirp"], c["mic_pos"], c["dirs"], fs=c["fs"], c=c["c"],
                               P=c["P"], R=c["R"], band=c["band"], mode=mode)
        np.testing.assert_allclose(E, ref[i * D:(i + 1) * D], rtol=1e-12, atol=1e-14)
