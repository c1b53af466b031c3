"""Variant readings on the GPU against the FP64 oracle: integer-delay delay-and-sum
(TD_NEAREST).  FP32 bar: relative L2 <= 1e-5 per energyscape."""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


@pytest.mark.parametrize("cfg,n_samples,n_dirs,frames", [("c1", None, None, 1), ("c2", 4096, 37, 2),
                                                         ("c2", 16384, 1500, 1)])
def test_td_nearest_matches_oracle(gpu, torch_mod, cfg, n_samples, n_dirs, frames):
    torch = torch_mod
    w = synth.make_workload(cfg, frames=frames, n_samples=n_samples, n_dirs=n_dirs)
    D = w.dirs.shape[0]
    _say(f"case td_nearest: {cfg} N={w.x.shape[2]} D={D} F={frames}")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                    decim=w.cfg.decim, mode="td_nearest", max_frames=frames)
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()
    # full size: every 50th direction of the oracle
    sel = np.arange(0, D, 50) if D > 200 else np.arange(D)
    for f in range(frames):
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                           band=w.cfg.band, mode="td_nearest", dir_index=sel)
        err = rel_l2(E[f][sel], Eo)
        _say(f"td_nearest {cfg} frame {f}: rel L2 {err:.2e}")
        assert err <= 1e-5
    # it is a different result from linear interpolation
    Et = O.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                       band=w.cfg.band, mode="td", dir_index=sel)
    assert rel_l2(E[0][sel], Et) > 1e-3


def test_td_nearest_positions_and_gradients(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=17)
    _say("case td_nearest set_positions / vjp")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, decim=w.cfg.decim, mode="td_nearest")
    pos2 = w.mic_pos + np.random.default_rng(np.random.SeedSequence([5, 0, 0, 1])).normal(0, 0.5e-3, w.mic_pos.shape)
    plan.set_positions(pos2)
    x = torch.from_numpy(w.x).cuda()
    E = plan.energyscape(x).cpu().numpy()[0]
    Eo = O.energyscape(w.x[0].astype(np.float64), w.chirp, pos2, w.dirs, fs=w.fs, c=w.c, P=plan.P, mode="td_nearest")
    assert rel_l2(E, Eo) <= 1e-5
    mf = plan.matched_filter(x)
    beam = plan.beamform(mf)
    dE = torch.ones((1, plan.D, plan.Q), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu.SonarError):
        plan.vjp(mf, beam, dE, want_dx=False, want_dpos=True)
