"""Every direction of the full 32 x 16384 x 1500 workload against the FP64 oracle (GPU).

The workload of the throughput figure (32 mics in 3.5 cm, 16384 samples, 1500 Fibonacci
hemisphere directions, 20-85 kHz band, R = 10, 16 frames per call, P = 32768) runs through
every beamformer mode, and all 1500 directions of frames 0, 7 and 15 are compared with the
oracle (§4.1: the image covers every direction of interest).  The oracle energyscapes are
computed once per session, spread over the host's cores (oracle.pool).

Bars, relative L2 over the whole energyscape [D][Q] of a frame: FP32 modes and FD_BF16X3
1e-5; TD_BF16, TD_BF16X2, FD_BF16 1e-3; TD_F16 2e-4 against its gridded-delay reading and 3e-4
against plain linear interpolation.  A fault confined to a few directions (one tile of 32, say)
could hide inside a whole-frame figure, so each direction is also held to ten times its
mode's bar relative to the frame's RMS direction norm (||E_d - Eo_d|| <= 10 bar ||Eo|| / sqrt(D)).
TD_BF16G (delays on a 1/256-sample grid) is held to 1e-3 against both its gridded reading and plain
linear interpolation.
"""

import sys

import numpy as np
import pytest

from oracle import pool
from workloads import synth

pytestmark = pytest.mark.gpu

FRAMES = (0, 7, 15)
F = 16
# mode: (oracle reading, bar) [, second reading checked too]
MODES = {
    "td": [("td", 1e-5)],
    "td_bf16": [("td", 1e-3)],
    "td_bf16x2": [("td", 1e-3)],
    "td_f16": [("td_grid2048", 2e-4), ("td", 3e-4)],
    "td_bf16g": [("td_grid256", 1e-3), ("td", 1e-3)],
    "fd_fp32": [("fd", 1e-5)],
    "fd_bf16": [("fd", 1e-3)],
    "fd_bf16x3": [("fd", 1e-5)],
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


@pytest.fixture(scope="module")
def c2():
    return synth.make_workload("c2", frames=F)


class _OracleCache:
    """Oracle energyscapes of the selected frames, all directions, per reading; computed on first use."""

    def __init__(self, w):
        self.w = w
        self.cache = {}

    def get(self, reading):
        if reading not in self.cache:
            w = self.w
            mode, steps = ("td", int(reading[7:])) if reading.startswith("td_grid") else (reading, None)
            jobs = [pool.Job(x=w.x[f], chirp=w.chirp, mic_pos=w.mic_pos, dirs=w.dirs, fs=w.fs, c=w.c, P=32768,
                             R=w.cfg.decim, band=w.cfg.band, mode=mode, alpha_steps=steps) for f in FRAMES]
            nw = pool.default_workers()
            _say(f"  oracle {reading}: frames {FRAMES}, all {w.dirs.shape[0]} directions, {nw} worker processes")
            Es, _, wall = pool.run(jobs, workers=nw, split=max(1, (2 * nw) // len(jobs)))
            _say(f"  oracle {reading}: {wall:.1f} s")
            self.cache[reading] = dict(zip(FRAMES, Es))
        return self.cache[reading]


@pytest.fixture(scope="module")
def oracle_c2(c2):
    return _OracleCache(c2)


def _check_frame(E, Eo, bar, label):
    D = Eo.shape[0]
    err = float(np.linalg.norm(E - Eo) / np.linalg.norm(Eo))
    rms = np.linalg.norm(Eo) / np.sqrt(D)
    per_dir = np.linalg.norm(E - Eo, axis=1) / rms
    worst = int(np.argmax(per_dir))
    _say(f"  {label}: rel L2 over all {D} directions = {err:.3e}; worst direction {worst}: "
         f"{per_dir[worst]:.3e} of the RMS direction norm")
    assert np.all(np.isfinite(E))
    assert err <= bar
    assert per_dir[worst] <= 10 * bar


@pytest.mark.parametrize("mode", list(MODES))
def test_c2_every_direction(gpu, torch_mod, c2, oracle_c2, mode):
    torch = torch_mod
    w = c2
    _say(f"case c2 full every direction: {mode}, F={F}")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 16384, fs=w.fs, c=w.c, band=w.cfg.band, decim=w.cfg.decim,
                    max_frames=F, mode=mode)
    assert plan.P == 32768
    x = torch.from_numpy(w.x).cuda()
    Et = plan.energyscape(x)
    E = Et.cpu().numpy()
    assert E.shape == (F, 1500, 1639)
    for reading, bar in MODES[mode]:
        ref = oracle_c2.get(reading)
        for f in FRAMES:
            _check_frame(E[f], ref[f], bar, f"{mode} frame {f} vs {reading}")
    assert torch.equal(plan.energyscape(x), Et)        # deterministic
    plan.close()
