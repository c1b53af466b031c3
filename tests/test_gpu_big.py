"""Matched filters beyond one workgroup's LDS (NF > 16384), up to the 64-mic stress configuration (GPU).

The four-step transform (radix-R pass over global memory + 16384-point LDS
transforms) must give the same matched filter, beam and energyscape as the
definition: FP32 paths within 1e-5 of the FP64 oracle, BF16 paths within 1e-3.
"""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu

BARS = {"td": 1e-5, "fd_fp32": 1e-5, "fd_bf16x3": 1e-5, "td_bf16": 1e-3, "fd_bf16": 1e-3}


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def test_big_matched_filter_rows(gpu, torch_mod):
    """P = 65536 (radix-2 pass): every stored matched-filter sample against the oracle."""
    torch = torch_mod
    w = synth.make_workload("c2", n_samples=40000, n_dirs=7, n_mics=4)
    _say("case mf rows: M=4 N=40000 P=65536")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 40000, fs=w.fs, c=w.c, band=w.cfg.band, mode="td")
    assert plan.P == 65536
    mf = plan.matched_filter(torch.from_numpy(w.x).cuda()).cpu().numpy()[0].reshape(plan.M, plan.mf_row)
    yhat = O.matched_filter(w.x[0].astype(np.float64), w.chirp, plan.P, w.fs, w.cfg.band)
    idx = (plan.mf_origin + np.arange(plan.mf_row)) % plan.P
    err = rel_l2(mf, yhat[:, idx])
    _say(f"  rows rel L2 = {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("case", [
    dict(N=40000, M=4, D=9, mode="td"),                       # R = 2
    dict(N=40000, M=4, D=9, mode="td_bf16"),
    dict(N=70000, M=3, D=5, mode="td", dtype="f16"),           # R = 8, half-precision samples
    dict(N=200000, M=2, D=3, mode="td"),                       # R = 8
    dict(N=300000, M=1, D=2, mode="td_bf16"),                  # R = 16, the largest transform
    dict(N=40000, M=6, D=8, mode="fd_fp32"),                   # band bins from the big split
    dict(N=40000, M=6, D=8, mode="fd_bf16x3"),
    dict(N=40000, M=32, D=8, mode="fd_bf16"),                 # one BF16 steering term: needs many mics
    dict(N=40000, M=12, D=40, mode="fd_fp32"),                # 9467 band bins: 8192-point phases, two bins per slot
    dict(N=100000, M=4, D=6, mode="fd_fp32"),                 # P = 131072 band: 16384-point phases, two per slot
])
def test_big_energyscape(gpu, torch_mod, case):
    torch = torch_mod
    w = synth.make_workload("c2", n_samples=case["N"], n_dirs=case["D"], n_mics=case["M"])
    _say(f"case {case}")
    dt = case.get("dtype", "f32")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, case["N"], fs=w.fs, c=w.c, band=w.cfg.band, mode=case["mode"],
                    sample_dtype=dt)
    xs = w.x if dt == "f32" else w.x.astype(np.float16)
    E = plan.energyscape(torch.from_numpy(xs).cuda()).cpu().numpy()[0]
    omode = "fd" if case["mode"].startswith("fd") else "td"
    Eo = O.energyscape(xs[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P, R=10,
                       band=w.cfg.band, mode=omode)
    err = rel_l2(E, Eo)
    _say(f"  P={plan.P} rel L2 = {err:.3e}")
    assert err <= BARS[case["mode"]]


STRESS_F = 16
STRESS_FULL = 1000      # directions of frame 0 checked against the oracle


@pytest.fixture(scope="module")
def c5():
    return synth.make_workload("c5", frames=STRESS_F)


class _StressOracle:
    """Oracle energyscapes of frame 0 of the stress workload on a seeded subset of 1000 directions,
    per reading, computed once on the host's cores."""

    def __init__(self, w):
        self.w = w
        self.idx = np.sort(np.random.default_rng(5).choice(w.dirs.shape[0], STRESS_FULL, replace=False))
        self.cache = {}

    def get(self, reading):
        if reading not in self.cache:
            from oracle import pool
            w = self.w
            job = pool.Job(x=w.x[0], chirp=w.chirp, mic_pos=w.mic_pos, dirs=w.dirs, fs=w.fs, c=w.c, P=131072,
                           R=w.cfg.decim, band=w.cfg.band, mode=reading, dir_index=self.idx)
            nw = pool.default_workers()
            Es, _, wall = pool.run([job], workers=nw, split=2 * nw)
            _say(f"  oracle {reading}: frame 0, {STRESS_FULL} directions, {nw} processes, {wall:.1f} s")
            self.cache[reading] = Es[0]
        return self.cache[reading]


@pytest.fixture(scope="module")
def oracle_c5(c5):
    return _StressOracle(c5)


@pytest.mark.parametrize("mode", ["td", "td_bf16x2", "fd_fp32", "fd_bf16"])
def test_stress_full_size(gpu, torch_mod, c5, oracle_c5, mode):
    """64 mics in 7 cm x 65536 samples x 10000 directions, 16 frames (P = 131072): frame 0 on a
    seeded subset of 1000 directions and frames 9 and 15 on 8 sampled directions against the oracle
    of the mode's reading (time-domain modes: linear interpolation; frequency-domain: exact phase)."""
    torch = torch_mod
    w = c5
    _say(f"case stress {mode}: M=64 N=65536 D=10000 F={STRESS_F}")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 65536, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=STRESS_F,
                    mode=mode)
    assert plan.P == 131072 and plan.Q == 6554
    E = plan.energyscape(torch.from_numpy(w.x).cuda())
    reading = "fd" if mode.startswith("fd") else "td"
    bar = {"td": 1e-5, "td_bf16x2": 1e-3, "fd_fp32": 1e-5, "fd_bf16": 1e-3}[mode]
    idx = oracle_c5.idx
    E0 = E[0][torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.all(np.isfinite(E0))
    err = rel_l2(E0, oracle_c5.get(reading))
    _say(f"  frame 0, {idx.size} directions: rel L2 = {err:.3e}")
    assert err <= bar
    rng = np.random.default_rng(6)
    sample = np.sort(np.concatenate([[0, 9999], rng.choice(10000, 6, replace=False)]))
    Es = E[:, torch.from_numpy(sample).cuda()].cpu().numpy()
    for f in (9, 15):
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                           R=10, band=w.cfg.band, mode=reading, dir_index=sample)
        e = rel_l2(Es[f], Eo)
        _say(f"  frame {f}: sampled rel L2 = {e:.3e}")
        assert e <= bar
    del E
    plan.close()
    torch.cuda.empty_cache()
