"""Parity of the BF16-MFMA time-domain beamformer with single-term samples (mode td_bf16x2)
with the FP64 oracle (GPU).

The mode is TD_BF16 with the samples carried as one BF16 term (weights still split): the
samples' rounding, independent from sample to sample and microphone to microphone, averages
down in the sum over the array.  Bar: relative L2 <= 1e-3 per energyscape against the
oracle's time-domain mode for arrays of 32 or more microphones (the mode's stated range);
smaller arrays are printed, not held to it.
"""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu

BAR = 1e-3


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _bf16_rne(v):
    u = np.ascontiguousarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def test_c1_td_bf16x2(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c1")
    _say("case c1 td_bf16x2: M=32 N=4096 D=91")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 4096, fs=w.fs, c=w.c, mode="td_bf16x2")
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()[0]
    Eo = O.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P, mode="td")
    err = rel_l2(E, Eo)
    _say(f"  rel L2 = {err:.3e}")
    assert err <= BAR


def test_td_bf16x2_planes_are_single_bf16_terms(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c2", n_samples=3000, n_dirs=45)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, fs=w.fs, c=w.c, band=w.cfg.band, mode="td_bf16x2")
    M, row = plan.M, plan.mf_row
    assert plan.mf_frame_elems == M * row * 3 // 2
    mf = plan.matched_filter(torch.from_numpy(w.x).cuda())
    fr = mf[0].cpu()
    y = fr[:M * row].numpy().reshape(M, row)
    pl = fr[M * row:].view(torch.int16).numpy().view(np.uint16).reshape(M, 2, row)
    assert np.array_equal(pl[:, 0], _bf16_rne(y.real))
    assert np.array_equal(pl[:, 1], _bf16_rne(y.imag))


@pytest.mark.parametrize("case", [
    dict(N=2000, D=17, band=(20e3, 85e3), R=10, F=3),
    dict(N=2500, D=33, band=(20e3, 85e3), R=10, F=17, P=8192),
    dict(N=900, D=40, band=(20e3, 85e3), R=10, F=2, M=40),
    dict(N=1500, D=100, band=(20e3, 85e3), R=10, F=1, M=64),
    dict(N=700, D=5, band=(20e3, 85e3), R=10, F=1, M=1),            # below the stated range: printed
    dict(N=3000, D=70, band=None, R=3, F=2, M=8),                   # below the stated range: printed
])
def test_td_bf16x2_shapes(gpu, torch_mod, case):
    torch = torch_mod
    w = synth.make_workload("c2", frames=case["F"], n_samples=case["N"], n_dirs=case["D"], n_mics=case.get("M"))
    _say(f"case td_bf16x2 {case}")
    noise = np.random.default_rng(case["N"] + case["D"]).standard_normal(w.x.shape).astype(np.float32)
    w.x = (w.x + 0.05 * noise).astype(np.float32)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, case["N"], fs=w.fs, c=w.c, band=case["band"], decim=case["R"],
                    fft_len=case.get("P", 0), max_frames=case["F"], mode="td_bf16x2")
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()
    errs = []
    for f in range(case["F"]):
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                           R=case["R"], band=case["band"], mode="td")
        errs.append(rel_l2(E[f], Eo))
    _say(f"  max rel L2 over frames = {max(errs):.3e}")
    if plan.M >= 32:
        assert max(errs) <= BAR
