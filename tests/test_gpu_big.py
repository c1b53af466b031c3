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


@pytest.mark.parametrize("mode", ["td", "td_bf16"])
def test_stress_full_size(gpu, torch_mod, mode):
    """64 mics in 7 cm x 65536 samples x 10000 directions, 16 frames (P = 131072):
    sampled directions of three frames against the oracle."""
    torch = torch_mod
    F = 16
    w = synth.make_workload("c5", frames=F)
    _say(f"case stress {mode}: M=64 N=65536 D=10000 F=16")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 65536, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=F, mode=mode)
    assert plan.P == 131072 and plan.Q == 6554
    E = plan.energyscape(torch.from_numpy(w.x).cuda())
    rng = np.random.default_rng(5)
    sample = np.sort(np.concatenate([[0, 9999], rng.choice(10000, 6, replace=False)]))
    Es = E[:, torch.from_numpy(sample).cuda()].cpu().numpy()
    assert np.all(np.isfinite(Es))
    errs = []
    for f in (0, 9, 15):
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                           R=10, band=w.cfg.band, mode="td", dir_index=sample)
        errs.append(rel_l2(Es[f], Eo))
        _say(f"  frame {f}: sampled rel L2 = {errs[-1]:.3e}")
    assert max(errs) <= BARS[mode]
