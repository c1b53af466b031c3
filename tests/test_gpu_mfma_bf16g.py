"""Parity of the BF16-MFMA time-domain beamformer with delays on a 1/256-sample grid (mode
td_bf16g) with the FP64 oracle (GPU).

The fractional delay is rounded to a multiple of 1/256 sample, so both interpolation weights are
exact single BF16 terms and each sample plane takes one product; the samples are one BF16 term,
as in td_bf16x2.  The oracle's gridded reading (das_td with alpha_steps=256) is the same
definition; plain linear interpolation differs from it by at most half a grid step per delay.
Bar: relative L2 <= 1e-3 per energyscape against both, for arrays of 32 or more microphones (the
mode's stated range); smaller arrays are printed, not held to it.
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


@pytest.mark.parametrize("case", [
    dict(N=4096, D=91, band=None, R=10, F=1, grid="c1"),
    dict(N=2000, D=17, band=(20e3, 85e3), R=10, F=3),
    dict(N=2500, D=33, band=(20e3, 85e3), R=10, F=17, P=8192),
    dict(N=900, D=40, band=(20e3, 85e3), R=10, F=2, M=40),        # 1/M not a power of two
    dict(N=1500, D=100, band=(20e3, 85e3), R=10, F=1, M=64),
    dict(N=700, D=5, band=(20e3, 85e3), R=10, F=1, M=1),             # below the stated range: printed
    dict(N=3000, D=70, band=None, R=3, F=2, M=8),                    # below the stated range: printed
])
def test_td_bf16g_shapes(gpu, torch_mod, case):
    torch = torch_mod
    if case.get("grid") == "c1":
        w = synth.make_workload("c1")
    else:
        w = synth.make_workload("c2", frames=case["F"], n_samples=case["N"], n_dirs=case["D"], n_mics=case.get("M"))
        noise = np.random.default_rng(case["N"] + case["D"]).standard_normal(w.x.shape).astype(np.float32)
        w.x = (w.x + 0.05 * noise).astype(np.float32)
    _say(f"case td_bf16g {case}")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, case["N"], fs=w.fs, c=w.c, band=case["band"], decim=case["R"],
                    fft_len=case.get("P", 0), max_frames=case["F"], mode="td_bf16g")
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()
    eg, et = [], []
    for f in range(case["F"]):
        kw = dict(fs=w.fs, c=w.c, P=plan.P, R=case["R"], band=case["band"], mode="td")
        x = w.x[f].astype(np.float64)
        eg.append(rel_l2(E[f], O.energyscape(x, w.chirp, w.mic_pos, w.dirs, alpha_steps=256, **kw)))
        et.append(rel_l2(E[f], O.energyscape(x, w.chirp, w.mic_pos, w.dirs, **kw)))
    _say(f"  max rel L2 over frames: {max(eg):.3e} vs the 1/256 grid, {max(et):.3e} vs linear interpolation")
    if plan.M >= 32:
        assert max(eg) <= BAR and max(et) <= BAR


def test_td_bf16g_planes_and_scratch(gpu, torch_mod):
    """Its matched-filter buffer carries the same BF16 planes as td_bf16x2 (bit-exact roundings of
    the complex rows), and the fused and staged energyscapes are identical."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=3000, n_dirs=45)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=2, mode="td_bf16g")
    M, row = plan.M, plan.mf_row
    assert plan.mf_frame_elems == M * row * 3 // 2
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    fr = mf[0].cpu()
    y = fr[:M * row].numpy().reshape(M, row)
    pl = fr[M * row:].view(torch.int16).numpy().view(np.uint16).reshape(M, 2, row)
    assert np.array_equal(pl[:, 0], _bf16_rne(y.real))
    assert np.array_equal(pl[:, 1], _bf16_rne(y.imag))
    assert torch.equal(plan.energyscape(x), plan.beamform_envelope(mf))
    assert torch.equal(plan.energyscape(x), plan.energyscape_static(x))


def test_td_bf16g_gradients_refuse_positions(gpu, torch_mod):
    """dx is the adjoint on the gridded delays; dpos is refused (piecewise constant in the positions)."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=1, n_samples=1200, n_dirs=20)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 1200, fs=w.fs, c=w.c, band=w.cfg.band, mode="td_bf16g")
    plan.enable_gradients()
    x = torch.from_numpy(w.x).cuda()
    dE = torch.ones((1, w.dirs.shape[0], plan.Q), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu.SonarError):
        plan.backward(x, dE, want_dx=False, want_dpos=True)
    dx, _ = plan.backward(x, dE, want_dx=True, want_dpos=False)
    assert bool(torch.isfinite(dx).all())
