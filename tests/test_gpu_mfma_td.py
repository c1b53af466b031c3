"""Parity of the BF16-MFMA time-domain beamformer (mode td_bf16) with the FP64 oracle (GPU).

The mode computes the same linear-interpolation delay-and-sum as the FP32
time-domain path, as a dense product on matrix cores: tap weights rounded to
BF16, samples carried as two BF16 terms, FP32 accumulation.  Bar: relative L2
<= 1e-3 per energyscape against the oracle's time-domain mode.  Its matched
filter and its stand-alone beamform/envelope calls are the FP32 kernels, held
to 1e-5.
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


def _oracle(w, f, plan, **kw):
    return O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                         mode="td", **kw)


def test_c1_td_bf16(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c1")
    _say("case c1 td_bf16: M=32 N=4096 D=91")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 4096, fs=w.fs, c=w.c, mode="td_bf16")
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()[0]
    err = rel_l2(E, _oracle(w, 0, plan, R=10))
    _say(f"  rel L2 = {err:.3e}")
    assert err <= BAR


def test_td_bf16_stages(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c2", n_samples=3000, n_dirs=45)
    _say("case td_bf16 stages: M=32 N=3000 D=45 band 20-85 kHz")
    kw = dict(fs=w.fs, c=w.c, band=w.cfg.band)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, mode="td_bf16", **kw)
    ref = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, mode="td", **kw)
    assert plan.mf_row == ref.mf_row and plan.mf_origin == ref.mf_origin
    assert plan.mf_frame_elems == 2 * plan.M * plan.mf_row
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    check_planes(mf, plan)
    beam = plan.beamform(mf)
    E = plan.envelope(beam)
    E2 = plan.beamform_envelope(mf)
    E3 = plan.energyscape(x)
    torch.cuda.synchronize()
    assert torch.equal(mf[:, :plan.M * plan.mf_row], ref.matched_filter(x))
    xf = w.x[0].astype(np.float64)
    yhat = O.matched_filter(xf, w.chirp, plan.P, w.fs, w.cfg.band)
    Dl = O.delays(w.mic_pos, w.dirs, w.fs, w.c)
    b_ref = O.das_td(yhat, Dl, O.beam_window_indices(0, plan.Q, 10, plan.K))
    e_b = rel_l2(beam.cpu().numpy()[0], b_ref)
    _say(f"  beamform (FP32) rel L2 = {e_b:.3e}")
    assert e_b <= 1e-5
    Eo = O.envelope(b_ref, O.default_lowpass(10), plan.Q, 10)
    e_env = rel_l2(E.cpu().numpy()[0], Eo)
    _say(f"  envelope (FP32) rel L2 = {e_env:.3e}")
    assert e_env <= 1e-5
    for name, got in (("beamform+envelope", E2), ("energyscape", E3)):
        e = rel_l2(got.cpu().numpy()[0], Eo)
        _say(f"  {name} rel L2 = {e:.3e}")
        assert e <= BAR
    assert torch.equal(E2, E3)


def _bf16_rne(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def check_planes(mf, plan):
    """The BF16 planes after the complex rows: bit-exact hi/lo split of the same samples."""
    import torch
    M, row = plan.M, plan.mf_row
    fr = mf[0].cpu()
    y = fr[:M * row].numpy().reshape(M, row)
    pl = fr[M * row:].view(torch.int16).numpy().view(np.uint16).reshape(M, 4, row)
    for c, part in enumerate((y.real, y.imag)):
        hi = _bf16_rne(part)
        hv = (hi.astype(np.uint32) << 16).view(np.float32)
        lo = _bf16_rne(part.astype(np.float32) - hv)
        assert np.array_equal(pl[:, 2 * c], hi)
        assert np.array_equal(pl[:, 2 * c + 1], lo)


def _sphere(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("case", [
    dict(N=2000, D=17, band=(20e3, 85e3), R=10, F=3),
    dict(N=1001, D=1, band=None, R=7, F=1),
    dict(N=3000, D=70, band=None, R=3, F=2, taps=5, gate=(100, 2950)),
    dict(N=700, D=5, band=(20e3, 85e3), R=10, F=1, M=1),
    dict(N=2500, D=33, band=(20e3, 85e3), R=10, F=17, P=8192),
    dict(N=900, D=40, band=(20e3, 85e3), R=10, F=2, M=40),          # three microphone chunks, ragged
    dict(N=1500, D=100, band=(20e3, 85e3), R=10, F=1, sphere=True),  # both hemispheres, random order
    dict(N=4000, D=64, band=(20e3, 85e3), R=1, F=1, taps=1),         # no decimation, single tap
])
def test_td_bf16_odd_shapes(gpu, torch_mod, case):
    torch = torch_mod
    w = synth.make_workload("c2", frames=case["F"], n_samples=case["N"], n_dirs=case["D"], n_mics=case.get("M"))
    if case.get("sphere"):
        w.dirs = _sphere(case["D"], 11)
    _say(f"case {case}")
    noise = np.random.default_rng(case["N"] + case["D"]).standard_normal(w.x.shape).astype(np.float32)
    w.x = (w.x + 0.05 * noise).astype(np.float32)
    taps = None
    if "taps" in case:
        taps = np.array([1.0]) if case["taps"] == 1 else np.array([0.1, 0.2, 0.4, 0.2, 0.1])
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, case["N"], fs=w.fs, c=w.c, band=case["band"],
                    decim=case["R"], taps=taps, gate=case.get("gate"), fft_len=case.get("P", 0),
                    max_frames=case["F"], mode="td_bf16")
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()
    for f in range(case["F"]):
        Eo = _oracle(w, f, plan, R=case["R"], taps=taps, band=case["band"], gate=case.get("gate"))
        err = rel_l2(E[f], Eo)
        _say(f"  frame {f}: rel L2 = {err:.3e}")
        assert err <= BAR


def test_td_bf16_deterministic(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=3000, n_dirs=40)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=2,
                    mode="td_bf16")
    x = torch.from_numpy(w.x).cuda()
    assert torch.equal(plan.energyscape(x).cpu(), plan.energyscape(x).cpu())
