"""Parity of the FP16-MFMA time-domain beamformer (mode td_f16) with the FP64 oracle (GPU).

The mode is the linear-interpolation beamformer with the fractional delays on a grid of
1/2048 sample (exact FP16 weights) and the samples as one FP16 term scaled per frame by a
power of two.  Bars: relative L2 <= 2e-4 against the oracle's gridded reading (what the
mode computes: the only differences are two FP16 roundings, of the samples and of |b| before
the low-pass, each at most 2^-12 relative, and FP32 sums; with one microphone nothing averages
them down), and <= 3e-4 against the oracle's plain time-domain mode (the grid moves each delay
by at most 1/4096 sample), for every array size including one microphone.  The sample scale is
checked bit by bit (planes = FP16 of 2^e yhat, header = 2^-e / M, 2^e max|yhat| < 2^14), and
a power-of-two change of the input's scale changes the energyscape by exactly that factor.
"""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu

BAR_GRID = 2e-4
BAR_TD = 3e-4
STEPS = 2048


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _check(w, E, P, R, band, f, label, dir_index=None):
    x = w.x[f].astype(np.float64)
    kw = dict(fs=w.fs, c=w.c, P=P, R=R, band=band, mode="td", dir_index=dir_index)
    Eg = O.energyscape(x, w.chirp, w.mic_pos, w.dirs, alpha_steps=STEPS, **kw)
    Et = O.energyscape(x, w.chirp, w.mic_pos, w.dirs, **kw)
    eg, et = rel_l2(E, Eg), rel_l2(E, Et)
    _say(f"  {label}: rel L2 vs gridded oracle {eg:.3e}, vs td oracle {et:.3e}")
    assert eg <= BAR_GRID and et <= BAR_TD
    return eg, et


def test_c1_td_f16(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c1")
    _say("case c1 td_f16: M=32 N=4096 D=91")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 4096, fs=w.fs, c=w.c, mode="td_f16")
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()[0]
    _check(w, E, plan.P, 10, None, 0, "c1")


def test_td_f16_planes_scale_and_header(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=3000, n_dirs=45)
    w.x[1] *= 3.0e-3                                   # a second frame of another scale
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=2, mode="td_f16")
    M, row = plan.M, plan.mf_row
    assert plan.mf_frame_elems == M * row * 3 // 2 + 2
    mf = plan.matched_filter(torch.from_numpy(w.x).cuda())
    for f in range(2):
        fr = mf[f].cpu()
        y = fr[:M * row].numpy().reshape(M, row)
        pl = fr[M * row:M * row * 3 // 2].view(torch.int16).numpy().view(np.uint16).reshape(M, 2, row)
        head = float(fr[M * row * 3 // 2:].view(torch.float32).numpy()[0])
        e = int(round(-np.log2(head * M)))
        assert head == np.float32(np.ldexp(np.float32(1.0) / np.float32(M), -e))
        s = np.float32(2.0) ** e
        assert np.array_equal(pl[:, 0], (y.real * s).astype(np.float16).view(np.uint16))
        assert np.array_equal(pl[:, 1], (y.imag * s).astype(np.float16).view(np.uint16))
        peak = float(np.max(np.abs(y))) * float(s)
        _say(f"  frame {f}: e = {e}, 2^e max|yhat| = {peak:.1f}")
        assert 2.0 ** 4 < peak < 2.0 ** 14


@pytest.mark.parametrize("case", [
    dict(N=2000, D=17, band=(20e3, 85e3), R=10, F=3),
    dict(N=2500, D=33, band=(20e3, 85e3), R=10, F=17, P=8192),
    dict(N=900, D=40, band=(20e3, 85e3), R=10, F=2, M=40),
    dict(N=1500, D=100, band=(20e3, 85e3), R=10, F=1, M=64),
    dict(N=700, D=5, band=(20e3, 85e3), R=10, F=1, M=1),
    dict(N=3000, D=70, band=None, R=3, F=2, M=8),
])
def test_td_f16_shapes(gpu, torch_mod, case):
    torch = torch_mod
    w = synth.make_workload("c2", frames=case["F"], n_samples=case["N"], n_dirs=case["D"], n_mics=case.get("M"))
    _say(f"case td_f16 {case}")
    noise = np.random.default_rng(case["N"] + case["D"]).standard_normal(w.x.shape).astype(np.float32)
    w.x = (w.x + 0.05 * noise).astype(np.float32)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, case["N"], fs=w.fs, c=w.c, band=case["band"], decim=case["R"],
                    fft_len=case.get("P", 0), max_frames=case["F"], mode="td_f16")
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()
    for f in sorted({0, case["F"] // 2, case["F"] - 1}):
        _check(w, E[f], plan.P, case["R"], case["band"], f, f"frame {f}")


def test_td_f16_power_of_two_scale_and_zero_input(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=2500, n_dirs=40)
    _say("case td_f16 scale invariance: x 2^40, x 2^-40, zeros")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 2500, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=2, mode="td_f16")
    x = torch.from_numpy(w.x).cuda()
    E = plan.energyscape(x)
    for k in (40, -40):
        Ek = plan.energyscape(x * (2.0 ** k))
        assert torch.equal(Ek, E * (2.0 ** k)), k
    Ez = plan.energyscape(torch.zeros_like(x))
    assert torch.count_nonzero(Ez).item() == 0


def test_td_f16_gradient_support(gpu, torch_mod):
    """dx is the adjoint on the gridded delays; dpos is refused (the gridded delays are piecewise
    constant in the positions)."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=1, n_samples=1200, n_dirs=20)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 1200, fs=w.fs, c=w.c, band=w.cfg.band, mode="td_f16")
    plan.enable_gradients()
    x = torch.from_numpy(w.x).cuda()
    dE = torch.ones((1, w.dirs.shape[0], plan.Q), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu.SonarError):
        plan.backward(x, dE, want_dx=False, want_dpos=True)


@pytest.mark.parametrize("mode", ["td_f16", "td_bf16x2", "td_bf16"])
def test_fused_energyscape_equals_staged_calls(gpu, torch_mod, mode):
    """The fused call (whose matched filter skips the complex rows in the MFMA modes) equals the
    matched filter into a caller buffer (rows and planes) followed by the fused beamformer +
    envelope, bit for bit."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=3, n_samples=2200, n_dirs=50)
    _say(f"case fused vs staged: {mode}")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 2200, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=3, mode=mode)
    x = torch.from_numpy(w.x).cuda()
    E1 = plan.energyscape(x)
    E2 = plan.beamform_envelope(plan.matched_filter(x))
    assert torch.equal(E1, E2)


@pytest.mark.parametrize("gain", [1.0e6, 4.0, 1.0e-4, 1.0e-9])
def test_two_plane_modes_any_tap_gain(gpu, torch_mod, gain):
    """The two-plane MFMA modes run the low-pass on FP16 taps, scaled at plan time by a power of two
    that puts the largest tap near 2^14 and undone at the store: a filter with any gain gives the
    oracle's energyscape for that filter within the modes' bars."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=1, n_samples=1500, n_dirs=20)
    taps = O.default_lowpass(10) * gain
    _say(f"case tap gain {gain:g}")
    Eo = O.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=2048, R=10,
                       taps=taps, band=w.cfg.band, mode="td")
    for mode in ("td_bf16x2", "td_f16"):
        plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 1500, fs=w.fs, c=w.c, band=w.cfg.band, taps=taps, mode=mode)
        assert plan.P == 2048
        E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()[0]
        err = rel_l2(E, Eo)
        _say(f"  {mode}: rel L2 vs td oracle {err:.3e}")
        assert err <= (BAR_TD if mode == "td_f16" else 1e-3)
