"""Parity of the frequency-domain beamformer modes with the FP64 oracle (GPU).

Each mode is compared with the oracle's exact-fractional-delay mode on the
same inputs.  Bars: FD_FP32 and FD_BF16X3 relative L2 <= 1e-5, FD_BF16
(operands rounded to BF16 on MFMA) <= 1e-3, per energyscape.
"""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu

BARS = {"fd_fp32": 1e-5, "fd_bf16x3": 1e-5, "fd_bf16": 1e-3}
# The beam spectrum before the envelope: FD_BF16 rounds each steering component to one BF16 term
# (relative error at most u = 2^-8, RMS at most u / sqrt(3)); away from the steered reflectors the
# sum over microphones is incoherent, so that relative error carries over to the spectrum instead of
# averaging down (the envelope's low-pass does average it: 1e-3 per energyscape)
STAGE_BARS = {"fd_fp32": 1e-5, "fd_bf16x3": 1e-5, "fd_bf16": 2.0 ** -8 / np.sqrt(3.0)}


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


@pytest.mark.parametrize("mode", ["fd_fp32", "fd_bf16x3", "fd_bf16"])
def test_c1_fd_energyscape(gpu, torch_mod, mode):
    torch = torch_mod
    w = synth.make_workload("c1")
    _say(f"case c1 {mode}: M=32 N=4096 D=91")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 4096, fs=w.fs, c=w.c, mode=mode)
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()[0]
    Eo = O.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                       R=10, mode="fd")
    err = rel_l2(E, Eo)
    _say(f"  {mode} rel L2 = {err:.3e}")
    assert err <= BARS[mode]


@pytest.mark.parametrize("mode", ["fd_fp32", "fd_bf16x3", "fd_bf16"])
def test_fd_beam_spectrum_stage(gpu, torch_mod, mode):
    """sonar_beam_spectrum (the per-bin GEMM alone) against the spectrum of the oracle's beam: the
    oracle's exact-delay beam over all of Z_P, transformed back, is B_d on every bin."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=3000, n_dirs=21)
    _say(f"case fd beam spectrum: {mode} M=32 N=3000 D=21 F=2")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=2, mode=mode)
    S = plan.query(gpu.Q_BEAM_SPEC_STRIDE)
    k_lo, kb = plan.band_lo_bin, plan.band_bins
    assert S >= kb and S % 16 == 0
    assert plan.query(gpu.Q_FD_FUSED) == 1 and plan.query(gpu.Q_FD_PHASE_LEN) >= kb // 2
    mf = plan.matched_filter(torch.from_numpy(w.x).cuda())
    B = plan.beam_spectrum(mf).cpu().numpy()
    Dl = O.delays(w.mic_pos, w.dirs, w.fs, w.c)
    for f in range(2):
        Y = O.matched_filter_spectrum(w.x[f].astype(np.float64), w.chirp, plan.P, w.fs, w.cfg.band)
        Bo = np.fft.fft(O.das_fd(Y, Dl, np.arange(plan.P)), axis=1)[:, k_lo:k_lo + kb]
        err = rel_l2(B[f][:, :kb], Bo)
        _say(f"  frame {f}: beam spectrum rel L2 = {err:.3e} (bar {STAGE_BARS[mode]:.2e})")
        assert err <= STAGE_BARS[mode]
    # the energyscape from the same plan is the spectrum's inverse + envelope
    assert torch.equal(plan.beamform_envelope(mf), plan.beamform_envelope(mf))


def test_fd_beam_spectrum_refused_for_time_domain(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=5)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 4096, fs=w.fs, c=w.c, mode="td")
    mf = plan.matched_filter(torch.from_numpy(w.x).cuda())
    out = torch.empty((1, 5, 16), dtype=torch.complex64, device="cuda")
    with pytest.raises(gpu.SonarError) as ei:
        gpu._check(gpu.load().sonar_beam_spectrum(plan._h, gpu.ctypes.c_void_p(mf.data_ptr()), 1,
                                                   gpu.ctypes.c_void_p(out.data_ptr()), gpu._stream_handle(None)),
                   "sonar_beam_spectrum")
    assert ei.value.status == gpu.SONAR_E_INVALID
    assert plan.query(gpu.Q_BEAM_SPEC_STRIDE) == 0


def test_fd_stages(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c2", n_samples=3000, n_dirs=21)
    _say("case fd stages: M=32 N=3000 D=21 band 20-85 kHz")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, fs=w.fs, c=w.c, band=w.cfg.band, mode="fd_fp32")
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    beam = plan.beamform(mf)
    E = plan.envelope(beam)
    E2 = plan.beamform_envelope(mf)
    torch.cuda.synchronize()
    xf = w.x[0].astype(np.float64)
    Y = O.matched_filter_spectrum(xf, w.chirp, plan.P, w.fs, w.cfg.band)
    k_lo, kb = plan.band_lo_bin, plan.band_bins
    assert np.all(Y[:, :k_lo] == 0) and np.all(Y[:, k_lo + kb:] == 0)
    band = mf.cpu().numpy()[0].reshape(kb, plan.M)
    e_mf = rel_l2(band, Y[:, k_lo:k_lo + kb].T)
    _say(f"  matched filter (band bins) rel L2 = {e_mf:.3e}")
    assert e_mf <= 1e-5
    Dl = O.delays(w.mic_pos, w.dirs, w.fs, w.c)
    b_ref = O.das_fd(Y, Dl, O.beam_window_indices(0, plan.Q, 10, plan.K))
    e_b = rel_l2(beam.cpu().numpy()[0], b_ref)
    _say(f"  beamform rel L2 = {e_b:.3e}")
    assert e_b <= 1e-5
    Eo = O.envelope(b_ref, O.default_lowpass(10), plan.Q, 10)
    for name, got in (("envelope", E), ("beamform+envelope", E2)):
        e = rel_l2(got.cpu().numpy()[0], Eo)
        _say(f"  {name} rel L2 = {e:.3e}")
        assert e <= 1e-5


@pytest.mark.parametrize("case", [
    dict(N=2000, D=17, band=(20e3, 85e3), R=10, F=3, mode="fd_fp32"),
    dict(N=1001, D=1, band=None, R=7, F=1, mode="fd_bf16x3"),
    dict(N=3000, D=70, band=None, R=3, F=2, taps=5, gate=(100, 2950), mode="fd_fp32"),
    dict(N=700, D=5, band=(20e3, 85e3), R=10, F=1, M=1, mode="fd_fp32"),
    dict(N=2500, D=33, band=(20e3, 85e3), R=10, F=17, P=8192, mode="fd_bf16"),
    dict(N=200, D=6, band=None, R=2, F=2, chirp=(25e3, 80e3, 1e-4), mode="fd_fp32"),   # unfused inverse
    dict(N=900, D=9, band=(20e3, 85e3), R=10, F=2, M=40, mode="fd_bf16x3"),            # two microphone chunks
])
def test_fd_odd_shapes(gpu, torch_mod, case):
    torch = torch_mod
    kw = {"chirp_params": case["chirp"]} if "chirp" in case else {}
    w = synth.make_workload("c2", frames=case["F"], n_samples=case["N"], n_dirs=case["D"],
                            n_mics=case.get("M"), **kw)
    _say(f"case {case}")
    noise = np.random.default_rng(case["N"] + case["D"]).standard_normal(w.x.shape).astype(np.float32)
    w.x = (w.x + 0.05 * noise).astype(np.float32)
    taps = np.array([0.1, 0.2, 0.4, 0.2, 0.1]) if "taps" in case else None
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, case["N"], fs=w.fs, c=w.c, band=case["band"],
                    decim=case["R"], taps=taps, gate=case.get("gate"), fft_len=case.get("P", 0),
                    max_frames=case["F"], mode=case["mode"])
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()
    for f in range(case["F"]):
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c,
                           P=plan.P, R=case["R"], taps=taps, band=case["band"], gate=case.get("gate"),
                           mode="fd")
        err = rel_l2(E[f], Eo)
        _say(f"  frame {f}: rel L2 = {err:.3e}")
        assert err <= BARS[case["mode"]]


def test_c2_no_band_fd_unfused(gpu, torch_mod):
    """No band mask: 16385 stored bins, inverse transform through the beam workspace."""
    torch = torch_mod
    w = synth.make_workload("c2")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 16384, fs=w.fs, c=w.c, band=None, mode="fd_fp32")
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()[0]
    sample = np.array([3, 400, 1200])
    Eo = O.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                       R=10, band=None, mode="fd", dir_index=sample)
    err = rel_l2(E[sample], Eo)
    _say(f"case c2 no band fd_fp32: sampled rel L2 = {err:.3e}")
    assert err <= 1e-5


def test_fd_deterministic(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=3000, n_dirs=40)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=2,
                    mode="fd_bf16")
    x = torch.from_numpy(w.x).cuda()
    assert torch.equal(plan.energyscape(x).cpu(), plan.energyscape(x).cpu())
