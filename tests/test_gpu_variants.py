"""Variant readings on the GPU against the FP64 oracle: integer-delay delay-and-sum
(TD_NEAREST), 4-point Lagrange fractional delay (TD_CUBIC) and the IIR (Butterworth,
causal lfilter) envelope.  FP32 bar: relative
L2 <= 1e-5 per energyscape."""

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


@pytest.mark.parametrize("mode,sections", [("td", 2), ("fd_fp32", 2), ("td_nearest", 1), ("td", 3)])
def test_iir_envelope_matches_oracle(gpu, torch_mod, mode, sections):
    import scipy.signal as ss
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=4096, n_dirs=13)
    _say(f"case iir envelope: mode={mode} sections={sections} N=4096 D=13 F=2")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                    decim=w.cfg.decim, mode=mode, max_frames=2)
    x = torch.from_numpy(w.x).cuda()
    E_fir = plan.energyscape(x).cpu().numpy()
    if sections == 3:
        sos = ss.butter(6, 0.15, output="sos")           # a custom cascade: order 6, -3 dB at 0.075 fs
        plan.set_envelope_iir(3, sos)
        bco, aco = np.array([1.0]), np.array([1.0])
        for q in sos:
            bco, aco = np.polymul(bco, q[:3]), np.polymul(aco, q[3:])
    else:
        plan.set_envelope_iir(sections)                  # Butterworth of order 2 S at fs / (2R)
        bco, aco = O.butterworth_lowpass(2 * sections, 1.0 / (2 * w.cfg.decim))
    E = plan.energyscape(x).cpu().numpy()
    omode = "fd" if mode.startswith("fd") else mode
    for f in range(2):
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                           band=w.cfg.band, mode=omode, iir=(bco, aco))
        err = rel_l2(E[f], Eo)
        _say(f"iir {mode} S={sections} frame {f}: rel L2 {err:.2e}")
        assert err <= 1e-5
    # the stage calls give the same result
    mf = plan.matched_filter(x)
    E_stage = plan.envelope(plan.beamform(mf)).cpu().numpy()
    assert np.array_equal(E_stage, E)
    # gradients stay with the FIR envelope
    with pytest.raises(gpu.SonarError):
        plan.vjp(mf, plan.beamform(mf), torch.zeros((2, plan.D, plan.Q), dtype=torch.float32, device="cuda"))
    # and switching back restores the FIR result exactly
    plan.set_envelope_iir(0)
    assert np.array_equal(plan.energyscape(x).cpu().numpy(), E_fir)


@pytest.mark.parametrize("cfg,n_samples,n_dirs,frames", [("c1", None, None, 1), ("c2", 4096, 37, 2),
                                                         ("c2", 16384, 1500, 1)])
def test_td_cubic_matches_oracle(gpu, torch_mod, cfg, n_samples, n_dirs, frames):
    torch = torch_mod
    w = synth.make_workload(cfg, frames=frames, n_samples=n_samples, n_dirs=n_dirs)
    D = w.dirs.shape[0]
    _say(f"case td_cubic: {cfg} N={w.x.shape[2]} D={D} F={frames}")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, band=w.cfg.band,
                    decim=w.cfg.decim, mode="td_cubic", max_frames=frames)
    x = torch.from_numpy(w.x).cuda()
    E = plan.energyscape(x).cpu().numpy()
    sel = np.arange(0, D, 50) if D > 200 else np.arange(D)
    for f in range(frames):
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                           band=w.cfg.band, mode="td_cubic", dir_index=sel)
        err = rel_l2(E[f][sel], Eo)
        _say(f"td_cubic {cfg} frame {f}: rel L2 {err:.2e}")
        assert err <= 1e-5
    # closer to the exact (FD) energyscape than linear interpolation
    Ef = O.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                       band=w.cfg.band, mode="fd", dir_index=sel)
    Et = O.energyscape(w.x[0].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P,
                       band=w.cfg.band, mode="td", dir_index=sel)
    _say(f"td_cubic vs exact {rel_l2(E[0][sel], Ef):.2e}, linear vs exact {rel_l2(Et, Ef):.2e}")
    assert rel_l2(E[0][sel], Ef) < rel_l2(Et, Ef)
    # the beam stage agrees with the fused path
    mf = plan.matched_filter(x)
    beam = plan.beamform(mf)
    assert rel_l2(plan.envelope(beam).cpu().numpy(), E) <= 1e-6
    # gradients of the cubic reading exist (their parity is in test_gpu_grad.py)
    _, dx, dpos = plan.vjp(mf, beam, torch.ones((frames, plan.D, plan.Q), dtype=torch.float32, device="cuda"))
    assert bool(torch.isfinite(dx).all()) and np.all(np.isfinite(dpos))


def test_td_cubic_positions_and_limits(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=11)
    _say("case td_cubic set_positions / 64-mic limit")
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, decim=w.cfg.decim, mode="td_cubic")
    pos2 = w.mic_pos + np.random.default_rng(np.random.SeedSequence([5, 0, 0, 2])).normal(0, 0.5e-3, w.mic_pos.shape)
    plan.set_positions(pos2)
    E = plan.energyscape(torch.from_numpy(w.x).cuda()).cpu().numpy()[0]
    Eo = O.energyscape(w.x[0].astype(np.float64), w.chirp, pos2, w.dirs, fs=w.fs, c=w.c, P=plan.P, mode="td_cubic")
    assert rel_l2(E, Eo) <= 1e-5
    pos65 = np.zeros((65, 3))
    pos65[:, 0] = np.linspace(-0.01, 0.01, 65)
    with pytest.raises(gpu.SonarError):
        gpu.Plan(pos65, w.chirp, w.dirs, w.x.shape[2], fs=w.fs, c=w.c, mode="td_cubic")
