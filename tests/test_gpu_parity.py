"""Parity of the HIP library with the FP64 oracle (GPU).

Every comparison runs the library through the C ABI (the ctypes binding) on
seeded synthetic inputs and checks it element by element against the oracle
on the same inputs.  FP32 path bar: relative L2 error <= 1e-5 per energyscape
(and per stage output); the error of every energyscape is printed.
"""

import math
import sys

import numpy as np
import pytest

import oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def _plan(gpu, w, **kw):
    args = dict(fs=w.fs, c=w.c, band=w.cfg.band, decim=w.cfg.decim)
    args.update(kw)
    return gpu.Plan(w.mic_pos, w.chirp, w.dirs, w.x.shape[2], **args)


def _fp64_oracle(w, frame, **kw):
    P = kw.pop("P")
    return O.energyscape(w.x[frame].astype(np.float64), w.chirp, w.mic_pos, w.dirs,
                         fs=w.fs, c=w.c, P=P, mode="td", **kw)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def test_c1_energyscape_matches_oracle(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c1")
    _say("case c1: M=32 N=4096 D=91 F=1")
    plan = _plan(gpu, w)
    x = torch.from_numpy(w.x).cuda()
    E = plan.energyscape(x).cpu().numpy()
    Eo = _fp64_oracle(w, 0, P=plan.P, R=10, band=w.cfg.band)
    err = rel_l2(E[0], Eo)
    _say(f"c1 energyscape rel L2 = {err:.3e}")
    assert E.shape == (1, 91, 410)
    assert err <= TOL_F32


def test_c1_stages_match_oracle(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=37)
    _say("case c1 stages: M=32 N=4096 D=37")
    plan = _plan(gpu, w)
    x = torch.from_numpy(w.x).cuda()
    mf = plan.matched_filter(x)
    beam = plan.beamform(mf)
    E = plan.envelope(beam)
    E2 = plan.beamform_envelope(mf)
    torch.cuda.synchronize()
    xf = w.x[0].astype(np.float64)
    yhat = O.matched_filter(xf, w.chirp, plan.P, w.fs, w.cfg.band)
    # MF rows: element i holds yhat[(origin + i) mod P]
    mf_np = mf.cpu().numpy()[0].reshape(plan.M, plan.mf_row)
    idx = np.mod(plan.mf_origin + np.arange(plan.mf_row), plan.P)
    e_mf = rel_l2(mf_np, yhat[:, idx])
    _say(f"matched filter rel L2 = {e_mf:.3e}")
    assert e_mf <= TOL_F32
    Dl = O.delays(w.mic_pos, w.dirs, w.fs, w.c)
    n_idx = O.beam_window_indices(0, plan.Q, 10, plan.K)
    b_ref = O.das_td(yhat, Dl, n_idx)
    e_b = rel_l2(beam.cpu().numpy()[0], b_ref)
    _say(f"beamform rel L2 = {e_b:.3e}")
    assert e_b <= TOL_F32
    # envelope stage in isolation: oracle envelope of the GPU's own beam
    taps = O.default_lowpass(10)
    Eo_stage = O.envelope(beam.cpu().numpy()[0].astype(np.complex128), taps, plan.Q, 10)
    e_env = rel_l2(E.cpu().numpy()[0], Eo_stage)
    _say(f"envelope rel L2 = {e_env:.3e}")
    assert e_env <= TOL_F32
    Eo = O.envelope(b_ref, taps, plan.Q, 10)
    e_fused = rel_l2(E2.cpu().numpy()[0], Eo)
    _say(f"beamform+envelope rel L2 = {e_fused:.3e}")
    assert e_fused <= TOL_F32


@pytest.mark.parametrize("case", [
    dict(name="c2", N=2000, D=17, band=(20e3, 85e3), R=10, F=3),           # ragged D tile, batch
    dict(name="c2", N=1001, D=1, band=None, R=7, F=1),                     # odd N, one direction
    dict(name="c2", N=3000, D=40, band=None, R=3, F=2, taps=5, gate=(100, 2950)),
    dict(name="c2", N=700, D=5, band=(20e3, 85e3), R=10, F=1, M=1),        # single microphone
    dict(name="c2", N=2500, D=33, band=(20e3, 85e3), R=10, F=1, P=8192),   # explicit larger P
    dict(name="c2", N=200, D=6, band=None, R=2, F=2, chirp=(25e3, 80e3, 1e-4)),   # short sweep, small P
])
def test_odd_shapes_match_oracle(gpu, torch_mod, case):
    torch = torch_mod
    kw = {}
    if "chirp" in case:
        kw["chirp_params"] = case["chirp"]
    w = synth.make_workload(case["name"], frames=case["F"], n_samples=case["N"], n_dirs=case["D"],
                            n_mics=case.get("M"), **kw)
    _say(f"case {case}")
    taps = None
    if "taps" in case:
        taps = np.array([0.1, 0.2, 0.4, 0.2, 0.1])
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, case["N"], fs=w.fs, c=w.c, band=case["band"],
                    decim=case["R"], taps=taps, gate=case.get("gate"), fft_len=case.get("P", 0),
                    max_frames=case["F"])
    # seeded broadband noise on top of the echoes, so that short windows without echoes still carry signal
    noise = np.random.default_rng(case["N"] + case["D"]).standard_normal(w.x.shape).astype(np.float32)
    w.x = (w.x + 0.05 * noise).astype(np.float32)
    x = torch.from_numpy(w.x).cuda()
    E = plan.energyscape(x).cpu().numpy()
    for f in range(case["F"]):
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c,
                           P=plan.P, R=case["R"], taps=taps, band=case["band"], gate=case.get("gate"),
                           mode="td")
        err = rel_l2(E[f], Eo)
        _say(f"  frame {f}: rel L2 = {err:.3e}  (Q={plan.Q}, P={plan.P})")
        assert E[f].shape == Eo.shape
        assert err <= TOL_F32


# compute-only bar per mode (against the oracle on the rounded samples) and its oracle reading
HALF_MODES = {"td": (1e-5, "td", None), "td_bf16x2": (1e-3, "td", None), "td_f16": (3e-4, "td", None),
              "fd_bf16": (1e-3, "fd", None), "fd_bf16x3": (1e-5, "fd", None), "td_bf16": (1e-3, "td", None),
              "td_bf16g": (1e-3, "td", None)}


@pytest.mark.parametrize("mode", list(HALF_MODES))
@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_half_precision_samples(gpu, torch_mod, dt, mode):
    """FP16 / BF16 samples into every mode: the compute-only error (against the oracle on the rounded
    samples) meets the mode's bar; the end-to-end error against the oracle on the FP32 samples, which
    adds the input rounding, stays within 1e-3."""
    torch = torch_mod
    w = synth.make_workload("c2", frames=2, n_samples=4000, n_dirs=96)
    _say(f"case half samples {dt} -> {mode}")
    bar, omode, _ = HALF_MODES[mode]
    tdt = {"f16": torch.float16, "bf16": torch.bfloat16}[dt]
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 4000, fs=w.fs, c=w.c, band=w.cfg.band, sample_dtype=dt,
                    max_frames=2, mode=mode)
    xh = torch.from_numpy(w.x).to(tdt)
    E = plan.energyscape(xh.cuda()).cpu().numpy()
    xr = xh.float().numpy().astype(np.float64)            # the rounded samples
    for f in range(2):
        Eo_r = O.energyscape(xr[f], w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, P=plan.P, R=10,
                             band=w.cfg.band, mode=omode)
        Eo = O.energyscape(w.x[f].astype(np.float64), w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c,
                           P=plan.P, R=10, band=w.cfg.band, mode=omode)
        e_compute = rel_l2(E[f], Eo_r)
        e_total = rel_l2(E[f], Eo)
        _say(f"  {dt} {mode} frame {f}: compute-only rel L2 = {e_compute:.3e}, vs FP32 samples = {e_total:.3e}")
        assert e_compute <= bar
        assert e_total <= 1e-3


def test_deterministic_and_batch_independent(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c2", frames=3, n_samples=3000, n_dirs=50)
    plan = gpu.Plan(w.mic_pos, w.chirp, w.dirs, 3000, fs=w.fs, c=w.c, band=w.cfg.band, max_frames=3)
    x = torch.from_numpy(w.x).cuda()
    E1 = plan.energyscape(x).cpu()
    E2 = plan.energyscape(x).cpu()
    assert torch.equal(E1, E2)
    E_single = plan.energyscape(x[1:2].contiguous()).cpu()
    assert torch.equal(E_single[0], E1[1])


def test_physics_reflectors_recovered(gpu, torch_mod):
    torch = torch_mod
    pos = synth.planar_array(32, 0.035, np.random.default_rng(123))
    refl = [(1.0, np.array([math.sin(math.radians(30)), 0, math.cos(math.radians(30))]), 1.0),
            (0.7, np.array([math.sin(math.radians(-50)), 0, math.cos(math.radians(-50))]), 0.8)]
    x = synth.simulate_frame(pos, (25e3, 80e3, 1e-3), refl, 4096, None, None)
    dirs = synth.azimuth_grid(91)
    plan = gpu.Plan(pos, synth.linear_chirp(), dirs, 4096, fs=synth.FS_HZ, c=synth.C_MPS)
    E = plan.energyscape(torch.from_numpy(x[None].astype(np.float32)).cuda()).cpu().numpy()[0]
    az = np.degrees(np.arctan2(dirs[:, 0], dirs[:, 2]))
    for r, u, _ in refl:
        q = int(round(2 * r * synth.FS_HZ / synth.C_MPS / 10))
        sub = E[:, q - 5:q + 6]
        d_pk = np.unravel_index(np.argmax(sub), sub.shape)[0]
        assert abs(az[d_pk] - math.degrees(math.atan2(u[0], u[2]))) <= 2.0


def test_exec_errors(gpu, torch_mod):
    torch = torch_mod
    w = synth.make_workload("c1", n_dirs=5)
    plan = _plan(gpu, w, max_frames=1)
    x2 = torch.zeros((2, 32, 4096), device="cuda")
    with pytest.raises(gpu.SonarError) as ei:
        plan.energyscape(x2)
    assert ei.value.status == gpu.SONAR_E_INVALID
    with pytest.raises(TypeError):
        plan.energyscape(torch.zeros((1, 32, 4096), device="cuda", dtype=torch.float16))
    with pytest.raises(gpu.SonarError) as ei:
        gpu.Plan(w.mic_pos, w.chirp, w.dirs, 4096, fs=w.fs, c=w.c, fft_len=1 << 20)
    assert ei.value.status == gpu.SONAR_E_UNSUPPORTED
