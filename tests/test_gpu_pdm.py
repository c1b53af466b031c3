"""PDM front end on the GPU (sonar_pdm_demodulate) against the FP64 oracle.

Bars: every output within 1e-6 sum|h| of the oracle (sum|h| is the full-scale output of
the +-1 input), and a relative L2 error <= 1e-6 per frame for recordings at least one
filter long (shorter ones have only edge windows, whose small outputs come from
full-scale arithmetic).  Two kernels: where 15 D + K <= 1024 the int8 matrix-core one
(taps rounded to 29-bit integers, exact integer sums, one rounding at the end), else the
byte-table one (4 ceil(K/32) FP32 table entries, each an FP64 sum of 8 taps rounded
once, plus an FP32 prefix-sum correction for windows reaching past the recording; the
case with D = 64 runs it).  Shapes cover one and several words per tick, partial
words, ragged last tiles, windows cut by both ends of the recording, custom filters, and
the full 32 x 16384 x 10 size of the headline workload.
"""

import sys

import numpy as np
import pytest

import oracle as O
from workloads import pdm

pytestmark = pytest.mark.gpu

TOL_REL = 1e-6
TOL_FULL_SCALE = 1e-6


def _say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _words_tensor(torch, words):
    return torch.from_numpy(np.ascontiguousarray(words).view(np.int32)).cuda()


def _check(x_gpu, words, M, N, D, taps, label):
    x_o = np.stack([O.pdm_demodulate(words[f], M, N, D, taps) for f in range(words.shape[0])])
    full_scale = float(np.sum(np.abs(taps)))
    err_abs = float(np.max(np.abs(x_gpu - x_o))) / full_scale
    err_rel = max(float(np.linalg.norm(x_gpu[f] - x_o[f]) / max(np.linalg.norm(x_o[f]), 1e-30))
                  for f in range(words.shape[0]))
    _say(f"pdm {label}: rel L2 {err_rel:.2e}, max abs / full scale {err_abs:.2e}")
    assert err_abs <= TOL_FULL_SCALE, (label, err_abs)
    if N * D >= np.asarray(taps).size:
        assert err_rel <= TOL_REL, (label, err_rel)


def test_pdm_sigma_delta_recording_matches_oracle(gpu, torch_mod):
    torch = torch_mod
    w = pdm.make_pdm_workload("c2", frames=2, n_samples=4096, n_dirs=37)
    M, N, D = w.base.mic_pos.shape[0], w.n_out, w.decim
    _say(f"case pdm sigma-delta: M={M} N={N} D={D} F=2")
    dem = gpu.Pdm(M, N, D, max_frames=2)
    x = dem.demodulate(_words_tensor(torch, w.words)).cpu().numpy()
    _check(x, w.words, M, N, D, O.pdm_default_taps(D), "sigma-delta c2 N=4096")


@pytest.mark.parametrize("M,N,D,K", [
    (1, 1, 10, 0), (6, 7, 10, 0), (32, 1000, 10, 0), (33, 300, 3, 0), (64, 257, 1, 0),
    (100, 129, 16, 0), (128, 513, 10, 0), (32, 500, 10, 1), (32, 500, 10, 9), (5, 333, 7, 161),
    (32, 64, 4, 513), (8, 100, 64, 161), (40, 200, 64, 129),
])
def test_pdm_shapes_match_oracle(gpu, torch_mod, M, N, D, K):
    torch = torch_mod
    _say(f"case pdm shape: M={M} N={N} D={D} K={K or 'default'}")
    rng = np.random.default_rng(np.random.SeedSequence([7, M, N, D, K]))
    F = 2
    bits = rng.integers(0, 2, size=(F, M, N * D)).astype(bool)
    words = np.stack([pdm.pack_words(bits[f]) for f in range(F)])
    if K == 0:
        taps = O.pdm_default_taps(D)
        dem = gpu.Pdm(M, N, D, max_frames=F)
    else:
        taps = rng.standard_normal(K)
        dem = gpu.Pdm(M, N, D, taps=taps, max_frames=F)
    x = dem.demodulate(_words_tensor(torch, words)).cpu().numpy()
    _check(x, words, M, N, D, taps, f"M={M} N={N} D={D} K={taps.size}")


def test_pdm_full_size_sampled(gpu, torch_mod):
    """32 mics x 16384 samples x 10 ticks, 16 frames per launch (the bench's batch); every
    sample of frames 0, 7 and 15 against the oracle."""
    torch = torch_mod
    M, N, D, F = 32, 16384, 10, 16
    _say(f"case pdm full size: M={M} N={N} D={D} F={F}")
    rng = np.random.default_rng(np.random.SeedSequence([7, 1, 2, 3]))
    words = rng.integers(0, 2**32, size=(F, N * D, 1), dtype=np.uint64).astype(np.uint32)
    dem = gpu.Pdm(M, N, D, max_frames=F)
    x = dem.demodulate(_words_tensor(torch, words)).cpu().numpy()
    idx = [0, 7, 15]
    _check(x[idx], words[idx], M, N, D, O.pdm_default_taps(D), "full size, frames 0/7/15")


def test_pdm_then_energyscape(gpu, torch_mod):
    """PDM words -> samples -> energyscape through the library equals the oracle's energyscape of the
    oracle's demodulated samples (<= 1e-5), and stays within 5 % of the energyscape of the analog
    signal sampled at 450 kHz (the modulator's in-band noise)."""
    torch = torch_mod
    w = pdm.make_pdm_workload("c2", frames=1, n_samples=4096, n_dirs=37)
    b = w.base
    M, N, D = b.mic_pos.shape[0], w.n_out, w.decim
    _say(f"case pdm -> energyscape: M={M} N={N} D=37")
    dem = gpu.Pdm(M, N, D)
    plan = gpu.Plan(b.mic_pos, b.chirp, b.dirs, N, fs=b.fs, c=b.c, band=b.cfg.band, decim=b.cfg.decim, mode="td")
    x = dem.demodulate(_words_tensor(torch, w.words))
    E = plan.energyscape(x).cpu().numpy()[0]
    x_o = O.pdm_demodulate(w.words[0], M, N, D, O.pdm_default_taps(D))
    E_o = O.energyscape(x_o, b.chirp, b.mic_pos, b.dirs, fs=b.fs, c=b.c, P=plan.P, band=b.cfg.band, mode="td")
    err = float(np.linalg.norm(E - E_o) / np.linalg.norm(E_o))
    E_a = O.energyscape(w.analog[0][:, ::D][:, :N], b.chirp, b.mic_pos, b.dirs, fs=b.fs, c=b.c, P=plan.P,
                        band=b.cfg.band, mode="td")
    phys = float(np.linalg.norm(E_o - E_a) / np.linalg.norm(E_a))
    _say(f"pdm -> energyscape: rel L2 vs oracle {err:.2e}; oracle PDM vs analog {phys:.2e}")
    assert err <= 1e-5
    assert phys <= 5e-2


def test_pdm_errors(gpu, torch_mod):
    torch = torch_mod
    dem = gpu.Pdm(32, 100, 10, max_frames=1)
    words = torch.zeros((2, 1000, 1), dtype=torch.int32, device="cuda")
    with pytest.raises(gpu.SonarError):
        dem.demodulate(words)                      # F above max_frames
    with pytest.raises(ValueError):
        dem.demodulate(torch.zeros((1, 999, 1), dtype=torch.int32, device="cuda"))
