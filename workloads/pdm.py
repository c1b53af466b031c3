"""Seeded 1-bit PDM recordings (the raw microphone format of the sensor, §2).

The sensor's microphones deliver 1-bit sigma-delta pulse-density modulated
streams; the paper gives neither the PDM clock nor the modulator.  Inputs here:

* PDM clock 4.5 MHz = 10 x the 450 kHz sample rate the pipeline runs at (§2), so
  one output sample is 10 PDM ticks;
* analog signal: the echo model of ``synth.simulate_frame`` evaluated at the PDM
  tick instants, scaled so its peak is 0.5 of full scale (a sigma-delta loop is
  stable well below full scale);
* modulator: the textbook second-order loop with two delay-free integrators and
  a sign quantiser (Candy's double-integration modulator):
      i1 <- i1 + u - y,   i2 <- i2 + i1 - y,   y <- sign(i2) in {-1, +1};
* packing: tick t of an M-microphone recording is ceil(M/32) little-endian 32-bit
  words, microphone m in bit m % 32 of word m // 32 (1 = +1, 0 = -1).

This module only draws inputs: it holds none of the demodulation arithmetic.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import synth

PDM_DECIM = 10                      # PDM ticks per 450 kHz sample
PDM_RATE_HZ = synth.FS_HZ * PDM_DECIM


def sigma_delta2(u: np.ndarray) -> np.ndarray:
    """Bits (bool, True = +1) of the second-order modulator for u [..., T], |u| < ~0.7."""
    u = np.asarray(u, dtype=np.float64)
    lanes = u.reshape(-1, u.shape[-1])
    i1 = np.zeros(lanes.shape[0])
    i2 = np.zeros(lanes.shape[0])
    y = np.ones(lanes.shape[0])
    out = np.empty(lanes.shape, dtype=bool)
    for t in range(lanes.shape[1]):
        i1 += lanes[:, t] - y
        i2 += i1 - y
        y = np.where(i2 >= 0.0, 1.0, -1.0)
        out[:, t] = y > 0
    return out.reshape(u.shape)


def pack_words(bits: np.ndarray) -> np.ndarray:
    """[M][T] bool -> [T][ceil(M/32)] uint32, microphone m in bit m % 32 of word m // 32."""
    M, T = bits.shape
    W = (M + 31) // 32
    words = np.zeros((T, W), dtype=np.uint64)
    for m in range(M):
        words[:, m // 32] |= bits[m].astype(np.uint64) << np.uint64(m % 32)
    return words.astype(np.uint32)


@dataclasses.dataclass
class PdmWorkload:
    words: np.ndarray      # [F][T][W] uint32, T = N * decim
    analog: np.ndarray     # [F][M][T] float64: the modulator's input
    base: synth.Workload   # geometry, chirp, directions, reflectors (x unused: None)
    decim: int
    n_out: int


def make_pdm_workload(name: str = "c2", frames: int = 1, n_samples: int | None = None,
                      n_dirs: int | None = None, n_mics: int | None = None, decim: int = PDM_DECIM,
                      chirp_params=(25e3, 80e3, 1e-3)) -> PdmWorkload:
    """PDM recordings of the named config's geometry and reflectors (same seeds as synth)."""
    cfg = synth.CONFIGS[name]
    N = n_samples or cfg.n_samples
    M = n_mics or cfg.n_mics
    cfg = dataclasses.replace(cfg, n_samples=N, n_mics=M)
    mic_pos = synth.planar_array(M, cfg.aperture, synth._rng(cfg.cfg_id, 0, 0, 0))
    dirs = synth.make_grid(cfg.grid) if n_dirs is None else synth.fibonacci_hemisphere(n_dirs)
    chirp = synth.linear_chirp(synth.FS_HZ, *chirp_params)
    fs_pdm = synth.FS_HZ * decim
    T = N * decim
    analog, refl = [], []
    for f in range(frames):
        rf = synth._draw_reflectors(cfg, synth._rng(cfg.cfg_id, 0, f, 1))
        a = synth.simulate_frame(mic_pos, chirp_params, rf, T, cfg.snr_db, synth._rng(cfg.cfg_id, 0, f, 2),
                                 fs=fs_pdm)
        peak = float(np.max(np.abs(a)))
        analog.append(a * (0.5 / peak) if peak > 0 else a)
        refl.append(rf)
    analog = np.stack(analog)
    bits = sigma_delta2(analog)
    words = np.stack([pack_words(bits[f]) for f in range(frames)])
    base = synth.Workload(cfg, None, chirp, mic_pos, dirs, refl)
    return PdmWorkload(words, analog, base, decim, N)


def sine_pdm(M: int, T: int, freq_hz: float, amp: float, fs_pdm: float = PDM_RATE_HZ, phase=None):
    """PDM words of M sines (phases seeded per microphone unless given) and the analog input."""
    if phase is None:
        phase = np.random.default_rng(np.random.SeedSequence([6, 0, 0, 0])).uniform(0, 2 * math.pi, size=M)
    t = np.arange(T) / fs_pdm
    u = amp * np.sin(2 * math.pi * freq_hz * t[None, :] + np.asarray(phase)[:, None])
    return pack_words(sigma_delta2(u)), u
