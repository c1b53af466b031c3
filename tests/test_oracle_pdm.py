"""Pins of the oracle's PDM front end (CPU): bit unpacking by Python integers, the
FIR-and-subsample against numpy's convolution, constant streams, the default filter's
response, and recovery of a sigma-delta modulated sine (the modulator's input is known)."""

import math

import numpy as np

import oracle as O
from workloads import pdm


def test_unpack_matches_python_integer_bits():
    rng = np.random.default_rng(11)
    M, T = 45, 37
    words = rng.integers(0, 2**32, size=(T, 2), dtype=np.uint64).astype(np.uint32)
    s = O.pdm_unpack(words, M)
    for t in range(T):
        for m in range(M):
            bit = (int(words[t, m // 32]) >> (m % 32)) & 1
            assert s[m, t] == (1.0 if bit else -1.0)


def test_packing_round_trip():
    rng = np.random.default_rng(12)
    bits = rng.integers(0, 2, size=(70, 50)).astype(bool)
    s = O.pdm_unpack(pdm.pack_words(bits), 70)
    assert np.array_equal(s > 0, bits)


def test_demodulate_matches_library_convolution():
    """x[n] is the full convolution s * h read at tick n decim + (K-1)/2."""
    rng = np.random.default_rng(13)
    M, N, D = 5, 120, 10
    h = O.pdm_default_taps(D)
    K = h.size
    bits = rng.integers(0, 2, size=(M, N * D)).astype(bool)
    x = O.pdm_demodulate(pdm.pack_words(bits), M, N, D, h)
    s = np.where(bits, 1.0, -1.0)
    for m in range(M):
        full = np.convolve(s[m], h)
        assert np.allclose(x[m], full[np.arange(N) * D + (K - 1) // 2], rtol=0, atol=1e-13)


def test_constant_streams():
    M, N, D = 3, 80, 10
    h = O.pdm_default_taps(D)
    hk = (h.size - 1) // 2
    ones = pdm.pack_words(np.ones((M, N * D), dtype=bool))
    zeros = pdm.pack_words(np.zeros((M, N * D), dtype=bool))
    interior = slice(hk // D + 1, N - hk // D - 1)
    assert np.allclose(O.pdm_demodulate(ones, M, N, D, h)[:, interior], 1.0, atol=1e-14)
    assert np.allclose(O.pdm_demodulate(zeros, M, N, D, h)[:, interior], -1.0, atol=1e-14)
    # at n = 0 only the taps reading ticks >= 0 contribute
    assert np.allclose(O.pdm_demodulate(ones, M, N, D, h)[:, 0], np.sum(h[:hk + 1]), atol=1e-14)


def test_default_filter_response():
    D = 10
    h = O.pdm_default_taps(D)
    K = h.size
    assert K == 32 * D + 1
    assert np.allclose(h, h[::-1])
    assert abs(np.sum(h) - 1.0) < 1e-14
    j = np.arange(K) - (K - 1) / 2

    def gain(f_over_fpdm):
        return abs(np.sum(h * np.exp(-2j * np.pi * f_over_fpdm * j)))
    # passband up to the sweep band's top (85 kHz of 4.5 MHz) within 0.05 dB, stopband from
    # a third of the output rate (150 kHz) below -60 dB
    for f in np.linspace(0.0, 85e3 / 4.5e6, 20):
        assert abs(20 * math.log10(gain(f))) < 0.05
    for f in np.linspace(150e3 / 4.5e6, 0.5, 200):
        assert gain(f) < 1e-3


def test_sigma_delta_sine_is_recovered():
    """Demodulating a second-order sigma-delta stream returns the modulator's input: a 50 kHz
    sine of amplitude 0.4 comes back within 1 % RMS at the subsampled instants (the residue is
    the in-band quantisation noise of the modulator), with no delay (zero-phase filter)."""
    M, N, D = 4, 600, 10
    words, u = pdm.sine_pdm(M, N * D, 50e3, 0.4)
    h = O.pdm_default_taps(D)
    x = O.pdm_demodulate(words, M, N, D, h)
    ref = u[:, ::D][:, :N]
    inner = slice(40, N - 40)
    err = np.sqrt(np.mean((x[:, inner] - ref[:, inner]) ** 2)) / np.sqrt(np.mean(ref[:, inner] ** 2))
    assert err < 1e-2, err
    # a one-sample (10-tick) delay would leave an error of |1 - exp(-2 pi i 50/450)| = 0.68
