"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: brute force on
tiny inputs, library routines that implement the same textbook operation
(numpy/scipy correlate, convolve, hilbert), closed forms, and invariants.  They
are chosen so that a dropped term, a wrong sign or index, or a transposed
operand in the oracle fails at least one of them.
"""

import math

import numpy as np
import pytest
import scipy.signal

import oracle as O
from workloads import synth

FS = 450e3
C = 343.0


def _rng(seed=0):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ matched filter

def test_mf_real_part_is_bruteforce_linear_correlation():
    rng = _rng(1)
    M, N, L, P = 3, 40, 7, 64
    x = rng.standard_normal((M, N))
    s = rng.standard_normal(L)
    y = O.matched_filter(x, s, P, FS)
    for m in range(M):
        for lag in range(-(L - 1), N):
            ref = 0.0
            for l in range(L):
                if 0 <= lag + l < N:
                    ref += s[l] * x[m, lag + l]
            assert abs(y[m, lag % P].real - ref) < 1e-12
    # lags that no sample reaches are exactly zero
    for lag in range(N, P - (L - 1)):
        assert np.all(np.abs(y[:, lag].real) < 1e-12)


def test_mf_real_part_matches_numpy_and_scipy_correlate():
    w = synth.make_workload("c1")
    x = w.x[0].astype(np.float64)
    s = w.chirp
    N, L = x.shape[1], len(s)
    P = 8192
    y = O.matched_filter(x[:4], s, P, FS)
    for m in range(4):
        full = np.correlate(x[m], s, mode="full")            # index lag + L - 1
        lags = np.arange(-(L - 1), N)
        got = y[m, lags % P].real
        assert np.max(np.abs(got - full)) < 1e-9 * np.max(np.abs(full))
        sc = scipy.signal.correlate(x[m], s, mode="full", method="direct")
        assert np.max(np.abs(got - sc)) < 1e-9 * np.max(np.abs(sc))


def test_mf_is_scipy_analytic_signal_of_circular_correlation():
    rng = _rng(2)
    M, N, L, P = 2, 100, 9, 128
    x = rng.standard_normal((M, N))
    s = rng.standard_normal(L)
    y = O.matched_filter(x, s, P, FS)
    for m in range(M):
        r = np.zeros(P)
        for n in range(P):                  # brute-force circular correlation
            r[n] = sum(s[l] * np.concatenate([x[m], np.zeros(P - N)])[(n + l) % P] for l in range(L))
        ana = scipy.signal.hilbert(r)
        assert np.max(np.abs(y[m] - ana)) < 1e-10 * np.max(np.abs(ana))


def test_mf_of_tone_with_unit_chirp_is_complex_exponential():
    P = 256
    n = np.arange(P)
    for k0 in (1, 17, 100, 127):
        x = np.cos(2 * np.pi * k0 * n / P)[None, :]
        y = O.matched_filter(x, np.array([1.0]), P, FS)
        assert np.max(np.abs(y[0] - np.exp(2j * np.pi * k0 * n / P))) < 1e-12


def test_mf_chirp_autocorrelation_peak_at_zero_lag():
    s = synth.linear_chirp()
    assert len(s) == 450
    N, P, n0 = 4096, 8192, 100
    x = np.zeros((1, N))
    x[0, n0:n0 + len(s)] = s
    y = O.matched_filter(x, s, P, FS)
    re = y[0, :N].real
    assert int(np.argmax(re)) == n0
    assert abs(re[n0] - np.sum(s * s)) < 1e-9
    # sum Hann^2 = 3L/8 exactly for the periodic window; sin^2 of the sweep averages 1/2
    assert abs(np.sum(s * s) - 3 * len(s) / 16) < 1e-6 * 84.375


def test_mf_linearity():
    rng = _rng(3)
    x1, x2 = rng.standard_normal((2, 4, 300))
    s = rng.standard_normal(20)
    P = 512
    a, b = 2.5, -0.75
    y = O.matched_filter(a * x1 + b * x2, s, P, FS, band=(10e3, 90e3))
    y12 = a * O.matched_filter(x1, s, P, FS, band=(10e3, 90e3)) + b * O.matched_filter(x2, s, P, FS, band=(10e3, 90e3))
    assert np.max(np.abs(y - y12)) < 1e-10


def test_mf_band_mask_passes_inband_and_removes_outband_tones():
    P = 1024
    n = np.arange(P)
    k_in, k_out = 100, 20                     # 43.9 kHz in band, 8.8 kHz out of band
    x = (np.cos(2 * np.pi * k_in * n / P) + np.cos(2 * np.pi * k_out * n / P))[None, :]
    y = O.matched_filter(x, np.array([1.0]), P, FS, band=(20e3, 85e3))
    assert np.max(np.abs(y[0] - np.exp(2j * np.pi * k_in * n / P))) < 1e-12


def test_band_mask_edges_inclusive():
    P = 1000
    beta = O.band_mask(P, 1000.0, (100.0, 200.0))   # bin k is k Hz
    assert beta[100] == 1 and beta[200] == 1 and beta[99] == 0 and beta[201] == 0
    assert np.all(O.band_mask(P, FS, None) == 1)


def test_analytic_weights():
    W = O.analytic_weights(8)
    assert list(W) == [1, 2, 2, 2, 1, 0, 0, 0]
    with pytest.raises(ValueError):
        O.analytic_weights(7)


# ------------------------------------------------------------------ delays

def test_delays_closed_form_and_sign():
    a = 0.01
    pos = np.array([[a, 0, 0], [0, a, 0], [0, 0, 0]])
    th = np.deg2rad(30.0)
    u = np.array([[np.sin(th), 0, np.cos(th)], [0, 0, 1]])
    Dl = O.delays(pos, u, FS, C)
    assert abs(Dl[0, 0] - FS * a * np.sin(th) / C) < 1e-12
    assert abs(Dl[0, 1]) < 1e-15 and abs(Dl[0, 2]) < 1e-15
    assert np.all(np.abs(Dl[1]) < 1e-15)          # broadside: zero delay for a z=0 array
    assert Dl.shape == (2, 3)


def test_td_offsets_ranges():
    Dl = np.array([[-2.25, 0.0, 3.5, -0.0, 1e-9]])
    o, a = O.td_offsets(Dl)
    assert list(o[0]) == [2, 0, -4, 0, -1]
    np.testing.assert_allclose(a[0], [0.25, 0.0, 0.5, 0.0, 1 - 1e-9], atol=1e-15)
    assert np.all((a >= 0) & (a < 1))


# ------------------------------------------------------------------ DAS

def _rand_yhat(M, P, seed=4):
    rng = _rng(seed)
    return rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))


def test_das_td_zero_delay_is_channel_mean():
    y = _rand_yhat(5, 64)
    n = np.arange(-10, 70)
    b = O.das_td(y, np.zeros((1, 5)), n)
    assert np.max(np.abs(b[0] - y.mean(axis=0)[n % 64])) < 1e-14


def test_das_td_integer_delay_is_circular_shift():
    M, P = 4, 64
    y = _rand_yhat(M, P)
    Dl = np.array([[3.0, -2.0, 0.0, 7.0]])
    n = np.arange(P)
    b = O.das_td(y, Dl, n)
    ref = np.mean([np.roll(y[m], int(Dl[0, m])) for m in range(M)], axis=0)  # y[n - Dl]
    assert np.max(np.abs(b[0] - ref)) < 1e-14


def test_das_td_half_sample_is_neighbour_average():
    P = 32
    y = _rand_yhat(1, P)
    b = O.das_td(y, np.array([[-2.5]]), np.arange(P))   # reads y[n + 2.5]
    ref = 0.5 * (np.roll(y[0], -2) + np.roll(y[0], -3))
    assert np.max(np.abs(b[0] - ref)) < 1e-14


def test_das_fd_integer_delays_equal_td():
    rng = _rng(5)
    M, N, L, P = 4, 100, 11, 128
    x = rng.standard_normal((M, N))
    s = rng.standard_normal(L)
    Y = O.matched_filter_spectrum(x, s, P, FS)
    y = np.fft.ifft(Y, axis=1)
    Dl = np.array([[1.0, -3.0, 0.0, 5.0], [2.0, 2.0, -1.0, 0.0]])
    n = np.arange(-20, 140)
    assert np.max(np.abs(O.das_fd(Y, Dl, n) - O.das_td(y, Dl, n))) < 1e-12


def test_das_fd_single_bin_is_phase_rotation():
    M, P, k0 = 3, 64, 5
    Y = np.zeros((M, P), dtype=complex)
    Y[1, k0] = 2.0 + 1.0j
    Dl = np.array([[0.3, -1.7, 2.2]])
    n = np.arange(P)
    b = O.das_fd(Y, Dl, n)[0]
    ref = (2.0 + 1.0j) / M * np.exp(-2j * np.pi * k0 * Dl[0, 1] / P) * np.exp(2j * np.pi * k0 * n / P) / P
    assert np.max(np.abs(b - ref)) < 1e-15


def test_das_fd_steering_to_true_direction_realigns_fractional_delays():
    # channels that are fractionally advanced copies of one analytic signal add coherently
    rng = _rng(6)
    M, P = 6, 256
    Y0 = np.zeros(P, dtype=complex)
    Y0[10:100] = rng.standard_normal(90) + 1j * rng.standard_normal(90)
    Dl = rng.uniform(-4, 4, size=(1, M))
    k = np.arange(P)
    Y = np.stack([Y0 * np.exp(2j * np.pi * k * Dl[0, m] / P) for m in range(M)])
    b = O.das_fd(Y, Dl, np.arange(P))[0]
    assert np.max(np.abs(b - np.fft.ifft(Y0))) < 1e-14


def test_das_linear_in_input():
    y1, y2 = _rand_yhat(3, 40, 7), _rand_yhat(3, 40, 8)
    Dl = np.array([[0.4, -1.3, 2.9]])
    n = np.arange(-5, 45)
    lhs = O.das_td(2 * y1 - 3j * y2, Dl, n)
    rhs = 2 * O.das_td(y1, Dl, n) - 3j * O.das_td(y2, Dl, n)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


# ------------------------------------------------------------------ envelope

def test_default_lowpass_shape_and_response():
    for R in (1, 4, 10):
        h = O.default_lowpass(R)
        K = 8 * R + 1
        assert h.size == K
        assert abs(h.sum() - 1.0) < 1e-14
        assert np.max(np.abs(h - h[::-1])) < 1e-15
    h = O.default_lowpass(10)
    f = np.linspace(0, 0.5, 2001)                    # cycles/sample
    H = np.abs(np.exp(-2j * np.pi * np.outer(f, np.arange(h.size))) @ h)
    assert abs(H[0] - 1) < 1e-12
    assert np.all(H[f <= 0.02] > 0.97)               # passband up to 9 kHz at 450 kHz
    assert abs(H[np.argmin(np.abs(f - 0.05))] - 0.5) < 0.05   # -6 dB at the cutoff fs/(2R)
    assert np.all(H[f >= 0.08] < 0.01)               # stopband


def test_envelope_of_unit_magnitude_tone_is_one():
    R, Q = 10, 30
    h = O.default_lowpass(R)
    G = (Q - 1) * R + h.size
    b = np.exp(2j * np.pi * 0.123 * np.arange(G))[None, :]
    E = O.envelope(b, h, Q, R)
    assert np.max(np.abs(E - 1.0)) < 1e-14


def test_envelope_matches_numpy_convolve_and_decimation():
    rng = _rng(9)
    R, Q, K = 4, 25, 13
    h = rng.standard_normal(K)
    G = (Q - 1) * R + K
    b = rng.standard_normal((2, G)) + 1j * rng.standard_normal((2, G))
    E = O.envelope(b, h, Q, R)
    for d in range(2):
        full = np.convolve(np.abs(b[d]), h, mode="full")    # full[n] = sum_j h[j] e[n-j]
        assert np.max(np.abs(E[d] - full[K - 1 + R * np.arange(Q)])) < 1e-12


def test_envelope_impulse_response_positions():
    R, Q, K = 3, 10, 7
    h = np.arange(1, K + 1, dtype=float)
    G = (Q - 1) * R + K
    for p in (0, 5, G - 1):
        b = np.zeros((1, G), dtype=complex)
        b[0, p] = -1.0
        E = O.envelope(b, h, Q, R)[0]
        for q in range(Q):
            j = q * R + K - 1 - p
            assert E[q] == (h[j] if 0 <= j < K else 0.0)


def test_window_indices_and_range_bins():
    assert O.num_range_bins(0, 16384, 10) == 1639
    assert O.num_range_bins(0, 4096, 10) == 410
    idx = O.beam_window_indices(0, 1639, 10, 81)
    assert idx.size == 16461 and idx[0] == -40 and idx[-1] == 16420


# ------------------------------------------------------------------ whole pipeline

def _small_case(seed=10, M=4, N=300, D=5):
    rng = _rng(seed)
    x = rng.standard_normal((M, N))
    s = synth.linear_chirp()[:40]
    pos = np.zeros((M, 3))
    pos[:, :2] = rng.uniform(-0.0175, 0.0175, size=(M, 2))
    dirs = synth.fibonacci_hemisphere(D)
    return x, s, pos, dirs


@pytest.mark.parametrize("mode", ["td", "fd"])
def test_pipeline_positive_homogeneity(mode):
    x, s, pos, dirs = _small_case()
    kw = dict(fs=FS, c=C, R=4, mode=mode, band=(20e3, 85e3))
    E1 = O.energyscape(x, s, pos, dirs, **kw)
    E2 = O.energyscape(-3.0 * x, s, pos, dirs, **kw)
    assert np.max(np.abs(E2 - 3.0 * E1)) < 1e-12 * np.max(np.abs(E1))


@pytest.mark.parametrize("mode", ["td", "fd"])
def test_pipeline_shift_by_R_shifts_one_range_bin(mode):
    x, s, pos, dirs = _small_case(N=400)
    R = 5
    x[:, -R:] = 0.0
    xs = np.concatenate([np.zeros((x.shape[0], R)), x[:, :-R]], axis=1)
    kw = dict(fs=FS, c=C, R=R, mode=mode, P=512)
    E = O.energyscape(x, s, pos, dirs, **kw)
    Es = O.energyscape(xs, s, pos, dirs, **kw)
    assert np.max(np.abs(Es[:, 1:] - E[:, :-1])) < 1e-11 * np.max(np.abs(E))


def test_pipeline_superposition_holds_at_beam_level():
    x, s, pos, dirs = _small_case()
    rng = _rng(11)
    x2 = rng.standard_normal(x.shape)
    kw = dict(fs=FS, c=C, R=4, mode="td", return_beam=True)
    _, b1 = O.energyscape(x, s, pos, dirs, **kw)
    _, b2 = O.energyscape(x2, s, pos, dirs, **kw)
    _, b12 = O.energyscape(x + x2, s, pos, dirs, **kw)
    assert np.max(np.abs(b12 - b1 - b2)) < 1e-11


def test_pipeline_dir_subset_rows_follow_index():
    x, s, pos, dirs = _small_case(D=7)
    E = O.energyscape(x, s, pos, dirs, fs=FS, c=C, R=4)
    Es = O.energyscape(x, s, pos, dirs, fs=FS, c=C, R=4, dir_index=[6, 2])
    assert np.array_equal(Es, E[[6, 2]])


def test_td_and_fd_agree_when_all_delays_are_integers():
    x, s, _, _ = _small_case(M=3)
    # one mic at the origin and directions/positions chosen so fs*(p.u)/c is an integer
    step = C / FS
    pos = np.array([[0, 0, 0], [2 * step, 0, 0], [0, -3 * step, 0]])
    dirs = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    Etd = O.energyscape(x, s, pos, dirs, fs=FS, c=C, R=4, mode="td")
    Efd = O.energyscape(x, s, pos, dirs, fs=FS, c=C, R=4, mode="fd")
    assert np.max(np.abs(Etd - Efd)) < 1e-11 * np.max(np.abs(Etd))


def test_point_reflectors_recovered_in_range_and_direction():
    """Physics: every reflector fully inside the window peaks at its azimuth and range."""
    w = synth.make_workload("c1")
    x = w.x[0].astype(np.float64)
    E = O.energyscape(x, w.chirp, w.mic_pos, w.dirs, fs=w.fs, c=w.c, R=10, mode="td")
    az_grid = np.degrees(np.arctan2(w.dirs[:, 0], w.dirs[:, 2]))
    n_checked = 0
    L = len(w.chirp)
    for (r, u, a) in w.reflectors[0]:
        n_echo = 2 * r * w.fs / w.c
        if n_echo + L > x.shape[1]:
            continue                               # echo leaves the recording window
        az = math.degrees(math.atan2(u[0], u[2]))
        q_true = n_echo / 10
        d_true = int(np.argmin(np.abs(az_grid - az)))
        # local neighbourhood of the true cell holds the global peak of that neighbourhood
        qlo, qhi = int(q_true) - 8, int(q_true) + 9
        sub = E[:, qlo:qhi]
        d_pk, q_pk = np.unravel_index(np.argmax(sub), sub.shape)
        assert abs(d_pk - d_true) <= 1, (az, az_grid[d_pk])
        # the chirp correlation peak sits within a few range bins of the round trip time
        assert abs((qlo + q_pk) - q_true) <= 2.5, (qlo + q_pk, q_true)
        n_checked += 1
    assert n_checked >= 1


def test_wrong_delay_sign_would_mirror_the_peak():
    """The sign of the steering delay is pinned by an off-axis reflector."""
    pos = synth.planar_array(32, 0.035, np.random.default_rng(123))
    s = synth.linear_chirp()
    refl = [(1.0, np.array([math.sin(math.radians(30)), 0, math.cos(math.radians(30))]), 1.0)]
    x = synth.simulate_frame(pos, (25e3, 80e3, 1e-3), refl, 4096, None, None)
    dirs = synth.azimuth_grid(91)
    E = O.energyscape(x, s, pos, dirs, fs=FS, c=C, R=10)
    d_pk, q_pk = np.unravel_index(np.argmax(E), E.shape)
    az = np.degrees(np.arctan2(dirs[d_pk, 0], dirs[d_pk, 2]))
    assert abs(az - 30.0) <= 2.0
    assert abs(q_pk * 10 * C / (2 * FS) - 1.0) < 0.02
