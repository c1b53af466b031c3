"""Pins of the oracle's variant readings (CPU): integer-delay delay-and-sum."""

import numpy as np
import pytest

import oracle as O


def test_nearest_offsets_follow_the_stated_rounding():
    """The delay rounded to the nearest sample with ties toward the later sample: beamforming reads
    channel m at n + o, o = -round(Dl), so a tie Dl = k + 1/2 reads sample n - k."""
    cases = [(-2.5, 3), (2.5, -2), (0.49, 0), (0.51, -1), (-0.49, 0), (-0.51, 1), (3.0, -3), (-3.0, 3)]
    for dl, o in cases:
        assert int(O.nearest_offsets(np.array([[dl]]))[0, 0]) == o, (dl, o)


def test_nearest_equals_linear_and_exact_at_integer_delays():
    rng = np.random.default_rng(21)
    M, P, D = 4, 128, 5
    Y = np.zeros((M, P), dtype=np.complex128)
    Y[:, :P // 2 + 1] = rng.standard_normal((M, P // 2 + 1)) + 1j * rng.standard_normal((M, P // 2 + 1))
    y = np.fft.ifft(Y, axis=1)
    Dl = rng.integers(-6, 7, size=(D, M)).astype(np.float64)
    n_idx = np.arange(-10, 90)
    bn = O.das_td_nearest(y, Dl, n_idx)
    assert np.allclose(bn, O.das_td(y, Dl, n_idx), rtol=0, atol=1e-14)
    assert np.allclose(bn, O.das_fd(Y, Dl, n_idx), rtol=0, atol=1e-12)


def test_nearest_moves_an_impulse_by_the_rounded_delay():
    """One channel holding a unit impulse at sample s: the beam has 1/M at n = s - o only."""
    M, P = 3, 64
    y = np.zeros((M, P), dtype=np.complex128)
    y[1, 20] = 1.0
    Dl = np.array([[0.0, 2.4, 0.0], [0.0, -3.6, 0.0]])     # channel 1: o = -2 and o = 4
    b = O.das_td_nearest(y, Dl, np.arange(P))
    for d, o in enumerate((-2, 4)):
        expect = np.zeros(P)
        expect[20 - o] = 1.0 / M
        assert np.array_equal(b[d], expect.astype(np.complex128))


def test_butterworth_design_matches_scipy():
    import scipy.signal as ss
    for order in (1, 2, 3, 4, 5, 8):
        for wn in (0.02, 0.1, 0.2, 0.45):
            b, a = O.butterworth_lowpass(order, wn / 2)          # fc / fs = Wn / 2
            bs, as_ = ss.butter(order, wn)
            assert np.allclose(b, bs, rtol=1e-10, atol=1e-15), (order, wn)
            assert np.allclose(a, as_, rtol=1e-10, atol=1e-13), (order, wn)


def test_butterworth_is_minus_3db_at_cutoff():
    b, a = O.butterworth_lowpass(4, 0.05)
    z = np.exp(-2j * np.pi * 0.05)
    H = np.polyval(b[::-1], z) / np.polyval(a[::-1], z)
    assert abs(abs(H) ** 2 - 0.5) < 1e-12
    assert abs(np.sum(b) / np.sum(a) - 1.0) < 1e-12


def test_lfilter_matches_scipy():
    import scipy.signal as ss
    rng = np.random.default_rng(22)
    b, a = O.butterworth_lowpass(4, 0.05)
    x = rng.standard_normal(500)
    assert np.allclose(O.lfilter(b, a, x), ss.lfilter(b, a, x), rtol=1e-10, atol=1e-13)
    b2, a2 = rng.standard_normal(3), np.array([2.0, -0.5, 0.1])
    assert np.allclose(O.lfilter(b2, a2, x), ss.lfilter(b2, a2, x), rtol=1e-10, atol=1e-13)


def test_envelope_iir_identity_filter_samples_the_magnitude():
    rng = np.random.default_rng(23)
    R, Q, K = 4, 9, 9
    bw = rng.standard_normal((3, (Q - 1) * R + K)) + 1j * rng.standard_normal((3, (Q - 1) * R + K))
    E = O.envelope_iir(bw, [1.0], [1.0], Q, R, K)
    assert np.array_equal(E, np.abs(bw)[:, (K - 1) // 2 + R * np.arange(Q)])


def test_lagrange4_weights_at_nodes_and_sum():
    for a, k in ((0.0, 1),):
        w = O.lagrange4_weights(np.array(a))
        assert np.allclose(w, np.eye(4)[k], atol=0)
    a = np.linspace(0, 1, 17, endpoint=False)
    assert np.allclose(O.lagrange4_weights(a).sum(axis=-1), 1.0, atol=1e-15)


def test_cubic_interpolation_is_exact_for_cubic_polynomials():
    """Away from the circular wrap, a cubic sample sequence is reproduced exactly at any fractional
    delay: b[n] = (1/M) sum_m poly(n - Dl[m]) (linear interpolation is not)."""
    rng = np.random.default_rng(24)
    M, P, D = 3, 256, 4
    c = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    n = np.arange(P, dtype=np.float64)
    poly = lambda t: c[0] + c[1] * t + c[2] * t ** 2 + c[3] * t ** 3   # noqa: E731
    y = np.tile(poly(n), (M, 1))
    Dl = rng.uniform(-5, 5, size=(D, M))
    n_idx = np.arange(20, 200)
    b = O.das_td_cubic(y, Dl, n_idx)
    expect = np.stack([np.mean([poly(n_idx - Dl[d, m]) for m in range(M)], axis=0) for d in range(D)])
    assert np.allclose(b, expect, rtol=1e-12, atol=1e-9)
    assert not np.allclose(O.das_td(y, Dl, n_idx), expect, rtol=1e-6)


def test_cubic_is_closer_to_the_exact_delay_than_linear():
    """On a band-limited analytic signal (the beamformer's input) the cubic interpolator's error
    against the exact per-bin phase delay is well below the linear one's."""
    rng = np.random.default_rng(25)
    M, P, D = 4, 512, 6
    Y = np.zeros((M, P), dtype=np.complex128)
    k = np.arange(P // 2 + 1)
    Y[:, :P // 2 + 1] = (rng.standard_normal((M, k.size)) + 1j * rng.standard_normal((M, k.size))) * (k < P // 10)
    y = np.fft.ifft(Y, axis=1)
    Dl = rng.uniform(-8, 8, size=(D, M))
    n_idx = np.arange(P)
    ex = O.das_fd(Y, Dl, n_idx)
    e_lin = np.linalg.norm(O.das_td(y, Dl, n_idx) - ex)
    e_cub = np.linalg.norm(O.das_td_cubic(y, Dl, n_idx) - ex)
    assert e_cub < 0.2 * e_lin, (e_cub, e_lin)


def _analytic_rows(rng, M, P):
    Y = np.zeros((M, P), dtype=np.complex128)
    Y[:, :P // 2 + 1] = rng.standard_normal((M, P // 2 + 1)) + 1j * rng.standard_normal((M, P // 2 + 1))
    return np.fft.ifft(Y, axis=1)


def test_gridded_offsets_round_to_the_grid():
    """alpha on multiples of 1/steps, half-way cases to even, alpha' = 1 moved to the next sample."""
    steps = 2048
    cases = [(-0.3, 0, round(0.3 * steps) / steps), (-(5 + 1.5 / steps), 5, 2 / steps),
             (-(5 + 2.5 / steps), 5, 2 / steps), (-(2 + 1 - 0.4 / steps), 3, 0.0), (-7.0, 7, 0.0),
             (1.25, -2, 0.75)]
    for dl, o_exp, a_exp in cases:
        o, a = O.gridded_offsets(np.array([[dl]]), steps)
        assert int(o[0, 0]) == o_exp and float(a[0, 0]) == a_exp, (dl, o, a)


def test_gridded_with_one_step_is_nearest():
    """A grid of one sample rounds alpha to 0 or 1: the nearest-sample delay (no ties drawn)."""
    rng = np.random.default_rng(31)
    M, P, D = 5, 96, 7
    y = _analytic_rows(rng, M, P)
    Dl = rng.uniform(-9, 9, size=(D, M))
    n_idx = np.arange(-12, 80)
    assert np.array_equal(O.das_td(y, Dl, n_idx, alpha_steps=1), O.das_td_nearest(y, Dl, n_idx))


@pytest.mark.parametrize("steps", [256, 2048])
def test_gridded_equals_linear_for_delays_on_the_grid(steps):
    rng = np.random.default_rng(32)
    M, P, D = 4, 128, 6
    y = _analytic_rows(rng, M, P)
    Dl = -(rng.integers(-6, 7, size=(D, M)) + rng.integers(0, steps, size=(D, M)) / steps)
    n_idx = np.arange(-10, 100)
    assert np.allclose(O.das_td(y, Dl, n_idx, alpha_steps=steps), O.das_td(y, Dl, n_idx), rtol=0, atol=1e-15)


def test_gridded_error_is_bounded_by_half_a_step():
    """b' - b = (1/M) sum_m (alpha' - alpha)(y[i+1] - y[i]) with |alpha' - alpha| <= 1/(2 steps)."""
    rng = np.random.default_rng(33)
    M, P, D, steps = 6, 128, 9, 16
    y = _analytic_rows(rng, M, P)
    Dl = rng.uniform(-8, 8, size=(D, M))
    n_idx = np.arange(-5, 110)
    diff = np.abs(O.das_td(y, Dl, n_idx, alpha_steps=steps) - O.das_td(y, Dl, n_idx))
    o, _ = O.td_offsets(Dl)
    for d in range(D):
        bound = np.zeros(n_idx.size)
        for m in range(M):
            i0 = np.mod(n_idx + o[d, m], P)
            bound += np.abs(y[m, np.mod(i0 + 1, P)] - y[m, i0])
        assert np.all(diff[d] <= bound / M / (2 * steps) + 1e-15)
    assert diff.max() > 0
