"""Pins of the oracle's reverse-mode derivatives (CPU): central finite differences of
L = sum(dE * E) with respect to microphone samples and microphone positions, the
adjoint identity of the matched filter, and the exactness of the envelope's VJP on a
linear case."""

import numpy as np

import oracle as O
from workloads import synth

FS, C = 450e3, 343.0


def _tiny(seed=0, M=4, N=300, D=3, band=(20e3, 85e3)):
    rng = np.random.default_rng(seed)
    w = synth.make_workload("c2", n_samples=N, n_dirs=D, n_mics=M)
    x = w.x[0].astype(np.float64) + 0.1 * rng.standard_normal((M, N))
    P = 1024
    dE = rng.standard_normal((D, O.num_range_bins(0, N, 5)))
    return w, x, P, dE, band


def _loss(x, w, P, dE, band, pos=None):
    E = O.energyscape(x, w.chirp, w.mic_pos if pos is None else pos, w.dirs, fs=FS, c=C, P=P, R=5,
                      band=band, mode="td")
    return float(np.sum(dE * E))


def test_vjp_samples_match_finite_differences():
    w, x, P, dE, band = _tiny()
    dx, _ = O.energyscape_vjp_td(x, w.chirp, w.mic_pos, w.dirs, dE, fs=FS, c=C, P=P, R=5, band=band)
    rng = np.random.default_rng(1)
    h = 1e-5
    for _ in range(12):
        m, t = int(rng.integers(x.shape[0])), int(rng.integers(x.shape[1]))
        xp, xm = x.copy(), x.copy()
        xp[m, t] += h
        xm[m, t] -= h
        fd = (_loss(xp, w, P, dE, band) - _loss(xm, w, P, dE, band)) / (2 * h)
        assert abs(fd - dx[m, t]) <= 1e-6 * max(1.0, abs(fd)), (m, t, fd, dx[m, t])


def test_vjp_positions_match_finite_differences():
    w, x, P, dE, band = _tiny(seed=2)
    _, dpos = O.energyscape_vjp_td(x, w.chirp, w.mic_pos, w.dirs, dE, fs=FS, c=C, P=P, R=5, band=band)
    h = 1e-6   # metres: well inside one sample cell (1 sample = 0.76 mm)
    for m in range(w.mic_pos.shape[0]):
        for k in range(3):
            pp, pm = w.mic_pos.copy(), w.mic_pos.copy()
            pp[m, k] += h
            pm[m, k] -= h
            fd = (_loss(x, w, P, dE, band, pp) - _loss(x, w, P, dE, band, pm)) / (2 * h)
            assert abs(fd - dpos[m, k]) <= 1e-5 * max(1.0, np.abs(dpos).max()), (m, k, fd, dpos[m, k])


def test_matched_filter_adjoint_identity():
    """<A x, G>_Re = <x, A^H G> for the matched filter A (x real, G complex)."""
    rng = np.random.default_rng(3)
    M, N, P = 3, 200, 512
    chirp = synth.linear_chirp(FS, 25e3, 80e3, 2e-4)
    x = rng.standard_normal((M, N))
    G = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    lhs = np.sum(np.real(np.conj(G) * O.matched_filter(x, chirp, P, FS, (20e3, 85e3))))
    rhs = np.sum(x * O.matched_filter_vjp(G, chirp, P, N, FS, (20e3, 85e3)))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_envelope_vjp_of_positive_real_beam_is_the_fir_transpose():
    """For b real and positive, |b| = b, so G_b is exactly the FIR's transpose applied to dE."""
    rng = np.random.default_rng(4)
    R, Q = 3, 7
    h = O.default_lowpass(R)
    K = h.size
    b = rng.uniform(0.5, 2.0, size=(2, (Q - 1) * R + K))
    dE = rng.standard_normal((2, Q))
    G = O.envelope_vjp(b, h, dE, Q, R)
    # the envelope is linear here: <E(b), dE> = <b, G>
    assert np.allclose(np.sum(O.envelope(b, h, Q, R) * dE), np.sum(b * G.real), rtol=1e-12)
    assert np.all(G.imag == 0)


def _loss_fd(x, w, P, dE, band, pos=None):
    E = O.energyscape(x, w.chirp, w.mic_pos if pos is None else pos, w.dirs, fs=FS, c=C, P=P, R=5,
                      band=band, mode="fd")
    return float(np.sum(dE * E))


def test_fd_vjp_samples_match_finite_differences():
    w, x, P, dE, band = _tiny(seed=5)
    dx, _ = O.energyscape_vjp_fd(x, w.chirp, w.mic_pos, w.dirs, dE, fs=FS, c=C, P=P, R=5, band=band)
    rng = np.random.default_rng(6)
    h = 1e-5
    for _ in range(12):
        m, t = int(rng.integers(x.shape[0])), int(rng.integers(x.shape[1]))
        xp, xm = x.copy(), x.copy()
        xp[m, t] += h
        xm[m, t] -= h
        fd = (_loss_fd(xp, w, P, dE, band) - _loss_fd(xm, w, P, dE, band)) / (2 * h)
        assert abs(fd - dx[m, t]) <= 1e-6 * max(1.0, abs(fd)), (m, t, fd, dx[m, t])


def test_fd_vjp_positions_match_finite_differences():
    """The exact-phase beamformer is smooth in the delays: central differences with
    h = 1e-6 m agree with the adjoint to the O(h^2) truncation error."""
    w, x, P, dE, band = _tiny(seed=7)
    _, dpos = O.energyscape_vjp_fd(x, w.chirp, w.mic_pos, w.dirs, dE, fs=FS, c=C, P=P, R=5, band=band)
    h = 1e-6
    for m in range(w.mic_pos.shape[0]):
        for k in range(3):
            pp, pm = w.mic_pos.copy(), w.mic_pos.copy()
            pp[m, k] += h
            pm[m, k] -= h
            fd = (_loss_fd(x, w, P, dE, band, pp) - _loss_fd(x, w, P, dE, band, pm)) / (2 * h)
            assert abs(fd - dpos[m, k]) <= 1e-6 * max(1.0, np.abs(dpos).max()), (m, k, fd, dpos[m, k])


def test_fd_beamformer_adjoint_identity():
    """b is linear in the spectra: Re<das_fd(V), G> = Re<V, G_Y> for random V, G (so G_Y is the
    true adjoint, including the one-sided bin range and the 1/P of the window read-out)."""
    rng = np.random.default_rng(8)
    M, P, D = 3, 256, 4
    V = np.zeros((M, P), dtype=np.complex128)
    V[:, :P // 2 + 1] = rng.standard_normal((M, P // 2 + 1)) + 1j * rng.standard_normal((M, P // 2 + 1))
    Dl = rng.uniform(-5, 5, size=(D, M))
    n_idx = np.arange(-20, 100)
    G = rng.standard_normal((D, n_idx.size)) + 1j * rng.standard_normal((D, n_idx.size))
    G_Y, _ = O.das_fd_vjp(V, Dl, n_idx, G)
    lhs = np.sum(np.real(np.conj(G) * O.das_fd(V, Dl, n_idx)))
    rhs = np.sum(np.real(np.conj(G_Y) * V))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_fd_matched_filter_spectrum_adjoint_identity():
    rng = np.random.default_rng(9)
    M, N, P = 3, 200, 512
    chirp = synth.linear_chirp(FS, 25e3, 80e3, 2e-4)
    x = rng.standard_normal((M, N))
    G = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    lhs = np.sum(np.real(np.conj(G) * O.matched_filter_spectrum(x, chirp, P, FS, (20e3, 85e3))))
    rhs = np.sum(x * O.matched_filter_spectrum_vjp(G, chirp, P, N, FS, (20e3, 85e3)))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_td_and_fd_position_gradients_agree_at_integer_delays():
    """With every delay an integer both beamformers read the matched-filter samples exactly,
    so the forward pass that the FD adjoint differentiates equals the TD one there."""
    w, x, P, dE, band = _tiny(seed=10, D=2)
    pos = np.round(w.mic_pos / (C / FS)) * (C / FS)           # positions on the sample lattice
    dirs = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])         # axes: every p . u is a lattice point
    Et = O.energyscape(x, w.chirp, pos, dirs, fs=FS, c=C, P=P, R=5, band=band, mode="td")
    Ef = O.energyscape(x, w.chirp, pos, dirs, fs=FS, c=C, P=P, R=5, band=band, mode="fd")
    assert np.allclose(Et, Ef, rtol=1e-9, atol=1e-12 * np.abs(Ef).max())


# ---------------------------------------------------------------------------
# TD_CUBIC (4-point Lagrange interpolation): the same pins as the linear reading
# ---------------------------------------------------------------------------

def _loss_cubic(x, w, P, dE, band, pos=None):
    E = O.energyscape(x, w.chirp, w.mic_pos if pos is None else pos, w.dirs, fs=FS, c=C, P=P, R=5,
                      band=band, mode="td_cubic")
    return float(np.sum(dE * E))


def test_lagrange4_slopes_are_the_weights_derivatives():
    """Closed forms: each L_k is a cubic with the nodes -1, 0, 1, 2; its slope matches a central
    difference, and the slopes sum to zero (the weights sum to one for every alpha)."""
    a = np.linspace(0.0, 0.999, 37)
    h = 1e-6
    num = (O.lagrange4_weights(a + h) - O.lagrange4_weights(a - h)) / (2 * h)
    S = O.lagrange4_weight_slopes(a)
    assert np.max(np.abs(num - S)) <= 1e-8
    assert np.max(np.abs(S.sum(axis=-1))) <= 1e-12
    # at the nodes: L_0'(0) = -1/2, L_1'(0) = 1, L_-1'(0) = -1/3, L_2'(0) = -1/6
    assert np.allclose(O.lagrange4_weight_slopes(0.0), [-1.0 / 3.0, -0.5, 1.0, -1.0 / 6.0], atol=1e-15)


def test_cubic_beamformer_adjoint_identity():
    """b is linear in yhat: Re <G_b, das_td_cubic(dy)> = Re <G_y, dy> for any dy."""
    rng = np.random.default_rng(7)
    M, P, D = 5, 256, 4
    Dl = rng.uniform(-20.0, 20.0, size=(D, M))
    n_idx = np.arange(40, 140)
    yhat = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    G_b = rng.standard_normal((D, n_idx.size)) + 1j * rng.standard_normal((D, n_idx.size))
    dy = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    G_y, _ = O.das_td_cubic_vjp(yhat, Dl, n_idx, G_b)
    lhs = np.real(np.vdot(G_b, O.das_td_cubic(dy, Dl, n_idx)))
    rhs = np.real(np.vdot(G_y, dy))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_cubic_delay_gradient_matches_finite_differences():
    """dDl of das_td_cubic_vjp against central differences of Re <G_b, b(Dl)> in each Dl[d][m]
    (delays kept inside their sample cells)."""
    rng = np.random.default_rng(8)
    M, P, D = 4, 256, 3
    Dl = np.floor(rng.uniform(-20.0, 20.0, size=(D, M))) + rng.uniform(0.2, 0.8, size=(D, M))
    n_idx = np.arange(30, 120)
    yhat = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    G_b = rng.standard_normal((D, n_idx.size)) + 1j * rng.standard_normal((D, n_idx.size))
    _, dDl = O.das_td_cubic_vjp(yhat, Dl, n_idx, G_b)
    h = 1e-6
    for d in range(D):
        for m in range(M):
            Dp, Dm = Dl.copy(), Dl.copy()
            Dp[d, m] += h
            Dm[d, m] -= h
            fd = (np.real(np.vdot(G_b, O.das_td_cubic(yhat, Dp, n_idx)))
                  - np.real(np.vdot(G_b, O.das_td_cubic(yhat, Dm, n_idx)))) / (2 * h)
            assert abs(fd - dDl[d, m]) <= 1e-6 * max(1.0, abs(fd)), (d, m, fd, dDl[d, m])


def test_cubic_vjp_samples_and_positions_match_finite_differences():
    w, x, P, dE, band = _tiny(seed=3)
    dx, dpos = O.energyscape_vjp_td(x, w.chirp, w.mic_pos, w.dirs, dE, fs=FS, c=C, P=P, R=5, band=band,
                                    interp="cubic")
    rng = np.random.default_rng(4)
    h = 1e-5
    for _ in range(8):
        m, t = int(rng.integers(x.shape[0])), int(rng.integers(x.shape[1]))
        xp, xm = x.copy(), x.copy()
        xp[m, t] += h
        xm[m, t] -= h
        fd = (_loss_cubic(xp, w, P, dE, band) - _loss_cubic(xm, w, P, dE, band)) / (2 * h)
        assert abs(fd - dx[m, t]) <= 1e-6 * max(1.0, abs(fd)), (m, t, fd, dx[m, t])
    h = 1e-6
    for m in range(w.mic_pos.shape[0]):
        for k in range(3):
            pp, pm = w.mic_pos.copy(), w.mic_pos.copy()
            pp[m, k] += h
            pm[m, k] -= h
            fd = (_loss_cubic(x, w, P, dE, band, pp) - _loss_cubic(x, w, P, dE, band, pm)) / (2 * h)
            assert abs(fd - dpos[m, k]) <= 1e-5 * max(1.0, np.abs(dpos).max()), (m, k, fd, dpos[m, k])


def test_cubic_and_linear_gradients_differ_only_by_the_interpolator():
    """With every delay on an integer sample (alpha = 0) both interpolators pass the samples through:
    the sample gradients agree, while the delay slopes differ (cubic: -sum_k L_k'(0) y[n+o+k] =
    y[n+o-1]/3 + y[n+o]/2 - y[n+o+1] + y[n+o+2]/6; linear: y[n+o] - y[n+o+1])."""
    rng = np.random.default_rng(9)
    M, P, D = 3, 128, 2
    Dl = np.floor(rng.uniform(-10.0, 10.0, size=(D, M)))
    n_idx = np.arange(20, 80)
    yhat = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    G_b = rng.standard_normal((D, n_idx.size)) + 1j * rng.standard_normal((D, n_idx.size))
    Gc, dc = O.das_td_cubic_vjp(yhat, Dl, n_idx, G_b)
    Gl, _ = O.das_td_vjp(yhat, Dl, n_idx, G_b)
    assert np.allclose(Gc, Gl, atol=1e-12)
    o = -Dl.astype(np.int64)
    for d in range(D):
        for m in range(M):
            y = lambda k: yhat[m, np.mod(n_idx + o[d, m] + k, P)]
            ref = -np.sum(np.real(np.conj(G_b[d]) * (-y(-1) / 3.0 - y(0) / 2.0 + y(1) - y(2) / 6.0))) / M
            assert abs(dc[d, m] - ref) <= 1e-10 * max(1.0, abs(ref))
