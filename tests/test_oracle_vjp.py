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
