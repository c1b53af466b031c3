"""Plain FP64 oracle of the energyscape pipeline (TEST INFRASTRUCTURE ONLY).

The paper (Jansen et al., "In-Air Imaging Sonar Sensor Network With Real-time
Processing Using GPUs") turns one multi-microphone recording of a broadband FM
sweep into a range x direction intensity image in three steps (Fig. 3 caption;
§4.1 Signal Processing): a matched filter against the emitted sweep, delay-and-sum
beamforming toward every direction of interest, and an envelope detector whose
output is subsampled (§4.3 GPU Algorithm Implementation).  The paper states
these steps in prose only; the precise definition implemented here fixes what
the paper leaves open (circular length-P arithmetic, analytic signal from
one-sided weights, zero-phase FIR low-pass, linear-interpolation or exact
fractional delays), and each function states the reading it takes.

Everything is numpy in float64 (complex128), with ``numpy.fft`` as the only
library primitive.  Nothing is blocked, fused or reordered beyond what the
definition states, so each function can be read against the definition.  Only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg
may use this module; the HIP library never does.

DFT convention: X[k] = sum_n x[n] exp(-2j*pi*k*n/P);
IDFT(X)[n] = (1/P) sum_k X[k] exp(+2j*pi*k*n/P).
"""

from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Matched filter (§4.1: each channel is matched-filtered against the emitted
# sweep; §4.3: on the GPU this filter is an FFT convolution whose group delay is
# removed afterwards).
# ---------------------------------------------------------------------------

def analytic_weights(P: int) -> np.ndarray:
    """One-sided weights that turn a real signal's DFT into its analytic signal.

    W[0] = 1, W[k] = 2 for 0 < k < P/2, W[P/2] = 1, W[k] = 0 above P/2 (the
    discrete analytic signal; the envelope of §4.1 is the magnitude of it).
    """
    if P % 2:
        raise ValueError("P must be even")
    W = np.zeros(P)
    W[0] = 1.0
    W[1:P // 2] = 2.0
    W[P // 2] = 1.0
    return W


def band_mask(P: int, fs: float, band=None) -> np.ndarray:
    """beta[k] = 1 where lo <= k*fs/P <= hi, else 0; all ones when band is None."""
    if band is None or (band[0] == 0 and band[1] == 0):
        return np.ones(P)
    lo, hi = band
    f = np.arange(P) * (fs / P)
    return ((f >= lo) & (f <= hi)).astype(np.float64)


def chirp_spectrum_filter(chirp, P: int, fs: float, band=None) -> np.ndarray:
    """C[k] = beta[k] * W[k] * conj(S[k]) with S = DFT_P(chirp zero-padded)."""
    s = np.asarray(chirp, dtype=np.float64)
    S = np.fft.fft(s, n=P)
    return band_mask(P, fs, band) * analytic_weights(P) * np.conj(S)


def matched_filter_spectrum(x, chirp, P: int, fs: float, band=None) -> np.ndarray:
    """Yhat_m[k] = X_m[k] * C[k], k in [0, P): the spectrum of the analytic MF output.

    x is [M][N] (zero-padded to P).  Correlation (not convolution) with the
    emitted chirp, so lag 0 of the output is the echo onset: the filter's group
    delay is removed by construction.
    """
    x = np.asarray(x, dtype=np.float64)
    if x.ndim != 2:
        raise ValueError("x must be [M][N]")
    if P < x.shape[1] + len(chirp) - 1:
        raise ValueError("P must be >= N + L - 1")
    X = np.fft.fft(x, n=P, axis=1)
    return X * chirp_spectrum_filter(chirp, P, fs, band)[None, :]


def matched_filter(x, chirp, P: int, fs: float, band=None) -> np.ndarray:
    """yhat_m[n] = IDFT_P(Yhat_m)[n] for n in Z_P, complex128 [M][P].

    Without a band mask, Re yhat_m[n] = sum_l chirp[l] * x_m[n + l] (the linear
    correlation; negative lags sit at P + n) and Im yhat is its discrete Hilbert
    transform.
    """
    return np.fft.ifft(matched_filter_spectrum(x, chirp, P, fs, band), axis=1)


# ---------------------------------------------------------------------------
# Delays (§4.1: for each direction of interest the delay relative to each
# channel of the array is computed; it depends on direction and channel only,
# i.e. far-field plane-wave steering).
# ---------------------------------------------------------------------------

def delays(mic_pos, dirs, fs: float, c: float) -> np.ndarray:
    """Dl[d][m] = fs * (p_m . u_d) / c in samples (float64).

    A plane wave arriving from unit direction u reaches microphone m earlier by
    p_m . u / c than it reaches the origin, so beamforming toward u reads
    channel m Dl[d][m] samples later.
    """
    pos = np.asarray(mic_pos, dtype=np.float64)
    u = np.asarray(dirs, dtype=np.float64)
    D, M = u.shape[0], pos.shape[0]
    Dl = np.empty((D, M))
    for d in range(D):
        for m in range(M):
            Dl[d, m] = fs * (pos[m, 0] * u[d, 0] + pos[m, 1] * u[d, 1] + pos[m, 2] * u[d, 2]) / c
    return Dl


def td_offsets(Dl):
    """Integer offset o = floor(-Dl) and interpolation weight alpha = -Dl - o in [0, 1)."""
    Dl = np.asarray(Dl, dtype=np.float64)
    o = np.floor(-Dl)
    return o.astype(np.int64), (-Dl - o)


def gridded_offsets(Dl, steps: int):
    """td_offsets with alpha rounded to a multiple of 1/steps (half-way cases to even):
    alpha' = rint(steps alpha) / steps; alpha' = 1 is taken as offset o + 1 with alpha' = 0.
    (A precision device of the library's FP16 mode, not a reading of the paper: the fractional
    delay on a grid of 1/steps sample makes the interpolation weights exact in a short
    floating-point format.)"""
    o, alpha = td_offsets(Dl)
    a = np.rint(alpha * steps) / steps
    up = a >= 1.0
    return o + up.astype(np.int64), np.where(up, 0.0, a)


# ---------------------------------------------------------------------------
# Delay-and-sum beamforming (§4.1: simple delay-and-sum steering; §4.3: a device
# kernel on the GPU).
# ---------------------------------------------------------------------------

def das_td(yhat, Dl, n_idx, alpha_steps: int | None = None) -> np.ndarray:
    """Fractional-delay DAS with linear interpolation, circular in P.

    b_d[n] = (1/M) sum_m [(1 - alpha) yhat_m[(n + o) mod P] + alpha yhat_m[(n + o + 1) mod P]]
    evaluated at the sample indices n_idx (which may be negative).  With alpha_steps, o and
    alpha come from gridded_offsets.
    Returns complex128 [D][len(n_idx)].
    """
    yhat = np.asarray(yhat)
    M, P = yhat.shape
    o, alpha = td_offsets(Dl) if alpha_steps is None else gridded_offsets(Dl, alpha_steps)
    n_idx = np.asarray(n_idx, dtype=np.int64)
    D = o.shape[0]
    b = np.zeros((D, n_idx.size), dtype=np.complex128)
    for d in range(D):
        acc = np.zeros(n_idx.size, dtype=np.complex128)
        for m in range(M):
            i0 = np.mod(n_idx + o[d, m], P)
            i1 = np.mod(n_idx + o[d, m] + 1, P)
            acc += (1.0 - alpha[d, m]) * yhat[m, i0] + alpha[d, m] * yhat[m, i1]
        b[d] = acc / M
    return b


def nearest_offsets(Dl):
    """Integer delay: the delay rounded to the nearest sample, ties toward the later sample
    (o = floor(-Dl + 1/2))."""
    return np.floor(-np.asarray(Dl, dtype=np.float64) + 0.5).astype(np.int64)


def das_td_nearest(yhat, Dl, n_idx) -> np.ndarray:
    """Integer-delay DAS (the plainest reading of "simple delay-and-sum"), circular in P:
    b_d[n] = (1/M) sum_m yhat_m[(n + o) mod P], o = nearest_offsets(Dl).  Complex128 [D][len(n_idx)]."""
    yhat = np.asarray(yhat)
    M, P = yhat.shape
    o = nearest_offsets(Dl)
    n_idx = np.asarray(n_idx, dtype=np.int64)
    b = np.zeros((o.shape[0], n_idx.size), dtype=np.complex128)
    for d in range(o.shape[0]):
        for m in range(M):
            b[d] += yhat[m, np.mod(n_idx + o[d, m], P)]
        b[d] /= M
    return b


def lagrange4_weights(alpha):
    """Weights of the 4-point Lagrange interpolator through samples -1, 0, 1, 2 evaluated at
    alpha in [0, 1): L_k(alpha) = prod_{j != k} (alpha - j) / (k - j).  Returns [..., 4]."""
    a = np.asarray(alpha, dtype=np.float64)
    nodes = (-1, 0, 1, 2)
    out = []
    for k in nodes:
        w = np.ones_like(a)
        for j in nodes:
            if j != k:
                w = w * (a - j) / (k - j)
        out.append(w)
    return np.stack(out, axis=-1)


def lagrange4_weight_slopes(alpha):
    """d L_k / d alpha of lagrange4_weights (nodes -1, 0, 1, 2): by the product rule,
    L_k'(alpha) = sum_{i != k} prod_{j != k, i} (alpha - j) / prod_{j != k} (k - j).  Returns [..., 4]."""
    a = np.asarray(alpha, dtype=np.float64)
    nodes = (-1, 0, 1, 2)
    out = []
    for k in nodes:
        den = 1.0
        for j in nodes:
            if j != k:
                den *= (k - j)
        s = np.zeros_like(a)
        for i in nodes:
            if i == k:
                continue
            t = np.ones_like(a)
            for j in nodes:
                if j != k and j != i:
                    t = t * (a - j)
            s = s + t
        out.append(s / den)
    return np.stack(out, axis=-1)


def das_td_cubic(yhat, Dl, n_idx) -> np.ndarray:
    """Fractional-delay DAS with 4-point (cubic) Lagrange interpolation, circular in P:
    o = floor(-Dl), alpha = -Dl - o,
    b_d[n] = (1/M) sum_m sum_{k=-1..2} L_k(alpha) yhat_m[(n + o + k) mod P]."""
    yhat = np.asarray(yhat)
    M, P = yhat.shape
    o, alpha = td_offsets(Dl)
    L = lagrange4_weights(alpha)
    n_idx = np.asarray(n_idx, dtype=np.int64)
    b = np.zeros((o.shape[0], n_idx.size), dtype=np.complex128)
    for d in range(o.shape[0]):
        for m in range(M):
            for i, k in enumerate((-1, 0, 1, 2)):
                b[d] += L[d, m, i] * yhat[m, np.mod(n_idx + o[d, m] + k, P)]
        b[d] /= M
    return b


def das_fd(Yspec, Dl, n_idx) -> np.ndarray:
    """Exact fractional-delay DAS by per-bin phase steering, circular in P.

    B_d[k] = (1/M) sum_m Yhat_m[k] exp(-2j pi k Dl[d][m] / P), b_d = IDFT_P(B_d),
    evaluated at n_idx.  Yhat vanishes above P/2 (analytic weights), so the
    sum over k runs over 0..P/2 only; the other bins of B_d are zero.
    """
    Y = np.asarray(Yspec)
    M, P = Y.shape
    Dl = np.asarray(Dl, dtype=np.float64)
    n_idx = np.mod(np.asarray(n_idx, dtype=np.int64), P)
    k = np.arange(P // 2 + 1, dtype=np.float64)
    D = Dl.shape[0]
    b = np.zeros((D, n_idx.size), dtype=np.complex128)
    for d in range(D):
        B = np.zeros(P, dtype=np.complex128)
        for m in range(M):
            B[:P // 2 + 1] += Y[m, :P // 2 + 1] * np.exp(-2j * np.pi * (k * Dl[d, m] / P))
        B /= M
        b[d] = np.fft.ifft(B)[n_idx]
    return b


# ---------------------------------------------------------------------------
# Envelope and subsampling (§4.1: the envelope of each beam is the reflector
# distribution along range; §4.3: filters run as FFT convolution with their
# group delay removed, and the envelope is subsampled afterwards).
# ---------------------------------------------------------------------------

def default_lowpass(R: int) -> np.ndarray:
    """Default zero-phase low-pass: K = 8R+1 Hamming-windowed sinc, cutoff fs/(2R), sum 1."""
    if R < 1:
        raise ValueError("R must be >= 1")
    K = 8 * R + 1
    j = np.arange(K, dtype=np.float64)
    w = 0.54 - 0.46 * np.cos(2.0 * np.pi * j / (K - 1))
    h = w * np.sinc((j - (K - 1) / 2) / R)
    return h / h.sum()


def num_range_bins(n0: int, n1: int, R: int) -> int:
    """Q = ceil((n1 - n0) / R)."""
    return -(-(n1 - n0) // R)


def beam_window_indices(n0: int, Q: int, R: int, K: int) -> np.ndarray:
    """Beam sample indices needed for Q outputs: n0 - (K-1)/2 ... n0 + (Q-1)R + (K-1)/2."""
    hk = (K - 1) // 2
    return np.arange(n0 - hk, n0 + (Q - 1) * R + hk + 1, dtype=np.int64)


def envelope(b_win, taps, Q: int, R: int) -> np.ndarray:
    """E[d][q] = sum_j h[j] |b_d[n0 + qR + (K-1)/2 - j]| from the beam window.

    b_win[d][i] holds b_d at sample n0 - (K-1)/2 + i, so the FIR tap j of output
    q reads window position qR + K - 1 - j.
    """
    h = np.asarray(taps, dtype=np.float64)
    K = h.size
    e = np.abs(np.asarray(b_win))
    D = e.shape[0]
    if e.shape[1] != (Q - 1) * R + K:
        raise ValueError("beam window has the wrong length")
    E = np.zeros((D, Q))
    for q in range(Q):
        seg = e[:, q * R:q * R + K]          # window positions qR .. qR+K-1
        E[:, q] = seg @ h[::-1]               # position qR+K-1-j pairs with h[j]
    return E


# IIR reading of the envelope filter (§4.3: the CPU implementation designs the
# filters as Butterworth filters and runs them with SciPy's lfilter, i.e. causal,
# group delay kept).  The IIR runs over the beam window from zero state at its
# first sample; output q is the filter's value at window position qR + (K-1)/2,
# the sample n0 + qR of the FIR reading.

def butterworth_lowpass(order: int, fc_over_fs: float):
    """(b, a) of the digital Butterworth low-pass of the given order with -3 dB at fc:
    analog prototype poles exp(i pi (2k + order + 1) / (2 order)), k < order, scaled to the
    prewarped cutoff W = 2 fs tan(pi fc / fs), mapped by the bilinear transform
    z = (2 fs + s) / (2 fs - s) (all zeros at z = -1); substituting s into W^order / prod(s - p)
    gives the gain W^order / prod(2 fs - p) of (z + 1)^order / prod(z - z_p) (unit gain at DC); a[0] = 1."""
    k = np.arange(order)
    poles_a = np.exp(1j * np.pi * (2 * k + order + 1) / (2 * order))
    fs = 1.0
    W = 2.0 * fs * np.tan(np.pi * fc_over_fs / fs)
    p = W * poles_a
    z_d = (2 * fs + p) / (2 * fs - p)
    a = np.real(np.poly(z_d))
    gain = np.real(W ** order / np.prod(2 * fs - p))
    b = gain * np.real(np.poly(-np.ones(order)))
    return b, a


def lfilter(b, a, x) -> np.ndarray:
    """Causal IIR from zero state: a[0] y[n] = sum_k b[k] x[n-k] - sum_{k>=1} a[k] y[n-k]."""
    b = np.asarray(b, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros(x.shape[-1])
    for n in range(x.shape[-1]):
        acc = 0.0
        for k in range(b.size):
            if n - k >= 0:
                acc += b[k] * x[n - k]
        for k in range(1, a.size):
            if n - k >= 0:
                acc -= a[k] * y[n - k]
        y[n] = acc / a[0]
    return y


def envelope_iir(b_win, bcoef, acoef, Q: int, R: int, K: int) -> np.ndarray:
    """E[d][q] = lfilter(bcoef, acoef, |b_d| over the window)[qR + (K-1)/2]."""
    e = np.abs(np.asarray(b_win))
    hk = (K - 1) // 2
    E = np.zeros((e.shape[0], Q))
    for d in range(e.shape[0]):
        y = lfilter(bcoef, acoef, e[d])
        E[d] = y[hk + R * np.arange(Q)]
    return E


# ---------------------------------------------------------------------------
# Whole pipeline (Fig. 3 order: matched filter, beamformer, envelope).
# ---------------------------------------------------------------------------

def energyscape(x, chirp, mic_pos, dirs, *, fs: float, c: float, P: int | None = None,
                gate=None, R: int = 10, taps=None, band=None, mode: str = "td",
                dir_index=None, return_beam: bool = False, iir=None, alpha_steps: int | None = None,
                timings: dict | None = None):
    """E[d][q] for one recording x[M][N]; mode 'td' (linear interpolation), 'td_nearest' (integer
    delays), 'td_cubic' (4-point Lagrange interpolation) or 'fd' (exact).  alpha_steps (mode
    'td') puts the fractional delays on a grid of 1/alpha_steps sample (gridded_offsets).

    dir_index selects a subset of directions (rows of the result follow it).
    With return_beam, also returns the complex beam window b[d][G'].
    iir = (b, a) selects the IIR envelope reading (envelope_iir) instead of the FIR.
    timings, if given, receives the wall-clock seconds of the three stages ('matched_filter',
    'beamform' (delays included), 'envelope'); it does not change what is computed.
    """
    import time
    clock = time.perf_counter
    x = np.asarray(x, dtype=np.float64)
    M, N = x.shape
    L = len(chirp)
    if P is None:
        P = 1
        while P < N + L - 1:
            P *= 2
    n0, n1 = (0, N) if gate is None else gate
    h = default_lowpass(R) if taps is None else np.asarray(taps, dtype=np.float64)
    K = h.size
    if K % 2 == 0:
        raise ValueError("FIR length must be odd")
    Q = num_range_bins(n0, n1, R)
    u = np.asarray(dirs, dtype=np.float64)
    if dir_index is not None:
        u = u[np.asarray(dir_index)]
    if mode not in ("td", "td_nearest", "td_cubic", "fd"):
        raise ValueError("mode must be 'td', 'td_nearest', 'td_cubic' or 'fd'")
    t0 = clock()
    y = matched_filter_spectrum(x, chirp, P, fs, band) if mode == "fd" else matched_filter(x, chirp, P, fs, band)
    t1 = clock()
    Dl = delays(mic_pos, u, fs, c)
    n_idx = beam_window_indices(n0, Q, R, K)
    if mode == "td":
        b = das_td(y, Dl, n_idx, alpha_steps)
    elif mode == "td_nearest":
        b = das_td_nearest(y, Dl, n_idx)
    elif mode == "td_cubic":
        b = das_td_cubic(y, Dl, n_idx)
    else:
        b = das_fd(y, Dl, n_idx)
    t2 = clock()
    E = envelope(b, h, Q, R) if iir is None else envelope_iir(b, iir[0], iir[1], Q, R, K)
    if timings is not None:
        timings.update(matched_filter=t1 - t0, beamform=t2 - t1, envelope=clock() - t2)
    return (E, b) if return_beam else E


# ---------------------------------------------------------------------------
# PDM front end (§2: the microphones deliver 1-bit sigma-delta pulse-density
# modulation; §4.3: on the GPU the binary data are unpacked, demodulated with a
# low-pass filter and subsampled before the matched filter).  The paper gives
# neither the PDM clock, the bit packing nor the filter; the readings taken:
# ceil(M/32) 32-bit words per PDM tick, microphone m in bit m % 32 of word
# m // 32 (set = +1, clear = -1); a zero-phase FIR low-pass at the PDM rate
# evaluated at every decim-th tick.
# ---------------------------------------------------------------------------

def pdm_default_taps(decim: int, K: int | None = None) -> np.ndarray:
    """Hamming-windowed sinc, K = 32 decim + 1 taps, cutoff a quarter of the output rate
    (1/(4 decim) of the PDM rate), normalised to unit DC gain."""
    K = 32 * decim + 1 if K is None else int(K)
    j = np.arange(K, dtype=np.float64)
    hk = (K - 1) / 2.0
    w = 0.54 - 0.46 * np.cos(2.0 * np.pi * j / (K - 1))
    h = w * np.sinc((j - hk) / (2.0 * decim))
    return h / np.sum(h)


def pdm_unpack(words, M: int) -> np.ndarray:
    """s[m][t] in {-1, +1} from words [T][ceil(M/32)] uint32."""
    words = np.asarray(words, dtype=np.uint32)
    s = np.empty((M, words.shape[0]))
    for m in range(M):
        bit = (words[:, m // 32] >> np.uint32(m % 32)) & np.uint32(1)
        s[m] = np.where(bit == 1, 1.0, -1.0)
    return s


def pdm_demodulate(words, M: int, N: int, decim: int, taps) -> np.ndarray:
    """x[m][n] = sum_{j<K} h[j] s_m[n decim + (K-1)/2 - j] with s = 0 outside the T recorded
    ticks: the zero-phase low-pass (group delay removed) evaluated only where the
    subsampler keeps it.  Returns float64 [M][N]."""
    s = pdm_unpack(words, M)
    T = s.shape[1]
    h = np.asarray(taps, dtype=np.float64)
    K = h.size
    if K % 2 == 0:
        raise ValueError("PDM filter length must be odd")
    hk = (K - 1) // 2
    x = np.zeros((M, N))
    n = np.arange(N)
    for j in range(K):
        t = n * decim + hk - j
        ok = (t >= 0) & (t < T)
        x[:, ok] += h[j] * s[:, t[ok]]
    return x


# ---------------------------------------------------------------------------
# Reverse-mode derivatives of the time-domain pipeline (the adjoint used for
# array self-calibration).  For a real loss L of the energyscape, dE = dL/dE.
# Complex quantities z carry the gradient G_z = dL/dRe z + i dL/dIm z, so that
# dL = sum Re(conj(G_z) dz).  Each step is the chain rule of the forward step
# above, written out term by term.
# ---------------------------------------------------------------------------

def envelope_vjp(b_win, taps, dE, Q: int, R: int) -> np.ndarray:
    """G_b[d][i] for E = envelope(b_win): dL/d|b| at window position i is
    sum over the outputs q that read it (i = qR + K-1-j) of dE[d][q] h[j]; then
    G_b = dL/d|b| * b/|b| (zero where b = 0)."""
    h = np.asarray(taps, dtype=np.float64)
    K = h.size
    b = np.asarray(b_win)
    dE = np.asarray(dE, dtype=np.float64)
    g_abs = np.zeros(b.shape)
    for q in range(Q):
        for j in range(K):
            g_abs[:, q * R + K - 1 - j] += dE[:, q] * h[j]
    mag = np.abs(b)
    unit = np.where(mag > 0, b / np.where(mag > 0, mag, 1.0), 0.0)
    return g_abs * unit


def das_td_vjp(yhat, Dl, n_idx, G_b):
    """Gradients of b = das_td(yhat, Dl, n_idx) given G_b [D][len(n_idx)].

    Returns (G_y [M][P] complex, dDl [D][M] real):
      G_y[m][(n+o) mod P]   += (1-alpha)/M * G_b[d][n],  G_y[m][(n+o+1) mod P] += alpha/M * G_b[d][n]
      dDl[d][m] = (1/M) sum_n Re(conj(G_b[d][n]) (yhat_m[n+o] - yhat_m[n+o+1]))
    (alpha = -Dl - o depends on Dl with slope -1 inside a sample cell; o is
    piecewise constant, so this is the derivative almost everywhere.)"""
    yhat = np.asarray(yhat)
    M, P = yhat.shape
    o, alpha = td_offsets(Dl)
    n_idx = np.asarray(n_idx, dtype=np.int64)
    G_b = np.asarray(G_b)
    D = o.shape[0]
    G_y = np.zeros((M, P), dtype=np.complex128)
    dDl = np.zeros((D, M))
    for d in range(D):
        for m in range(M):
            i0 = np.mod(n_idx + o[d, m], P)
            i1 = np.mod(n_idx + o[d, m] + 1, P)
            np.add.at(G_y[m], i0, (1.0 - alpha[d, m]) / M * G_b[d])
            np.add.at(G_y[m], i1, alpha[d, m] / M * G_b[d])
            dDl[d, m] = np.sum(np.real(np.conj(G_b[d]) * (yhat[m, i0] - yhat[m, i1]))) / M
    return G_y, dDl


def das_td_cubic_vjp(yhat, Dl, n_idx, G_b):
    """Gradients of b = das_td_cubic(yhat, Dl, n_idx) given G_b [D][len(n_idx)].

    Returns (G_y [M][P] complex, dDl [D][M] real):
      G_y[m][(n+o+k) mod P] += L_k(alpha)/M * G_b[d][n]                   (k = -1 .. 2)
      dDl[d][m] = -(1/M) sum_n Re(conj(G_b[d][n]) sum_k L_k'(alpha) yhat_m[n+o+k])
    (alpha = -Dl - o has slope -1 in Dl inside a sample cell; o is piecewise constant, so this
    is the derivative almost everywhere.)"""
    yhat = np.asarray(yhat)
    M, P = yhat.shape
    o, alpha = td_offsets(Dl)
    Lw = lagrange4_weights(alpha)
    Ls = lagrange4_weight_slopes(alpha)
    n_idx = np.asarray(n_idx, dtype=np.int64)
    G_b = np.asarray(G_b)
    D = o.shape[0]
    G_y = np.zeros((M, P), dtype=np.complex128)
    dDl = np.zeros((D, M))
    for d in range(D):
        for m in range(M):
            acc = np.zeros(n_idx.size, dtype=np.complex128)
            for i, k in enumerate((-1, 0, 1, 2)):
                idx = np.mod(n_idx + o[d, m] + k, P)
                np.add.at(G_y[m], idx, Lw[d, m, i] / M * G_b[d])
                acc += Ls[d, m, i] * yhat[m, idx]
            dDl[d, m] = -np.sum(np.real(np.conj(G_b[d]) * acc)) / M
    return G_y, dDl


def matched_filter_vjp(G_y, chirp, P: int, N: int, fs: float, band=None) -> np.ndarray:
    """dx [M][N] for yhat = matched_filter(x) (x real, zero-padded to P): the filter is
    yhat = IDFT(C . DFT(x)), so its adjoint is dx = Re IDFT(conj(C) . DFT(G_y)), cut to N."""
    C = chirp_spectrum_filter(chirp, P, fs, band)
    G_hat = np.fft.fft(np.asarray(G_y), axis=1)
    return np.real(np.fft.ifft(np.conj(C)[None, :] * G_hat, axis=1))[:, :N]


def delays_vjp(dDl, dirs, fs: float, c: float) -> np.ndarray:
    """dpos [M][3] for Dl = delays(pos, dirs): dDl[d][m] * fs/c * u_d summed over d."""
    u = np.asarray(dirs, dtype=np.float64)
    return (fs / c) * (np.asarray(dDl, dtype=np.float64).T @ u)


def das_fd_vjp(Yspec, Dl, n_idx, G_b):
    """Gradients of b = das_fd(Yspec, Dl, n_idx) given G_b [D][len(n_idx)].

    b_d = IDFT_P(B_d) on the window, B_d[k] = (1/M) sum_m Yhat_m[k] exp(-2j pi k Dl[d][m] / P)
    for k <= P/2.  The window read-out is linear, so G_B_d = DFT_P(G_b scattered onto Z_P) / P;
    then, bin by bin,
      G_Y[m][k] = (1/M) sum_d exp(+2j pi k Dl[d][m] / P) G_B_d[k]              (k <= P/2, else 0)
      dDl[d][m] = (1/M) sum_k Re(conj(G_B_d[k]) Yhat_m[k] (-2j pi k / P) exp(-2j pi k Dl[d][m] / P)).
    The steering phase is smooth in Dl, so these are exact derivatives everywhere.
    Returns (G_Y [M][P] complex, dDl [D][M] real)."""
    Y = np.asarray(Yspec)
    M, P = Y.shape
    Dl = np.asarray(Dl, dtype=np.float64)
    n_idx = np.mod(np.asarray(n_idx, dtype=np.int64), P)
    G_b = np.asarray(G_b)
    D = Dl.shape[0]
    k = np.arange(P // 2 + 1, dtype=np.float64)
    G_Y = np.zeros((M, P), dtype=np.complex128)
    dDl = np.zeros((D, M))
    for d in range(D):
        g = np.zeros(P, dtype=np.complex128)
        np.add.at(g, n_idx, G_b[d])
        GB = np.fft.fft(g)[:P // 2 + 1] / P
        for m in range(M):
            ph = np.exp(-2j * np.pi * (k * Dl[d, m] / P))
            G_Y[m, :P // 2 + 1] += np.conj(ph) * GB / M
            dDl[d, m] = np.sum(np.real(np.conj(GB) * Y[m, :P // 2 + 1] * (-2j * np.pi * k / P) * ph)) / M
    return G_Y, dDl


def matched_filter_spectrum_vjp(G_Y, chirp, P: int, N: int, fs: float, band=None) -> np.ndarray:
    """dx [M][N] for Yhat = matched_filter_spectrum(x) = C . DFT_P(x) (x real, zero-padded):
    G_X = conj(C) G_Y and dL/dx[n] = Re sum_k G_X[k] exp(+2j pi k n / P), cut to N."""
    C = chirp_spectrum_filter(chirp, P, fs, band)
    return np.real(P * np.fft.ifft(np.conj(C)[None, :] * np.asarray(G_Y), axis=1))[:, :N]


def energyscape_vjp_fd(x, chirp, mic_pos, dirs, dE, *, fs: float, c: float, P: int | None = None,
                       gate=None, R: int = 10, taps=None, band=None):
    """(dx [M][N], dpos [M][3]) of L = sum(dE * energyscape(..., mode='fd')) by the chain rule:
    envelope -> exact-phase delay-and-sum -> matched-filter spectrum and delays."""
    x = np.asarray(x, dtype=np.float64)
    M, N = x.shape
    L = len(chirp)
    if P is None:
        P = 1
        while P < N + L - 1:
            P *= 2
    n0, n1 = (0, N) if gate is None else gate
    h = default_lowpass(R) if taps is None else np.asarray(taps, dtype=np.float64)
    K = h.size
    Q = num_range_bins(n0, n1, R)
    Dl = delays(mic_pos, dirs, fs, c)
    n_idx = beam_window_indices(n0, Q, R, K)
    Y = matched_filter_spectrum(x, chirp, P, fs, band)
    b = das_fd(Y, Dl, n_idx)
    G_b = envelope_vjp(b, h, dE, Q, R)
    G_Y, dDl = das_fd_vjp(Y, Dl, n_idx, G_b)
    dx = matched_filter_spectrum_vjp(G_Y, chirp, P, N, fs, band)
    dpos = delays_vjp(dDl, dirs, fs, c)
    return dx, dpos


def energyscape_vjp_td(x, chirp, mic_pos, dirs, dE, *, fs: float, c: float, P: int | None = None,
                       gate=None, R: int = 10, taps=None, band=None, interp: str = "linear"):
    """(dx [M][N], dpos [M][3]) of L = sum(dE * energyscape(..., mode='td')) (interp 'linear') or
    of mode='td_cubic' (interp 'cubic') by the chain rule: envelope -> delay-and-sum -> matched
    filter and delays."""
    if interp not in ("linear", "cubic"):
        raise ValueError("interp must be 'linear' or 'cubic'")
    x = np.asarray(x, dtype=np.float64)
    M, N = x.shape
    L = len(chirp)
    if P is None:
        P = 1
        while P < N + L - 1:
            P *= 2
    n0, n1 = (0, N) if gate is None else gate
    h = default_lowpass(R) if taps is None else np.asarray(taps, dtype=np.float64)
    K = h.size
    Q = num_range_bins(n0, n1, R)
    Dl = delays(mic_pos, dirs, fs, c)
    n_idx = beam_window_indices(n0, Q, R, K)
    yhat = matched_filter(x, chirp, P, fs, band)
    b = das_td(yhat, Dl, n_idx) if interp == "linear" else das_td_cubic(yhat, Dl, n_idx)
    G_b = envelope_vjp(b, h, dE, Q, R)
    G_y, dDl = (das_td_vjp if interp == "linear" else das_td_cubic_vjp)(yhat, Dl, n_idx, G_b)
    dx = matched_filter_vjp(G_y, chirp, P, N, fs, band)
    dpos = delays_vjp(dDl, dirs, fs, c)
    return dx, dpos
