"""Synthetic recordings with the shapes of the paper's workload.

The paper measures on real recordings of a 32-microphone eRTIS sensor sampled
at 450 kHz (§2 Sonar Synchronisation), processed with 90, 1850 and 3000
directions of interest (§5 Experimental Validation).  Those recordings, the
array layout (Fig. 1a) and the sweep parameters are not published, so every
input here is seeded and synthetic:

* array: microphones uniform in a square planar aperture in the z = 0 plane
  (the paper only says "known, irregularly positioned");
* emitted sweep: Hann-windowed linear FM sweep (the paper says "broadband
  FM-sweep");
* echoes: point reflectors with 1/r amplitude spreading and exact spherical
  round-trip travel time from an emitter at the origin, with the continuous
  sweep evaluated at each sample instant (no interpolation);
* noise: white Gaussian at a stated SNR, sigma^2 = mean(clean^2) / 10^(SNR/10).

Seeds: numpy SeedSequence([config_id, sensor, frame, stream]) with stream
0 = geometry, 1 = reflectors, 2 = noise; frames of one sensor share geometry.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

FS_HZ = 450e3      # §2: the eRTIS samples at 450 kHz
C_MPS = 343.0      # speed of sound in air at 20 C (not stated in the paper)
N_MICS = 32        # §2: 32 digital microphones


def _rng(cfg_id: int, sensor: int, frame: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg_id, sensor, frame, stream]))


def linear_chirp(fs: float = FS_HZ, f0: float = 25e3, f1: float = 80e3, T: float = 1e-3) -> np.ndarray:
    """Samples s[l] = s(l/fs), l < round(T*fs), of the Hann-windowed linear sweep."""
    L = int(round(T * fs))
    t = np.arange(L) / fs
    return _chirp_at(t, f0, f1, T)


def _chirp_at(t, f0, f1, T):
    t = np.asarray(t, dtype=np.float64)
    inside = (t >= 0.0) & (t < T)
    w = 0.5 * (1.0 - np.cos(2.0 * np.pi * t / T))
    s = w * np.sin(2.0 * np.pi * (f0 * t + (f1 - f0) * t * t / (2.0 * T)))
    return np.where(inside, s, 0.0)


def planar_array(M: int, aperture: float, rng: np.random.Generator) -> np.ndarray:
    """[M][3] positions, uniform in [-a/2, a/2]^2 in the z = 0 plane (metres)."""
    pos = np.zeros((M, 3))
    pos[:, :2] = rng.uniform(-aperture / 2, aperture / 2, size=(M, 2))
    return pos


def azimuth_grid(n: int = 91, lo_deg: float = -90.0, step_deg: float = 2.0) -> np.ndarray:
    """Horizontal-plane directions u = (sin az, 0, cos az) (2D image of §5)."""
    az = np.deg2rad(lo_deg + step_deg * np.arange(n))
    return np.stack([np.sin(az), np.zeros(n), np.cos(az)], axis=1)


def fibonacci_hemisphere(D: int) -> np.ndarray:
    """D near-uniform directions on the frontal (z > 0) hemisphere (golden-angle spiral)."""
    i = np.arange(D, dtype=np.float64)
    z = (i + 0.5) / D
    phi = i * np.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(1.0 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def restricted_grid(D_target: int = 1850, half_deg: float = 45.0) -> np.ndarray:
    """Fibonacci directions with |azimuth|, |elevation| <= half_deg (the 1850-direction case of §5).

    The spiral density is chosen so that about D_target points survive the cut.
    """
    best = None
    for D in range(D_target, 20 * D_target):
        u = fibonacci_hemisphere(D)
        az = np.degrees(np.arctan2(u[:, 0], u[:, 2]))
        el = np.degrees(np.arcsin(np.clip(u[:, 1], -1, 1)))
        keep = u[(np.abs(az) <= half_deg) & (np.abs(el) <= half_deg)]
        if keep.shape[0] >= D_target:
            best = keep
            break
    return best


@dataclasses.dataclass(frozen=True)
class Config:
    cfg_id: int
    name: str
    n_mics: int
    aperture: float
    n_samples: int
    n_reflectors: int
    r_range: tuple
    snr_db: float
    grid: str                 # "az91" or "fib<D>"
    band: tuple | None        # matched-filter band mask in Hz, or None
    decim: int = 10
    planar_reflectors: bool = False   # True: elevation 0, azimuth within +-80 deg


CONFIGS = {
    # plain method, 1 sensor, horizontal plane (small enough for the oracle in seconds)
    "c1": Config(1, "c1", 32, 0.035, 4096, 3, (0.5, 4.0), 20.0, "az91", None, planar_reflectors=True),
    # single sensor, full 3D, the throughput workload: 32 mics x 16384 samples x 1500 directions
    "c2": Config(2, "c2", 32, 0.035, 16384, 20, (0.3, 6.0), 20.0, "fib1500", (20e3, 85e3)),
    # sensor network (one entry per sensor; sizes per sensor come from network_sensor_shape)
    "c3": Config(3, "c3", 32, 0.035, 16384, 20, (0.3, 6.0), 20.0, "fib1500", (20e3, 85e3)),
    # stress: 64 mics in 7 cm, 65536 samples, 10000 directions
    "c5": Config(5, "c5", 64, 0.070, 65536, 50, (0.3, 24.0), 10.0, "fib10000", (20e3, 85e3)),
}


@dataclasses.dataclass
class Workload:
    cfg: Config
    x: np.ndarray          # [F][M][N] float32
    chirp: np.ndarray      # [L] float64
    mic_pos: np.ndarray    # [M][3] float64
    dirs: np.ndarray       # [D][3] float64
    reflectors: list       # per frame: list of (r, u[3], amplitude)
    fs: float = FS_HZ
    c: float = C_MPS


def make_grid(grid: str) -> np.ndarray:
    if grid == "az91":
        return azimuth_grid(91)
    if grid.startswith("fib"):
        return fibonacci_hemisphere(int(grid[3:]))
    raise ValueError(grid)


def simulate_frame(mic_pos, chirp_params, reflectors, n_samples, snr_db, rng_noise,
                   fs: float = FS_HZ, c: float = C_MPS) -> np.ndarray:
    """x[m][n] = sum_i (a_i/r_i) s(n/fs - tau_im) + noise, tau_im = (r_i + |r_i u_i - p_m|)/c."""
    f0, f1, T = chirp_params
    M = mic_pos.shape[0]
    x = np.zeros((M, n_samples))
    L = int(round(T * fs))
    for (r, u, a) in reflectors:
        pt = r * np.asarray(u)
        for m in range(M):
            tau = (r + np.linalg.norm(pt - mic_pos[m])) / c
            n_first = int(math.floor(tau * fs))
            lo = max(n_first, 0)
            hi = min(n_first + L + 2, n_samples)
            if lo >= hi:
                continue
            n = np.arange(lo, hi)
            x[m, lo:hi] += (a / r) * _chirp_at(n / fs - tau, f0, f1, T)
    p_sig = float(np.mean(x * x))
    if snr_db is not None and p_sig > 0:
        sigma = math.sqrt(p_sig / (10.0 ** (snr_db / 10.0)))
        x += rng_noise.normal(0.0, sigma, size=x.shape)
    return x


def _draw_reflectors(cfg: Config, rng: np.random.Generator):
    out = []
    for _ in range(cfg.n_reflectors):
        r = rng.uniform(*cfg.r_range)
        if cfg.planar_reflectors:
            az = np.deg2rad(rng.uniform(-80.0, 80.0))
            u = np.array([np.sin(az), 0.0, np.cos(az)])
        else:
            z = rng.uniform(0.0, 1.0)
            ph = rng.uniform(0.0, 2 * np.pi)
            s = math.sqrt(1.0 - z * z)
            u = np.array([s * math.cos(ph), s * math.sin(ph), z])
        a = rng.uniform(0.2, 1.0)
        out.append((r, u, a))
    return out


def make_workload(name: str, frames: int = 1, sensor: int = 0, n_samples: int | None = None,
                  n_dirs: int | None = None, n_mics: int | None = None,
                  chirp_params=(25e3, 80e3, 1e-3)) -> Workload:
    """Seeded synthetic batch of `frames` recordings of one sensor for a named config.

    n_samples / n_dirs / n_mics override the config's sizes (for reduced test shapes);
    the seeds stay those of the named config.
    """
    cfg = CONFIGS[name]
    if n_samples is not None or n_mics is not None:
        cfg = dataclasses.replace(cfg, n_samples=n_samples or cfg.n_samples,
                                  n_mics=n_mics or cfg.n_mics)
    mic_pos = planar_array(cfg.n_mics, cfg.aperture, _rng(cfg.cfg_id, sensor, 0, 0))
    dirs = make_grid(cfg.grid) if n_dirs is None else fibonacci_hemisphere(n_dirs)
    if n_dirs is not None and cfg.grid == "az91":
        dirs = azimuth_grid(n_dirs, -90.0, 180.0 / max(n_dirs - 1, 1))
    chirp = linear_chirp(FS_HZ, *chirp_params)
    xs, refl = [], []
    for f in range(frames):
        rf = _draw_reflectors(cfg, _rng(cfg.cfg_id, sensor, f, 1))
        x = simulate_frame(mic_pos, chirp_params, rf, cfg.n_samples, cfg.snr_db,
                           _rng(cfg.cfg_id, sensor, f, 2))
        xs.append(x.astype(np.float32))
        refl.append(rf)
    return Workload(cfg, np.stack(xs), chirp, mic_pos, dirs, refl)


NETWORK_LENGTHS = (8192, 16384, 32768)


def network_sensor_shape(sensor: int) -> tuple:
    """(N, grid) of one sensor of the heterogeneous network: N cycles through NETWORK_LENGTHS
    from a seeded offset, the grid alternates between the 91-azimuth 2D image and the
    1500-direction hemisphere."""
    off = int(_rng(3, 0, 0, 3).integers(len(NETWORK_LENGTHS)))
    n = NETWORK_LENGTHS[(sensor * 2 + off) % len(NETWORK_LENGTHS)]
    grid = "az91" if sensor % 2 == 0 else "fib1500"
    return n, grid


def make_network(sensors: int = 8, frames: int = 4, n_dirs: int | None = None) -> list:
    """Seeded sensor network: one Workload per sensor, each with its own array geometry,
    recording length and direction grid (n_dirs overrides the 3D grid's size for tests)."""
    out = []
    for s in range(sensors):
        n, grid = network_sensor_shape(s)
        cfg = dataclasses.replace(CONFIGS["c3"], n_samples=n, grid=grid,
                                  planar_reflectors=(grid == "az91"))
        mic_pos = planar_array(cfg.n_mics, cfg.aperture, _rng(3, s, 0, 0))
        dirs = make_grid(grid)
        if n_dirs is not None and grid != "az91":
            dirs = fibonacci_hemisphere(n_dirs)
        chirp_params = (25e3, 80e3, 1e-3)
        chirp = linear_chirp(FS_HZ, *chirp_params)
        xs, refl = [], []
        for f in range(frames):
            rf = _draw_reflectors(cfg, _rng(3, s, f, 1))
            xs.append(simulate_frame(mic_pos, chirp_params, rf, n, cfg.snr_db, _rng(3, s, f, 2)).astype(np.float32))
            refl.append(rf)
        out.append(Workload(cfg, np.stack(xs), chirp, mic_pos, dirs, refl))
    return out


@dataclasses.dataclass
class CalibrationWorkload:
    x: np.ndarray          # [F][M][N] float32, recorded with true_pos
    chirp: np.ndarray      # [L] float64
    true_pos: np.ndarray   # [M][3] float64
    start_pos: np.ndarray  # [M][3] float64: true_pos plus the seeded perturbation
    dirs: np.ndarray       # [D][3] float64
    cells: list            # per frame: list of (d, q) energyscape cells of the reflectors
    band: tuple
    decim: int
    fs: float = FS_HZ
    c: float = C_MPS


def make_calibration(frames: int = 10, reflectors: int = 5, sigma: float = 0.5e-3, n_samples: int = 16384,
                     n_dirs: int = 1500, n_mics: int = N_MICS, snr_db: float = 20.0,
                     chirp_params=(25e3, 80e3, 1e-3)) -> CalibrationWorkload:
    """Seeded array self-calibration workload (cfg_id 4).

    Reflectors sit in the far field of the 3.5 cm array, so the echo at microphone m
    arrives after tau = (2 r - p_m . u) / c (the plane-wave model of the §4.1 delays),
    with a common amplitude per reflector (no spreading loss).  Each reflector is placed
    exactly on a grid direction d and at a range r = q R c / (2 fs) that puts its beam
    peak on the centre of range cell q, so the energyscape cells (d, q) are known and
    the ideal geometry maximises E there.  Ranges of one frame are distinct multiples of
    25 cells, so the compressed echoes of one frame do not overlap in range.
    Seeds: SeedSequence([4, 0, frame, stream]), stream 0 = geometry, 1 = reflectors,
    2 = noise, 4 = position perturbation (Gaussian, sigma metres per coordinate).
    """
    R = 10
    fs, c = FS_HZ, C_MPS
    true_pos = planar_array(n_mics, 0.035, _rng(4, 0, 0, 0))
    start_pos = true_pos + _rng(4, 0, 0, 4).normal(0.0, sigma, size=true_pos.shape)
    dirs = fibonacci_hemisphere(n_dirs)
    f0, f1, T = chirp_params
    chirp = linear_chirp(fs, f0, f1, T)
    L = chirp.size
    q_hi = (n_samples - L - 8) // R
    slots = np.arange(50, q_hi, 25)
    xs, cells = [], []
    for f in range(frames):
        rng = _rng(4, 0, f, 1)
        ds = rng.choice(n_dirs, size=reflectors, replace=False)
        qs = rng.choice(slots, size=reflectors, replace=False)
        amps = rng.uniform(0.5, 1.0, size=reflectors)
        x = np.zeros((n_mics, n_samples))
        n = np.arange(n_samples)
        for d, q, a in zip(ds, qs, amps):
            r = q * R * c / (2.0 * fs)
            for m in range(n_mics):
                tau = (2.0 * r - true_pos[m] @ dirs[d]) / c
                x[m] += a * _chirp_at(n / fs - tau, f0, f1, T)
        p_sig = float(np.mean(x * x))
        sig = math.sqrt(p_sig / (10.0 ** (snr_db / 10.0)))
        x += _rng(4, 0, f, 2).normal(0.0, sig, size=x.shape)
        xs.append(x.astype(np.float32))
        cells.append([(int(d), int(q)) for d, q in zip(ds, qs)])
    return CalibrationWorkload(np.stack(xs), chirp, true_pos, start_pos, dirs, cells, (20e3, 85e3), R)
