"""Thin ctypes binding of the C ABI in include/sonar.h.

Argument marshalling only: every step of the pipeline runs in the HIP
library.  PyTorch supplies device memory (tensors) and the stream handle; the
library never sees a torch type.  Loading fails loudly when the library has
not been built: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libsonar.so")

SONAR_OK = 0
SONAR_E_INVALID = -1
SONAR_E_NOMEM = -2
SONAR_E_HIP = -3
SONAR_E_UNSUPPORTED = -4

PRECISIONS = {"fp32": 0, "bf16": 1}
BF_MODES = {"td": 0, "fd_fp32": 1, "fd_bf16": 2, "fd_bf16x3": 3, "td_bf16": 4, "td_nearest": 5, "td_cubic": 6, "td_bf16x2": 7, "td_f16": 8,
            "td_bf16g": 9}
DTYPES = {"f32": 0, "f16": 1, "bf16": 2}

Q_RANGE_BINS, Q_BEAM_LEN, Q_FFT_LEN, Q_MF_ROW, Q_MF_ORIGIN = 0, 1, 2, 3, 4
Q_BAND_LO_BIN, Q_BAND_BINS, Q_WORKSPACE_BYTES, Q_LPF_LEN, Q_MF_FRAME_ELEMS = 5, 6, 7, 8, 9
Q_MATRIX_FLOP_PER_FRAME = 10
Q_MT_WAVES = 11
Q_BEAM_SPEC_STRIDE, Q_FD_PHASE_LEN, Q_FD_FUSED = 12, 13, 14

_dp = ctypes.POINTER(ctypes.c_double)


class PlanDesc(ctypes.Structure):
    """Mirror of sonar_plan_desc (field order and types as in include/sonar.h)."""
    _fields_ = [
        ("n_mics", ctypes.c_int32), ("mic_pos", _dp),
        ("chirp_len", ctypes.c_int32), ("chirp", _dp),
        ("fs_hz", ctypes.c_double), ("c_mps", ctypes.c_double),
        ("n_dirs", ctypes.c_int32), ("dirs", _dp),
        ("n_samples", ctypes.c_int32),
        ("gate_begin", ctypes.c_int32), ("gate_end", ctypes.c_int32),
        ("decim", ctypes.c_int32),
        ("lpf_len", ctypes.c_int32), ("lpf_taps", _dp),
        ("band_lo_hz", ctypes.c_double), ("band_hi_hz", ctypes.c_double),
        ("fft_len", ctypes.c_int32),
        ("bf_mode", ctypes.c_int32), ("sample_dtype", ctypes.c_int32), ("max_frames", ctypes.c_int32),
    ]


class PdmDesc(ctypes.Structure):
    """Mirror of sonar_pdm_desc."""
    _fields_ = [
        ("n_mics", ctypes.c_int32), ("n_out", ctypes.c_int32), ("decim", ctypes.c_int32),
        ("n_taps", ctypes.c_int32), ("taps", _dp), ("max_frames", ctypes.c_int32),
    ]


_lib = None

# name -> (restype, argtypes); every function declared in include/sonar.h
_SIGNATURES = {
    "sonar_plan_create": (ctypes.c_int, [ctypes.POINTER(PlanDesc), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sonar_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sonar_plan_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "sonar_matched_filter": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sonar_beamform": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sonar_envelope": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sonar_beam_spectrum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "sonar_beamform_envelope": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sonar_energyscape_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sonar_energyscape_batch_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                       ctypes.c_void_p]),
    "sonar_energyscape_multi": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_void_p),
                                                ctypes.c_int32, ctypes.c_void_p]),
    "sonar_plan_create_tuned": (ctypes.c_int, [ctypes.POINTER(PlanDesc), ctypes.c_int32, ctypes.c_void_p,
                                                ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int32)]),
    "sonar_plan_enable_gradients": (ctypes.c_int, [ctypes.c_void_p]),
    "sonar_tune_cache": (ctypes.c_int, [ctypes.c_char_p]),
    "sonar_energyscape_vjp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "sonar_plan_set_positions": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sonar_energyscape_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sonar_energyscape_cells": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p]),
    "sonar_pdm_create": (ctypes.c_int, [ctypes.POINTER(PdmDesc), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sonar_pdm_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sonar_pdm_demodulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "sonar_plan_set_envelope_iir": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sonar_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sonar_last_error": (ctypes.c_char_p, []),
}


def load():
    """Load libsonar.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class SonarError(RuntimeError):
    def __init__(self, status: int, what: str):
        lib = load()
        msg = lib.sonar_last_error().decode()
        super().__init__(f"{what}: {lib.sonar_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _check(status: int, what: str):
    if status != SONAR_OK:
        raise SonarError(status, what)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A plan: array geometry, sweep, directions and range gate, with its device workspace."""

    def __init__(self, mic_pos, chirp, dirs, n_samples: int, *, fs: float, c: float,
                 gate=None, decim: int = 10, taps=None, band=None, fft_len: int = 0,
                 mode: str = "td", sample_dtype: str = "f32", max_frames: int = 1, stream=None,
                 tune: str | None = None):
        """tune = "fp32" or "bf16" lets sonar_plan_create_tuned pick the fastest mode of that
        precision class (mode is then ignored; the choice is in self.mode)."""
        lib = load()
        self._keep = []
        pos = _f64(mic_pos)
        u = _f64(dirs)
        s = _f64(chirp).reshape(-1)
        h = None if taps is None else _f64(taps).reshape(-1)
        self._keep += [pos, u, s, h]
        d = PlanDesc()
        d.n_mics = pos.shape[0]
        d.mic_pos = _ptr(pos)
        d.chirp_len = s.size
        d.chirp = _ptr(s)
        d.fs_hz = fs
        d.c_mps = c
        d.n_dirs = u.shape[0]
        d.dirs = _ptr(u)
        d.n_samples = int(n_samples)
        d.gate_begin, d.gate_end = (0, 0) if gate is None else (int(gate[0]), int(gate[1]))
        d.decim = int(decim)
        d.lpf_len = 0 if h is None else h.size
        d.lpf_taps = _ptr(h)
        d.band_lo_hz, d.band_hi_hz = (0.0, 0.0) if band is None else (float(band[0]), float(band[1]))
        d.fft_len = int(fft_len)
        d.bf_mode = BF_MODES[mode]
        d.sample_dtype = DTYPES[sample_dtype]
        d.max_frames = int(max_frames)
        self.mode = mode
        self.sample_dtype = sample_dtype
        self.M, self.D, self.N = d.n_mics, d.n_dirs, d.n_samples
        self.max_frames = d.max_frames
        handle = ctypes.c_void_p()
        if tune is None:
            _check(lib.sonar_plan_create(ctypes.byref(d), _stream_handle(stream), ctypes.byref(handle)),
                   "sonar_plan_create")
        else:
            chosen = ctypes.c_int32(-1)
            _check(lib.sonar_plan_create_tuned(ctypes.byref(d), PRECISIONS[tune], _stream_handle(stream),
                                               ctypes.byref(handle), ctypes.byref(chosen)),
                   "sonar_plan_create_tuned")
            self.mode = {v: k for k, v in BF_MODES.items()}[chosen.value]
        self._h = handle
        self.Q = self.query(Q_RANGE_BINS)
        self.G = self.query(Q_BEAM_LEN)
        self.P = self.query(Q_FFT_LEN)
        self.K = self.query(Q_LPF_LEN)
        self.mf_row = self.query(Q_MF_ROW)
        self.mf_origin = self.query(Q_MF_ORIGIN)
        self.mf_frame_elems = self.query(Q_MF_FRAME_ELEMS)
        self.band_lo_bin = self.query(Q_BAND_LO_BIN)
        self.band_bins = self.query(Q_BAND_BINS)

    # -- plumbing -------------------------------------------------------------
    def query(self, what: int) -> int:
        v = ctypes.c_int64()
        _check(load().sonar_plan_query(self._h, what, ctypes.byref(v)), "sonar_plan_query")
        return int(v.value)

    def close(self):
        if getattr(self, "_h", None):
            load().sonar_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _frames(self, t, per_frame_shape, what):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{what} must be a CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if tuple(t.shape[1:]) != tuple(per_frame_shape):
            raise ValueError(f"{what} must have shape [F]{list(per_frame_shape)}, got {list(t.shape)}")
        return t.shape[0]

    def _samples(self, x):
        import torch
        want = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[self.sample_dtype]
        if x.dtype != want:
            raise TypeError(f"x must be {want}, got {x.dtype}")
        return self._frames(x, (self.M, self.N), "x")

    def _out(self, out, shape, dtype, device):
        import torch
        if out is None:
            return torch.empty(shape, dtype=dtype, device=device)
        if tuple(out.shape) != tuple(shape) or out.dtype != dtype or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous {dtype} tensor of shape {list(shape)}")
        return out

    # -- pipeline -------------------------------------------------------------
    def energyscape(self, x, out=None, stream=None):
        """E[F][D][Q] (float32) for samples x[F][M][N]."""
        import torch
        F = self._samples(x)
        E = self._out(out, (F, self.D, self.Q), torch.float32, x.device)
        _check(load().sonar_energyscape_batch(self._h, ctypes.c_void_p(x.data_ptr()), F,
                                              ctypes.c_void_p(E.data_ptr()), _stream_handle(stream)),
               "sonar_energyscape_batch")
        return E

    def energyscape_static(self, x, out=None, stream=None):
        """sonar_energyscape_batch_static: E[F][D][Q] with the per-frame buffers in the library's static
        device scratch (no allocation in the call; calls on one device must not overlap).  `out`
        should be given by callers that cannot allocate."""
        import torch
        F = self._samples(x)
        E = self._out(out, (F, self.D, self.Q), torch.float32, x.device)
        _check(load().sonar_energyscape_batch_static(self._h, ctypes.c_void_p(x.data_ptr()), F,
                                                     ctypes.c_void_p(E.data_ptr()), _stream_handle(stream)),
               "sonar_energyscape_batch_static")
        return E

    def matched_filter(self, x, out=None, stream=None):
        """Matched-filter buffer, complex64 [F][mf_frame_elems] (layout per mode, see sonar.h)."""
        import torch
        F = self._samples(x)
        mf = self._out(out, (F, self.mf_frame_elems), torch.complex64, x.device)
        _check(load().sonar_matched_filter(self._h, ctypes.c_void_p(x.data_ptr()), F,
                                           ctypes.c_void_p(mf.data_ptr()), _stream_handle(stream)),
               "sonar_matched_filter")
        return mf

    def beamform(self, mf, out=None, stream=None):
        """Beam window b[F][D][G'] (complex64) from a matched-filter buffer."""
        import torch
        F = self._frames(mf, (self.mf_frame_elems,), "mf")
        b = self._out(out, (F, self.D, self.G), torch.complex64, mf.device)
        _check(load().sonar_beamform(self._h, ctypes.c_void_p(mf.data_ptr()), F,
                                     ctypes.c_void_p(b.data_ptr()), _stream_handle(stream)),
               "sonar_beamform")
        return b

    def beam_spectrum(self, mf, out=None, stream=None):
        """Frequency-domain plans: per-bin beam spectra B[F][D][S] (complex64, S = the padded row of
        stored bins; the first band_bins of each row are B_d at bins band_lo_bin + j)."""
        import torch
        F = self._frames(mf, (self.mf_frame_elems,), "mf")
        S = self.query(Q_BEAM_SPEC_STRIDE)
        B = self._out(out, (F, self.D, S), torch.complex64, mf.device)
        _check(load().sonar_beam_spectrum(self._h, ctypes.c_void_p(mf.data_ptr()), F,
                                          ctypes.c_void_p(B.data_ptr()), _stream_handle(stream)),
               "sonar_beam_spectrum")
        return B

    def envelope(self, beam, out=None, stream=None):
        """E[F][D][Q] from a beam window b[F][D][G']."""
        import torch
        F = self._frames(beam, (self.D, self.G), "beam")
        E = self._out(out, (F, self.D, self.Q), torch.float32, beam.device)
        _check(load().sonar_envelope(self._h, ctypes.c_void_p(beam.data_ptr()), F,
                                     ctypes.c_void_p(E.data_ptr()), _stream_handle(stream)),
               "sonar_envelope")
        return E

    def set_envelope_iir(self, n_sections: int = 2, sos=None, stream=None):
        """IIR envelope reading: n_sections second-order sections [S][6] (b0, b1, b2, a0, a1, a2), or the
        default Butterworth of order 2 n_sections at fs/(2R); n_sections = 0 returns to the FIR."""
        arr = None if sos is None else _f64(sos, (int(n_sections), 6))
        _check(load().sonar_plan_set_envelope_iir(self._h, int(n_sections), _ptr(arr), _stream_handle(stream)),
               "sonar_plan_set_envelope_iir")
        self._keep_sos = arr

    def enable_gradients(self):
        _check(load().sonar_plan_enable_gradients(self._h), "sonar_plan_enable_gradients")

    def set_positions(self, mic_pos, stream=None):
        """New microphone positions [M][3] (TD_LINEAR plans): rebuilds the delay table."""
        pos = _f64(mic_pos, (self.M, 3))
        _check(load().sonar_plan_set_positions(self._h, _ptr(pos), _stream_handle(stream)), "sonar_plan_set_positions")

    def vjp(self, mf, beam, dE, want_dx=True, want_dpos=True, stream=None):
        """sonar_energyscape_vjp.  Returns (G_mf, dx, dpos): G_mf is the gradient of the
        matched-filter output (TD modes: complex64 [F][M][P] over Z_P; FD modes: complex64
        [F][Kb][M] on the band bins), dx float32 [F][M][N] or None, dpos float64 numpy [M][3]
        or None.  beam (the forward beam window) is overwritten with G_b."""
        import torch
        self.enable_gradients()
        F = self._frames(mf, (self.mf_frame_elems,), "mf")
        self._frames(beam, (self.D, self.G), "beam")
        self._frames(dE, (self.D, self.Q), "dE")
        if dE.dtype != torch.float32 or beam.dtype != torch.complex64:
            raise TypeError("dE must be float32 and beam complex64")
        if beam.shape[0] != F or dE.shape[0] != F:
            raise ValueError("mf, beam and dE must hold the same number of frames")
        dy = dx = dpos = None
        if want_dx:
            shape = (F, self.M, self.P) if self.mode.startswith("td") else (F, self.band_bins, self.M)
            dy = torch.empty(shape, dtype=torch.complex64, device=mf.device)
            dx = torch.empty((F, self.M, self.N), dtype=torch.float32, device=mf.device)
        if want_dpos:
            dpos = torch.empty((self.M, 3), dtype=torch.float64, device=mf.device)
        _check(load().sonar_energyscape_vjp(self._h, ctypes.c_void_p(mf.data_ptr()), ctypes.c_void_p(beam.data_ptr()),
                                            ctypes.c_void_p(dE.data_ptr()), F,
                                            ctypes.c_void_p(dy.data_ptr() if dy is not None else 0),
                                            ctypes.c_void_p(dx.data_ptr() if dx is not None else 0),
                                            ctypes.c_void_p(dpos.data_ptr() if dpos is not None else 0),
                                            _stream_handle(stream)), "sonar_energyscape_vjp")
        return dy, dx, (dpos.cpu().numpy() if dpos is not None else None)

    def backward(self, x, dE, want_dx=True, want_dpos=True, stream=None):
        """sonar_energyscape_backward: (dx [F][M][N] float32 or None, dpos [M][3] float64 numpy or None)."""
        import torch
        self.enable_gradients()
        F = self._samples(x)
        self._frames(dE, (self.D, self.Q), "dE")
        if dE.dtype != torch.float32 or dE.shape[0] != F:
            raise ValueError("dE must be float32 [F][D][Q] with the frames of x")
        dx = torch.empty((F, self.M, self.N), dtype=torch.float32, device=x.device) if want_dx else None
        dpos = torch.empty((self.M, 3), dtype=torch.float64, device=x.device) if want_dpos else None
        _check(load().sonar_energyscape_backward(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(dE.data_ptr()),
                                                 F, ctypes.c_void_p(dx.data_ptr() if dx is not None else 0),
                                                 ctypes.c_void_p(dpos.data_ptr() if dpos is not None else 0),
                                                 _stream_handle(stream)), "sonar_energyscape_backward")
        return dx, (dpos.cpu().numpy() if dpos is not None else None)

    def cells(self, mf, cells, dE, want_E=True, want_dpos=True, stream=None):
        """sonar_energyscape_cells: (E [n] float32 tensor or None, dpos [M][3] float64 numpy or None)
        for cells int32 [n][3] (f, d, q) and weights dE float32 [n] on the device."""
        import torch
        self.enable_gradients()
        F = self._frames(mf, (self.mf_frame_elems,), "mf")
        if not (isinstance(cells, torch.Tensor) and cells.is_cuda and cells.dtype == torch.int32 and cells.dim() == 2
                and cells.shape[1] == 3 and cells.is_contiguous()):
            raise ValueError("cells must be a contiguous int32 CUDA tensor [n][3]")
        n = cells.shape[0]
        if not (isinstance(dE, torch.Tensor) and dE.is_cuda and dE.dtype == torch.float32 and tuple(dE.shape) == (n,)
                and dE.is_contiguous()):
            raise ValueError("dE must be a contiguous float32 CUDA tensor [n]")
        E = torch.empty((n,), dtype=torch.float32, device=mf.device) if want_E else None
        dpos = torch.empty((self.M, 3), dtype=torch.float64, device=mf.device) if want_dpos else None
        _check(load().sonar_energyscape_cells(self._h, ctypes.c_void_p(mf.data_ptr()), ctypes.c_void_p(cells.data_ptr()),
                                              n, ctypes.c_void_p(dE.data_ptr()), F,
                                              ctypes.c_void_p(E.data_ptr() if E is not None else 0),
                                              ctypes.c_void_p(dpos.data_ptr() if dpos is not None else 0),
                                              _stream_handle(stream)), "sonar_energyscape_cells")
        return E, (dpos.cpu().numpy() if dpos is not None else None)

    def beamform_envelope(self, mf, out=None, stream=None):
        """E[F][D][Q] from a matched-filter buffer, beam kept on chip."""
        import torch
        F = self._frames(mf, (self.mf_frame_elems,), "mf")
        E = self._out(out, (F, self.D, self.Q), torch.float32, mf.device)
        _check(load().sonar_beamform_envelope(self._h, ctypes.c_void_p(mf.data_ptr()), F,
                                              ctypes.c_void_p(E.data_ptr()), _stream_handle(stream)),
               "sonar_beamform_envelope")
        return E


class Pdm:
    """PDM front end: packed 1-bit words [F][N*decim][ceil(M/32)] (uint32 viewed as int32 in torch)
    -> samples [F][M][N] float32 on the device (sonar_pdm_demodulate)."""

    def __init__(self, n_mics: int, n_out: int, decim: int = 10, taps=None, max_frames: int = 1, stream=None):
        d = PdmDesc()
        d.n_mics, d.n_out, d.decim, d.max_frames = int(n_mics), int(n_out), int(decim), int(max_frames)
        self._keep = None
        if taps is None:
            d.n_taps, d.taps = 0, None
        else:
            self._keep = _f64(taps)
            d.n_taps, d.taps = self._keep.size, _ptr(self._keep)
        h = ctypes.c_void_p()
        _check(load().sonar_pdm_create(ctypes.byref(d), _stream_handle(stream), ctypes.byref(h)), "sonar_pdm_create")
        self._h = h
        self.M, self.N, self.decim, self.max_frames = d.n_mics, d.n_out, d.decim, d.max_frames
        self.W = (self.M + 31) // 32

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().sonar_pdm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def demodulate(self, words, out=None, stream=None):
        import torch
        if not isinstance(words, torch.Tensor) or not words.is_cuda or not words.is_contiguous():
            raise TypeError("words must be a contiguous CUDA tensor")
        if words.dtype not in (torch.int32, torch.uint32):
            raise TypeError("words must hold 32-bit words (int32 or uint32)")
        if tuple(words.shape[1:]) != (self.N * self.decim, self.W):
            raise ValueError(f"words must have shape [F][{self.N * self.decim}][{self.W}], got {list(words.shape)}")
        F = words.shape[0]
        x = torch.empty((F, self.M, self.N), dtype=torch.float32, device=words.device) if out is None else out
        if tuple(x.shape) != (F, self.M, self.N) or x.dtype != torch.float32 or not x.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor [F][M][N]")
        _check(load().sonar_pdm_demodulate(self._h, ctypes.c_void_p(words.data_ptr()), F, ctypes.c_void_p(x.data_ptr()),
                                           _stream_handle(stream)), "sonar_pdm_demodulate")
        return x


class Energyscape:
    """Differentiable energyscape of one TD_LINEAR or FD plan: E = f(x, positions).

    Energyscape.apply(x, pos, plan): x [F][M][N] float32 CUDA tensor, pos [M][3] float64
    CPU tensor (written into the plan with sonar_plan_set_positions), returns E [F][D][Q].
    The backward pass is sonar_energyscape_vjp: dL/dx on the device, dL/dpos on the host."""

    _fn = None

    @staticmethod
    def _make():
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, x, pos, plan):
                pos_np = np.array(pos.detach().cpu().numpy(), dtype=np.float64, copy=True)
                plan.set_positions(pos_np)
                mf = plan.matched_filter(x)
                beam = plan.beamform(mf)
                E = plan.envelope(beam)
                ctx.plan = plan
                # the VJP kernels read the plan's delay tables: a later forward on the same plan
                # moves them, so backward puts this forward's geometry back first
                ctx.pos = pos_np
                ctx.save_for_backward(mf, beam)
                return E

            @staticmethod
            def backward(ctx, dE):
                mf, beam = ctx.saved_tensors
                want_dx, want_dpos = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
                ctx.plan.set_positions(ctx.pos)
                _, dx, dpos = ctx.plan.vjp(mf, beam.clone(), dE.contiguous(), want_dx=want_dx, want_dpos=want_dpos)
                return dx, (torch.from_numpy(dpos) if dpos is not None else None), None

        return _Fn

    @classmethod
    def apply(cls, x, pos, plan):
        if cls._fn is None:
            cls._fn = cls._make()
        return cls._fn.apply(x, pos, plan)


def tune_cache(path):
    """sonar_tune_cache: JSON-lines file that persists tuned plan choices (None switches it off)."""
    _check(load().sonar_tune_cache(None if path is None else os.fsencode(path)), "sonar_tune_cache")


def energyscape_multi(plans, xs, outs=None, stream=None):
    """sonar_energyscape_multi: E_i for each (plan_i, x_i[F_i][M_i][N_i]); returns the list of E_i."""
    import torch
    n = len(plans)
    if len(xs) != n or (outs is not None and len(outs) != n):
        raise ValueError("plans, xs (and outs) must have the same length")
    Es = []
    for i, (pl, x) in enumerate(zip(plans, xs)):
        F = pl._samples(x)
        Es.append(pl._out(None if outs is None else outs[i], (F, pl.D, pl.Q), torch.float32, x.device))
    arr_p = (ctypes.c_void_p * n)(*[pl._h.value for pl in plans])
    arr_x = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    arr_f = (ctypes.c_int32 * n)(*[x.shape[0] for x in xs])
    arr_e = (ctypes.c_void_p * n)(*[E.data_ptr() for E in Es])
    _check(load().sonar_energyscape_multi(arr_p, arr_x, arr_f, arr_e, n, _stream_handle(stream)),
           "sonar_energyscape_multi")
    return Es


def header_functions(header_path=None):
    """Names of the functions declared in include/sonar.h."""
    import re
    if header_path is None:
        header_path = os.path.join(os.path.dirname(PKG), "include", "sonar.h")
    with open(header_path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sonar_[a-z_]+)\s*\(", text)))
