"""CPU-side checks of the C ABI: the library loads, exports every declared symbol,
and rejects bad descriptors in host code before any device work."""

import ctypes
import os

import numpy as np
import pytest

from paper_2208_10839_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_pipeline_calls():
    names = binding.header_functions()
    for n in ("sonar_plan_create", "sonar_plan_destroy", "sonar_plan_query", "sonar_matched_filter",
              "sonar_beamform", "sonar_envelope", "sonar_beamform_envelope", "sonar_energyscape_batch",
              "sonar_status_string", "sonar_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for n in binding.header_functions():
        assert hasattr(lib, n), n
    # the binding covers exactly the declared surface
    assert sorted(binding._SIGNATURES) == binding.header_functions()


def test_status_strings():
    lib = binding.load()
    assert lib.sonar_status_string(0) == b"success"
    assert lib.sonar_status_string(-1) == b"invalid argument"
    assert lib.sonar_status_string(-4) == b"unsupported configuration"
    assert lib.sonar_status_string(12345) == b"unknown status"


def test_descriptor_layout_matches_header_field_order():
    import re
    with open(os.path.join(ROOT, "include", "sonar.h")) as f:
        text = f.read()
    body = text[text.index("typedef struct {"):text.index("} sonar_plan_desc;")]
    fields = re.findall(r"\b(?:int32_t|double|const double\*)\s+(\w+);", body)
    assert fields == [f[0] for f in binding.PlanDesc._fields_]


def _desc(**over):
    pos = np.zeros((4, 3))
    pos[:, 0] = [0.0, 0.01, -0.01, 0.005]
    dirs = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.8]])
    chirp = np.ones(8)
    keep = [pos, dirs, chirp]
    d = binding.PlanDesc()
    d.n_mics, d.mic_pos = 4, pos.ctypes.data_as(binding._dp)
    d.chirp_len, d.chirp = 8, chirp.ctypes.data_as(binding._dp)
    d.fs_hz, d.c_mps = 450e3, 343.0
    d.n_dirs, d.dirs = 2, dirs.ctypes.data_as(binding._dp)
    d.n_samples, d.decim, d.max_frames = 100, 4, 1
    for k, v in over.items():
        setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("field,value,status", [
    ("n_mics", 0, binding.SONAR_E_INVALID),
    ("n_dirs", 0, binding.SONAR_E_INVALID),
    ("n_samples", 4, binding.SONAR_E_INVALID),        # N < L
    ("decim", 0, binding.SONAR_E_INVALID),
    ("max_frames", 0, binding.SONAR_E_INVALID),
    ("fs_hz", -1.0, binding.SONAR_E_INVALID),
    ("fft_len", 107, binding.SONAR_E_INVALID),        # odd (N + L - 1 = 107): not a valid length
    ("fft_len", 64, binding.SONAR_E_INVALID),         # below N + L - 1
    ("fft_len", 106, binding.SONAR_E_INVALID),        # even, but below N + L - 1
    ("fft_len", 108, binding.SONAR_E_UNSUPPORTED),    # valid (even, >= N + L - 1), not a power of two
    ("fft_len", 120, binding.SONAR_E_UNSUPPORTED),    # valid: 2^3 3 5, radices the library does not have
    ("fft_len", 1048576, binding.SONAR_E_UNSUPPORTED),  # above 2 x 16 x 16384
    ("gate_begin", 50, binding.SONAR_E_INVALID),      # gate_end 0 -> n0 >= n1
    ("lpf_len", 4, binding.SONAR_E_INVALID),          # even, and no taps
    ("bf_mode", 10, binding.SONAR_E_INVALID),
    ("sample_dtype", 9, binding.SONAR_E_INVALID),
])
def test_bad_descriptor_rejected_on_host(field, value, status):
    lib = binding.load()
    d, keep = _desc(**{field: value})
    h = ctypes.c_void_p()
    assert lib.sonar_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == status
    assert h.value is None
    assert len(lib.sonar_last_error()) > 0


@pytest.mark.parametrize("fft_len,band", [
    (131072, (0.0, 0.0)),        # 65537 stored bins: 16384-point phases, 5 bins folded per slot (beam window path)
    (131072, (20e3, 85e3)),      # the stress size: two bins per slot, fused inverse + envelope
    (524288, (0.0, 0.0)),        # the largest transform
])
def test_frequency_domain_sizes_pass_host_validation(fft_len, band):
    """Frequency-domain plans of any supported FFT length pass the host-side checks: without a
    device here, creation stops at the first HIP call (SONAR_E_HIP), not at a size refusal."""
    lib = binding.load()
    d, keep = _desc(fft_len=fft_len, bf_mode=binding.BF_MODES["fd_fp32"], band_lo_hz=band[0], band_hi_hz=band[1])
    h = ctypes.c_void_p()
    assert lib.sonar_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == binding.SONAR_E_HIP
    assert b"hipGetDevice" in lib.sonar_last_error()


def test_multi_and_tuned_reject_bad_arguments_on_host():
    lib = binding.load()
    assert lib.sonar_energyscape_multi(None, None, None, None, 0, None) == binding.SONAR_OK   # nothing to do
    assert lib.sonar_energyscape_multi(None, None, None, None, 2, None) == binding.SONAR_E_INVALID
    assert lib.sonar_energyscape_multi(None, None, None, None, -1, None) == binding.SONAR_E_INVALID
    d, keep = _desc()
    h = ctypes.c_void_p()
    m = ctypes.c_int32()
    assert lib.sonar_plan_create_tuned(ctypes.byref(d), 7, None, ctypes.byref(h), ctypes.byref(m)) == \
        binding.SONAR_E_INVALID
    assert lib.sonar_plan_create_tuned(None, 0, None, ctypes.byref(h), None) == binding.SONAR_E_INVALID


def test_non_unit_direction_rejected():
    lib = binding.load()
    d, keep = _desc()
    bad = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.81]])
    keep.append(bad)
    d.dirs = bad.ctypes.data_as(binding._dp)
    h = ctypes.c_void_p()
    assert lib.sonar_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == binding.SONAR_E_INVALID
    assert b"unit" in lib.sonar_last_error()


def test_null_arguments_rejected():
    lib = binding.load()
    h = ctypes.c_void_p()
    assert lib.sonar_plan_create(None, None, ctypes.byref(h)) == binding.SONAR_E_INVALID
    v = ctypes.c_int64()
    assert lib.sonar_plan_query(None, 0, ctypes.byref(v)) == binding.SONAR_E_INVALID
    assert lib.sonar_energyscape_batch(None, None, 1, None, None) == binding.SONAR_E_INVALID
    assert lib.sonar_plan_destroy(None) == 0
    assert lib.sonar_plan_enable_gradients(None) == binding.SONAR_E_INVALID
    assert lib.sonar_energyscape_vjp(None, None, None, None, 1, None, None, None, None) == binding.SONAR_E_INVALID
    assert lib.sonar_plan_set_positions(None, None, None) == binding.SONAR_E_INVALID
    assert lib.sonar_pdm_create(None, None, None) == binding.SONAR_E_INVALID
    assert lib.sonar_pdm_demodulate(None, None, 1, None, None) == binding.SONAR_E_INVALID
    assert lib.sonar_pdm_destroy(None) == binding.SONAR_OK
    assert lib.sonar_plan_set_envelope_iir(None, 2, None, None) == binding.SONAR_E_INVALID
    assert lib.sonar_energyscape_backward(None, None, None, 1, None, None, None) == binding.SONAR_E_INVALID


@pytest.mark.parametrize("field,value,status", [
    ("n_mics", 0, -1), ("n_mics", 129, -1), ("n_out", 0, -1), ("decim", 0, -1), ("max_frames", 0, -1),
    ("n_taps", 4, -1),            # even length: not zero-phase
    ("n_taps", 515, -4),          # above the supported length
])
def test_bad_pdm_descriptor_rejected_on_host(field, value, status):
    lib = binding.load()
    d = binding.PdmDesc(n_mics=32, n_out=1024, decim=10, n_taps=0, taps=None, max_frames=1)
    keep = None
    if field == "n_taps":
        keep = np.ones(value)
        d.n_taps, d.taps = value, keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    else:
        setattr(d, field, value)
    h = ctypes.c_void_p()
    assert lib.sonar_pdm_create(ctypes.byref(d), None, ctypes.byref(h)) == status
    assert h.value is None


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2208_10839_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                with open(os.path.join(dirpath, fn)) as f:
                    src = f.read()
                assert "import oracle" not in src and "from oracle" not in src, fn
                assert "oracle/" not in src, fn
