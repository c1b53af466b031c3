"""FP64 CPU oracle of the eRTIS energyscape pipeline.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (``paper_2208_10839_amd``) never imports, calls or
links anything here, and nothing here imports the product path: the two share
no code.
"""

from .sonar_oracle import (  # noqa: F401
    analytic_weights,
    band_mask,
    beam_window_indices,
    butterworth_lowpass,
    chirp_spectrum_filter,
    das_fd,
    das_fd_vjp,
    das_td,
    das_td_cubic,
    das_td_cubic_vjp,
    das_td_nearest,
    das_td_vjp,
    default_lowpass,
    delays,
    delays_vjp,
    energyscape,
    energyscape_vjp_fd,
    energyscape_vjp_td,
    gridded_offsets,
    lagrange4_weight_slopes,
    lagrange4_weights,
    lfilter,
    envelope,
    envelope_iir,
    envelope_vjp,
    matched_filter,
    matched_filter_spectrum,
    matched_filter_spectrum_vjp,
    matched_filter_vjp,
    nearest_offsets,
    num_range_bins,
    pdm_default_taps,
    pdm_demodulate,
    pdm_unpack,
    td_offsets,
)
