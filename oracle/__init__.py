"""FP64 CPU oracle for the DAS -> envelope -> log-compression -> B-mode path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
implementation (``paper_1811_01566_amd``); both consume inputs made by the
seeded generators in ``phantom/``.

The paper (WaveFlow, arXiv 1811.01566) names the pipeline - Delay-and-Sum
beamforming for STAI and PWI (Sec. II-B), analytic signal via the FFT-based
Hilbert transform and its absolute value (Sec. II-B; Fig. 2), dynamic range
clipping in dB (Fig. 2; Sec. III), the FIR pre-filter (Sec. II-B) and the
windowed moments feeding the qUS estimator (Fig. 3) - but prints no
equation.  Each function
below is the plain textbook definition of the named step, written in float64
with no blocking, fusion or reordering; every point the paper leaves open is
a stated reading (geometry, time origin, interpolation, apodisation, FFT
length, dB reference).

Pins (see ``tests/test_oracle_pins.py``): closed-form times of flight, the
sign/offset convention of plane-wave transmits, constant and linear-ramp RF
with closed-form sums, a point scatterer focusing at its pixel, linearity,
mirror symmetry, STAI reciprocity, brute-force scalar loops on tiny grids,
the envelope of a cosine / Gaussian-modulated pulse / constant and the
scipy Hilbert routine, closed-form dB values, the FIR's impulse response,
moving-average tone gain and edge sums, and closed-form window moments of
constant, ramp and Rayleigh envelopes.  No part is "parity
unpinned" except agreement with the paper's own images, which it does not
print.
"""

from .das import (
    element_positions,
    pixel_positions,
    tof_receive,
    tof_stai_transmit,
    tof_pwi_transmit,
    pwi_time_offset,
    fractional_index,
    interp_linear,
    receive_weight,
    das_sum,
    das_stai,
    das_pwi,
    das_workload,
    workload_tof,
)
from .adjoint import (
    das_adjoint_sum,
    das_dydc_sum,
    das_adjoint_workload,
    das_dydc_workload,
)
from .analytic import hilbert_multiplier, analytic_signal, envelope
from .dbclip import log_compress, bmode
from .fir import fir_same
from .moments import moment_map_shape, moment_maps

__all__ = [
    "element_positions", "pixel_positions", "tof_receive", "tof_stai_transmit",
    "tof_pwi_transmit", "pwi_time_offset", "fractional_index", "interp_linear",
    "receive_weight", "das_sum", "das_stai", "das_pwi", "das_workload", "workload_tof",
    "hilbert_multiplier", "analytic_signal", "envelope", "log_compress", "bmode",
    "das_adjoint_sum", "das_dydc_sum", "das_adjoint_workload", "das_dydc_workload",
    "fir_same", "moment_map_shape", "moment_maps",
]
