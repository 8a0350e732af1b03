"""Seeded synthetic inputs for the DAS -> B-mode path.

This package is the only code shared by the FP64 oracle (``oracle/``) and the
HIP path (``paper_1811_01566_amd``).  It holds workload descriptions
(probe, transmit sequence, pixel grid, phantom recipe) and a forward acoustic
model that synthesises int16 RF channel data from point scatterers.  It holds
none of the beamforming, envelope or log-compression arithmetic: the
scattering simulation below is the data source that the paper's Ultrasound
Environment stands for (Sec. II-A), not the method.

The paper measured wire and cyst phantoms whose data are not available here;
the recipes in :mod:`phantom.configs` stand in for them with seeded synthetic
scatterer fields of the same kind.
"""

from .configs import (
    Workload,
    WORKLOADS,
    get_workload,
    tiny_stai,
    tiny_pwi,
)
from .synth import synth_rf, scatterers_for, point_echo_rf
from .taps import bandpass_taps, workload_taps

__all__ = [
    "bandpass_taps",
    "workload_taps",
    "Workload",
    "WORKLOADS",
    "get_workload",
    "tiny_stai",
    "tiny_pwi",
    "synth_rf",
    "scatterers_for",
    "point_echo_rf",
]
