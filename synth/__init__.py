"""Seeded synthetic inputs for the ptychography loss + gradient path.

This package only *generates inputs*: objects, probes, scan positions,
detector-pad sizes, the tilted-plane resampling table and photon-count
sampling.  It holds none of the forward model, loss or gradient arithmetic,
so both the FP64 oracle (tests) and the HIP path (benchmarks) can draw the
same inputs from it without sharing any of the method's computation.

The workload recipes stand in for the paper's experimental dataset, which is
not available: see ``synth.configs`` for the five workloads.
"""

from .configs import WORKLOADS, Workload, get_workload, reduced
from .geometry import smooth_pad, pads_for, ratios_for, is_smooth7
from .fields import make_truth, make_start, sample_counts, synthetic_counts

__all__ = [
    "WORKLOADS", "Workload", "get_workload", "reduced",
    "smooth_pad", "pads_for", "ratios_for", "is_smooth7",
    "make_truth", "make_start", "sample_counts", "synthetic_counts",
]
