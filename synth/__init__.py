"""Seeded synthetic XPCS inputs shared by the oracle tests, the GPU tests and the bench.

This package only *makes inputs*: speckle photon-count frames and annular
q-ROI label maps.  It contains none of the method's arithmetic (no Gram
products, no decomposition, no correlation), so both the CPU oracle and the
HIP path can consume its output without sharing any computation.
"""

from .speckle import (  # noqa: F401
    SpeckleSpec,
    WORKLOADS,
    annular_labels,
    whole_detector_labels,
    split_tau_map,
    speckle_frames_numpy,
    speckle_frames_torch,
    low_rank_frames_numpy,
    workload_labels,
    workload_tau,
    seed_for,
)
