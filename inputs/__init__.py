"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the imaging method: no DFT, no phase, no
operator, no thresholding.  It only draws random numbers (scene content,
sampling masks, noise) and records the radar parameter sets and workload
descriptions as plain numbers.  Both the FP64 oracle and the HIP path consume
what it produces; neither of them is imported here.
"""

from .params import (RADAR_STRIPMAP, RADAR_TABLE2_SIM, RADAR_LBAND_STRESS,
                      params_with)
from .scenes import (rng, random_complex, point_targets, targets_to_image,
                     sparse_field, extended_patches, random_mask,
                     circular_noise, batched_shapes)
from .workloads import WORKLOADS, workload, gradient_problem_parts

__all__ = [
    "RADAR_STRIPMAP", "RADAR_TABLE2_SIM", "RADAR_LBAND_STRESS", "params_with",
    "rng", "random_complex", "point_targets", "targets_to_image",
    "sparse_field", "extended_patches", "random_mask", "circular_noise",
    "batched_shapes", "WORKLOADS", "workload", "gradient_problem_parts",
]
