"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package holds no arithmetic of the reconstruction method itself: it only
fixes the scanner/workload parameters and draws the random quantities (ellipse
phantoms, standard-normal noise vectors, request streams).  Everything that
turns these into a system matrix, a sinogram or a solution lives either in the
oracle or in the HIP library, each written independently.
"""
from .workloads import SCANNER, Workload, WORKLOADS, get_workload  # noqa: F401
from .phantom import (  # noqa: F401
    ellipse_params, phantom_image, phantom_batch, noise_vector, noise_batch,
    NOISE_REL_LEVEL, request_stream,
)
