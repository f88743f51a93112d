"""Seeded synthetic inputs for parallel-beam CT reconstruction.

This package generates phantoms, exact analytic sinograms and noise. It holds
none of the reconstruction method's arithmetic (no system matrix, no TV, no
conjugate gradient): both the FP64 oracle and the HIP path take their inputs
from here, so neither depends on the other.
"""
from .phantom import (  # noqa: F401
    Ellipse,
    geometry_angles,
    bin_centres,
    random_ellipses,
    texture_disks,
    analytic_sinogram,
    rasterize,
    add_gaussian_noise,
    add_poisson_like_noise,
    default_bins,
)
from .workloads import Workload, make_workload, CONFIGS  # noqa: F401
