"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle
checks.  This package simulates data (objects, PSFs, Poisson noise); it holds
none of the deconvolution arithmetic and imports neither the oracle nor the
HIP library."""
from .workloads import (  # noqa: F401
    Workload, rng_for, gaussian_psf, airy_psf, fringe_psf, blur_periodic,
    point_sources, sersic_image, config0, config1, config2, config3, config4,
    small_single, small_multi, small_boundary,
)
