"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only generates inputs (meshes and random vectors).  It holds none
of the boundary element method's arithmetic, and neither the oracle nor the HIP
library imports the other through it.
"""
from .meshes import (octa_sphere, ellipsoid, perturbed_sphere, flat_plate,
                     single_pair, random_vector, real_sph_harm)

__all__ = ["octa_sphere", "ellipsoid", "perturbed_sphere", "flat_plate",
           "single_pair", "random_vector", "real_sph_harm"]
