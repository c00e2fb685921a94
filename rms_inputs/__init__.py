"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only builds inputs: label volumes (x fastest in memory, stored as
numpy arrays of shape [nz, ny, nx]), gradient waveforms and direction sets.
It holds none of the walk's arithmetic and imports neither the oracle nor the
GPU library.
"""
from .substrates import (uniform_volume, cylinder_z, slab_x, cube_cell, sphere_cell,
                         ellipsoid_packing, axon_bundle)
from .protocols import pgse, ogse_cos, six_dirs, fibonacci_hemisphere
from . import configs

__all__ = ["uniform_volume", "cylinder_z", "slab_x", "cube_cell", "sphere_cell",
           "ellipsoid_packing", "axon_bundle", "pgse", "ogse_cos", "six_dirs",
           "fibonacci_hemisphere", "configs"]
