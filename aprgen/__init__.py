"""Seeded synthetic inputs for APR convolution: sphere-field images and the
particle cells of their Adaptive Particle Representation.

This package only *produces inputs* (particle cells, particle values, and the
LinearAccess arrays that encode them).  It holds none of the convolution
method's arithmetic: no tree fill, no patch reconstruction, no stencils.  Both
the FP64 oracle and the HIP path consume what it emits.
"""
from .apr_input import (AprInput, SphereConfig, CONFIGS, random_apr,
                        sphere_apr, encode_cells, level_dims, lmax_for)

__all__ = ["AprInput", "SphereConfig", "CONFIGS", "random_apr", "sphere_apr",
           "encode_cells", "level_dims", "lmax_for"]
