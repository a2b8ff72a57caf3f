"""Seeded synthetic inputs shared by the library's tests, the bench and the oracle.

This package holds point clouds and workload descriptions only. It contains none
of the method's arithmetic (no trees, no kernels, no compression): both the HIP
library and the CPU oracle receive the same point arrays from here and do all
further work with their own code.
"""

from .points import (  # noqa: F401
    fibonacci_sphere,
    ellipsoid,
    cube_surface,
    jitter,
    batched_geometries,
)
from .configs import CONFIGS, Workload, KernelSpec  # noqa: F401
