"""Named workloads (sizes, geometries, kernels, tolerances).

Each entry is data only: the point cloud comes from `points.py`, the kernel is
named by kind plus diagonal value and diagonal shift, and the tolerances are
the input compression tolerance and the product tolerance.
"""

from dataclasses import dataclass, field

import numpy as np

from . import points as P


@dataclass(frozen=True)
class KernelSpec:
    kind: str  # "laplace_4pi" = 1/(4 pi r), "inv_dist" = 1/r, "exp" = exp(-r)
    diag: float = 1.0  # value used for the i == j entry
    shift: float = 0.0  # added to every diagonal entry (B = K + shift * I)


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    geometry: str  # "sphere", "ellipsoid", "cube"
    leaf: int
    eta: float
    kernel_a: KernelSpec
    kernel_b: KernelSpec
    eps_in: float
    eps: float
    jitter: float = 0.0
    seed: int = 0
    axes: tuple = (1.0, 0.7, 0.5)
    split: int = 0  # 0 = bounding-box midpoint bisection, 1 = median
    same_ab: bool = False
    extra: dict = field(default_factory=dict)

    def points(self) -> np.ndarray:
        if self.geometry == "sphere":
            p = P.fibonacci_sphere(self.n)
        elif self.geometry == "ellipsoid":
            p = P.ellipsoid(self.n, self.axes)
        elif self.geometry == "cube":
            p = P.cube_surface(self.n, self.seed)
        else:
            raise ValueError(self.geometry)
        if self.jitter > 0.0:
            p = P.jitter(p, self.jitter, self.seed)
        return p


LAPLACE = KernelSpec("laplace_4pi", 1.0, 0.0)
EXP_PLUS_I = KernelSpec("exp", 1.0, 1.0)

CONFIGS = {
    # n = 2048 sphere, A = B = 1/(4 pi r) with unit diagonal, leaf 32.
    "sphere2k": Workload("sphere2k", 2048, "sphere", 32, 0.8, LAPLACE, LAPLACE, 1e-8, 1e-6,
                         same_ab=True),
    # n = 65536 jittered sphere, A = 1/(4 pi r), B = exp(-r) + I, leaf 64.
    "sphere64k": Workload("sphere64k", 65536, "sphere", 64, 0.8, LAPLACE, EXP_PLUS_I, 1e-8, 1e-6,
                          jitter=1e-3),
    # n = 262144 ellipsoid (1, 0.7, 0.5), kernels as sphere64k.
    "ellipsoid256k": Workload("ellipsoid256k", 262144, "ellipsoid", 64, 0.8, LAPLACE, EXP_PLUS_I,
                              1e-8, 1e-6, jitter=1e-3),
    # n = 262144 jittered sphere, kernels as sphere64k (the headline workload).
    "sphere256k": Workload("sphere256k", 262144, "sphere", 64, 0.8, LAPLACE, EXP_PLUS_I, 1e-8, 1e-6,
                           jitter=1e-3),
}
