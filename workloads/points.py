"""Point-cloud generators for the synthetic kernel-matrix workloads.

The paper's experiments use Galerkin matrices on the unit sphere (numerical
examples section, exponential-kernel and single-layer examples). The meshes,
quadrature and assembly behind them are not available, so the workloads here
use collocation-style kernel matrices on points of closed surfaces instead:
the unit sphere, ellipsoids and the surface of the unit cube.

All generators return float64 arrays of shape (n, 3), row-major, and are fully
determined by their arguments (and the seed, where one is taken).
"""

import math

import numpy as np

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


def fibonacci_sphere(n: int) -> np.ndarray:
    """n points of a Fibonacci lattice on the unit sphere.

    z_i = 1 - (2i+1)/n, r_i = sqrt(1 - z_i^2), phi_i = i * pi * (3 - sqrt 5),
    x_i = (r_i cos phi_i, r_i sin phi_i, z_i), i = 0..n-1.
    """
    if n < 1:
        raise ValueError("n must be positive")
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * GOLDEN_ANGLE
    return np.ascontiguousarray(np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1))


def ellipsoid(n: int, axes=(1.0, 0.7, 0.5)) -> np.ndarray:
    """Fibonacci-sphere points scaled coordinate-wise by the ellipsoid's semi-axes."""
    p = fibonacci_sphere(n)
    return np.ascontiguousarray(p * np.asarray(axes, dtype=np.float64)[None, :])


def cube_surface(n: int, seed: int = 0) -> np.ndarray:
    """n points on the surface of [-1/2, 1/2]^3: a face drawn uniformly, then a
    point drawn uniformly in that face."""
    rng = np.random.default_rng(seed)
    face = rng.integers(0, 6, size=n)
    uv = rng.uniform(-0.5, 0.5, size=(n, 2))
    pts = np.empty((n, 3), dtype=np.float64)
    axis = face // 2
    sign = np.where(face % 2 == 0, -0.5, 0.5)
    for a in range(3):
        sel = axis == a
        others = [b for b in range(3) if b != a]
        pts[sel, a] = sign[sel]
        pts[sel, others[0]] = uv[sel, 0]
        pts[sel, others[1]] = uv[sel, 1]
    return pts


def jitter(points: np.ndarray, amplitude: float = 1e-3, seed: int = 0) -> np.ndarray:
    """Adds U(-amplitude, amplitude) to every coordinate (no re-projection)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(points + rng.uniform(-amplitude, amplitude, size=points.shape))


def batched_geometries(count: int = 64, n_lo: int = 4096, n_hi: int = 65536, seed: int = 0):
    """Draws `count` independent product workloads: n log-uniform in [n_lo, n_hi],
    a geometry from {sphere, ellipsoid with axes U[0.4, 1], cube surface} and a
    kernel pair from {1/r, exp(-r)}. Returns a list of dicts with the points and
    the kernel kinds of the two factors."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        geo = int(rng.integers(0, 3))
        if geo == 0:
            pts, name = fibonacci_sphere(n), "sphere"
        elif geo == 1:
            axes = tuple(float(a) for a in rng.uniform(0.4, 1.0, size=3))
            pts, name = ellipsoid(n, axes), "ellipsoid%.3f,%.3f,%.3f" % axes
        else:
            pts, name = cube_surface(n, seed=int(rng.integers(0, 2**31))), "cube"
        ka = ["inv_dist", "exp"][int(rng.integers(0, 2))]
        kb = ["inv_dist", "exp"][int(rng.integers(0, 2))]
        out.append({"n": n, "points": pts, "geometry": name, "kernel_a": ka, "kernel_b": kb})
    return out
