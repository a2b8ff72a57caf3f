"""Kernel-matrix entries of the synthetic workloads (oracle).

Entries are indexed by original point index. Off the diagonal the entry is the
kernel of the distance r = ||x_i - x_j||_2 (evaluated as sqrt(dx*dx+dy*dy+dz*dz)):
  laplace_4pi: 1 / (4 pi r)
  inv_dist:    1 / r
  exp:         exp(-r)
On the diagonal it is `diag + shift`.
"""

import math

import numpy as np


def kernel_block(points: np.ndarray, rows: np.ndarray, cols: np.ndarray, kind: str,
                 diag: float = 1.0, shift: float = 0.0) -> np.ndarray:
    """Dense block K[rows, cols] (rows/cols are arrays of original point indices)."""
    x = points[rows]
    y = points[cols]
    dx = x[:, None, 0] - y[None, :, 0]
    dy = x[:, None, 1] - y[None, :, 1]
    dz = x[:, None, 2] - y[None, :, 2]
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    same = rows[:, None] == cols[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        if kind == "laplace_4pi":
            k = 1.0 / (4.0 * math.pi * r)
        elif kind == "inv_dist":
            k = 1.0 / r
        elif kind == "exp":
            k = np.exp(-r)
        else:
            raise ValueError(kind)
    return np.where(same, diag + shift, k)


def kernel_matrix(points: np.ndarray, kind: str, diag: float = 1.0, shift: float = 0.0) -> np.ndarray:
    idx = np.arange(points.shape[0])
    return kernel_block(points, idx, idx, kind, diag, shift)
