"""H-matrix container for the oracle (Section 2: low-rank set, H-matrix set,
block structure, H-matrix-vector product).

An H-matrix is held as its list of leaves. Index ranges are positions in the
cluster ordering (clusters are contiguous ranges of positions). A farfield leaf
stores M = L R^T with L (m x k) and R (n x k); a nearfield leaf stores M densely.
"""

from dataclasses import dataclass, field

import numpy as np

KIND_F, KIND_N = 1, 2


@dataclass
class Leaf:
    r0: int  # first row position
    m: int
    c0: int  # first column position
    n: int
    kind: int
    L: np.ndarray = None  # (m, k) for KIND_F
    R: np.ndarray = None  # (n, k) for KIND_F
    D: np.ndarray = None  # (m, n) for KIND_N
    level: int = 0

    @property
    def rank(self):
        return self.L.shape[1] if self.kind == KIND_F else None

    def dense(self) -> np.ndarray:
        if self.kind == KIND_F:
            return self.L @ self.R.T
        return self.D


@dataclass
class HMatrix:
    n: int
    perm: np.ndarray  # position -> original point index
    leaves: list = field(default_factory=list)

    def to_dense(self, order: int = 1) -> np.ndarray:
        """Dense n x n matrix; order 1 = cluster order, 0 = original point order."""
        M = np.zeros((self.n, self.n))
        for b in self.leaves:
            M[b.r0:b.r0 + b.m, b.c0:b.c0 + b.n] = b.dense()
        if order == 0:
            out = np.empty_like(M)
            out[np.ix_(self.perm, self.perm)] = M
            return out
        return M

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = H x (cluster order), visiting every leaf once as the recursion of
        Algorithm 2 does; x may be a matrix of several columns."""
        y = np.zeros((self.n,) + x.shape[1:])
        for b in self.leaves:
            xs = x[b.c0:b.c0 + b.n]
            if b.kind == KIND_F:
                y[b.r0:b.r0 + b.m] += b.L @ (b.R.T @ xs)
            else:
                y[b.r0:b.r0 + b.m] += b.D @ xs
        return y

    def rmatvec(self, x: np.ndarray) -> np.ndarray:
        """y = H^T x (cluster order)."""
        y = np.zeros((self.n,) + x.shape[1:])
        for b in self.leaves:
            xs = x[b.r0:b.r0 + b.m]
            if b.kind == KIND_F:
                y[b.c0:b.c0 + b.n] += b.R @ (b.L.T @ xs)
            else:
                y[b.c0:b.c0 + b.n] += b.D.T @ xs
        return y

    def row_strip(self, r0: int, r1: int) -> np.ndarray:
        """Dense rows [r0, r1) of H (cluster order), all n columns."""
        S = np.zeros((r1 - r0, self.n))
        for b in self.leaves:
            lo, hi = max(r0, b.r0), min(r1, b.r0 + b.m)
            if lo >= hi:
                continue
            if b.kind == KIND_F:
                S[lo - r0:hi - r0, b.c0:b.c0 + b.n] = b.L[lo - b.r0:hi - b.r0] @ b.R.T
            else:
                S[lo - r0:hi - r0, b.c0:b.c0 + b.n] = b.D[lo - b.r0:hi - b.r0]
        return S

    def col_strip(self, c0: int, c1: int) -> np.ndarray:
        """Dense columns [c0, c1) of H (cluster order), all n rows."""
        S = np.zeros((self.n, c1 - c0))
        for b in self.leaves:
            lo, hi = max(c0, b.c0), min(c1, b.c0 + b.n)
            if lo >= hi:
                continue
            if b.kind == KIND_F:
                S[b.r0:b.r0 + b.m, lo - c0:hi - c0] = b.L @ b.R[lo - b.c0:hi - b.c0].T
            else:
                S[b.r0:b.r0 + b.m, lo - c0:hi - c0] = b.D[:, lo - b.c0:hi - b.c0]
        return S

    def frob2(self) -> float:
        return float(sum(np.sum(b.dense() ** 2) for b in self.leaves))


def leaf_key(b: Leaf):
    return (b.r0, b.m, b.c0, b.n)
