"""Exact product blocks, best approximation and acceptance (oracle).

What the product path must compute has a plain definition: for every farfield
leaf tau x sigma of the block-cluster tree, the best approximation at relative
Frobenius tolerance eps of the exact block (A_H B_H)[tau, sigma] (the epsilon-rank
notion of the numerical-examples section; Eckart-Young gives the optimum), and
for every nearfield leaf the exact block itself (evaluate() in Algorithm 4).

Two ways of getting exact blocks, both written out from that definition:
  * brute force: densify A_H and B_H, one GEMM (small n only);
  * strips: D[tau, sigma] = A_H[tau, :] @ B_H[:, sigma] with both strips densified
    (any n; used on sampled blocks).
"""

from dataclasses import dataclass

import numpy as np

from .assemble import eps_rank, truncate
from .hmatrix import HMatrix, KIND_F


class StripIndex:
    """Vectorised leaf lookup for strip densification of large H-matrices."""

    def __init__(self, H: HMatrix):
        self.H = H
        self.r0 = np.array([b.r0 for b in H.leaves], dtype=np.int64)
        self.r1 = self.r0 + np.array([b.m for b in H.leaves], dtype=np.int64)
        self.c0 = np.array([b.c0 for b in H.leaves], dtype=np.int64)
        self.c1 = self.c0 + np.array([b.n for b in H.leaves], dtype=np.int64)

    def row_strip(self, a: int, b: int) -> np.ndarray:
        S = np.zeros((b - a, self.H.n))
        for i in np.nonzero((self.r0 < b) & (self.r1 > a))[0]:
            lf = self.H.leaves[i]
            lo, hi = max(a, lf.r0), min(b, lf.r0 + lf.m)
            if lf.kind == KIND_F:
                S[lo - a:hi - a, lf.c0:lf.c0 + lf.n] = lf.L[lo - lf.r0:hi - lf.r0] @ lf.R.T
            else:
                S[lo - a:hi - a, lf.c0:lf.c0 + lf.n] = lf.D[lo - lf.r0:hi - lf.r0]
        return S

    def col_strip(self, a: int, b: int) -> np.ndarray:
        S = np.zeros((self.H.n, b - a))
        for i in np.nonzero((self.c0 < b) & (self.c1 > a))[0]:
            lf = self.H.leaves[i]
            lo, hi = max(a, lf.c0), min(b, lf.c0 + lf.n)
            if lf.kind == KIND_F:
                S[lf.r0:lf.r0 + lf.m, lo - a:hi - a] = lf.L @ lf.R[lo - lf.c0:hi - lf.c0].T
            else:
                S[lf.r0:lf.r0 + lf.m, lo - a:hi - a] = lf.D[:, lo - lf.c0:hi - lf.c0]
        return S


def exact_block_strips(ia: StripIndex, ib: StripIndex, r0, m, c0, n) -> np.ndarray:
    """(A_H B_H)[r0:r0+m, c0:c0+n] = A_H[rows, :] @ B_H[:, cols]."""
    return ia.row_strip(r0, r0 + m) @ ib.col_strip(c0, c0 + n)


def brute_force_product(A: HMatrix, B: HMatrix) -> np.ndarray:
    """Dense A_H @ B_H in cluster order."""
    return A.to_dense(1) @ B.to_dense(1)


def best_approximation(D: np.ndarray, eps: float):
    """Eckart-Young best approximation of D at relative Frobenius tolerance eps."""
    return truncate(D, eps)


@dataclass
class BlockCheck:
    kind: int
    err: float  # relative Frobenius error of the candidate
    rank: int  # candidate rank (farfield)
    kstar: int  # oracle's epsilon-rank (farfield)
    ok: bool


def check_block(D: np.ndarray, kind: int, eps: float, U=None, V=None, Dc=None,
                err_factor: float = 1.01, rank_slack: int = 2, near_tol: float = 1e-12) -> BlockCheck:
    """Acceptance of one candidate block against the exact block D.

    Farfield: ||D - U V^T||_F <= err_factor * eps * ||D||_F and
              rank <= k* + rank_slack, with k* the epsilon-rank of D.
    Nearfield: ||D - Dc||_F <= near_tol * ||D||_F.
    """
    nd = float(np.linalg.norm(D))
    if kind == KIND_F:
        s = np.linalg.svd(D, compute_uv=False) if D.size else np.zeros(0)
        kstar = eps_rank(s, eps)
        approx = U @ V.T if U.shape[1] else np.zeros_like(D)
        e = float(np.linalg.norm(D - approx))
        rel = e / nd if nd > 0 else (0.0 if e == 0.0 else np.inf)
        ok = (e <= err_factor * eps * nd) and (U.shape[1] <= kstar + rank_slack)
        return BlockCheck(kind, rel, U.shape[1], kstar, ok)
    e = float(np.linalg.norm(D - Dc))
    rel = e / nd if nd > 0 else (0.0 if e == 0.0 else np.inf)
    return BlockCheck(kind, rel, -1, -1, e <= near_tol * nd or e == 0.0)


def blockwise_best_product(A: HMatrix, B: HMatrix, eps: float) -> HMatrix:
    """The whole target: blockwise best approximation of A_H B_H on B's partition
    (brute force; small n)."""
    D = brute_force_product(A, B)
    C = HMatrix(n=A.n, perm=A.perm.copy())
    from .hmatrix import Leaf, KIND_N  # local import keeps the public surface small
    for lf in B.leaves:
        blk = D[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
        if lf.kind == KIND_F:
            L, R, _, _ = truncate(blk, eps)
            C.leaves.append(Leaf(lf.r0, lf.m, lf.c0, lf.n, KIND_F, L=L, R=R, level=lf.level))
        else:
            C.leaves.append(Leaf(lf.r0, lf.m, lf.c0, lf.n, KIND_N, D=blk.copy(), level=lf.level))
    return C


def global_error_estimate(C: HMatrix, A: HMatrix, B: HMatrix, iters: int = 10, size: int = 100,
                          seed: int = 0):
    """Frobenius-norm estimate of C - A B by subspace iteration on
    v -> C v - A (B v) (the error estimator of the numerical-examples section).
    Returns (estimate of ||C - AB||_F, estimate of ||AB||_F)."""
    rng = np.random.default_rng(seed)
    n = A.n
    size = min(size, n)

    def err_op(X):
        return C.matvec(X) - A.matvec(B.matvec(X))

    def err_opT(X):
        return C.rmatvec(X) - B.rmatvec(A.rmatvec(X))

    X = rng.standard_normal((n, size))
    for _ in range(iters):
        Y, _ = np.linalg.qr(err_op(X))
        X, _ = np.linalg.qr(err_opT(Y))
    Y = err_op(X)
    est_err = float(np.linalg.norm(Y))
    Xp = rng.standard_normal((n, size))
    for _ in range(iters):
        Yp, _ = np.linalg.qr(A.matvec(B.matvec(Xp)))
        Xp, _ = np.linalg.qr(B.rmatvec(A.rmatvec(Yp)))
    est_norm = float(np.linalg.norm(A.matvec(B.matvec(Xp))))
    return est_err, est_norm


def subspace_frobenius(op, opT, X0, iters):
    """Frobenius-norm estimate of an operator E given through op(X) = E X and
    opT(Y) = E^T Y: subspace iteration from the start block X0 (n x p),
    Y = orth(E X), X = orth(E^T Y), repeated `iters` times, then ||E X||_F. With
    orthonormal X this is the norm of E on the p-dimensional subspace that the
    iteration converges to (its dominant right singular subspace), the
    estimator of the numerical-examples section. Orthonormalization is a thin QR."""
    X = np.linalg.qr(np.asarray(X0, dtype=np.float64))[0]
    for _ in range(iters):
        Y = np.linalg.qr(op(X))[0]
        X = np.linalg.qr(opT(Y))[0]
    return float(np.linalg.norm(op(X)))


def product_error_estimate(C: HMatrix, A: HMatrix, B: HMatrix, X0, iters: int):
    """(estimate of ||C - A B||_F, estimate of ||A B||_F) by subspace_frobenius
    on v -> C v - A (B v) and on v -> A (B v), both from the start block X0
    (cluster order)."""
    err = subspace_frobenius(lambda X: C.matvec(X) - A.matvec(B.matvec(X)),
                             lambda Y: C.rmatvec(Y) - B.rmatvec(A.rmatvec(Y)), X0, iters)
    nrm = subspace_frobenius(lambda X: A.matvec(B.matvec(X)), lambda Y: B.rmatvec(A.rmatvec(Y)), X0, iters)
    return err, nrm


class LeafStrips:
    """Strip densification from an arbitrary source of leaves: arrays of the
    leaves' row/column ranges and a callable returning a leaf's dense block.
    Used on large H-matrices where only the leaves a strip touches are fetched."""

    def __init__(self, n, r0, r1, c0, c1, get_dense):
        self.n = n
        self.r0, self.r1, self.c0, self.c1 = (np.asarray(a, dtype=np.int64) for a in (r0, r1, c0, c1))
        self.get = get_dense
        self.cache = {}

    def leaf(self, i):
        if i not in self.cache:
            self.cache[i] = self.get(int(i))
        return self.cache[i]

    def rows_needed(self, a, b):
        return np.nonzero((self.r0 < b) & (self.r1 > a))[0]

    def cols_needed(self, a, b):
        return np.nonzero((self.c0 < b) & (self.c1 > a))[0]

    def row_strip(self, a, b):
        S = np.zeros((b - a, self.n))
        for i in self.rows_needed(a, b):
            D = self.leaf(i)
            lo, hi = max(a, self.r0[i]), min(b, self.r1[i])
            S[lo - a:hi - a, self.c0[i]:self.c1[i]] = D[lo - self.r0[i]:hi - self.r0[i]]
        return S

    def col_strip(self, a, b):
        S = np.zeros((self.n, b - a))
        for i in self.cols_needed(a, b):
            D = self.leaf(i)
            lo, hi = max(a, self.c0[i]), min(b, self.c1[i])
            S[self.r0[i]:self.r1[i], lo - a:hi - a] = D[:, lo - self.c0[i]:hi - self.c0[i]]
        return S


def exact_block_chunked(sa: LeafStrips, sb: LeafStrips, r0, r1, c0, c1, chunk=8192):
    """(A_H B_H)[r0:r1, c0:c1] = sum over column ranges K of A_H[rows, K] @ B_H[K, cols]:
    the strip product of exact_block_strips with the inner dimension taken in pieces of
    `chunk`, so that host memory stays at (r1 - r0 + c1 - c0) * chunk doubles."""
    m, n = r1 - r0, c1 - c0
    D = np.zeros((m, n))
    rows = sa.rows_needed(r0, r1)
    cols = sb.cols_needed(c0, c1)
    for k0 in range(0, sa.n, chunk):
        k1 = min(sa.n, k0 + chunk)
        As = np.zeros((m, k1 - k0))
        for i in rows[(sa.c0[rows] < k1) & (sa.c1[rows] > k0)]:
            L = sa.leaf(i)
            lo, hi = max(r0, sa.r0[i]), min(r1, sa.r1[i])
            cl, ch = max(k0, sa.c0[i]), min(k1, sa.c1[i])
            As[lo - r0:hi - r0, cl - k0:ch - k0] = L[lo - sa.r0[i]:hi - sa.r0[i], cl - sa.c0[i]:ch - sa.c0[i]]
        Bs = np.zeros((k1 - k0, n))
        for i in cols[(sb.r0[cols] < k1) & (sb.r1[cols] > k0)]:
            L = sb.leaf(i)
            rl, rh = max(k0, sb.r0[i]), min(k1, sb.r1[i])
            lo, hi = max(c0, sb.c0[i]), min(c1, sb.c1[i])
            Bs[rl - k0:rh - k0, lo - c0:hi - c0] = L[rl - sb.r0[i]:rh - sb.r0[i], lo - sb.c0[i]:hi - sb.c0[i]]
        D += As @ Bs
    return D


def oracle_block(sa: LeafStrips, sb: LeafStrips, r0, r1, c0, c1, kind, eps):
    """The oracle's answer for one leaf of the product: the exact block and, for a
    farfield leaf, its singular values and epsilon-rank (Eckart-Young)."""
    D = sa.row_strip(r0, r1) @ sb.col_strip(c0, c1)
    if kind == KIND_F:
        s = np.linalg.svd(D, compute_uv=False)
        return D, s, eps_rank(s, eps)
    return D, None, None
