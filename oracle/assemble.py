"""Input compression by per-block truncated SVD (oracle).

Each farfield leaf of a kernel matrix is replaced by its best approximation at
relative Frobenius tolerance eps_in (Eckart-Young): the smallest k with
sqrt(sum_{i>k} s_i^2) <= eps_in * ||M||_F, stored as L = U_k diag(s_k), R = V_k.
Nearfield leaves are stored densely. This is the epsilon-rank notion of the
numerical-examples section, applied block by block.
"""

import numpy as np

from .hmatrix import HMatrix, Leaf, KIND_F, KIND_N
from .kernels import kernel_block
from .tree import BlockTree, KIND_F as T_F


def eps_rank(s: np.ndarray, eps: float) -> int:
    """Smallest k with tail_k = sqrt(sum_{i>=k} s_i^2) <= eps * ||s||_2 (k = 0 if
    the matrix is zero). `s` holds the singular values in decreasing order."""
    s = np.asarray(s, dtype=np.float64)
    total = float(np.sqrt(np.sum(s * s)))
    if total == 0.0:
        return 0
    # tail[k] = sqrt(sum_{i >= k} s_i^2), k = 0..len(s)
    sq = s * s
    tail = np.sqrt(np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]]))
    for k in range(len(s) + 1):
        if tail[k] <= eps * total:
            return k
    return len(s)


def truncate(M: np.ndarray, eps: float):
    """Best approximation of M at relative Frobenius tolerance eps: returns
    (L, R, s, k) with M ~= L R^T, L = U_k diag(s_k), R = V_k."""
    if M.size == 0:
        return np.zeros((M.shape[0], 0)), np.zeros((M.shape[1], 0)), np.zeros(0), 0
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    k = eps_rank(s, eps)
    return U[:, :k] * s[:k][None, :], Vt[:k].T.copy(), s, k


def assemble(bt: BlockTree, points: np.ndarray, kind: str, diag: float, shift: float,
             eps_in: float) -> HMatrix:
    ct = bt.ct
    H = HMatrix(n=points.shape[0], perm=ct.perm.copy())
    for b in bt.leaves():
        t, s = bt.tau[b], bt.sigma[b]
        r0, m, c0, n = int(ct.begin[t]), int(ct.size[t]), int(ct.begin[s]), int(ct.size[s])
        K = kernel_block(points, ct.perm[r0:r0 + m], ct.perm[c0:c0 + n], kind, diag, shift)
        if bt.kind[b] == T_F:
            L, R, _, _ = truncate(K, eps_in)
            H.leaves.append(Leaf(r0, m, c0, n, KIND_F, L=L, R=R, level=int(bt.level[b])))
        else:
            H.leaves.append(Leaf(r0, m, c0, n, KIND_N, D=K, level=int(bt.level[b])))
    return H
