"""Cluster tree, admissibility and block-cluster tree (oracle).

Follows Section 2 of the paper: the tree definition (Def. 2.1), the cluster
tree (Def. 2.2), the admissibility condition (Def. 2.3) and the construction
of the block-cluster tree (Algorithm 1, BuildBlockClusterTree).

The paper leaves the cluster-tree construction and the concrete admissibility
condition open. Readings used here:
  * split 0 (bounding-box bisection): tight axis-aligned box of the cluster's
    points, longest edge (ties to the lowest axis), cut at its midpoint
    0.5*(lo+hi); points with coordinate <= mid go to the first son, keeping
    their order. Stop when #tau <= leaf size, when the box extent is zero, or
    when a son would be empty.
  * split 1 (median): along the same longest edge, stable sort by
    (coordinate, position); the first floor(#tau/2) form the first son.
  * diam(tau) = ||bmax - bmin||_2 of the tight box;
    dist(tau, sigma) = || max(0, bmin_s - bmax_t, bmin_t - bmax_s) ||_2;
    adm <=> dist > 0 and max(diam tau, diam sigma) <= eta * dist.
  * Algorithm 1 prints the sons as sigma' x tau'; they are read as tau' x sigma'
    (tau-son major order).
Norms are evaluated as sqrt(x*x + y*y + z*z) with that association, in float64.
"""

import math
from dataclasses import dataclass

import numpy as np

KIND_INNER, KIND_F, KIND_N = 0, 1, 2


@dataclass
class ClusterTree:
    perm: np.ndarray  # perm[i] = original index of the point at cluster position i
    begin: np.ndarray  # per cluster, first position
    size: np.ndarray
    level: np.ndarray
    parent: np.ndarray
    children: list  # list of lists of cluster ids (empty for leaves)
    bmin: np.ndarray  # (nc, 3)
    bmax: np.ndarray

    @property
    def count(self):
        return len(self.begin)

    def is_leaf(self, c):
        return len(self.children[c]) == 0


def _norm3(v):
    return math.sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2])


def diam(ct: ClusterTree, c: int) -> float:
    d = ct.bmax[c] - ct.bmin[c]
    return _norm3((float(d[0]), float(d[1]), float(d[2])))


def dist(ct: ClusterTree, t: int, s: int) -> float:
    g = []
    for a in range(3):
        u = float(ct.bmin[s][a]) - float(ct.bmax[t][a])
        w = float(ct.bmin[t][a]) - float(ct.bmax[s][a])
        g.append(max(0.0, u, w))
    return _norm3(g)


def admissible(ct: ClusterTree, t: int, s: int, eta: float) -> bool:
    """Admissibility condition (Def. 2.3 reading above)."""
    d = dist(ct, t, s)
    if not d > 0.0:
        return False
    return max(diam(ct, t), diam(ct, s)) <= eta * d


def build_cluster_tree(points: np.ndarray, leaf_size: int, split: int = 0) -> ClusterTree:
    """Cluster tree by recursive bisection (Def. 2.2), breadth-first cluster ids."""
    pts = np.asarray(points, dtype=np.float64)
    n = pts.shape[0]
    perm = np.arange(n, dtype=np.int64)
    begin, size, level, parent, children, bmin, bmax = [], [], [], [], [], [], []

    def add(b, s, lev, par):
        idx = perm[b:b + s]
        p = pts[idx]
        begin.append(b)
        size.append(s)
        level.append(lev)
        parent.append(par)
        children.append([])
        bmin.append(p.min(axis=0))
        bmax.append(p.max(axis=0))
        return len(begin) - 1

    add(0, n, 0, -1)
    head = 0
    while head < len(begin):
        c = head
        head += 1
        s = size[c]
        if s <= leaf_size:
            continue
        ext = bmax[c] - bmin[c]
        axis = 0
        for a in (1, 2):
            if ext[a] > ext[axis]:
                axis = a
        if not ext[axis] > 0.0:
            continue
        b = begin[c]
        idx = perm[b:b + s].copy()
        coord = pts[idx, axis]
        if split == 0:
            mid = 0.5 * (float(bmin[c][axis]) + float(bmax[c][axis]))
            first = coord <= mid
            n1 = int(first.sum())
            if n1 == 0 or n1 == s:
                continue
            new = np.concatenate([idx[first], idx[~first]])
        elif split == 1:
            order = np.lexsort((np.arange(s), coord))  # by coordinate, then position
            new = idx[order]
            n1 = s // 2
        else:
            raise ValueError("split must be 0 or 1")
        perm[b:b + s] = new
        c1 = add(b, n1, level[c] + 1, c)
        c2 = add(b + n1, s - n1, level[c] + 1, c)
        children[c] = [c1, c2]

    return ClusterTree(
        perm=perm,
        begin=np.asarray(begin, dtype=np.int64),
        size=np.asarray(size, dtype=np.int64),
        level=np.asarray(level, dtype=np.int64),
        parent=np.asarray(parent, dtype=np.int64),
        children=children,
        bmin=np.asarray(bmin),
        bmax=np.asarray(bmax),
    )


@dataclass
class BlockTree:
    ct: ClusterTree
    eta: float
    tau: np.ndarray  # per block, row cluster id
    sigma: np.ndarray  # per block, column cluster id
    level: np.ndarray
    kind: np.ndarray  # KIND_INNER, KIND_F or KIND_N
    children: list  # list of lists of block ids
    lookup: dict  # (tau, sigma) -> block id

    @property
    def count(self):
        return len(self.tau)

    def leaves(self, kind=None):
        if kind is None:
            return [b for b in range(self.count) if self.kind[b] != KIND_INNER]
        return [b for b in range(self.count) if self.kind[b] == kind]

    @property
    def depth(self):
        return int(self.level.max())

    def csp(self) -> int:
        """Sparsity constant: max over clusters of the number of blocks it heads."""
        cnt = np.zeros(self.ct.count, dtype=np.int64)
        np.add.at(cnt, self.tau, 1)
        cnt2 = np.zeros(self.ct.count, dtype=np.int64)
        np.add.at(cnt2, self.sigma, 1)
        return int(max(cnt.max(), cnt2.max()))


def build_block_tree(ct: ClusterTree, eta: float) -> BlockTree:
    """Algorithm 1 (BuildBlockClusterTree) from the root I x I, breadth first."""
    tau, sigma, level, kind, children = [0], [0], [0], [KIND_INNER], [[]]
    head = 0
    while head < len(tau):
        b = head
        head += 1
        t, s = tau[b], sigma[b]
        if admissible(ct, t, s, eta):
            kind[b] = KIND_F
        elif ct.children[t] and ct.children[s]:
            kind[b] = KIND_INNER
            kids = []
            for t2 in ct.children[t]:
                for s2 in ct.children[s]:
                    tau.append(t2)
                    sigma.append(s2)
                    level.append(level[b] + 1)
                    kind.append(KIND_INNER)
                    children.append([])
                    kids.append(len(tau) - 1)
            children[b] = kids
        else:
            kind[b] = KIND_N
    lookup = {(tau[b], sigma[b]): b for b in range(len(tau))}
    return BlockTree(
        ct=ct,
        eta=eta,
        tau=np.asarray(tau, dtype=np.int64),
        sigma=np.asarray(sigma, dtype=np.int64),
        level=np.asarray(level, dtype=np.int64),
        kind=np.asarray(kind, dtype=np.int64),
        children=children,
        lookup=lookup,
    )
