"""Test helpers: conversion of the library's exported H-matrices into the
oracle's container (the oracle's only view of library results), and GPU
presence checks."""

import numpy as np

from oracle.hmatrix import HMatrix, Leaf, KIND_F, KIND_N


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def exported_to_oracle(H, tree, M):
    """Builds an oracle HMatrix from hmat_export of M (leaves in breadth-first order)."""
    info = H.hmat_tree_info(tree)
    perm = H.hmat_tree_perm(tree).astype(np.int64)
    cl = H.hmat_tree_clusters(tree)
    bl = H.hmat_tree_blocks(tree)
    ranks, offs, pool = H.hmat_export(M)
    leaves_ids = np.nonzero(bl["kind"] != 0)[0]
    out = HMatrix(n=info["n"], perm=perm)
    for i, b in enumerate(leaves_ids):
        t, s = bl["tau"][b], bl["sigma"][b]
        r0, m, c0, n = int(cl["begin"][t]), int(cl["size"][t]), int(cl["begin"][s]), int(cl["size"][s])
        o = int(offs[i])
        if bl["kind"][b] == 1:
            k = int(ranks[i])
            L = pool[o:o + m * k].reshape(k, m).T.copy()
            R = pool[o + m * k:o + m * k + n * k].reshape(k, n).T.copy()
            out.leaves.append(Leaf(r0, m, c0, n, KIND_F, L=L, R=R, level=int(bl["level"][b])))
        else:
            D = pool[o:o + m * n].reshape(n, m).T.copy()
            out.leaves.append(Leaf(r0, m, c0, n, KIND_N, D=D, level=int(bl["level"][b])))
    return out


def oracle_to_blocks(Hm: HMatrix):
    """(ranks, offsets, pool) of an oracle HMatrix for hmat_from_blocks (leaves in
    the order of Hm.leaves, which must be the library's breadth-first leaf order)."""
    ranks, offs, parts = [], [], []
    pos = 0
    for lf in Hm.leaves:
        offs.append(pos)
        if lf.kind == KIND_F:
            ranks.append(lf.L.shape[1])
            a = np.concatenate([lf.L.T.ravel(), lf.R.T.ravel()])
        else:
            ranks.append(0)
            a = lf.D.T.ravel()
        parts.append(a)
        pos += a.size
    pool = np.concatenate(parts) if parts else np.zeros(1)
    return np.array(ranks, dtype=np.int32), np.array(offs, dtype=np.int64), pool
