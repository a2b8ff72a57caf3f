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


def leaf_source(H, tree, M):
    """LeafStrips over a library H-matrix, fetching leaves with hmat_block_get."""
    from oracle.product import LeafStrips
    cl = H.hmat_tree_clusters(tree)
    bl = H.hmat_tree_blocks(tree)
    n = H.hmat_tree_info(tree)["n"]
    leaf_ids = np.nonzero(bl["kind"] != 0)[0]
    t, s = bl["tau"][leaf_ids], bl["sigma"][leaf_ids]
    r0 = cl["begin"][t].astype(np.int64)
    c0 = cl["begin"][s].astype(np.int64)

    def get(i):
        d, U, V = H.hmat_block_get(M, i)
        return (U @ V.T) if d["kind"] == 1 else V

    src = LeafStrips(n, r0, r0 + cl["size"][t], c0, c0 + cl["size"][s], get)
    src.kind = bl["kind"][leaf_ids]
    src.level = bl["level"][leaf_ids]
    return src


def sampled_check(H, tree, A, B, C, eps, per_level=3, seed=0, max_rows=2048, largest_rows=0, log=print):
    """Checks a stratified sample of C's leaves (per level and kind, at most max_rows
    rows) against exact blocks A_H[tau, :] B_H[:, sigma] built from strips, plus, per
    level, the largest farfield leaf of at most `largest_rows` rows (0: none). Returns
    the list of (level, kind, rows, cols, err, rank, kstar, ok)."""
    from oracle.product import check_block, exact_block_chunked
    pa, pb, pc = leaf_source(H, tree, A), leaf_source(H, tree, B), leaf_source(H, tree, C)
    rng = np.random.default_rng(seed)
    rows = pc.r1 - pc.r0
    area = rows * (pc.c1 - pc.c0)
    out = []
    for L in np.unique(pc.level):
        for kind in (1, 2):
            cand = np.nonzero((pc.level == L) & (pc.kind == kind) & (rows <= max_rows))[0]
            pick = list(rng.choice(cand, min(per_level, cand.size), replace=False)) if cand.size else []
            if kind == 1 and largest_rows:
                big = np.nonzero((pc.level == L) & (pc.kind == 1) & (rows <= largest_rows))[0]
                if big.size:
                    j = int(big[np.argmax(area[big])])
                    if j not in pick:
                        pick.append(j)
            for i in pick:
                r0, r1, c0, c1 = pc.r0[i], pc.r1[i], pc.c0[i], pc.c1[i]
                D = exact_block_chunked(pa, pb, r0, r1, c0, c1)
                d, U, V = H.hmat_block_get(C, int(i))
                if kind == 1:
                    r = check_block(D, 1, eps, U=U, V=V)
                else:
                    r = check_block(D, 2, eps, Dc=V)
                out.append((int(L), kind, int(r1 - r0), int(c1 - c0), r.err, r.rank, r.kstar, r.ok))
                log(f"  level {L} kind {kind} {r1 - r0}x{c1 - c0}: err {r.err:.3e} rank {r.rank} k* {r.kstar} "
                    f"{'ok' if r.ok else 'FAIL'}")
    # leaves fetched for the strips are cached per source; free them
    for src in (pa, pb, pc):
        src.cache.clear()
    return out
