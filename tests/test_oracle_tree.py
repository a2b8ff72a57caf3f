"""Pins of the oracle's cluster tree, admissibility and block tree against the
definitions of Section 2 (Def. 2.1-2.3, Algorithm 1) and brute force."""

import itertools

import numpy as np
import pytest

from workloads import fibonacci_sphere, cube_surface, ellipsoid, jitter
from oracle.tree import (build_cluster_tree, build_block_tree, admissible, diam, dist,
                         KIND_F, KIND_N, KIND_INNER)


def test_fibonacci_points_on_sphere():
    p = fibonacci_sphere(1000)
    assert p.shape == (1000, 3)
    assert np.allclose(np.linalg.norm(p, axis=1), 1.0, atol=1e-14)
    # z is the closed form 1 - (2i+1)/n
    assert np.allclose(p[:, 2], 1.0 - (2 * np.arange(1000) + 1) / 1000.0)
    assert len(np.unique(np.round(p, 12), axis=0)) == 1000


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("gen", ["sphere", "cube", "ellipsoid"])
def test_cluster_tree_definition(split, gen):
    n = 3000
    pts = {"sphere": fibonacci_sphere(n), "cube": cube_surface(n, 3),
           "ellipsoid": jitter(ellipsoid(n), 1e-3, 1)}[gen]
    leaf = 40
    ct = build_cluster_tree(pts, leaf, split)
    # perm is a permutation; the root is I
    assert sorted(ct.perm.tolist()) == list(range(n))
    assert ct.begin[0] == 0 and ct.size[0] == n
    leaves = []
    for c in range(ct.count):
        assert ct.size[c] > 0  # Def. 2.2 (3): non-empty
        kids = ct.children[c]
        if not kids:
            leaves.append(c)
            assert ct.size[c] <= leaf or np.all(ct.bmax[c] == ct.bmin[c])
            continue
        # Def. 2.2 (2): disjoint union of the sons, contiguous ranges in order
        assert len(kids) == 2
        assert ct.begin[kids[0]] == ct.begin[c]
        assert ct.begin[kids[1]] == ct.begin[kids[0]] + ct.size[kids[0]]
        assert ct.size[kids[0]] + ct.size[kids[1]] == ct.size[c]
        for k in kids:
            assert ct.parent[k] == c and ct.level[k] == ct.level[c] + 1
        # tight bounding boxes
        p = pts[ct.perm[ct.begin[c]:ct.begin[c] + ct.size[c]]]
        assert np.array_equal(p.min(0), ct.bmin[c]) and np.array_equal(p.max(0), ct.bmax[c])
        ext = ct.bmax[c] - ct.bmin[c]
        ax = int(np.argmax(ext))  # first maximal axis
        p1 = pts[ct.perm[ct.begin[kids[0]]:ct.begin[kids[0]] + ct.size[kids[0]]], ax]
        p2 = pts[ct.perm[ct.begin[kids[1]]:ct.begin[kids[1]] + ct.size[kids[1]]], ax]
        if split == 0:
            mid = 0.5 * (ct.bmin[c][ax] + ct.bmax[c][ax])
            assert np.all(p1 <= mid) and np.all(p2 > mid)
        else:
            assert ct.size[kids[0]] == ct.size[c] // 2
            assert p1.max() <= p2.min()
    # leaves partition I
    cover = np.zeros(n, dtype=int)
    for c in leaves:
        cover[ct.begin[c]:ct.begin[c] + ct.size[c]] += 1
    assert np.all(cover == 1)


def _point_diam(p):
    d = p[:, None, :] - p[None, :, :]
    return np.sqrt((d ** 2).sum(-1)).max()


def _point_dist(p, q):
    d = p[:, None, :] - q[None, :, :]
    return np.sqrt((d ** 2).sum(-1)).min()


def test_admissibility_symmetric_monotone_and_geometric():
    pts = fibonacci_sphere(1500)
    ct = build_cluster_tree(pts, 24, 0)
    rng = np.random.default_rng(0)
    ids = rng.choice(ct.count, size=60, replace=False)
    for t, s in itertools.product(ids, ids):
        assert admissible(ct, t, s, 0.8) == admissible(ct, s, t, 0.8)
        if admissible(ct, t, s, 0.8):
            # box distance and diameter bound the point-set quantities
            pt = pts[ct.perm[ct.begin[t]:ct.begin[t] + ct.size[t]]]
            ps = pts[ct.perm[ct.begin[s]:ct.begin[s] + ct.size[s]]]
            assert _point_dist(pt, ps) >= dist(ct, t, s) - 1e-15
            assert max(_point_diam(pt), _point_diam(ps)) <= 0.8 * _point_dist(pt, ps) + 1e-15
            for t2 in ct.children[t]:
                for s2 in ct.children[s]:
                    assert admissible(ct, t2, s2, 0.8)  # Def. 2.3 monotone


@pytest.mark.parametrize("split", [0, 1])
def test_block_tree_partition(split):
    n = 2048
    pts = fibonacci_sphere(n)
    ct = build_cluster_tree(pts, 32, split)
    bt = build_block_tree(ct, 0.8)
    cover = np.zeros((n, n), dtype=np.int8)
    for b in range(bt.count):
        t, s = bt.tau[b], bt.sigma[b]
        assert bt.level[b] == ct.level[t] == ct.level[s]  # level-conserving
        if bt.kind[b] == KIND_F:
            assert admissible(ct, t, s, 0.8) and not bt.children[b]
        elif bt.kind[b] == KIND_N:
            assert not admissible(ct, t, s, 0.8) and not bt.children[b]
            assert not ct.children[t] or not ct.children[s]
        else:
            assert ct.children[t] and ct.children[s]
            assert [(bt.tau[c], bt.sigma[c]) for c in bt.children[b]] == \
                [(t2, s2) for t2 in ct.children[t] for s2 in ct.children[s]]
        if bt.kind[b] != KIND_INNER:
            cover[ct.begin[t]:ct.begin[t] + ct.size[t], ct.begin[s]:ct.begin[s] + ct.size[s]] += 1
    assert np.all(cover == 1)  # F and N leaves partition I x I


def test_block_tree_sizes_of_sphere2k():
    """The n = 2048 workload's tree (midpoint split, leaf 32, eta 0.8)."""
    pts = fibonacci_sphere(2048)
    ct = build_cluster_tree(pts, 32, 0)
    bt = build_block_tree(ct, 0.8)
    assert ct.count == 197
    assert (bt.kind == KIND_F).sum() == 3020 and (bt.kind == KIND_N).sum() == 2627
    assert bt.depth == 7 and bt.csp() == 64
