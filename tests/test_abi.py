"""Host-side checks of the C ABI (no GPU needed): every declared symbol is
exported, argument errors are reported, and the library's trees are identical
to the oracle's (permutation, clusters, blocks and their kinds)."""

import os
import re

import numpy as np
import pytest

from workloads import fibonacci_sphere, cube_surface, ellipsoid, jitter
from oracle.tree import build_cluster_tree, build_block_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


def test_header_symbols_exported(H):
    hdr = open(os.path.join(ROOT, "include", "hmat.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(hmat_[a-z_0-9]+)\s*\(", hdr))
    assert len(declared) >= 25
    import ctypes
    L = ctypes.CDLL(H.LIB_PATH)
    missing = [s for s in declared if not hasattr(L, s)]
    assert not missing, missing
    assert declared == set(H.exported_symbols())


def test_argument_errors(H):
    pts = fibonacci_sphere(100)
    with pytest.raises(H.HmatError) as e:
        H.hmat_build_tree(pts, 0, 0.8)
    assert e.value.code == H.HMAT_ERR_ARG
    with pytest.raises(H.HmatError):
        H.hmat_build_tree(pts, 16, -1.0)
    bad = pts.copy()
    bad[3, 1] = np.nan
    with pytest.raises(H.HmatError):
        H.hmat_build_tree(bad, 16, 0.8)
    with pytest.raises(H.HmatError):
        H.hmat_build_tree(pts, 16, 0.8, split=7)


CASES = [
    ("sphere2k", lambda: fibonacci_sphere(2048), 32, 0),
    ("sphere2k-median", lambda: fibonacci_sphere(2048), 32, 1),
    ("jitter", lambda: jitter(fibonacci_sphere(6000), 1e-3, 0), 64, 0),
    ("cube", lambda: cube_surface(5000, 2), 40, 0),
    ("ellipsoid-median", lambda: ellipsoid(7000, (1.0, 0.45, 0.8)), 50, 1),
    ("tiny", lambda: fibonacci_sphere(5), 2, 0),
    ("single", lambda: fibonacci_sphere(1), 1, 0),
]


@pytest.mark.parametrize("name,gen,leaf,split", CASES, ids=[c[0] for c in CASES])
def test_tree_equals_oracle(H, name, gen, leaf, split):
    pts = gen()
    ct = build_cluster_tree(pts, leaf, split)
    bt = build_block_tree(ct, 0.8)
    t = H.hmat_build_tree(pts, leaf, 0.8, split)
    try:
        info = H.hmat_tree_info(t)
        assert info["n"] == len(pts) and info["n_clusters"] == ct.count
        assert info["n_blocks"] == bt.count and info["depth"] == bt.depth
        assert info["csp"] == bt.csp()
        assert np.array_equal(H.hmat_tree_perm(t), ct.perm)
        cl = H.hmat_tree_clusters(t)
        assert np.array_equal(cl["begin"], ct.begin) and np.array_equal(cl["size"], ct.size)
        assert np.array_equal(cl["parent"], ct.parent) and np.array_equal(cl["level"], ct.level)
        bl = H.hmat_tree_blocks(t)
        assert np.array_equal(bl["tau"], bt.tau) and np.array_equal(bl["sigma"], bt.sigma)
        assert np.array_equal(bl["kind"], bt.kind) and np.array_equal(bl["level"], bt.level)
    finally:
        H.hmat_tree_destroy(t)
