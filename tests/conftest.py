import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def small_case():
    """n = 2048 Fibonacci sphere, 1/(4 pi r) with unit diagonal, leaf 32, eta 0.8."""
    from workloads import fibonacci_sphere
    from oracle.tree import build_cluster_tree, build_block_tree
    from oracle.assemble import assemble

    pts = fibonacci_sphere(2048)
    ct = build_cluster_tree(pts, 32, 0)
    bt = build_block_tree(ct, 0.8)
    A = assemble(bt, pts, "laplace_4pi", 1.0, 0.0, 1e-8)
    return pts, ct, bt, A
