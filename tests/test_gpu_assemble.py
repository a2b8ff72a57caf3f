"""GPU assembly vs the oracle: every farfield block of the assembled kernel
matrix meets the input tolerance (relative Frobenius error <= 1.01 eps_in) with
rank <= the epsilon-rank + 2; nearfield blocks equal the kernel entries."""

import numpy as np
import pytest

from workloads import fibonacci_sphere, jitter
from oracle.kernels import kernel_block
from oracle.assemble import eps_rank
from tests.helpers import exported_to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


@pytest.mark.parametrize("kind,diag,shift,n,leaf", [
    ("laplace_4pi", 1.0, 0.0, 2048, 32),
    ("exp", 1.0, 1.0, 3000, 64),
    ("inv_dist", 1.0, 0.0, 1500, 20),
])
@pytest.mark.parametrize("budget", [0, 1 << 20])
def test_assembly_blocks(H, kind, diag, shift, n, leaf, budget):
    """budget 1 MB forces many assembly chunks (regression: chunk offsets)."""
    print(f"[assembly] kind={kind} n={n} leaf={leaf} budget={budget}", flush=True)
    pts = jitter(fibonacci_sphere(n), 1e-3, 0) if kind == "exp" else fibonacci_sphere(n)
    t = H.hmat_build_tree(pts, leaf, 0.8, 0)
    M, code = H.hmat_assemble(t, kind, diag, shift, 1e-8, opts=H.hmat_opts_default(workspace_limit=budget))
    Hm = exported_to_oracle(H, t, M)
    perm = Hm.perm
    worst, slack = 0.0, -99
    for lf in Hm.leaves:
        K = kernel_block(pts, perm[lf.r0:lf.r0 + lf.m], perm[lf.c0:lf.c0 + lf.n], kind, diag, shift)
        if lf.kind == 1:
            nk = np.linalg.norm(K)
            e = np.linalg.norm(K - lf.L @ lf.R.T) / nk
            kstar = eps_rank(np.linalg.svd(K, compute_uv=False), 1e-8)
            worst = max(worst, e)
            slack = max(slack, lf.L.shape[1] - kstar)
            assert e <= 1.01e-8, (lf.r0, lf.c0, e)
            assert lf.L.shape[1] <= kstar + 2
        else:
            assert np.allclose(lf.D, K, rtol=1e-14, atol=0)
    print(f"worst rel err {worst:.3e}, max rank - k* = {slack}")
    H.hmat_destroy(M)
    H.hmat_tree_destroy(t)
