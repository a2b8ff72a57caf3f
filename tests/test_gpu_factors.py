"""Structure of the product's farfield factors, which pins the orthogonalisation and the
core SVD of the randomized scheme (Section 4.3) through their outputs.

A farfield block of C is written as L R^T with L = Q W and R = Q_Z J, where
  Q    orthonormal basis of the sketch and probe columns (CGS2, k_orth_append),
  Q_Z  the Q factor of Z = S^T Q (CGS2 in k_core),
  W, J the one-sided Jacobi SVD of R_Z^T: R_Z^T J = W, with W's columns orthogonal and
       their norms the singular values, sorted descending and truncated to k columns.
So, for every farfield block:
  * R^T R = I_k;
  * L^T L is diagonal; its diagonal, sigma_j^2, descends;
  * sigma_j are the singular values of L R^T (LAPACK's SVD of the output);
  * Weyl's inequality bounds sigma_j against the singular values of the exact block D
    (the oracle's brute-force product): |sigma_j - s_j(D)| <= ||D - L R^T||_2.
A basis that lost orthogonality (one Gram-Schmidt pass instead of two), a Jacobi
iteration stopped early or a wrong sort order fails one of these."""

import ctypes

import numpy as np
import pytest

from oracle.hmatrix import KIND_F
from oracle.product import brute_force_product
from tests.helpers import exported_to_oracle
from workloads import fibonacci_sphere, jitter

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


@pytest.fixture(scope="module")
def case(H):
    pts = jitter(fibonacci_sphere(4096), 1e-3, seed=5)
    t = H.hmat_build_tree(pts, 32, 0.8, 0)
    A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-10)
    B, _ = H.hmat_assemble(t, "exp", 1.0, 1.0, eps_in=1e-10)
    P = brute_force_product(exported_to_oracle(H, t, A), exported_to_oracle(H, t, B))
    yield t, A, B, P
    H.hmat_destroy(A)
    H.hmat_destroy(B)
    H.hmat_tree_destroy(t)


@pytest.mark.parametrize("eps,exact", [(1e-6, 0), (1e-10, 0), (1e-6, 1)])
def test_farfield_factor_structure(H, case, eps, exact):
    t, A, B, P = case
    st = H.hmat_stats()
    o = H.hmat_opts_default()
    o.exact_lowrank = exact
    o.stats = ctypes.pointer(st)
    C, code = H.hmat_multiply(A, B, eps, o)
    assert code == 0
    Co = exported_to_oracle(H, t, C)
    H.hmat_destroy(C)
    orth_r = gram_l = sort_bad = sv_out = weyl = 0.0
    nblk = 0
    for lf in Co.leaves:
        if lf.kind != KIND_F or lf.L.shape[1] == 0:
            continue
        nblk += 1
        L, R = lf.L, lf.R
        k = L.shape[1]
        orth_r = max(orth_r, np.abs(R.T @ R - np.eye(k)).max())
        sig = np.linalg.norm(L, axis=0)
        assert sig.min() > 0.0
        G = (L.T @ L) / np.outer(sig, sig)
        gram_l = max(gram_l, np.abs(G - np.eye(k)).max())
        if k > 1:
            sort_bad = max(sort_bad, np.max(np.diff(sig)) / sig[0])
        s_out = np.linalg.svd(L @ R.T, compute_uv=False)[:k]
        sv_out = max(sv_out, np.abs(s_out - sig).max() / sig[0])
        D = P[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
        s_d = np.linalg.svd(D, compute_uv=False)
        e2 = np.linalg.norm(D - L @ R.T, 2)
        weyl = max(weyl, (np.abs(sig - s_d[:k]).max() - e2) / s_d[0])
    print(f"eps {eps} exact {exact}: {nblk} farfield blocks, max |R^T R - I| {orth_r:.2e}, "
          f"max normalised |L^T L - diag| {gram_l:.2e}, sort {sort_bad:.1e}, "
          f"|sigma - svd(L R^T)|/sigma_1 {sv_out:.2e}, Weyl excess/s_1 {weyl:.2e}, "
          f"exact blocks {st.n_exact_lowrank}", flush=True)
    assert nblk > 100
    if exact:
        assert st.n_exact_lowrank > 0
    assert orth_r <= 1e-12
    assert gram_l <= 1e-12
    assert sort_bad <= 0.0
    assert sv_out <= 1e-13
    assert weyl <= 1e-13
