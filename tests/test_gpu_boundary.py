"""Boundary calls and special cases of the product on the GPU.

* hmat_to_dense in both point orders against the oracle's densification of the
  library's exported leaves;
* HMAT_FP32_APPLY rejected below its accuracy floor;
* special cases of the product with a plain answer: A = B symmetric (mirrored
  blocks have equal epsilon-ranks, so the library's ranks agree within the rank
  slack), eps = 1e-14 (no truncation: C equals A_H B_H up to rounding, the exact
  product in low-rank format of Section 3), and a global rank-one factor (every
  block of C has rank <= 1).
"""

import ctypes

import numpy as np
import pytest

from oracle.hmatrix import HMatrix, Leaf, KIND_F, KIND_N
from oracle.product import brute_force_product, check_block
from tests.helpers import exported_to_oracle, oracle_to_blocks
from workloads import fibonacci_sphere, jitter

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


def _export_all(H, t, M):
    ranks, offs, pool = H.hmat_export(M)
    return ranks.copy(), offs.copy(), pool.copy()


def test_to_dense_both_orders(H):
    print("[boundary] hmat_to_dense, 1500 jittered sphere points, leaf 24, A and C = A B", flush=True)
    pts = jitter(fibonacci_sphere(1500), 1e-3, 2)
    t = H.hmat_build_tree(pts, 24, 0.8, 0)
    A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
    B, _ = H.hmat_assemble(t, "exp", 1.0, 1.0, eps_in=1e-8)
    C, _ = H.hmat_multiply(A, B, 1e-6)
    n = 1500
    for M in (A, C):
        Mo = exported_to_oracle(H, t, M)
        for order in (0, 1):
            D = H.hmat_to_dense(M, n, order)
            ref = Mo.to_dense(order)
            err = np.abs(D - ref).max()
            print(f"  order {order}: max |to_dense - oracle| = {err:.3e}", flush=True)
            assert err <= 1e-15 * np.abs(ref).max()
    # leading dimension larger than n
    import paper_1805_08998_amd.hmat as HM
    out = np.full((n + 7, n), np.nan, order="F")
    HM._check(HM.lib().hmat_to_dense(A, out.ctypes.data_as(HM._D), n + 7, 1))
    assert np.array_equal(out[:n], H.hmat_to_dense(A, n, 1)) and np.isnan(out[n:]).all()
    # argument errors
    assert HM.lib().hmat_to_dense(A, out.ctypes.data_as(HM._D), n - 1, 1) == H.HMAT_ERR_ARG
    assert HM.lib().hmat_to_dense(A, out.ctypes.data_as(HM._D), n, 2) == H.HMAT_ERR_ARG
    for h in (A, B, C):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)


def test_fp32_apply_floor(H):
    print("[boundary] HMAT_FP32_APPLY below its accuracy floor", flush=True)
    pts = fibonacci_sphere(600)
    t = H.hmat_build_tree(pts, 24, 0.8, 0)
    A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
    o = H.hmat_opts_default(precision=H.HMAT_FP32_APPLY)
    with pytest.raises(H.HmatError) as e:
        H.hmat_multiply(A, A, 1e-8, o)
    assert e.value.code == H.HMAT_ERR_ARG and "1e-6" in str(e.value)
    with pytest.raises(H.HmatError):
        H.hmat_multiply_batched([A], [A], 1e-7, o)
    C, code = H.hmat_multiply(A, A, 1e-6, o)
    assert code == 0
    H.hmat_destroy(C)
    H.hmat_destroy(A)
    H.hmat_tree_destroy(t)


def _product_check(H, t, A, B, C, eps):
    Ao, Bo, Co = exported_to_oracle(H, t, A), exported_to_oracle(H, t, B), exported_to_oracle(H, t, C)
    P = brute_force_product(Ao, Bo)
    return P, Co


def test_symmetric_product_mirrored_ranks(H):
    """A = B = A^T: C = A^2 is symmetric, k*(tau x sigma) = k*(sigma x tau), so the
    library's ranks of mirrored blocks agree within the rank slack of 2."""
    print("[special] A = B symmetric, n = 2048: mirrored ranks", flush=True)
    pts = fibonacci_sphere(2048)
    t = H.hmat_build_tree(pts, 32, 0.8, 0)
    A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
    C, _ = H.hmat_multiply(A, A, 1e-6)
    P, Co = _product_check(H, t, A, A, C, 1e-6)
    ranks = {(l.r0, l.c0): l.L.shape[1] for l in Co.leaves if l.kind == KIND_F}
    diff = [abs(ranks[(c, r)] - k) for (r, c), k in ranks.items()]
    bad = sum(not (check_block(P[l.r0:l.r0 + l.m, l.c0:l.c0 + l.n], KIND_F, 1e-6, U=l.L, V=l.R).ok)
              for l in Co.leaves if l.kind == KIND_F)
    print(f"  {len(ranks)} farfield blocks, max |rank - mirrored rank| = {max(diff)}, {bad} outside the bound",
          flush=True)
    assert max(diff) <= 2 and bad == 0
    H.hmat_destroy(C)
    H.hmat_destroy(A)
    H.hmat_tree_destroy(t)


def test_tiny_eps_is_exact_product(H):
    """eps = 1e-13 and 1e-14: no truncation to speak of; C equals A_H B_H up to rounding.
    The largest blocks of this tree then keep 33-43 columns of near-rank-deficient cores,
    where the core SVD's rotations must stay identical across the lanes of a wave (an
    earlier build lost the orthogonality of its right factor on two such blocks)."""
    pts = jitter(fibonacci_sphere(2048), 1e-3, 3)
    t = H.hmat_build_tree(pts, 32, 0.8, 0)
    A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
    B, _ = H.hmat_assemble(t, "exp", 1.0, 1.0, eps_in=1e-8)
    for eps in (1e-13, 1e-14):
        print(f"[special] eps = {eps:g}, n = 2048: C = A_H B_H to rounding", flush=True)
        st = H.hmat_stats()
        o = H.hmat_opts_default(max_growth=7)  # panel capacity 64: every block of this tree fits
        o.stats = ctypes.pointer(st)
        C, code = H.hmat_multiply(A, B, eps, o)
        P, Co = _product_check(H, t, A, B, C, eps)
        E = Co.to_dense(1) - P
        rel = np.linalg.norm(E) / np.linalg.norm(P)
        worst = max(np.linalg.norm(E[l.r0:l.r0 + l.m, l.c0:l.c0 + l.n]) /
                    np.linalg.norm(P[l.r0:l.r0 + l.m, l.c0:l.c0 + l.n]) for l in Co.leaves)
        print(f"  status {code}, global relative error {rel:.3e}, worst block {worst:.3e}, "
              f"Jacobi sweep caps {st.n_svd_sweep_cap}", flush=True)
        assert code == 0
        assert rel <= 1e-13 and worst <= 1e-12
        H.hmat_destroy(C)
    for h in (A, B):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)


def test_rank_one_factor(H):
    """A = u u^T (global rank one, stored on the tree's partition): every block of
    C = A B has rank <= 1, and meets the acceptance bound."""
    print("[special] global rank-one A, n = 1024", flush=True)
    pts = fibonacci_sphere(1024)
    t = H.hmat_build_tree(pts, 24, 0.8, 0)
    B, _ = H.hmat_assemble(t, "inv_dist", 1.0, 0.0, eps_in=1e-8)
    Bo = exported_to_oracle(H, t, B)
    perm = H.hmat_tree_perm(t)
    u = np.cos(3 * pts[perm, 0]) + pts[perm, 2]
    R1 = HMatrix(n=1024, perm=Bo.perm)
    for lf in Bo.leaves:
        if lf.kind == KIND_F:
            R1.leaves.append(Leaf(lf.r0, lf.m, lf.c0, lf.n, KIND_F, L=u[lf.r0:lf.r0 + lf.m, None].copy(),
                                  R=u[lf.c0:lf.c0 + lf.n, None].copy()))
        else:
            R1.leaves.append(Leaf(lf.r0, lf.m, lf.c0, lf.n, KIND_N,
                                  D=np.outer(u[lf.r0:lf.r0 + lf.m], u[lf.c0:lf.c0 + lf.n])))
    A = H.hmat_from_blocks(t, *oracle_to_blocks(R1))
    C, code = H.hmat_multiply(A, B, 1e-6)
    P, Co = _product_check(H, t, A, B, C, 1e-6)
    kmax, bad = 0, 0
    for l in Co.leaves:
        D = P[l.r0:l.r0 + l.m, l.c0:l.c0 + l.n]
        if l.kind == KIND_F:
            kmax = max(kmax, l.L.shape[1])
            bad += not check_block(D, KIND_F, 1e-6, U=l.L, V=l.R).ok
        else:
            bad += not check_block(D, KIND_N, 1e-6, Dc=l.D).ok
    print(f"  max farfield rank {kmax}, {bad} blocks outside the bound", flush=True)
    assert code == 0 and kmax <= 1 and bad == 0
    for h in (A, B, C):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)
