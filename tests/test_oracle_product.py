"""Pins of the oracle's assembly, H-matrix-vector product, best approximation,
sum-expressions and product against closed forms, brute force and special cases."""

import numpy as np
import pytest

from workloads import fibonacci_sphere
from oracle.assemble import eps_rank, truncate, assemble
from oracle.hmatrix import HMatrix, Leaf, KIND_F, KIND_N
from oracle.kernels import kernel_matrix
from oracle.product import (StripIndex, brute_force_product, check_block, exact_block_strips,
                            blockwise_best_product, global_error_estimate)
from oracle.sumexpr import build_sum_expressions, apply_identity, hmult
from oracle.tree import build_cluster_tree, build_block_tree, KIND_F as T_F


def test_eps_rank_closed_form():
    s = np.array([1.0, 0.5, 1e-3, 1e-5, 1e-7, 0.0])
    nrm = np.sqrt((s ** 2).sum())
    # tail after keeping 3 values = sqrt(1e-10 + 1e-14)
    assert eps_rank(s, 1.001e-5 / nrm * 1.0001) == 3
    assert eps_rank(s, 0.99e-5 / nrm) == 4
    assert eps_rank(s, 1.0) == 0
    assert eps_rank(np.zeros(4), 1e-6) == 0


def test_truncate_is_eckart_young():
    rng = np.random.default_rng(1)
    U, _ = np.linalg.qr(rng.standard_normal((40, 12)))
    V, _ = np.linalg.qr(rng.standard_normal((30, 12)))
    s = 10.0 ** (-1.3 * np.arange(12))
    M = (U * s) @ V.T
    L, R, sv, k = truncate(M, 1e-6)
    assert np.allclose(sv[:12], s, rtol=1e-10, atol=1e-15)
    # relative tails: from index 5 about 10**-6.5 (kept below 1e-6), from 4 about 10**-5.2
    assert k == 5
    err = np.linalg.norm(M - L @ R.T)
    assert abs(err - np.sqrt((s[5:] ** 2).sum())) < 1e-14


def test_assembly_blockwise_and_global(small_case):
    pts, ct, bt, A = small_case
    K = kernel_matrix(pts[ct.perm], "laplace_4pi", 1.0, 0.0)
    for lf in A.leaves:
        blk = K[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
        nb = np.linalg.norm(blk)
        if lf.kind == KIND_F:
            assert np.linalg.norm(blk - lf.L @ lf.R.T) <= 1e-8 * nb * (1 + 1e-12)
            k = lf.L.shape[1]
            if k > 0:  # minimality: one rank fewer misses the tolerance
                s = np.linalg.svd(blk, compute_uv=False)
                assert np.sqrt((s[k - 1:] ** 2).sum()) > 1e-8 * nb
        else:
            assert np.array_equal(lf.D, blk)
    # global error follows from the blockwise ones (theorem after eq. (ACAblockerror))
    assert np.linalg.norm(A.to_dense(1) - K) <= 1e-8 * np.linalg.norm(K) * (1 + 1e-12)
    # diagonal value
    assert np.allclose(np.diag(A.to_dense(0)), 1.0)


def test_matvec_and_strips_match_dense(small_case):
    pts, ct, bt, A = small_case
    D = A.to_dense(1)
    x = np.random.default_rng(2).standard_normal((A.n, 3))
    assert np.allclose(A.matvec(x), D @ x, rtol=0, atol=1e-12 * np.abs(D @ x).max())
    assert np.allclose(A.rmatvec(x), D.T @ x, rtol=0, atol=1e-12 * np.abs(D.T @ x).max())
    si = StripIndex(A)
    assert np.array_equal(si.row_strip(100, 180), D[100:180])
    assert np.array_equal(si.col_strip(5, 70), D[:, 5:70])
    # original order is the inverse permutation of the cluster order
    D0 = A.to_dense(0)
    assert np.array_equal(D0[np.ix_(ct.perm, ct.perm)], D)


def test_strip_oracle_equals_brute_force(small_case):
    pts, ct, bt, A = small_case
    P = brute_force_product(A, A)
    si = StripIndex(A)
    for lf in A.leaves[::97]:
        blk = exact_block_strips(si, si, lf.r0, lf.m, lf.c0, lf.n)
        ref = P[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
        assert np.allclose(blk, ref, rtol=0, atol=1e-13 * np.abs(P).max())


def _small_tree(n=1024, leaf=24, split=0):
    pts = fibonacci_sphere(n)
    ct = build_cluster_tree(pts, leaf, split)
    return pts, ct, build_block_tree(ct, 0.8)


@pytest.mark.parametrize("split", [0, 1])
def test_sum_expressions_are_exact(split):
    """Restriction is lossless: S(tau, sigma) I = (A B)[tau, sigma] for every block."""
    pts, ct, bt = _small_tree(1024, 24, split)
    A = assemble(bt, pts, "laplace_4pi", 1.0, 0.0, 1e-8)
    B = assemble(bt, pts, "exp", 1.0, 1.0, 1e-8)
    P = brute_force_product(A, B)
    S = build_sum_expressions(A, B, bt)
    scale = np.abs(P).max()
    n_leafrho = 0
    for b in range(bt.count):
        t, s = bt.tau[b], bt.sigma[b]
        D = apply_identity(S, bt, b)
        ref = P[ct.begin[t]:ct.begin[t] + ct.size[t], ct.begin[s]:ct.begin[s] + ct.size[s]]
        assert np.abs(D - ref).max() <= 1e-13 * scale
    # the midpoint split produces pairs whose middle cluster is a leaf
    if split == 0:
        for b in range(bt.count):
            _, H = S[b]
            n_leafrho += sum(1 for r in H if not ct.children[r])
        S2 = build_sum_expressions(A, B, bt, drop_leaf_rho=True)
        worst = 0.0
        for b in bt.leaves():
            t, s = bt.tau[b], bt.sigma[b]
            ref = P[ct.begin[t]:ct.begin[t] + ct.size[t], ct.begin[s]:ct.begin[s] + ct.size[s]]
            worst = max(worst, np.linalg.norm(apply_identity(S2, bt, b) - ref) / np.linalg.norm(ref))
        assert worst > 1e-2  # dropping those pairs is visibly wrong


def test_hmult_equals_blockwise_best():
    pts, ct, bt = _small_tree(1024, 24, 0)
    A = assemble(bt, pts, "laplace_4pi", 1.0, 0.0, 1e-8)
    B = assemble(bt, pts, "exp", 1.0, 1.0, 1e-8)
    C1 = hmult(A, B, bt, 1e-6)
    C2 = blockwise_best_product(A, B, 1e-6)
    P = brute_force_product(A, B)
    for l1, l2 in zip(C1.leaves, C2.leaves):
        assert (l1.r0, l1.m, l1.c0, l1.n, l1.kind) == (l2.r0, l2.m, l2.c0, l2.n, l2.kind)
        ref = P[l1.r0:l1.r0 + l1.m, l1.c0:l1.c0 + l1.n]
        if l1.kind == KIND_F:
            c = check_block(ref, KIND_F, 1e-6, U=l1.L, V=l1.R, rank_slack=0)
            assert c.ok and c.rank == c.kstar == l2.L.shape[1]
        else:
            assert check_block(ref, KIND_N, 1e-6, Dc=l1.D).ok


def _identity_like(A: HMatrix, scale=1.0):
    I = HMatrix(n=A.n, perm=A.perm.copy())
    for lf in A.leaves:
        if lf.kind == KIND_F:
            I.leaves.append(Leaf(lf.r0, lf.m, lf.c0, lf.n, KIND_F, L=np.zeros((lf.m, 0)),
                                 R=np.zeros((lf.n, 0)), level=lf.level))
        else:
            D = scale * np.eye(lf.m) if (lf.r0 == lf.c0 and lf.m == lf.n) else np.zeros((lf.m, lf.n))
            I.leaves.append(Leaf(lf.r0, lf.m, lf.c0, lf.n, KIND_N, D=D, level=lf.level))
    return I


def test_special_cases(small_case):
    pts, ct, bt, A = small_case
    eps = 1e-6
    # B = identity: C is the blockwise eps-truncation of A
    C = hmult(A, _identity_like(A), bt, eps)
    for lc, la in zip(C.leaves, A.leaves):
        if la.kind == KIND_F:
            _, _, s, k = truncate(la.L @ la.R.T, eps)
            assert lc.L.shape[1] == k
            assert np.linalg.norm(lc.L @ lc.R.T - la.L @ la.R.T) <= eps * np.linalg.norm(s)
        else:
            assert np.allclose(lc.D, la.D, rtol=0, atol=1e-15)
    # B = 0: C = 0 with all ranks 0
    C0 = hmult(A, _identity_like(A, 0.0), bt, eps)
    assert all((l.kind == KIND_F and l.L.shape[1] == 0) or (l.kind == KIND_N and not l.D.any())
               for l in C0.leaves)


def test_rank_one_and_symmetry():
    pts, ct, bt = _small_tree(768, 24, 0)
    u = np.cos(3 * pts[ct.perm, 0]) + pts[ct.perm, 2]
    R1 = HMatrix(n=768, perm=ct.perm.copy())
    for b in bt.leaves():
        t, s = bt.tau[b], bt.sigma[b]
        r0, m, c0, n = ct.begin[t], ct.size[t], ct.begin[s], ct.size[s]
        if bt.kind[b] == T_F:
            R1.leaves.append(Leaf(r0, m, c0, n, KIND_F, L=u[r0:r0 + m, None].copy(), R=u[c0:c0 + n, None].copy()))
        else:
            R1.leaves.append(Leaf(r0, m, c0, n, KIND_N, D=np.outer(u[r0:r0 + m], u[c0:c0 + n])))
    A = assemble(bt, pts, "inv_dist", 1.0, 0.0, 1e-8)
    C = hmult(R1, A, bt, 1e-6)
    assert all(l.L.shape[1] <= 1 for l in C.leaves if l.kind == KIND_F)
    # A A is symmetric: mirrored blocks have equal eps-ranks
    C2 = hmult(A, A, bt, 1e-6)
    ranks = {(l.r0, l.c0): l.L.shape[1] for l in C2.leaves if l.kind == KIND_F}
    assert all(ranks[(c, r)] == k for (r, c), k in ranks.items())


def test_global_error_is_sum_of_block_errors():
    pts, ct, bt = _small_tree(1024, 24, 0)
    A = assemble(bt, pts, "laplace_4pi", 1.0, 0.0, 1e-8)
    B = assemble(bt, pts, "exp", 1.0, 1.0, 1e-8)
    C = blockwise_best_product(A, B, 1e-6)
    P = brute_force_product(A, B)
    E = C.to_dense(1) - P
    blocks = sum(np.linalg.norm(E[l.r0:l.r0 + l.m, l.c0:l.c0 + l.n]) ** 2 for l in C.leaves)
    assert abs(np.linalg.norm(E) ** 2 - blocks) <= 1e-12 * blocks
    assert np.linalg.norm(E) <= 1e-6 * np.linalg.norm(P)
    est, nrm = global_error_estimate(C, A, B, iters=3, size=40)
    assert 0.3 * np.linalg.norm(E, 2) <= est <= 1.01 * np.linalg.norm(E)
