"""Pins of the oracle functions every GPU parity verdict rests on: the acceptance
rule (check_block), the kernel entries (kernel_block) and the strip oracle used
at full size (LeafStrips, oracle_block).

Each test is built so that a plausible mistake fails it: an acceptance rule
made lenient (relative error compared against an absolute bound, a dropped rank
slack, a nearfield tolerance loosened), a kernel with a wrong constant or a
missing diagonal shift, or a strip that misplaces a leaf.
"""

import math

import numpy as np
import pytest

from oracle.assemble import assemble, eps_rank
from oracle.hmatrix import KIND_F, KIND_N
from oracle.kernels import kernel_block, kernel_matrix
from oracle.product import LeafStrips, brute_force_product, check_block, oracle_block


def _spectrum_block(scale, m=40, n=30, seed=3):
    """D = U diag(s) V^T with orthonormal U, V and a geometric spectrum, scaled so that
    ||D||_F = scale (large, so that relative and absolute errors differ)."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, 14)))
    V, _ = np.linalg.qr(rng.standard_normal((n, 14)))
    s = 10.0 ** (-0.9 * np.arange(14))
    s *= scale / np.linalg.norm(s)
    return U, s, V, (U * s) @ V.T


def _tail(s, k):
    return float(np.sqrt(np.sum(s[k:] ** 2)))


@pytest.mark.parametrize("scale", [1e3, 1e-3])
def test_check_block_farfield_bounds(scale):
    """Acceptance of a farfield block (the epsilon-rank of the numerical-examples
    section, Eckart-Young): error <= 1.01 eps ||D||_F and rank <= k* + 2."""
    eps = 1e-6
    U, s, V, D = _spectrum_block(scale)
    nd = float(np.linalg.norm(D))
    k = eps_rank(s, eps)
    assert 0 < k < 12
    assert _tail(s, k) <= eps * nd < _tail(s, k - 1)

    def cand(rank, delta=0.0):
        """rank-`rank` truncation with its first singular value moved by delta:
        error^2 = tail(rank)^2 + delta^2 (orthogonal pieces)."""
        sv = s[:rank].copy()
        if rank:
            sv[0] += delta
        return U[:, :rank] * sv, V[:, :rank].copy()

    # the optimum passes, with k* reported
    L, R = cand(k)
    r = check_block(D, KIND_F, eps, U=L, V=R)
    assert r.ok and r.kstar == k and r.rank == k and r.err <= eps
    # one rank fewer misses the tolerance
    L, R = cand(k - 1)
    r = check_block(D, KIND_F, eps, U=L, V=R)
    assert not r.ok and r.err > eps
    # rank k* + 2 is allowed, k* + 3 is not, although both are more accurate
    assert check_block(D, KIND_F, eps, *cand(k + 2)).ok
    r = check_block(D, KIND_F, eps, *cand(k + 3))
    assert not r.ok and r.err < eps
    # error exactly 1.0 eps passes, 1.02 eps fails, at the optimal rank
    t = _tail(s, k)
    for target, ok in ((1.0, True), (1.02, False)):
        delta = math.sqrt((target * eps * nd) ** 2 - t * t)
        L, R = cand(k, delta)
        r = check_block(D, KIND_F, eps, U=L, V=R)
        assert abs(r.err - target * eps) <= 1e-6 * eps
        assert r.ok is ok


def test_check_block_zero_and_empty_farfield():
    D = np.zeros((8, 5))
    r = check_block(D, KIND_F, 1e-6, U=np.zeros((8, 0)), V=np.zeros((5, 0)))
    assert r.ok and r.kstar == 0 and r.err == 0.0
    # a nonzero candidate for a zero block is wrong
    r = check_block(D, KIND_F, 1e-6, U=np.ones((8, 1)), V=np.ones((5, 1)))
    assert not r.ok


def test_check_block_nearfield():
    """Nearfield blocks are exact up to rounding (evaluate() in Algorithm 4)."""
    rng = np.random.default_rng(4)
    D = 1e3 * rng.standard_normal((33, 21))
    assert check_block(D, KIND_N, 1e-6, Dc=D.copy()).ok
    assert check_block(D, KIND_N, 1e-6, Dc=D * (1 + 1e-14)).ok
    P = D.copy()
    P[3, 4] += 1e-10 * np.linalg.norm(D)
    r = check_block(D, KIND_N, 1e-6, Dc=P)
    assert not r.ok and 0.9e-10 <= r.err <= 1.1e-10
    assert check_block(np.zeros((4, 4)), KIND_N, 1e-6, Dc=np.zeros((4, 4))).ok
    assert not check_block(np.zeros((4, 4)), KIND_N, 1e-6, Dc=np.full((4, 4), 1e-100)).ok


def test_kernel_block_hand_values():
    """Entries at distances 5, 3 and 1 computed by hand, and the diagonal rule
    (diag + shift on i == j only)."""
    pts = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0], [1.0, 2.0, 2.0], [0.0, 0.0, 1.0]])
    rows, cols = np.array([0]), np.array([0, 1, 2, 3])
    want = {
        "laplace_4pi": [0.015915494309189534, 0.026525823848649224, 0.07957747154594767],  # 1/(20pi), 1/(12pi), 1/(4pi)
        "inv_dist": [0.2, 1.0 / 3.0, 1.0],
        "exp": [0.006737946999085467, 0.049787068367863944, 0.36787944117144233],  # e^-5, e^-3, e^-1
    }
    for kind, v in want.items():
        K = kernel_block(pts, rows, cols, kind, diag=0.25, shift=0.0)
        assert K.shape == (1, 4)
        assert K[0, 0] == 0.25
        assert np.allclose(K[0, 1:], v, rtol=1e-15, atol=0)
        # B = K + I: the diagonal becomes diag + 1 = 2 for diag 1 (kernel exp(-r) + I)
        K2 = kernel_block(pts, np.array([2, 1]), np.array([1, 2]), kind, diag=1.0, shift=1.0)
        assert K2[0, 1] == 2.0 and K2[1, 0] == 2.0
        d12 = math.dist(pts[1], pts[2])  # sqrt(4 + 4 + 4)
        ref = {"laplace_4pi": 1 / (4 * math.pi * d12), "inv_dist": 1 / d12, "exp": math.exp(-d12)}[kind]
        assert abs(K2[0, 0] - ref) <= 1e-15 * ref and abs(K2[1, 1] - ref) <= 1e-15 * ref
    # the full matrix is symmetric with the diagonal rule applied exactly once
    M = kernel_matrix(pts, "exp", diag=1.0, shift=1.0)
    assert np.array_equal(M, M.T) and np.all(np.diag(M) == 2.0)


def test_leafstrips_and_oracle_block_equal_brute_force(small_case):
    """The strip oracle used on sampled blocks at full size reproduces the
    brute-force product block by block, and its epsilon-rank is the one of the
    exact block."""
    pts, ct, bt, A = small_case
    B = assemble(bt, pts, "exp", 1.0, 1.0, 1e-8)
    P = brute_force_product(A, B)

    def src(H):
        r0 = [lf.r0 for lf in H.leaves]
        c0 = [lf.c0 for lf in H.leaves]
        r1 = [lf.r0 + lf.m for lf in H.leaves]
        c1 = [lf.c0 + lf.n for lf in H.leaves]
        return LeafStrips(H.n, r0, r1, c0, c1, lambda i: H.leaves[i].dense())

    sa, sb = src(A), src(B)
    DA, DB = A.to_dense(1), B.to_dense(1)
    assert np.array_equal(sa.row_strip(37, 301), DA[37:301])
    assert np.array_equal(sb.col_strip(1000, 1077), DB[:, 1000:1077])
    scale = np.abs(P).max()
    rng = np.random.default_rng(5)
    far = [i for i, lf in enumerate(B.leaves) if lf.kind == KIND_F]
    near = [i for i, lf in enumerate(B.leaves) if lf.kind == KIND_N]
    for i in list(rng.choice(far, 25, replace=False)) + list(rng.choice(near, 10, replace=False)):
        lf = B.leaves[i]
        D, s, k = oracle_block(sa, sb, lf.r0, lf.r0 + lf.m, lf.c0, lf.c0 + lf.n, lf.kind, 1e-6)
        ref = P[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
        assert np.abs(D - ref).max() <= 1e-13 * scale
        if lf.kind == KIND_F:
            sref = np.linalg.svd(ref, compute_uv=False)
            assert k == eps_rank(sref, 1e-6)
            assert np.allclose(s, sref, rtol=0, atol=1e-12 * sref[0])
        else:
            assert s is None and k is None
    # the inner-dimension chunked strip product (bounded host memory at full size) equals
    # the brute-force block for chunk sizes that cut leaves in the middle
    from oracle.product import exact_block_chunked
    for (r0, r1, c0, c1), chunk in (((37, 301, 1000, 1077), 500), ((0, 2048, 1900, 2048), 333), ((64, 128, 0, 64), 2048)):
        D = exact_block_chunked(sa, sb, r0, r1, c0, c1, chunk=chunk)
        assert np.abs(D - P[r0:r1, c0:c1]).max() <= 1e-13 * scale
