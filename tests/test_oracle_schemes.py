"""Pins of the oracle's generator and of its other low-rank schemes (CPU only).

Each scheme is checked against facts the paper and the mathematics fix, not
against its own formula:
  * Philox4x32-10: the published known-answer vectors of the generator;
    Box-Muller: one output evaluated by hand, and the first four moments;
  * ACA (Algorithm 6): a 3 x 3 example worked by hand (pivots, cross), exact
    recovery of a rank-r matrix in r steps, the interpolation property (the
    residual vanishes on every pivot row and column), and the stopping rule on a
    diagonal matrix with known spectrum;
  * Lanczos (Algorithm 7): Q^T D W equals the upper bidiagonal B built from
    alpha and beta (a transposed or shifted beta fails), full steps reproduce
    the singular values of D, and the stopping rule on a known spectrum;
  * Algorithm 9: exact when rank(D) <= k; never better than the Eckart-Young
    optimum; R = D^T L with orthonormal L;
  * Algorithm 5: equals the dense truncated SVD of L R^T.
"""

import numpy as np
import pytest

from oracle.assemble import truncate
from oracle.philox import philox4x32_10, gaussian_from_words, omega
from oracle.schemes import aca, lanczos, randomized_fixed, lowrank_svd


# ---------------------------------------------------------------- generator
@pytest.mark.parametrize("ctr,key,out", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, out):
    got = tuple(int(v) for v in philox4x32_10(list(ctr), key))
    assert got == out


def test_box_muller_by_hand():
    # words chosen so that a = 2^52 - 1 + ... : x = 0x80000000, y = 0 -> a = 2^52, u1 = (2^52 + 1) 2^-53
    # z = 0x40000000, w = 0 -> b = 2^51, u2 = 1/4: cos(pi/2) = 0 up to rounding
    g = gaussian_from_words(np.array([0x80000000, 0, 0x40000000, 0], dtype=np.uint64))
    u1 = (2.0 ** 52 + 1) * 2.0 ** -53
    assert abs(float(g) - np.sqrt(-2 * np.log(u1)) * np.cos(np.pi / 2)) < 1e-15
    # u2 = 0: g = sqrt(-2 ln u1)
    g0 = gaussian_from_words(np.array([0x80000000, 0, 0, 0], dtype=np.uint64))
    assert float(g0) == pytest.approx(np.sqrt(-2 * np.log(u1)), rel=1e-15)


def test_gaussian_moments_and_keying():
    Om = omega(np.arange(20000), np.arange(8), seed=0x5eed)
    x = Om.ravel()
    assert abs(x.mean()) < 0.02
    assert abs(x.var() - 1.0) < 0.02
    assert abs(np.mean(x ** 3)) < 0.05
    assert abs(np.mean(x ** 4) - 3.0) < 0.1
    # entries depend only on (row, column, seed): a sub-block equals the block of a larger draw
    sub = omega(np.arange(100, 140), np.arange(2, 5), seed=0x5eed)
    assert np.array_equal(sub, Om[100:140, 2:5])
    assert not np.array_equal(omega(np.arange(10), [0], 1), omega(np.arange(10), [0], 2))
    # columns are not shifted copies of each other
    c = np.corrcoef(Om[:, 0], Om[:, 1])[0, 1]
    assert abs(c) < 0.03


# ---------------------------------------------------------------- ACA
def test_aca_hand_example():
    D = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0], [7.0, 8.0, 10.0]])
    # step 1: row 0 = (1, 2, 3), column pivot 2, u1 = (1/3, 2/3, 1), l1 = D[:, 2] = (3, 6, 10)
    r1 = aca(D, 0.0, k_fixed=1)
    A1 = np.outer([3.0, 6.0, 10.0], [1 / 3, 2 / 3, 1.0])
    assert np.allclose(r1.L @ r1.R.T, A1, rtol=0, atol=1e-14)
    # step 2: next row = largest |l1| among rows 1, 2 -> row 2; residual row
    # (7, 8, 10) - 10 u1 = (11/3, 4/3, 0), pivot column 0; u2 = (1, 4/11, 0);
    # l2 = D[:, 0] - u1[0] l1 = (1, 4, 7) - (1, 2, 10/3) = (0, 2, 11/3)
    r2 = aca(D, 0.0, k_fixed=2)
    A2 = A1 + np.outer([0.0, 2.0, 11 / 3], [1.0, 4 / 11, 0.0])
    assert np.allclose(r2.L @ r2.R.T, A2, rtol=0, atol=1e-13)
    # three steps on a 3 x 3 matrix interpolate every row: exact
    r3 = aca(D, 0.0, k_fixed=3)
    assert np.allclose(r3.L @ r3.R.T, D, rtol=0, atol=1e-13)


def test_aca_recovers_low_rank_and_interpolates():
    rng = np.random.default_rng(3)
    for r in (1, 4, 9):
        D = rng.standard_normal((40, r)) @ rng.standard_normal((r, 30))
        res = aca(D, 1e-12)
        assert res.converged and res.steps == r
        assert np.linalg.norm(res.L @ res.R.T - D) <= 1e-12 * np.linalg.norm(D)
    # interpolation: after k fixed steps the residual vanishes on the pivot rows/columns
    D = rng.standard_normal((25, 20))
    D = D @ np.diag(0.5 ** np.arange(20)) @ rng.standard_normal((20, 20))
    res = aca(D, 0.0, k_fixed=6)
    Rm = D - res.L @ res.R.T
    rows = np.argsort(np.abs(Rm).max(axis=1))[:6]
    cols = np.argsort(np.abs(Rm).max(axis=0))[:6]
    assert np.abs(Rm[rows]).max() <= 1e-10 * np.abs(D).max()
    assert np.abs(Rm[:, cols]).max() <= 1e-10 * np.abs(D).max()


def test_aca_stopping_rule_on_known_spectrum():
    D = np.diag([1.0, 1e-3, 1e-9, 0.0])
    res = aca(D, 1e-6)
    # steps: 1, 1e-3 kept; the 1e-9 update is below 1e-6 * ||L U|| and is discarded
    assert res.steps == 2 and res.converged
    assert res.e2 == pytest.approx(1e-18, rel=1e-12)
    assert res.L.shape[1] == 2
    # zero block: rank 0
    z = aca(np.zeros((5, 4)), 1e-6)
    assert z.L.shape[1] == 0 and z.converged


# ---------------------------------------------------------------- Lanczos
def test_lanczos_bidiagonal_relation_and_spectrum():
    rng = np.random.default_rng(5)
    D = rng.standard_normal((12, 9))
    w1 = rng.standard_normal(9)
    res = lanczos(D, 0.0, w1, k_fixed=9)
    s_ref = np.linalg.svd(D, compute_uv=False)
    s_got = np.linalg.svd(res.L @ res.R.T, compute_uv=False)
    assert np.allclose(s_got, s_ref, rtol=1e-12, atol=0)
    # B = Q^T D W is upper bidiagonal with alpha on the diagonal and beta above it:
    # rebuild the recurrence by hand for 4 steps
    w = w1 / np.linalg.norm(w1)
    q = D @ w
    a1 = np.linalg.norm(q)
    q = q / a1
    v = D.T @ q - a1 * w
    b1 = np.linalg.norm(v)
    v = v / b1
    q2 = D @ v - b1 * q
    a2 = np.linalg.norm(q2)
    r2 = lanczos(D, 0.0, w1, k_fixed=2)
    # the rank-2 approximation is Q_2 B_2 W_2^T with B_2 = [[a1, b1], [0, a2]]
    B2 = np.array([[a1, b1], [0.0, a2]])
    A2 = np.stack([q, q2 / a2], 1) @ B2 @ np.stack([w, v], 1).T
    assert np.allclose(r2.L @ r2.R.T, A2, rtol=0, atol=1e-12 * np.abs(D).max())


def test_lanczos_stopping_rule():
    U = np.linalg.qr(np.random.default_rng(1).standard_normal((30, 6)))[0]
    V = np.linalg.qr(np.random.default_rng(2).standard_normal((20, 6)))[0]
    s = np.array([1.0, 0.1, 1e-2, 1e-9, 1e-10, 1e-11])
    D = U @ np.diag(s) @ V.T
    res = lanczos(D, 1e-6, np.ones(20))
    # the Krylov space needs a step beyond the rank it resolves before the updates fall below eps
    assert res.converged and 3 <= res.steps <= 5
    k = res.L.shape[1]
    assert k == 3
    assert np.linalg.norm(D - res.L @ res.R.T) <= 1e-6 * np.linalg.norm(D)
    # exactly rank 2, start vector with a part outside the row space: the right Krylov space
    # span(w1, D^T D w1, (D^T D)^2 w1) holds the row space after 3 steps, and the result is exact
    D2 = U[:, :2] @ np.diag([1.0, 0.5]) @ V[:, :2].T
    r2 = lanczos(D2, 1e-12, np.ones(20))
    assert r2.steps == 3 and r2.L.shape[1] == 2 and np.linalg.norm(D2 - r2.L @ r2.R.T) <= 1e-13


# ---------------------------------------------------------------- Algorithm 9
def test_randomized_fixed_rank():
    rng = np.random.default_rng(7)
    D = rng.standard_normal((50, 5)) @ rng.standard_normal((5, 40))
    Om = rng.standard_normal((40, 8))
    res = randomized_fixed(D, Om, q=1)
    assert np.allclose(res.L.T @ res.L, np.eye(8), atol=1e-12)
    assert np.allclose(res.R, D.T @ res.L, atol=1e-12)
    assert np.linalg.norm(D - res.L @ res.R.T) <= 1e-12 * np.linalg.norm(D)
    # full-rank block: never better than the best rank-k approximation, and close to it
    D = rng.standard_normal((60, 60)) @ np.diag(0.6 ** np.arange(60)) @ rng.standard_normal((60, 60))
    s = np.linalg.svd(D, compute_uv=False)
    opt = np.sqrt(np.sum(s[8:] ** 2))
    mean = {}
    for q in (0, 1, 3):
        errs = []
        for _ in range(6):
            r = randomized_fixed(D, rng.standard_normal((60, 8)), q=q)
            errs.append(np.linalg.norm(D - r.L @ r.R.T))
        assert min(errs) >= opt * (1 - 1e-12)
        mean[q] = np.mean(errs) / opt
    # subspace iterations converge to the optimum: q = 0 is far off, q = 3 within 1 %
    assert mean[3] < mean[1] < mean[0] and mean[1] <= 1.6 and mean[3] <= 1.01


# ---------------------------------------------------------------- Algorithm 5
def test_lowrank_svd_equals_dense_truncation():
    rng = np.random.default_rng(11)
    L = rng.standard_normal((70, 12)) @ np.diag(0.3 ** np.arange(12))
    R = rng.standard_normal((45, 12))
    for eps in (1e-2, 1e-6, 1e-12):
        Lo, Ro = lowrank_svd(L, R, eps)
        Ld, Rd, _, k = truncate(L @ R.T, eps)
        assert Lo.shape[1] == k
        assert np.linalg.norm(Lo @ Ro.T - Ld @ Rd.T) <= 1e-12 * np.linalg.norm(L @ R.T)


# ---------------------------------------------------------------- subspace estimator
def test_subspace_frobenius_pins():
    from oracle.product import subspace_frobenius
    rng = np.random.default_rng(13)
    # rank-6 operator: a block of p >= 6 directions captures all of it -> exactly ||E||_F
    E = rng.standard_normal((80, 6)) @ rng.standard_normal((6, 70))
    est = subspace_frobenius(lambda X: E @ X, lambda Y: E.T @ Y, rng.standard_normal((70, 8)), 3)
    assert est == pytest.approx(np.linalg.norm(E), rel=1e-12)
    # decaying spectrum, p = 5: converges to the norm of the top-5 part, below ||E||_F
    U = np.linalg.qr(rng.standard_normal((60, 20)))[0]
    V = np.linalg.qr(rng.standard_normal((50, 20)))[0]
    s = 0.5 ** np.arange(20)
    E = U @ np.diag(s) @ V.T
    est = subspace_frobenius(lambda X: E @ X, lambda Y: E.T @ Y, rng.standard_normal((50, 5)), 12)
    assert est == pytest.approx(np.sqrt(np.sum(s[:5] ** 2)), rel=1e-8)
    assert est < np.linalg.norm(E)
    # the transpose must be E^T: with E itself in its place (a transposed-operand slip) the
    # estimate is wrong
    Esq = E[:50]
    good = subspace_frobenius(lambda X: Esq @ X, lambda Y: Esq.T @ Y, rng.standard_normal((50, 5)), 12)
    wrong = subspace_frobenius(lambda X: Esq @ X, lambda Y: Esq @ Y, rng.standard_normal((50, 5)), 12)
    assert abs(wrong - good) > 1e-3 * good
