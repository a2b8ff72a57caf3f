"""GPU rank predictor: forward, gradient and Adam kernels against the float64
reference, feature extraction from a product, and the learned product mode
(accuracy unchanged, fewer growth rounds, fallback when the prediction is
too small)."""

import ctypes

import numpy as np
import pytest

from oracle import mlp
from oracle.hmatrix import KIND_F
from oracle.product import brute_force_product, check_block
from tests.helpers import exported_to_oracle
from workloads import fibonacci_sphere, jitter

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


def data(seed, n):
    rng = np.random.default_rng(seed)
    feats = np.column_stack([rng.integers(2, 12, n), rng.normal(-1, 1, n), rng.normal(-1, 1, n),
                             rng.normal(0, 1, n), rng.normal(4, 1, n), rng.integers(1, 30, n)])
    ranks = np.maximum(1, np.round(3 * feats[:, 0] - 4 * feats[:, 3] + feats[:, 4] + rng.normal(0, 1, n)))
    return feats.astype(np.float32), ranks.astype(np.float32)


def ref_params(H, model, feats, ranks):
    """The model's parameters with the standardisation of (feats, ranks) (float32)."""
    p = H.hmat_rank_model_get(model).astype(np.float64)
    fm, fs, rm, rs = mlp.standardisation(feats, ranks)
    p[mlp.NPARAM:] = np.concatenate([fm, fs, [rm, rs]]).astype(np.float32)
    return p


def test_predict_matches_reference(H):
    feats, ranks = data(1, 300)
    m = H.hmat_rank_model_create(7)
    try:
        p = ref_params(H, m, feats, ranks)
        H.hmat_rank_model_set(m, p)
        got = H.hmat_rank_model_predict(m, feats)
        want = mlp.predict(p, feats.astype(np.float64))
        assert np.max(np.abs(got - want)) <= 1e-4 * max(1.0, np.max(np.abs(want)))
        assert H.hmat_rank_model_predict(m, feats[:0]).size == 0
    finally:
        H.hmat_rank_model_destroy(m)


def test_gradient_matches_reference(H):
    feats, ranks = data(2, 256)
    m = H.hmat_rank_model_create(3)
    try:
        p = ref_params(H, m, feats, ranks)
        H.hmat_rank_model_set(m, p)
        g, loss = H.hmat_rank_model_grad(m, feats, ranks)
        gr = mlp.grad(p, feats.astype(np.float64), ranks.astype(np.float64))
        lr = mlp.loss(p, feats.astype(np.float64), ranks.astype(np.float64))
        assert abs(loss - lr) <= 1e-4 * lr
        scale = np.max(np.abs(gr))
        err = np.abs(g - gr)
        assert np.all(err <= 1e-4 * np.abs(gr) + 1e-5 * scale), float(np.max(err / (np.abs(gr) + scale)))
    finally:
        H.hmat_rank_model_destroy(m)


def test_adam_step_matches_reference(H):
    feats, ranks = data(4, 200)
    m = H.hmat_rank_model_create(5)
    try:
        p0 = ref_params(H, m, feats, ranks)
        H.hmat_rank_model_set(m, p0)
        lr = 1e-3
        H.hmat_rank_model_train(m, feats, ranks, H.hmat_train_opts_default(epochs=1, batch=200, lr=lr))
        p1 = H.hmat_rank_model_get(m).astype(np.float64)
        g = mlp.grad(p0, feats.astype(np.float64), ranks.astype(np.float64))
        z = np.zeros_like(p0)
        pr, _, _ = mlp.adam_step(p0, z, z, g, 1, lr)
        k = mlp.NPARAM
        assert np.allclose(p1[k:], p0[k:], rtol=1e-6)
        big = np.abs(g[:k]) > 1e-3 * np.max(np.abs(g[:k]))
        d_gpu, d_ref = p1[:k] - p0[:k], pr[:k] - p0[:k]
        assert np.all(np.abs(d_gpu) <= lr * (1 + 1e-3) + 1e-6 * np.abs(p0[:k]))
        assert np.allclose(d_gpu[big], d_ref[big], rtol=2e-3, atol=2e-6 * (1 + np.max(np.abs(p0))))
    finally:
        H.hmat_rank_model_destroy(m)


def test_save_load_roundtrip(H, tmp_path):
    feats, ranks = data(8, 100)
    m = H.hmat_rank_model_create(2)
    try:
        H.hmat_rank_model_set(m, ref_params(H, m, feats, ranks))
        path = str(tmp_path / "model.bin")
        H.hmat_rank_model_save(m, path)
        m2 = H.hmat_rank_model_load(path)
        try:
            assert np.array_equal(H.hmat_rank_model_get(m2), H.hmat_rank_model_get(m))
            assert np.array_equal(H.hmat_rank_model_predict(m2, feats), H.hmat_rank_model_predict(m, feats))
        finally:
            H.hmat_rank_model_destroy(m2)
        (tmp_path / "bad.bin").write_bytes(b"not a model")
        with pytest.raises(H.HmatError):
            H.hmat_rank_model_load(str(tmp_path / "bad.bin"))
    finally:
        H.hmat_rank_model_destroy(m)


def test_training_lowers_loss(H):
    feats, ranks = data(6, 2000)
    m = H.hmat_rank_model_create(9)
    try:
        losses = H.hmat_rank_model_train(m, feats, ranks, H.hmat_train_opts_default(epochs=60, batch=128, lr=2e-3))
        assert losses[-1] < 0.2 * losses[0], losses[[0, -1]]
        pred = H.hmat_rank_model_predict(m, feats)
        assert np.sqrt(np.mean((pred - ranks) ** 2)) < 0.5 * np.std(ranks)
    finally:
        H.hmat_rank_model_destroy(m)


@pytest.fixture(scope="module")
def product_case(H):
    pts = jitter(fibonacci_sphere(4096), 1e-3, seed=2)
    t = H.hmat_build_tree(pts, 32, 0.8, 0)
    A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
    B, _ = H.hmat_assemble(t, "exp", 1.0, 1.0, eps_in=1e-8)
    P = brute_force_product(exported_to_oracle(H, t, A), exported_to_oracle(H, t, B))
    yield t, A, B, P
    H.hmat_destroy(A)
    H.hmat_destroy(B)
    H.hmat_tree_destroy(t)


def multiply(H, t, A, B, eps, **kw):
    st = H.hmat_stats()
    o = H.hmat_opts_default(**kw)
    o.stats = ctypes.pointer(st)
    C, code = H.hmat_multiply(A, B, eps, o)
    return C, st


def count_bad(H, t, C, P, eps):
    Co = exported_to_oracle(H, t, C)
    bad = 0
    for lf in Co.leaves:
        D = P[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
        r = check_block(D, KIND_F, eps, U=lf.L, V=lf.R) if lf.kind == KIND_F else check_block(D, 2, eps, Dc=lf.D)
        bad += not r.ok
    return bad


def test_features(H, product_case):
    t, A, B, P = product_case
    eps = 1e-6
    C0, st0 = multiply(H, t, A, B, eps)
    feats, ranks = H.hmat_product_features(C0)
    assert feats.shape == (st0.n_far, 6) and ranks.shape == (st0.n_far,)
    # ranks are those of C's farfield blocks; level feature matches the block levels
    bl = H.hmat_tree_blocks(t)
    far = np.nonzero(bl["kind"] == 1)[0]
    rk, _, _ = H.hmat_export(C0)
    leaf = np.nonzero(bl["kind"] != 0)[0]
    far_ranks = rk[np.isin(leaf, far)]
    assert np.array_equal(np.sort(ranks), np.sort(far_ranks.astype(np.float32)))
    assert np.array_equal(np.sort(feats[:, 0]), np.sort(bl["level"][far].astype(np.float32)))
    assert np.all(np.isfinite(feats))
    # sketch widths at which the residual check passed: at least the block's rank and at
    # most the panel capacity; blocks that grew need more than the first width b0 (8)
    widths = H.hmat_product_widths(C0)
    assert widths.shape == ranks.shape
    assert np.all(widths >= ranks) and np.all(widths <= 64)
    assert int(np.sum(widths > 8)) <= st0.n_grown_blocks
    assert count_bad(H, t, C0, P, eps) == 0
    H.hmat_destroy(C0)


@pytest.mark.parametrize("eps", [1e-6, 1e-8])
def test_learned_mode(H, product_case, eps):
    """The predictor is trained out of sample: on the sketch widths (hmat_product_widths)
    of a product on other points (another jitter draw of the sphere and the ellipsoid
    with axes 1, 0.7, 0.5), then applied to this product. The learned mode keeps every
    block within the bound. At eps = 1e-8, where most blocks grow, it grows at most half
    as many blocks as the plain form and makes fewer operator passes (its wider first
    sketches take passes of their own). At eps = 1e-6 (ranks around 6, inside the plain
    width) a block is widened only where the prediction is three quarters into the first
    growth step: it grows at most three quarters as many blocks, with at most 5 % more
    passes."""
    from workloads import ellipsoid
    t, A, B, P = product_case
    C0, st0 = multiply(H, t, A, B, eps)
    H.hmat_destroy(C0)
    feats, widths = [], []
    for pts in (jitter(fibonacci_sphere(4096), 1e-3, seed=9), ellipsoid(4096, (1.0, 0.7, 0.5))):
        tt = H.hmat_build_tree(pts, 32, 0.8, 0)
        At, _ = H.hmat_assemble(tt, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
        Bt, _ = H.hmat_assemble(tt, "exp", 1.0, 1.0, eps_in=1e-8)
        Ct, _ = multiply(H, tt, At, Bt, eps)
        f, _ = H.hmat_product_features(Ct)
        feats.append(f)
        widths.append(H.hmat_product_widths(Ct))
        for h in (At, Bt, Ct):
            H.hmat_destroy(h)
        H.hmat_tree_destroy(tt)
    feats, widths = np.concatenate(feats), np.concatenate(widths)
    m = H.hmat_rank_model_create(1)
    try:
        losses = H.hmat_rank_model_train(m, feats, widths, H.hmat_train_opts_default(epochs=200, batch=128, lr=2e-3))
        assert losses[-1] < losses[0]
        C1, st1 = multiply(H, t, A, B, eps, rank_mode=H.HMAT_RANK_PREDICT, rank_model=m)
        assert count_bad(H, t, C1, P, eps) == 0
        assert st1.n_not_converged == 0
        print(f"eps {eps}: training widths {np.bincount(widths.astype(int))[8::8]} (8, 16, ...); plain: grown "
              f"{st0.n_grown_blocks}, columns {st0.sketch_columns}, target passes {st0.target_passes}; learned: grown "
              f"{st1.n_grown_blocks}, columns {st1.sketch_columns}, fallback {st1.n_fallback}, target passes "
              f"{st1.target_passes}", flush=True)
        assert 0 <= st1.n_fallback <= st1.n_grown_blocks
        if eps < 1e-7:
            assert st1.n_grown_blocks <= 0.5 * max(st0.n_grown_blocks, 1)
            assert st1.target_passes < st0.target_passes
        else:
            assert st1.n_grown_blocks <= 0.75 * max(st0.n_grown_blocks, 1)
            assert st1.target_passes <= 1.05 * st0.target_passes
        H.hmat_destroy(C1)
    finally:
        H.hmat_rank_model_destroy(m)


def test_under_prediction_falls_back(H, product_case):
    t, A, B, P = product_case
    eps = 1e-6
    m = H.hmat_rank_model_create(1)
    try:
        p = H.hmat_rank_model_get(m)
        p[mlp.NPARAM - 1] = -1e4  # output bias: every prediction far below 1
        H.hmat_rank_model_set(m, p)
        C, st = multiply(H, t, A, B, eps, rank_mode=H.HMAT_RANK_PREDICT, rank_model=m, p_l=0, max_growth=16)
        assert 0 < st.n_fallback <= st.n_grown_blocks  # blocks vs block-rounds
        assert st.n_not_converged == 0
        assert count_bad(H, t, C, P, eps) == 0
        H.hmat_destroy(C)
    finally:
        H.hmat_rank_model_destroy(m)


def test_growth_budget_exhausted_is_reported(H, product_case):
    t, A, B, P = product_case
    st = H.hmat_stats()
    o = H.hmat_opts_default(b0=1, max_growth=0)
    o.stats = ctypes.pointer(st)
    C, code = H.hmat_multiply(A, B, 1e-6, o, allow_not_converged=True)
    assert code == H.HMAT_ERR_NOT_CONVERGED
    assert st.n_not_converged > 0
    # the blocks are listed: converged = 0 exactly on the farfield blocks that ran out
    n = H.hmat_block_count(C)
    flags = [H.hmat_block_get(C, i, with_data=False)[0] for i in range(n)]
    assert sum(1 for d in flags if d["converged"] == 0) == st.n_not_converged
    assert all(d["kind"] == 1 for d in flags if d["converged"] == 0)
    H.hmat_destroy(C)
    with pytest.raises(H.HmatError):
        H.hmat_multiply(A, B, 1e-6, o)
