"""Pins of the rank-predictor reference (oracle/mlp.py) that do not rely on it.

- gradient: central finite differences of the loss (h = 1e-6, float64);
- forward: a hand-built network whose output has a closed form;
- Adam: the first update moves every weight by lr * g / (|g| + eps), opposite
  to the gradient (bias corrections make m_hat = g and v_hat = g^2);
- training: full-batch Adam on a target the network can represent lowers the loss.
"""

import numpy as np
import pytest

from oracle import mlp


def random_params(rng, feats=None, ranks=None):
    parts = []
    for _, shape in mlp.SHAPES:
        fan_in = shape[1] if len(shape) == 2 else 64
        parts.append(rng.standard_normal(int(np.prod(shape))) * np.sqrt(2.0 / fan_in))
    if feats is None:
        norm = np.concatenate([rng.standard_normal(6), 0.5 + rng.random(6), [10.0, 4.0]])
    else:
        fm, fs, rm, rs = mlp.standardisation(feats, ranks)
        norm = np.concatenate([fm, fs, [rm, rs]])
    return np.concatenate(parts + [norm])


def test_layout_size():
    assert mlp.NPARAM == 64 * 6 + 64 + 2 * (64 * 64 + 64) + 64 + 1
    p = np.arange(mlp.NPARAM + mlp.NNORM, dtype=np.float64)
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    feats = rng.standard_normal((40, 6)) * 2 + 1
    ranks = rng.integers(1, 40, size=40).astype(np.float64)
    p = random_params(rng, feats, ranks)
    g = mlp.grad(p, feats, ranks)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 60, replace=False), [mlp.NPARAM - 1, 0, 64 * 6]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, feats, ranks) - mlp.loss(p - e, feats, ranks)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert np.all(g[mlp.NPARAM:] == 0)


def test_forward_closed_form():
    # h1[0] = relu(z0), passed through layers 2 and 3 unchanged; output 3 h3[0] - 1
    w = mlp.unpack(np.zeros(mlp.NPARAM + mlp.NNORM))
    w = {k: np.array(v, copy=True) for k, v in w.items()}
    w["W1"][0, 0] = 1.0
    w["W2"][0, 0] = 1.0
    w["W3"][0, 0] = 1.0
    w["W4"][0, 0] = 3.0
    w["b4"][0] = -1.0
    w["fmean"] = np.full(6, 2.0)
    w["fstd"] = np.full(6, 4.0)
    w["rmean"], w["rstd"] = 5.0, 2.0
    p = mlp.pack(w)
    feats = np.array([[10.0, 0, 0, 0, 0, 0], [-6.0, 9, 9, 9, 9, 9]])
    o, _ = mlp.forward(p, feats)
    assert np.allclose(o, [3 * 2.0 - 1, -1.0])
    assert np.allclose(mlp.predict(p, feats), [5.0 * 2 + 5, -1.0 * 2 + 5])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(mlp.NPARAM + mlp.NNORM)
    g = rng.standard_normal(mlp.NPARAM + mlp.NNORM)
    g[mlp.NPARAM:] = 0
    lr = 1e-2
    p1, m1, v1 = mlp.adam_step(p, np.zeros_like(p), np.zeros_like(p), g, 1, lr)
    k = mlp.NPARAM
    assert np.allclose(p1[:k] - p[:k], -lr * g[:k] / (np.abs(g[:k]) + 1e-8), rtol=1e-12, atol=0)
    assert np.array_equal(p1[k:], p[k:])
    assert np.allclose(m1[:k], 0.1 * g[:k]) and np.allclose(v1[:k], 0.001 * g[:k] ** 2)


def test_full_batch_adam_lowers_loss():
    rng = np.random.default_rng(11)
    feats = rng.standard_normal((128, 6))
    ranks = 12 + 3 * feats[:, 0] - 2 * np.abs(feats[:, 3])
    p = random_params(rng, feats, ranks)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = mlp.loss(p, feats, ranks)
    for step in range(1, 201):
        p, m, v = mlp.adam_step(p, m, v, mlp.grad(p, feats, ranks), step, 3e-3)
    assert mlp.loss(p, feats, ranks) < 0.1 * l0
