"""Rank predictor reference (test infrastructure; float64, numpy).

The learned component of the product predicts the epsilon-rank of a farfield
block of C from cheap geometric and structural features, so that the
randomized compression (the blocked scheme of Section 4) starts with a sketch
whose width is close to the final rank.  The model is a multi-layer perceptron
6 -> 64 -> 64 -> 64 -> 1 with ReLU activations, trained with the mean squared
error on standardised ranks and the Adam update (Kingma and Ba, 2015).

Parameter vector layout (shared with the library's get/set entry points):
W1 (64x6), b1 (64), W2 (64x64), b2 (64), W3 (64x64), b3 (64), W4 (1x64), b4 (1),
then the standardisation: feature means (6), feature standard deviations (6),
rank mean, rank standard deviation.  Weight matrices are row-major (out x in).

This module is written for clarity, not speed; only tests, the smoke check and
the CPU baseline of the benchmark use it.
"""

import numpy as np

NF, NH = 6, 64
SHAPES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (1, NH)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
NNORM = 2 * NF + 2


def unpack(p):
    """Split a flat parameter vector into named weights and the standardisation."""
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    norm = p[o:o + NNORM]
    out["fmean"], out["fstd"] = norm[:NF], norm[NF:2 * NF]
    out["rmean"], out["rstd"] = norm[2 * NF], norm[2 * NF + 1]
    return out


def pack(w):
    parts = [np.asarray(w[name], dtype=np.float64).ravel() for name, _ in SHAPES]
    parts += [np.asarray(w["fmean"]).ravel(), np.asarray(w["fstd"]).ravel(),
              np.array([w["rmean"], w["rstd"]], dtype=np.float64)]
    return np.concatenate(parts)


def standardisation(feats, ranks):
    """Mean and population standard deviation of features and ranks (floored at 1e-6)."""
    f = np.asarray(feats, dtype=np.float64)
    r = np.asarray(ranks, dtype=np.float64)
    return (f.mean(0), np.maximum(f.std(0), 1e-6), r.mean(), max(r.std(), 1e-6))


def forward(p, feats):
    """Network output on standardised features; returns (output, activations)."""
    w = unpack(p)
    z = (np.asarray(feats, dtype=np.float64) - w["fmean"]) / w["fstd"]
    h1 = np.maximum(z @ w["W1"].T + w["b1"], 0.0)
    h2 = np.maximum(h1 @ w["W2"].T + w["b2"], 0.0)
    h3 = np.maximum(h2 @ w["W3"].T + w["b3"], 0.0)
    o = (h3 @ w["W4"].T + w["b4"])[:, 0]
    return o, (z, h1, h2, h3)


def predict(p, feats):
    """Predicted rank: the output mapped back from standardised rank units."""
    w = unpack(p)
    o, _ = forward(p, feats)
    return o * w["rstd"] + w["rmean"]


def loss(p, feats, ranks):
    """Mean squared error between the output and the standardised ranks."""
    w = unpack(p)
    o, _ = forward(p, feats)
    t = (np.asarray(ranks, dtype=np.float64) - w["rmean"]) / w["rstd"]
    return float(np.mean((o - t) ** 2))


def grad(p, feats, ranks):
    """Gradient of `loss` with respect to the weights (reverse-mode chain rule).

    Returns a vector in the parameter layout; the standardisation entries are 0.
    """
    w = unpack(p)
    n = len(ranks)
    o, (z, h1, h2, h3) = forward(p, feats)
    t = (np.asarray(ranks, dtype=np.float64) - w["rmean"]) / w["rstd"]
    do = (2.0 / n) * (o - t)[:, None]              # n x 1
    g = {"W4": do.T @ h3, "b4": do.sum(0)}
    d3 = (do @ w["W4"]) * (h3 > 0)
    g["W3"], g["b3"] = d3.T @ h2, d3.sum(0)
    d2 = (d3 @ w["W3"]) * (h2 > 0)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ w["W2"]) * (h1 > 0)
    g["W1"], g["b1"] = d1.T @ z, d1.sum(0)
    g["fmean"], g["fstd"], g["rmean"], g["rstd"] = np.zeros(NF), np.zeros(NF), 0.0, 0.0
    return pack(g)


def adam_step(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One Adam update of the weights (standardisation entries untouched).

    step is the 1-based update count used in the bias corrections.
    """
    p = np.array(p, dtype=np.float64)
    m = np.array(m, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    k = NPARAM
    gk = np.asarray(g, dtype=np.float64)[:k] + weight_decay * p[:k]
    m[:k] = beta1 * m[:k] + (1 - beta1) * gk
    v[:k] = beta2 * v[:k] + (1 - beta2) * gk * gk
    mh = m[:k] / (1 - beta1 ** step)
    vh = v[:k] / (1 - beta2 ** step)
    p[:k] = p[:k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
