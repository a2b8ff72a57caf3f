"""Parity at the full workload sizes, in the configuration bench.py times.

At n = 65536 and n = 262144 the oracle cannot form the whole product, so a
stratified sample of leaves is checked: per level and kind a few random leaves of
at most 256 rows, plus the largest farfield leaf of the level up to 2048 rows
(65536 points) or 1024 rows (262144 points). Each exact block
A_H[tau, :] B_H[:, sigma] is built from densified strips of the library's own A_H
and B_H, with the inner dimension in pieces so that host memory stays bounded, and
compared with C's block (farfield: error <= 1.01 eps and rank <= eps-rank + 2;
nearfield: error <= 1e-12).

Cases: plain float64 at both sizes; learned widths at 262144 points (model trained
on the 65536-point sphere's plain ranks, as bench.py does); the 262144-point
ellipsoid (axes 1, 0.7, 0.5) with float32 sketch panels at eps = 1e-4 and 1e-6,
whose errors are reported (max, p99, median of error / eps) and gated like float64."""

import ctypes

import numpy as np
import pytest

from tests.helpers import sampled_check
from workloads import CONFIGS

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


def build(H, name):
    w = CONFIGS[name]
    t = H.hmat_build_tree(w.points(), w.leaf, w.eta, w.split)
    A, _ = H.hmat_assemble(t, w.kernel_a.kind, w.kernel_a.diag, w.kernel_a.shift, w.eps_in)
    B, _ = H.hmat_assemble(t, w.kernel_b.kind, w.kernel_b.diag, w.kernel_b.shift, w.eps_in)
    return w, t, A, B


def check(H, w, t, A, B, C, st, label, eps=None):
    eps = w.eps if eps is None else eps
    big = 2048 if w.n <= 65536 else 1024
    res = sampled_check(H, t, A, B, C, eps, per_level=2 if w.n <= 65536 else 1, max_rows=256, seed=1,
                        largest_rows=big, log=lambda s: print(s, flush=True))
    bad = [r for r in res if not r[-1]]
    far = np.array([r[4] for r in res if r[1] == 1]) / eps
    rows = max(r[2] for r in res if r[1] == 1)
    print(f"{label}: {len(res)} sampled blocks (largest farfield {rows} rows), {len(bad)} outside the bound; "
          f"farfield error/eps max {far.max():.3f} p99 {np.percentile(far, 99):.3f} median {np.median(far):.3f}; "
          f"growth rounds {st.n_growth_rounds}, not converged {st.n_not_converged}", flush=True)
    assert st.n_not_converged == 0
    assert len(res) >= 10 and not bad
    assert rows > 256  # the large targets were reached


def run(H, A, B, eps, **kw):
    st = H.hmat_stats()
    o = H.hmat_opts_default(**kw)
    o.stats = ctypes.pointer(st)
    C, code = H.hmat_multiply(A, B, eps, o, allow_not_converged=True)
    assert code == H.HMAT_OK
    return C, st


@pytest.mark.parametrize("name", ["sphere64k", "sphere256k"])
def test_fullsize_plain(H, name):
    print(f"[fullsize] {name} plain", flush=True)
    w, t, A, B = build(H, name)
    C, st = run(H, A, B, w.eps)
    check(H, w, t, A, B, C, st, f"{name} plain")
    for h in (A, B, C):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)


def _train_on_sphere64k(H):
    w, t, A, B = build(H, "sphere64k")
    C0, _ = run(H, A, B, w.eps)
    f, r = H.hmat_product_features(C0)
    for h in (A, B, C0):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)
    m = H.hmat_rank_model_create(1)
    H.hmat_rank_model_train(m, f, r, H.hmat_train_opts_default(epochs=20, batch=512, lr=2e-3))
    return m


def test_fullsize_learned_and_fp32_64k(H):
    """Learned widths and the fp32 sketch at n = 65536."""
    print("[fullsize] sphere64k learned + fp32 apply", flush=True)
    m = _train_on_sphere64k(H)
    w, t, A, B = build(H, "sphere64k")
    for label, kw in (("learned", dict(rank_mode=H.HMAT_RANK_PREDICT, rank_model=m)),
                      ("fp32 apply", dict(precision=H.HMAT_FP32_APPLY))):
        C, st = run(H, A, B, w.eps, **kw)
        check(H, w, t, A, B, C, st, f"sphere64k {label}")
        H.hmat_destroy(C)
    H.hmat_rank_model_destroy(m)
    for h in (A, B):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)


def test_fullsize_learned_256k(H):
    """The headline configuration: learned widths on the 262144-point sphere."""
    print("[fullsize] sphere256k learned (model from the 65536-point sphere)", flush=True)
    m = _train_on_sphere64k(H)
    w, t, A, B = build(H, "sphere256k")
    C, st = run(H, A, B, w.eps, rank_mode=H.HMAT_RANK_PREDICT, rank_model=m)
    check(H, w, t, A, B, C, st, "sphere256k learned")
    for h in (A, B, C):
        H.hmat_destroy(h)
    H.hmat_rank_model_destroy(m)
    H.hmat_tree_destroy(t)


def test_fullsize_ellipsoid_fp32(H):
    """The 262144-point ellipsoid with float32 sketch panels at eps = 1e-4 and 1e-6."""
    print("[fullsize] ellipsoid256k fp32 apply", flush=True)
    w, t, A, B = build(H, "ellipsoid256k")
    for eps in (1e-4, 1e-6):
        C, st = run(H, A, B, eps, precision=H.HMAT_FP32_APPLY)
        check(H, w, t, A, B, C, st, f"ellipsoid256k fp32 eps={eps:g}", eps=eps)
        H.hmat_destroy(C)
    for h in (A, B):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)
