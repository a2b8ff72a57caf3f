"""Parity at the full workload sizes, in the configuration bench.py times.

At n = 65536 and n = 262144 the oracle cannot form the whole product, so a
stratified sample of leaves (per level and kind, at most 256 rows) is checked:
each exact block A_H[tau, :] B_H[:, sigma] is built from densified strips of the
library's own A_H and B_H and compared with C's block (farfield: error <= 1.01
eps and rank <= eps-rank + 2; nearfield: error <= 1e-12)."""

import ctypes

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


def check(H, w, t, A, B, C, st, label):
    res = sampled_check(H, t, A, B, C, w.eps, per_level=2 if w.n <= 65536 else 1, max_rows=256, seed=1,
                        log=lambda s: print(s, flush=True))
    bad = [r for r in res if not r[-1]]
    print(f"{label}: {len(res)} sampled blocks, {len(bad)} outside the bound; growth rounds "
          f"{st.n_growth_rounds}, not converged {st.n_not_converged}", flush=True)
    assert st.n_not_converged == 0
    assert len(res) >= 10 and not bad


@pytest.mark.parametrize("name", ["sphere64k", "sphere256k"])
def test_fullsize_plain(H, name):
    print(f"[fullsize] {name} plain", flush=True)
    w, t, A, B = build(H, name)
    st = H.hmat_stats()
    o = H.hmat_opts_default()
    o.stats = ctypes.pointer(st)
    C, code = H.hmat_multiply(A, B, w.eps, o, allow_not_converged=True)
    assert code == H.HMAT_OK
    check(H, w, t, A, B, C, st, f"{name} plain")
    for h in (A, B, C):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)


def test_fullsize_learned_and_fp32_64k(H):
    """Learned widths (model trained on this product's own plain ranks) and the
    fp32 sketch at n = 65536; the fp32 errors are reported and gated like fp64 here."""
    print("[fullsize] sphere64k learned + fp32 apply", flush=True)
    w, t, A, B = build(H, "sphere64k")
    st0 = H.hmat_stats()
    o = H.hmat_opts_default()
    o.stats = ctypes.pointer(st0)
    C0, _ = H.hmat_multiply(A, B, w.eps, o)
    f, r = H.hmat_product_features(C0)
    H.hmat_destroy(C0)
    m = H.hmat_rank_model_create(1)
    H.hmat_rank_model_train(m, f, r, H.hmat_train_opts_default(epochs=20, batch=512, lr=2e-3))
    for label, kw in (("learned", dict(rank_mode=H.HMAT_RANK_PREDICT, rank_model=m)),
                      ("fp32 apply", dict(precision=H.HMAT_FP32_APPLY))):
        st = H.hmat_stats()
        o = H.hmat_opts_default(**kw)
        o.stats = ctypes.pointer(st)
        C, code = H.hmat_multiply(A, B, w.eps, o, allow_not_converged=True)
        check(H, w, t, A, B, C, st, f"sphere64k {label}")
        H.hmat_destroy(C)
    H.hmat_rank_model_destroy(m)
    for h in (A, B):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)
