"""hmat_matvec_noalloc against hmat_matvec (same kernels, scratch in the library's
static device array instead of allocated memory): two calls in a row, the second
on a smaller input (fewer points, fewer vectors, the other direction and point
order), each bit-identical to hmat_matvec on the same input; and a request whose
scratch exceeds the static array is rejected before any work is enqueued."""

import numpy as np
import pytest

from workloads import fibonacci_sphere, jitter

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


def _dev(X, pad=0):
    import torch
    n, nv = X.shape
    d = torch.zeros((nv, n + pad), dtype=torch.float64, device="cuda")
    d[:, :n] = torch.from_numpy(X.T.copy()).cuda()
    return d


def test_noalloc_matches_matvec(H):
    import torch
    mats = []
    for n, leaf in ((2048, 32), (1500, 24)):
        t = H.hmat_build_tree(jitter(fibonacci_sphere(n), 1e-3, 6), leaf, 0.8, 0)
        A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
        B, _ = H.hmat_assemble(t, "exp", 1.0, 1.0, eps_in=1e-8)
        C, _ = H.hmat_multiply(A, B, 1e-6)
        mats.append((n, t, A, B, C))
    rng = np.random.default_rng(8)
    calls = [(mats[0][4], mats[0][0], 3, 0, 0, 4), (mats[1][2], mats[1][0], 1, 1, 1, 0)]
    for M, n, nv, trans, order, pad in calls:
        X = rng.standard_normal((n, nv))
        xd = _dev(X, pad)
        y_ref = torch.full((nv, n + pad), float("nan"), dtype=torch.float64, device="cuda")
        y_na = torch.full((nv, n + pad), float("nan"), dtype=torch.float64, device="cuda")
        H.hmat_matvec(M, xd.data_ptr(), n + pad, y_ref.data_ptr(), n + pad, nv, trans, order)
        H.hmat_matvec_noalloc(M, xd.data_ptr(), n + pad, y_na.data_ptr(), n + pad, nv, trans, order)
        torch.cuda.synchronize()
        a, b = y_ref.cpu().numpy(), y_na.cpu().numpy()
        print(f"[noalloc] n={n} nvec={nv} trans={trans} order={order}: bit-identical {np.array_equal(a[:, :n], b[:, :n])}",
              flush=True)
        assert np.array_equal(a[:, :n], b[:, :n]) and np.isfinite(b[:, :n]).all()
        assert np.isnan(b[:, n:]).all()
    # a scratch request above the static array is rejected, and nothing is written
    n, t, A, B, C = mats[0]
    ranks, offs, pool = H.hmat_export(C)
    nb = int(H.hmat_tree_info(t)["n_blocks"])
    ksum = int(ranks.sum())
    nv = (H.HMAT_MATVEC_NOALLOC_BYTES // 8 - nb) // max(ksum, 1) + 1
    X = np.ones((n, nv))
    xd = _dev(X)
    yd = torch.full((nv, n), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(H.HmatError) as e:
        H.hmat_matvec_noalloc(C, xd.data_ptr(), n, yd.data_ptr(), n, nv, 0, 1)
    assert e.value.code == H.HMAT_ERR_ARG and "static" in str(e.value)
    torch.cuda.synchronize()
    assert torch.isnan(yd).all().item()
    for n, t, A, B, C in mats:
        for h in (A, B, C):
            H.hmat_destroy(h)
        H.hmat_tree_destroy(t)
