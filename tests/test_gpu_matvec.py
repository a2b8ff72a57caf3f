"""H-matrix times vectors on the GPU (Algorithm 2) against the oracle.

y = M x and y = M^T x for the library's assembled A and a product C = A B,
n = 2048 (leaf 32) and n = 1500 (leaf 24, median split), in both point orders,
with 1, 3 and 17 vectors and padded leading dimensions. The reference is the
oracle's densification of the library's exported leaves times x (float64): the
two differ only by summation order (1e-13 relative). Argument errors are
checked, and the output is deterministic (two calls bit-identical)."""

import numpy as np
import pytest

from tests.helpers import exported_to_oracle
from workloads import fibonacci_sphere, jitter

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


@pytest.fixture(scope="module")
def mats(H):
    out = []
    for n, leaf, split in ((2048, 32, 0), (1500, 24, 1)):
        pts = jitter(fibonacci_sphere(n), 1e-3, 5)
        t = H.hmat_build_tree(pts, leaf, 0.8, split)
        A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
        B, _ = H.hmat_assemble(t, "exp", 1.0, 1.0, eps_in=1e-8)
        C, _ = H.hmat_multiply(A, B, 1e-6)
        out.append((n, t, A, B, C))
    yield out
    for n, t, A, B, C in out:
        for h in (A, B, C):
            H.hmat_destroy(h)
        H.hmat_tree_destroy(t)


def _matvec(H, M, X, trans, order, pad=0):
    import torch
    n, nv = X.shape
    xd = torch.zeros((nv, n + pad), dtype=torch.float64, device="cuda")
    xd[:, :n] = torch.from_numpy(X.T.copy()).cuda()
    yd = torch.full((nv, n + pad + 3), float("nan"), dtype=torch.float64, device="cuda")
    H.hmat_matvec(M, xd.data_ptr(), n + pad, yd.data_ptr(), n + pad + 3, nv, trans, order)
    torch.cuda.synchronize()
    Y = yd.cpu().numpy()
    assert np.isnan(Y[:, n:]).all()  # padding untouched
    return Y[:, :n].T.copy()


@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("order", [0, 1])
def test_matvec_matches_dense(H, mats, trans, order):
    rng = np.random.default_rng(10 + 2 * trans + order)
    for n, t, A, B, C in mats:
        for name, M in (("A", A), ("C", C)):
            D = exported_to_oracle(H, t, M).to_dense(order)
            Op = D.T if trans else D
            for nv, pad in ((1, 0), (3, 5), (17, 0)):
                X = rng.standard_normal((n, nv))
                Y = _matvec(H, M, X, trans, order, pad)
                ref = Op @ X
                err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
                assert err <= 1e-13, (n, name, nv, err)
            print(f"[matvec] n={n} {name} trans={trans} order={order}: ok", flush=True)


def test_matvec_deterministic_and_errors(H, mats):
    import torch
    import paper_1805_08998_amd.hmat as HM
    n, t, A, B, C = mats[0]
    X = np.random.default_rng(3).standard_normal((n, 4))
    Y1 = _matvec(H, C, X, 0, 0)
    Y2 = _matvec(H, C, X, 0, 0)
    assert np.array_equal(Y1, Y2)
    xd = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    yd = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    L = HM.lib()
    p = lambda a: __import__("ctypes").c_void_p(a)
    ok = L.hmat_matvec(A, 0, 1, 2, p(xd.data_ptr()), n, p(yd.data_ptr()), n, None)
    assert ok == H.HMAT_OK
    for args in ((2, 1, 2, xd.data_ptr(), n, yd.data_ptr(), n),      # trans
                 (0, 2, 2, xd.data_ptr(), n, yd.data_ptr(), n),      # order
                 (0, 1, 0, xd.data_ptr(), n, yd.data_ptr(), n),      # nvec
                 (0, 1, 2, xd.data_ptr(), n - 1, yd.data_ptr(), n),  # ldx
                 (0, 1, 2, xd.data_ptr(), n, xd.data_ptr() + 8, n),  # overlap
                 (0, 1, 2, 0, n, yd.data_ptr(), n)):                 # NULL
        tr, od, nv, xp, lx, yp, ly = args
        assert L.hmat_matvec(A, tr, od, nv, p(xp), lx, p(yp), ly, None) == H.HMAT_ERR_ARG
    torch.cuda.synchronize()


def test_error_estimate_matches_oracle(H, mats):
    """hmat_error_estimate against the oracle's subspace iteration from the same start
    block: same operator products, same iteration, so the estimates agree to rounding;
    and the estimated relative error of C = A B at eps = 1e-6 is of order eps."""
    import torch
    from oracle.product import product_error_estimate
    for n, t, A, B, C in mats:
        p, iters = 12, 4
        X0 = np.random.default_rng(21).standard_normal((n, p))
        xd = torch.from_numpy(X0.T.copy()).cuda()
        err, nrm = H.hmat_error_estimate(C, A, B, xd.data_ptr(), p, iters)
        Ao, Bo, Co = (exported_to_oracle(H, t, M) for M in (A, B, C))
        err_o, nrm_o = product_error_estimate(Co, Ao, Bo, X0, iters)
        print(f"[estimate] n={n}: err {err:.6e} (oracle {err_o:.6e}), norm {nrm:.6e} (oracle {nrm_o:.6e}), "
              f"relative {err / nrm:.3e}", flush=True)
        assert abs(nrm - nrm_o) <= 1e-10 * nrm_o
        assert abs(err - err_o) <= 1e-6 * err_o + 1e-14 * nrm_o
        assert 0 < err / nrm <= 1.05e-6
    # argument errors
    n, t, A, B, C = mats[0]
    n2, t2, A2, B2, C2 = mats[1]
    xd = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    with pytest.raises(H.HmatError) as e:
        H.hmat_error_estimate(C, A, B2, xd.data_ptr(), 2, 1)
    assert e.value.code == H.HMAT_ERR_TREE_MISMATCH
    for p, it in ((0, 1), (n + 1, 1), (2, -1), (2, 101)):
        with pytest.raises(H.HmatError) as e:
            H.hmat_error_estimate(C, A, B, xd.data_ptr(), p, it)
        assert e.value.code == H.HMAT_ERR_ARG
