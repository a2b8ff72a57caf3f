"""Mixed precision (HMAT_FP32_APPLY): the sketch and probe passes read float32
copies of the panels; projection, core and truncation stay float64.

The error of every block against the exact float64 product is reported (max,
99th percentile and median of error / eps, and rank - eps-rank). The gates are
loose on purpose: the float32 panels perturb S by about 1e-7 relative, which
the float64 projection and the kappa margin of the truncation absorb, so the
bound 1.01 eps is expected to hold at eps = 1e-4 and to hold for nearly every
block at eps = 1e-6."""

import ctypes

import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def case(H):
    pts = jitter(fibonacci_sphere(4096), 1e-3, seed=5)
    t = H.hmat_build_tree(pts, 32, 0.8, 0)
    A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
    B, _ = H.hmat_assemble(t, "exp", 1.0, 1.0, eps_in=1e-8)
    P = brute_force_product(exported_to_oracle(H, t, A), exported_to_oracle(H, t, B))
    yield t, A, B, P
    H.hmat_destroy(A)
    H.hmat_destroy(B)
    H.hmat_tree_destroy(t)


def errors(H, t, C, P, eps):
    far, slack, near = [], [], []
    for lf in exported_to_oracle(H, t, C).leaves:
        D = P[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
        if lf.kind == KIND_F:
            r = check_block(D, KIND_F, eps, U=lf.L, V=lf.R)
            far.append(r.err / eps)
            slack.append(r.rank - r.kstar)
        else:
            near.append(check_block(D, 2, eps, Dc=lf.D).err)
    return np.array(far), np.array(slack), np.array(near)


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_fp32_apply_errors(H, case, eps):
    t, A, B, P = case
    st = H.hmat_stats()
    o = H.hmat_opts_default(precision=H.HMAT_FP32_APPLY)
    o.stats = ctypes.pointer(st)
    C, code = H.hmat_multiply(A, B, eps, o, allow_not_converged=True)
    far, slack, near = errors(H, t, C, P, eps)
    H.hmat_destroy(C)
    print(f"fp32 apply, eps {eps}: error/eps max {far.max():.4f} p99 {np.percentile(far, 99):.4f} "
          f"median {np.median(far):.4f}; rank - k* max {slack.max()} p99 {np.percentile(slack, 99):.0f}; "
          f"nearfield max {near.max():.2e}; growth rounds {st.n_growth_rounds}, not converged "
          f"{st.n_not_converged}", flush=True)
    assert code == H.HMAT_OK and st.n_not_converged == 0
    assert near.max() <= 1e-12  # the nearfield is evaluated in float64
    assert np.median(far) <= 1.01
    if eps >= 1e-4:
        assert far.max() <= 1.01 and slack.max() <= 2
    else:
        assert far.max() <= 1.5 and np.mean(far > 1.01) <= 0.01 and np.percentile(slack, 99) <= 2


def test_fp32_apply_close_to_fp64(H, case):
    """The float32 sketch changes the basis, not the quality: ranks agree with the
    float64 product to within one on almost every block."""
    t, A, B, P = case
    C64, _ = H.hmat_multiply(A, B, 1e-6)
    C32, _ = H.hmat_multiply(A, B, 1e-6, H.hmat_opts_default(precision=H.HMAT_FP32_APPLY),
                             allow_not_converged=True)
    r64, _, _ = H.hmat_export(C64)
    r32, _, _ = H.hmat_export(C32)
    assert np.mean(np.abs(r64.astype(int) - r32.astype(int)) <= 1) >= 0.99
    H.hmat_destroy(C64)
    H.hmat_destroy(C32)


def test_bf16_sketch_rejected(H, case):
    t, A, B, P = case
    with pytest.raises(H.HmatError) as e:
        H.hmat_multiply(A, B, 1e-4, H.hmat_opts_default(precision=H.HMAT_BF16_SKETCH))
    assert e.value.code == H.HMAT_ERR_ARG
