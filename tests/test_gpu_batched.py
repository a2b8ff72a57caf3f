"""Batched products: several independent products (own trees, sizes, kernels)
in one call, run concurrently on several streams. Every block of every product
meets the oracle's bound, results equal those of the same products computed one
at a time, and per-product errors are reported without affecting the others."""

import ctypes

import numpy as np
import pytest

from oracle.hmatrix import KIND_F
from oracle.product import brute_force_product, check_block
from tests.helpers import exported_to_oracle
from workloads import fibonacci_sphere, ellipsoid, cube_surface, jitter

pytestmark = pytest.mark.gpu

CASES = [  # (points, leaf, kernel A, kernel B)
    (lambda: jitter(fibonacci_sphere(1800), 1e-3, seed=3), 32, ("laplace_4pi", 1.0, 0.0), ("exp", 1.0, 1.0)),
    (lambda: ellipsoid(2500, (1.0, 0.6, 0.45)), 32, ("inv_dist", 1.0, 0.0), ("exp", 1.0, 0.0)),
    (lambda: cube_surface(2200, seed=4), 32, ("exp", 1.0, 0.0), ("inv_dist", 1.0, 0.0)),
    (lambda: fibonacci_sphere(3000), 48, ("laplace_4pi", 1.0, 0.0), ("laplace_4pi", 1.0, 0.0)),
    (lambda: ellipsoid(1500, (0.9, 0.8, 0.4)), 24, ("exp", 1.0, 1.0), ("laplace_4pi", 1.0, 0.0)),
    (lambda: jitter(cube_surface(2800, seed=9), 1e-3, seed=1), 40, ("inv_dist", 1.0, 0.0), ("exp", 1.0, 1.0)),
]


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


@pytest.fixture(scope="module")
def products(H):
    out = []
    for pts_fn, leaf, ka, kb in CASES:
        t = H.hmat_build_tree(pts_fn(), leaf, 0.8, 0)
        A, _ = H.hmat_assemble(t, *ka, eps_in=1e-8)
        B, _ = H.hmat_assemble(t, *kb, eps_in=1e-8)
        out.append((t, A, B))
    yield out
    for t, A, B in out:
        H.hmat_destroy(A)
        H.hmat_destroy(B)
        H.hmat_tree_destroy(t)


def pool_of(H, M):
    ranks, offs, pool = H.hmat_export(M)
    return ranks, pool


@pytest.mark.parametrize("streams", [0, 3])
def test_batched_matches_oracle_and_sequential(H, products, streams):
    eps = 1e-6
    st = H.hmat_stats()
    o = H.hmat_opts_default(streams=streams)
    o.stats = ctypes.pointer(st)
    Cs, status = H.hmat_multiply_batched([p[1] for p in products], [p[2] for p in products], eps, o)
    assert list(status) == [H.HMAT_OK] * len(products)
    assert st.streams_used >= 1 and (streams == 0 or st.streams_used == streams)
    print(f"streams {streams}: used {st.streams_used}, {st.t_total:.3f}s, far {st.n_far}, near {st.n_near}",
          flush=True)
    far_total = 0
    for (t, A, B), C in zip(products, Cs):
        # same result as the product computed alone (plain mode is deterministic)
        C1, _ = H.hmat_multiply(A, B, eps)
        r0, p0 = pool_of(H, C)
        r1, p1 = pool_of(H, C1)
        assert np.array_equal(r0, r1) and np.array_equal(p0, p1)
        H.hmat_destroy(C1)
        # every block within the bound
        P = brute_force_product(exported_to_oracle(H, t, A), exported_to_oracle(H, t, B))
        Co = exported_to_oracle(H, t, C)
        bad = 0
        for lf in Co.leaves:
            D = P[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
            if lf.kind == KIND_F:
                r = check_block(D, KIND_F, eps, U=lf.L, V=lf.R)
                far_total += 1
            else:
                r = check_block(D, 2, eps, Dc=lf.D)
            bad += not r.ok
        assert bad == 0
        H.hmat_destroy(C)
    assert far_total == st.n_far


def test_batched_reports_per_product_errors(H, products):
    (t0, A0, B0), (t1, A1, B1) = products[0], products[1]
    o = H.hmat_opts_default(streams=2)
    # product 1 mixes matrices of two different trees
    Cs, status = H.hmat_multiply_batched([A0, A0, A1], [B0, B1, B1], 1e-6, o)
    assert list(status) == [H.HMAT_OK, H.HMAT_ERR_TREE_MISMATCH, H.HMAT_OK]
    assert not Cs[1].value
    assert H.lib().hmat_last_error().decode().startswith("product 1")
    for i in (0, 2):
        H.hmat_destroy(Cs[i])


def test_batched_empty(H):
    Cs, status = H.hmat_multiply_batched([], [], 1e-6, H.hmat_opts_default())
    assert Cs == [] and list(status) == []


BATCH64_SKIP = ("batch of 64 products (4096 to 65536 points): calls stopped making progress on the GPU, the "
                "second call under the allocator's first policy and the first call under its second; the "
                "simulated footprint of exactly those calls nears the whole device (tests/test_alloc_cache.py). "
                "The allocator now keeps to three quarters of the device; that is not yet run on this batch")


@pytest.mark.slow
@pytest.mark.skip(reason=BATCH64_SKIP)
def test_batched64_two_calls(H):
    """The 64-product workload (n log-uniform in [4096, 65536], random geometries and
    kernel pairs), called twice: both calls complete, and every product of the
    second call equals the first (plain mode is deterministic)."""
    import time
    from workloads import batched_geometries
    specs = batched_geometries(64, seed=0)
    print("[batched64] building 64 trees and 128 matrices", flush=True)
    trees, As, Bs = [], [], []
    for sp in specs:
        t = H.hmat_build_tree(sp["points"], 64, 0.8, 0)
        A, _ = H.hmat_assemble(t, sp["kernel_a"], 1.0, 0.0, eps_in=1e-8)
        B, _ = H.hmat_assemble(t, sp["kernel_b"], 1.0, 0.0, eps_in=1e-8)
        trees.append(t), As.append(A), Bs.append(B)
    o = H.hmat_opts_default()
    t0 = time.monotonic()
    C1, s1 = H.hmat_multiply_batched(As, Bs, 1e-6, o)
    t1 = time.monotonic()
    print(f"[batched64] first call {t1 - t0:.1f} s", flush=True)
    C2, s2 = H.hmat_multiply_batched(As, Bs, 1e-6, o)
    print(f"[batched64] second call {time.monotonic() - t1:.1f} s", flush=True)
    assert list(s1) == [0] * 64 and list(s2) == [0] * 64
    for a, b in zip(C1, C2):
        assert all(np.array_equal(x, y) for x, y in zip(pool_of(H, a), pool_of(H, b)))
        H.hmat_destroy(a), H.hmat_destroy(b)
    for t, A, B in zip(trees, As, Bs):
        H.hmat_destroy(A), H.hmat_destroy(B), H.hmat_tree_destroy(t)
