"""GPU product vs the oracle's exact blocks (brute force, small n).

Farfield blocks: relative Frobenius error <= 1.01 eps and rank <= eps-rank + 2.
Nearfield blocks: relative error <= 1e-12. The oracle ingests the library's own
exported A and B, so input compression errors cancel out of the comparison.
"""

import numpy as np
import pytest

from workloads import fibonacci_sphere, jitter, cube_surface
from oracle.product import brute_force_product, check_block
from oracle.hmatrix import KIND_F
from tests.helpers import exported_to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1805_08998_amd import hmat
    hmat.lib()
    return hmat


def run_case(H, pts, leaf, split, ka, kb, eps, same=False, opts=None):
    t = H.hmat_build_tree(pts, leaf, 0.8, split)
    A, _ = H.hmat_assemble(t, *ka, eps_in=1e-8)
    B = A if same else H.hmat_assemble(t, *kb, eps_in=1e-8)[0]
    st = H.hmat_stats()
    o = opts or H.hmat_opts_default()
    import ctypes
    o.stats = ctypes.pointer(st)
    C, code = H.hmat_multiply(A, B, eps, o)
    Ao = exported_to_oracle(H, t, A)
    Bo = Ao if same else exported_to_oracle(H, t, B)
    Co = exported_to_oracle(H, t, C)
    P = brute_force_product(Ao, Bo)
    worst_f, worst_n, slack, nbad = 0.0, 0.0, -99, 0
    for lf in Co.leaves:
        D = P[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
        if lf.kind == KIND_F:
            r = check_block(D, KIND_F, eps, U=lf.L, V=lf.R)
            worst_f = max(worst_f, r.err)
            slack = max(slack, r.rank - r.kstar)
        else:
            r = check_block(D, 2, eps, Dc=lf.D)
            worst_n = max(worst_n, r.err)
        nbad += (not r.ok)
    for h in ([A, C] if same else [A, B, C]):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)
    print(f"far worst {worst_f:.3e} (eps {eps}), rank-k* max {slack}, near worst {worst_n:.3e}, "
          f"bad {nbad}, growth rounds {st.n_growth_rounds}, not conv {st.n_not_converged}", flush=True)
    return nbad, worst_f, worst_n, code


@pytest.mark.parametrize("name,n,leaf,split", [
    ("sphere2k-laplace", 2048, 32, 0),
    ("sphere1500-median", 1500, 24, 1),
])
def test_product_laplace_square(H, name, n, leaf, split):
    print(f"[product] {name}", flush=True)
    pts = fibonacci_sphere(n)
    nbad, wf, wn, code = run_case(H, pts, leaf, split, ("laplace_4pi", 1.0, 0.0), None, 1e-6, same=True)
    assert code == 0 and nbad == 0


def test_product_mixed_kernels(H):
    print("[product] jittered sphere 3000, laplace x (exp + I)", flush=True)
    pts = jitter(fibonacci_sphere(3000), 1e-3, 0)
    nbad, wf, wn, code = run_case(H, pts, 48, 0, ("laplace_4pi", 1.0, 0.0), ("exp", 1.0, 1.0), 1e-6)
    assert code == 0 and nbad == 0


def test_product_cube_eps4(H):
    print("[product] cube 2500, 1/r x exp, eps 1e-4", flush=True)
    pts = cube_surface(2500, 1)
    nbad, wf, wn, code = run_case(H, pts, 32, 0, ("inv_dist", 1.0, 0.0), ("exp", 1.0, 0.0), 1e-4)
    assert code == 0 and nbad == 0


def test_product_root_is_leaf(H):
    print("[product] n = 40 with leaf 64 (single dense block)", flush=True)
    pts = fibonacci_sphere(40)
    nbad, wf, wn, code = run_case(H, pts, 64, 0, ("exp", 1.0, 0.0), ("inv_dist", 1.0, 0.0), 1e-6)
    assert code == 0 and nbad == 0


def test_product_many_chunks(H):
    """A tiny workspace budget splits the targets into many chunks."""
    print("[product] sphere2k with a 4 MB workspace budget", flush=True)
    pts = fibonacci_sphere(2048)
    o = H.hmat_opts_default()
    o.workspace_limit = 4 << 20
    nbad, wf, wn, code = run_case(H, pts, 32, 0, ("laplace_4pi", 1.0, 0.0), None, 1e-6, same=True, opts=o)
    assert code == 0 and nbad == 0


@pytest.mark.slow
def test_product_sphere8k(H):
    print("[product] jittered sphere 8192, leaf 64, laplace x (exp + I)", flush=True)
    pts = jitter(fibonacci_sphere(8192), 1e-3, 0)
    nbad, wf, wn, code = run_case(H, pts, 64, 0, ("laplace_4pi", 1.0, 0.0), ("exp", 1.0, 1.0), 1e-6)
    assert code == 0 and nbad == 0


def test_product_duplicate_points(H):
    """Every point twice: zero-extent clusters (Def. 2.2 allows no split there)."""
    print("[product] 700 points, each twice, exp x exp", flush=True)
    import numpy as np
    p = fibonacci_sphere(700)
    pts = np.ascontiguousarray(np.concatenate([p, p]))
    nbad, wf, wn, code = run_case(H, pts, 32, 0, ("exp", 1.0, 0.0), ("exp", 1.0, 1.0), 1e-6)
    assert code == 0 and nbad == 0


def test_product_with_identity_and_zero(H):
    """A I = A and A 0 = 0 with I and 0 given as H-matrices on the same tree
    (rank-0 farfield leaves, dense identity or zero nearfield leaves)."""
    import numpy as np
    from oracle.hmatrix import HMatrix, Leaf, KIND_N
    from tests.helpers import oracle_to_blocks
    print("[product] sphere 2048: A I and A 0", flush=True)
    pts = fibonacci_sphere(2048)
    t = H.hmat_build_tree(pts, 32, 0.8, 0)
    A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-8)
    Ao = exported_to_oracle(H, t, A)
    for which in ("identity", "zero"):
        Io = HMatrix(n=Ao.n, perm=Ao.perm)
        for lf in Ao.leaves:
            if lf.kind == KIND_F:
                Io.leaves.append(Leaf(lf.r0, lf.m, lf.c0, lf.n, KIND_F, L=np.zeros((lf.m, 0)), R=np.zeros((lf.n, 0))))
            else:
                D = np.eye(lf.m) if (which == "identity" and lf.r0 == lf.c0 and lf.m == lf.n) else np.zeros((lf.m, lf.n))
                Io.leaves.append(Leaf(lf.r0, lf.m, lf.c0, lf.n, KIND_N, D=D))
        I = H.hmat_from_blocks(t, *oracle_to_blocks(Io))
        C, code = H.hmat_multiply(A, I, 1e-6)
        P = brute_force_product(Ao, exported_to_oracle(H, t, I))
        Co = exported_to_oracle(H, t, C)
        bad = 0
        for lf in Co.leaves:
            D = P[lf.r0:lf.r0 + lf.m, lf.c0:lf.c0 + lf.n]
            r = check_block(D, KIND_F, 1e-6, U=lf.L, V=lf.R) if lf.kind == KIND_F else check_block(D, 2, 1e-6, Dc=lf.D)
            bad += not r.ok
            if which == "zero":
                assert (lf.kind == KIND_F and lf.L.shape[1] == 0) or (lf.kind != KIND_F and not lf.D.any())
        print(f"A {which}: {bad} blocks outside the bound", flush=True)
        assert code == 0 and bad == 0
        H.hmat_destroy(C)
        H.hmat_destroy(I)
    H.hmat_destroy(A)
    H.hmat_tree_destroy(t)


@pytest.mark.parametrize("eps,precision", [(1e-6, 0), (1e-9, 0), (1e-6, 1)])
def test_sparse_passes_bit_identical(H, eps, precision):
    """A pass in which at most an eighth of a chunk's targets are active (growth rounds,
    the later identity panels of a chunk's widest targets) launches only their work items.
    The product equals, bit for bit, the one whose passes launch every work item."""
    import ctypes
    pts = jitter(fibonacci_sphere(8192), 1e-3, seed=11)
    t = H.hmat_build_tree(pts, 32, 0.8, 0)
    A, _ = H.hmat_assemble(t, "laplace_4pi", 1.0, 0.0, eps_in=1e-10)
    B, _ = H.hmat_assemble(t, "exp", 1.0, 1.0, eps_in=1e-10)
    out = []
    for full in (0, 1):
        st = H.hmat_stats()
        o = H.hmat_opts_default(full_passes=full, precision=precision)
        o.stats = ctypes.pointer(st)
        C, code = H.hmat_multiply(A, B, eps, o)
        assert code == 0
        out.append((H.hmat_export(C), st.n_passes, st.n_sparse_passes, st.n_growth_rounds, st.t_total))
        H.hmat_destroy(C)
    for h in (A, B):
        H.hmat_destroy(h)
    H.hmat_tree_destroy(t)
    (r0, o0, p0), n0, s0, g0, t0 = out[0]
    (r1, o1, p1), n1, s1, g1, t1 = out[1]
    print(f"eps {eps} precision {precision}: passes {n0} ({s0} sparse) vs {n1} ({s1}), growth rounds {g0}, "
          f"product {t0:.3f} s vs {t1:.3f} s", flush=True)
    assert s0 > 0 and s1 == 0 and n0 == n1
    assert np.array_equal(r0, r1) and np.array_equal(o0, o1)
    assert p0.tobytes() == p1.tobytes()
