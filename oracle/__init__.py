"""CPU oracle for the hierarchical-matrix product (test infrastructure only).

A plain, slow, float64 implementation of what the product path computes,
written from the paper (Doelz, Harbrecht, Multerer, "On the best approximation
of the hierarchical matrix product"). It shares no code with the HIP library.
Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py`
may import it; the library never calls into it.

Modules:
  tree      cluster tree, admissibility, block-cluster tree (Section 2)
  kernels   kernel-matrix entries of the synthetic workloads
  hmatrix   H-matrix container, densification, H-matrix-vector product
  assemble  input compression by per-block truncated SVD
  product   brute-force product, strip oracle, best approximation, acceptance
  sumexpr   sum-expressions, restriction and the recursive product (Section 3)
  mlp       float64 reference of the rank-predictor network
"""
