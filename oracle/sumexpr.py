"""Sum-expressions and the recursive product (oracle, small n).

Section 3 of the paper: a sum-expression S(tau, sigma) = S_R + S_H holds a list
of low-rank matrices A_j B_j^T (S_R) and a list of pairs of H-matrix blocks
(H[tau, rho_j], K[rho_j, sigma]) (S_H) (Def. 3.1). Restriction to a son
tau' x sigma' (Algorithm 3) restricts every low-rank term by index shift and
splits every pair over the sons rho' of rho; a pair with an admissible factor is
multiplied out into a low-rank term, a pair of two inadmissible factors stays a
pair. Algorithm 4 recurses from S(I, I) = {(H, K)} and, at a leaf, truncates
(farfield) or evaluates (nearfield).

Readings:
  * Def. 3.1 and the proof of Lemma 5.1 print H where K is meant in places; the
    pair is (H[tau, rho], K[rho, sigma]).
  * When rho is a leaf cluster (tau and sigma are not), Algorithm 3's loop over
    sons(rho) is empty. Then tau x rho and rho x sigma are both nearfield leaves;
    the pair is kept with rho' = rho as the product of the row restriction of
    H[tau, rho] and the column restriction of K[rho, sigma], entered as a
    low-rank term of rank #rho. `drop_leaf_rho=True` drops it instead (only for
    the test that shows the reading matters).
  * Truncation of a farfield sum-expression uses the dense SVD of S applied to
    the identity, the reference operator of the numerical-examples section.
Dense sub-blocks of the factors are read from their densified matrices, which
restricts this module to small n.
"""

import numpy as np

from .assemble import truncate
from .hmatrix import HMatrix, Leaf, KIND_F as H_F, KIND_N as H_N
from .tree import BlockTree, KIND_F, KIND_N, KIND_INNER


def build_sum_expressions(A: HMatrix, B: HMatrix, bt: BlockTree, drop_leaf_rho: bool = False):
    """Runs Algorithm 3 from the root over the whole block tree. Returns a dict
    block id -> (list of (L, R) low-rank terms, list of rho cluster ids)."""
    ct = bt.ct
    Ad = A.to_dense(1)
    Bd = B.to_dense(1)
    beg, siz = ct.begin, ct.size

    def rng(c):
        return slice(int(beg[c]), int(beg[c] + siz[c]))

    def lowrank_of(Mdense, M: HMatrix, blk):
        """Stored factors of a farfield leaf of M (by block id)."""
        key = (int(beg[bt.tau[blk]]), int(siz[bt.tau[blk]]), int(beg[bt.sigma[blk]]), int(siz[bt.sigma[blk]]))
        lf = M._leaf_by_key[key]
        return lf.L, lf.R

    for M in (A, B):
        M._leaf_by_key = {(lf.r0, lf.m, lf.c0, lf.n): lf for lf in M.leaves}

    S = {0: ([], [0])}  # root: S_H(I, I) = {(A, B)} with rho = I
    order = np.argsort(bt.level, kind="stable")
    for b in order:
        if bt.kind[b] != KIND_INNER:
            continue
        R_par, H_par = S[b]
        for c in bt.children[b]:
            t2, s2 = int(bt.tau[c]), int(bt.sigma[c])
            r_off = int(beg[t2] - beg[bt.tau[b]])
            c_off = int(beg[s2] - beg[bt.sigma[b]])
            # S_R restriction: index shift of every low-rank term
            R_new = [(L[r_off:r_off + siz[t2]], R[c_off:c_off + siz[s2]]) for (L, R) in R_par]
            H_new = []
            for rho in H_par:
                kids = ct.children[rho]
                if not kids:
                    if drop_leaf_rho:
                        continue
                    # both factors are nearfield leaves; keep their restricted product
                    R_new.append((Ad[rng(t2), rng(rho)], Bd[rng(rho), rng(s2)].T))
                    continue
                for r2 in kids:
                    b1 = bt.lookup[(t2, r2)]
                    b2 = bt.lookup[(r2, s2)]
                    f1 = bt.kind[b1] == KIND_F
                    f2 = bt.kind[b2] == KIND_F
                    if f1 and f2:
                        La, Ra = lowrank_of(Ad, A, b1)
                        Lb, Rb = lowrank_of(Bd, B, b2)
                        R_new.append((La @ (Ra.T @ Lb), Rb))
                    elif f1:
                        La, Ra = lowrank_of(Ad, A, b1)
                        K = Bd[rng(r2), rng(s2)]
                        R_new.append((La, K.T @ Ra))
                    elif f2:
                        Lb, Rb = lowrank_of(Bd, B, b2)
                        Hm = Ad[rng(t2), rng(r2)]
                        R_new.append((Hm @ Lb, Rb))
                    else:
                        H_new.append(r2)
            S[c] = (R_new, H_new)
    S["_dense"] = (Ad, Bd)
    return S


def apply_identity(S, bt: BlockTree, blk: int) -> np.ndarray:
    """S(tau, sigma) applied to the identity of size #sigma: the dense block."""
    ct = bt.ct
    Ad, Bd = S["_dense"]
    t, s = int(bt.tau[blk]), int(bt.sigma[blk])
    m, n = int(ct.size[t]), int(ct.size[s])
    D = np.zeros((m, n))
    R_terms, H_terms = S[blk]
    for L, R in R_terms:
        D += L @ R.T
    tb, sb = int(ct.begin[t]), int(ct.begin[s])
    for rho in H_terms:
        rb, rs = int(ct.begin[rho]), int(ct.size[rho])
        D += Ad[tb:tb + m, rb:rb + rs] @ Bd[rb:rb + rs, sb:sb + n]
    return D


def hmult(A: HMatrix, B: HMatrix, bt: BlockTree, eps: float, drop_leaf_rho: bool = False) -> HMatrix:
    """Algorithm 4 with dense-SVD truncation at farfield leaves."""
    S = build_sum_expressions(A, B, bt, drop_leaf_rho)
    ct = bt.ct
    C = HMatrix(n=A.n, perm=A.perm.copy())
    for b in bt.leaves():
        D = apply_identity(S, bt, b)
        t, s = int(bt.tau[b]), int(bt.sigma[b])
        r0, m, c0, n = int(ct.begin[t]), int(ct.size[t]), int(ct.begin[s]), int(ct.size[s])
        if bt.kind[b] == KIND_F:
            L, R, _, _ = truncate(D, eps)
            C.leaves.append(Leaf(r0, m, c0, n, H_F, L=L, R=R, level=int(bt.level[b])))
        else:
            C.leaves.append(Leaf(r0, m, c0, n, H_N, D=D, level=int(bt.level[b])))
    return C
