"""The paper's other low-rank schemes, applied to one exact target block (oracle).

Section 4 approximates a target block A = S(tau, sigma) through products with
vectors only. Besides the adaptive randomized range finder (the default path),
it lists:

  * adaptive cross approximation with partial pivoting (Algorithm 6);
  * Golub-Kahan-Lanczos bidiagonalization with reorthogonalization (Algorithm 7);
  * the randomized rank-k approximation with q subspace iterations (Algorithm 9),
    the fixed-rank form of the randomized scheme;
and Section 3 uses the SVD of a low-rank matrix (Algorithm 5) to truncate a sum
of low-rank terms exactly.

Every function here takes the exact dense block D (from the oracle's own
sum-expressions, or from strips of the densified factors) and runs the scheme on
it with plain numpy in float64, step by step in the paper's order. The library
touches S only through S X and S^T X; on D these products are plain GEMVs, so
the two must agree up to rounding wherever the scheme's integer decisions
(pivots, stopping step, kept rank) agree.

Readings (the paper is silent on these):
  * ACA starts at row 0. The next row pivot is the row of largest modulus of the
    newest column l_r among the rows not used yet (first index on ties); the
    column pivot is the first index of largest modulus of the residual row (the
    partial pivoting the paper describes).
  * A residual row that is exactly zero ends ACA (the Schur complement has no
    pivot left in that row).
  * Stopping (eq. (truncaca)): step r is computed, and ACA / Lanczos stop when
    the norm of its update is at most eps times the Frobenius norm of the
    approximation built by the previous steps. The update of that step is
    discarded, as in the paper; its squared norm e2 is the error proxy.
    For Lanczos the update of step r is alpha_r q_r w_r^T + beta_{r-1} q_{r-1}
    w_r^T, of norm sqrt(alpha_r^2 + beta_{r-1}^2); the approximation of k steps
    is Q_k B_k W_k^T with the k x k upper bidiagonal B_k.
  * Final recompression (the epsilon-rank of the numerical examples): the
    approximation is brought to SVD form (Algorithm 5 for ACA's L U^T, the SVD of
    B_k for Lanczos) and truncated to the smallest rank k' with
    tail(k')^2 <= eps^2 ||approximation||_F^2 - e2, so that truncation and the
    discarded update together stay within eps (same split of the error budget as
    the randomized path's truncation rule).
  * Fixed-rank mode (k_fixed > 0, the "fixed rank" experiments): ACA and Lanczos
    stop when k_fixed steps are kept (no eps test); the randomized scheme draws
    k_fixed Gaussian columns. There is no truncation in fixed-rank mode.
  * Orthonormalization in Algorithm 9 is a thin QR of the columns.
  * The Lanczos start vector is column 0 of the shared Gaussian matrix Omega
    (rows = the positions of sigma), normalised; Algorithm 9 uses columns
    0 .. k-1 of Omega (see philox.py for the generator).
  * Steps are capped at kcap and at min(m, n). A block whose adaptive
    iteration reaches kcap < min(m, n) without meeting the stopping test is
    reported as not converged.
"""

from dataclasses import dataclass

import numpy as np

from .assemble import eps_rank


@dataclass
class SchemeResult:
    L: np.ndarray       # m x k
    R: np.ndarray       # n x k, block ~= L R^T
    steps: int          # iterations kept before recompression
    converged: bool
    e2: float           # squared norm of the discarded update (error proxy)


def _truncate_svd(P, Qr, M, eps, e2, fixed):
    """SVD of the small core M, truncation by tail^2 <= eps^2 ||M||^2 - e2 (none in
    fixed mode), factors L = P U_k s_k, R = Qr V_k."""
    if M.size == 0:
        return np.zeros((P.shape[0], 0)), np.zeros((Qr.shape[0], 0))
    U, s, Vt = np.linalg.svd(M)
    if fixed:
        k = len(s)
    else:
        budget = eps * eps * float(np.sum(s * s)) - e2
        sq = s * s
        tail2 = np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]])
        k = len(s)
        if budget >= 0:
            for kk in range(len(s) + 1):
                if tail2[kk] <= budget:
                    k = kk
                    break
    return (P @ U[:, :k]) * s[:k][None, :], Qr @ Vt[:k].T


def aca(D, eps, kcap=64, k_fixed=0):
    """Adaptive cross approximation with partial pivoting (Algorithm 6), then
    recompression by Algorithm 5 and epsilon-truncation."""
    m, n = D.shape
    fixed = k_fixed > 0
    lim = min(m, n, kcap, k_fixed if fixed else kcap)
    Ls, Us = [], []
    used = np.zeros(m, dtype=bool)
    i = 0
    nrm2 = 0.0
    e2 = 0.0
    converged = False
    while True:
        r = len(Ls)
        if r == lim:
            converged = fixed or r == min(m, n)
            break
        row = D[i, :].copy()
        for L_j, U_j in zip(Ls, Us):
            row -= L_j[i] * U_j
        used[i] = True
        jp = int(np.argmax(np.abs(row)))
        piv = row[jp]
        if piv == 0.0:
            converged = True
            break
        u = row / piv
        col = D[:, jp].copy()
        for L_j, U_j in zip(Ls, Us):
            col -= U_j[jp] * L_j
        nl, nu = float(col @ col), float(u @ u)
        if not fixed and nl * nu <= eps * eps * nrm2:
            e2 = nl * nu
            converged = True
            break
        cross = sum(float(L_j @ col) * float(U_j @ u) for L_j, U_j in zip(Ls, Us))
        nrm2 += 2.0 * cross + nl * nu
        Ls.append(col)
        Us.append(u)
        cand = np.abs(col)
        cand[used] = -1.0
        i = int(np.argmax(cand))
    k = len(Ls)
    if k == 0:
        return SchemeResult(np.zeros((m, 0)), np.zeros((n, 0)), 0, converged, e2)
    Lm, Um = np.stack(Ls, axis=1), np.stack(Us, axis=1)
    Ql, Rl = np.linalg.qr(Lm)
    Qu, Ru = np.linalg.qr(Um)
    L, R = _truncate_svd(Ql, Qu, Rl @ Ru.T, eps, e2, fixed)
    return SchemeResult(L, R, k, converged, e2)


def _reorth(v, basis):
    """Two passes of classical Gram-Schmidt against the columns in `basis`."""
    for _ in range(2):
        for b in basis:
            v = v - (b @ v) * b
    return v


def lanczos(D, eps, w1, kcap=64, k_fixed=0):
    """Golub-Kahan-Lanczos bidiagonalization (Algorithm 7) with full
    reorthogonalization, the stopping rule above, SVD of B_k and truncation."""
    m, n = D.shape
    fixed = k_fixed > 0
    lim = min(m, n, kcap, k_fixed if fixed else kcap)
    w = np.asarray(w1, dtype=np.float64)
    w = w / np.linalg.norm(w)
    Ws, Qs, alpha, beta = [w], [], [], []
    nrm2, e2, beta_prev = 0.0, 0.0, 0.0
    converged = False
    while True:
        r = len(alpha)
        q = D @ Ws[r]
        if r > 0:
            q = q - beta_prev * Qs[r - 1]
        q = _reorth(q, Qs)
        a = float(np.linalg.norm(q))
        upd2 = a * a + beta_prev * beta_prev
        if (not fixed and upd2 <= eps * eps * nrm2) or a == 0.0:
            e2 = upd2
            converged = True
            break
        Qs.append(q / a)
        alpha.append(a)
        nrm2 += upd2
        r += 1
        wn = D.T @ Qs[r - 1] - a * Ws[r - 1]
        wn = _reorth(wn, Ws)
        b = float(np.linalg.norm(wn))
        if r == lim:
            e2 = 0.0 if fixed else b * b
            converged = fixed or r == min(m, n)
            break
        if b == 0.0:
            converged = True
            break
        Ws.append(wn / b)
        beta.append(b)
        beta_prev = b
    k = len(alpha)
    if k == 0:
        return SchemeResult(np.zeros((m, 0)), np.zeros((n, 0)), 0, converged, e2)
    Bk = np.diag(alpha) + np.diag(beta[:k - 1], 1)
    Qk, Wk = np.stack(Qs, axis=1), np.stack(Ws[:k], axis=1)
    L, R = _truncate_svd(Qk, Wk, Bk, eps, e2, fixed)
    return SchemeResult(L, R, k, converged, e2)


def randomized_fixed(D, Om, q=1):
    """Randomized rank-k approximation with q subspace iterations (Algorithm 9):
    returns L (orthonormal columns) and R = A^T L, with k = Om.shape[1]."""
    Lp = np.linalg.qr(D @ Om)[0]
    for _ in range(q):
        U = np.linalg.qr(D.T @ Lp)[0]
        Lp = np.linalg.qr(D @ U)[0]
    return SchemeResult(Lp, D.T @ Lp, Om.shape[1], True, 0.0)


def lowrank_svd(L, R, eps):
    """SVD of a low-rank matrix L R^T (Algorithm 5) and its epsilon-truncation:
    QR of both factors, SVD of R_L R_R^T, factors Q_L U_k s_k and Q_R V_k."""
    if L.shape[1] == 0:
        return np.zeros((L.shape[0], 0)), np.zeros((R.shape[0], 0))
    Ql, Rl = np.linalg.qr(L)
    Qr, Rr = np.linalg.qr(R)
    U, s, Vt = np.linalg.svd(Rl @ Rr.T)
    k = eps_rank(s, eps)
    return (Ql @ U[:, :k]) * s[:k][None, :], Qr @ Vt[:k].T
