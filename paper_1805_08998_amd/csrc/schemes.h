// The paper's other low-rank schemes for a target block S = S(tau, sigma),
// run over all targets of a chunk at once (one workgroup per target per step):
//
//  * adaptive cross approximation with partial pivoting (Section 4, ACA,
//    Algorithm 6): each step fetches one row e_i^T S (a transposed pass with a
//    unit vector) and one column S e_j (a forward pass), subtracts the crosses
//    found so far, and stops on the update-size criterion eq. (truncaca);
//  * Golub-Kahan-Lanczos bidiagonalization (Section 4, Algorithm 7) with full
//    reorthogonalization: one forward and one transposed pass per step;
//  * the randomized rank-k approximation with q subspace iterations
//    (Algorithm 9), the fixed-rank form of the randomized scheme.
//
// The passes themselves are the product's apply kernels (the caller runs them);
// these kernels hold the per-target vector work between passes and the final
// recompression: QR of both ACA factors and SVD of R_L R_U^T (Algorithm 5), or
// SVD of the bidiagonal B_k, followed by the truncation
//   tail(k)^2 <= eps^2 ||approximation||_F^2 - e2,
// where e2 is the squared norm of the update that stopped the iteration.
#pragma once

#include "hmat_internal.h"

namespace hm {

struct ITarget {
  double* L;     // m x cap: ACA columns l_r / Lanczos q_r / Algorithm 9 range basis
  double* U;     // n x (cap + 1): ACA rows u_r / Lanczos w_r / Algorithm 9 co-range
  double* xf;    // n: input of the forward pass (unit vector e_j, or w_r)
  double* xt;    // m: input of the transposed pass (unit vector e_i, or q_r)
  double* yf;    // m: output of the forward pass
  double* yt;    // n: output of the transposed pass
  double* work;  // 2 cap^2 (core, then W and J) + cap (sigma) + 2 cap (alpha, beta)
  int32_t* used; // m: ACA rows already used as pivots
  int32_t m, n;
  int32_t row0, col0;  // first row / column position of the block
  int32_t r;           // steps kept (columns of L)
  int32_t rz;          // columns of U (Algorithm 9)
  int32_t state;       // 0 running, 1 finished, 2 step cap reached before the stopping test held
  int32_t pi, pj;      // ACA pivots of the current step
  int32_t lim;         // step limit min(m, n, cap, k_fixed)
  int32_t k;           // output rank
  int32_t block;
  int32_t svd_sweeps;  // Jacobi sweeps of the final SVD (-1: sweep cap reached)
  int32_t pad;
  double nrm2;       // ||approximation||_F^2
  double e2;         // squared norm of the discarded update
  double beta_prev;  // Lanczos beta_{r-1}
  double pad2;
  int64_t out_off;   // element offset of the output L (then R) in the result pool
};

struct IParams {
  int32_t cap;    // panel capacity (steps)
  int32_t fixed;  // 1: fixed-rank mode (no eps test, no truncation)
  double eps;
};

constexpr int ISCHEME_CAP = 64;

// Zeroes xf, xt and used; ACA starts at row 0 (xt = e_0).
void launch_aca_init(ITarget* t, int nt, hipStream_t s);
// Residual row u = yt - sum_j L[pi, j] U[:, j], column pivot, u / pivot, xf = e_pj.
void launch_aca_row(ITarget* t, int nt, const IParams& p, hipStream_t s);
// Residual column l = yf - sum_j U[pj, j] L[:, j], stopping test, norm update, next row pivot.
void launch_aca_col(ITarget* t, int nt, const IParams& p, int32_t* state_out, hipStream_t s);
// QR of L[:, :r] and U[:, :r] in place, core R_L R_U^T into work.
void launch_aca_core(ITarget* t, int nt, const IParams& p, hipStream_t s);

// w_1 = column 0 of Omega on sigma, normalised; xf = w_1.
void launch_gkl_init(ITarget* t, int nt, const double* omega, hipStream_t s);
// q = yf - beta_{r-1} q_{r-1}, reorthogonalization, alpha, stopping test.
void launch_gkl_fwd(ITarget* t, int nt, const IParams& p, hipStream_t s);
// w = yt - alpha_r w_r, reorthogonalization, beta, step limit.
void launch_gkl_bwd(ITarget* t, int nt, const IParams& p, int32_t* state_out, hipStream_t s);
// Core = B_k (alpha on the diagonal, beta above it) into work.
void launch_gkl_core(ITarget* t, int nt, const IParams& p, hipStream_t s);

// One-sided Jacobi SVD of the r x r core in work, sorted, truncated (sets k and
// svd_sweeps); rmax = the largest r among the targets.
void launch_iter_svd(ITarget* t, int nt, const IParams& p, int rmax, hipStream_t s);
// L_out = L W[:, :k], R_out = U J[:, :k] into pool + out_off.
void launch_iter_write(ITarget* t, int nt, const IParams& p, double* pool, hipStream_t s);

// Algorithm 9: orthonormalise columns [0, cnt_t) of L (side 0, count in r) or of U
// (side 1, count in rz) in place, CGS2, dropping columns whose relative residual is
// below 1e-13 (cnt_t = the target's previous count, or `cnt` for the first sketch).
void launch_orth_cols(ITarget* t, int nt, int side, int cnt, int32_t* counts_out, hipStream_t s);
// Output of Algorithm 9: L_out = L[:, :r], R_out = U[:, :r] (k = r).
void launch_copy_out(ITarget* t, int nt, double* pool, hipStream_t s);

}  // namespace hm
