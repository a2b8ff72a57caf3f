// Randomized compression of implicitly given blocks (shared by assembly and product).
//
// Per farfield target tau x sigma (m = #tau, n = #sigma) the blocked randomized
// range finder of Section 4 (randomized low-rank approximation) runs as:
//   Y = S Omega (b0 columns) and P = S G (probe columns) in one pass,
//   Q = orth(Y) (CGS2, rank revealing), P' = (I - Q Q^T) P, E^2 = ||P'||_F^2 / g,
//   Z = S^T Q (projection), ||B||_F^2 = ||Z||_F^2 with B = Q^T S,
//   while E > delta * eps * sqrt(||B||^2 + E^2): Q += orth(P'), new probe, new
//     projection columns (adaptive growth),
//   Z = Qz Rz, one-sided Jacobi on Rz^T = W J^T, output L = Q W_k, R = Qz J_k with
//   the smallest k such that tail_k^2 <= eps^2 (||B||^2 + E^2) - kappa E^2.
// The block error is E_true^2 + tail_k^2 (orthogonal pieces); kappa > 1 keeps it
// below eps ||S|| unless the probe underestimates the residual norm by more than
// sqrt(kappa).
// Only the products S X and S^T X depend on the operator; they are supplied by
// the caller (kernel evaluation for assembly, sum-expressions for the product).
#pragma once

#include "hmat_internal.h"
#include "product_kernels.h"

namespace hm {

struct CTarget {
  double* Y;     // m x (cap + g), ld m: Q in columns [0, cap), probe area [cap, cap + g)
  double* Z;     // n x cap, ld n: projections S^T Q
  double* core;  // cap*cap (Rz, then W) + cap*cap (J) + cap (sigma)
  int32_t m, n;
  int32_t row0, col0;  // first row / column position of the block
  int32_t r;           // columns of Q so far
  int32_t rz;          // columns of Z so far
  int32_t k;           // output rank
  int32_t done;        // residual check passed
  int32_t active;      // participates in the current pass
  int32_t rounds;      // growth rounds used
  double E2, nB2;
  int64_t out_off;     // element offset of the output L (then R) in the result pool
  int32_t block;       // block id
  int32_t w0;          // initial sketch width of this target (b0 or predicted)
  int32_t svd_capped;  // 1: the core's Jacobi iteration reached its sweep cap
  int32_t pad;
};

constexpr int CAPMAX_CORE = 64;  // largest column count of the per-target panels and cores

struct CParams {
  int32_t cap;     // column capacity of Q / Z
  int32_t g;       // probe columns
  double eps;
  double delta;
  double kappa;  // safety factor on the estimated residual in the truncation rule
};

// Omega: n x ncol Gaussian matrix (column-major, ld = n) keyed by (seed, position, column).
void launch_fill_gaussian(double* omega, int64_t n, int32_t ncol, uint64_t seed, hipStream_t s);

// Orthonormalise columns [src, src + cnt) of Y against Q[:, :r] and among themselves,
// appending the kept ones at Q[:, r...] (r updated). Targets with active == 0 skip.
void launch_orth_append(CTarget* t, int nt, int src, int cnt, const CParams& p, hipStream_t s);
// Probe residual of columns [cap, cap + g): P' = (I - Q Q^T) P twice; E2 = ||P'||^2 / g.
void launch_probe_residual(CTarget* t, int nt, const CParams& p, hipStream_t s);
// nB2 = ||Z[:, :rz]||^2 and done = (E <= delta * eps * sqrt(nB2 + E2)); also marks
// targets without room for another round (r + g > cap) as finished.
void launch_check(CTarget* t, int nt, const CParams& p, int32_t* n_pending, hipStream_t s);
// QR of Z, Jacobi SVD of the core, truncation: sets k and keeps W, J, sigma in core.
// rmax: the largest rz among the targets (0: use the capacity)
void launch_core(CTarget* t, int nt, const CParams& p, hipStream_t s, int rmax = 0);
// Algorithm 5 (SVD of a low-rank sum): columns [c0, c0 + cnt) of the target's stacked
// term factor [L_1 core_1, L_2 core_2, ...] (restricted to tau, terms of the block and
// of its ancestors in creation order) into Y[:, cap .. cap + cnt); zero past the last
// term column.
void launch_term_columns(CTarget* t, int nt, const TreeView& tv, int c0, int cnt, int cap, hipStream_t s);
// L = Q W[:, :k] and R = Qz J[:, :k] into pool + out_off.
void launch_write_factors(CTarget* t, int nt, const CParams& p, double* pool, hipStream_t s);

}  // namespace hm
