// H-matrix times a block of vectors (Algorithm 2): launches of matvec.hip.
#pragma once

#include "hmat_internal.h"

namespace hm {

// Scratch of one product y = M x with nvec vectors, in doubles: one int64 offset per
// block of the tree, then the leaf products R^T x (or L^T x) of every farfield leaf.
int64_t matvec_scratch_doubles(const HMat* M, int32_t nvec);

// Enqueues y = M x (trans 0) or y = M^T x (trans 1) on stream s. x, y: device
// column-major n x nvec (leading dimensions ldx, ldy), rows in original point order
// (order 0) or cluster order (order 1). scratch: matvec_scratch_doubles(M, nvec) doubles
// of device memory, in use until the stream passes this point. The tree's device copy
// must exist.
void matvec_launch(const HMat* M, int32_t trans, int32_t order, int32_t nvec, const double* x, int64_t ldx,
                   double* y, int64_t ldy, double* scratch, hipStream_t s);

// Frobenius-norm estimates of C - A B and of A B by subspace iteration from the
// start block X0 (device, n x p, cluster order); synchronous on stream s.
void error_estimate(const HMat* C, const HMat* A, const HMat* B, const double* X0, int32_t p, int32_t iters,
                    hipStream_t s, double* err, double* norm_ab);

// Argument checks of the matvec entry points (HMAT_ERR_ARG via Error); returns M.
HMat* check_matvec_args(hmat mh, int32_t trans, int32_t order, int32_t nvec, const double* x, int64_t ldx,
                        const double* y, int64_t ldy);

}  // namespace hm
