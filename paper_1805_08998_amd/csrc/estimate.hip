// Frobenius-norm estimate of the product error C - A B (the accuracy instrument of
// the numerical-examples section): subspace iteration on the operator
// E v = C v - A (B v), whose products with a block of vectors are three H-matrix
// products (Algorithm 2). From a start block X (n x p, cluster order):
//   repeat iters times: Y = orth(E X), X = orth(E^T Y);  estimate = ||E X||_F,
// and the same on v -> A (B v) for the reference norm ||A B||_F. Orthonormalization
// is classical Gram-Schmidt applied twice, one column at a time, with deterministic
// reductions (fixed summation order).
#include <algorithm>
#include <cmath>

#include "hmat_internal.h"
#include "device_common.h"
#include "matvec.h"

namespace hm {

namespace {

constexpr int NT = 256;
constexpr int NR = 1024;  // threads of the single-workgroup reductions

// h[i] = V[:, i] . V[:, j] for i < j; workgroup i.
__global__ void __launch_bounds__(NT) k_col_dots(const double* __restrict__ V, int64_t n, int j, double* __restrict__ h) {
  __shared__ double red[NT / 64];
  const int i = blockIdx.x;
  const double* a = V + int64_t(i) * n;
  const double* b = V + int64_t(j) * n;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += NT) acc += a[r] * b[r];
  acc = block_sum<NT>(acc, red);
  if (threadIdx.x == 0) h[i] = acc;
}

// V[:, j] -= V[:, :j] h
__global__ void __launch_bounds__(NT) k_col_sub(double* __restrict__ V, int64_t n, int j, const double* __restrict__ h) {
  const int64_t r = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (r >= n) return;
  double v = V[int64_t(j) * n + r];
  for (int i = 0; i < j; ++i) v -= V[int64_t(i) * n + r] * h[i];
  V[int64_t(j) * n + r] = v;
}

// out = sum of squares of x[0 .. len) (one workgroup, fixed order)
__global__ void __launch_bounds__(NR) k_sumsq(const double* __restrict__ x, int64_t len, double* __restrict__ out) {
  __shared__ double red[NR / 64];
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < len; r += NR) acc += x[r] * x[r];
  acc = block_sum<NR>(acc, red);
  if (threadIdx.x == 0) *out = acc;
}

// x[0 .. len) *= 1 / sqrt(*s2) (zero when s2 == 0)
__global__ void __launch_bounds__(NT) k_scale_inv_sqrt(double* __restrict__ x, int64_t len, const double* __restrict__ s2) {
  const int64_t r = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (r >= len) return;
  const double v = *s2;
  x[r] = v > 0.0 ? x[r] / sqrt(v) : 0.0;
}

__global__ void __launch_bounds__(NT) k_sub(double* __restrict__ y, const double* __restrict__ t, int64_t len) {
  const int64_t r = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (r < len) y[r] -= t[r];
}

unsigned grid_of(int64_t len) { return unsigned((len + NT - 1) / NT); }

// Orthonormal columns of V (n x p) in place; h: p doubles, s2: one double.
void orth_panel(double* V, int64_t n, int p, double* h, double* s2, hipStream_t s) {
  for (int j = 0; j < p; ++j) {
    for (int pass = 0; pass < 2 && j > 0; ++pass) {
      hipLaunchKernelGGL(k_col_dots, dim3(unsigned(j)), dim3(NT), 0, s, V, n, j, h);
      hipLaunchKernelGGL(k_col_sub, dim3(grid_of(n)), dim3(NT), 0, s, V, n, j, h);
    }
    hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(NR), 0, s, V + int64_t(j) * n, n, s2);
    hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(grid_of(n)), dim3(NT), 0, s, V + int64_t(j) * n, n, s2);
  }
  HM_CHECK_HIP(hipGetLastError());
}

struct EstimateWork {
  const HMat* C;  // null: the operator is A B alone
  const HMat* A;
  const HMat* B;
  int64_t n;
  int p;
  double* t1;
  double* t2;
  double* scratch;
  hipStream_t s;
  // Y = E X (trans 0) or X = E^T Y (trans 1), E = C - A B or A B
  void apply(const double* X, double* Y, int trans) const {
    const HMat* first = trans ? A : B;
    const HMat* second = trans ? B : A;
    matvec_launch(first, trans, 1, p, X, n, t1, n, scratch, s);
    if (!C) {
      matvec_launch(second, trans, 1, p, t1, n, Y, n, scratch, s);
      return;
    }
    matvec_launch(second, trans, 1, p, t1, n, t2, n, scratch, s);
    matvec_launch(C, trans, 1, p, X, n, Y, n, scratch, s);
    hipLaunchKernelGGL(k_sub, dim3(grid_of(n * p)), dim3(NT), 0, s, Y, t2, n * p);
    HM_CHECK_HIP(hipGetLastError());
  }
};

double subspace_estimate(const EstimateWork& w, const double* X0, double* V, double* W, double* h, double* s2,
                         int iters) {
  const int64_t len = w.n * w.p;
  HM_CHECK_HIP(hipMemcpyAsync(V, X0, 8 * len, hipMemcpyDeviceToDevice, w.s));
  orth_panel(V, w.n, w.p, h, s2, w.s);
  for (int it = 0; it < iters; ++it) {
    w.apply(V, W, 0);
    orth_panel(W, w.n, w.p, h, s2, w.s);
    w.apply(W, V, 1);
    orth_panel(V, w.n, w.p, h, s2, w.s);
  }
  w.apply(V, W, 0);
  hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(NR), 0, w.s, W, len, s2);
  HM_CHECK_HIP(hipGetLastError());
  double out = 0.0;
  HM_CHECK_HIP(hipMemcpyAsync(&out, s2, 8, hipMemcpyDeviceToHost, w.s));
  HM_CHECK_HIP(hipStreamSynchronize(w.s));
  return std::sqrt(out);
}

}  // namespace

void error_estimate(const HMat* C, const HMat* A, const HMat* B, const double* X0, int32_t p, int32_t iters,
                    hipStream_t s, double* err, double* norm_ab) {
  const int64_t n = A->tree->n;
  set_current_stream(s);
  const int64_t sc = std::max({matvec_scratch_doubles(A, p), matvec_scratch_doubles(B, p), matvec_scratch_doubles(C, p)});
  const size_t len = size_t(n) * size_t(p);
  DevBuf<double> V{len}, W{len}, t1{len}, t2{len}, scratch{size_t(sc)}, h{size_t(p) + 1};
  EstimateWork w{C, A, B, n, p, t1.p, t2.p, scratch.p, s};
  *err = subspace_estimate(w, X0, V.p, W.p, h.p, h.p + p, iters);
  w.C = nullptr;
  *norm_ab = subspace_estimate(w, X0, V.p, W.p, h.p, h.p + p, iters);
}

}  // namespace hm
