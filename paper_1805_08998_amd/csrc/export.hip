// Dense expansion of an H-matrix on the device (hmat_to_dense).
//
// Every leaf of the block-cluster tree holds either L R^T (farfield, low-rank
// set of Def. 2.6) or a dense block (nearfield). The leaves partition I x I, so
// every entry of the dense matrix is written exactly once. The matrix is built
// in column slabs of bounded size and copied slab by slab into the caller's
// host buffer.
#include <algorithm>
#include <cstring>

#include "hmat_internal.h"

namespace hm {

// One workgroup per (leaf, 64-column tile of the leaf); threads run over rows.
// A column of the leaf lands in output column cj = (order ? pos : perm[pos]);
// only columns inside the slab [j0, j0 + ncol) are written, at row
// ri = (order ? pos : perm[pos]).
__global__ void __launch_bounds__(256) k_leaves_to_dense(const int32_t* __restrict__ leaves,
                                                         const int32_t* __restrict__ b_tau,
                                                         const int32_t* __restrict__ b_sigma,
                                                         const int32_t* __restrict__ b_kind,
                                                         const int32_t* __restrict__ c_begin,
                                                         const int32_t* __restrict__ c_size,
                                                         const int32_t* __restrict__ rank,
                                                         const int64_t* __restrict__ off,
                                                         const double* __restrict__ pool,
                                                         const int32_t* __restrict__ perm, int32_t order,
                                                         int64_t j0, int64_t ncol, int64_t n,
                                                         double* __restrict__ out) {
  const int32_t b = leaves[blockIdx.x];
  const int32_t m = c_size[b_tau[b]], nn = c_size[b_sigma[b]];
  const int32_t r0 = c_begin[b_tau[b]], c0 = c_begin[b_sigma[b]];
  const int jt = int(blockIdx.y) * 64;
  if (jt >= nn) return;
  const bool far = b_kind[b] == KIND_F;
  const int k = far ? rank[b] : 0;
  const double* d = pool + off[b];
  const int jend = min(nn, jt + 64);
  for (int j = jt; j < jend; ++j) {
    const int64_t cpos = int64_t(c0) + j;
    const int64_t cj = order ? cpos : int64_t(perm[cpos]);
    if (cj < j0 || cj >= j0 + ncol) continue;
    double* col = out + (cj - j0) * n;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      double v;
      if (far) {
        v = 0.0;
        for (int c = 0; c < k; ++c) v = fma(d[i + int64_t(c) * m], d[int64_t(m) * k + j + int64_t(c) * nn], v);
      } else {
        v = d[i + int64_t(j) * m];
      }
      const int64_t rpos = int64_t(r0) + i;
      col[order ? rpos : int64_t(perm[rpos])] = v;
    }
  }
}

void expand_to_dense(HMat* M, double* out, int64_t ld, int32_t order, hipStream_t s) {
  Tree* t = M->tree;
  set_current_stream(s);
  t->ensure_device(s);
  const int64_t n = t->n;
  DevBuf<int32_t> d_leaves, d_perm;
  d_leaves.upload(t->leaves, s);
  d_perm.upload(t->perm, s);
  int32_t max_cols = 1;
  for (int32_t b : t->leaves) max_cols = std::max(max_cols, t->c_size[t->b_sigma[b]]);
  // slab of at most 1 GiB of output columns
  const int64_t slab = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t(1) << 27) / std::max<int64_t>(n, 1)));
  DevBuf<double> buf(size_t(n) * size_t(slab));
  const dim3 grid(unsigned(t->leaves.size()), unsigned((max_cols + 63) / 64));
  for (int64_t j0 = 0; j0 < n; j0 += slab) {
    const int64_t nc = std::min(slab, n - j0);
    HM_CHECK_HIP(hipMemsetAsync(buf.p, 0, size_t(n) * size_t(nc) * 8, s));
    if (!t->leaves.empty()) {
      hipLaunchKernelGGL(k_leaves_to_dense, grid, dim3(256), 0, s, d_leaves.p, t->dev->b_tau.p, t->dev->b_sigma.p,
                         t->dev->b_kind.p, t->dev->c_begin.p, t->dev->c_size.p, M->d_rank.p, M->d_off.p, M->pool.p,
                         d_perm.p, order, j0, nc, n, buf.p);
      HM_CHECK_HIP(hipGetLastError());
    }
    HM_CHECK_HIP(hipMemcpy2DAsync(out + j0 * ld, size_t(ld) * 8, buf.p, size_t(n) * 8, size_t(n) * 8, size_t(nc),
                                  hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
  }
}

}  // namespace hm
