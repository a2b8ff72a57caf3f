// H-matrix times a block of vectors (Algorithm 2, HtimesV): y = M x or y = M^T x.
//
// Every leaf tau x sigma of the block-cluster tree contributes L (R^T x[sigma])
// (farfield, low-rank) or D x[sigma] (nearfield) to y[tau] (Algorithm 2 run
// over the leaves; the leaves partition I x I). Two launches:
//   1. per farfield leaf, t_b = R_b^T x[sigma] (transposed: L_b^T x[tau]) into a
//      scratch buffer at an offset given by an exclusive prefix over the ranks;
//   2. per leaf cluster c, one thread per row of c: the rows of c are covered by
//      the leaves whose row cluster is c or one of its ancestors, so the thread
//      walks the ancestor chain and sums every leaf of their block rows in a fixed
//      order (deterministic, no atomics).
// Vectors are in the caller's point order (order 0: original indices, gathered
// and scattered through the permutation) or in cluster order (order 1).
#include <algorithm>
#include <mutex>
#include <string>

#include "hmat_internal.h"
#include "device_common.h"
#include "matvec.h"

namespace hm {

namespace {

constexpr int NT = 256;
constexpr int NV = 8;  // vectors per register block

__device__ __forceinline__ int64_t vec_row(const int32_t* perm, int32_t order, int64_t pos) {
  return order ? pos : int64_t(perm[pos]);
}

// Exclusive prefix over blocks of (farfield ? rank : 0) * nvec; one workgroup of 1024
// threads, each thread sums a contiguous segment.
__global__ void __launch_bounds__(1024) k_rank_prefix(const int32_t* __restrict__ kind, const int32_t* __restrict__ rank,
                                                      int64_t nb, int32_t nvec, int64_t* __restrict__ toff) {
  __shared__ int64_t part[1024];
  const int tid = threadIdx.x;
  const int64_t seg = (nb + 1023) / 1024;
  const int64_t lo = std::min<int64_t>(nb, tid * seg), hi = std::min<int64_t>(nb, lo + seg);
  int64_t s = 0;
  for (int64_t b = lo; b < hi; ++b) s += kind[b] == KIND_F ? int64_t(rank[b]) * nvec : 0;
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    int64_t acc = 0;
    for (int i = 0; i < 1024; ++i) {
      const int64_t v = part[i];
      part[i] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int64_t acc = part[tid];
  for (int64_t b = lo; b < hi; ++b) {
    toff[b] = acc;
    acc += kind[b] == KIND_F ? int64_t(rank[b]) * nvec : 0;
  }
}

// t_b(c, v) = sum_j F_b(j, c) x(other0 + j, v) for every farfield leaf b, F = R (forward)
// or L (transposed); one wave per column c.
__global__ void __launch_bounds__(NT) k_leaf_rt(const int32_t* __restrict__ kind, const int32_t* __restrict__ rank,
                                                const int64_t* __restrict__ off, const int32_t* __restrict__ b_tau,
                                                const int32_t* __restrict__ b_sigma, const int32_t* __restrict__ c_begin,
                                                const int32_t* __restrict__ c_size, const double* __restrict__ pool,
                                                const int32_t* __restrict__ perm, int32_t order, int32_t trans,
                                                int32_t nvec, const double* __restrict__ x, int64_t ldx,
                                                const int64_t* __restrict__ toff, double* __restrict__ tbuf) {
  const int64_t b = blockIdx.x;
  if (kind[b] != KIND_F) return;
  const int k = rank[b];
  if (k == 0) return;
  const int m = c_size[b_tau[b]], n = c_size[b_sigma[b]];
  // forward: R (n x k, after L in the leaf's data) against x[sigma]; transposed: L (m x k) against x[tau]
  const double* F = pool + off[b] + (trans ? 0 : int64_t(m) * k);
  const int rows = trans ? m : n;
  const int64_t x0 = c_begin[trans ? b_tau[b] : b_sigma[b]];
  double* t = tbuf + toff[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int v0 = 0; v0 < nvec; v0 += NV) {
    const int nv = min(NV, nvec - v0);
    for (int c = w; c < k; c += NT / 64) {
      double acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = 0.0;
      for (int j = lane; j < rows; j += 64) {
        const double f = F[j + int64_t(c) * rows];
        const int64_t xr = vec_row(perm, order, x0 + j);
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (v < nv) acc[v] += f * x[xr + int64_t(v0 + v) * ldx];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double s = wave_sum(acc[v]);
        if (lane == 0 && v < nv) t[c + int64_t(v0 + v) * k] = s;
      }
    }
  }
}

// y(row) for the rows of one leaf cluster (forward: block rows of its ancestors,
// transposed: block columns).
__global__ void __launch_bounds__(NT) k_rows_mv(const int32_t* __restrict__ leaf_clusters, const int32_t* __restrict__ c_begin,
                                                const int32_t* __restrict__ c_size, const int32_t* __restrict__ c_parent,
                                                const int32_t* __restrict__ lptr, const int32_t* __restrict__ lblk,
                                                const int32_t* __restrict__ b_tau, const int32_t* __restrict__ b_sigma,
                                                const int32_t* __restrict__ kind, const int32_t* __restrict__ rank,
                                                const int64_t* __restrict__ off, const double* __restrict__ pool,
                                                const int32_t* __restrict__ perm, int32_t order, int32_t trans,
                                                int32_t nvec, const double* __restrict__ x, int64_t ldx,
                                                const int64_t* __restrict__ toff, const double* __restrict__ tbuf,
                                                double* __restrict__ y, int64_t ldy) {
  const int32_t cl = leaf_clusters[blockIdx.x];
  const int32_t r0 = c_begin[cl], nr = c_size[cl];
  for (int li = threadIdx.x; li < nr; li += NT) {
    const int64_t pos = int64_t(r0) + li;
    for (int v0 = 0; v0 < nvec; v0 += NV) {
      const int nv = min(NV, nvec - v0);
      double acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = 0.0;
      for (int32_t a = cl; a >= 0; a = c_parent[a]) {
        const int32_t a0 = c_begin[a], am = c_size[a];
        const int ia = int(pos - a0);  // row of the leaf inside its own cluster
        for (int32_t p = lptr[a]; p < lptr[a + 1]; ++p) {
          const int32_t b = lblk[p];
          const int32_t oc = trans ? b_tau[b] : b_sigma[b];  // the other cluster of the leaf
          const int32_t o0 = c_begin[oc], on = c_size[oc];
          const double* d = pool + off[b];
          if (kind[b] == KIND_F) {
            const int k = rank[b];
            // forward: L (am x k), row ia; transposed: R (am x k after L of on x k), row ia
            const double* P = trans ? d + int64_t(on) * k : d;
            const double* t = tbuf + toff[b];
            for (int c = 0; c < k; ++c) {
              const double pv = P[ia + int64_t(c) * am];
#pragma unroll
              for (int v = 0; v < NV; ++v)
                if (v < nv) acc[v] += pv * t[c + int64_t(v0 + v) * k];
            }
          } else {
            // forward: D (am x on) row ia against x[other]; transposed: D (on x am) column ia
            for (int j = 0; j < on; ++j) {
              const double dv = trans ? d[j + int64_t(ia) * on] : d[ia + int64_t(j) * am];
              const int64_t xr = vec_row(perm, order, int64_t(o0) + j);
#pragma unroll
              for (int v = 0; v < NV; ++v)
                if (v < nv) acc[v] += dv * x[xr + int64_t(v0 + v) * ldx];
            }
          }
        }
      }
      const int64_t yr = vec_row(perm, order, pos);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (v < nv) y[yr + int64_t(v0 + v) * ldy] = acc[v];
    }
  }
}

}  // namespace

int64_t matvec_scratch_doubles(const HMat* M, int32_t nvec) {
  const Tree& t = *M->tree;
  int64_t ks = 0;
  for (int32_t b : t.leaves)
    if (t.b_kind[b] == KIND_F) ks += M->rank[b];
  const int64_t nb = int64_t(t.b_tau.size());
  return nb + ks * int64_t(nvec);  // int64 offsets (one double each), then the leaf products
}

void matvec_launch(const HMat* M, int32_t trans, int32_t order, int32_t nvec, const double* x, int64_t ldx,
                   double* y, int64_t ldy, double* scratch_p, hipStream_t s) {
  const Tree& t = *M->tree;
  const DeviceTree& dv = *t.dev;
  const int64_t nb = int64_t(t.b_tau.size());
  int64_t* toff = reinterpret_cast<int64_t*>(scratch_p);
  double* tbuf = scratch_p + nb;
  hipLaunchKernelGGL(k_rank_prefix, dim3(1), dim3(1024), 0, s, dv.b_kind.p, M->d_rank.p, nb, nvec, toff);
  HM_CHECK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_leaf_rt, dim3(unsigned(nb)), dim3(NT), 0, s, dv.b_kind.p, M->d_rank.p, M->d_off.p, dv.b_tau.p,
                     dv.b_sigma.p, dv.c_begin.p, dv.c_size.p, M->pool.p, dv.perm.p, order, trans, nvec, x, ldx, toff,
                     tbuf);
  HM_CHECK_HIP(hipGetLastError());
  const unsigned nlc = unsigned(t.leaf_clusters.size());
  hipLaunchKernelGGL(k_rows_mv, dim3(nlc), dim3(NT), 0, s, dv.leaf_clusters.p, dv.c_begin.p, dv.c_size.p,
                     dv.c_parent.p, trans ? dv.bcol_ptr.p : dv.brow_ptr.p, trans ? dv.bcol_blk.p : dv.brow_blk.p,
                     dv.b_tau.p, dv.b_sigma.p, dv.b_kind.p, M->d_rank.p, M->d_off.p, M->pool.p, dv.perm.p, order,
                     trans, nvec, x, ldx, toff, tbuf, y, ldy);
  HM_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- no-allocation variant
// Scratch of hmat_matvec_noalloc: a static device array, one copy per GPU the library
// runs on, allocated with the code object and held until the process ends. In host code
// `scratch` only names the symbol; its device address on each GPU comes from
// hipGetSymbolAddress (once per device, with that device current).
static __device__ __align__(256) double scratch[HMAT_MATVEC_NOALLOC_BYTES / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

double* scratch_of_device(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  HM_REQUIRE(dev >= 0 && dev < kMaxDevices, HMAT_ERR_ARG, "device id out of range");
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HM_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_dev[dev];
}
}  // namespace

}  // namespace hm

extern "C" hmat_status hmat_matvec_noalloc(hmat mh, int32_t trans, int32_t order, int32_t nvec, const double* x,
                                           int64_t ldx, double* y, int64_t ldy, void* stream) {
  using namespace hm;
  try {
    HMat* M = check_matvec_args(mh, trans, order, nvec, x, ldx, y, ldy);
    const int64_t need = matvec_scratch_doubles(M, nvec) * int64_t(sizeof(double));
    HM_REQUIRE(need <= int64_t(HMAT_MATVEC_NOALLOC_BYTES), HMAT_ERR_ARG,
               "hmat_matvec_noalloc needs " + std::to_string(need) + " bytes of scratch, above its static " +
                   std::to_string(int64_t(HMAT_MATVEC_NOALLOC_BYTES)) + " (use hmat_matvec or fewer vectors)");
    int dev = 0;
    HM_CHECK_HIP(hipGetDevice(&dev));
    double* sp = scratch_of_device(dev);
    matvec_launch(M, trans, order, nvec, x, ldx, y, ldy, sp, reinterpret_cast<hipStream_t>(stream));
    return HMAT_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return HMAT_ERR_INTERNAL;
  }
}
