// Product kernels: products of sum-expressions with blocks of vectors.
//
// A sum-expression S(tau, sigma) = sum_i L_i core_i R_i^T + sum_j A[tau, rho_j] B[rho_j, sigma]
// (Def. 3.1) is applied to a panel X as in the identity that closes Section 3:
//   S X = sum_i L_i (core_i (R_i^T X)) + sum_j A[tau, rho_j] (B[rho_j, sigma] X),
// and S^T X likewise with the roles of the factors exchanged. The low-rank
// terms are views into the factor pools (restriction by index shift), the
// pairs are products with whole subtrees of A and B (Algorithm 2 on a block).
//
// Work decomposition (one 64-lane wave per work item, PW = 16 columns per pass):
//   k_term_p1   per (target, term): V = core (R^T X)        (reduction over input rows)
//   k_leaf_p1   per (subtree task, low-rank leaf): T = R^T X (or L^T X)
//   k_subtree_p2 per (subtree task, output leaf cluster): Y = sum over the
//               leaves whose rows contain it of L T or D X (or the transposes)
//   k_gather    per (target, output leaf cluster): Y = sum_i L_i V_i + sum_j pair_j
// Every output row is written by exactly one work item, in a fixed order, so
// results do not depend on scheduling.
#include "product_kernels.h"
#include "device_common.h"
#include "hmat_internal.h"

namespace hm {

// ---------------------------------------------------------------- wave helpers
// Us[c * PW + col] = sum_r M(r, c) X(r, col) for c < k, col < w.
// M(r, c) = mtrans ? M[c + r * ldm] : M[r + c * ldm].
// X(r, col) = xident ? (r == xc0 + col) : X[r + col * ldx].
__device__ void reduce_wave(const double* __restrict__ M, int ldm, int mtrans, int rows, int k,
                            const double* __restrict__ X, int ldx, int xident, int xc0, int w,
                            double* Us) {
  const int lane = threadIdx.x;
  const int G = k >= 64 ? 1 : 64 / k;
  const int c = lane % k, g = lane / k;
  const bool act = g < G;
  double acc[PW];
#pragma unroll
  for (int s = 0; s < PW; ++s) acc[s] = 0.0;
  if (act) {
    if (xident) {
#pragma unroll
      for (int s = 0; s < PW; ++s) {
        int col = g + s * G;
        int r = xc0 + col;
        if (col < w && r >= 0 && r < rows) acc[s] = mtrans ? M[c + int64_t(r) * ldm] : M[r + int64_t(c) * ldm];
      }
    } else if (mtrans) {
      for (int r = 0; r < rows; ++r) {
        double mv = M[c + int64_t(r) * ldm];
#pragma unroll
        for (int s = 0; s < PW; ++s) {
          int col = g + s * G;
          if (col < w) acc[s] += mv * X[r + int64_t(col) * ldx];
        }
      }
    } else {
      const double* Mc = M + int64_t(c) * ldm;
      for (int r = 0; r < rows; ++r) {
        double mv = Mc[r];
#pragma unroll
        for (int s = 0; s < PW; ++s) {
          int col = g + s * G;
          if (col < w) acc[s] += mv * X[r + int64_t(col) * ldx];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < PW; ++s) {
      int col = g + s * G;
      if (col < w) Us[c * PW + col] = acc[s];
    }
  }
  __syncthreads();
}

// acc[col] += sum_c P(row, c) Vs[c * PW + col] for this lane's row.
__device__ __forceinline__ void expand_row(const double* __restrict__ P, int64_t rowidx, int ldp, int ptrans,
                                           int k, const double* Vs, int w, double* acc) {
  for (int c = 0; c < k; ++c) {
    double p = ptrans ? P[c + rowidx * ldp] : P[rowidx + int64_t(c) * ldp];
#pragma unroll
    for (int col = 0; col < PW; ++col)
      if (col < w) acc[col] += p * Vs[c * PW + col];
  }
}

// Vs (k x w, ld PW) <- V (k x w column-major, ld k)
__device__ __forceinline__ void stage_v(const double* __restrict__ V, int k, int w, double* Vs) {
  for (int i = threadIdx.x; i < k * w; i += 64) {
    int c = i % k, col = i / k;
    Vs[c * PW + col] = V[i];
  }
  __syncthreads();
}

// ---------------------------------------------------------------- term reductions
__global__ void __launch_bounds__(64) k_term_p1(const TermItem* __restrict__ items, const TDesc* __restrict__ td,
                                               const TInfo* __restrict__ ti, TreeView tv, double* __restrict__ vbuf) {
  __shared__ double Us[64 * PW];
  const TermItem it = items[blockIdx.x];
  const TDesc d = td[it.t];
  if (d.w == 0) return;
  const Term T = tv.terms[it.term];
  const int tb = ti[it.t].block;
  const int tau = tv.b_tau[tb], sig = tv.b_sigma[tb];
  const double* M;
  int ldm, mtrans, rows, k, kout, mode;
  if (!d.trans) {  // V = core (R[sigma]^T X)
    const int rr = tv.c_begin[sig] - T.rrow0;
    M = T.rtrans ? T.R + int64_t(rr) * T.ldr : T.R + rr;
    ldm = T.ldr;
    mtrans = T.rtrans;
    rows = tv.c_size[sig];
    k = T.kr;
    kout = T.kl;
    mode = T.core ? 1 : 0;
  } else {  // V = core^T (L[tau]^T X)
    M = T.L + (tv.c_begin[tau] - T.lrow0);
    ldm = T.ldl;
    mtrans = 0;
    rows = tv.c_size[tau];
    k = T.kl;
    kout = T.kr;
    mode = T.core ? 2 : 0;
  }
  if (k == 0 || kout == 0) return;
  reduce_wave(M, ldm, mtrans, rows, k, d.X, d.ldx, d.xident, d.xcol0, d.w, Us);
  double* V = vbuf + it.voff;
  for (int p = threadIdx.x; p < kout * d.w; p += 64) {
    int i = p % kout, col = p / kout;
    double v;
    if (mode == 0) {
      v = Us[i * PW + col];
    } else if (mode == 1) {
      v = 0.0;
      for (int c = 0; c < T.kr; ++c) v += T.core[i + int64_t(c) * T.kl] * Us[c * PW + col];
    } else {
      v = 0.0;
      for (int c = 0; c < T.kl; ++c) v += T.core[c + int64_t(i) * T.kl] * Us[c * PW + col];
    }
    V[p] = v;
  }
}

// ---------------------------------------------------------------- subtree tasks
__device__ __forceinline__ void task_input(const Task& tk, const TDesc* td, const double*& X, int& ldx, int& w,
                                           int& xident, int& xc0) {
  if (tk.t >= 0) {
    const TDesc& d = td[tk.t];
    w = d.w;
    if (tk.X) {
      X = tk.X;
      ldx = tk.ldx;
      xident = 0;
      xc0 = 0;
    } else {
      X = d.X;
      ldx = d.ldx;
      xident = d.xident;
      xc0 = d.xcol0;
    }
  } else {
    X = tk.X;
    ldx = tk.ldx;
    w = tk.w;
    xident = 0;
    xc0 = 0;
  }
}

__global__ void __launch_bounds__(64) k_leaf_p1(const LeafItem* __restrict__ items, const Task* __restrict__ tasks,
                                               const TDesc* __restrict__ td, TreeView tv, MatView ma, MatView mb,
                                               double* __restrict__ ws) {
  __shared__ double Us[64 * PW];
  const LeafItem it = items[blockIdx.x];
  const Task tk = tasks[it.task];
  const double* X;
  int ldx, w, xident, xc0;
  task_input(tk, td, X, ldx, w, xident, xc0);
  if (w == 0) return;
  const MatView& mv = tk.mat ? mb : ma;
  const int b = it.block;
  const int k = mv.rank[b];
  if (k == 0) return;
  const int qt = tv.b_tau[tk.q], qs = tv.b_sigma[tk.q];
  const int bt = tv.b_tau[b], bs = tv.b_sigma[b];
  const int m = tv.c_size[bt], n = tv.c_size[bs];
  const double* base = mv.pool + mv.off[b];
  const double* M;
  int rows, ro, ldm;
  if (!tk.trans) {  // T = R^T X[sigma_b]
    M = base + int64_t(k) * m;
    ldm = n;
    rows = n;
    ro = tv.c_begin[bs] - tv.c_begin[qs];
  } else {  // T = L^T X[tau_b]
    M = base;
    ldm = m;
    rows = m;
    ro = tv.c_begin[bt] - tv.c_begin[qt];
  }
  const double* Xr = xident ? X : X + ro;
  reduce_wave(M, ldm, 0, rows, k, Xr, ldx, xident, xc0 - ro, w, Us);
  double* T = ws + tk.tws + (mv.kpref[tv.b_dfs[b]] - mv.kpref[tk.lo]) * PW;
  for (int p = threadIdx.x; p < k * w; p += 64) {
    int i = p % k, col = p / k;
    T[p] = Us[i * PW + col];
  }
}

__global__ void __launch_bounds__(64) k_subtree_p2(const RowItem* __restrict__ items, const Task* __restrict__ tasks,
                                                  const TDesc* __restrict__ td, TreeView tv, MatView ma, MatView mb,
                                                  const double* __restrict__ ws) {
  __shared__ double Vs[64 * PW];
  const RowItem it = items[blockIdx.x];
  const Task tk = tasks[it.owner];
  const double* X;
  int ldx, w, xident, xc0;
  task_input(tk, td, X, ldx, w, xident, xc0);
  if (w == 0) return;
  const MatView& mv = tk.mat ? mb : ma;
  const int qt = tv.b_tau[tk.q], qs = tv.b_sigma[tk.q];
  const int outc = tk.trans ? qs : qt, inc = tk.trans ? qt : qs;
  const int in0 = tv.c_begin[inc], in1 = in0 + tv.c_size[inc];
  const int c = tv.leaf_clusters[it.lc];
  const int row_lo = tv.c_begin[c] + it.chunk * 64;
  const int nr = min(64, tv.c_begin[c] + tv.c_size[c] - row_lo);
  const int lane = threadIdx.x;
  const bool rok = lane < nr;
  const int row = row_lo + (rok ? lane : 0);
  double acc[PW];
#pragma unroll
  for (int s = 0; s < PW; ++s) acc[s] = 0.0;
  for (int a = c; a >= 0; a = tv.c_parent[a]) {
    const int p0 = tk.trans ? tv.bcol_ptr[a] : tv.brow_ptr[a];
    const int p1 = tk.trans ? tv.bcol_ptr[a + 1] : tv.brow_ptr[a + 1];
    for (int p = p0; p < p1; ++p) {
      const int b = tk.trans ? tv.bcol_blk[p] : tv.brow_blk[p];
      const int oth = tk.trans ? tv.b_tau[b] : tv.b_sigma[b];
      const int o0 = tv.c_begin[oth], o1 = o0 + tv.c_size[oth];
      if (o0 < in0 || o1 > in1) continue;
      const int bt = tv.b_tau[b], bs = tv.b_sigma[b];
      const int m = tv.c_size[bt], n = tv.c_size[bs];
      const double* base = mv.pool + mv.off[b];
      const int64_t ridx = row - tv.c_begin[a];
      if (tv.b_kind[b] == KIND_F) {
        const int k = mv.rank[b];
        if (k == 0) continue;
        const double* V = ws + tk.tws + (mv.kpref[tv.b_dfs[b]] - mv.kpref[tk.lo]) * PW;
        stage_v(V, k, w, Vs);
        if (rok) {
          if (!tk.trans) expand_row(base, ridx, m, 0, k, Vs, w, acc);
          else expand_row(base + int64_t(k) * m, ridx, n, 0, k, Vs, w, acc);
        }
        __syncthreads();
      } else {
        // dense leaf: stream its input rows through LDS in chunks of 64
        const int nin = tk.trans ? m : n;
        const int xo = o0 - in0;
        for (int j0 = 0; j0 < nin; j0 += 64) {
          const int jn = min(64, nin - j0);
          for (int i = lane; i < jn * w; i += 64) {
            int j = i % jn, col = i / jn;
            int r = xo + j0 + j;
            Vs[j * PW + col] = xident ? (r == xc0 + col ? 1.0 : 0.0) : X[r + int64_t(col) * ldx];
          }
          __syncthreads();
          if (rok) {
            for (int j = 0; j < jn; ++j) {
              double dv = tk.trans ? base[(j0 + j) + ridx * m] : base[ridx + int64_t(j0 + j) * m];
#pragma unroll
              for (int col = 0; col < PW; ++col)
                if (col < w) acc[col] += dv * Vs[j * PW + col];
            }
          }
          __syncthreads();
        }
      }
    }
    if (a == outc) break;
  }
  if (rok) {
    const int64_t orow = row - tv.c_begin[outc];
#pragma unroll
    for (int col = 0; col < PW; ++col)
      if (col < w) tk.Y[orow + int64_t(col) * tk.ldy] = acc[col];
  }
}

// ---------------------------------------------------------------- target gather
__global__ void __launch_bounds__(64) k_gather(const RowItem* __restrict__ items, const TDesc* __restrict__ td,
                                              const TInfo* __restrict__ ti, const HPair* __restrict__ hp, TreeView tv,
                                              const double* __restrict__ vbuf) {
  __shared__ double Vs[64 * PW];
  const RowItem it = items[blockIdx.x];
  const TDesc d = td[it.owner];
  if (d.w == 0) return;
  const TInfo inf = ti[it.owner];
  const int tb = inf.block;
  const int outc = d.trans ? tv.b_sigma[tb] : tv.b_tau[tb];
  const int c = tv.leaf_clusters[it.lc];
  const int row_lo = tv.c_begin[c] + it.chunk * 64;
  const int nr = min(64, tv.c_begin[c] + tv.c_size[c] - row_lo);
  const int lane = threadIdx.x;
  const bool rok = lane < nr;
  const int row = row_lo + (rok ? lane : 0);
  const int w = d.w;
  double acc[PW];
#pragma unroll
  for (int s = 0; s < PW; ++s) acc[s] = 0.0;
  int64_t voff = inf.vbase;
  for (int a = tb; a >= 0; a = tv.b_parent[a]) {
    for (int i = tv.group_ptr[a]; i < tv.group_ptr[a + 1]; ++i) {
      const Term T = tv.terms[i];
      const int kout = d.trans ? T.kr : T.kl;
      const double* V = vbuf + voff;
      voff += int64_t(T.kl > T.kr ? T.kl : T.kr) * PW;
      if (kout == 0) continue;
      stage_v(V, kout, w, Vs);
      if (rok) {
        if (!d.trans) expand_row(T.L, row - T.lrow0, T.ldl, 0, kout, Vs, w, acc);
        else expand_row(T.R, row - T.rrow0, T.ldr, T.rtrans, kout, Vs, w, acc);
      }
      __syncthreads();
    }
  }
  const int64_t orow = row - tv.c_begin[outc];
  const int ld2 = tv.c_size[outc];
  if (rok) {
    for (int j = inf.hp_begin; j < inf.hp_end; ++j) {
      const double* T2 = hp[j].temp2;
#pragma unroll
      for (int col = 0; col < PW; ++col)
        if (col < w) acc[col] += T2[orow + int64_t(col) * ld2];
    }
#pragma unroll
    for (int col = 0; col < PW; ++col)
      if (col < w) {
        int jo = col < d.split ? col : col + d.gap;
        d.Y[orow + int64_t(jo) * d.ldy] = acc[col];
      }
  }
}

// ---------------------------------------------------------------- launch wrappers
template <class ItemT>
static void launch_items(void (*kern)(const ItemT*, const Task*, const TDesc*, TreeView, MatView, MatView, double*),
                         const ItemT* items, size_t n, const Task* tasks, const TDesc* td, const TreeView& tv,
                         const MatView& ma, const MatView& mb, double* ws, hipStream_t s) {
  const size_t maxg = size_t(1) << 30;
  for (size_t b = 0; b < n; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, n - b));
    hipLaunchKernelGGL(kern, dim3(cnt), dim3(64), 0, s, items + b, tasks, td, tv, ma, mb, ws);
    HM_CHECK_HIP(hipGetLastError());
  }
}

void launch_leaf_p1(const LeafItem* items, size_t n, const Task* tasks, const TDesc* td, const TreeView& tv,
                    const MatView& ma, const MatView& mb, double* ws, hipStream_t s) {
  if (n) launch_items(k_leaf_p1, items, n, tasks, td, tv, ma, mb, ws, s);
}

void launch_subtree_p2(const RowItem* items, size_t n, const Task* tasks, const TDesc* td, const TreeView& tv,
                       const MatView& ma, const MatView& mb, const double* ws, hipStream_t s) {
  const size_t maxg = size_t(1) << 30;
  for (size_t b = 0; b < n; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, n - b));
    hipLaunchKernelGGL(k_subtree_p2, dim3(cnt), dim3(64), 0, s, items + b, tasks, td, tv, ma, mb, ws);
    HM_CHECK_HIP(hipGetLastError());
  }
}

void launch_term_p1(const TermItem* items, size_t n, const TDesc* td, const TInfo* ti, const TreeView& tv,
                    double* vbuf, hipStream_t s) {
  const size_t maxg = size_t(1) << 30;
  for (size_t b = 0; b < n; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, n - b));
    hipLaunchKernelGGL(k_term_p1, dim3(cnt), dim3(64), 0, s, items + b, td, ti, tv, vbuf);
    HM_CHECK_HIP(hipGetLastError());
  }
}

void launch_gather(const RowItem* items, size_t n, const TDesc* td, const TInfo* ti, const HPair* hp,
                   const TreeView& tv, const double* vbuf, hipStream_t s) {
  const size_t maxg = size_t(1) << 30;
  for (size_t b = 0; b < n; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, n - b));
    hipLaunchKernelGGL(k_gather, dim3(cnt), dim3(64), 0, s, items + b, td, ti, hp, tv, vbuf);
    HM_CHECK_HIP(hipGetLastError());
  }
}

}  // namespace hm
