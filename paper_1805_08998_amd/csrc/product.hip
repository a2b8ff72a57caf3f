// Product kernels: products of sum-expressions with blocks of vectors.
//
// A sum-expression S(tau, sigma) = sum_i L_i core_i R_i^T + sum_j A[tau, rho_j] B[rho_j, sigma]
// (Def. 3.1) is applied to a panel X as in the identity that closes Section 3:
//   S X = sum_i L_i (core_i (R_i^T X)) + sum_j A[tau, rho_j] (B[rho_j, sigma] X),
// and S^T X likewise with the roles of the factors exchanged. The low-rank
// terms are views into the factor pools (restriction by index shift), the
// pairs are products with whole subtrees of A and B (Algorithm 2 on a block).
//
// Work decomposition (64-lane waves, PW = 16 columns per pass, all products on
// v_mfma_f64_16x16x4f64):
//   k_fused_terms / k_fused_terms4  per target with clusters of <= 64 / <= 256 rows:
//               Y = sum_i P_i (core_i (M_i^T X)) + sum_j pair_j in one kernel
//   k_term_reduce per (large target, term): V = core (M^T X)
//   k_gather_mfma per (large target, output leaf cluster): Y = sum_i P_i V_i + sum_j pair_j
//   k_leaf_reduce per (subtree task, low-rank leaf): T = R^T X (or L^T X)
//   k_subtree_expand per (subtree task, output leaf cluster): Y = sum over the
//               leaves whose rows contain it of L T or D X (or the transposes)
// Every output row is written by exactly one work item, in a fixed order, so
// results do not depend on scheduling.
#include "product_kernels.h"
#include "device_common.h"
#include "hmat_internal.h"

namespace hm {

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

// ---------------------------------------------------------------- fused small targets
// One wave applies a whole target whose input and output clusters have at most
// 64 rows: for every low-rank term of every ancestor, U = M^T X (M = R forward,
// L transposed), V = core U (or core^T U), Y += P V (P = L forward, R transposed),
// all on v_mfma_f64_16x16x4f64. Operand layouts on gfx950: A[i][k] at lane i + 16k,
// B[k][j] at lane j + 16k, and accumulator register v of lane l holds D[l/16 + 4v][l%16]
// -- so accumulator register v is exactly the B operand of K-step v of the next product.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// v if c else 0. v is loaded unconditionally from an in-bounds (clamped) address and
// scaled by 0 or 1, so the compiler keeps the load outside any branch and the steps of a
// loop stay straight-line (panel values are finite).
__device__ __forceinline__ double masked(bool c, double v) { return v * (c ? 1.0 : 0.0); }

// Panels and factors live in device global memory. Pointers read from descriptors are
// generic, and loads through them compile to flat loads; through a global-address-space
// pointer they are global loads.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ dbl4 mfma4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <class TS>
__global__ void __launch_bounds__(64) k_fused_terms(const int32_t* __restrict__ tlist, const TDesc* __restrict__ td,
                                                   const TInfo* __restrict__ ti, const HPair* __restrict__ hp,
                                                   TreeView tv) {
  const int t = tlist[blockIdx.x];
  const TDesc d = td[t];
  if (d.w == 0) return;
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  const TInfo inf = ti[t];
  const int tb = inf.block;
  const int tau = tv.b_tau[tb], sig = tv.b_sigma[tb];
  const int outc = d.trans ? sig : tau, inc = d.trans ? tau : sig;
  const int nout = tv.c_size[outc], nin = tv.c_size[inc];
  const int out0 = tv.c_begin[outc], in0 = tv.c_begin[inc];
  const int w = d.w;
  const int ksteps = (nin + 3) >> 2;  // K-steps over the input rows
  const int ntile = (nout + 15) >> 4;
  // X as B operands: xb[s] = X(4s + lk, li)
  double xb[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int r = 4 * s + lk;
    double v = 0.0;
    if (r < nin && li < w) v = d.xident ? (r == d.xcol0 + li ? 1.0 : 0.0) : d.X[r + int64_t(li) * d.ldx];
    xb[s] = v;
  }
  dbl4 y[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) y[q] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int a = d.accum ? -1 : tb; a >= 0; a = tv.b_parent[a]) {
    for (int it = tv.group_ptr[a]; it < tv.group_ptr[a + 1]; ++it) {
      const TermT<TS> T = tree_terms<TS>(tv)[it];
      // reduction operand M (rows = input cluster), expansion operand P (rows = output cluster)
      const TS* M;
      int ldm, mtr, kin;
      const TS* P;
      int ldp, ptr, kp;
      if (!d.trans) {
        const int rr = in0 - T.rrow0;
        M = T.rtrans ? T.R + int64_t(rr) * T.ldr : T.R + rr;
        ldm = T.ldr;
        mtr = T.rtrans;
        kin = T.kr;
        P = T.L + (out0 - T.lrow0);
        ldp = T.ldl;
        ptr = 0;
        kp = T.kl;
      } else {
        M = T.L + (in0 - T.lrow0);
        ldm = T.ldl;
        mtr = 0;
        kin = T.kl;
        const int rr = out0 - T.rrow0;
        P = T.rtrans ? T.R + int64_t(rr) * T.ldr : T.R + rr;
        ldp = T.ldr;
        ptr = T.rtrans;
        kp = T.kr;
      }
      const int nkb = (kin + 15) >> 4;
      dbl4 U[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        U[kb] = dbl4{0.0, 0.0, 0.0, 0.0};
        if (kb < nkb) {
          const int c = 16 * kb + li;
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            if (s < ksteps) {
              const int r = 4 * s + lk;
              double av = 0.0;
              if (c < kin && r < nin) av = mtr ? M[c + int64_t(r) * ldm] : M[r + int64_t(c) * ldm];
              U[kb] = mfma4(av, xb[s], U[kb]);
            }
          }
        }
      }
      dbl4 V[4];
      int nob;
      if (T.core) {
        nob = (kp + 15) >> 4;
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
          V[ob] = dbl4{0.0, 0.0, 0.0, 0.0};
          if (ob < nob) {
            const int i = 16 * ob + li;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
              if (kb < nkb) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                  const int cc = 16 * kb + 4 * s4 + lk;
                  double av = 0.0;
                  if (i < kp && cc < kin) av = d.trans ? T.core[cc + int64_t(i) * T.kl] : T.core[i + int64_t(cc) * T.kl];
                  V[ob] = mfma4(av, U[kb][s4], V[ob]);
                }
              }
            }
          }
        }
      } else {
        nob = nkb;
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) V[ob] = U[ob];
      }
#pragma unroll
      for (int tile = 0; tile < 4; ++tile) {
        if (tile < ntile) {
          const int row = 16 * tile + li;
#pragma unroll
          for (int ob = 0; ob < 4; ++ob) {
            if (ob < nob) {
#pragma unroll
              for (int s4 = 0; s4 < 4; ++s4) {
                const int cc = 16 * ob + 4 * s4 + lk;
                double av = 0.0;
                if (cc < kp && row < nout) av = ptr ? P[cc + int64_t(row) * ldp] : P[row + int64_t(cc) * ldp];
                y[tile] = mfma4(av, V[ob][s4], y[tile]);
              }
            }
          }
        }
      }
    }
  }
  // pair results and output: y[tile][v] = Y(16 tile + lk + 4v, li)
#pragma unroll
  for (int tile = 0; tile < 4; ++tile) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * tile + lk + 4 * v;
      if (tile < ntile && row < nout && li < w) {
        const int jo = li < d.split ? li : li + d.gap;
        double val = d.accum ? d.Y[row + int64_t(jo) * d.ldy] : y[tile][v];
        for (int j = inf.hp_begin; j < inf.hp_end; ++j) val += hp[j].temp2[row + int64_t(li) * nout];
        d.Y[row + int64_t(jo) * d.ldy] = val;
      }
    }
  }
}

// ---------------------------------------------------------------- subtree products on MFMA
// Work items: item g belongs to the task k with pre[k] <= g < pre[k+1], and is the
// (g - pre[k])-th depth-first leaf of the task's subtree (reduction) or leaf cluster of its
// output (expansion). The subtree kernels read (k, g - pre[k]) from a table written on the
// device when the task list is uploaded (one load instead of a search of dependent loads).

// u = M[:, 16 kb : 16 kb + 16]^T X for one 16-column block of M (element (r, c) of the block
// at r * msr + mcol, lane column c) and X's column li (Xg points at it). Groups of four
// K-steps: the loads of a group are issued together from clamped in-bounds addresses, then
// masked. XID: X is the identity shifted by xcol0 (no X loads; Xg unused).
template <bool XID, class TS>
__device__ __forceinline__ dbl4 reduce_rows(const __attribute__((address_space(1))) TS* Mg, int64_t msr, int64_t mcol,
                                            const __attribute__((address_space(1))) double* Xg, int nin, int ks,
                                            int lk, int li, bool cok, bool lok, int xcol0) {
  dbl4 u = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < ks; s0 += 4) {
    double av[4], bv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rc = min(4 * (s0 + q) + lk, nin - 1);
      av[q] = double(Mg[int64_t(rc) * msr + mcol]);
      if constexpr (!XID) bv[q] = Xg[rc];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 4 * (s0 + q) + lk;
      double b;
      if constexpr (XID) b = (r < nin && lok && r == xcol0 + li) ? 1.0 : 0.0;
      else b = masked(r < nin && lok, bv[q]);
      u = mfma4(masked(cok && r < nin, av[q]), b, u);
    }
  }
  return u;
}

// y[tile] += D[roff + 16 tile + li, :] X for a dense leaf D (element (i, j) at
// i * dsr + j * dsj: rows of D, or of D^T for the transposed product), nin columns, X's
// column li at Xg. Groups of two K-steps: loads first (clamped), then masked MFMAs; rows
// past nr are masked, not branched. XID: X is the identity shifted by xoff (no X loads).
template <bool XID, class TS>
__device__ __forceinline__ void expand_dense(dbl4 (&y)[4], const __attribute__((address_space(1))) TS* Dg, int64_t dsr,
                                             int64_t dsj, int roff, int nr,
                                             const __attribute__((address_space(1))) double* Xg, int nin, int lk,
                                             int li, bool lok, int xoff) {
  const int ks = (nin + 3) >> 2;
  for (int s0 = 0; s0 < ks; s0 += 2) {
    double bv[2], av[2][4];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int jc = min(4 * (s0 + q) + lk, nin - 1);
      if constexpr (!XID) bv[q] = Xg[jc];
#pragma unroll
      for (int tile = 0; tile < 4; ++tile) {
        const int rcl = min(16 * tile + li, nr - 1);
        av[q][tile] = double(Dg[int64_t(roff + rcl) * dsr + int64_t(jc) * dsj]);
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int j = 4 * (s0 + q) + lk;
      const bool jok = j < nin;
      double b;
      if constexpr (XID) b = (jok && lok && j == xoff + li) ? 1.0 : 0.0;
      else b = masked(jok && lok, bv[q]);
#pragma unroll
      for (int tile = 0; tile < 4; ++tile) y[tile] = mfma4(masked(jok && 16 * tile + li < nr, av[q][tile]), b, y[tile]);
    }
  }
}

template <class TS>
__global__ void __launch_bounds__(64) k_leaf_reduce(const int32_t* __restrict__ owner, int64_t g0,
                                                   const Task* __restrict__ tasks, const TDesc* __restrict__ td,
                                                   TreeView tv, MatView ma, MatView mb, double* __restrict__ ws) {
  const int64_t g = g0 + blockIdx.x;
  const int k = owner[2 * g], item = owner[2 * g + 1];
  const Task tk = tasks[k];
  const int dfs = tk.lo + item;
  const MatView& mv = tk.mat ? mb : ma;
  const DfsRec L = mv.dfs_rec[dfs];
  const int kr = L.k;
  if (kr <= 0) return;  // nearfield leaf (-1) or rank 0
  const double* X;
  int ldx, w, xident, xc0;
  task_input(tk, td, X, ldx, w, xident, xc0);
  if (w == 0) return;
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  const int m = L.m, n = L.n;
  const TS* base = mat_pool<TS>(mv) + L.off;
  const TS* M;
  int rows, ro, ldm;
  if (!tk.trans) {
    M = base + int64_t(kr) * m;
    ldm = n;
    rows = n;
    ro = L.c0 - tv.c_begin[tv.b_sigma[tk.q]];
  } else {
    M = base;
    ldm = m;
    rows = m;
    ro = L.r0 - tv.c_begin[tv.b_tau[tk.q]];
  }
  const int nkb = (kr + 15) >> 4;
  const int ks = (rows + 3) >> 2;
  double* T = ws + tk.tws + (mv.kpref[dfs] - mv.kpref[tk.lo]) * PW;
  const int lic = min(li, w - 1);
  const bool lok = li < w;
  for (int kb = 0; kb < nkb; ++kb) {
    const int c = 16 * kb + li;
    const bool cok = c < kr;
    const int cc = min(c, kr - 1);
    const dbl4 U = xident ? reduce_rows<true>(gmem(M), 1, int64_t(cc) * ldm, gmem(X), rows, ks, lk, li, cok, lok,
                                              xc0 - ro)
                          : reduce_rows<false>(gmem(M), 1, int64_t(cc) * ldm, gmem(X + ro + int64_t(lic) * ldx), rows,
                                               ks, lk, li, cok, lok, 0);
    // U[v] = T(16 kb + lk + 4v, li); T is kr x w column-major
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * kb + lk + 4 * v;
      if (i < kr && li < w) T[i + int64_t(li) * kr] = U[v];
    }
  }
}

template <class TS>
__global__ void __launch_bounds__(64) k_subtree_expand(const int32_t* __restrict__ owner, int64_t g0,
                                                      const Task* __restrict__ tasks, const TDesc* __restrict__ td,
                                                      TreeView tv, MatView ma, MatView mb,
                                                      const double* __restrict__ ws) {
  const int64_t g = g0 + blockIdx.x;
  const int kt = owner[2 * g], item = owner[2 * g + 1];
  const Task tk = tasks[kt];
  const double* X;
  int ldx, w, xident, xc0;
  task_input(tk, td, X, ldx, w, xident, xc0);
  if (w == 0) return;
  const MatView& mv = tk.mat ? mb : ma;
  const int qt = tv.b_tau[tk.q], qs = tv.b_sigma[tk.q];
  const int outc = tk.trans ? qs : qt, inc = tk.trans ? qt : qs;
  const int in0 = tv.c_begin[inc], in1 = in0 + tv.c_size[inc];
  const int c = tv.leaf_clusters[tv.c_lc_begin[outc] + item];
  const int row_lo = tv.c_begin[c];
  const int nr = tv.c_size[c];  // leaf clusters have at most 64 rows
  const int ntile = (nr + 15) >> 4;
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  dbl4 y[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) y[q] = dbl4{0.0, 0.0, 0.0, 0.0};
  const LeafRec* lst = tk.trans ? mv.col_rec : mv.row_rec;
  const int* lptr = tk.trans ? tv.bcol_ptr : tv.brow_ptr;
  const int64_t kp_lo = mv.kpref[tk.lo];
  for (int a = c; a >= 0; a = tv.c_parent[a]) {
    int p0 = lptr[a];
    const int p1 = lptr[a + 1];
    {  // the list is sorted by the first position of the other cluster: skip to in0
      int lo = p0, hi = p1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lst[mid].o0 < in0) lo = mid + 1;
        else hi = mid;
      }
      p0 = lo;
    }
    const int roff = row_lo - tv.c_begin[a];  // first output row inside the leaves' rows
    for (int p = p0; p < p1; ++p) {
      const LeafRec L = lst[p];
      const int o0 = L.o0, o1 = o0 + L.on;
      if (o0 >= in1) break;
      if (o1 > in1) continue;
      const int m = L.m, n = L.n;
      const TS* base = mat_pool<TS>(mv) + L.off;
      if (L.k >= 0) {
        const int k = L.k;
        if (k == 0) continue;
        const double* Tm = ws + tk.tws + (int64_t(L.kp) - kp_lo) * PW;
        const TS* P = tk.trans ? base + int64_t(k) * m : base;
        const int ldp = tk.trans ? n : m;
        const int ks = (k + 3) >> 2;
        const int lic = min(li, w - 1);
        const auto Tg = gmem(Tm + int64_t(lic) * k);
        const auto Pg = gmem(P + roff);
        // groups of two K-steps, loads first (clamped), then masked MFMAs
        for (int s0 = 0; s0 < ks; s0 += 2) {
          double bv[2], av[2][4];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int ccl = min(4 * (s0 + q) + lk, k - 1);
            bv[q] = Tg[ccl];
#pragma unroll
            for (int tile = 0; tile < 4; ++tile) av[q][tile] = double(Pg[min(16 * tile + li, nr - 1) + int64_t(ccl) * ldp]);
          }
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int cc = 4 * (s0 + q) + lk;
            const double b = masked(cc < k && li < w, bv[q]);
#pragma unroll
            for (int tile = 0; tile < 4; ++tile)
              y[tile] = mfma4(masked(cc < k && 16 * tile + li < nr, av[q][tile]), b, y[tile]);
          }
        }
      } else {
        // D X (or D^T X): D is m x n column-major
        const int nin = tk.trans ? m : n;
        const int xo = o0 - in0;
        const int lic = min(li, w - 1);
        const bool lok = li < w;
        const int64_t dsr = tk.trans ? int64_t(m) : 1, dsj = tk.trans ? 1 : int64_t(m);
        if (xident)
          expand_dense<true>(y, gmem(base), dsr, dsj, roff, nr, gmem(X), nin, lk, li, lok, xc0 - xo);
        else
          expand_dense<false>(y, gmem(base), dsr, dsj, roff, nr, gmem(X + xo + int64_t(lic) * ldx), nin, lk, li, lok,
                              0);
      }
    }
    if (a == outc) break;
  }
  const int orow0 = row_lo - tv.c_begin[outc];
#pragma unroll
  for (int tile = 0; tile < 4; ++tile) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * tile + lk + 4 * v;
      if (tile < ntile && r < nr && li < w) tk.Y[(orow0 + r) + int64_t(li) * tk.ldy] = y[tile][v];
    }
  }
}

// Large targets: per (target, term) V = core (M^T X) on MFMA (M = R forward, L
// transposed), written to the target's slot; the expansion is k_gather_mfma.
template <class TS>
__global__ void __launch_bounds__(64) k_term_reduce(const TermItem* __restrict__ items, const TDesc* __restrict__ td,
                                                   const TInfo* __restrict__ ti, TreeView tv,
                                                   double* __restrict__ vbuf) {
  const TermItem it = items[blockIdx.x];
  const TDesc d = td[it.t];
  if (d.w == 0) return;
  const TermT<TS> T = tree_terms<TS>(tv)[it.term];
  const int tb = ti[it.t].block;
  const int tau = tv.b_tau[tb], sig = tv.b_sigma[tb];
  const TS* M;
  int ldm, mtr, nin, kin, kout;
  if (!d.trans) {
    const int rr = tv.c_begin[sig] - T.rrow0;
    M = T.rtrans ? T.R + int64_t(rr) * T.ldr : T.R + rr;
    ldm = T.ldr;
    mtr = T.rtrans;
    nin = tv.c_size[sig];
    kin = T.kr;
    kout = T.kl;
  } else {
    M = T.L + (tv.c_begin[tau] - T.lrow0);
    ldm = T.ldl;
    mtr = 0;
    nin = tv.c_size[tau];
    kin = T.kl;
    kout = T.kr;
  }
  if (kin == 0 || kout == 0) return;
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  const int w = d.w;
  const int nkb = (kin + 15) >> 4;
  const int nob = (kout + 15) >> 4;
  const int ks = (nin + 3) >> 2;
  const int lic = min(li, w - 1);
  const bool lok = li < w;
  double* Vout = vbuf + it.voff;  // kout x w, column-major
  // One accumulator chain per 16 columns of M, with no branches between its MFMAs:
  // loads come from clamped in-bounds addresses and are masked, so several steps'
  // loads are in flight together and the accumulator stays in place.
  dbl4 V[4];
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) V[ob] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int kb = 0; kb < nkb; ++kb) {
    const int c = 16 * kb + li;
    const bool cok = c < kin;
    const int cc = min(c, kin - 1);
    dbl4 u;
    // element (r, c) of M at r * msr + mcol
    const int64_t msr = mtr ? int64_t(ldm) : 1, mcol = mtr ? int64_t(cc) : int64_t(cc) * ldm;
    if (d.xident)
      u = reduce_rows<true>(gmem(M), msr, mcol, gmem(Vout), nin, ks, lk, li, cok, lok, d.xcol0);
    else
      u = reduce_rows<false>(gmem(M), msr, mcol, gmem(d.X + int64_t(lic) * d.ldx), nin, ks, lk, li, cok, lok, 0);
    if (T.core) {
      // V += core[:, 16 kb : 16 kb + 16] u (transposed core for the transposed pass)
      const auto Cg = gmem(T.core);
      const int64_t csr = d.trans ? 1 : T.kl, csc = d.trans ? T.kl : 1;
#pragma unroll
      for (int ob = 0; ob < 4; ++ob) {
        if (ob < nob) {
          const int i = 16 * ob + li;
          const int ic = min(i, kout - 1);
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int ccr = 16 * kb + 4 * s4 + lk;
            const int ccc = min(ccr, kin - 1);
            double av = double(Cg[int64_t(ccc) * csr + int64_t(ic) * csc]);
            av = masked(i < kout && ccr < kin, av);
            V[ob] = mfma4(av, u[s4], V[ob]);
          }
        }
      }
    } else {
      // kin == kout: u holds rows 16 kb + lk + 4 v of V
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * kb + lk + 4 * v;
        if (row < kout && lok) Vout[row + int64_t(li) * kout] = u[v];
      }
    }
  }
  if (T.core) {
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      if (ob < nob) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * ob + lk + 4 * v;
          if (row < kout && lok) Vout[row + int64_t(li) * kout] = V[ob][v];
        }
      }
    }
  }
}

template <class TS>
__global__ void __launch_bounds__(64) k_gather_mfma(const RowItem* __restrict__ items, const TDesc* __restrict__ td,
                                                   const TInfo* __restrict__ ti, const HPair* __restrict__ hp,
                                                   TreeView tv, const double* __restrict__ vbuf) {
  const RowItem it = items[blockIdx.x];
  const TDesc d = td[it.owner];
  if (d.w == 0) return;
  const TInfo inf = ti[it.owner];
  const int tb = inf.block;
  const int outc = d.trans ? tv.b_sigma[tb] : tv.b_tau[tb];
  const int c = tv.leaf_clusters[it.lc];
  const int row_lo = tv.c_begin[c];
  const int nr = tv.c_size[c];
  const int ntile = (nr + 15) >> 4;
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  const int w = d.w;
  dbl4 y[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) y[q] = dbl4{0.0, 0.0, 0.0, 0.0};
  int64_t voff = inf.vbase;
  for (int a = tb; a >= 0; a = tv.b_parent[a]) {
    for (int i = tv.group_ptr[a]; i < tv.group_ptr[a + 1]; ++i) {
      const TermT<TS> T = tree_terms<TS>(tv)[i];
      const int kout = d.trans ? T.kr : T.kl;
      const double* V = vbuf + voff;
      voff += int64_t(T.kl > T.kr ? T.kl : T.kr) * PW;
      if (kout == 0) continue;
      const TS* P;
      int ldp, ptr;
      int64_t r0;
      if (!d.trans) {
        P = T.L;
        ldp = T.ldl;
        ptr = 0;
        r0 = row_lo - T.lrow0;
      } else {
        P = T.R;
        ldp = T.ldr;
        ptr = T.rtrans;
        r0 = row_lo - T.rrow0;
      }
      const int ks = (kout + 3) >> 2;
      const int lic = min(li, w - 1);
      // element (row, col) of P at row * psr + col * psc
      const int64_t psr = ptr ? int64_t(ldp) : 1, psc = ptr ? 1 : int64_t(ldp);
      const auto Pg = gmem(P + r0 * psr);
      const auto Vg = gmem(V + int64_t(lic) * kout);
      // groups of two K-steps (five loads each), loads first, then the masked MFMAs;
      // rows past nr are masked, not branched
      for (int s0 = 0; s0 < ks; s0 += 2) {
        double bv[2], av[2][4];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int ccl = min(4 * (s0 + q) + lk, kout - 1);
          bv[q] = Vg[ccl];
#pragma unroll
          for (int tile = 0; tile < 4; ++tile) {
            const int rcl = min(16 * tile + li, nr - 1);
            av[q][tile] = double(Pg[int64_t(rcl) * psr + int64_t(ccl) * psc]);
          }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int cc = 4 * (s0 + q) + lk;
          const double b = masked(cc < kout && li < w, bv[q]);
#pragma unroll
          for (int tile = 0; tile < 4; ++tile)
            y[tile] = mfma4(masked(cc < kout && 16 * tile + li < nr, av[q][tile]), b, y[tile]);
        }
      }
    }
  }
  const int orow0 = row_lo - tv.c_begin[outc];
  const int ld2 = tv.c_size[outc];
#pragma unroll
  for (int tile = 0; tile < 4; ++tile) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * tile + lk + 4 * v;
      if (tile < ntile && r < nr && li < w) {
        const int64_t orow = orow0 + r;
        double val = y[tile][v];
        for (int j = inf.hp_begin; j < inf.hp_end; ++j) val += hp[j].temp2[orow + int64_t(li) * ld2];
        const int jo = li < d.split ? li : li + d.gap;
        d.Y[orow + int64_t(jo) * d.ldy] = val;
      }
    }
  }
}

void launch_term_reduce(const TermItem* items, size_t n, const TDesc* td, const TInfo* ti, const TreeView& tv,
                        double* vbuf, hipStream_t s, bool lowp) {
  const size_t maxg = size_t(max_groups(64));
  for (size_t b = 0; b < n; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, n - b));
    if (lowp) hipLaunchKernelGGL(k_term_reduce<float>, dim3(cnt), dim3(64), 0, s, items + b, td, ti, tv, vbuf);
    else hipLaunchKernelGGL(k_term_reduce<double>, dim3(cnt), dim3(64), 0, s, items + b, td, ti, tv, vbuf);
    HM_CHECK_HIP(hipGetLastError());
  }
}

void launch_gather_mfma(const RowItem* items, size_t n, const TDesc* td, const TInfo* ti, const HPair* hp,
                        const TreeView& tv, const double* vbuf, hipStream_t s, bool lowp) {
  const size_t maxg = size_t(max_groups(64));
  for (size_t b = 0; b < n; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, n - b));
    if (lowp) hipLaunchKernelGGL(k_gather_mfma<float>, dim3(cnt), dim3(64), 0, s, items + b, td, ti, hp, tv, vbuf);
    else hipLaunchKernelGGL(k_gather_mfma<double>, dim3(cnt), dim3(64), 0, s, items + b, td, ti, hp, tv, vbuf);
    HM_CHECK_HIP(hipGetLastError());
  }
}

// owner[2 g] = k and owner[2 g + 1] = g - pre[k] for pre[k] <= g < pre[k + 1]: one
// workgroup per task
__global__ void __launch_bounds__(64) k_fill_owner(const int64_t* __restrict__ pre, int ntask,
                                                  int32_t* __restrict__ owner) {
  const int k = blockIdx.x;
  if (k >= ntask) return;
  const int64_t g0 = pre[k], g1 = pre[k + 1];
  for (int64_t g = g0 + threadIdx.x; g < g1; g += 64) {
    owner[2 * g] = k;
    owner[2 * g + 1] = int32_t(g - g0);
  }
}

void launch_fill_owner(const int64_t* pre, int ntask, int32_t* owner, hipStream_t s) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(k_fill_owner, dim3(unsigned(ntask)), dim3(64), 0, s, pre, ntask, owner);
  HM_CHECK_HIP(hipGetLastError());
}

void launch_leaf_reduce(const int32_t* owner, int64_t nitems, const Task* tasks, const TDesc* td, const TreeView& tv,
                        const MatView& ma, const MatView& mb, double* ws, hipStream_t s, bool lowp) {
  const int64_t maxg = max_groups(64);
  for (int64_t b = 0; b < nitems; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, nitems - b));
    if (lowp)
      hipLaunchKernelGGL(k_leaf_reduce<float>, dim3(cnt), dim3(64), 0, s, owner, b, tasks, td, tv, ma, mb, ws);
    else
      hipLaunchKernelGGL(k_leaf_reduce<double>, dim3(cnt), dim3(64), 0, s, owner, b, tasks, td, tv, ma, mb, ws);
    HM_CHECK_HIP(hipGetLastError());
  }
}

void launch_subtree_expand(const int32_t* owner, int64_t nitems, const Task* tasks, const TDesc* td,
                           const TreeView& tv, const MatView& ma, const MatView& mb, const double* ws,
                           hipStream_t s, bool lowp) {
  const int64_t maxg = max_groups(64);
  for (int64_t b = 0; b < nitems; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, nitems - b));
    if (lowp)
      hipLaunchKernelGGL(k_subtree_expand<float>, dim3(cnt), dim3(64), 0, s, owner, b, tasks, td, tv, ma, mb, ws);
    else
      hipLaunchKernelGGL(k_subtree_expand<double>, dim3(cnt), dim3(64), 0, s, owner, b, tasks, td, tv, ma, mb, ws);
    HM_CHECK_HIP(hipGetLastError());
  }
}

// Four waves per target for clusters of up to 256 rows: wave q reduces input rows
// [64q, 64q + 64) and expands output rows [64q, 64q + 64); the partial products
// M^T X of the four waves are summed through double-buffered LDS (one barrier per term).
template <class TS>
__global__ void __launch_bounds__(256) k_fused_terms4(const int32_t* __restrict__ tlist, const TDesc* __restrict__ td,
                                                     const TInfo* __restrict__ ti, const HPair* __restrict__ hp,
                                                     TreeView tv) {
  __shared__ double ulds[2][4][4][4][64];  // buffer, wave, k-block, register, lane
  const int t = tlist[blockIdx.x];
  const TDesc d = td[t];
  if (d.w == 0) return;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const TInfo inf = ti[t];
  const int tb = inf.block;
  const int tau = tv.b_tau[tb], sig = tv.b_sigma[tb];
  const int outc = d.trans ? sig : tau, inc = d.trans ? tau : sig;
  const int nout = tv.c_size[outc], nin = tv.c_size[inc];
  const int out0 = tv.c_begin[outc], in0 = tv.c_begin[inc];
  const int w = d.w;
  const int rin0 = 64 * wid, rout0 = 64 * wid;  // this wave's input / output row offset
  const int nin_w = max(0, min(64, nin - rin0)), nout_w = max(0, min(64, nout - rout0));
  const int ksteps = (nin_w + 3) >> 2;
  const int ntile = (nout_w + 15) >> 4;
  double xb[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int r = 4 * s + lk;
    double v = 0.0;
    if (r < nin_w && li < w) {
      const int rr = rin0 + r;
      v = d.xident ? (rr == d.xcol0 + li ? 1.0 : 0.0) : d.X[rr + int64_t(li) * d.ldx];
    }
    xb[s] = v;
  }
  dbl4 y[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) y[q] = dbl4{0.0, 0.0, 0.0, 0.0};
  int buf = 0;
  for (int a = d.accum ? -1 : tb; a >= 0; a = tv.b_parent[a]) {
    for (int it = tv.group_ptr[a]; it < tv.group_ptr[a + 1]; ++it) {
      const TermT<TS> T = tree_terms<TS>(tv)[it];
      const TS* M;
      int ldm, mtr, kin;
      const TS* P;
      int ldp, ptr, kp;
      if (!d.trans) {
        const int rr = in0 - T.rrow0;
        M = T.rtrans ? T.R + int64_t(rr) * T.ldr : T.R + rr;
        ldm = T.ldr;
        mtr = T.rtrans;
        kin = T.kr;
        P = T.L + (out0 - T.lrow0);
        ldp = T.ldl;
        ptr = 0;
        kp = T.kl;
      } else {
        M = T.L + (in0 - T.lrow0);
        ldm = T.ldl;
        mtr = 0;
        kin = T.kl;
        const int rr = out0 - T.rrow0;
        P = T.rtrans ? T.R + int64_t(rr) * T.ldr : T.R + rr;
        ldp = T.ldr;
        ptr = T.rtrans;
        kp = T.kr;
      }
      const int nkb = (kin + 15) >> 4;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        if (kb < nkb) {
          dbl4 u = dbl4{0.0, 0.0, 0.0, 0.0};
          const int c = 16 * kb + li;
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            if (s < ksteps) {
              const int r = rin0 + 4 * s + lk;
              double av = 0.0;
              if (c < kin && 4 * s + lk < nin_w) av = mtr ? M[c + int64_t(r) * ldm] : M[r + int64_t(c) * ldm];
              u = mfma4(av, xb[s], u);
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) ulds[buf][wid][kb][v][lane] = u[v];
        }
      }
      __syncthreads();
      dbl4 U[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        U[kb] = dbl4{0.0, 0.0, 0.0, 0.0};
        if (kb < nkb) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            U[kb][v] = ulds[buf][0][kb][v][lane] + ulds[buf][1][kb][v][lane] + ulds[buf][2][kb][v][lane] +
                       ulds[buf][3][kb][v][lane];
        }
      }
      buf ^= 1;
      dbl4 V[4];
      int nob;
      if (T.core) {
        nob = (kp + 15) >> 4;
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
          V[ob] = dbl4{0.0, 0.0, 0.0, 0.0};
          if (ob < nob) {
            const int i = 16 * ob + li;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
              if (kb < nkb) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                  const int cc = 16 * kb + 4 * s4 + lk;
                  double av = 0.0;
                  if (i < kp && cc < kin) av = d.trans ? T.core[cc + int64_t(i) * T.kl] : T.core[i + int64_t(cc) * T.kl];
                  V[ob] = mfma4(av, U[kb][s4], V[ob]);
                }
              }
            }
          }
        }
      } else {
        nob = nkb;
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) V[ob] = U[ob];
      }
#pragma unroll
      for (int tile = 0; tile < 4; ++tile) {
        if (tile < ntile) {
          const int r = 16 * tile + li;
#pragma unroll
          for (int ob = 0; ob < 4; ++ob) {
            if (ob < nob) {
#pragma unroll
              for (int s4 = 0; s4 < 4; ++s4) {
                const int cc = 16 * ob + 4 * s4 + lk;
                double av = 0.0;
                if (cc < kp && r < nout_w) {
                  const int row = rout0 + r;
                  av = ptr ? P[cc + int64_t(row) * ldp] : P[row + int64_t(cc) * ldp];
                }
                y[tile] = mfma4(av, V[ob][s4], y[tile]);
              }
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int tile = 0; tile < 4; ++tile) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * tile + lk + 4 * v;
      if (tile < ntile && r < nout_w && li < w) {
        const int row = rout0 + r;
        const int jo = li < d.split ? li : li + d.gap;
        double val = d.accum ? d.Y[row + int64_t(jo) * d.ldy] : y[tile][v];
        for (int j = inf.hp_begin; j < inf.hp_end; ++j) val += hp[j].temp2[row + int64_t(li) * nout];
        d.Y[row + int64_t(jo) * d.ldy] = val;
      }
    }
  }
}

void launch_fused_terms4(const int32_t* tlist, size_t n, const TDesc* td, const TInfo* ti, const HPair* hp,
                         const TreeView& tv, hipStream_t s, bool lowp) {
  const size_t maxg = size_t(max_groups(256));
  for (size_t b = 0; b < n; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, n - b));
    if (lowp) hipLaunchKernelGGL(k_fused_terms4<float>, dim3(cnt), dim3(256), 0, s, tlist + b, td, ti, hp, tv);
    else hipLaunchKernelGGL(k_fused_terms4<double>, dim3(cnt), dim3(256), 0, s, tlist + b, td, ti, hp, tv);
    HM_CHECK_HIP(hipGetLastError());
  }
}

void launch_fused_terms(const int32_t* tlist, size_t n, const TDesc* td, const TInfo* ti, const HPair* hp,
                        const TreeView& tv, hipStream_t s, bool lowp) {
  const size_t maxg = size_t(max_groups(64));
  for (size_t b = 0; b < n; b += maxg) {
    unsigned cnt = unsigned(std::min(maxg, n - b));
    if (lowp) hipLaunchKernelGGL(k_fused_terms<float>, dim3(cnt), dim3(64), 0, s, tlist + b, td, ti, hp, tv);
    else hipLaunchKernelGGL(k_fused_terms<double>, dim3(cnt), dim3(64), 0, s, tlist + b, td, ti, hp, tv);
    HM_CHECK_HIP(hipGetLastError());
  }
}

}  // namespace hm

namespace hm {

// Nearfield targets of at most 256 x 256: C[tau, sigma] = sum_i L_i core_i R_i^T +
// sum_j A[tau, rho_j] B[rho_j, sigma] over the pairs of two dense leaves,
// evaluated directly (S applied to the identity, the nearfield step of
// Algorithm 4, without forming S I column block by column block). Pairs with a
// subdivided factor are added afterwards through identity panels. One
// workgroup per 64-row block of a target (item = target, row block), which takes
// the target's 64-column blocks in turn; wave q owns columns [16q, 16q + 16) of
// each, so every term panel is read once per 64 x 64 sub-block instead of once
// per 16 columns, and from L2 after the first column block. Every term of a direct target has
// kl, kr <= NEAR_TERM_MAX (the host routes other targets to the identity panels), so
// V below holds a whole term.
__global__ void __launch_bounds__(256) k_near_direct(const int32_t* __restrict__ items,
                                                    const int32_t* __restrict__ blocks,
                                                    const int64_t* __restrict__ coff,
                                                    const int32_t* __restrict__ pptr,
                                                    const int32_t* __restrict__ pairs, TreeView tv, MatView ma,
                                                    MatView mb, double* __restrict__ cpool) {
  const int t = items[2 * blockIdx.x], rc = items[2 * blockIdx.x + 1];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int tb = blocks[t];
  const int tau = tv.b_tau[tb], sig = tv.b_sigma[tb];
  const int mt = tv.c_size[tau], nt = tv.c_size[sig];
  const int rb0 = 64 * (rc >> 16);   // row block origin
  const int m = min(64, mt - rb0);   // rows of this row block
  const int n = nt;
  const int out0 = tv.c_begin[tau] + rb0, in0 = tv.c_begin[sig];
  // the column blocks of the row block one after the other: the term panels and A rows
  // this workgroup reads for the first come from L2 for the others
  for (int cb0 = 0; cb0 < n; cb0 += 64) {
  const int col0 = cb0 + 16 * wid;
  if (col0 >= min(n, cb0 + 64)) break;  // no columns for this wave here or further right; no barriers follow
  const int ntile = (m + 15) >> 4;
  const int jc = col0 + li;  // column of this lane in B operands and in the output
  const bool jok = jc < n && jc < cb0 + 64;
  const int jcl = min(jc, min(n, cb0 + 64) - 1);  // clamped: every lane loads in bounds
  // All loads below come from clamped in-bounds addresses and are masked, so the MFMA
  // chains run without branches and the loads of a group are in flight together.
  dbl4 y[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) y[q] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int a = tb; a >= 0; a = tv.b_parent[a]) {
    for (int it = tv.group_ptr[a]; it < tv.group_ptr[a + 1]; ++it) {
      const Term T = tv.terms[it];
      const int kl = T.kl, kr = T.kr;
      const int64_t rrow = int64_t(in0 + jcl - T.rrow0);  // R row of this lane's column
      const int rt = T.rtrans;
      // V = core R_slab^T (kl x 16) in accumulator layout: V[ob][v] = V(16 ob + lk + 4 v, li)
      const int nob = (kl + 15) >> 4;
      dbl4 V[4];
      if (T.core) {
        const int ks = (kr + 3) >> 2;
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
          V[ob] = dbl4{0.0, 0.0, 0.0, 0.0};
          if (ob < nob) {
            const int i = 16 * ob + li;
            const int icl = min(i, kl - 1);
            for (int s0 = 0; s0 < ks; s0 += 4) {
              double av[4], bv[4];
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int ccl = min(4 * (s0 + q) + lk, kr - 1);
                av[q] = T.core[icl + int64_t(ccl) * kl];
                bv[q] = rt ? T.R[ccl + rrow * T.ldr] : T.R[rrow + int64_t(ccl) * T.ldr];
              }
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int cc = 4 * (s0 + q) + lk;
                V[ob] = mfma4(masked(i < kl && cc < kr, av[q]), masked(cc < kr && jok, bv[q]), V[ob]);
              }
            }
          }
        }
      } else {
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int cc = 16 * ob + lk + 4 * v;
            const int ccl = min(cc, kr - 1);
            const double val = rt ? T.R[ccl + rrow * T.ldr] : T.R[rrow + int64_t(ccl) * T.ldr];
            V[ob][v] = masked(ob < nob && cc < kr && jok, val);
          }
        }
      }
      // y += L_tau V: all four row tiles, rows past m masked
      const int64_t lr = int64_t(out0 - T.lrow0);
#pragma unroll
      for (int ob = 0; ob < 4; ++ob) {
        if (ob < nob) {
          double av[4][4];
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int ccl = min(16 * ob + 4 * s4 + lk, kl - 1);
#pragma unroll
            for (int tile = 0; tile < 4; ++tile)
              av[s4][tile] = T.L[(lr + min(16 * tile + li, m - 1)) + int64_t(ccl) * T.ldl];
          }
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int cc = 16 * ob + 4 * s4 + lk;
#pragma unroll
            for (int tile = 0; tile < 4; ++tile)
              y[tile] = mfma4(masked(cc < kl && 16 * tile + li < m, av[s4][tile]), V[ob][s4], y[tile]);
          }
        }
      }
    }
  }
  // dense pairs: y += A[tau, rho] B[rho, sigma][:, slab], two K-steps per group
  for (int p = pptr[t]; p < pptr[t + 1]; ++p) {
    const int qa = pairs[2 * p], qb = pairs[2 * p + 1];
    const int nr = tv.c_size[tv.b_sigma[qa]];
    const double* Ab = ma.pool + ma.off[qa] + rb0;  // rows of this sub-block, leading dimension mt
    const double* Bb = mb.pool + mb.off[qb];        // nr x n, column-major
    const int ks = (nr + 3) >> 2;
    for (int s0 = 0; s0 < ks; s0 += 2) {
      double bv[2], av[2][4];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ccl = min(4 * (s0 + q) + lk, nr - 1);
        bv[q] = Bb[ccl + int64_t(jcl) * nr];
#pragma unroll
        for (int tile = 0; tile < 4; ++tile) av[q][tile] = Ab[min(16 * tile + li, m - 1) + int64_t(ccl) * mt];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int cc = 4 * (s0 + q) + lk;
        const double b = masked(cc < nr && jok, bv[q]);
#pragma unroll
        for (int tile = 0; tile < 4; ++tile)
          y[tile] = mfma4(masked(cc < nr && 16 * tile + li < m, av[q][tile]), b, y[tile]);
      }
    }
  }
  double* Cb = cpool + coff[t] + rb0;  // C block is mt x n, column-major
#pragma unroll
  for (int tile = 0; tile < 4; ++tile) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * tile + lk + 4 * v;
      if (tile < ntile && r < m && jok) Cb[r + int64_t(jc) * mt] = y[tile][v];
    }
  }
  }
}

void launch_near_direct(const int32_t* items, int64_t nitems, const int32_t* blocks, const int64_t* coff,
                        const int32_t* pptr, const int32_t* pairs, const TreeView& tv, const MatView& ma,
                        const MatView& mb, double* cpool, hipStream_t s) {
  const int64_t maxg = max_groups(256);
  for (int64_t b = 0; b < nitems; b += maxg) {
    const unsigned cnt = unsigned(std::min(maxg, nitems - b));
    hipLaunchKernelGGL(k_near_direct, dim3(cnt), dim3(256), 0, s, items + 2 * b, blocks, coff, pptr, pairs, tv, ma,
                       mb, cpool);
    HM_CHECK_HIP(hipGetLastError());
  }
}

__global__ void k_to_float(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = float(src[i]);
}

void launch_to_float(const double* src, float* dst, int64_t n, hipStream_t s) {
  const int64_t per = int64_t(256) * max_groups(256);
  for (int64_t b = 0; b < n; b += per) {
    const int64_t cnt = std::min(per, n - b);
    hipLaunchKernelGGL(k_to_float, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, s, src + b, dst + b, cnt);
    HM_CHECK_HIP(hipGetLastError());
  }
}

__global__ void k_scatter_terms(const int32_t* __restrict__ ids, const Term* __restrict__ src, Term* __restrict__ dst,
                                int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[ids[i]] = src[i];
}

void launch_scatter_terms(const int32_t* ids, const Term* src, Term* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter_terms, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, ids, src, dst, n);
  HM_CHECK_HIP(hipGetLastError());
}

}  // namespace hm
