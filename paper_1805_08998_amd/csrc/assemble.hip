// Assembly of kernel matrices as H-matrices on the device.
//
// Nearfield leaves are filled with kernel entries. Every farfield leaf is
// compressed to relative Frobenius tolerance eps_in by the randomized scheme of
// compress.h, whose operator products K[tau, sigma] X are evaluated on the fly
// from the points (the kernels are symmetric, so K^T X uses the same routine
// with rows and columns exchanged).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "compress.h"
#include "device_common.h"

namespace hm {

struct KernelDev {
  int32_t kind;
  double diag;  // diag + shift
};

__device__ __forceinline__ double kernel_eval(const KernelDev& k, double dx, double dy, double dz) {
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  if (k.kind == HMAT_KERNEL_LAPLACE_4PI) return 1.0 / (12.566370614359172 * r);
  if (k.kind == HMAT_KERNEL_INV_DIST) return 1.0 / r;
  return exp(-r);
}

// ---------------------------------------------------------------- nearfield fill
struct DenseJob {
  int64_t off;
  int32_t row0, m, col0, n;
};

__global__ void k_fill_dense(const DenseJob* __restrict__ jobs, const double* __restrict__ xyz,
                             KernelDev k, double* __restrict__ pool) {
  const DenseJob J = jobs[blockIdx.x];
  const int64_t total = int64_t(J.m) * J.n;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    int i = int(e % J.m), j = int(e / J.m);
    int pi = J.row0 + i, pj = J.col0 + j;
    double v;
    if (pi == pj) {
      v = k.diag;
    } else {
      v = kernel_eval(k, xyz[3 * pi] - xyz[3 * pj], xyz[3 * pi + 1] - xyz[3 * pj + 1],
                      xyz[3 * pi + 2] - xyz[3 * pj + 2]);
    }
    pool[J.off + e] = v;
  }
}

// ---------------------------------------------------------------- kernel apply
// Y[:, j'] (+)= K[rows, cols] X[:, j] for j < w, with output column j' = j for
// j < split and j + gap otherwise. One wave per 64-row chunk of a target.
struct KApplyItem {
  const double* X;  // n x w, ld ldx
  double* Y;        // m x *, ld ldy
  int32_t ldx, ldy;
  int32_t row0, m;  // output positions
  int32_t col0, n;  // input positions
  int32_t chunk;    // 64-row chunk index
  int32_t w, split, gap;
};

constexpr int KW = 24;  // max columns per kernel-apply pass

__global__ void __launch_bounds__(64) k_kernel_apply(const KApplyItem* __restrict__ items,
                                                     const double* __restrict__ xyz, KernelDev kd) {
  __shared__ double px[64], py[64], pz[64];
  __shared__ double xs[64 * KW];
  const KApplyItem it = items[blockIdx.x];
  const int lane = threadIdx.x;
  const int i = it.chunk * 64 + lane;
  const bool row_ok = i < it.m;
  const int pi = it.row0 + (row_ok ? i : 0);
  const double xi = xyz[3 * pi], yi = xyz[3 * pi + 1], zi = xyz[3 * pi + 2];
  double acc[KW];
#pragma unroll
  for (int j = 0; j < KW; ++j) acc[j] = 0.0;
  for (int c0 = 0; c0 < it.n; c0 += 64) {
    const int c = c0 + lane;
    __syncthreads();
    if (c < it.n) {
      const int pj = it.col0 + c;
      px[lane] = xyz[3 * pj];
      py[lane] = xyz[3 * pj + 1];
      pz[lane] = xyz[3 * pj + 2];
      for (int j = 0; j < it.w; ++j) xs[lane * KW + j] = it.X[int64_t(j) * it.ldx + c];
    }
    __syncthreads();
    const int cn = min(64, it.n - c0);
    for (int cc = 0; cc < cn; ++cc) {
      const int pj = it.col0 + c0 + cc;
      double kv = (pj == pi) ? kd.diag : kernel_eval(kd, xi - px[cc], yi - py[cc], zi - pz[cc]);
#pragma unroll
      for (int j = 0; j < KW; ++j)
        if (j < it.w) acc[j] += kv * xs[cc * KW + j];
    }
  }
  if (row_ok) {
#pragma unroll
    for (int j = 0; j < KW; ++j)
      if (j < it.w) {
        int jo = j < it.split ? j : j + it.gap;
        it.Y[int64_t(jo) * it.ldy + i] = acc[j];
      }
  }
}

// ---------------------------------------------------------------- driver
namespace {

struct Pass {
  std::vector<KApplyItem> items;
  void add(const double* X, int ldx, double* Y, int ldy, int row0, int m, int col0, int n, int w,
           int split, int gap) {
    for (int c = 0; c * 64 < m; ++c)
      items.push_back(KApplyItem{X, Y, ldx, ldy, row0, m, col0, n, c, w, split, gap});
  }
  void run(const double* xyz, KernelDev kd, hipStream_t s) {
    if (items.empty()) return;
    DevBuf<KApplyItem> d(items.size());
    d.upload(items, s);
    const size_t maxg = size_t(max_groups(64));
    for (size_t b = 0; b < items.size(); b += maxg) {
      unsigned cnt = unsigned(std::min(maxg, items.size() - b));
      hipLaunchKernelGGL(k_kernel_apply, dim3(cnt), dim3(64), 0, s, d.p + b, xyz, kd);
      HM_CHECK_HIP(hipGetLastError());
    }
    HM_CHECK_HIP(hipStreamSynchronize(s));
  }
};

}  // namespace

HMat* assemble_kernel(Tree* t, const hmat_kernel* k, double eps_in, const Opts& opts,
                      int64_t* n_not_converged) {
  HM_REQUIRE(k != nullptr, HMAT_ERR_ARG, "kernel is NULL");
  HM_REQUIRE(k->kind >= 0 && k->kind <= 2, HMAT_ERR_ARG, "unknown kernel kind");
  HM_REQUIRE(eps_in > 0.0 && eps_in < 1.0, HMAT_ERR_ARG, "eps_in must be in (0, 1)");
  HM_REQUIRE(std::isfinite(k->diag) && std::isfinite(k->shift), HMAT_ERR_ARG, "non-finite diagonal");
  hipStream_t s = opts.stream();
  set_current_stream(s);
  t->ensure_device(s);
  KernelDev kd{k->kind, k->diag + k->shift};
  const double* xyz = t->dev->xyz_perm.p;

  HMat* M = new HMat();
  M->tree = t;
  tree_retain(t);
  const int64_t nb = int64_t(t->b_tau.size());
  M->rank.assign(nb, 0);
  M->off.assign(nb, -1);

  // nearfield leaves first in the pool
  int64_t pos = 0;
  std::vector<DenseJob> dense;
  std::vector<int32_t> far;
  for (int32_t b : t->leaves) {
    int32_t ta = t->b_tau[b], sg = t->b_sigma[b];
    if (t->b_kind[b] == KIND_N) {
      M->off[b] = pos;
      dense.push_back(DenseJob{pos, t->c_begin[ta], t->c_size[ta], t->c_begin[sg], t->c_size[sg]});
      pos += int64_t(t->c_size[ta]) * t->c_size[sg];
    } else {
      far.push_back(b);
    }
  }
  const int64_t dense_len = pos;

  // farfield compression in chunks bounded by a workspace budget
  const int b0 = 16, g = 8, cap = 48;
  CParams cp{cap, g, eps_in, opts.o.delta, 9.0};
  const int max_rounds = (cap - b0) / g;
  struct ChunkOut {
    DevBuf<double> buf;
    std::vector<int32_t> blocks;
    std::vector<int32_t> ranks;
    std::vector<int64_t> offs;  // inside buf
  };
  std::vector<ChunkOut> outs;
  DevBuf<double> omega(size_t(t->n) * size_t(b0 + g * (max_rounds + 1)));
  const int ncol_omega = b0 + g * (max_rounds + 1);
  launch_fill_gaussian(omega.p, t->n, ncol_omega, opts.o.seed ^ 0xA55E3B1Eull, s);

  const int64_t budget = opts.o.workspace_limit > 0 ? opts.o.workspace_limit : (int64_t(2) << 30);
  size_t fi = 0;
  int64_t not_conv = 0;
  while (fi < far.size()) {
    // chunk of targets
    std::vector<int32_t> blocks;
    int64_t need = 0;
    while (fi < far.size()) {
      int32_t b = far[fi];
      int64_t m = t->c_size[t->b_tau[b]], n = t->c_size[t->b_sigma[b]];
      int64_t bytes = 8 * (m * (cap + g) + n * cap + 2 * cap * cap + cap);
      if (!blocks.empty() && need + bytes > budget) break;
      need += bytes;
      blocks.push_back(b);
      ++fi;
    }
    const int nt = int(blocks.size());
    DevBuf<double> ws(size_t(need / 8));
    std::vector<CTarget> h(nt);
    int64_t o = 0;
    for (int i = 0; i < nt; ++i) {
      int32_t b = blocks[i];
      CTarget& T = h[i];
      std::memset(&T, 0, sizeof(T));
      T.m = t->c_size[t->b_tau[b]];
      T.n = t->c_size[t->b_sigma[b]];
      T.row0 = t->c_begin[t->b_tau[b]];
      T.col0 = t->c_begin[t->b_sigma[b]];
      T.Y = ws.p + o;
      o += int64_t(T.m) * (cap + g);
      T.Z = ws.p + o;
      o += int64_t(T.n) * cap;
      T.core = ws.p + o;
      o += 2 * cap * cap + cap;
      T.active = 1;
      T.block = b;
      T.w0 = b0;
    }
    DevBuf<CTarget> dt(nt);
    dt.upload(h, s);
    // sketch + probe in one pass
    {
      Pass p;
      for (auto& T : h)
        p.add(omega.p + T.col0, int(t->n), T.Y, T.m, T.row0, T.m, T.col0, T.n, b0 + g, b0, cap - b0);
      p.run(xyz, kd, s);
    }
    launch_orth_append(dt.p, nt, 0, b0, cp, s);
    launch_probe_residual(dt.p, nt, cp, s);
    HM_CHECK_HIP(hipMemcpyAsync(h.data(), dt.p, sizeof(CTarget) * nt, hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    // projection Z = K^T Q (K symmetric: K[sigma, tau] Q)
    {
      Pass p;
      for (auto& T : h)
        if (T.r > 0) p.add(T.Y, T.m, T.Z, T.n, T.col0, T.n, T.row0, T.m, T.r, T.r, 0);
      p.run(xyz, kd, s);
    }
    for (auto& T : h) T.rz = T.r;
    dt.upload(h, s);
    DevBuf<int32_t> pending(nt);
    std::vector<int32_t> hp(nt);
    for (int round = 0; round < max_rounds; ++round) {
      launch_check(dt.p, nt, cp, pending.p, s);
      HM_CHECK_HIP(hipMemcpyAsync(hp.data(), pending.p, 4 * nt, hipMemcpyDeviceToHost, s));
      HM_CHECK_HIP(hipMemcpyAsync(h.data(), dt.p, sizeof(CTarget) * nt, hipMemcpyDeviceToHost, s));
      HM_CHECK_HIP(hipStreamSynchronize(s));
      int cnt = 0;
      for (int i = 0; i < nt; ++i) {
        h[i].active = hp[i];
        cnt += hp[i];
      }
      if (!cnt) break;
      dt.upload(h, s);
      std::vector<int32_t> r_old(nt);
      for (int i = 0; i < nt; ++i) r_old[i] = h[i].r;
      launch_orth_append(dt.p, nt, cap, g, cp, s);
      HM_CHECK_HIP(hipMemcpyAsync(h.data(), dt.p, sizeof(CTarget) * nt, hipMemcpyDeviceToHost, s));
      HM_CHECK_HIP(hipStreamSynchronize(s));
      const int col = b0 + g * (round + 1);
      Pass probe, proj;
      for (int i = 0; i < nt; ++i) {
        CTarget& T = h[i];
        if (!T.active) continue;
        T.rounds++;
        probe.add(omega.p + int64_t(col) * t->n + T.col0, int(t->n), T.Y + int64_t(cap) * T.m, T.m,
                  T.row0, T.m, T.col0, T.n, g, g, 0);
        int nw = T.r - r_old[i];
        if (nw > 0)
          proj.add(T.Y + int64_t(r_old[i]) * T.m, T.m, T.Z + int64_t(r_old[i]) * T.n, T.n, T.col0, T.n,
                   T.row0, T.m, nw, nw, 0);
        T.rz = T.r;
      }
      probe.run(xyz, kd, s);
      proj.run(xyz, kd, s);
      dt.upload(h, s);
      launch_probe_residual(dt.p, nt, cp, s);
    }
    launch_check(dt.p, nt, cp, pending.p, s);
    for (int i = 0; i < nt; ++i) h[i].active = 1;
    launch_core(dt.p, nt, cp, s);
    HM_CHECK_HIP(hipMemcpyAsync(h.data(), dt.p, sizeof(CTarget) * nt, hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    ChunkOut co;
    int64_t olen = 0;
    for (int i = 0; i < nt; ++i) {
      CTarget& T = h[i];
      if (!T.done) ++not_conv;
      co.blocks.push_back(T.block);
      co.ranks.push_back(T.k);
      co.offs.push_back(olen);
      T.out_off = olen;
      olen += int64_t(T.k) * (T.m + T.n);
    }
    co.buf.alloc(size_t(std::max<int64_t>(olen, 1)));
    dt.upload(h, s);
    launch_write_factors(dt.p, nt, cp, co.buf.p, s);
    HM_CHECK_HIP(hipStreamSynchronize(s));
    outs.push_back(std::move(co));
  }

  // final pool: nearfield blocks then the farfield chunks, each chunk at its own base
  int64_t total = dense_len;
  std::vector<int64_t> chunk_base, chunk_len;
  for (auto& co : outs) {
    int64_t len = 0;
    for (size_t i = 0; i < co.blocks.size(); ++i) {
      int32_t b = co.blocks[i];
      M->rank[b] = co.ranks[i];
      M->off[b] = total + co.offs[i];
      len += int64_t(co.ranks[i]) * (t->c_size[t->b_tau[b]] + t->c_size[t->b_sigma[b]]);
    }
    chunk_base.push_back(total);
    chunk_len.push_back(len);
    total += len;
  }
  M->pool_len = total;
  M->pool.alloc(size_t(std::max<int64_t>(total, 1)));
  if (!dense.empty()) {
    DevBuf<DenseJob> dj(dense.size());
    dj.upload(dense, s);
    hipLaunchKernelGGL(k_fill_dense, dim3(unsigned(dense.size())), dim3(256), 0, s, dj.p, xyz, kd,
                       M->pool.p);
    HM_CHECK_HIP(hipGetLastError());
    HM_CHECK_HIP(hipStreamSynchronize(s));
  }
  for (size_t c = 0; c < outs.size(); ++c)
    if (chunk_len[c])
      HM_CHECK_HIP(hipMemcpyAsync(M->pool.p + chunk_base[c], outs[c].buf.p, 8 * chunk_len[c],
                                  hipMemcpyDeviceToDevice, s));
  M->upload_meta(s);
  HM_CHECK_HIP(hipStreamSynchronize(s));
  if (n_not_converged) *n_not_converged = not_conv;
  return M;
}

}  // namespace hm
