// Cluster tree and block-cluster tree on the host (Section 2 of the paper:
// Def. 2.2 cluster tree, Def. 2.3 admissibility, Algorithm 1).
//
// Compiled with -ffp-contract=off: the admissibility test must take the same
// decisions as any other IEEE float64 evaluation of the same formulas, so no
// multiply-add may be fused.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "hmat_internal.h"

namespace hm {

static double norm3(double a, double b, double c) { return std::sqrt(a * a + b * b + c * c); }

double cluster_dist(const Tree& t, int32_t a, int32_t b) {
  double g[3];
  for (int k = 0; k < 3; ++k) {
    double u = t.c_bmin[3 * b + k] - t.c_bmax[3 * a + k];
    double w = t.c_bmin[3 * a + k] - t.c_bmax[3 * b + k];
    double m = 0.0;
    if (u > m) m = u;
    if (w > m) m = w;
    g[k] = m;
  }
  return norm3(g[0], g[1], g[2]);
}

bool admissible(const Tree& t, int32_t a, int32_t b) {
  double d = cluster_dist(t, a, b);
  if (!(d > 0.0)) return false;
  double da = t.c_diam[a], db = t.c_diam[b];
  double m = da > db ? da : db;
  return m <= t.eta * d;
}

int32_t Tree::find_block(int32_t tau, int32_t sigma) const {
  auto b = row_all_blk.begin() + row_all_ptr[tau];
  auto e = row_all_blk.begin() + row_all_ptr[tau + 1];
  auto it = std::lower_bound(b, e, sigma, [&](int32_t blk, int32_t s) { return b_sigma[blk] < s; });
  if (it != e && b_sigma[*it] == sigma) return *it;
  return -1;
}

Tree* build_tree(const double* xyz, int64_t n, int32_t leaf, double eta, int32_t split) {
  HM_REQUIRE(xyz != nullptr, HMAT_ERR_ARG, "xyz is NULL");
  HM_REQUIRE(n >= 1 && n < (int64_t(1) << 31), HMAT_ERR_ARG, "n must be in [1, 2^31)");
  HM_REQUIRE(leaf >= 1, HMAT_ERR_ARG, "leaf_size must be >= 1");
  HM_REQUIRE(std::isfinite(eta) && eta > 0.0, HMAT_ERR_ARG, "eta must be finite and > 0");
  HM_REQUIRE(split == HMAT_SPLIT_MIDPOINT || split == HMAT_SPLIT_MEDIAN, HMAT_ERR_ARG,
             "unknown split rule");
  for (int64_t i = 0; i < 3 * n; ++i)
    HM_REQUIRE(std::isfinite(xyz[i]), HMAT_ERR_ARG, "non-finite coordinate");

  Tree* t = new Tree();
  t->n = n;
  t->leaf_size = leaf;
  t->eta = eta;
  t->split = split;
  t->xyz.assign(xyz, xyz + 3 * n);
  t->perm.resize(n);
  std::iota(t->perm.begin(), t->perm.end(), 0);

  auto add_cluster = [&](int32_t b, int32_t s, int32_t lev, int32_t par) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = b; i < b + s; ++i) {
      const double* p = &t->xyz[3 * int64_t(t->perm[i])];
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], p[k]);
        hi[k] = std::max(hi[k], p[k]);
      }
    }
    t->c_begin.push_back(b);
    t->c_size.push_back(s);
    t->c_level.push_back(lev);
    t->c_parent.push_back(par);
    t->c_child0.push_back(-1);
    t->c_nchild.push_back(0);
    for (int k = 0; k < 3; ++k) {
      t->c_bmin.push_back(lo[k]);
      t->c_bmax.push_back(hi[k]);
    }
    t->c_diam.push_back(norm3(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]));
    return int32_t(t->c_begin.size() - 1);
  };

  add_cluster(0, int32_t(n), 0, -1);
  std::vector<int32_t> tmp;
  for (size_t head = 0; head < t->c_begin.size(); ++head) {
    int32_t c = int32_t(head);
    int32_t s = t->c_size[c];
    if (s <= leaf) continue;
    double ext[3];
    for (int k = 0; k < 3; ++k) ext[k] = t->c_bmax[3 * c + k] - t->c_bmin[3 * c + k];
    int axis = 0;
    for (int k = 1; k < 3; ++k)
      if (ext[k] > ext[axis]) axis = k;
    if (!(ext[axis] > 0.0)) continue;
    int32_t b = t->c_begin[c];
    int32_t* idx = t->perm.data() + b;
    int32_t n1;
    if (split == HMAT_SPLIT_MIDPOINT) {
      double mid = 0.5 * (t->c_bmin[3 * c + axis] + t->c_bmax[3 * c + axis]);
      tmp.clear();
      for (int32_t i = 0; i < s; ++i)
        if (t->xyz[3 * int64_t(idx[i]) + axis] <= mid) tmp.push_back(idx[i]);
      n1 = int32_t(tmp.size());
      if (n1 == 0 || n1 == s) continue;
      for (int32_t i = 0; i < s; ++i)
        if (!(t->xyz[3 * int64_t(idx[i]) + axis] <= mid)) tmp.push_back(idx[i]);
      std::copy(tmp.begin(), tmp.end(), idx);
    } else {
      std::stable_sort(idx, idx + s, [&](int32_t p, int32_t q) {
        return t->xyz[3 * int64_t(p) + axis] < t->xyz[3 * int64_t(q) + axis];
      });
      n1 = s / 2;
    }
    int32_t lev = t->c_level[c] + 1;
    int32_t c1 = add_cluster(b, n1, lev, c);
    add_cluster(b + n1, s - n1, lev, c);
    t->c_child0[c] = c1;
    t->c_nchild[c] = 2;
  }
  const int32_t nc = int32_t(t->c_begin.size());

  // leaf clusters by position and the range of them inside every cluster
  for (int32_t c = 0; c < nc; ++c)
    if (t->c_nchild[c] == 0) t->leaf_clusters.push_back(c);
  std::sort(t->leaf_clusters.begin(), t->leaf_clusters.end(),
            [&](int32_t a, int32_t b) { return t->c_begin[a] < t->c_begin[b]; });
  t->c_lc_begin.resize(nc);
  t->c_lc_end.resize(nc);
  for (int32_t c = 0; c < nc; ++c) {
    auto lo = std::lower_bound(t->leaf_clusters.begin(), t->leaf_clusters.end(), t->c_begin[c],
                               [&](int32_t lc, int32_t pos) { return t->c_begin[lc] < pos; });
    auto hi = std::lower_bound(t->leaf_clusters.begin(), t->leaf_clusters.end(),
                               t->c_begin[c] + t->c_size[c],
                               [&](int32_t lc, int32_t pos) { return t->c_begin[lc] < pos; });
    t->c_lc_begin[c] = int32_t(lo - t->leaf_clusters.begin());
    t->c_lc_end[c] = int32_t(hi - t->leaf_clusters.begin());
  }

  // Algorithm 1, breadth first
  auto add_block = [&](int32_t tau, int32_t sigma, int32_t lev, int32_t par) {
    t->b_tau.push_back(tau);
    t->b_sigma.push_back(sigma);
    t->b_level.push_back(lev);
    t->b_kind.push_back(KIND_INNER);
    t->b_child0.push_back(-1);
    t->b_nchild.push_back(0);
    t->b_parent.push_back(par);
  };
  add_block(0, 0, 0, -1);
  for (size_t head = 0; head < t->b_tau.size(); ++head) {
    int32_t b = int32_t(head);
    int32_t tau = t->b_tau[b], sigma = t->b_sigma[b];
    if (admissible(*t, tau, sigma)) {
      t->b_kind[b] = KIND_F;
    } else if (t->c_nchild[tau] && t->c_nchild[sigma]) {
      t->b_kind[b] = KIND_INNER;
      int32_t first = int32_t(t->b_tau.size());
      int32_t cnt = 0;
      for (int32_t i = 0; i < t->c_nchild[tau]; ++i)
        for (int32_t j = 0; j < t->c_nchild[sigma]; ++j) {
          add_block(t->c_child0[tau] + i, t->c_child0[sigma] + j, t->b_level[b] + 1, b);
          ++cnt;
        }
      t->b_child0[b] = first;
      t->b_nchild[b] = cnt;
    } else {
      t->b_kind[b] = KIND_N;
    }
  }
  const int64_t nb = int64_t(t->b_tau.size());
  HM_REQUIRE(nb < (int64_t(1) << 31), HMAT_ERR_ARG, "too many blocks");
  t->leaf_index.assign(nb, -1);
  for (int64_t b = 0; b < nb; ++b)
    if (t->b_kind[b] != KIND_INNER) {
      t->leaf_index[b] = int32_t(t->leaves.size());
      t->leaves.push_back(int32_t(b));
    }
  t->depth = 0;
  for (int64_t b = 0; b < nb; ++b) t->depth = std::max(t->depth, t->b_level[b]);
  t->level_begin.assign(t->depth + 2, nb);
  for (int64_t b = nb - 1; b >= 0; --b) t->level_begin[t->b_level[b]] = b;
  for (int l = t->depth; l >= 0; --l)
    t->level_begin[l] = std::min(t->level_begin[l], t->level_begin[l + 1]);

  // sparsity constant and block-row / block-column lists
  std::vector<int32_t> crow(nc, 0), ccol(nc, 0);
  for (int64_t b = 0; b < nb; ++b) {
    crow[t->b_tau[b]]++;
    ccol[t->b_sigma[b]]++;
  }
  t->csp = 0;
  for (int32_t c = 0; c < nc; ++c) t->csp = std::max(t->csp, std::max(crow[c], ccol[c]));

  auto build_csr = [&](bool rows, bool leaves_only, std::vector<int32_t>& ptr,
                       std::vector<int32_t>& blk) {
    ptr.assign(nc + 1, 0);
    for (int64_t b = 0; b < nb; ++b) {
      if (leaves_only && t->b_kind[b] == KIND_INNER) continue;
      ptr[(rows ? t->b_tau[b] : t->b_sigma[b]) + 1]++;
    }
    for (int32_t c = 0; c < nc; ++c) ptr[c + 1] += ptr[c];
    blk.assign(ptr[nc], 0);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t b = 0; b < nb; ++b) {
      if (leaves_only && t->b_kind[b] == KIND_INNER) continue;
      blk[fill[rows ? t->b_tau[b] : t->b_sigma[b]]++] = int32_t(b);
    }
    for (int32_t c = 0; c < nc; ++c) {
      auto key = [&](int32_t x) { return rows ? t->c_begin[t->b_sigma[x]] : t->c_begin[t->b_tau[x]]; };
      std::sort(blk.begin() + ptr[c], blk.begin() + ptr[c + 1],
                [&](int32_t x, int32_t y) { return key(x) < key(y); });
    }
  };
  build_csr(true, true, t->brow_ptr, t->brow_blk);
  build_csr(false, true, t->bcol_ptr, t->bcol_blk);
  build_csr(true, false, t->row_all_ptr, t->row_all_blk);
  for (int32_t c = 0; c < nc; ++c)
    std::sort(t->row_all_blk.begin() + t->row_all_ptr[c], t->row_all_blk.begin() + t->row_all_ptr[c + 1],
              [&](int32_t x, int32_t y) { return t->b_sigma[x] < t->b_sigma[y]; });
  return t;
}

void Tree::ensure_device(hipStream_t s) {
  std::lock_guard<std::mutex> lk(dev_mu);
  int d = 0;
  HM_CHECK_HIP(hipGetDevice(&d));
  if (dev && dev_id == d) return;
  delete dev;
  dev = new DeviceTree();
  dev_id = d;
  dev->c_begin.upload(c_begin, s);
  dev->c_size.upload(c_size, s);
  dev->c_parent.upload(c_parent, s);
  dev->c_level.upload(c_level, s);
  dev->c_lc_begin.upload(c_lc_begin, s);
  dev->c_lc_end.upload(c_lc_end, s);
  dev->leaf_clusters.upload(leaf_clusters, s);
  dev->b_tau.upload(b_tau, s);
  dev->b_sigma.upload(b_sigma, s);
  dev->b_kind.upload(b_kind, s);
  dev->brow_ptr.upload(brow_ptr, s);
  dev->brow_blk.upload(brow_blk, s);
  dev->bcol_ptr.upload(bcol_ptr, s);
  dev->bcol_blk.upload(bcol_blk, s);
  dev->perm.upload(perm, s);
  std::vector<double> xp(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) xp[3 * i + k] = xyz[3 * int64_t(perm[i]) + k];
  dev->xyz_perm.upload(xp, s);
  HM_CHECK_HIP(hipStreamSynchronize(s));
}

Tree::~Tree() { delete dev; }

void tree_release(Tree* t) {
  if (t && t->refs.fetch_sub(1) == 1) delete t;
}

}  // namespace hm
