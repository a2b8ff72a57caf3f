// Host driver of the product C = A B (Algorithms 3 and 4 of the paper, breadth
// first, with the blocked randomized compression of Section 4).
//
// 1. Symbolic restriction over the whole block tree (Algorithm 3): for every
//    block the low-rank terms created at it and its list of pairs
//    (A[tau, rho], B[rho, sigma]). Terms of ancestors are inherited by index
//    shift and never copied.
// 2. Creation of the low-rank terms in subtree batches (memory bound):
//    FF: core R_A^T L_B; FH: B[rho', sigma']^T R_A; HF: A[tau', rho'] L_B; a pair
//    whose middle cluster is a leaf keeps both dense factors as a term.
// 3. Targets in chunks: farfield leaves are compressed (sketch + probe, CGS2,
//    projection, growth, core SVD, truncation); nearfield leaves are evaluated
//    by applying their sum-expression to the identity.
#include <algorithm>
#include <cmath>
#include <limits>
#include <cstring>
#include <deque>
#include <future>
#include <map>
#include <unordered_map>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

#include "compress.h"
#include "product_kernels.h"
#include "schemes.h"

namespace hm {

void launch_leaf_reduce(const int32_t* owner, int64_t nitems, const Task* tasks, const TDesc* td, const TreeView& tv,
                        const MatView& ma, const MatView& mb, double* ws, hipStream_t s, bool lowp);
void launch_subtree_expand(const int32_t* owner, int64_t nitems, const Task* tasks, const TDesc* td,
                           const TreeView& tv, const MatView& ma, const MatView& mb, const double* ws,
                           hipStream_t s, bool lowp);
void launch_fill_owner(const int64_t* pre, int ntask, int32_t* owner, hipStream_t s);
void launch_term_reduce(const TermItem* items, size_t n, const TDesc* td, const TInfo* ti, const TreeView& tv,
                        double* vbuf, hipStream_t s, bool lowp);
void launch_gather_mfma(const RowItem* items, size_t n, const TDesc* td, const TInfo* ti, const HPair* hp,
                        const TreeView& tv, const double* vbuf, hipStream_t s, bool lowp);
void launch_fused_terms(const int32_t* tlist, size_t n, const TDesc* td, const TInfo* ti, const HPair* hp,
                        const TreeView& tv, hipStream_t s, bool lowp);
void launch_scatter_terms(const int32_t* ids, const Term* src, Term* dst, int64_t n, hipStream_t s);
void launch_fused_terms4(const int32_t* tlist, size_t n, const TDesc* td, const TInfo* ti, const HPair* hp,
                         const TreeView& tv, hipStream_t s, bool lowp);
void launch_to_float(const double* src, float* dst, int64_t n, hipStream_t s);
void launch_near_direct(const int32_t* items, int64_t nitems, const int32_t* blocks, const int64_t* coff,
                        const int32_t* pptr, const int32_t* pairs, const TreeView& tv, const MatView& ma,
                        const MatView& mb, double* cpool, hipStream_t s);

namespace {

enum { T_FF = 0, T_FH = 1, T_HF = 2, T_GAP = 3 };

struct SymTerm {
  int32_t type;
  int32_t child;  // block the term belongs to
  int32_t a_blk, b_blk;
  int32_t kl, kr;
  int32_t batch;
  int64_t data_off;  // offset of created data in the batch's pool (-1 none)
};

// Depth-first order of the leaves, the leaf range of every block, and per matrix
// prefix sums of farfield ranks over that order.
struct DfsInfo {
  std::vector<int32_t> dfs_of_block;  // leaf block -> dfs index (else -1)
  std::vector<int32_t> lo, hi;        // per block
  std::vector<int32_t> dfs_block;     // dfs index -> block
};

DfsInfo dfs_order(const Tree& t) {
  const int64_t nb = int64_t(t.b_tau.size());
  DfsInfo d;
  d.dfs_of_block.assign(nb, -1);
  d.lo.assign(nb, 0);
  d.hi.assign(nb, 0);
  std::vector<std::pair<int32_t, int>> st;  // (block, state)
  st.push_back({0, 0});
  while (!st.empty()) {
    auto [b, s] = st.back();
    st.pop_back();
    if (s == 0) {
      d.lo[b] = int32_t(d.dfs_block.size());
      if (t.b_nchild[b] == 0) {
        d.dfs_of_block[b] = int32_t(d.dfs_block.size());
        d.dfs_block.push_back(b);
        d.hi[b] = int32_t(d.dfs_block.size());
      } else {
        st.push_back({b, 1});
        for (int i = t.b_nchild[b] - 1; i >= 0; --i) st.push_back({t.b_child0[b] + i, 0});
      }
    } else {
      d.hi[b] = int32_t(d.dfs_block.size());
    }
  }
  return d;
}

struct DevMat {
  DevBuf<int64_t> kpref;
  std::vector<int64_t> hkpref;
  DevBuf<LeafRec> row_rec, col_rec;
  DevBuf<DfsRec> dfs_rec;
  MatView view(const HMat* M) const {
    return MatView{M->pool.p, M->d_rank.p, M->d_off.p, kpref.p, M->pool32.p, row_rec.p, col_rec.p, dfs_rec.p};
  }
};

// Packed leaf records of M for the subtree kernels (block-row and block-column lists,
// depth-first order).
void build_leaf_recs(const HMat* M, const DfsInfo& d, DevMat& dm, hipStream_t s) {
  const Tree& t = *M->tree;
  auto rec = [&](int32_t b, bool row) {
    LeafRec r{};
    const int32_t oth = row ? t.b_sigma[b] : t.b_tau[b];
    r.off = M->off[b];
    r.o0 = t.c_begin[oth];
    r.on = t.c_size[oth];
    r.k = t.b_kind[b] == KIND_F ? M->rank[b] : -1;
    r.m = t.c_size[t.b_tau[b]];
    r.n = t.c_size[t.b_sigma[b]];
    r.kp = int32_t(dm.hkpref[d.dfs_of_block[b]]);
    return r;
  };
  HM_REQUIRE(dm.hkpref.back() < int64_t(INT32_MAX), HMAT_ERR_ARG, "too many farfield ranks for 32-bit offsets");
  std::vector<LeafRec> rr(t.brow_blk.size()), cr(t.bcol_blk.size());
  for (size_t p = 0; p < rr.size(); ++p) rr[p] = rec(t.brow_blk[p], true);
  for (size_t p = 0; p < cr.size(); ++p) cr[p] = rec(t.bcol_blk[p], false);
  std::vector<DfsRec> dr(d.dfs_block.size());
  for (size_t i = 0; i < dr.size(); ++i) {
    const int32_t b = d.dfs_block[i];
    DfsRec& x = dr[i];
    x.off = M->off[b];
    x.r0 = t.c_begin[t.b_tau[b]];
    x.c0 = t.c_begin[t.b_sigma[b]];
    x.m = t.c_size[t.b_tau[b]];
    x.n = t.c_size[t.b_sigma[b]];
    x.k = t.b_kind[b] == KIND_F ? M->rank[b] : -1;
    x.pad = 0;
  }
  dm.row_rec.upload(rr, s);
  dm.col_rec.upload(cr, s);
  dm.dfs_rec.upload(dr, s);
}

void build_kpref(const HMat* M, const DfsInfo& d, DevMat& dm, hipStream_t s) {
  dm.hkpref.assign(d.dfs_block.size() + 1, 0);
  const Tree& t = *M->tree;
  for (size_t i = 0; i < d.dfs_block.size(); ++i) {
    int32_t b = d.dfs_block[i];
    dm.hkpref[i + 1] = dm.hkpref[i] + (t.b_kind[b] == KIND_F ? M->rank[b] : 0);
  }
  dm.kpref.upload(dm.hkpref, s);
}

// Algorithmic work of one kernel family for one target in one pass direction:
// bytes = a + b * w, flops = f * w for a pass of width w.
struct Coef {
  double a = 0, b = 0, f = 0;
};
enum { K_TERM = 0, K_LEAF = 1, K_EXPAND = 2, K_GATHER = 3, K_COMPRESS = 4, K_FUSED = 5, K_FUSED4 = 6, K_NEAR = 7 };
// nearfield targets whose clusters both have at most FUSED_MAX (one wave) or FUSED4_MAX
// (four waves) rows use the fused MFMA kernels for their pairs
constexpr int FUSED_MAX = 64;
constexpr int FUSED4_MAX = 256;

// Per matrix, prefix sums over the depth-first leaf order of the quantities the
// subtree kernels stream (forward f / transposed t).
struct SubSums {
  std::vector<double> in_f, in_t, rin_f, rin_t, klr, out_f, out_t, vin_f, vin_t;
};

// HIP-event timing of kernel launches on the product's stream.
struct KernTimer {
  bool on = false;
  hipStream_t s = 0;
  // events are created once and reused by later products (creation is costly)
  static std::vector<hipEvent_t>& pool() {
    static std::vector<hipEvent_t> p;
    return p;
  }
  static std::mutex& pool_mu() {
    static std::mutex m;
    return m;
  }
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  hipEvent_t get() {
    {
      std::lock_guard<std::mutex> lk(pool_mu());
      if (!pool().empty()) {
        hipEvent_t e = pool().back();
        pool().pop_back();
        return e;
      }
    }
    hipEvent_t e;
    HM_CHECK_HIP(hipEventCreate(&e));
    return e;
  }
  void begin(int kind) {
    if (!on) return;
    hipEvent_t a = get(), b = get();
    HM_CHECK_HIP(hipEventRecord(a, s));
    ev.push_back({kind, {a, b}});
  }
  void end() {
    if (!on) return;
    HM_CHECK_HIP(hipEventRecord(ev.back().second.second, s));
  }
  void resolve(hmat_stats& st) {
    if (!on) return;
    HM_CHECK_HIP(hipStreamSynchronize(s));
    std::lock_guard<std::mutex> lk(pool_mu());
    for (auto& e : ev) {
      float ms = 0.f;
      HM_CHECK_HIP(hipEventElapsedTime(&ms, e.second.first, e.second.second));
      st.kern_time[e.first] += 1e-3 * ms;
      st.kern_launches[e.first] += 1;
      pool().push_back(e.second.first);
      pool().push_back(e.second.second);
    }
    ev.clear();
  }
};

struct Ctx {
  const Tree* t;
  const HMat* A;
  const HMat* B;
  hipStream_t s;
  DfsInfo dfs;
  DevMat da, db;
  MatView ma, mb;
  TreeView tv;
  DevBuf<int32_t> b_parent, b_dfs, group_ptr;
  DevBuf<Term> terms;
  std::vector<SymTerm> sym;
  std::vector<int32_t> group_ptr_h;
  std::vector<int32_t> hptr, hrho;  // pairs per block: hptr over blocks, hrho = (rho, A block, B block) triples
  std::vector<Term> hterms;
  hmat_stats st{};
  double eps;
  Opts opts;
  DevBuf<double> omega;  // Gaussian columns shared by all targets, rows keyed by position
  int64_t omega_cols = 0;
  KernTimer timer;
  SubSums sa, sb;
  double alg_flops = 0, alg_bytes = 0;  // minimum algorithmic work (final ranks as widths)
  std::vector<double> bflops;           // per block: the part of alg_flops charged to it as a target
  void charge(int32_t b, double by, double fl) {
    alg_bytes += by;
    alg_flops += fl;
    bflops[b] += fl;
  }
  // mixed precision: the forward sketch passes read float copies of every panel pool
  bool lowp = false;
  struct PoolPair {
    const double* b64;
    int64_t len;
    const float* b32;
  };
  std::vector<PoolPair> pools;  // double pool -> its float copy
  std::vector<Term32> hterms32;
  DevBuf<Term32> terms32;
  DevBuf<float> gpool32, bpool32;  // float copies of the created-term pools
  void register_pool(const double* b64, int64_t len, const float* b32) {
    for (auto& q : pools)
      if (q.b64 == b64) {
        q.len = len;
        q.b32 = b32;
        return;
      }
    pools.push_back(PoolPair{b64, len, b32});
  }
  const float* to32(const double* p) const {
    if (!p) return nullptr;
    for (const auto& q : pools)
      if (p >= q.b64 && p <= q.b64 + q.len) return q.b32 + (p - q.b64);
    throw Error(HMAT_ERR_INTERNAL, "term panel outside the registered pools");
  }

  ~Ctx();
  int32_t m_of(int32_t b) const { return t->c_size[t->b_tau[b]]; }
  int32_t n_of(int32_t b) const { return t->c_size[t->b_sigma[b]]; }
  int32_t rank_a(int32_t b) const { return A->rank[b]; }
  int32_t rank_b(int32_t b) const { return B->rank[b]; }
};

// ------------------------------------------------------------------ symbolic restriction
// Capacity of the large plan arrays is kept per host thread between products: they
// reach hundreds of megabytes, and fresh allocations would be page-faulted in again
// by every product. Only the capacity is reused; every product rebuilds the contents.
struct PlanArena {
  std::vector<SymTerm> sym;
  std::vector<int32_t> hrho;
  std::vector<Term> hterms;
  std::vector<std::vector<SymTerm>> part_sym;
  std::vector<std::vector<int32_t>> part_nxt, part_leaf;
};
PlanArena& plan_arena() {
  static thread_local PlanArena a;
  return a;
}
constexpr size_t kArenaKeepBytes = size_t(4) << 30;  // larger arrays are released after use

Ctx::~Ctx() {
  PlanArena& a = plan_arena();
  if (sym.capacity() * sizeof(SymTerm) <= kArenaKeepBytes) {
    sym.clear();
    a.sym.swap(sym);
  }
  if (hrho.capacity() * sizeof(int32_t) <= kArenaKeepBytes) {
    hrho.clear();
    a.hrho.swap(hrho);
  }
  if (hterms.capacity() * sizeof(Term) <= kArenaKeepBytes) {
    hterms.clear();
    a.hterms.swap(hterms);
  }
}

void symbolic(Ctx& c) {
  const Tree& t = *c.t;
  const int64_t nb = int64_t(t.b_tau.size());
  c.group_ptr_h.assign(nb + 1, 0);
  c.hptr.assign(nb + 1, 0);
  PlanArena& arena = plan_arena();
  c.sym.swap(arena.sym);
  c.hrho.swap(arena.hrho);
  c.sym.clear();
  c.hrho.clear();
  // Breadth-first: the sons of the blocks of one level are generated in block-id
  // order, so terms and pair lists are appended in block order and both CSR arrays
  // are filled directly. Pair lists of inner blocks live only for one level.
  // Pair entries are triples (rho, block tau x rho, block rho x sigma); the blocks of
  // a son pair follow from the parents' ids because sons of a block are stored
  // tau-son-major and contiguously: son (i, j) of block x is child0[x] + i * #sons(sigma_x) + j.
  // The blocks of a level are split into contiguous ranges handled by worker threads;
  // their outputs are concatenated in block order, so the result does not depend on
  // the number of threads.
  std::vector<int32_t> cur_ptr{0, 1}, cur_rho{0, 0, 0};  // level 0: the root, rho = I
  int64_t lev_first = 0;                                  // first block id of the current level
  if (t.b_kind[0] != KIND_INNER) {
    c.hrho.insert(c.hrho.end(), cur_rho.begin(), cur_rho.end());
    c.hptr[1] = 1;
  }
  struct Part {
    std::vector<SymTerm> sym;
    std::vector<int32_t> nxt_rho, leaf_rho;
    std::vector<int32_t> n_terms, n_nxt, n_leaf;  // per son, in son order
    int64_t first_child = -1;
    std::string err;
  };
  const unsigned hw = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  for (int lev = 0; lev < t.depth; ++lev) {
    const int64_t lb = t.level_begin[lev], le = t.level_begin[lev + 1];
    const int64_t nlev = le - lb;
    const int nparts = nlev >= 4096 ? int(hw) : 1;
    std::vector<Part> parts(nparts);
    if (arena.part_sym.size() < size_t(nparts)) {
      arena.part_sym.resize(nparts);
      arena.part_nxt.resize(nparts);
      arena.part_leaf.resize(nparts);
    }
    for (int pi = 0; pi < nparts; ++pi) {  // reuse capacity
      parts[pi].sym.swap(arena.part_sym[pi]);
      parts[pi].nxt_rho.swap(arena.part_nxt[pi]);
      parts[pi].leaf_rho.swap(arena.part_leaf[pi]);
      parts[pi].sym.clear();
      parts[pi].nxt_rho.clear();
      parts[pi].leaf_rho.clear();
    }
    auto work = [&](int pi) {
      Part& P = parts[pi];
      const int64_t b0 = lb + nlev * pi / nparts, b1 = lb + nlev * (pi + 1) / nparts;
      for (int64_t b = b0; b < b1; ++b) {
        if (t.b_kind[b] != KIND_INNER) continue;
        const int32_t* rb = cur_rho.data() + 3 * cur_ptr[b - lev_first];
        const int nr = cur_ptr[b - lev_first + 1] - cur_ptr[b - lev_first];
        const int ns = t.c_nchild[t.b_sigma[b]];
        for (int ci = 0; ci < t.b_nchild[b]; ++ci) {
          const int32_t ch = t.b_child0[b] + ci;
          if (P.first_child < 0) P.first_child = ch;
          const int it = ci / ns, is = ci % ns;  // son indices in tau_b and sigma_b
          const size_t s0 = P.sym.size(), h0 = P.nxt_rho.size();
          for (int q = 0; q < nr; ++q) {
            const int32_t rho = rb[3 * q], qa = rb[3 * q + 1], qb = rb[3 * q + 2];
            if (t.c_nchild[rho] == 0) {
              // middle cluster is a leaf: both factors are nearfield leaves of the parent level
              P.sym.push_back(SymTerm{T_GAP, ch, qa, qb, t.c_size[rho], t.c_size[rho], 0, -1});
              continue;
            }
            const int nrho = t.c_nchild[rho];
            for (int i = 0; i < nrho; ++i) {
              const int32_t r2 = t.c_child0[rho] + i;
              const int32_t b1x = t.b_child0[qa] + it * nrho + i;  // tau' x rho'
              const int32_t b2x = t.b_child0[qb] + i * ns + is;    // rho' x sigma'
              const bool f1 = t.b_kind[b1x] == KIND_F, f2 = t.b_kind[b2x] == KIND_F;
              if (f1 && f2) {
                if (c.rank_a(b1x) && c.rank_b(b2x))
                  P.sym.push_back(SymTerm{T_FF, ch, b1x, b2x, c.rank_a(b1x), c.rank_b(b2x), 0, -1});
              } else if (f1) {
                if (c.rank_a(b1x)) P.sym.push_back(SymTerm{T_FH, ch, b1x, b2x, c.rank_a(b1x), c.rank_a(b1x), 0, -1});
              } else if (f2) {
                if (c.rank_b(b2x)) P.sym.push_back(SymTerm{T_HF, ch, b1x, b2x, c.rank_b(b2x), c.rank_b(b2x), 0, -1});
              } else {
                P.nxt_rho.push_back(r2);
                P.nxt_rho.push_back(b1x);
                P.nxt_rho.push_back(b2x);
              }
            }
          }
          P.n_terms.push_back(int32_t(P.sym.size() - s0));
          const int cnt = int((P.nxt_rho.size() - h0) / 3);
          if (t.b_kind[ch] != KIND_INNER) {  // a leaf keeps its pairs; they leave the next level's list
            P.leaf_rho.insert(P.leaf_rho.end(), P.nxt_rho.begin() + h0, P.nxt_rho.end());
            P.nxt_rho.resize(h0);
            P.n_leaf.push_back(cnt);
            P.n_nxt.push_back(0);
          } else {
            P.n_leaf.push_back(0);
            P.n_nxt.push_back(cnt);
          }
        }
      }
    };
    if (nparts == 1) {
      work(0);
    } else {
      std::vector<std::thread> th;
      for (int pi = 0; pi < nparts; ++pi) th.emplace_back([&, pi]() {
        try {
          work(pi);
        } catch (const std::exception& e) {
          parts[pi].err = e.what();
        }
      });
      for (auto& x : th) x.join();
      for (auto& P : parts)
        if (!P.err.empty()) throw Error(HMAT_ERR_INTERNAL, P.err);
    }
    // concatenate in block order and fill the CSR pointers of the sons (= the next level)
    std::vector<int32_t> nxt_ptr{0}, nxt_rho;
    int64_t next_expected = t.level_begin[lev + 1];
    size_t sym_total = c.sym.size(), nxt_total = 0;
    for (auto& P : parts) sym_total += P.sym.size(), nxt_total += P.nxt_rho.size();
    c.sym.reserve(sym_total);
    nxt_rho.reserve(nxt_total);
    for (auto& P : parts) {
      if (P.n_terms.empty()) continue;
      if (P.first_child != next_expected) throw Error(HMAT_ERR_INTERNAL, "block order");
      size_t lp = 0;
      next_expected += int64_t(P.n_terms.size());
      const int64_t ch0 = P.first_child;
      int64_t spos = int64_t(c.sym.size());
      c.sym.insert(c.sym.end(), P.sym.begin(), P.sym.end());
      nxt_rho.insert(nxt_rho.end(), P.nxt_rho.begin(), P.nxt_rho.end());
      for (size_t k = 0; k < P.n_terms.size(); ++k) {
        const int64_t ch = ch0 + int64_t(k);
        spos += P.n_terms[k];
        c.group_ptr_h[ch + 1] = int32_t(spos);
        if (P.n_leaf[k]) c.hrho.insert(c.hrho.end(), P.leaf_rho.begin() + 3 * lp, P.leaf_rho.begin() + 3 * (lp + P.n_leaf[k]));
        lp += P.n_leaf[k];
        c.hptr[ch + 1] = int32_t(c.hrho.size() / 3);
        nxt_ptr.push_back(nxt_ptr.back() + P.n_nxt[k]);
      }
    }
    for (int pi = 0; pi < nparts; ++pi) {
      arena.part_sym[pi].swap(parts[pi].sym);
      arena.part_nxt[pi].swap(parts[pi].nxt_rho);
      arena.part_leaf[pi].swap(parts[pi].leaf_rho);
    }
    if (int64_t(nxt_ptr.size()) != t.level_begin[lev + 2] - t.level_begin[lev + 1] + 1)
      throw Error(HMAT_ERR_INTERNAL, "level size");
    cur_ptr.swap(nxt_ptr);
    cur_rho.swap(nxt_rho);
    lev_first = t.level_begin[lev + 1];
  }
}

// ------------------------------------------------------------------ subtree task lists
// Tasks of one launch pair (leaf reductions, then output expansion). The device
// enumerates the work items from two prefix sums: leaves of each task's subtree
// (depth-first range) and leaf clusters of each task's output cluster.
struct TaskList {
  std::vector<Task> tasks;
  std::vector<int64_t> lpre{0}, rpre{0};
  DevBuf<Task> d_tasks;
  DevBuf<int64_t> d_lpre, d_rpre;
  DevBuf<int32_t> d_lown, d_rown;  // per work item: (task, item within the task)
  int64_t ws_len = 0;
  void add(const Ctx& c, const Task& tk, bool expand) {
    const Tree& t = *c.t;
    tasks.push_back(tk);
    lpre.push_back(lpre.back() + (c.dfs.hi[tk.q] - c.dfs.lo[tk.q]));
    const int32_t outc = tk.trans ? t.b_sigma[tk.q] : t.b_tau[tk.q];
    rpre.push_back(rpre.back() + (expand ? (t.c_lc_end[outc] - t.c_lc_begin[outc]) : 0));
  }
  int ntask() const { return int(tasks.size()); }
  void upload(hipStream_t s) {
    HM_REQUIRE(lpre.back() < int64_t(INT32_MAX) && rpre.back() < int64_t(INT32_MAX), HMAT_ERR_INTERNAL,
               "too many subtree work items in one list");
    d_tasks.upload(tasks, s);
    d_lpre.upload(lpre, s);
    d_rpre.upload(rpre, s);
    // the per-item tables are written on the device from the prefixes
    d_lown.alloc(size_t(2 * std::max<int64_t>(lpre.back(), 1)));
    d_rown.alloc(size_t(2 * std::max<int64_t>(rpre.back(), 1)));
    launch_fill_owner(d_lpre.p, ntask(), d_lown.p, s);
    launch_fill_owner(d_rpre.p, ntask(), d_rown.p, s);
  }
};

void add_subtree_rows(const Tree& t, int32_t owner, int32_t cluster, std::vector<RowItem>& rows) {
  for (int32_t lc = t.c_lc_begin[cluster]; lc < t.c_lc_end[cluster]; ++lc) {
    int32_t cl = t.leaf_clusters[lc];
    for (int ch = 0; ch * 64 < t.c_size[cl]; ++ch) rows.push_back(RowItem{owner, lc, ch, 0});
  }
}

void build_subsums(const Ctx& c, const HMat* M, SubSums& S) {
  const Tree& t = *c.t;
  const size_t nl = c.dfs.dfs_block.size();
  for (auto* v : {&S.in_f, &S.in_t, &S.rin_f, &S.rin_t, &S.klr, &S.out_f, &S.out_t, &S.vin_f, &S.vin_t})
    v->assign(nl + 1, 0.0);
  for (size_t i = 0; i < nl; ++i) {
    const int32_t b = c.dfs.dfs_block[i];
    const double m = t.c_size[t.b_tau[b]], n = t.c_size[t.b_sigma[b]];
    const double lct = t.c_lc_end[t.b_tau[b]] - t.c_lc_begin[t.b_tau[b]];
    const double lcs = t.c_lc_end[t.b_sigma[b]] - t.c_lc_begin[t.b_sigma[b]];
    double in_f = 0, in_t = 0, rin_f = 0, rin_t = 0, klr = 0, out_f, out_t, vin_f, vin_t;
    if (t.b_kind[b] == KIND_F) {
      const double k = M->rank[b];
      in_f = n * k, in_t = m * k, rin_f = k > 0 ? n : 0, rin_t = k > 0 ? m : 0, klr = k;
      out_f = m * k, out_t = n * k, vin_f = k * lct, vin_t = k * lcs;
    } else {
      out_f = out_t = m * n, vin_f = n * lct, vin_t = m * lcs;
    }
    S.in_f[i + 1] = S.in_f[i] + in_f;
    S.in_t[i + 1] = S.in_t[i] + in_t;
    S.rin_f[i + 1] = S.rin_f[i] + rin_f;
    S.rin_t[i + 1] = S.rin_t[i] + rin_t;
    S.klr[i + 1] = S.klr[i] + klr;
    S.out_f[i + 1] = S.out_f[i] + out_f;
    S.out_t[i + 1] = S.out_t[i] + out_t;
    S.vin_f[i + 1] = S.vin_f[i] + vin_f;
    S.vin_t[i + 1] = S.vin_t[i] + vin_t;
  }
}

// Work of a subtree product of width w on block q of matrix mat (trans: M^T X):
// leaf reductions and output expansion.
void subtree_coef(const Ctx& c, int mat, int32_t q, int trans, Coef& leaf, Coef& expand) {
  const SubSums& S = mat ? c.sb : c.sa;
  const int32_t lo = c.dfs.lo[q], hi = c.dfs.hi[q];
  auto d = [&](const std::vector<double>& v) { return v[hi] - v[lo]; };
  const double in = trans ? d(S.in_t) : d(S.in_f), rin = trans ? d(S.rin_t) : d(S.rin_f);
  const double out = trans ? d(S.out_t) : d(S.out_f), vin = trans ? d(S.vin_t) : d(S.vin_f);
  const double mout = c.t->c_size[trans ? c.t->b_sigma[q] : c.t->b_tau[q]];
  leaf.a += 8 * in;
  leaf.b += 8 * (rin + d(S.klr));
  leaf.f += 2 * in;
  expand.a += 8 * out;
  expand.b += 8 * (vin + mout);
  expand.f += 2 * out;
}

void account(hmat_stats& st, int kind, const Coef& k, double w) {
  st.kern_bytes[kind] += k.a + k.b * w;
  st.kern_flops[kind] += k.f * w;
}

// workspace (doubles) the leaf reductions of a subtree task need
int64_t subtree_ws(const Ctx& c, int mat, int32_t q) {
  const DevMat& dm = mat ? c.db : c.da;
  return (dm.hkpref[c.dfs.hi[q]] - dm.hkpref[c.dfs.lo[q]]) * PW;
}

// Leaf reductions (and expansions) of nl (nr) work items of a task array, owner tables
// lown and rown; X and widths of target tasks come from td.
void run_task_items(Ctx& c, const Task* tasks, int64_t nl, const int32_t* lown, int64_t nr, const int32_t* rown,
                    const TDesc* td, double* ws, bool expand, bool lowp) {
  if (nl > 0) {
    c.timer.begin(K_LEAF);
    launch_leaf_reduce(lown, nl, tasks, td, c.tv, c.ma, c.mb, ws, c.s, lowp);
    c.timer.end();
  }
  if (expand && nr > 0) {
    c.timer.begin(K_EXPAND);
    launch_subtree_expand(rown, nr, tasks, td, c.tv, c.ma, c.mb, ws, c.s, lowp);
    c.timer.end();
  }
}

void run_tasks(Ctx& c, TaskList& L, const TDesc* td, double* ws, bool expand, bool lowp = false) {
  if (L.tasks.empty()) return;
  run_task_items(c, L.d_tasks.p, L.lpre.back(), L.d_lown.p, L.rpre.back(), L.d_rown.p, td, ws, expand, lowp);
}

// Term creation is split so that the host part of a subtree batch can be prepared on a
// worker thread while the previous batch's targets run on the device:
//   layout_terms  - data offsets of the created terms in their pool;
//   prepare_terms - creation task lists and term descriptors (host only; its work
//                   counters go to the CreatePrep, not to the shared statistics);
//   execute_terms - uploads, creation kernels, float copies (device, calling thread).
struct CreatePrep {
  TaskList ff, fh;
  int64_t pos = 0;
  double kern_bytes[8] = {}, kern_flops[8] = {};
  double alg_bytes = 0, alg_flops = 0, t_lists = 0;
  // the terms' device descriptors in the order of `which`, packed and uploaded by the
  // preparing thread (stage_terms): publish_terms then only scatters them
  std::vector<Term> packed;
  DevBuf<int32_t> d_ids;
  DevBuf<Term> d_src;
  bool staged = false;
};

int64_t layout_terms(Ctx& c, const std::vector<int32_t>& which) {
  int64_t pos = 0;
  for (int32_t i : which) {
    SymTerm& st = c.sym[i];
    if (st.type == T_FF) st.data_off = pos, pos += int64_t(st.kl) * st.kr;
    else if (st.type == T_FH) st.data_off = pos, pos += int64_t(st.kl) * c.n_of(st.child);
    else if (st.type == T_HF) st.data_off = pos, pos += int64_t(st.kl) * c.m_of(st.child);
    else st.data_off = -1;
  }
  return pos;
}

void prepare_terms(Ctx& c, const std::vector<int32_t>& which, double* P, int64_t pos, CreatePrep& pr) {
  const Tree& t = *c.t;
  const double th0 = now_seconds();
  pr.pos = pos;
  pr.staged = false;
  for (int k = 0; k < 8; ++k) pr.kern_bytes[k] = pr.kern_flops[k] = 0;
  pr.alg_bytes = pr.alg_flops = 0;
  TaskList& ff = pr.ff;
  TaskList& fh = pr.fh;
  for (TaskList* L : {&ff, &fh}) {  // empty, keeping capacity
    L->tasks.clear();
    L->lpre.assign(1, 0);
    L->rpre.assign(1, 0);
    L->ws_len = 0;
  }
  auto acc = [&](int kind, const Coef& k, double w) {
    pr.kern_bytes[kind] += k.a + k.b * w;
    pr.kern_flops[kind] += k.f * w;
  };
  for (int32_t i : which) {
    const SymTerm& st = c.sym[i];
    if (st.type == T_FF) {
      const int32_t rho = t.b_sigma[st.a_blk];
      const double* LB = c.B->pool.p + c.B->off[st.b_blk];
      for (int j0 = 0; j0 < st.kr; j0 += PW) {
        Task tk{};
        tk.X = LB + int64_t(j0) * t.c_size[rho];
        tk.ldx = t.c_size[rho];
        tk.mat = 0;
        tk.q = st.a_blk;
        tk.trans = 0;
        tk.t = -1;
        tk.w = std::min(PW, st.kr - j0);
        tk.lo = c.dfs.lo[st.a_blk];
        tk.tws = st.data_off + int64_t(j0) * st.kl;
        ff.add(c, tk, false);
        {
          const double nr = t.c_size[rho], w = tk.w;
          Coef k{8 * nr * st.kl, 8 * (nr + st.kl), 2 * nr * st.kl};
          acc(K_LEAF, k, w);
          pr.alg_bytes += k.a + k.b * w;
          pr.alg_flops += k.f * w;
        }
      }
    } else if (st.type == T_FH || st.type == T_HF) {
      const bool isfh = st.type == T_FH;
      const int32_t rho = isfh ? t.b_tau[st.b_blk] : t.b_sigma[st.a_blk];
      const int32_t nrho = t.c_size[rho];
      const double* X;
      if (isfh) X = c.A->pool.p + c.A->off[st.a_blk] + int64_t(st.kl) * c.m_of(st.a_blk);  // R_A
      else X = c.B->pool.p + c.B->off[st.b_blk];                                            // L_B
      const int32_t outn = isfh ? c.n_of(st.child) : c.m_of(st.child);
      for (int j0 = 0; j0 < st.kl; j0 += PW) {
        Task tk{};
        tk.X = X + int64_t(j0) * nrho;
        tk.ldx = nrho;
        tk.Y = P + st.data_off + int64_t(j0) * outn;
        tk.ldy = outn;
        tk.mat = isfh ? 1 : 0;
        tk.q = isfh ? st.b_blk : st.a_blk;
        tk.trans = isfh ? 1 : 0;
        tk.t = -1;
        tk.w = std::min(PW, st.kl - j0);
        tk.lo = c.dfs.lo[tk.q];
        tk.tws = fh.ws_len;
        fh.ws_len += subtree_ws(c, tk.mat, tk.q);
        fh.add(c, tk, true);
        {
          Coef kl, ke;
          subtree_coef(c, tk.mat, tk.q, tk.trans, kl, ke);
          acc(K_LEAF, kl, tk.w);
          acc(K_EXPAND, ke, tk.w);
          pr.alg_bytes += kl.a + kl.b * tk.w + ke.a + ke.b * tk.w;
          pr.alg_flops += (kl.f + ke.f) * tk.w;
        }
      }
    }
  }
  // device descriptors of these terms
  for (int32_t i : which) {
    const SymTerm& st = c.sym[i];
    Term& T = c.hterms[i];
    const double* pa = c.A->pool.p + c.A->off[st.a_blk];
    const double* pb = c.B->pool.p + c.B->off[st.b_blk];
    const int32_t tau2 = t.b_tau[st.child], sig2 = t.b_sigma[st.child];
    T.kl = st.kl;
    T.kr = st.kr;
    T.rtrans = 0;
    T.core = nullptr;
    switch (st.type) {
      case T_FF: {
        const int32_t m = c.m_of(st.a_blk), nrho = c.n_of(st.a_blk), nsig = c.n_of(st.b_blk);
        (void)nrho;
        T.L = pa;  // L_A (tau' x kA)
        T.ldl = m;
        T.lrow0 = t.c_begin[tau2];
        T.R = pb + int64_t(st.kr) * c.m_of(st.b_blk);  // R_B (sigma' x kB)
        T.ldr = nsig;
        T.rrow0 = t.c_begin[sig2];
        T.core = P + st.data_off;
        break;
      }
      case T_FH:
        T.L = pa;
        T.ldl = c.m_of(st.a_blk);
        T.lrow0 = t.c_begin[tau2];
        T.R = P + st.data_off;
        T.ldr = c.n_of(st.child);
        T.rrow0 = t.c_begin[sig2];
        break;
      case T_HF:
        T.L = P + st.data_off;
        T.ldl = c.m_of(st.child);
        T.lrow0 = t.c_begin[tau2];
        T.R = pb + int64_t(st.kr) * c.m_of(st.b_blk);
        T.ldr = c.n_of(st.b_blk);
        T.rrow0 = t.c_begin[sig2];
        break;
      default: {  // both factors dense leaves of the parent level: A[tau, rho] and B[rho, sigma]
        T.L = pa;
        T.ldl = c.m_of(st.a_blk);
        T.lrow0 = t.c_begin[t.b_tau[st.a_blk]];
        T.R = pb;  // stored rho x sigma, read as R(j, c) = B[c + j * #rho]
        T.ldr = c.m_of(st.b_blk);
        T.rrow0 = t.c_begin[t.b_sigma[st.b_blk]];
        T.rtrans = 1;
        break;
      }
    }
  }
  pr.t_lists = now_seconds() - th0;
}

// Packs the descriptors of the terms in `which` (final once prepare_terms has run) and
// uploads them on stream s, on the preparing thread, so that the device does not wait for
// this between a batch's term creation and its targets.
void stage_terms(const Ctx& c, const std::vector<int32_t>& which, CreatePrep& pr, hipStream_t s) {
  pr.packed.resize(which.size());
  for (size_t i = 0; i < which.size(); ++i) pr.packed[i] = c.hterms[size_t(which[i])];
  pr.d_ids.upload(which, s);
  pr.d_src.upload(pr.packed, s);
  pr.staged = true;
}

void execute_terms(Ctx& c, CreatePrep& pr, double* P, DevBuf<float>& pool32_out) {
  hipStream_t s = c.s;
  for (int k = 0; k < 8; ++k) {
    c.st.kern_bytes[k] += pr.kern_bytes[k];
    c.st.kern_flops[k] += pr.kern_flops[k];
  }
  c.alg_bytes += pr.alg_bytes;
  c.alg_flops += pr.alg_flops;
  c.st.t_host[1] += pr.t_lists;
  TaskList& ff = pr.ff;
  TaskList& fh = pr.fh;
  double tu = now_seconds();
  if (!ff.tasks.empty()) ff.upload(s);
  if (!fh.tasks.empty()) fh.upload(s);
  c.st.t_host[5] += now_seconds() - tu;
  tu = now_seconds();
  if (!ff.tasks.empty()) run_tasks(c, ff, nullptr, P, false);
  if (!fh.tasks.empty()) {
    DevBuf<double> ws(size_t(std::max<int64_t>(fh.ws_len, 1)));
    run_tasks(c, fh, nullptr, ws.p, true);
  }
  const int64_t pos = pr.pos;
  if (c.lowp) {
    if (pool32_out.n < size_t(std::max<int64_t>(pos, 1))) pool32_out.alloc(size_t(std::max<int64_t>(pos, 1)));
    if (pos) launch_to_float(P, pool32_out.p, pos, s);
    c.register_pool(P, pos, pool32_out.p);
  }
  HM_CHECK_HIP(hipStreamSynchronize(s));
  c.st.t_host[6] += now_seconds() - tu;
}

// All three steps on the calling thread (terms of levels <= L0).
void create_terms(Ctx& c, const std::vector<int32_t>& which, DevBuf<double>& pool_out, DevBuf<float>& pool32_out,
                  CreatePrep& pr) {
  const int64_t pos = layout_terms(c, which);
  if (pool_out.n < size_t(std::max<int64_t>(pos, 1))) {  // callers may pass a pool sized for several calls
    const double ta = now_seconds();
    pool_out.alloc(size_t(std::max<int64_t>(pos, 1)));
    c.st.t_host[4] += now_seconds() - ta;
  }
  prepare_terms(c, which, pool_out.p, pos, pr);
  execute_terms(c, pr, pool_out.p, pool32_out);
}

// Device descriptors of the terms in `which` (only these changed since the last call);
// `pr`, when given and staged, holds them packed and uploaded already.
void publish_terms(Ctx& c, const std::vector<int32_t>& which, CreatePrep* pr = nullptr) {
  const double t0 = now_seconds();
  struct Acc {
    Ctx& c;
    double t0;
    ~Acc() { c.st.t_host[7] += now_seconds() - t0; }
  } acc{c, t0};
  if (c.terms.n < c.hterms.size()) c.terms.alloc(c.hterms.size());
  if (which.empty()) return;
  static thread_local std::vector<Term> packed_keep;
  DevBuf<int32_t> ids_here;
  DevBuf<Term> src_here;
  const int32_t* ids;
  const Term* src;
  const std::vector<Term>* packed_p;
  if (pr && pr->staged && pr->packed.size() == which.size()) {
    ids = pr->d_ids.p;
    src = pr->d_src.p;
    packed_p = &pr->packed;
  } else {
    std::vector<Term>& packed = packed_keep;
    packed.resize(which.size());
    for (size_t i = 0; i < which.size(); ++i) packed[i] = c.hterms[which[i]];
    ids_here.upload(which, c.s);
    src_here.upload(packed, c.s);
    ids = ids_here.p;
    src = src_here.p;
    packed_p = &packed;
  }
  const std::vector<Term>& packed = *packed_p;
  launch_scatter_terms(ids, src, c.terms.p, int64_t(which.size()), c.s);
  if (c.lowp) {
    // the same terms over the float copies (TermT<float> has the layout of TermT<double>)
    static_assert(sizeof(Term32) == sizeof(Term), "term layouts differ");
    if (c.terms32.n < c.hterms.size()) c.terms32.alloc(c.hterms.size());
    static thread_local std::vector<Term32> p32_keep;  // capacity kept: no page faults per product
    std::vector<Term32>& p32 = p32_keep;
    p32.resize(which.size());
    for (size_t i = 0; i < which.size(); ++i) {
      const Term& T = packed[i];
      Term32& U = p32[i];
      U.L = c.to32(T.L);
      U.R = c.to32(T.R);
      U.core = c.to32(T.core);
      U.ldl = T.ldl;
      U.ldr = T.ldr;
      U.lrow0 = T.lrow0;
      U.rrow0 = T.rrow0;
      U.kl = T.kl;
      U.kr = T.kr;
      U.rtrans = T.rtrans;
      U.pad = 0;
    }
    DevBuf<Term32> src32;
    src32.upload(p32, c.s);
    launch_scatter_terms(ids, reinterpret_cast<const Term*>(src32.p), reinterpret_cast<Term*>(c.terms32.p),
                         int64_t(which.size()), c.s);
    c.tv.terms32 = c.terms32.p;
  }
  HM_CHECK_HIP(hipStreamSynchronize(c.s));
}

// ------------------------------------------------------------------ target chunks
struct Chunk {
  std::vector<int32_t> blocks;  // target blocks
  std::vector<TInfo> info;
  std::vector<HPair> pairs;
  // pair stages: forward B-side (1f) then A-side (2f); transposed A-side (1t) then B-side (2t)
  TaskList t1f, t2f, t1t, t2t;
  std::vector<TermItem> term_items;
  std::vector<RowItem> gf, gt;  // gather items forward / transposed (large targets)
  // pair temporaries start at offset PW so that no stage-2 input offset is 0 (0 = "input from
  // the target's pass descriptor")
  int64_t vlen = 0, tws_f = 0, tws_t = 0, pair_len = PW;
  // device
  DevBuf<TInfo> d_info;
  DevBuf<HPair> d_pairs;
  DevBuf<RowItem> d_gf, d_gt;
  DevBuf<TermItem> d_terms;
  DevBuf<double> vbuf, wsf, wst, pairbuf;
  DevBuf<TDesc> d_td;
  std::vector<Coef> coef[4][2];  // per kernel family and direction, per target
  std::vector<int32_t> small;    // targets applied by the one-wave fused kernel
  std::vector<int32_t> small4;   // targets applied by the four-wave fused kernel
  std::vector<uint8_t> is_small;
  DevBuf<int32_t> d_small, d_small4;
  std::vector<float> feats;  // HMAT_N_FEATURES per target (farfield chunks, when needed)
  // nearfield chunks: targets of at most NEAR_MAX rows and columns are evaluated by the
  // direct kernel (terms and dense x dense pairs); their other pairs stay in `pairs`
  bool near = false;
  // Forward stage-1 sharing holds when every target's input is fixed by sigma (rows of
  // Omega, identity columns). The ACA, Lanczos and fixed-rank schemes apply S to inputs of
  // their own (unit vectors at per-target pivots, Lanczos vectors, power-iteration bases):
  // their chunks give every pair its own stage-1 task.
  bool share_s1 = true;
  std::vector<uint8_t> direct;
  std::vector<int32_t> dpptr, dpairs;  // per direct target (chunk order): dense pairs (A block, B block)
  // direct kernel work, prepared by the builder: (direct target, 64-row block << 16) items,
  // the direct targets' chunk positions, and their algorithmic bytes and flops
  std::vector<int32_t> ditems, dpos;
  std::vector<double> dby, dfl;
  DevBuf<int32_t> d_ditems, d_dblk, d_dpptr, d_dpairs;
  DevBuf<int64_t> d_dco;
  // Forward stage 1 of a pair, B[rho, sigma] X, depends only on the pair block and on X, and
  // in a forward pass X is fixed by sigma (rows of Omega, or identity columns, at a column
  // offset common to the pass). One stage-1 task per pair block serves all targets that hold
  // it; its pass descriptor is entry nt + g, the widest of its targets' descriptors.
  std::vector<int32_t> g_ptr, g_mem;  // CSR: targets of stage-1 group g
  std::vector<Coef> g_leaf, g_exp;    // work of group g's task (per column)
  std::vector<Coef> s1_leaf, s1_exp;  // per target: its stage-1 work as if run alone
  std::vector<TDesc> tdx;             // pass descriptors of the targets, then of the groups
  // Sparse passes. In a pass where few of the chunk's targets are active (a growth round,
  // the later 16-column identity panels of a chunk's widest targets), launching every work
  // item of the chunk costs far more than the active ones' work: each inactive item still
  // reads its task and descriptor before it exits. Such a pass launches only the work items
  // of its active descriptors. `sp_ptr` / `sp_idx`: per list (t1f, t2f, t1t, t2t, term
  // items, gf, gt, small, small4), the entries of each descriptor (targets, then stage-1
  // groups; entries with no descriptor last), built with the chunk.
  bool sp_built = false;
  std::vector<int32_t> sp_ptr[9], sp_idx[9];
  std::vector<char> sp_host;
  DevBuf<char> sp_dev;
  DevBuf<int32_t> sp_own[4];  // owner tables of the compact lists: leaf and expand, two lists
  // recorded on the product's stream after the chunk's last kernel when the chunk is
  // recycled: the builder's stream waits on it before reusing or freeing the device buffers
  hipEvent_t done = nullptr;
  bool pending = false;
  Chunk() = default;
  Chunk(const Chunk&) = delete;
  Chunk& operator=(const Chunk&) = delete;
  ~Chunk() {
    if (done) (void)hipEventDestroy(done);
  }
  void mark_done(hipStream_t s) {
    if (!done) HM_CHECK_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    HM_CHECK_HIP(hipEventRecord(done, s));
    pending = true;
  }
  // empties the chunk for reuse, keeping host capacity and device buffers
  void reset() {
    blocks.clear();
    info.clear();
    pairs.clear();
    for (TaskList* L : {&t1f, &t2f, &t1t, &t2t}) {
      L->tasks.clear();
      L->lpre.assign(1, 0);
      L->rpre.assign(1, 0);
      L->ws_len = 0;
    }
    term_items.clear();
    gf.clear();
    gt.clear();
    vlen = tws_f = tws_t = 0;
    pair_len = PW;
    for (auto& row : coef)
      for (auto& v : row) v.clear();
    small.clear();
    small4.clear();
    is_small.clear();
    feats.clear();
    near = false;
    share_s1 = true;
    direct.clear();
    dpptr.clear();
    dpairs.clear();
    ditems.clear();
    dpos.clear();
    dby.clear();
    dfl.clear();
    g_ptr.clear();
    g_mem.clear();
    g_leaf.clear();
    g_exp.clear();
    s1_leaf.clear();
    s1_exp.clear();
    sp_built = false;
  }
};

constexpr int NEAR_MAX = 256;

// Features of a farfield target for the rank predictor: level, log diam tau,
// log diam sigma, log dist(tau, sigma), log(1 + sum of the ranks of the
// sum-expression's terms, each H-pair counted by min(#rho, m, n)), number of
// terms and pairs.
void target_features(const Ctx& c, int32_t b, float* f) {
  const Tree& t = *c.t;
  const int32_t tau = t.b_tau[b], sig = t.b_sigma[b];
  const int32_t m = t.c_size[tau], n = t.c_size[sig];
  double rsum = 0;
  int cnt = 0;
  for (int32_t a = b; a >= 0; a = t.b_parent[a])
    for (int32_t j = c.group_ptr_h[a]; j < c.group_ptr_h[a + 1]; ++j) {
      rsum += std::min(c.sym[j].kl, c.sym[j].kr);
      ++cnt;
    }
  for (int32_t j = c.hptr[b]; j < c.hptr[b + 1]; ++j) {
    rsum += std::min(t.c_size[c.hrho[3 * j]], std::min(m, n));
    ++cnt;
  }
  f[0] = float(t.b_level[b]);
  f[1] = float(std::log(std::max(t.c_diam[tau], 1e-12)));
  f[2] = float(std::log(std::max(t.c_diam[sig], 1e-12)));
  f[3] = float(std::log(std::max(cluster_dist(t, tau, sig), 1e-12)));
  f[4] = float(std::log1p(rsum));
  f[5] = float(cnt);
}

int64_t target_cost(const Ctx& c, int32_t b, bool far, const Opts& o, int cap) {
  const Tree& t = *c.t;
  int64_t m = c.m_of(b), n = c.n_of(b);
  int64_t v = 0;
  for (int32_t a = b; a >= 0; a = t.b_parent[a])
    for (int32_t i = c.group_ptr_h[a]; i < c.group_ptr_h[a + 1]; ++i)
      v += int64_t(std::max(c.sym[i].kl, c.sym[i].kr)) * PW;
  int64_t pr = 0;
  for (int32_t j = c.hptr[b]; j < c.hptr[b + 1]; ++j) {
    int32_t rho = c.hrho[3 * j], qa = c.hrho[3 * j + 1], qb = c.hrho[3 * j + 2];
    pr += (2 * t.c_size[rho] + std::max(m, n)) * PW;
    pr += 2 * (c.da.hkpref[c.dfs.hi[qa]] - c.da.hkpref[c.dfs.lo[qa]] + c.db.hkpref[c.dfs.hi[qb]] -
               c.db.hkpref[c.dfs.lo[qb]]) * PW;
  }
  int64_t panels = far ? (m * (cap + o.o.probes) + n * cap + 2 * cap * cap + cap) : 0;
  return 8 * (v + pr + panels) + 512;
}

void build_sparse_index(Chunk& ch);

// Work items of the direct nearfield kernel and each direct target's algorithmic bytes and
// flops (terms of the target and of its ancestors, dense x dense pairs): on the builder's
// thread, so that the device does not wait for them.
void prepare_direct(const Ctx& c, Chunk& ch) {
  const Tree& t = *c.t;
  const int nt = int(ch.blocks.size());
  for (int i = 0; i < nt; ++i) {
    if (!ch.direct[i]) continue;
    const int32_t b = ch.blocks[i];
    const int m = c.m_of(b), n = c.n_of(b);
    const int k = int32_t(ch.dpos.size());
    for (int rb = 0; rb < (m + 63) / 64; ++rb) {
      ch.ditems.push_back(k);
      ch.ditems.push_back(rb << 16);
    }
    double by = 8.0 * m * n, fl = 0.0;
    for (int32_t a = b; a >= 0; a = t.b_parent[a])
      for (int32_t j = c.group_ptr_h[a]; j < c.group_ptr_h[a + 1]; ++j) {
        const SymTerm& sy = c.sym[j];
        const double core = sy.type == T_FF ? double(sy.kl) * sy.kr : 0.0;
        by += 8.0 * (double(m) * sy.kl + double(n) * sy.kr + core);
        fl += 2.0 * n * (core + double(m) * sy.kl);
      }
    for (int32_t p = ch.dpptr[k]; p < ch.dpptr[k + 1]; ++p) {
      const double nr = t.c_size[t.b_sigma[ch.dpairs[2 * p]]];
      by += 8.0 * (m * nr + nr * n);
      fl += 2.0 * m * nr * n;
    }
    ch.dpos.push_back(i);
    ch.dby.push_back(by);
    ch.dfl.push_back(fl);
  }
}

void build_chunk(const Ctx& c, Chunk& ch, bool features) {
  const Tree& t = *c.t;
  const int nt = int(ch.blocks.size());
  if (features) {
    ch.feats.resize(size_t(nt) * HMAT_N_FEATURES);
    for (int i = 0; i < nt; ++i) target_features(c, ch.blocks[i], &ch.feats[size_t(i) * HMAT_N_FEATURES]);
  }
  ch.info.resize(nt);
  for (int k = 0; k < 4; ++k)
    for (int d = 0; d < 2; ++d) ch.coef[k][d].assign(nt, Coef{});
  ch.is_small.assign(nt, 0);
  ch.direct.assign(nt, 0);
  ch.dpptr.assign(1, 0);
  ch.dpairs.clear();
  ch.s1_leaf.assign(nt, Coef{});
  ch.s1_exp.assign(nt, Coef{});
  ch.g_leaf.clear();
  ch.g_exp.clear();
  // pair block B[rho, sigma] (and, without sharing, the target) -> stage-1 group
  std::unordered_map<int64_t, int32_t> group_of;
  std::vector<int64_t> group_off;                 // its temporary
  std::vector<std::pair<int32_t, int32_t>> members;
  for (int i = 0; i < nt; ++i) {
    const int32_t b = ch.blocks[i];
    TInfo& ti = ch.info[i];
    ti.block = b;
    ti.vbase = ch.vlen;
    // the direct and fused kernels hold a term of width kl, kr <= 64 in registers and LDS
    // tiles; a target with a wider term (a leaf cluster of duplicate points can exceed the
    // leaf size) goes to term_reduce + gather
    bool narrow_terms = true;
    if (ch.near)
      for (int32_t a = b; narrow_terms && a >= 0; a = t.b_parent[a])
        for (int32_t j = c.group_ptr_h[a]; j < c.group_ptr_h[a + 1]; ++j)
          if (c.sym[j].kl > NEAR_TERM_MAX || c.sym[j].kr > NEAR_TERM_MAX) narrow_terms = false;
    const bool direct = ch.near && narrow_terms && c.m_of(b) <= NEAR_MAX && c.n_of(b) <= NEAR_MAX;
    ch.direct[i] = direct;
    const double mt = t.c_size[t.b_tau[b]], nt_ = t.c_size[t.b_sigma[b]];
    // the fused kernels serve nearfield targets that add pair results to the direct
    // kernel's output; farfield targets of every size use term_reduce + gather, which
    // measured faster on them than the fused kernels
    const bool small1 = ch.near && narrow_terms && mt <= FUSED_MAX && nt_ <= FUSED_MAX;
    const bool small = small1 || (ch.near && narrow_terms && mt <= FUSED4_MAX && nt_ <= FUSED4_MAX);
    ch.is_small[i] = small1 ? 1 : small ? 2 : 0;
    if (small1) ch.small.push_back(i);
    else if (small) ch.small4.push_back(i);
    double skl = 0, skr = 0;
    for (int32_t a = b; a >= 0; a = t.b_parent[a])
      for (int32_t j = c.group_ptr_h[a]; j < c.group_ptr_h[a + 1]; ++j) {
        if (!small) {
          ch.term_items.push_back(TermItem{i, j, ch.vlen});
          ch.vlen += int64_t(std::max(c.sym[j].kl, c.sym[j].kr)) * PW;
        }
        const SymTerm& sy = c.sym[j];
        const double core = sy.type == T_FF ? double(sy.kl) * sy.kr : 0.0;
        Coef& f = ch.coef[K_TERM][0][i];
        f.a += 8 * (nt_ * sy.kr + core);
        f.b += 8 * (nt_ + sy.kl);
        f.f += 2 * (nt_ * sy.kr + core);
        Coef& tr = ch.coef[K_TERM][1][i];
        tr.a += 8 * (mt * sy.kl + core);
        tr.b += 8 * (mt + sy.kr);
        tr.f += 2 * (mt * sy.kl + core);
        skl += sy.kl;
        skr += sy.kr;
      }
    {
      const int32_t np = c.hptr[b + 1] - c.hptr[b];
      const double nchf = t.c_lc_end[t.b_tau[b]] - t.c_lc_begin[t.b_tau[b]];
      const double ncht = t.c_lc_end[t.b_sigma[b]] - t.c_lc_begin[t.b_sigma[b]];
      Coef& gf = ch.coef[K_GATHER][0][i];
      gf.a = 8 * mt * skl;
      gf.b = 8 * (skl * nchf + mt * (np + 1));
      gf.f = 2 * mt * skl + mt * np;
      Coef& gt = ch.coef[K_GATHER][1][i];
      gt.a = 8 * nt_ * skr;
      gt.b = 8 * (skr * ncht + nt_ * (np + 1));
      gt.f = 2 * nt_ * skr + nt_ * np;
    }
    ti.hp_begin = int32_t(ch.pairs.size());
    const int32_t tau = t.b_tau[b], sig = t.b_sigma[b];
    const int32_t m = t.c_size[tau], n = t.c_size[sig];
    for (int32_t j = c.hptr[b]; j < c.hptr[b + 1]; ++j) {
      const int32_t rho = c.hrho[3 * j], qa = c.hrho[3 * j + 1], qb = c.hrho[3 * j + 2];
      if (qa < 0 || qb < 0) throw Error(HMAT_ERR_INTERNAL, "pair blocks missing");
      if (direct && t.b_kind[qa] == KIND_N && t.b_kind[qb] == KIND_N) {  // done by the direct kernel
        ch.dpairs.push_back(qa);
        ch.dpairs.push_back(qb);
        continue;
      }
      subtree_coef(c, 1, qb, 0, ch.s1_leaf[i], ch.s1_exp[i]);
      subtree_coef(c, 0, qa, 0, ch.coef[K_LEAF][0][i], ch.coef[K_EXPAND][0][i]);
      subtree_coef(c, 0, qa, 1, ch.coef[K_LEAF][1][i], ch.coef[K_EXPAND][1][i]);
      subtree_coef(c, 1, qb, 1, ch.coef[K_LEAF][1][i], ch.coef[K_EXPAND][1][i]);
      const int64_t off1 = ch.pair_len;  // transposed stage 1 (per pair)
      ch.pair_len += int64_t(t.c_size[rho]) * PW;
      const int64_t off2 = ch.pair_len;
      ch.pair_len += int64_t(std::max(m, n)) * PW;
      ch.pairs.push_back(HPair{reinterpret_cast<double*>(off2)});  // offset, rebased on upload
      auto stage = [&](TaskList& L, int64_t& tws, int mat, int32_t q, int trans, int64_t xoff, int64_t yoff,
                       int ldy, int32_t tdi) {
        Task tk{};
        tk.X = xoff < 0 ? nullptr : reinterpret_cast<double*>(xoff);
        tk.ldx = t.c_size[rho];
        tk.Y = reinterpret_cast<double*>(yoff);
        tk.ldy = ldy;
        tk.mat = mat;
        tk.q = q;
        tk.trans = trans;
        tk.t = tdi;
        tk.lo = c.dfs.lo[q];
        tk.tws = tws;
        tws += subtree_ws(c, mat, q);
        L.add(c, tk, true);
      };
      // forward: B[rho, sigma] X -> temp1 of the pair block's group, then A[tau, rho] temp1 -> temp2
      const int64_t gkey = ch.share_s1 ? int64_t(qb) : (int64_t(i) << 32) | int64_t(uint32_t(qb));
      auto gi = group_of.find(gkey);
      if (gi == group_of.end()) {
        const int32_t g = int32_t(group_off.size());
        gi = group_of.emplace(gkey, g).first;
        group_off.push_back(ch.pair_len);
        ch.pair_len += int64_t(t.c_size[rho]) * PW;
        ch.g_leaf.emplace_back();
        ch.g_exp.emplace_back();
        subtree_coef(c, 1, qb, 0, ch.g_leaf.back(), ch.g_exp.back());
        stage(ch.t1f, ch.tws_f, 1, qb, 0, -1, group_off[g], t.c_size[rho], nt + g);
      }
      members.emplace_back(gi->second, i);
      stage(ch.t2f, ch.tws_f, 0, qa, 0, group_off[gi->second], off2, m, i);
      // transposed: A[tau, rho]^T X -> temp1, then B[rho, sigma]^T temp1 -> temp2
      stage(ch.t1t, ch.tws_t, 0, qa, 1, -1, off1, t.c_size[rho], i);
      stage(ch.t2t, ch.tws_t, 1, qb, 1, off1, off2, n, i);
    }
    ti.hp_end = int32_t(ch.pairs.size());
    if (direct) {
      ch.dpptr.push_back(int32_t(ch.dpairs.size() / 2));
      for (int d = 0; d < 2; ++d) ch.coef[K_TERM][d][i] = ch.coef[K_GATHER][d][i] = Coef{};  // terms: direct kernel
    }
    if (!small) {
      add_subtree_rows(t, i, tau, ch.gf);
      add_subtree_rows(t, i, sig, ch.gt);
    }
  }
  // members of each stage-1 group (CSR, targets in chunk order)
  const int32_t ng = int32_t(group_off.size());
  ch.g_ptr.assign(size_t(ng) + 1, 0);
  for (const auto& gm : members) ch.g_ptr[gm.first + 1]++;
  for (int32_t g = 0; g < ng; ++g) ch.g_ptr[g + 1] += ch.g_ptr[g];
  ch.g_mem.resize(members.size());
  {
    std::vector<int32_t> fill(ch.g_ptr.begin(), ch.g_ptr.end() - 1);
    for (const auto& gm : members) ch.g_mem[fill[gm.first]++] = gm.second;
  }
  // built here, on the builder's thread while the device runs the previous chunk, rather
  // than at the chunk's first sparse pass, when the device would wait for it
  build_sparse_index(ch);
  if (ch.near) prepare_direct(c, ch);
}

void upload_chunk(Chunk& ch, hipStream_t s) {
  ch.pairbuf.alloc(size_t(std::max<int64_t>(ch.pair_len, 1)));
  double* base = ch.pairbuf.p;
  auto rebase = [&](const double* p) { return base + reinterpret_cast<intptr_t>(p); };
  for (auto& hp : ch.pairs) hp.temp2 = rebase(hp.temp2);
  for (auto* L : {&ch.t1f, &ch.t2f, &ch.t1t, &ch.t2t})
    for (Task& tk : L->tasks) {
      tk.Y = rebase(tk.Y);
      if (tk.X) tk.X = rebase(tk.X);
    }
  ch.d_info.upload(ch.info, s);
  ch.d_pairs.upload(ch.pairs, s);
  for (auto* L : {&ch.t1f, &ch.t2f, &ch.t1t, &ch.t2t}) L->upload(s);
  ch.d_gf.upload(ch.gf, s);
  ch.d_gt.upload(ch.gt, s);
  ch.d_terms.upload(ch.term_items, s);
  ch.d_small.upload(ch.small, s);
  ch.d_small4.upload(ch.small4, s);
  ch.vbuf.alloc(size_t(std::max<int64_t>(ch.vlen, 1)));
  ch.wsf.alloc(size_t(std::max<int64_t>(ch.tws_f, 1)));
  ch.wst.alloc(size_t(std::max<int64_t>(ch.tws_t, 1)));
  ch.d_td.alloc(ch.blocks.size() + ch.g_leaf.size());
  if (!ch.dpos.empty()) {
    std::vector<int32_t> dblk(ch.dpos.size());
    for (size_t k = 0; k < ch.dpos.size(); ++k) dblk[k] = ch.blocks[size_t(ch.dpos[k])];
    ch.d_ditems.upload(ch.ditems, s);
    ch.d_dblk.upload(dblk, s);
    ch.d_dpptr.upload(ch.dpptr, s);
    if (ch.dpairs.empty()) {
      const int32_t none[2] = {0, 0};
      ch.d_dpairs.upload(none, 2, s);
    } else {
      ch.d_dpairs.upload(ch.dpairs, s);
    }
  }
  HM_CHECK_HIP(hipStreamSynchronize(s));  // the work-item tables are written by kernels on s
}

// One application of every target's operator in the chunk (forward: S X, transposed: S^T X).
// Index of the chunk's work items by pass descriptor (see Chunk::sp_ptr).
void build_sparse_index(Chunk& ch) {
  const int32_t nd = int32_t(ch.blocks.size() + ch.g_leaf.size());  // targets, then stage-1 groups
  auto csr = [&](int li, size_t n, auto key) {
    std::vector<int32_t>& ptr = ch.sp_ptr[li];
    std::vector<int32_t>& idx = ch.sp_idx[li];
    ptr.assign(size_t(nd) + 2, 0);
    for (size_t i = 0; i < n; ++i) {
      const int32_t k = key(i);
      ptr[size_t(k >= 0 && k < nd ? k : nd) + 1]++;
    }
    for (size_t j = 0; j + 1 < ptr.size(); ++j) ptr[j + 1] += ptr[j];
    idx.resize(n);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (size_t i = 0; i < n; ++i) {
      const int32_t k = key(i);
      idx[size_t(fill[size_t(k >= 0 && k < nd ? k : nd)]++)] = int32_t(i);
    }
  };
  TaskList* lists[4] = {&ch.t1f, &ch.t2f, &ch.t1t, &ch.t2t};
  for (int li = 0; li < 4; ++li) {
    const TaskList& L = *lists[li];
    csr(li, L.tasks.size(), [&](size_t i) { return L.tasks[i].t; });
  }
  csr(4, ch.term_items.size(), [&](size_t i) { return ch.term_items[i].t; });
  csr(5, ch.gf.size(), [&](size_t i) { return ch.gf[i].owner; });
  csr(6, ch.gt.size(), [&](size_t i) { return ch.gt[i].owner; });
  csr(7, ch.small.size(), [&](size_t i) { return ch.small[i]; });
  csr(8, ch.small4.size(), [&](size_t i) { return ch.small4[i]; });
  ch.sp_built = true;
}

// One pass over the work items of the active descriptors only (ch.tdx holds the pass's
// descriptors; they go up in the same copy as the compact lists). Every launched item does
// what it does in a full pass, so the results are the same bit for bit.
void run_pass_sparse(Ctx& c, Chunk& ch, bool trans, bool lowp) {
  hipStream_t s = c.s;
  if (!ch.sp_built) build_sparse_index(ch);
  const int32_t nd = int32_t(ch.tdx.size());
  HM_REQUIRE(size_t(nd) + 2 == ch.sp_ptr[0].size(), HMAT_ERR_INTERNAL, "sparse pass index out of date");
  std::vector<int32_t> act;
  for (int32_t j = 0; j < nd; ++j)
    if (ch.tdx[j].w > 0) act.push_back(j);
  act.push_back(nd);  // entries with no descriptor
  std::vector<char>& h = ch.sp_host;
  h.clear();
  auto section = [&](size_t bytes) {
    const size_t off = (h.size() + 255) & ~size_t(255);
    h.resize(off + bytes);
    return off;
  };
  const size_t td_off = section(ch.tdx.size() * sizeof(TDesc));
  std::memcpy(h.data() + td_off, ch.tdx.data(), ch.tdx.size() * sizeof(TDesc));
  // gathers the active entries of list li from src into a new section; returns (offset, count)
  auto gather = [&](int li, const auto& src) {
    using T = typename std::decay_t<decltype(src)>::value_type;
    size_t cnt = 0;
    for (int32_t j : act) cnt += size_t(ch.sp_ptr[li][size_t(j) + 1] - ch.sp_ptr[li][size_t(j)]);
    const size_t off = section(cnt * sizeof(T));
    T* out = reinterpret_cast<T*>(h.data() + off);
    size_t k = 0;
    for (int32_t j : act)
      for (int32_t e = ch.sp_ptr[li][size_t(j)]; e < ch.sp_ptr[li][size_t(j) + 1]; ++e) out[k++] = src[size_t(ch.sp_idx[li][size_t(e)])];
    return std::make_pair(off, cnt);
  };
  // task lists of this direction: tasks, and the prefix sums of their leaf and expansion items
  struct Compact {
    size_t tasks = 0, lpre = 0, rpre = 0, n = 0;
    int64_t nl = 0, nr = 0;
  } cl[2];
  TaskList* lists[2] = {trans ? &ch.t1t : &ch.t1f, trans ? &ch.t2t : &ch.t2f};
  for (int x = 0; x < 2; ++x) {
    const int li = (trans ? 2 : 0) + x;
    const TaskList& L = *lists[x];
    auto tk = gather(li, L.tasks);
    cl[x].tasks = tk.first;
    cl[x].n = tk.second;
    cl[x].lpre = section((tk.second + 1) * sizeof(int64_t));
    cl[x].rpre = section((tk.second + 1) * sizeof(int64_t));
    int64_t* lp = reinterpret_cast<int64_t*>(h.data() + cl[x].lpre);
    int64_t* rp = reinterpret_cast<int64_t*>(h.data() + cl[x].rpre);
    lp[0] = rp[0] = 0;
    size_t k = 0;
    for (int32_t j : act)
      for (int32_t e = ch.sp_ptr[li][size_t(j)]; e < ch.sp_ptr[li][size_t(j) + 1]; ++e, ++k) {
        const size_t i = size_t(ch.sp_idx[li][size_t(e)]);
        lp[k + 1] = lp[k] + (L.lpre[i + 1] - L.lpre[i]);
        rp[k + 1] = rp[k] + (L.rpre[i + 1] - L.rpre[i]);
      }
    cl[x].nl = lp[k];
    cl[x].nr = rp[k];
  }
  const auto terms = gather(4, ch.term_items);
  const auto rows = trans ? gather(6, ch.gt) : gather(5, ch.gf);
  const auto small = gather(7, ch.small);
  const auto small4 = gather(8, ch.small4);
  ch.sp_dev.upload(h, s);  // one synchronous copy
  const char* d = ch.sp_dev.p;
  const TDesc* dtd = reinterpret_cast<const TDesc*>(d + td_off);
  double* ws = trans ? ch.wst.p : ch.wsf.p;
  for (int x = 0; x < 2; ++x) {
    if (cl[x].n == 0) continue;
    DevBuf<int32_t>& lown = ch.sp_own[2 * x];
    DevBuf<int32_t>& rown = ch.sp_own[2 * x + 1];
    if (lown.n < size_t(2 * std::max<int64_t>(cl[x].nl, 1))) lown.alloc(size_t(2 * std::max<int64_t>(cl[x].nl, 1)));
    if (rown.n < size_t(2 * std::max<int64_t>(cl[x].nr, 1))) rown.alloc(size_t(2 * std::max<int64_t>(cl[x].nr, 1)));
    launch_fill_owner(reinterpret_cast<const int64_t*>(d + cl[x].lpre), int(cl[x].n), lown.p, s);
    launch_fill_owner(reinterpret_cast<const int64_t*>(d + cl[x].rpre), int(cl[x].n), rown.p, s);
    run_task_items(c, reinterpret_cast<const Task*>(d + cl[x].tasks), cl[x].nl, lown.p, cl[x].nr, rown.p, dtd, ws,
                   true, lowp);
  }
  if (terms.second) {
    c.timer.begin(K_TERM);
    launch_term_reduce(reinterpret_cast<const TermItem*>(d + terms.first), terms.second, dtd, ch.d_info.p, c.tv,
                       ch.vbuf.p, s, lowp);
    c.timer.end();
  }
  if (rows.second) {
    c.timer.begin(K_GATHER);
    launch_gather_mfma(reinterpret_cast<const RowItem*>(d + rows.first), rows.second, dtd, ch.d_info.p, ch.d_pairs.p,
                       c.tv, ch.vbuf.p, s, lowp);
    c.timer.end();
  }
  if (small.second) {
    c.timer.begin(K_FUSED);
    launch_fused_terms(reinterpret_cast<const int32_t*>(d + small.first), small.second, dtd, ch.d_info.p,
                       ch.d_pairs.p, c.tv, s, lowp);
    c.timer.end();
  }
  if (small4.second) {
    c.timer.begin(K_FUSED4);
    launch_fused_terms4(reinterpret_cast<const int32_t*>(d + small4.first), small4.second, dtd, ch.d_info.p,
                        ch.d_pairs.p, c.tv, s, lowp);
    c.timer.end();
  }
}

void run_pass(Ctx& c, Chunk& ch, const std::vector<TDesc>& td, bool trans, bool lowp = false) {
  hipStream_t s = c.s;
  // descriptors of the targets, then of the stage-1 groups (forward passes): a group takes
  // the descriptor of its widest target (same X for all of them; the others read a prefix
  // of the columns)
  const size_t nt = td.size(), ngr = ch.g_leaf.size();
  ch.tdx.assign(td.begin(), td.end());
  ch.tdx.resize(nt + ngr);
  for (size_t g = 0; g < ngr; ++g) {
    TDesc& e = ch.tdx[nt + g];
    std::memset(&e, 0, sizeof(e));
    if (trans) continue;
    for (int32_t k = ch.g_ptr[g]; k < ch.g_ptr[g + 1]; ++k)
      if (td[ch.g_mem[k]].w > e.w) e = td[ch.g_mem[k]];
    e.Y = nullptr;  // stage 1 writes the group's temporary
    if (e.w) {
      account(c.st, K_LEAF, ch.g_leaf[g], e.w);
      account(c.st, K_EXPAND, ch.g_exp[g], e.w);
    }
  }
  const int d = trans ? 1 : 0;
  for (size_t i = 0; i < nt; ++i)
    if (td[i].w) {
      c.st.target_passes++;
      account(c.st, K_LEAF, ch.coef[K_LEAF][d][i], td[i].w);
      account(c.st, K_EXPAND, ch.coef[K_EXPAND][d][i], td[i].w);
      if (ch.is_small[i]) {
        const int kf = ch.is_small[i] == 1 ? K_FUSED : K_FUSED4;
        account(c.st, kf, ch.coef[K_TERM][d][i], td[i].w);
        account(c.st, kf, ch.coef[K_GATHER][d][i], td[i].w);
      } else {
        account(c.st, K_TERM, ch.coef[K_TERM][d][i], td[i].w);
        account(c.st, K_GATHER, ch.coef[K_GATHER][d][i], td[i].w);
      }
    }
  size_t nact = 0;
  for (size_t i = 0; i < nt; ++i) nact += td[i].w > 0;
  c.st.n_passes++;
  if (!c.opts.o.full_passes && nact * 8 <= nt && nt >= 64) {
    c.st.n_sparse_passes++;
    run_pass_sparse(c, ch, trans, lowp);  // uploads the descriptors with its lists
    return;
  }
  ch.d_td.upload(ch.tdx, s);  // synchronous: the descriptors are rewritten for the next pass
  const TDesc* dtd = ch.d_td.p;
  if (!trans) {
    run_tasks(c, ch.t1f, dtd, ch.wsf.p, true, lowp);
    run_tasks(c, ch.t2f, dtd, ch.wsf.p, true, lowp);
  } else {
    run_tasks(c, ch.t1t, dtd, ch.wst.p, true, lowp);
    run_tasks(c, ch.t2t, dtd, ch.wst.p, true, lowp);
  }
  if (!ch.term_items.empty()) {
    c.timer.begin(K_TERM);
    launch_term_reduce(ch.d_terms.p, ch.term_items.size(), dtd, ch.d_info.p, c.tv, ch.vbuf.p, s, lowp);
    c.timer.end();
  }
  const size_t ng = trans ? ch.gt.size() : ch.gf.size();
  if (ng) {
    c.timer.begin(K_GATHER);
    launch_gather_mfma(trans ? ch.d_gt.p : ch.d_gf.p, ng, dtd, ch.d_info.p, ch.d_pairs.p, c.tv, ch.vbuf.p, s, lowp);
    c.timer.end();
  }
  if (!ch.small.empty()) {
    c.timer.begin(K_FUSED);
    launch_fused_terms(ch.d_small.p, ch.small.size(), dtd, ch.d_info.p, ch.d_pairs.p, c.tv, s, lowp);
    c.timer.end();
  }
  if (!ch.small4.empty()) {
    c.timer.begin(K_FUSED4);
    launch_fused_terms4(ch.d_small4.p, ch.small4.size(), dtd, ch.d_info.p, ch.d_pairs.p, c.tv, s, lowp);
    c.timer.end();
  }
}

struct FarOut {
  DevBuf<double> buf;
  std::vector<int32_t> blocks, ranks;
  std::vector<int32_t> widths;  // randomized scheme: columns of Q when the residual check passed
  std::vector<uint8_t> done;
  std::vector<int64_t> offs;
  int64_t len = 0;
};

// Minimum algorithmic work of farfield target i of a chunk at final rank k: one forward
// and one transposed pass of width k, the core factorisations and the factor output.
void charge_far(Ctx& c, const Chunk& ch, int i, int32_t block, int m, int n, int k) {
  const double w = std::max(k, 1);
  for (int kk = 0; kk < 4; ++kk)
    for (int d = 0; d < 2; ++d) {
      const Coef& cf = ch.coef[kk][d][i];
      c.charge(block, cf.a + cf.b * w, cf.f * w);
    }
  for (const Coef* cf : {&ch.s1_leaf[i], &ch.s1_exp[i]})  // forward stage 1, counted per target
    c.charge(block, cf->a + cf->b * w, cf->f * w);
  c.charge(block, 8.0 * (m + n) * k, 4.0 * (m + n) * w * w + 22.0 * w * w * w);
}

// Omega with at least ncol columns (rows keyed by position, so regenerating it for more
// columns keeps the existing ones).
void ensure_omega(Ctx& c, int64_t ncol) {
  if (c.omega_cols >= ncol) return;
  c.omega.alloc(size_t(c.t->n) * size_t(ncol));
  launch_fill_gaussian(c.omega.p, c.t->n, int32_t(ncol), c.opts.o.seed, c.s);
  c.omega_cols = ncol;
}

// Randomized compression of the chunk's farfield targets.
void compress_chunk(Ctx& c, Chunk& ch, const std::vector<int32_t>& w0, FarOut& out) {
  const Tree& t = *c.t;
  hipStream_t s = c.s;
  const int g = c.opts.o.probes;
  int b0max = 0;
  for (int x : w0) b0max = std::max(b0max, x);
  const int cap = std::min(64, std::max(b0max, c.opts.o.b0) + c.opts.o.max_growth * g);
  CParams cp{cap, g, c.eps, c.opts.o.delta, 9.0};
  const int nt = int(ch.blocks.size());
  const int64_t ncol_om = std::max(b0max, c.opts.o.b0) + int64_t(g) * (c.opts.o.max_growth + 1);
  // panels
  int64_t need = 0;
  for (int32_t b : ch.blocks) need += int64_t(c.m_of(b)) * (cap + g) + int64_t(c.n_of(b)) * cap + 2 * cap * cap + cap;
  DevBuf<double> ws{size_t(need)};
  std::vector<CTarget> h(nt);
  int64_t o = 0;
  for (int i = 0; i < nt; ++i) {
    const int32_t b = ch.blocks[i];
    CTarget& T = h[i];
    std::memset(&T, 0, sizeof(T));
    T.m = c.m_of(b);
    T.n = c.n_of(b);
    T.row0 = t.c_begin[t.b_tau[b]];
    T.col0 = t.c_begin[t.b_sigma[b]];
    T.Y = ws.p + o;
    o += int64_t(T.m) * (cap + g);
    T.Z = ws.p + o;
    o += int64_t(T.n) * cap;
    T.core = ws.p + o;
    o += 2 * cap * cap + cap;
    T.active = 1;
    T.block = b;
    T.w0 = w0[i];
  }
  // Gaussian columns shared by all targets (rows keyed by position), generated once
  ensure_omega(c, ncol_om);
  const double* omega_p = c.omega.p;
  DevBuf<CTarget> dt(nt);
  dt.upload(h, s);
  std::vector<TDesc> td(nt);
  auto clear_td = [&]() {
    for (auto& d : td) std::memset(&d, 0, sizeof(d));
  };
  // forward pass over global columns [j0, j0 + w) of [sketch (w0) | probe (g)]
  auto sketch_probe = [&](const std::vector<int>& active, int col_probe) {
    // widths differ per target: run chunks of PW columns over the max total width
    int maxw = 0;
    for (int i = 0; i < nt; ++i)
      if (active[i]) maxw = std::max(maxw, h[i].w0 + g);
    for (int j0 = 0; j0 < maxw; j0 += PW) {
      clear_td();
      bool any = false;
      for (int i = 0; i < nt; ++i) {
        if (!active[i]) continue;
        const CTarget& T = h[i];
        const int tot = col_probe < 0 ? T.w0 + g : g;
        if (j0 >= tot) continue;
        TDesc& d = td[i];
        d.w = std::min(PW, tot - j0);
        d.trans = 0;
        d.ldx = int32_t(t.n);
        d.ldy = T.m;
        if (col_probe < 0) {
          // columns [0, w0) of Omega -> Q area; [w0, w0 + g) -> probe area at cap
          d.X = omega_p + int64_t(j0) * t.n + T.col0;
          if (j0 < T.w0) {
            d.Y = T.Y + int64_t(j0) * T.m;
            d.split = T.w0 - j0;
            d.gap = cap - T.w0;
          } else {
            d.Y = T.Y + int64_t(j0 - T.w0 + cap) * T.m;
            d.split = d.w;
            d.gap = 0;
          }
          // probe columns of the first pass come from Omega columns [w0, w0 + g): they are
          // distinct from the sketch columns by construction
        } else {
          d.X = omega_p + int64_t(col_probe + j0) * t.n + T.col0;
          d.Y = T.Y + int64_t(cap + j0) * T.m;
          d.split = d.w;
          d.gap = 0;
        }
        any = true;
      }
      if (any) run_pass(c, ch, td, false, c.lowp);
    }
  };
  auto project = [&](const std::vector<int>& r_from, const std::vector<int>& r_to) {
    int maxw = 0;
    for (int i = 0; i < nt; ++i) maxw = std::max(maxw, r_to[i] - r_from[i]);
    for (int j0 = 0; j0 < maxw; j0 += PW) {
      clear_td();
      bool any = false;
      for (int i = 0; i < nt; ++i) {
        const CTarget& T = h[i];
        const int nw = r_to[i] - r_from[i];
        if (j0 >= nw) continue;
        TDesc& d = td[i];
        d.w = std::min(PW, nw - j0);
        d.trans = 1;
        d.X = T.Y + int64_t(r_from[i] + j0) * T.m;
        d.ldx = T.m;
        d.Y = T.Z + int64_t(r_from[i] + j0) * T.n;
        d.ldy = T.n;
        d.split = d.w;
        any = true;
      }
      if (any) run_pass(c, ch, td, true);
    }
  };
  auto fetch = [&]() {
    const double t0 = now_seconds();
    HM_CHECK_HIP(hipMemcpyAsync(h.data(), dt.p, sizeof(CTarget) * nt, hipMemcpyDeviceToHost, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    c.st.t_host[3] += now_seconds() - t0;
  };
  std::vector<int> all(nt, 1);
  double t0 = now_seconds();
  sketch_probe(all, -1);
  // orthonormalise the sketch columns (per-target counts differ: run with the max and let
  // targets with fewer columns see zero-width extra columns)
  {
    int maxw0 = 0;
    for (auto& T : h) maxw0 = std::max(maxw0, T.w0);
    c.timer.begin(K_COMPRESS);
    launch_orth_append(dt.p, nt, 0, maxw0, cp, s);
    c.timer.end();  // each target uses its own w0 columns
  }
  c.timer.begin(K_COMPRESS);
    launch_probe_residual(dt.p, nt, cp, s);
    c.timer.end();
  fetch();
  double t1 = now_seconds();
  c.st.t_sketch += t1 - t0;
  std::vector<int> rf(nt, 0), rt(nt);
  for (int i = 0; i < nt; ++i) rt[i] = h[i].r;
  project(rf, rt);
  for (auto& T : h) T.rz = T.r;
  dt.upload(h, s);
  double t2 = now_seconds();
  c.st.t_project += t2 - t1;
  DevBuf<int32_t> pending(nt);
  std::vector<int32_t> hp(nt);
  for (auto& T : h) c.st.sketch_columns += T.w0;
  for (int round = 0; round < c.opts.o.max_growth; ++round) {
    launch_check(dt.p, nt, cp, pending.p, s);
    HM_CHECK_HIP(hipMemcpyAsync(hp.data(), pending.p, 4 * nt, hipMemcpyDeviceToHost, s));
    fetch();
    int cnt = 0;
    for (int i = 0; i < nt; ++i) {
      h[i].active = hp[i];
      cnt += hp[i];
    }
    if (!cnt) break;
    c.st.n_growth_rounds++;
    c.st.n_grown_blocks += cnt;
    double ta = now_seconds();
    const double tg0 = ta;
    dt.upload(h, s);
    std::vector<int> r_old(nt);
    for (int i = 0; i < nt; ++i) r_old[i] = h[i].r;
    c.timer.begin(K_COMPRESS);
    launch_orth_append(dt.p, nt, cap, g, cp, s);
    c.timer.end();
    fetch();
    std::vector<int> act(nt);
    for (int i = 0; i < nt; ++i) {
      act[i] = h[i].active;
      if (act[i]) {
        h[i].rounds++;
        c.st.sketch_columns += g;
      }
    }
    // next probe columns of Omega: [w0 + g * (round + 1), ...) keyed per round
    sketch_probe(act, std::max(b0max, c.opts.o.b0) + g * (round + 1));
    double tb = now_seconds();
    c.st.t_sketch += tb - ta;
    std::vector<int> rto(nt);
    for (int i = 0; i < nt; ++i) rto[i] = act[i] ? h[i].r : r_old[i];
    for (int i = 0; i < nt; ++i)
      if (!act[i]) r_old[i] = rto[i];
    project(r_old, rto);
    for (int i = 0; i < nt; ++i) h[i].rz = h[i].r;
    dt.upload(h, s);
    c.timer.begin(K_COMPRESS);
    launch_probe_residual(dt.p, nt, cp, s);
    c.timer.end();
    c.st.t_project += now_seconds() - tb;
    c.st.t_growth += now_seconds() - tg0;
  }
  double t3 = now_seconds();
  launch_check(dt.p, nt, cp, pending.p, s);
  c.timer.begin(K_COMPRESS);
    int rmax = 1;
    for (const auto& T : h) rmax = std::max(rmax, T.rz);
    launch_core(dt.p, nt, cp, s, rmax);
    c.timer.end();
  fetch();
  out.blocks.clear();
  out.ranks.clear();
  out.widths.clear();
  out.done.clear();
  out.offs.clear();
  out.len = 0;
  for (int i = 0; i < nt; ++i) {
    CTarget& T = h[i];
    out.widths.push_back(T.r);
    if (!T.done) c.st.n_not_converged++;
    if (T.svd_capped) c.st.n_svd_sweep_cap++;
    if (T.rounds > 0 && c.opts.o.rank_mode == HMAT_RANK_PREDICT) c.st.n_fallback++;
    out.blocks.push_back(T.block);
    out.ranks.push_back(T.k);
    out.done.push_back(uint8_t(T.done ? 1 : 0));
    out.offs.push_back(out.len);
    T.out_off = out.len;
    out.len += int64_t(T.k) * (T.m + T.n);
    c.st.rank_hist[std::min(T.k, 64)]++;
    charge_far(c, ch, i, T.block, T.m, T.n, T.k);
  }
  out.buf.alloc(size_t(std::max<int64_t>(out.len, 1)));
  dt.upload(h, s);
  c.timer.begin(K_COMPRESS);
    launch_write_factors(dt.p, nt, cp, out.buf.p, s);
    c.timer.end();
  HM_CHECK_HIP(hipStreamSynchronize(s));
  c.st.t_core += now_seconds() - t3;
}

// ------------------------------------------------------------------ Algorithm 5
// Columns of the stacked term factor of a farfield target (sum of the widths of its
// terms and of its ancestors' terms; every term contributes L core, of kr columns).
int64_t term_columns(const Ctx& c, int32_t b) {
  const Tree& t = *c.t;
  int64_t K = 0;
  for (int32_t a = b; a >= 0; a = t.b_parent[a])
    for (int32_t j = c.group_ptr_h[a]; j < c.group_ptr_h[a + 1]; ++j) K += c.sym[j].kr;
  return K;
}

// A farfield target is truncated exactly by Algorithm 5 when its sum-expression holds no
// H-pairs (S_H empty) and its stacked factor spans at most `cap` columns.
bool exact_eligible(const Ctx& c, int32_t b, int cap) {
  if (c.hptr[b + 1] != c.hptr[b]) return false;
  return std::min<int64_t>(c.m_of(b), term_columns(c, b)) <= cap;
}

// SVD of the low-rank sum S = sum_j L_j core_j R_j^T of targets with S_H empty
// (Algorithm 5), with the second QR taken of R R_L^T: Q = orth([L_1 core_1, ...]) (the
// range of S, by CGS2 in batches of PW stacked columns), Z = S^T Q (= R R_L^T up to the
// basis), QR of Z, SVD of its triangular factor, truncation at eps relative to ||S||_F
// (no estimated residual: E = 0).
void compress_chunk_exact(Ctx& c, Chunk& ch, FarOut& out) {
  const Tree& t = *c.t;
  hipStream_t s = c.s;
  const int nt = int(ch.blocks.size());
  const int cap = CAPMAX_CORE;
  const CParams cp{cap, PW, c.eps, c.opts.o.delta, 0.0};
  int64_t need = 0, kmax = 0;
  std::vector<int64_t> K(nt);
  for (int i = 0; i < nt; ++i) {
    const int32_t b = ch.blocks[i];
    K[i] = term_columns(c, b);
    kmax = std::max(kmax, K[i]);
    need += int64_t(c.m_of(b)) * (cap + PW) + int64_t(c.n_of(b)) * cap + 2 * cap * cap + cap;
  }
  DevBuf<double> ws{size_t(std::max<int64_t>(need, 1))};
  std::vector<CTarget> h(nt);
  int64_t o = 0;
  for (int i = 0; i < nt; ++i) {
    const int32_t b = ch.blocks[i];
    CTarget& T = h[i];
    std::memset(&T, 0, sizeof(T));
    T.m = c.m_of(b);
    T.n = c.n_of(b);
    T.row0 = t.c_begin[t.b_tau[b]];
    T.col0 = t.c_begin[t.b_sigma[b]];
    T.Y = ws.p + o;
    o += int64_t(T.m) * (cap + PW);
    T.Z = ws.p + o;
    o += int64_t(T.n) * cap;
    T.core = ws.p + o;
    o += 2 * cap * cap + cap;
    T.active = 1;
    T.block = b;
  }
  DevBuf<CTarget> dt(nt);
  dt.upload(h, s);
  const double t0 = now_seconds();
  for (int64_t c0 = 0; c0 < kmax; c0 += PW) {
    c.timer.begin(K_COMPRESS);
    launch_term_columns(dt.p, nt, c.tv, int(c0), PW, cap, s);
    launch_orth_append(dt.p, nt, cap, PW, cp, s);
    c.timer.end();
  }
  HM_CHECK_HIP(hipMemcpyAsync(h.data(), dt.p, sizeof(CTarget) * nt, hipMemcpyDeviceToHost, s));
  HM_CHECK_HIP(hipStreamSynchronize(s));
  const double t1 = now_seconds();
  c.st.t_sketch += t1 - t0;
  // Z = S^T Q
  int maxw = 0;
  for (const auto& T : h) maxw = std::max(maxw, T.r);
  std::vector<TDesc> td(nt);
  for (int j0 = 0; j0 < maxw; j0 += PW) {
    bool any = false;
    for (int i = 0; i < nt; ++i) {
      TDesc& d = td[i];
      std::memset(&d, 0, sizeof(d));
      const CTarget& T = h[i];
      if (j0 >= T.r) continue;
      d.w = std::min(PW, T.r - j0);
      d.trans = 1;
      d.X = T.Y + int64_t(j0) * T.m;
      d.ldx = T.m;
      d.Y = T.Z + int64_t(j0) * T.n;
      d.ldy = T.n;
      d.split = d.w;
      any = true;
    }
    if (any) run_pass(c, ch, td, true);
  }
  const double t2 = now_seconds();
  c.st.t_project += t2 - t1;
  int rmax = 1;
  for (auto& T : h) {
    T.rz = T.r;
    T.E2 = 0.0;
    T.done = 1;
    rmax = std::max(rmax, T.rz);
  }
  dt.upload(h, s);
  c.timer.begin(K_COMPRESS);
  launch_core(dt.p, nt, cp, s, rmax);
  c.timer.end();
  HM_CHECK_HIP(hipMemcpyAsync(h.data(), dt.p, sizeof(CTarget) * nt, hipMemcpyDeviceToHost, s));
  HM_CHECK_HIP(hipStreamSynchronize(s));
  out.blocks.clear();
  out.ranks.clear();
  out.done.clear();
  out.offs.clear();
  out.len = 0;
  for (int i = 0; i < nt; ++i) {
    CTarget& T = h[i];
    out.blocks.push_back(T.block);
    out.ranks.push_back(T.k);
    out.done.push_back(1);
    out.offs.push_back(out.len);
    T.out_off = out.len;
    out.len += int64_t(T.k) * (T.m + T.n);
    c.st.rank_hist[std::min(T.k, 64)]++;
    c.st.n_exact_lowrank++;
    if (T.svd_capped) c.st.n_svd_sweep_cap++;
    charge_far(c, ch, i, T.block, T.m, T.n, T.k);
  }
  out.buf.alloc(size_t(std::max<int64_t>(out.len, 1)));
  dt.upload(h, s);
  c.timer.begin(K_COMPRESS);
  launch_write_factors(dt.p, nt, cp, out.buf.p, s);
  c.timer.end();
  HM_CHECK_HIP(hipStreamSynchronize(s));
  c.st.t_core += now_seconds() - t2;
}

// ------------------------------------------------------------------ other schemes
// Per-target panels of the ACA, Lanczos and fixed-rank schemes.
struct IterPanels {
  DevBuf<double> ws;
  DevBuf<int32_t> used, state;
  DevBuf<ITarget> dt;
  std::vector<ITarget> h;
  std::vector<int32_t> hs;  // per target: state (or column count) read back after a step
};

void setup_iter(Ctx& c, Chunk& ch, IterPanels& P, int cap, int kfixed) {
  const Tree& t = *c.t;
  const int nt = int(ch.blocks.size());
  int64_t need = 0, needi = 0;
  for (int32_t b : ch.blocks) {
    const int64_t m = c.m_of(b), n = c.n_of(b);
    need += m * cap + n * (cap + 1) + 2 * (m + n) + 2 * int64_t(cap) * cap + 3 * cap;
    needi += m;
  }
  P.ws.alloc(size_t(std::max<int64_t>(need, 1)));
  P.used.alloc(size_t(std::max<int64_t>(needi, 1)));
  P.state.alloc(size_t(std::max(nt, 1)));
  P.h.assign(size_t(nt), ITarget{});
  P.hs.assign(size_t(nt), 0);
  int64_t o = 0, oi = 0;
  for (int i = 0; i < nt; ++i) {
    const int32_t b = ch.blocks[i];
    ITarget& T = P.h[i];
    std::memset(&T, 0, sizeof(T));
    T.m = c.m_of(b);
    T.n = c.n_of(b);
    T.row0 = t.c_begin[t.b_tau[b]];
    T.col0 = t.c_begin[t.b_sigma[b]];
    T.L = P.ws.p + o;
    o += int64_t(T.m) * cap;
    T.U = P.ws.p + o;
    o += int64_t(T.n) * (cap + 1);
    T.xf = P.ws.p + o;
    o += T.n;
    T.xt = P.ws.p + o;
    o += T.m;
    T.yf = P.ws.p + o;
    o += T.m;
    T.yt = P.ws.p + o;
    o += T.n;
    T.work = P.ws.p + o;
    o += 2 * int64_t(cap) * cap + 3 * cap;
    T.used = P.used.p + oi;
    oi += T.m;
    T.block = b;
    T.lim = std::min({T.m, T.n, cap, kfixed > 0 ? kfixed : cap});
  }
  P.dt.upload(P.h, c.s);
}

void fetch_iter(Ctx& c, IterPanels& P) {
  const double t0 = now_seconds();
  HM_CHECK_HIP(hipMemcpyAsync(P.h.data(), P.dt.p, sizeof(ITarget) * P.h.size(), hipMemcpyDeviceToHost, c.s));
  HM_CHECK_HIP(hipStreamSynchronize(c.s));
  c.st.t_host[3] += now_seconds() - t0;
}

void fetch_counts(Ctx& c, IterPanels& P) {
  const double t0 = now_seconds();
  HM_CHECK_HIP(hipMemcpyAsync(P.hs.data(), P.state.p, 4 * P.hs.size(), hipMemcpyDeviceToHost, c.s));
  HM_CHECK_HIP(hipStreamSynchronize(c.s));
  c.st.t_host[3] += now_seconds() - t0;
}

// Lays out the outputs of the chunk's targets (rank T.k each) and records them in `out`.
void layout_outputs(Ctx& c, Chunk& ch, IterPanels& P, FarOut& out) {
  out.blocks.clear();
  out.ranks.clear();
  out.done.clear();
  out.offs.clear();
  out.len = 0;
  for (size_t i = 0; i < P.h.size(); ++i) {
    ITarget& T = P.h[i];
    const bool ok = T.state != 2;
    if (!ok) c.st.n_not_converged++;
    if (T.svd_sweeps < 0) c.st.n_svd_sweep_cap++;
    out.blocks.push_back(T.block);
    out.ranks.push_back(T.k);
    out.done.push_back(uint8_t(ok ? 1 : 0));
    out.offs.push_back(out.len);
    T.out_off = out.len;
    out.len += int64_t(T.k) * (T.m + T.n);
    c.st.rank_hist[std::min(T.k, 64)]++;
    charge_far(c, ch, int(i), T.block, T.m, T.n, T.k);
  }
  out.buf.alloc(size_t(std::max<int64_t>(out.len, 1)));
  P.dt.upload(P.h, c.s);
}

// ACA (Algorithm 6) or Lanczos bidiagonalization (Algorithm 7) of the chunk's farfield
// targets: one transposed and one forward pass of width 1 per step for every target
// still running, the per-target vector work in between, then recompression.
void compress_chunk_iter(Ctx& c, Chunk& ch, FarOut& out) {
  const Tree& t = *c.t;
  hipStream_t s = c.s;
  const int nt = int(ch.blocks.size());
  const int cap = ISCHEME_CAP;
  const int kf = c.opts.o.k_fixed;
  const IParams ip{cap, kf > 0 ? 1 : 0, c.eps};
  const bool aca = c.opts.o.scheme == HMAT_SCHEME_ACA;
  IterPanels P;
  setup_iter(c, ch, P, cap, kf);
  const double t0 = now_seconds();
  for (int i = 0; i < nt; ++i) P.hs[i] = P.h[i].lim == 0 ? 1 : 0;
  if (aca) {
    launch_aca_init(P.dt.p, nt, s);
  } else {
    ensure_omega(c, 1);
    launch_gkl_init(P.dt.p, nt, c.omega.p, s);
  }
  std::vector<TDesc> td(nt);
  // one pass of width 1 over the running targets: forward yf = S xf, transposed yt = S^T xt
  auto vec_pass = [&](bool trans) {
    bool any = false;
    for (int i = 0; i < nt; ++i) {
      TDesc& d = td[i];
      std::memset(&d, 0, sizeof(d));
      if (P.hs[i] != 0) continue;
      const ITarget& T = P.h[i];
      d.w = 1;
      d.split = 1;
      d.trans = trans ? 1 : 0;
      d.X = trans ? T.xt : T.xf;
      d.ldx = trans ? T.m : T.n;
      d.Y = trans ? T.yt : T.yf;
      d.ldy = trans ? T.n : T.m;
      any = true;
    }
    if (any) run_pass(c, ch, td, trans);
  };
  for (int step = 0; step <= cap; ++step) {
    if (std::none_of(P.hs.begin(), P.hs.end(), [](int32_t v) { return v == 0; })) break;
    if (aca) {
      vec_pass(true);  // row e_i^T S of every running target
      c.timer.begin(K_COMPRESS);
      launch_aca_row(P.dt.p, nt, ip, s);
      c.timer.end();
      vec_pass(false);  // column S e_j
      c.timer.begin(K_COMPRESS);
      launch_aca_col(P.dt.p, nt, ip, P.state.p, s);
      c.timer.end();
    } else {
      vec_pass(false);  // S w_r
      c.timer.begin(K_COMPRESS);
      launch_gkl_fwd(P.dt.p, nt, ip, s);
      c.timer.end();
      vec_pass(true);  // S^T q_r
      c.timer.begin(K_COMPRESS);
      launch_gkl_bwd(P.dt.p, nt, ip, P.state.p, s);
      c.timer.end();
    }
    fetch_counts(c, P);
  }
  const double t1 = now_seconds();
  c.st.t_sketch += t1 - t0;
  c.timer.begin(K_COMPRESS);
  if (aca) launch_aca_core(P.dt.p, nt, ip, s);
  else launch_gkl_core(P.dt.p, nt, ip, s);
  c.timer.end();
  fetch_iter(c, P);
  int rmax = 1;
  for (const auto& T : P.h) {
    rmax = std::max(rmax, T.r);
    c.st.scheme_steps += T.r;
  }
  c.timer.begin(K_COMPRESS);
  launch_iter_svd(P.dt.p, nt, ip, rmax, s);
  c.timer.end();
  fetch_iter(c, P);
  for (int i = 0; i < nt; ++i)
    if (P.h[i].state == 0) P.h[i].state = 2;  // still running after the step cap
  layout_outputs(c, ch, P, out);
  c.timer.begin(K_COMPRESS);
  launch_iter_write(P.dt.p, nt, ip, out.buf.p, s);
  c.timer.end();
  HM_CHECK_HIP(hipStreamSynchronize(s));
  c.st.t_core += now_seconds() - t1;
  (void)t;
}

// Fixed-rank randomized scheme (Algorithm 9): L = orth(S Omega_k), q subspace iterations
// (U = orth(S^T L), L = orth(S U)), output L and R = S^T L.
void compress_chunk_fixed(Ctx& c, Chunk& ch, FarOut& out) {
  const Tree& t = *c.t;
  hipStream_t s = c.s;
  const int nt = int(ch.blocks.size());
  const int cap = ISCHEME_CAP;
  const int k = c.opts.o.k_fixed;
  IterPanels P;
  setup_iter(c, ch, P, cap, k);
  const double t0 = now_seconds();
  ensure_omega(c, k);
  std::vector<TDesc> td(nt);
  std::vector<int32_t> r(nt, k), rz(nt, 0);
  // passes over per-target column counts cnt[i], PW columns at a time
  auto passes = [&](bool trans, const std::vector<int32_t>& cnt, bool sketch) {
    int maxw = 0;
    for (int v : cnt) maxw = std::max(maxw, v);
    for (int j0 = 0; j0 < maxw; j0 += PW) {
      bool any = false;
      for (int i = 0; i < nt; ++i) {
        TDesc& d = td[i];
        std::memset(&d, 0, sizeof(d));
        if (j0 >= cnt[i]) continue;
        const ITarget& T = P.h[i];
        d.w = std::min(PW, cnt[i] - j0);
        d.split = d.w;
        d.trans = trans ? 1 : 0;
        if (sketch) {
          d.X = c.omega.p + int64_t(j0) * t.n + T.col0;
          d.ldx = int32_t(t.n);
        } else {
          d.X = trans ? T.L + int64_t(j0) * T.m : T.U + int64_t(j0) * T.n;
          d.ldx = trans ? T.m : T.n;
        }
        d.Y = trans ? T.U + int64_t(j0) * T.n : T.L + int64_t(j0) * T.m;
        d.ldy = trans ? T.n : T.m;
        any = true;
      }
      if (any) run_pass(c, ch, td, trans);
    }
  };
  auto orth = [&](int side, int cnt, std::vector<int32_t>& dst) {
    c.timer.begin(K_COMPRESS);
    launch_orth_cols(P.dt.p, nt, side, cnt, P.state.p, s);
    c.timer.end();
    fetch_counts(c, P);
    dst = P.hs;
  };
  passes(false, r, true);  // L = S Omega[:, :k]
  orth(0, k, r);
  for (int it = 0; it < c.opts.o.subspace_iters; ++it) {
    passes(true, r, false);  // U = S^T L
    orth(1, 0, rz);
    passes(false, rz, false);  // L = S U
    orth(0, 0, r);
  }
  const double t1 = now_seconds();
  c.st.t_sketch += t1 - t0;
  passes(true, r, false);  // R = S^T L
  c.st.t_project += now_seconds() - t1;
  const double t2 = now_seconds();
  fetch_iter(c, P);
  for (auto& T : P.h) {
    T.k = T.r;
    T.state = 1;
    c.st.scheme_steps += k;
  }
  layout_outputs(c, ch, P, out);
  c.timer.begin(K_COMPRESS);
  launch_copy_out(P.dt.p, nt, out.buf.p, s);
  c.timer.end();
  HM_CHECK_HIP(hipStreamSynchronize(s));
  c.st.t_core += now_seconds() - t2;
}

// Nearfield targets: S applied to the identity, PW columns at a time, straight into C.
void evaluate_chunk(Ctx& c, Chunk& ch, double* cpool, const std::vector<int64_t>& coff) {
  const int nt = int(ch.blocks.size());
  // direct kernel: terms and dense x dense pairs of the targets of at most NEAR_MAX x NEAR_MAX,
  // one work item per 64-row block (the kernel takes its column blocks in turn); its lists
  // were prepared and uploaded with the chunk
  const size_t nd = ch.dpos.size();
  c.st.n_near_direct += int64_t(nd);
  if (nd) {
    std::vector<int64_t> dco(nd);
    for (size_t k = 0; k < nd; ++k) {
      const int i = ch.dpos[k];
      dco[k] = coff[size_t(i)];
      c.st.kern_bytes[K_NEAR] += ch.dby[k];
      c.st.kern_flops[K_NEAR] += ch.dfl[k];
      c.charge(ch.blocks[size_t(i)], ch.dby[k], ch.dfl[k]);
    }
    ch.d_dco.upload(dco, c.s);
    c.timer.begin(K_NEAR);
    launch_near_direct(ch.d_ditems.p, int64_t(ch.ditems.size() / 2), ch.d_dblk.p, ch.d_dco.p, ch.d_dpptr.p,
                       ch.d_dpairs.p, c.tv, c.ma, c.mb, cpool, c.s);
    c.timer.end();
  }
  // identity panels, PW columns at a time: whole targets beyond NEAR_MAX, and the pairs
  // with a subdivided factor of direct targets (added to what the direct kernel wrote)
  const double tp0 = now_seconds();
  int maxn = 0;
  std::vector<uint8_t> panel(nt, 0);
  for (int i = 0; i < nt; ++i) {
    panel[i] = !ch.direct[i] || ch.info[i].hp_end > ch.info[i].hp_begin;
    if (panel[i]) maxn = std::max(maxn, c.n_of(ch.blocks[i]));
  }
  std::vector<TDesc> td(nt);
  for (int j0 = 0; j0 < maxn; j0 += PW) {
    for (int i = 0; i < nt; ++i) {
      TDesc& d = td[i];
      std::memset(&d, 0, sizeof(d));
      const int32_t b = ch.blocks[i];
      const int n = c.n_of(b), m = c.m_of(b);
      if (!panel[i] || j0 >= n) continue;
      d.w = std::min(PW, n - j0);
      d.trans = 0;
      d.xident = 1;
      d.xcol0 = j0;
      d.X = nullptr;
      d.Y = cpool + coff[i] + int64_t(j0) * m;
      d.ldy = m;
      d.split = d.w;
      d.accum = ch.direct[i];
    }
    run_pass(c, ch, td, false);
  }
  for (int i = 0; i < nt; ++i) {
    if (!panel[i]) continue;
    const double w = c.n_of(ch.blocks[i]);
    for (int k = 0; k < 4; ++k) {  // term coefficients of direct targets are zero
      const Coef& cf = ch.coef[k][0][i];
      c.charge(ch.blocks[i], cf.a + cf.b * w, cf.f * w);
    }
    for (const Coef* cf : {&ch.s1_leaf[i], &ch.s1_exp[i]})  // forward stage 1, counted per target
      c.charge(ch.blocks[i], cf->a + cf->b * w, cf->f * w);
  }
  HM_CHECK_HIP(hipStreamSynchronize(c.s));
  c.st.t_near_panels += now_seconds() - tp0;
}

}  // namespace

hmat_status multiply(HMat* A, HMat* B, double eps, const Opts& opts, HMat** Cout) {
  const double t_start = now_seconds();
  const AllocCounters alloc0 = alloc_counters();
  HM_REQUIRE(A->tree == B->tree, HMAT_ERR_TREE_MISMATCH, "A and B must be built on the same tree");
  Tree* t = A->tree;
  HM_REQUIRE(t->leaf_size <= 64, HMAT_ERR_ARG, "the product needs leaf_size <= 64");
  for (int32_t b : t->leaves)
    if (t->b_kind[b] == KIND_F)
      HM_REQUIRE(A->rank[b] <= 64 && B->rank[b] <= 64, HMAT_ERR_ARG, "input ranks above 64 are not supported");
  Ctx c;
  c.t = t;
  c.A = A;
  c.B = B;
  c.s = opts.stream();
  c.eps = eps;
  c.opts = opts;
  hipStream_t s = c.s;
  set_current_stream(s);
  t->ensure_device(s);

  // plan
  c.dfs = dfs_order(*t);
  build_kpref(A, c.dfs, c.da, s);
  build_kpref(B, c.dfs, c.db, s);
  build_leaf_recs(A, c.dfs, c.da, s);
  build_leaf_recs(B, c.dfs, c.db, s);
  c.lowp = opts.o.precision == HMAT_FP32_APPLY;
  if (c.lowp) {
    for (HMat* M : {A, B}) {
      std::lock_guard<std::mutex> lk(M->mu32);
      if (!M->pool32.p || M->pool32.n < size_t(std::max<int64_t>(M->pool_len, 1))) {
        M->pool32.alloc(size_t(std::max<int64_t>(M->pool_len, 1)));
        if (M->pool_len) launch_to_float(M->pool.p, M->pool32.p, M->pool_len, s);
        HM_CHECK_HIP(hipStreamSynchronize(s));
      }
    }
    c.register_pool(A->pool.p, A->pool_len, A->pool32.p);
    c.register_pool(B->pool.p, B->pool_len, B->pool32.p);
  }
  c.ma = c.da.view(A);
  c.mb = c.db.view(B);
  build_subsums(c, A, c.sa);
  build_subsums(c, B, c.sb);
  c.timer.on = opts.o.time_kernels != 0;
  c.timer.s = s;
  {
    const double t0 = now_seconds();
    symbolic(c);
    c.st.t_host[0] += now_seconds() - t0;
    c.st.n_terms = int64_t(c.sym.size());
    c.st.n_leaf_pairs = int64_t(c.hrho.size() / 3);
  }
  c.b_parent.upload(t->b_parent, s);
  c.b_dfs.upload(c.dfs.dfs_of_block, s);
  c.group_ptr.upload(c.group_ptr_h, s);
  c.hterms.swap(plan_arena().hterms);
  c.hterms.assign(c.sym.size(), Term{});
  c.tv = TreeView{t->dev->c_begin.p, t->dev->c_size.p, t->dev->c_parent.p, t->dev->leaf_clusters.p,
                  t->dev->b_tau.p, t->dev->b_sigma.p, t->dev->b_kind.p, c.b_parent.p, c.b_dfs.p,
                  t->dev->brow_ptr.p, t->dev->brow_blk.p, t->dev->bcol_ptr.p, t->dev->bcol_blk.p,
                  c.group_ptr.p, nullptr, t->dev->c_lc_begin.p};
  c.st.t_plan = now_seconds() - t_start;

  // memory of the data each term creates, and the level of the block it belongs to
  const int64_t nsym = int64_t(c.sym.size());
  std::vector<int64_t> tmem(nsym);
  for (int64_t i = 0; i < nsym; ++i) {
    const SymTerm& st = c.sym[i];
    tmem[i] = st.type == T_FF ? int64_t(st.kl) * st.kr
            : st.type == T_FH ? int64_t(st.kl) * c.n_of(st.child)
            : st.type == T_HF ? int64_t(st.kl) * c.m_of(st.child) : 0;
    tmem[i] *= 8;
  }
  // Subtree batches: terms of blocks deeper than level L0 live only while the targets
  // of their level-L0 subtree group are processed (the paper's recursion is depth
  // first; this is the same order at the granularity of a batch of subtrees).
  int64_t term_budget;
  {
    // terms of one subtree batch: at most 0.45 of the available memory (shared by the
    // products in flight; with float copies of the terms, which take half as much again,
    // two thirds of that) and at most 16 GiB of float64 terms (more batches cost little;
    // very large pools are slow to map and make the budget depend on what earlier products
    // left in the block cache)
    const size_t fb = dev_free_bytes() / size_t(std::max(1, opts.concurrency));
    const double share = c.lowp ? 0.45 * 2.0 / 3.0 : 0.45;
    term_budget = opts.o.workspace_limit > 0 ? 8 * opts.o.workspace_limit
                                             : std::min<int64_t>(int64_t(share * double(fb)), int64_t(16) << 30);
    if (c.lowp && opts.o.workspace_limit > 0) term_budget = term_budget / 3 * 2;
  }
  const int depth = t->depth;
  std::vector<int64_t> cum(depth + 2, 0);
  for (int64_t i = 0; i < nsym; ++i) cum[t->b_level[c.sym[i].child]] += tmem[i];
  for (int l = 1; l <= depth + 1; ++l) cum[l] += cum[l - 1];
  int L0 = depth;
  if (cum[depth] > term_budget) {
    L0 = 0;
    for (int l = 0; l <= depth; ++l)
      if (cum[l] <= term_budget / 4) L0 = l;
  }
  const int64_t nb = int64_t(t->b_tau.size());
  std::vector<int32_t> root0(nb, -1);  // level-L0 ancestor of blocks at levels >= L0
  for (int64_t b = 0; b < nb; ++b) {
    if (t->b_level[b] == L0) root0[b] = int32_t(b);
    else if (t->b_level[b] > L0) root0[b] = root0[t->b_parent[b]];
  }
  // group level-L0 blocks into batches by the memory of their subtrees' terms
  std::vector<int64_t> sub_mem(nb, 0);
  for (int64_t i = 0; i < nsym; ++i) {
    int32_t ch = c.sym[i].child;
    if (t->b_level[ch] > L0) sub_mem[root0[ch]] += tmem[i];
  }
  std::vector<int32_t> batch_of(nb, -1);
  int nbatch = 0;
  {
    int64_t used = 0;
    const int64_t room = std::max<int64_t>(term_budget - cum[std::min(L0, depth)], term_budget / 2);
    bool open = false;
    for (int64_t b = t->level_begin[L0]; b < t->level_begin[L0 + 1]; ++b) {
      if (sub_mem[b] == 0 && t->b_kind[b] != KIND_INNER) continue;
      if (open && used + sub_mem[b] > room) {
        ++nbatch;
        used = 0;
      }
      batch_of[b] = nbatch;
      used += sub_mem[b];
      open = true;
    }
    if (open) ++nbatch;
  }
  c.st.n_batches = nbatch + 1;

  // output matrix
  std::unique_ptr<HMat> C_owner(new HMat());  // freed if the product fails part-way
  HMat* C = C_owner.get();
  C->tree = t;
  tree_retain(t);
  C->rank.assign(nb, 0);
  C->off.assign(nb, -1);
  c.bflops.assign(nb, 0.0);
  const bool predict = opts.o.rank_mode == HMAT_RANK_PREDICT;
  const bool collect = !predict && opts.o.stats != nullptr;
  std::vector<int32_t> far_all, near_all;
  for (int32_t b : t->leaves) (t->b_kind[b] == KIND_F ? far_all : near_all).push_back(b);
  c.st.n_far = int64_t(far_all.size());
  c.st.n_near = int64_t(near_all.size());
  // Learned mode: one prediction per farfield target, made before the targets are put
  // into chunks. The prediction estimates the sketch width a target needs. A target is
  // widened only where the prediction is well into the first growth step: a chunk's
  // operator passes run as long as its widest target needs them, so a widened target that
  // did not need it costs its chunk a pass, while one that did saves only the growth
  // round's check and synchronisation (its extra pass is paid either way).
  std::vector<float> pred_of;  // per block
  const double widen_at = opts.o.b0 + 0.75 * opts.o.growth;
  if (predict && !far_all.empty()) {
    const double tq = now_seconds();
    std::vector<float> fe(far_all.size() * size_t(HMAT_N_FEATURES));
    {
      const size_t nthr = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
      std::vector<std::thread> th;
      for (size_t w = 0; w < nthr; ++w)
        th.emplace_back([&, w] {
          for (size_t i = w; i < far_all.size(); i += nthr)
            target_features(c, far_all[i], &fe[i * HMAT_N_FEATURES]);
        });
      for (auto& x : th) x.join();
    }
    std::vector<float> pv;
    predict_ranks(opts.o.rank_model, fe, pv, s);
    pred_of.assign(size_t(nb), std::numeric_limits<float>::quiet_NaN());
    for (size_t i = 0; i < far_all.size(); ++i) pred_of[far_all[i]] = pv[i];
    c.st.t_predict += now_seconds() - tq;
  }
  auto predicted_wide = [&](int32_t b) {
    const float pv = pred_of[b];
    return std::isfinite(pv) && double(pv) > widen_at;
  };
  int64_t near_len = 0;
  std::vector<int64_t> near_off(nb, -1);
  for (int32_t b : near_all) {
    near_off[b] = near_len;
    near_len += int64_t(c.m_of(b)) * c.n_of(b);
  }
  DevBuf<double> near_buf(size_t(std::max<int64_t>(near_len, 1)));
  // device workspace of one chunk of targets: larger chunks mean fewer, fuller launches
  // (measured: 3 GiB 6.62 s, 8 GiB 6.37 s, 16 GiB 6.31 s per 262144-point product); three
  // chunks can be alive at once (one running, two built ahead), so at most 1/16 of the
  // available memory each, shared by the products in flight (the cache would otherwise
  // overflow and free blocks, and a device free waits for all streams)
  const int64_t budget = opts.o.workspace_limit > 0
                             ? opts.o.workspace_limit
                             : std::min<int64_t>(int64_t(16) << 30,
                                                 int64_t(dev_free_bytes() / (16 * std::max(1, opts.concurrency))));
  // ACA, Lanczos and the fixed-rank scheme apply S to per-target vectors
  const bool own_inputs = opts.o.scheme != HMAT_SCHEME_RANDOMIZED || opts.o.k_fixed > 0;
  const int cap_est = own_inputs ? ISCHEME_CAP + 4 : std::min(64, opts.o.b0 + opts.o.max_growth * opts.o.probes);
  std::vector<FarOut> outs;

  // Targets are processed in chunks; the host work lists of chunk k+1 are built on a
  // worker thread while the device runs chunk k.
  auto partition = [&](const std::vector<int32_t>& list, bool far) {
    std::vector<std::vector<int32_t>> parts;
    for (size_t i = 0; i < list.size();) {
      std::vector<int32_t> blk;
      int64_t used = 0;
      while (i < list.size()) {
        int64_t cst = target_cost(c, list[i], far, opts, cap_est);
        if (!blk.empty() && used + cst > budget) break;
        used += cst;
        blk.push_back(list[i++]);
      }
      parts.push_back(std::move(blk));
    }
    return parts;
  };
  std::vector<std::unique_ptr<Chunk>> spare_chunks;  // finished chunks, reused by later ones
  // A product alone on the device builds the next chunk on a worker thread, which uploads
  // it on its own non-blocking stream (its copies overlap the work on the product's stream
  // even when that is the null stream), and prepares the next subtree batch on another.
  // Products in flight next to others (batched calls) do both on their own thread and
  // stream: the other products keep the device busy meanwhile, and each product then uses
  // one host thread and one stream.
  const bool overlap = opts.concurrency <= 1;
  struct UploadStream {
    hipStream_t s = nullptr;
    explicit UploadStream(bool create) {
      if (create) HM_CHECK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    }
    ~UploadStream() {
      if (!s) return;
      (void)hipStreamSynchronize(s);
      forget_stream(s);
      (void)hipStreamDestroy(s);
    }
  } s_up(overlap);
  struct Job {
    bool far;
    std::vector<int32_t> blocks;
    bool exact = false;  // farfield targets truncated by Algorithm 5
  };
  // chunk partition of a batch's targets; reads only the plan, so it may run on another
  // thread (its time goes to `secs`, not to the shared statistics)
  auto make_jobs_t = [&](const std::vector<int32_t>& near, const std::vector<int32_t>& far, double* secs) {
    std::vector<Job> jobs;
    const double tp = now_seconds();
    for (auto& p : partition(near, false)) jobs.push_back(Job{false, std::move(p)});
    std::vector<int32_t> far_rest, far_exact;
    if (opts.o.exact_lowrank) {
      for (int32_t b : far) (exact_eligible(c, b, CAPMAX_CORE) ? far_exact : far_rest).push_back(b);
    }
    const std::vector<int32_t>& rest = opts.o.exact_lowrank ? far_rest : far;
    for (auto& p : partition(far_exact, true)) jobs.push_back(Job{true, std::move(p), true});
    for (auto& p : partition(rest, true)) jobs.push_back(Job{true, std::move(p)});
    *secs += now_seconds() - tp;
    return jobs;
  };
  auto make_jobs = [&](const std::vector<int32_t>& near, const std::vector<int32_t>& far) {
    double secs = 0;
    std::vector<Job> jobs = make_jobs_t(near, far, &secs);
    c.st.t_host[2] += secs;
    return jobs;
  };
  // The next subtree batch's jobs: partitioned on a worker thread while the current batch
  // runs, and collected when the chunk pipeline first reaches them.
  struct NextJobs {
    std::future<std::vector<Job>> f;
    std::vector<Job> v;
    double secs = 0;
    bool ready = true;
    const std::vector<Job>* get() {
      if (!ready) {
        v = f.get();
        ready = true;
      }
      return &v;
    }
  };
  // the worker builds the next chunk's work lists and uploads them on its own stream
  // while the device runs the current chunk
  auto build = [&c, &s_up](std::unique_ptr<Chunk> ch, bool features) {
    set_current_stream(s_up.s);
    // a recycled chunk's buffers may still be read by its last kernels on the product's
    // stream: uploads into them, and frees (whose events are recorded on s_up), come after
    if (ch->pending) HM_CHECK_HIP(hipStreamWaitEvent(s_up.s, ch->done, 0));
    ch->pending = false;
    build_chunk(c, *ch, features);
    upload_chunk(*ch, s_up.s);  // each upload waits for its copy on s_up
    return ch;
  };
  auto build_here = [&c, s](std::unique_ptr<Chunk> ch, bool features) {
    build_chunk(c, *ch, features);
    upload_chunk(*ch, s);  // on the product's stream: after the recycled chunk's kernels
    ch->pending = false;
    return ch;
  };
  // the chunks being built, in job order; declared after s_up so that pending builds end
  // before s_up does. Two builds run ahead of the device: one build at a time fell behind
  // it on the heavier chunks (the first nearfield chunk of a subtree batch among them).
  std::deque<std::future<std::unique_ptr<Chunk>>> pending;
  const size_t build_depth = overlap ? 2 : 1;
  size_t carried = 0;  // jobs of the next process_targets call already in `pending`
  auto launch_build = [&](const Job& job) {
    std::unique_ptr<Chunk> ch;
    if (!spare_chunks.empty()) {  // reuse: host arrays keep their capacity
      ch = std::move(spare_chunks.back());
      spare_chunks.pop_back();
      ch->reset();
    } else {
      ch = std::make_unique<Chunk>();
    }
    ch->blocks = job.blocks;
    ch->near = !job.far;
    ch->share_s1 = !(job.far && own_inputs);
    const bool features = job.far && collect;
    if (overlap) {
      pending.push_back(std::async(std::launch::async, build, std::move(ch), features));
    } else {
      std::promise<std::unique_ptr<Chunk>> ready;
      ready.set_value(build_here(std::move(ch), features));
      pending.push_back(ready.get_future());
    }
  };
  // Runs the chunks of `jobs`, keeping `build_depth` chunks in build ahead of the one running.
  // With `then` (the jobs of the next call), the first chunks of the next call are built
  // while the last ones of this call run; the next call finds them in `pending`. Building
  // reads only the plan, so it may overlap the next subtree batch's term creation.
  auto process_targets = [&](const std::vector<Job>& jobs, NextJobs* then) {
    size_t launched = std::min(carried, jobs.size()), then_launched = 0;
    carried = 0;
    auto top_up = [&]() {
      while (pending.size() < build_depth) {
        if (launched < jobs.size()) {
          launch_build(jobs[launched++]);
          continue;
        }
        const std::vector<Job>* tj = then ? then->get() : nullptr;
        if (tj && then_launched < tj->size()) launch_build((*tj)[then_launched++]);
        else break;
      }
    };
    top_up();
    for (size_t k = 0; k < jobs.size(); ++k) {
      const double th = now_seconds();
      std::unique_ptr<Chunk> chp = pending.front().get();
      pending.pop_front();
      top_up();
      Chunk& ch = *chp;
      c.st.t_host[2] += now_seconds() - th;
      if (!jobs[k].far) {
        double tn = now_seconds();
        std::vector<int64_t> coff;
        for (int32_t b : ch.blocks) coff.push_back(near_off[b]);
        evaluate_chunk(c, ch, near_buf.p, coff);
        c.st.t_near += now_seconds() - tn;
      } else {
        std::vector<int32_t> w0(ch.blocks.size(), opts.o.b0);
        if (predict) {
          // learned initial widths (the residual check still grows the sketch where the
          // prediction is too small)
          for (size_t i = 0; i < w0.size(); ++i) {
            const int mn = std::min(c.m_of(ch.blocks[i]), c.n_of(ch.blocks[i]));
            const double pv = double(pred_of[ch.blocks[i]]);
            const int g = opts.o.probes;
            // a prediction below three quarters of the first growth step keeps the plain
            // initial width (a regression trained mostly on blocks of that width scatters
            // around it); above, the width is the prediction plus p_l
            int w = !predicted_wide(ch.blocks[i])
                        ? opts.o.b0
                        : int(std::clamp(std::ceil(pv) + opts.o.p_l, 1.0, double(64 - g)));
            // operator passes run PW columns at a time: widen the sketch as far as it
            // costs no extra pass of the sketch (w + g columns) or of the projection (w)
            const int up_s = (w + g + PW - 1) / PW * PW - g, up_p = (w + PW - 1) / PW * PW;
            w = std::min({up_s, up_p, 64 - g});
            w0[i] = int32_t(std::max(1, std::min(w, mn)));
          }
        }
        outs.emplace_back();
        if (jobs[k].exact) compress_chunk_exact(c, ch, outs.back());
        else if (opts.o.scheme != HMAT_SCHEME_RANDOMIZED) compress_chunk_iter(c, ch, outs.back());
        else if (opts.o.k_fixed > 0) compress_chunk_fixed(c, ch, outs.back());
        else compress_chunk(c, ch, w0, outs.back());
        if (collect) {
          const FarOut& fo = outs.back();
          C->features.feats.insert(C->features.feats.end(), ch.feats.begin(), ch.feats.end());
          for (int32_t k : fo.ranks) C->features.ranks.push_back(float(k));
          for (size_t j = 0; j < fo.ranks.size(); ++j)
            C->features.widths.push_back(float(j < fo.widths.size() ? fo.widths[j] : fo.ranks[j]));
        }
      }
      chp->mark_done(s);
      spare_chunks.push_back(std::move(chp));
    }
    carried = then_launched;
  };

  // global terms and targets (levels <= L0)
  std::vector<int32_t> gterms;
  for (int64_t i = 0; i < nsym; ++i)
    if (t->b_level[c.sym[i].child] <= L0) gterms.push_back(int32_t(i));
  DevBuf<double> global_pool;
  // The subtree batches' setup (their term and target lists, the batch pool, batch 0's
  // preparation and chunk partition) reads only the plan and touches only batch 0's terms:
  // it runs on a worker thread while the global terms and targets run, and the global
  // targets' chunk pipeline builds batch 0's first chunks.
  const bool batches = L0 < depth;
  std::vector<std::vector<int32_t>> bterms, bnear, bfar;
  DevBuf<double> batch_pool;
  // the host part of batch k + 1 (layout, lists, descriptors) is prepared on a worker
  // thread while batch k's targets run; its creation kernels start once batch k is done,
  // because both batches use the same pool
  CreatePrep preps[2];
  auto prep_batch = [&](int k) {
    const int64_t pos = layout_terms(c, bterms[k]);
    prepare_terms(c, bterms[k], batch_pool.p, pos, preps[k & 1]);
    // the descriptors go up on the upload stream, so that publishing them is one
    // device-side scatter (the previous use of these buffers, batch k - 2's scatter,
    // completed before batch k - 1's targets started)
    if (s_up.s) {
      set_current_stream(s_up.s);
      stage_terms(c, bterms[k], preps[k & 1], s_up.s);
      set_current_stream(s);  // the calling thread may be the product's own
    }
  };
  double setup_alloc_s = 0, setup_jobs_s = 0;  // written by the setup, read after it
  auto batch_setup = [&]() {
    set_current_stream(s);
    bterms.assign(size_t(nbatch), {});
    bnear.assign(size_t(nbatch), {});
    bfar.assign(size_t(nbatch), {});
    for (int64_t i = 0; i < nsym; ++i) {
      int32_t ch = c.sym[i].child;
      if (t->b_level[ch] > L0) bterms[batch_of[root0[ch]]].push_back(int32_t(i));
    }
    for (int32_t b : near_all)
      if (t->b_level[b] > L0) bnear[batch_of[root0[b]]].push_back(b);
    for (int32_t b : far_all)
      if (t->b_level[b] > L0) bfar[batch_of[root0[b]]].push_back(b);
    // one pool, sized for the largest batch, serves every batch in turn
    int64_t maxpool = 1;
    for (int k = 0; k < nbatch; ++k) {
      int64_t sz = 0;
      for (int32_t i : bterms[k]) sz += tmem[i] / 8;
      maxpool = std::max(maxpool, sz);
    }
    const double ta = now_seconds();
    batch_pool.alloc(size_t(maxpool));
    // float copies of the batches' terms: one pool of the largest batch's size, so that it
    // is not reallocated as the batches grow
    if (c.lowp && c.bpool32.n < size_t(maxpool)) c.bpool32.alloc(size_t(maxpool));
    setup_alloc_s = now_seconds() - ta;
    prep_batch(0);
    return make_jobs_t(bnear[0], bfar[0], &setup_jobs_s);
  };
  NextJobs jobs0;
  if (batches) {
    if (overlap) {
      jobs0.ready = false;
      jobs0.f = std::async(std::launch::async, batch_setup);
    } else {
      jobs0.v = batch_setup();
    }
  }
  {
    double tc = now_seconds();
    CreatePrep gprep;
    create_terms(c, gterms, global_pool, c.gpool32, gprep);
    publish_terms(c, gterms);
    c.tv.terms = c.terms.p;
    c.st.t_restrict += now_seconds() - tc;
  }
  {
    std::vector<int32_t> nf, ff;
    for (int32_t b : near_all)
      if (t->b_level[b] <= L0) nf.push_back(b);
    for (int32_t b : far_all)
      if (t->b_level[b] <= L0) ff.push_back(b);
    process_targets(make_jobs(nf, ff), batches && overlap ? &jobs0 : nullptr);
  }
  // batches of deeper subtrees
  if (batches) {
    std::vector<Job> jobs_cur = std::move(*jobs0.get());
    c.st.t_host[4] += setup_alloc_s;
    c.st.t_host[2] += setup_jobs_s;
    NextJobs jobs_next;
    std::future<void> next_prep;
    for (int k = 0; k < nbatch; ++k) {
      double tc = now_seconds();
      if (next_prep.valid()) next_prep.get();
      execute_terms(c, preps[k & 1], batch_pool.p, c.bpool32);
      publish_terms(c, bterms[k], &preps[k & 1]);
      c.tv.terms = c.terms.p;
      if (k + 1 < nbatch) {
        if (overlap) next_prep = std::async(std::launch::async, prep_batch, k + 1);
        else prep_batch(k + 1);
      }
      c.st.t_restrict += now_seconds() - tc;
      jobs_next.v.clear();
      jobs_next.secs = 0;
      jobs_next.ready = true;
      if (k + 1 < nbatch) {
        if (overlap) {
          jobs_next.ready = false;
          jobs_next.f = std::async(std::launch::async, make_jobs_t, std::cref(bnear[k + 1]), std::cref(bfar[k + 1]),
                                   &jobs_next.secs);
        } else {
          jobs_next.v = make_jobs_t(bnear[k + 1], bfar[k + 1], &jobs_next.secs);
        }
      }
      process_targets(jobs_cur, overlap ? &jobs_next : nullptr);
      jobs_cur = std::move(*jobs_next.get());
      c.st.t_host[2] += jobs_next.secs;
    }
    batch_pool.release();  // before C's pool is allocated
  }

  // assemble C's pool: nearfield blocks, then farfield chunks
  int64_t total = near_len;
  std::vector<int64_t> base;
  for (auto& o : outs) {
    base.push_back(total);
    total += o.len;
  }
  C->pool_len = total;
  C->pool.alloc(size_t(std::max<int64_t>(total, 1)));
  if (near_len)
    HM_CHECK_HIP(hipMemcpyAsync(C->pool.p, near_buf.p, 8 * near_len, hipMemcpyDeviceToDevice, s));
  for (int32_t b : near_all) C->off[b] = near_off[b];
  for (size_t k = 0; k < outs.size(); ++k) {
    auto& o = outs[k];
    if (o.len) HM_CHECK_HIP(hipMemcpyAsync(C->pool.p + base[k], o.buf.p, 8 * o.len, hipMemcpyDeviceToDevice, s));
    for (size_t j = 0; j < o.blocks.size(); ++j) {
      C->rank[o.blocks[j]] = o.ranks[j];
      C->off[o.blocks[j]] = base[k] + o.offs[j];
      if (!o.done[j]) {
        if (C->notconv.empty()) C->notconv.assign(nb, 0);
        C->notconv[o.blocks[j]] = 1;
      }
    }
  }
  C->upload_meta(s);
  HM_CHECK_HIP(hipStreamSynchronize(s));
  c.timer.resolve(c.st);
  c.st.flops_alg = c.alg_flops;
  c.st.bytes_alg = c.alg_bytes;
  c.st.t_total = now_seconds() - t_start;
  {
    const AllocCounters a1 = alloc_counters();
    c.st.t_alloc = a1.seconds - alloc0.seconds;
    c.st.n_malloc = a1.mallocs - alloc0.mallocs;
    c.st.n_cache_release = a1.releases - alloc0.releases;
  }
  if (opts.o.stats) *opts.o.stats = c.st;
  C->block_flops.swap(c.bflops);
  *Cout = C_owner.release();
  if (c.st.n_not_converged > 0) {
    set_last_error(std::to_string(c.st.n_not_converged) + " farfield blocks exhausted the growth budget");
    return HMAT_ERR_NOT_CONVERGED;
  }
  return HMAT_OK;
}

// ------------------------------------------------------------------ batched products
// Independent products run concurrently, one host thread and one HIP stream per
// product in flight, so that small products (whose levels are too narrow to fill
// 256 CUs) overlap. The number in flight is autotuned per size class.
namespace {
std::mutex g_tune_mu;
std::map<int, int> g_tuned_streams;  // size class (rounded mean log2 n) -> streams

void add_stats(hmat_stats& a, const hmat_stats& b) {
  a.t_plan += b.t_plan;
  a.t_restrict += b.t_restrict;
  a.t_sketch += b.t_sketch;
  a.t_project += b.t_project;
  a.t_core += b.t_core;
  a.t_near += b.t_near;
  a.t_predict += b.t_predict;
  a.flops_alg += b.flops_alg;
  a.bytes_alg += b.bytes_alg;
  a.n_far += b.n_far;
  a.n_near += b.n_near;
  a.n_growth_rounds += b.n_growth_rounds;
  a.n_grown_blocks += b.n_grown_blocks;
  a.n_not_converged += b.n_not_converged;
  a.n_fallback += b.n_fallback;
  a.sketch_columns += b.sketch_columns;
  a.peak_bytes = std::max(a.peak_bytes, b.peak_bytes);
  a.n_batches += b.n_batches;
  for (int k = 0; k < 65; ++k) a.rank_hist[k] += b.rank_hist[k];
  for (int k = 0; k < 8; ++k) {
    a.kern_launches[k] += b.kern_launches[k];
    a.kern_time[k] += b.kern_time[k];
    a.kern_bytes[k] += b.kern_bytes[k];
    a.kern_flops[k] += b.kern_flops[k];
    a.t_host[k] += b.t_host[k];
  }
  a.t_alloc += b.t_alloc;
  a.n_malloc += b.n_malloc;
  a.n_cache_release += b.n_cache_release;
  a.target_passes += b.target_passes;
  a.n_near_direct += b.n_near_direct;
  a.n_terms += b.n_terms;
  a.n_leaf_pairs += b.n_leaf_pairs;
  a.t_near_panels += b.t_near_panels;
  a.scheme_steps += b.scheme_steps;
  a.n_exact_lowrank += b.n_exact_lowrank;
  a.n_svd_sweep_cap += b.n_svd_sweep_cap;
  a.t_growth += b.t_growth;
  a.n_passes += b.n_passes;
  a.n_sparse_passes += b.n_sparse_passes;
}
}  // namespace

hmat_status multiply_batched(HMat* const* A, HMat* const* B, int32_t count, double eps, const Opts& opts,
                             HMat** C, int32_t* status) {
  const double t0 = now_seconds();
  int dev = 0;
  HM_CHECK_HIP(hipGetDevice(&dev));
  for (int32_t i = 0; i < count; ++i) {
    HM_REQUIRE(A[i] && B[i], HMAT_ERR_ARG, "NULL H-matrix in batch");
    C[i] = nullptr;
  }
  std::vector<hmat_stats> pst(size_t(std::max(count, 1)));
  std::vector<hmat_status> pstat(size_t(std::max(count, 1)), HMAT_OK);
  std::vector<std::string> perr(size_t(std::max(count, 1)));
  // products idx[lo, hi) on S streams; returns the wall time
  std::vector<int32_t> idx(size_t(std::max(count, 1)));
  for (int32_t i = 0; i < count; ++i) idx[i] = i;
  auto run_range = [&](int32_t lo, int32_t hi, int S) {
    std::atomic<int32_t> next{lo};
    std::vector<std::thread> th;
    const double ts = now_seconds();
    for (int w = 0; w < S; ++w)
      th.emplace_back([&]() {
        hipStream_t s = nullptr;
        if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
          (void)hipGetLastError();
          s = nullptr;
        }
        for (;;) {
          const int32_t k = next.fetch_add(1);
          if (k >= hi) break;
          const int32_t i = idx[k];
          if (!s) {
            pstat[i] = HMAT_ERR_DEVICE;
            perr[i] = "stream creation failed";
            continue;
          }
          Opts o = opts;
          o.o.stream = s;
          o.o.stats = &pst[i];
          o.concurrency = S;
          try {
            pstat[i] = multiply(A[i], B[i], eps, o, &C[i]);
            if (pstat[i] != HMAT_OK) perr[i] = "product " + std::to_string(i) + ": " + hmat_last_error();
          } catch (const Error& e) {
            pstat[i] = e.code;
            perr[i] = "product " + std::to_string(i) + ": " + e.what();
          } catch (const std::exception& e) {
            pstat[i] = HMAT_ERR_INTERNAL;
            perr[i] = "product " + std::to_string(i) + ": " + e.what();
          }
        }
        if (s) {
          (void)hipStreamSynchronize(s);
          forget_stream(s);
          (void)hipStreamDestroy(s);
        }
      });
    for (auto& x : th) x.join();
    return now_seconds() - ts;
  };
  int S = opts.o.streams;
  int32_t done = 0;
  if (count > 0 && S <= 0) {
    double lg = 0;
    for (int32_t i = 0; i < count; ++i) lg += std::log2(double(std::max<int64_t>(A[i]->tree->n, 2)));
    const int cls = int(std::lround(lg / count));
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tuned_streams.find(cls);
      if (it != g_tuned_streams.end()) S = it->second;
    }
    if (S <= 0) {
      // trials: 2 x S products each with S = 1, 2, 4; the best rate runs the rest
      double best = -1.0;
      int best_s = 1;
      bool complete = true;
      for (int cand : {1, 2, 4}) {
        const int32_t take = std::min<int32_t>(2 * cand, count - done);
        if (take < cand) {
          complete = false;
          break;
        }
        const double sec = run_range(done, done + take, cand);
        double fl = 0;
        for (int32_t i = done; i < done + take; ++i) fl += pst[i].flops_alg;
        const double rate = fl / std::max(sec, 1e-9);
        if (rate > best) best = rate, best_s = cand;
        done += take;
      }
      S = best_s;
      if (complete) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned_streams[cls] = S;
      }
    }
  }
  if (S <= 0) S = 1;
  if (done < count) run_range(done, count, std::min<int>(S, count - done));
  // products that ran out of device memory next to others are run again alone
  {
    int32_t nre = 0;
    for (int32_t i = 0; i < count; ++i)
      if (pstat[i] == HMAT_ERR_OOM) {
        if (C[i]) hmat_release(C[i]);
        C[i] = nullptr;
        pst[i] = hmat_stats{};
        perr[i].clear();
        idx[nre++] = i;
      }
    if (nre) run_range(0, nre, 1);
  }
  hmat_status worst = HMAT_OK;
  std::string first_err;
  hmat_stats tot{};
  for (int32_t i = 0; i < count; ++i) {
    if (status) status[i] = pstat[i];
    if (pstat[i] != HMAT_OK && worst == HMAT_OK) {
      worst = pstat[i];
      first_err = perr[i];
    }
    add_stats(tot, pst[i]);
  }
  tot.t_total = now_seconds() - t0;
  tot.streams_used = S;
  if (opts.o.stats) *opts.o.stats = tot;
  set_last_error(first_err);
  return worst;
}

}  // namespace hm
