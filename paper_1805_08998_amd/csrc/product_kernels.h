// Device-side data of the product: low-rank terms of the sum-expressions,
// subtree product tasks, per-target pass descriptors and work items.
#pragma once

#include <cstdint>

namespace hm {

constexpr int PW = 16;  // columns per apply pass (wider passes are split)
constexpr int NEAR_TERM_MAX = 64;  // largest term width (kl, kr) of a target of the direct nearfield kernel

// One low-rank term of a sum-expression, L * core * R^T (Def. 3.1), stored
// through views into the factor pools. Restriction to a sub-block (Algorithm 3)
// is an index shift: row position p of the target maps to panel row p - lrow0.
// T is the storage type of the panels (double, or float for the fp32 copies).
template <class T>
struct TermT {
  const T* L;     // element (i, c) at L[i + c * ldl]
  const T* R;     // rtrans == 0: (j, c) at R[j + c * ldr]; rtrans == 1: at R[c + j * ldr]
  const T* core;  // kl x kr column-major (ld kl), or null when kl == kr and the core is I
  int32_t ldl, ldr;
  int32_t lrow0, rrow0;
  int32_t kl, kr;
  int32_t rtrans, pad;
};
using Term = TermT<double>;
using Term32 = TermT<float>;

// A leaf block of one matrix as seen from a block row (or column) list: one 32-byte
// record instead of a chain of dependent index loads.
struct LeafRec {
  int64_t off;     // element offset of the leaf's data in the pool
  int32_t o0, on;  // position and size of the other cluster (sigma in a row list, tau in a column list)
  int32_t k;       // farfield rank, -1 for a nearfield (dense) leaf
  int32_t m, n;    // rows and columns of the leaf
  int32_t kp;      // rank prefix of the leaf in depth-first order (kpref[dfs]): its leaf products'
                   // offset in a subtree task's workspace, without a lookup
};
// The same, indexed by depth-first leaf index.
struct DfsRec {
  int64_t off;
  int32_t r0, c0;  // first row and column position
  int32_t m, n;
  int32_t k;       // farfield rank, -1 for nearfield
  int32_t pad;
};

struct MatView {
  const double* pool;
  const int32_t* rank;   // per block
  const int64_t* off;    // per block, element offset of the leaf data in pool
  const int64_t* kpref;  // per depth-first leaf index: prefix sum of farfield ranks
  const float* pool32;   // float copy of pool (mixed precision), else null
  const LeafRec* row_rec;  // aligned with the tree's block-row lists (brow_blk)
  const LeafRec* col_rec;  // aligned with the block-column lists (bcol_blk)
  const DfsRec* dfs_rec;   // per depth-first leaf index
};

struct TreeView {
  const int32_t* c_begin;
  const int32_t* c_size;
  const int32_t* c_parent;
  const int32_t* leaf_clusters;
  const int32_t* b_tau;
  const int32_t* b_sigma;
  const int32_t* b_kind;
  const int32_t* b_parent;
  const int32_t* b_dfs;  // depth-first leaf index of a leaf block
  const int32_t* brow_ptr;
  const int32_t* brow_blk;
  const int32_t* bcol_ptr;
  const int32_t* bcol_blk;
  const int32_t* group_ptr;  // terms created at each block
  const Term* terms;
  const int32_t* c_lc_begin;  // first index into leaf_clusters of each cluster
  const Term32* terms32;      // the same terms over the float panel copies (mixed precision)
};

// Storage-type views: the kernels are instantiated for double panels and for
// their float copies; arithmetic is float64 in both.
template <class T> __host__ __device__ inline const T* mat_pool(const MatView& m);
template <> __host__ __device__ inline const double* mat_pool<double>(const MatView& m) { return m.pool; }
template <> __host__ __device__ inline const float* mat_pool<float>(const MatView& m) { return m.pool32; }
template <class T> __host__ __device__ inline const TermT<T>* tree_terms(const TreeView& v);
template <> __host__ __device__ inline const Term* tree_terms<double>(const TreeView& v) { return v.terms; }
template <> __host__ __device__ inline const Term32* tree_terms<float>(const TreeView& v) { return v.terms32; }

// Pass descriptor of one target: the target's operator is applied to X
// (forward: S X with X rows = sigma, output rows = tau; transposed: S^T X with
// X rows = tau, output rows = sigma). w == 0 marks an inactive target.
struct TDesc {
  const double* X;
  double* Y;
  int32_t ldx, ldy;
  int32_t w;
  int32_t split, gap;  // output column j goes to j (j < split) or j + gap
  int32_t trans;
  int32_t xident;      // X is the identity restricted to columns [xcol0, xcol0 + w)
  int32_t xcol0;
  int32_t accum;       // 1: Y += the pair results only (the terms were evaluated elsewhere)
};

struct TInfo {
  int32_t block;
  int32_t hp_begin, hp_end;  // H-pairs of the target
  int32_t pad;
  int64_t vbase;             // first slot of the target's term results
};

// Product of a subtree of A or B with a panel: trans == 0: Y[tau_q] = M[q] X[sigma_q];
// trans == 1: Y[sigma_q] = M[q]^T X[tau_q]. When t >= 0 the width and, if X is
// null, the input come from the target's pass descriptor.
struct Task {
  const double* X;
  double* Y;
  int32_t ldx, ldy;
  int32_t mat;  // 0 = A, 1 = B
  int32_t q;
  int32_t trans;
  int32_t t;
  int32_t w;    // fixed width when t < 0
  int32_t lo;   // first depth-first leaf index of subtree(q)
  int64_t tws;  // workspace of the leaf products R^T X (or L^T X)
};

struct TermItem {
  int32_t t, term;
  int64_t voff;
};

struct LeafItem {
  int32_t task, block;
};

struct RowItem {  // output rows: leaf cluster lc (index into leaf_clusters), 64-row chunk
  int32_t owner;  // task or target
  int32_t lc;
  int32_t chunk;
  int32_t pad;
};

struct HPair {
  double* temp2;  // output of the second stage (rows of the target's output cluster, ld = its size)
};

}  // namespace hm
