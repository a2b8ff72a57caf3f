// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hmat.h"

namespace hm {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  hmat_status code;
  Error(hmat_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define HM_CHECK_HIP(expr)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::hm::Error(HMAT_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_) + \
                                             " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

#define HM_REQUIRE(cond, code, msg)                                \
  do {                                                             \
    if (!(cond)) throw ::hm::Error((code), std::string(msg));      \
  } while (0)

// ---------------------------------------------------------------- device memory
void* dev_alloc(size_t bytes);
void dev_free(void* p);
// stream on which freed blocks may still be in use (set by every entry point that launches work)
void set_current_stream(hipStream_t s);
// Before destroying a stream the library created: marks the cached blocks freed on it
// as idle (the stream must have been synchronized).
void forget_stream(hipStream_t s);
struct AllocCounters {
  double seconds = 0;  // in hipMalloc / hipFree
  int64_t mallocs = 0, releases = 0;
};
AllocCounters alloc_counters();
// device memory available to the library: free memory plus blocks held by its cache,
// within the share of the device the library keeps to (three quarters)
size_t dev_free_bytes();
// Copies host memory to the device and waits; large copies go through a pinned
// staging buffer (allocated with hipHostMalloc and kept for reuse).
void host_to_device(void* dst, const void* src, size_t bytes, hipStream_t s);

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count) p = static_cast<T*>(dev_alloc(count * sizeof(T)));
  }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    n = 0;
  }
  void upload(const T* h, size_t count, hipStream_t s) {
    if (count > n) alloc(count);
    if (count) host_to_device(p, h, count * sizeof(T), s);  // synchronous: h may change right after
  }
  void upload(const std::vector<T>& v, hipStream_t s) { upload(v.data(), v.size(), s); }
};

// ---------------------------------------------------------------- tree
enum { KIND_INNER = 0, KIND_F = 1, KIND_N = 2 };

struct DeviceTree {
  DevBuf<int32_t> c_begin, c_size, c_parent, c_level, c_lc_begin, c_lc_end, leaf_clusters;
  DevBuf<int32_t> b_tau, b_sigma, b_kind;
  DevBuf<int32_t> brow_ptr, brow_blk, bcol_ptr, bcol_blk;
  DevBuf<double> xyz_perm;  // points in cluster order, n x 3
  DevBuf<int32_t> perm;     // cluster position -> original point index
};

struct Tree {
  std::atomic<int> refs{1};
  int64_t n = 0;
  int32_t leaf_size = 0, split = 0;
  double eta = 0;
  std::vector<double> xyz;  // original order, row-major n x 3
  std::vector<int32_t> perm;
  // clusters (breadth-first ids)
  std::vector<int32_t> c_begin, c_size, c_parent, c_level, c_child0, c_nchild;
  std::vector<double> c_bmin, c_bmax;  // 3 per cluster
  std::vector<double> c_diam;
  std::vector<int32_t> leaf_clusters;           // leaf clusters ordered by position
  std::vector<int32_t> c_lc_begin, c_lc_end;    // range of leaf_clusters inside each cluster
  // blocks (breadth-first ids; sons of a block are contiguous)
  std::vector<int32_t> b_tau, b_sigma, b_level, b_kind, b_child0, b_nchild, b_parent;
  std::vector<int32_t> leaves;      // leaf block ids, breadth-first
  std::vector<int32_t> leaf_index;  // block id -> position in `leaves` or -1
  std::vector<int64_t> level_begin; // blocks of level l are [level_begin[l], level_begin[l+1])
  int32_t depth = 0, csp = 0;
  // leaf blocks with row cluster c (sorted by column position) and column cluster c
  std::vector<int32_t> brow_ptr, brow_blk, bcol_ptr, bcol_blk;
  // (tau, sigma) -> block id lookup for restriction: per cluster tau the blocks of its
  // block row (all kinds), sorted by sigma id
  std::vector<int32_t> row_all_ptr, row_all_blk;

  DeviceTree* dev = nullptr;
  int dev_id = -1;
  std::mutex dev_mu;  // guards the lazy device copy

  int32_t find_block(int32_t tau, int32_t sigma) const;  // -1 if absent
  bool is_leaf_cluster(int32_t c) const { return c_nchild[c] == 0; }
  void ensure_device(hipStream_t s);
  ~Tree();
};

Tree* build_tree(const double* xyz, int64_t n, int32_t leaf, double eta, int32_t split);
bool admissible(const Tree& t, int32_t a, int32_t b);
double cluster_dist(const Tree& t, int32_t a, int32_t b);

inline void tree_retain(Tree* t) { t->refs.fetch_add(1); }
void tree_release(Tree* t);

// ---------------------------------------------------------------- H-matrix
struct ProductFeatures {
  std::vector<float> feats;  // n_far x 6
  std::vector<float> ranks;
  std::vector<float> widths;  // sketch columns at which the residual check passed
};

struct HMat {
  Tree* tree = nullptr;
  // per block id (all blocks): rank for F leaves, 0 otherwise; element offset of the
  // leaf's data in `pool` (-1 for inner blocks)
  std::vector<int32_t> rank;
  std::vector<int64_t> off;
  std::vector<uint8_t> notconv;  // per block: 1 for a farfield block whose compression did not converge
  int64_t pool_len = 0;
  DevBuf<double> pool;
  DevBuf<int32_t> d_rank;
  DevBuf<int64_t> d_off;
  DevBuf<float> pool32;  // float copy of `pool`, built on demand for mixed precision
  std::mutex mu32;       // guards building pool32
  ProductFeatures features;
  std::vector<double> block_flops;  // product output: algorithmic flops charged to each block as a target
  ~HMat();
  void upload_meta(hipStream_t s);
};

void hmat_release(HMat* m);

// ---------------------------------------------------------------- options
struct Opts {
  hmat_opts o;
  int concurrency = 1;  // products in flight at once (set by the batched driver)
  hipStream_t stream() const { return reinterpret_cast<hipStream_t>(o.stream); }
};
Opts resolve_opts(const hmat_opts* o);
// HMAT_ERR_ARG for a precision mode below its accuracy floor
void check_precision_floor(const Opts& o, double eps);

double now_seconds();

// Rank predictor inference: feats holds HMAT_N_FEATURES floats per target; out receives
// one predicted rank per target (synchronous on stream s).
void predict_ranks(hmat_rank_model model, const std::vector<float>& feats, std::vector<float>& out, hipStream_t s);

}  // namespace hm
