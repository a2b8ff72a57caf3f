// C ABI entry points: handles, error reporting, device allocator, tree queries,
// assembly, import/export. Every entry point catches everything and reports
// through hmat_last_error().
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

#include "block_cache.h"
#include "compress.h"
#include "hmat_internal.h"
#include "matvec.h"

namespace hm {

HMat* assemble_kernel(Tree* t, const hmat_kernel* k, double eps_in, const Opts& opts,
                      int64_t* n_not_converged);
hmat_status multiply(HMat* A, HMat* B, double eps, const Opts& opts, HMat** C);
hmat_status multiply_batched(HMat* const* A, HMat* const* B, int32_t count, double eps, const Opts& opts,
                             HMat** C, int32_t* status);
void expand_to_dense(HMat* M, double* out, int64_t ld, int32_t order, hipStream_t s);

static thread_local std::string g_err;
void set_last_error(const std::string& msg) { g_err = msg; }

// Device memory comes from a cache of blocks (block_cache.h) over hipMalloc/hipFree.
// The stream that orders a block's reuse is the calling thread's current stream.
static thread_local hipStream_t g_stream = 0;  // per host thread (concurrent products)

namespace {
struct HipOps {
  void* malloc(size_t b) {
    void* p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void release(void* p) { (void)hipFree(p); }
  void* record(void* s) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    if (hipEventRecord(ev, static_cast<hipStream_t>(s)) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipEventDestroy(ev);
      return nullptr;
    }
    return ev;
  }
  bool done(void* ev) {
    const hipError_t q = hipEventQuery(static_cast<hipEvent_t>(ev));
    if (q != hipSuccess) (void)hipGetLastError();  // not ready (or unusable): not done
    return q == hipSuccess;
  }
  void wait(void* ev) {
    if (hipEventSynchronize(static_cast<hipEvent_t>(ev)) != hipSuccess) (void)hipGetLastError();
  }
  void destroy(void* ev) { (void)hipEventDestroy(static_cast<hipEvent_t>(ev)); }
  double now() { return now_seconds(); }
};

size_t device_total() {
  size_t fb = 0, tb = 0;
  if (hipMemGetInfo(&fb, &tb) != hipSuccess) {
    (void)hipGetLastError();
    return size_t(128) << 30;
  }
  return tb;
}

// The library holds at most three quarters of the device memory (live and cached
// blocks): before an allocation would go past that, idle cached blocks are released.
// A device run close to full has made products stall. trim() would hand idle blocks back
// down to an eighth of the memory; the library releases them only before or after an
// allocation (block_cache.h), never when a block is freed.
BlockCache<HipOps>& cache() {
  static BlockCache<HipOps> c(HipOps{}, device_total() / 4, false, device_total() / 4 * 3);
  // HMAT_ALLOC_TRACE=<file>: one line per allocation, free and release (block_cache.h)
  static const bool traced = [] {
    const char* f = std::getenv("HMAT_ALLOC_TRACE");
    if (f && *f) c.set_trace(std::fopen(f, "w"));
    return true;
  }();
  (void)traced;
  return c;
}
}  // namespace

void set_current_stream(hipStream_t s) { g_stream = s; }

void forget_stream(hipStream_t s) { cache().forget_stream(s); }

size_t dev_free_bytes() {
  size_t fb = 0, tb = 0;
  HM_CHECK_HIP(hipMemGetInfo(&fb, &tb));
  BlockCache<HipOps>& c = cache();
  const size_t cached = c.cached_bytes(), held = c.held_bytes();
  const size_t live = held - std::min(held, cached);
  const size_t room = c.soft_cap() > live ? c.soft_cap() - live : 0;
  return std::min(fb + cached, room);
}

AllocCounters alloc_counters() {
  const CacheCounters c = cache().counters();
  AllocCounters a;
  a.seconds = c.seconds;
  a.mallocs = c.mallocs;
  a.releases = c.releases;
  return a;
}

void* dev_alloc(size_t bytes) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  void* p = cache().alloc(bytes, dev, g_stream);
  if (!p) throw Error(HMAT_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  if (!cache().free(p, g_stream)) (void)hipFree(p);
}

// Pinned staging buffers for large host-to-device copies: a pool shared by the host
// threads. A copy holds one buffer for its whole duration but no lock while it waits
// for its stream, so concurrent products do not queue behind each other's streams.
static std::mutex g_pin_mu;
static std::vector<void*> g_pin_free;
static constexpr size_t kPinChunk = size_t(64) << 20;

namespace {
struct PinnedLease {
  void* p = nullptr;
  PinnedLease() {
    {
      std::lock_guard<std::mutex> lk(g_pin_mu);
      if (!g_pin_free.empty()) {
        p = g_pin_free.back();
        g_pin_free.pop_back();
        return;
      }
    }
    if (hipHostMalloc(&p, kPinChunk) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
  }
  ~PinnedLease() {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.push_back(p);
  }
};
}  // namespace

void host_to_device(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t small = size_t(4) << 20;
  if (bytes <= small) {
    HM_CHECK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    return;
  }
  PinnedLease pin;
  if (!pin.p) {  // no pinned memory: plain copy
    HM_CHECK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
    return;
  }
  const char* hs = static_cast<const char*>(src);
  char* dd = static_cast<char*>(dst);
  for (size_t off = 0; off < bytes; off += kPinChunk) {
    const size_t len = std::min(kPinChunk, bytes - off);
    std::memcpy(pin.p, hs + off, len);
    HM_CHECK_HIP(hipMemcpyAsync(dd + off, pin.p, len, hipMemcpyHostToDevice, s));
    HM_CHECK_HIP(hipStreamSynchronize(s));
  }
}

double now_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

Opts resolve_opts(const hmat_opts* o) {
  Opts r;
  hmat_opts_default(&r.o);
  if (o) r.o = *o;
  HM_REQUIRE(r.o.b0 >= 1 && r.o.b0 <= 32, HMAT_ERR_ARG, "b0 must be in [1, 32]");
  HM_REQUIRE(r.o.growth >= 1 && r.o.growth <= 16, HMAT_ERR_ARG, "growth must be in [1, 16]");
  HM_REQUIRE(r.o.probes >= 1 && r.o.probes <= 16, HMAT_ERR_ARG, "probes must be in [1, 16]");
  HM_REQUIRE(r.o.max_growth >= 0 && r.o.max_growth <= 16, HMAT_ERR_ARG, "max_growth must be in [0, 16]");
  HM_REQUIRE(r.o.p_l >= 0 && r.o.p_l <= 16, HMAT_ERR_ARG, "p_l must be in [0, 16]");
  HM_REQUIRE(r.o.delta > 0.0 && r.o.delta <= 1.0, HMAT_ERR_ARG, "delta must be in (0, 1]");
  HM_REQUIRE(r.o.precision >= 0 && r.o.precision <= 2, HMAT_ERR_ARG, "unknown precision");
  HM_REQUIRE(r.o.precision != HMAT_BF16_SKETCH, HMAT_ERR_ARG,
             "HMAT_BF16_SKETCH is not supported: bf16 panels perturb S by ~4e-3 relative, far above any "
             "tolerance the product targets, so the sketch would need as many fp64 growth rounds as it saves");
  HM_REQUIRE(r.o.rank_mode == HMAT_RANK_ADAPTIVE || r.o.rank_mode == HMAT_RANK_PREDICT, HMAT_ERR_ARG,
             "unknown rank mode");
  HM_REQUIRE(r.o.rank_mode != HMAT_RANK_PREDICT || r.o.rank_model != nullptr, HMAT_ERR_ARG,
             "HMAT_RANK_PREDICT needs opts.rank_model");
  HM_REQUIRE(r.o.streams >= 0 && r.o.streams <= 4, HMAT_ERR_ARG, "streams must be in [0, 4]");
  HM_REQUIRE(r.o.scheme >= HMAT_SCHEME_RANDOMIZED && r.o.scheme <= HMAT_SCHEME_LANCZOS, HMAT_ERR_ARG,
             "unknown scheme");
  HM_REQUIRE(r.o.k_fixed >= 0 && r.o.k_fixed <= 64, HMAT_ERR_ARG, "k_fixed must be in [0, 64]");
  HM_REQUIRE(r.o.subspace_iters >= 0 && r.o.subspace_iters <= 8, HMAT_ERR_ARG, "subspace_iters must be in [0, 8]");
  HM_REQUIRE(r.o.exact_lowrank == 0 || r.o.exact_lowrank == 1, HMAT_ERR_ARG, "exact_lowrank must be 0 or 1");
  HM_REQUIRE(r.o.full_passes == 0 || r.o.full_passes == 1, HMAT_ERR_ARG, "full_passes must be 0 or 1");
  const bool plain_randomized = r.o.scheme == HMAT_SCHEME_RANDOMIZED && r.o.k_fixed == 0;
  HM_REQUIRE(r.o.rank_mode != HMAT_RANK_PREDICT || plain_randomized, HMAT_ERR_ARG,
             "HMAT_RANK_PREDICT sizes the first sketch of the adaptive randomized scheme only");
  HM_REQUIRE(r.o.precision != HMAT_FP32_APPLY || plain_randomized, HMAT_ERR_ARG,
             "HMAT_FP32_APPLY applies to the sketch passes of the adaptive randomized scheme only");
  return r;
}

// The float32 panels of HMAT_FP32_APPLY perturb S by about 1e-7 relative, and the residual
// probe, computed from the same panels, cannot see that perturbation; the truncation margin
// absorbs it only down to the smallest tolerance at which the mode was checked against the
// oracle.
void check_precision_floor(const Opts& o, double eps) {
  HM_REQUIRE(o.o.precision != HMAT_FP32_APPLY || eps >= HMAT_FP32_APPLY_EPS_MIN, HMAT_ERR_ARG,
             "HMAT_FP32_APPLY needs eps >= 1e-6: below that the float32 panel rounding (about 1e-7 relative) "
             "is not covered by the residual check");
}

HMat::~HMat() { tree_release(tree); }

void HMat::upload_meta(hipStream_t s) {
  d_rank.upload(rank, s);
  d_off.upload(off, s);
}

void hmat_release(HMat* m) { delete m; }

// Checks shared by the matvec entry points; returns M.
HMat* check_matvec_args(hmat mh, int32_t trans, int32_t order, int32_t nvec, const double* x, int64_t ldx,
                        const double* y, int64_t ldy) {
  HM_REQUIRE(mh && x && y, HMAT_ERR_ARG, "NULL argument");
  HMat* M = reinterpret_cast<HMat*>(mh);
  const int64_t n = M->tree->n;
  HM_REQUIRE(trans == 0 || trans == 1, HMAT_ERR_ARG, "trans must be 0 or 1");
  HM_REQUIRE(order == 0 || order == 1, HMAT_ERR_ARG, "order must be 0 or 1");
  HM_REQUIRE(nvec >= 1, HMAT_ERR_ARG, "nvec must be >= 1");
  HM_REQUIRE(ldx >= n && ldy >= n, HMAT_ERR_ARG, "ldx and ldy must be >= n");
  const char* xb = reinterpret_cast<const char*>(x);
  const char* yb = reinterpret_cast<const char*>(y);
  const int64_t xl = 8 * (ldx * (nvec - 1) + n), yl = 8 * (ldy * (nvec - 1) + n);
  HM_REQUIRE(xb + xl <= yb || yb + yl <= xb, HMAT_ERR_ARG, "x and y overlap");
  int dev = 0;
  HM_CHECK_HIP(hipGetDevice(&dev));
  HM_REQUIRE(M->tree->dev != nullptr && M->tree->dev_id == dev, HMAT_ERR_ARG,
             "the current device is not the one the H-matrix lives on");
  return M;
}

}  // namespace hm

using namespace hm;

#define API_BEGIN try {
#define API_END                                   \
  }                                               \
  catch (const hm::Error& e) {                    \
    set_last_error(e.what());                     \
    return e.code;                                \
  }                                               \
  catch (const std::bad_alloc&) {                 \
    set_last_error("host allocation failed");     \
    return HMAT_ERR_OOM;                          \
  }                                               \
  catch (const std::exception& e) {               \
    set_last_error(e.what());                     \
    return HMAT_ERR_INTERNAL;                     \
  }                                               \
  catch (...) {                                   \
    set_last_error("unknown error");              \
    return HMAT_ERR_INTERNAL;                     \
  }                                               \
  set_last_error("");                             \
  return HMAT_OK;

extern "C" {

const char* hmat_last_error(void) { return g_err.c_str(); }
const char* hmat_version(void) { return "hmat-mi355x 0.1"; }

void hmat_opts_default(hmat_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = HMAT_FP64;
  o->rank_mode = HMAT_RANK_ADAPTIVE;
  o->b0 = 8;
  o->growth = 8;
  o->probes = 8;
  o->max_growth = 6;
  o->p_l = 2;
  o->delta = 0.2;
  o->seed = 0x5eedull;
  o->scheme = HMAT_SCHEME_RANDOMIZED;
  o->subspace_iters = 1;
}

hmat_status hmat_build_tree(const double* xyz, int64_t n, int32_t leaf_size, double eta, int32_t split,
                            hmat_tree* out) {
  API_BEGIN
  HM_REQUIRE(out != nullptr, HMAT_ERR_ARG, "out is NULL");
  *out = reinterpret_cast<hmat_tree>(build_tree(xyz, n, leaf_size, eta, split));
  API_END
}

hmat_status hmat_tree_destroy(hmat_tree t) {
  API_BEGIN
  tree_release(reinterpret_cast<Tree*>(t));
  API_END
}

hmat_status hmat_tree_info(hmat_tree th, hmat_tree_info_t* out) {
  API_BEGIN
  HM_REQUIRE(th && out, HMAT_ERR_ARG, "NULL argument");
  Tree* t = reinterpret_cast<Tree*>(th);
  out->n = t->n;
  out->leaf_size = t->leaf_size;
  out->split = t->split;
  out->eta = t->eta;
  out->depth = t->depth;
  out->n_clusters = int32_t(t->c_begin.size());
  out->n_blocks = int64_t(t->b_tau.size());
  int64_t nf = 0, nn = 0;
  for (int32_t b : t->leaves) (t->b_kind[b] == KIND_F ? nf : nn)++;
  out->n_far = nf;
  out->n_near = nn;
  out->csp = t->csp;
  API_END
}

hmat_status hmat_tree_perm(hmat_tree th, int32_t* perm) {
  API_BEGIN
  HM_REQUIRE(th && perm, HMAT_ERR_ARG, "NULL argument");
  Tree* t = reinterpret_cast<Tree*>(th);
  std::memcpy(perm, t->perm.data(), sizeof(int32_t) * t->perm.size());
  API_END
}

hmat_status hmat_tree_clusters(hmat_tree th, int32_t* begin, int32_t* size, int32_t* parent, int32_t* level) {
  API_BEGIN
  HM_REQUIRE(th, HMAT_ERR_ARG, "NULL tree");
  Tree* t = reinterpret_cast<Tree*>(th);
  size_t nc = t->c_begin.size();
  if (begin) std::memcpy(begin, t->c_begin.data(), 4 * nc);
  if (size) std::memcpy(size, t->c_size.data(), 4 * nc);
  if (parent) std::memcpy(parent, t->c_parent.data(), 4 * nc);
  if (level) std::memcpy(level, t->c_level.data(), 4 * nc);
  API_END
}

hmat_status hmat_tree_blocks(hmat_tree th, int32_t* tau, int32_t* sigma, int32_t* level, int32_t* kind) {
  API_BEGIN
  HM_REQUIRE(th, HMAT_ERR_ARG, "NULL tree");
  Tree* t = reinterpret_cast<Tree*>(th);
  size_t nb = t->b_tau.size();
  if (tau) std::memcpy(tau, t->b_tau.data(), 4 * nb);
  if (sigma) std::memcpy(sigma, t->b_sigma.data(), 4 * nb);
  if (level) std::memcpy(level, t->b_level.data(), 4 * nb);
  if (kind) std::memcpy(kind, t->b_kind.data(), 4 * nb);
  API_END
}

hmat_status hmat_assemble(hmat_tree th, const hmat_kernel* k, double eps_in, const hmat_opts* opts, hmat* out) {
  API_BEGIN
  HM_REQUIRE(th && k && out, HMAT_ERR_ARG, "NULL argument");
  Opts o = resolve_opts(opts);
  int64_t nc = 0;
  HMat* M = assemble_kernel(reinterpret_cast<Tree*>(th), k, eps_in, o, &nc);
  *out = reinterpret_cast<hmat>(M);
  if (nc > 0) {
    set_last_error(std::to_string(nc) + " farfield blocks did not reach eps_in");
    return HMAT_ERR_NOT_CONVERGED;
  }
  API_END
}

hmat_status hmat_from_blocks(hmat_tree th, const int32_t* ranks, const int64_t* offsets, const double* pool,
                             hmat* out) {
  API_BEGIN
  HM_REQUIRE(th && ranks && offsets && pool && out, HMAT_ERR_ARG, "NULL argument");
  Tree* t = reinterpret_cast<Tree*>(th);
  HMat* M = new HMat();
  M->tree = t;
  tree_retain(t);
  const int64_t nb = int64_t(t->b_tau.size());
  M->rank.assign(nb, 0);
  M->off.assign(nb, -1);
  int64_t total = 0;
  std::vector<int64_t> len(t->leaves.size());
  for (size_t i = 0; i < t->leaves.size(); ++i) {
    int32_t b = t->leaves[i];
    int64_t m = t->c_size[t->b_tau[b]], n = t->c_size[t->b_sigma[b]];
    if (t->b_kind[b] == KIND_F) {
      if (ranks[i] < 0 || ranks[i] > std::min(m, n)) {
        delete M;
        throw Error(HMAT_ERR_ARG, "rank out of range at leaf " + std::to_string(i));
      }
      M->rank[b] = ranks[i];
      len[i] = int64_t(ranks[i]) * (m + n);
    } else {
      len[i] = m * n;
    }
    M->off[b] = total;
    total += len[i];
  }
  std::vector<double> h(size_t(std::max<int64_t>(total, 1)));
  for (size_t i = 0; i < t->leaves.size(); ++i)
    std::memcpy(h.data() + M->off[t->leaves[i]], pool + offsets[i], 8 * len[i]);
  M->pool_len = total;
  hipStream_t s = 0;
  M->pool.upload(h, s);
  M->upload_meta(s);
  HM_CHECK_HIP(hipStreamSynchronize(s));
  *out = reinterpret_cast<hmat>(M);
  API_END
}

hmat_status hmat_destroy(hmat m) {
  API_BEGIN
  hmat_release(reinterpret_cast<HMat*>(m));
  API_END
}

hmat_status hmat_multiply(hmat A, hmat B, double eps, const hmat_opts* opts, hmat* C) {
  API_BEGIN
  HM_REQUIRE(A && B && C, HMAT_ERR_ARG, "NULL argument");
  HM_REQUIRE(eps > 0.0 && eps < 1.0, HMAT_ERR_ARG, "eps must be in (0, 1)");
  Opts o = resolve_opts(opts);
  check_precision_floor(o, eps);
  HMat* out = nullptr;
  hmat_status st = multiply(reinterpret_cast<HMat*>(A), reinterpret_cast<HMat*>(B), eps, o, &out);
  *C = reinterpret_cast<hmat>(out);
  if (st != HMAT_OK) return st;
  API_END
}

hmat_status hmat_multiply_batched(const hmat* A, const hmat* B, int32_t count, double eps, const hmat_opts* opts,
                                  hmat* C, int32_t* status) {
  API_BEGIN
  HM_REQUIRE(A && B && C && count >= 0, HMAT_ERR_ARG, "bad argument");
  HM_REQUIRE(eps > 0.0 && eps < 1.0, HMAT_ERR_ARG, "eps must be in (0, 1)");
  Opts o = resolve_opts(opts);
  check_precision_floor(o, eps);
  hmat_status st = multiply_batched(reinterpret_cast<HMat* const*>(A), reinterpret_cast<HMat* const*>(B),
                                    count, eps, o, reinterpret_cast<HMat**>(C), status);
  if (st != HMAT_OK) return st;
  API_END
}


hmat_status hmat_matvec(hmat mh, int32_t trans, int32_t order, int32_t nvec, const double* x, int64_t ldx,
                        double* y, int64_t ldy, void* stream) {
  API_BEGIN
  HMat* M = check_matvec_args(mh, trans, order, nvec, x, ldx, y, ldy);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  set_current_stream(s);
  DevBuf<double> scratch(size_t(matvec_scratch_doubles(M, nvec)));
  matvec_launch(M, trans, order, nvec, x, ldx, y, ldy, scratch.p, s);
  API_END
}

hmat_status hmat_error_estimate(hmat Ch, hmat Ah, hmat Bh, const double* X0, int32_t p, int32_t iters, void* stream,
                                double* err, double* norm_ab) {
  API_BEGIN
  HM_REQUIRE(Ch && Ah && Bh && X0 && err && norm_ab, HMAT_ERR_ARG, "NULL argument");
  HMat* C = reinterpret_cast<HMat*>(Ch);
  HMat* A = reinterpret_cast<HMat*>(Ah);
  HMat* B = reinterpret_cast<HMat*>(Bh);
  HM_REQUIRE(A->tree == B->tree && C->tree == A->tree, HMAT_ERR_TREE_MISMATCH, "C, A and B must share one tree");
  HM_REQUIRE(p >= 1 && p <= A->tree->n, HMAT_ERR_ARG, "p must be in [1, n]");
  HM_REQUIRE(iters >= 0 && iters <= 100, HMAT_ERR_ARG, "iters must be in [0, 100]");
  int dev = 0;
  HM_CHECK_HIP(hipGetDevice(&dev));
  HM_REQUIRE(A->tree->dev != nullptr && A->tree->dev_id == dev, HMAT_ERR_ARG,
             "the current device is not the one the H-matrices live on");
  error_estimate(C, A, B, X0, p, iters, reinterpret_cast<hipStream_t>(stream), err, norm_ab);
  API_END
}

hmat_status hmat_gaussian_panel(int64_t n, int32_t ncol, uint64_t seed, double* out, void* stream) {
  API_BEGIN
  HM_REQUIRE(out != nullptr, HMAT_ERR_ARG, "out is NULL");
  HM_REQUIRE(n >= 0 && ncol >= 0 && n < (int64_t(1) << 38), HMAT_ERR_ARG, "n must be in [0, 2^38) and ncol >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_fill_gaussian(out, n, ncol, seed, s);
  HM_CHECK_HIP(hipStreamSynchronize(s));
  API_END
}

hmat_status hmat_to_dense(hmat mh, double* out, int64_t ld, int32_t order) {
  API_BEGIN
  HM_REQUIRE(mh && out, HMAT_ERR_ARG, "NULL argument");
  HMat* M = reinterpret_cast<HMat*>(mh);
  HM_REQUIRE(ld >= M->tree->n, HMAT_ERR_ARG, "ld < n");
  HM_REQUIRE(order == 0 || order == 1, HMAT_ERR_ARG, "order must be 0 or 1");
  expand_to_dense(M, out, ld, order, 0);
  API_END
}

hmat_status hmat_block_count(hmat mh, int64_t* count) {
  API_BEGIN
  HM_REQUIRE(mh && count, HMAT_ERR_ARG, "NULL argument");
  *count = int64_t(reinterpret_cast<HMat*>(mh)->tree->leaves.size());
  API_END
}

hmat_status hmat_block_get(hmat mh, int64_t i, hmat_block_desc* d, double* U, double* V) {
  API_BEGIN
  HM_REQUIRE(mh && d, HMAT_ERR_ARG, "NULL argument");
  HMat* M = reinterpret_cast<HMat*>(mh);
  Tree* t = M->tree;
  HM_REQUIRE(i >= 0 && i < int64_t(t->leaves.size()), HMAT_ERR_ARG, "block index out of range");
  int32_t b = t->leaves[i];
  d->row_begin = t->c_begin[t->b_tau[b]];
  d->rows = t->c_size[t->b_tau[b]];
  d->col_begin = t->c_begin[t->b_sigma[b]];
  d->cols = t->c_size[t->b_sigma[b]];
  d->level = t->b_level[b];
  d->kind = t->b_kind[b];
  d->rank = t->b_kind[b] == KIND_F ? M->rank[b] : 0;
  d->block = b;
  d->converged = (!M->notconv.empty() && M->notconv[b]) ? 0 : 1;
  d->pad = 0;
  if (t->b_kind[b] == KIND_F) {
    int64_t k = M->rank[b];
    if (U && k) HM_CHECK_HIP(hipMemcpy(U, M->pool.p + M->off[b], 8 * k * d->rows, hipMemcpyDeviceToHost));
    if (V && k)
      HM_CHECK_HIP(hipMemcpy(V, M->pool.p + M->off[b] + k * d->rows, 8 * k * d->cols, hipMemcpyDeviceToHost));
  } else if (V) {
    HM_CHECK_HIP(hipMemcpy(V, M->pool.p + M->off[b], 8 * d->rows * d->cols, hipMemcpyDeviceToHost));
  }
  API_END
}

hmat_status hmat_product_block_flops(hmat mh, double* flops) {
  API_BEGIN
  HM_REQUIRE(mh && flops, HMAT_ERR_ARG, "NULL argument");
  HMat* M = reinterpret_cast<HMat*>(mh);
  Tree* t = M->tree;
  for (size_t i = 0; i < t->leaves.size(); ++i)
    flops[i] = M->block_flops.empty() ? 0.0 : M->block_flops[t->leaves[i]];
  API_END
}

hmat_status hmat_export(hmat mh, int32_t* ranks, int64_t* offsets, double* pool, int64_t* pool_len) {
  API_BEGIN
  HM_REQUIRE(mh && pool_len, HMAT_ERR_ARG, "NULL argument");
  HMat* M = reinterpret_cast<HMat*>(mh);
  Tree* t = M->tree;
  for (size_t i = 0; i < t->leaves.size(); ++i) {
    int32_t b = t->leaves[i];
    if (ranks) ranks[i] = M->rank[b];
    if (offsets) offsets[i] = M->off[b];
  }
  if (pool) {
    HM_REQUIRE(*pool_len >= M->pool_len, HMAT_ERR_ARG, "pool buffer too small");
    if (M->pool_len)
      HM_CHECK_HIP(hipMemcpy(pool, M->pool.p, 8 * size_t(M->pool_len), hipMemcpyDeviceToHost));
  }
  *pool_len = M->pool_len;
  API_END
}

}  // extern "C"
