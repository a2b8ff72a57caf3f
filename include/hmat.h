/*
 * hmat.h -- C ABI of the MI355X hierarchical-matrix product library.
 *
 * The library computes the product C = A B of two H-matrices that live on one
 * block-cluster tree and, for every admissible (farfield) leaf tau x sigma of
 * that tree, stores the best approximation at relative Frobenius tolerance eps
 * of the exact block (A B)[tau, sigma]; inadmissible (nearfield) leaves of C
 * hold the exact dense block. This is the product of Doelz, Harbrecht and
 * Multerer, "On the best approximation of the hierarchical matrix product":
 * sum-expressions (Def. 3.1) built by restriction (Algorithm 3) inside the
 * recursive product (Algorithm 4), compressed by the blocked randomized scheme
 * (Section 4, randomized low-rank approximation) that touches each sum only
 * through its products with blocks of vectors (the sum-expression-times-vector
 * identity ending Section 3).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an hmat_status; HMAT_OK is 0. On failure a message
 *    is available from hmat_last_error() (thread-local, valid until the next
 *    call on that thread). No C++ exception crosses this interface.
 *  - Pointers documented as "host" are CPU memory owned by the caller; the
 *    library copies what it needs before returning and never keeps them.
 *  - Handles (hmat_tree, hmat, hmat_rank_model) are owned by the caller and
 *    released with the matching *_destroy call. An hmat keeps a reference to
 *    its tree, so a tree may be destroyed while matrices built on it live.
 *  - Positions: a tree orders the points so that every cluster is a contiguous
 *    range of positions ("cluster order"); perm[pos] is the original index of
 *    the point at that position.
 *  - Dense matrices exchanged with the caller are column-major with a leading
 *    dimension argument.
 *  - All device work runs on the HIP stream given in hmat_opts.stream (the
 *    null stream when 0); entry points that return data to the host
 *    synchronise that stream before returning.
 *  - Errors are never swallowed: a call either completes its whole job or
 *    returns a non-zero status (HMAT_ERR_NOT_CONVERGED additionally returns a
 *    usable result, see hmat_multiply).
 */
#ifndef HMAT_H
#define HMAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hmat_status;
enum {
  HMAT_OK = 0,
  HMAT_ERR_ARG = 1,            /* invalid argument (size, tolerance, null pointer, NaN point) */
  HMAT_ERR_TREE_MISMATCH = 2,  /* factors do not share one block-cluster tree */
  HMAT_ERR_NOT_CONVERGED = 3,  /* some farfield blocks exhausted the growth budget */
  HMAT_ERR_DEVICE = 4,         /* HIP runtime error */
  HMAT_ERR_OOM = 5,            /* device allocation failed */
  HMAT_ERR_INTERNAL = 6
};

typedef struct hmat_tree_s* hmat_tree;
typedef struct hmat_s* hmat;
typedef struct hmat_rank_model_s* hmat_rank_model;

/* Last error message of the calling thread (never NULL). */
const char* hmat_last_error(void);

/* Library version string. */
const char* hmat_version(void);


/* ------------------------------------------------------------------------ */
/* Cluster tree and block-cluster tree (Section 2: Def. 2.2, Def. 2.3,       */
/* Algorithm 1).                                                             */
/* ------------------------------------------------------------------------ */

enum { HMAT_SPLIT_MIDPOINT = 0, HMAT_SPLIT_MEDIAN = 1 };

/*
 * Builds the cluster tree of n points and the block-cluster tree on it.
 *  xyz        host, n x 3 row-major float64 coordinates (copied).
 *  leaf_size  a cluster with at most leaf_size points is a leaf (>= 1).
 *  eta        admissibility: dist > 0 and max(diam tau, diam sigma) <= eta*dist,
 *             with diam/dist taken on tight axis-aligned bounding boxes (> 0).
 *  split      HMAT_SPLIT_MIDPOINT: halve the longest box edge (ties to the
 *             lowest axis) at its midpoint, points <= mid to the first son;
 *             HMAT_SPLIT_MEDIAN: first floor(#tau/2) points after a stable
 *             sort along that edge. A cluster whose box has zero extent, or
 *             whose midpoint cut would leave a son empty, stays a leaf.
 *  out        receives the new tree handle.
 * Sons of a block are tau' x sigma' in tau'-major order (Algorithm 1).
 * Errors: HMAT_ERR_ARG for n < 1, leaf_size < 1, eta <= 0 or not finite, a
 * non-finite coordinate, an unknown split or a NULL pointer.
 */
hmat_status hmat_build_tree(const double* xyz, int64_t n, int32_t leaf_size, double eta,
                            int32_t split, hmat_tree* out);
hmat_status hmat_tree_destroy(hmat_tree t);

typedef struct {
  int64_t n;
  int32_t leaf_size;
  int32_t split;
  double eta;
  int32_t depth;       /* depth of the block-cluster tree */
  int32_t n_clusters;
  int64_t n_blocks;    /* all blocks, inner ones included */
  int64_t n_far;       /* admissible leaves (F) */
  int64_t n_near;      /* inadmissible leaves (N) */
  int32_t csp;         /* sparsity constant: max blocks per cluster (row or column) */
} hmat_tree_info_t;

hmat_status hmat_tree_info(hmat_tree t, hmat_tree_info_t* out);
/* perm: host int32[n], perm[pos] = original index. */
hmat_status hmat_tree_perm(hmat_tree t, int32_t* perm);
/* Clusters in breadth-first order; each output is host int32[n_clusters]. */
hmat_status hmat_tree_clusters(hmat_tree t, int32_t* begin, int32_t* size, int32_t* parent,
                               int32_t* level);
/* Blocks in breadth-first order; each output host int32[n_blocks]; kind is
 * 0 = inner, 1 = farfield leaf (F), 2 = nearfield leaf (N). */
hmat_status hmat_tree_blocks(hmat_tree t, int32_t* tau, int32_t* sigma, int32_t* level,
                             int32_t* kind);

/* ------------------------------------------------------------------------ */
/* Options and statistics                                                   */
/* ------------------------------------------------------------------------ */

/*
 * Precision of the sum-expression applies:
 *  HMAT_FP64        everything in float64;
 *  HMAT_FP32_APPLY  the forward sketch and probe passes read float32 copies of
 *                   every panel (inputs and created terms; arithmetic stays
 *                   float64 on MFMA), while projection, orthogonalisation,
 *                   core SVD, truncation and the nearfield stay float64; the
 *                   float copies of A and B are kept with the matrices. Only
 *                   for eps >= HMAT_FP32_APPLY_EPS_MIN (HMAT_ERR_ARG below):
 *                   the float rounding of the panels (about 1e-7 relative) is
 *                   invisible to the residual probe, which reads the same
 *                   panels, and the truncation margin covers it only there;
 *  HMAT_BF16_SKETCH rejected with HMAT_ERR_ARG (bf16 panels perturb S by about
 *                   4e-3 relative, above every supported tolerance).
 */
enum { HMAT_FP64 = 0, HMAT_FP32_APPLY = 1, HMAT_BF16_SKETCH = 2 };
#define HMAT_FP32_APPLY_EPS_MIN 1e-6
enum { HMAT_RANK_ADAPTIVE = 0, HMAT_RANK_PREDICT = 1 };

typedef struct {
  double t_total;      /* seconds, entry to completion (stream synchronised) */
  double t_plan;       /* host planning of the work lists */
  double t_restrict;   /* creation of low-rank terms (Algorithm 3 products) */
  double t_sketch;     /* range finding incl. probes and growth rounds */
  double t_project;    /* projection passes */
  double t_core;       /* orthogonalisation, core SVD, truncation, output */
  double t_near;       /* nearfield evaluation */
  double t_predict;    /* rank-predictor inference */
  double flops_alg;    /* algorithmic flops of the passes actually run */
  double bytes_alg;    /* algorithmic operand bytes of the passes actually run */
  int64_t n_far, n_near;
  int64_t n_growth_rounds;   /* total growth rounds over all levels */
  int64_t n_grown_blocks;    /* block-rounds that needed growth */
  int64_t n_not_converged;
  int64_t n_fallback;        /* learned mode: blocks whose prediction failed the check */
  int64_t sketch_columns;    /* sum over farfield blocks of sketch columns used */
  int64_t peak_bytes;        /* peak device workspace of the call */
  int32_t n_batches;         /* subtree batches the product was split into */
  int32_t rank_hist[65];     /* output ranks; index 64 counts ranks >= 64 */
  /* Per kernel family (HMAT_KERN_*): launches, summed launch durations measured
   * with HIP events on the product's stream (only with opts.time_kernels), and
   * the algorithmic operand bytes and flops those launches processed. */
  int64_t kern_launches[8];
  double kern_time[8];
  double kern_bytes[8];
  double kern_flops[8];
  /* Time split: [0] symbolic plan, [1] term-creation lists, [2] chunk
   * partition + upload + waiting for the chunk builder, [3] waiting on the device
   * inside the compression loop, [4] term-pool allocation, [5] creation-list
   * upload, [6] creation kernels incl. synchronisation, [7] term publication. */
  double t_host[8];
  /* device memory of the product: seconds in hipMalloc/hipFree, hipMalloc calls,
   * times the block cache was emptied to make room */
  double t_alloc;
  int64_t n_malloc;
  int64_t n_cache_release;
  /* operator applications: sum over passes of the targets taking part (a pass
   * applies a target's sum-expression, or its transpose, to up to 16 columns) */
  int64_t target_passes;
  /* hmat_multiply_batched: products in flight at once (chosen or autotuned) */
  int32_t streams_used;
  int32_t pad_s;
  /* nearfield targets evaluated by the direct kernel, and seconds spent on the
   * other nearfield targets (identity panels) */
  int64_t n_near_direct;
  double t_near_panels;
  /* size of the symbolic plan: low-rank terms created, pairs kept at leaves */
  int64_t n_terms;
  int64_t n_leaf_pairs;
  /* farfield blocks: iterations of ACA / Lanczos kept (summed), columns of the
   * fixed-rank sketch, blocks truncated exactly by Algorithm 5, and final SVDs whose
   * Jacobi iteration reached its sweep cap (their factors are still exact, their
   * truncation may keep more columns than needed) */
  int64_t scheme_steps;
  int64_t n_exact_lowrank;
  int64_t n_svd_sweep_cap;
  /* seconds spent in the growth rounds of the adaptive randomized scheme (extra probes,
   * orthogonalisation and projections after the first residual check): the most that a
   * better first sketch width (HMAT_RANK_PREDICT) can save */
  double t_growth;
  /* passes over chunks of targets (sketch, projection and identity-panel passes), and those
   * of them that launched only the work items of their active targets (full_passes) */
  int64_t n_passes;
  int64_t n_sparse_passes;
} hmat_stats;

/* Kernel families of hmat_stats.kern_* */
enum {
  HMAT_KERN_TERM_REDUCE = 0,   /* core (R^T X) per (target, low-rank term) */
  HMAT_KERN_LEAF_REDUCE = 1,   /* R^T X per (subtree product, low-rank leaf) */
  HMAT_KERN_SUBTREE_EXPAND = 2,/* subtree products: L T and D X per output leaf cluster */
  HMAT_KERN_GATHER = 3,        /* per target: sum of L V over its terms and pair results */
  HMAT_KERN_COMPRESS = 4,      /* orthogonalisation, probe residual, core SVD, output */
  HMAT_KERN_FUSED_TERMS = 5,   /* fused term reduce + expand, targets of <= 64 rows/columns */
  HMAT_KERN_FUSED_TERMS4 = 6,  /* the same with four waves, targets of <= 256 rows/columns */
  HMAT_KERN_NEAR_DIRECT = 7    /* nearfield targets of <= 256 x 256: low-rank terms and dense x dense
                                  pairs evaluated per 64 x 64 sub-block, all columns at once */
};

typedef struct {
  int32_t precision;   /* HMAT_FP64 (default) or HMAT_FP32_APPLY */
  int32_t rank_mode;   /* HMAT_RANK_ADAPTIVE (default) or HMAT_RANK_PREDICT: the model's output
                          per farfield block is read as the sketch width the block needs; a
                          prediction up to b0 + 3 growth / 4 keeps the first width b0, above it the
                          first width is the prediction plus p_l (rounded up to the 16-column
                          pass granularity) */
  int32_t b0;          /* initial sketch width (default 8) */
  int32_t growth;      /* columns added per growth round (default 8) */
  int32_t probes;      /* probe columns of the a-posteriori check (default 8) */
  int32_t max_growth;  /* growth rounds before HMAT_ERR_NOT_CONVERGED (default 6) */
  int32_t p_l;         /* oversampling added to a prediction that widens the first sketch (default 2) */
  int32_t time_kernels;/* 1: time every kernel launch with HIP events into stats */
  double delta;        /* residual target: E <= delta * eps * ||S||_F (default 0.2) */
  uint64_t seed;       /* random stream of the sketches (default 0x5eed) */
  void* stream;        /* hipStream_t (0 = null stream) */
  hmat_rank_model rank_model;  /* required for HMAT_RANK_PREDICT */
  hmat_stats* stats;   /* optional output */
  int64_t workspace_limit;     /* bytes of device workspace per subtree batch (0 = auto) */
  int32_t streams;     /* hmat_multiply_batched: products in flight at once, each on its own
                          stream and host thread, 1..4 (0 = autotuned, default) */
  int32_t scheme;      /* low-rank scheme of the farfield targets, HMAT_SCHEME_* (default
                          HMAT_SCHEME_RANDOMIZED) */
  int32_t k_fixed;     /* 0 (default): eps-adaptive ranks; 1..64: fixed-rank mode (Section 4,
                          fixed rank approximation): ACA and Lanczos stop after k_fixed steps,
                          the randomized scheme runs Algorithm 9 with k_fixed columns; eps is
                          then not used for the farfield blocks */
  int32_t subspace_iters; /* q of Algorithm 9 (fixed-rank randomized scheme), 0..8 (default 1) */
  int32_t exact_lowrank;  /* 1: farfield targets whose sum-expression has no H-pairs left
                             (S_H empty) are truncated exactly by the SVD of their low-rank sum
                             (Algorithm 5) when it fits the 64-column panels; 0 (default): every
                             target uses `scheme` */
  int32_t full_passes; /* 0 (default): a pass over a chunk of targets in which at most an
                          eighth of them are active (a growth round, the later 16-column
                          identity panels of a chunk's widest targets) launches only the work
                          items of the active ones; each launched item computes what it computes
                          in a full pass, so results are bit-identical. 1: every pass launches
                          all work items of its chunk (inactive ones exit at once) */
} hmat_opts;

/* Low-rank schemes of Section 4 (hmat_opts.scheme). Every scheme touches a target's
 * sum-expression only through products S X and S^T X:
 *  HMAT_SCHEME_RANDOMIZED  blocked randomized range finder with the a-posteriori
 *                          residual check and adaptive growth (Algorithm 8 in blocked form),
 *                          or Algorithm 9 in fixed-rank mode;
 *  HMAT_SCHEME_ACA         adaptive cross approximation with partial pivoting
 *                          (Algorithm 6), stopping rule eq. (truncaca), recompressed by
 *                          Algorithm 5 to the eps-rank;
 *  HMAT_SCHEME_LANCZOS     Golub-Kahan-Lanczos bidiagonalization with reorthogonalization
 *                          (Algorithm 7), same stopping rule, SVD of the bidiagonal.
 * ACA and Lanczos take one matrix-vector product with S and one with S^T per step and
 * stop after at most 64 steps (HMAT_ERR_NOT_CONVERGED if a block needs more). Their
 * start values: ACA starts at the block's first row; Lanczos starts from column 0 of the
 * product's Gaussian matrix (opts.seed). */
enum { HMAT_SCHEME_RANDOMIZED = 0, HMAT_SCHEME_ACA = 1, HMAT_SCHEME_LANCZOS = 2 };

/* Fills *o with the defaults listed above. */
void hmat_opts_default(hmat_opts* o);

/* ------------------------------------------------------------------------ */
/* Assembly of kernel matrices                                              */
/* ------------------------------------------------------------------------ */

enum { HMAT_KERNEL_LAPLACE_4PI = 0, HMAT_KERNEL_INV_DIST = 1, HMAT_KERNEL_EXP = 2 };

typedef struct {
  int32_t kind;   /* 1/(4 pi r), 1/r or exp(-r) of r = ||x_i - x_j||_2 */
  int32_t pad;
  double diag;    /* entry used for i == j */
  double shift;   /* added to every diagonal entry */
} hmat_kernel;

/*
 * Assembles the kernel matrix on the tree's points as an H-matrix in the set
 * H(B, k) of Def. 2.6 (farfield leaves in the low-rank set R(tau x sigma, k),
 * nearfield leaves dense; the paper's inputs come from boundary elements, these
 * from point kernels). Nearfield
 * leaves dense, farfield leaves compressed on the device to relative Frobenius
 * tolerance eps_in per block (same randomized compression as the product,
 * applied to the kernel block evaluated on the fly).
 * Errors: HMAT_ERR_ARG (unknown kind, eps_in not in (0,1), NULL), device errors,
 * HMAT_ERR_NOT_CONVERGED with the result still returned.
 */
hmat_status hmat_assemble(hmat_tree t, const hmat_kernel* k, double eps_in, const hmat_opts* opts,
                          hmat* out);

/*
 * Builds an H-matrix on tree t from host data: for every leaf block i (in the
 * order of hmat_block_count/hmat_block_get) ranks[i] (farfield) and the leaf's
 * data at pool + offsets[i]: farfield L (rows x rank) then R (cols x rank),
 * nearfield the dense rows x cols block, all column-major.
 */
hmat_status hmat_from_blocks(hmat_tree t, const int32_t* ranks, const int64_t* offsets,
                             const double* pool, hmat* out);

hmat_status hmat_destroy(hmat M);

/* ------------------------------------------------------------------------ */
/* Product                                                                  */
/* ------------------------------------------------------------------------ */

/*
 * C = A B on the common block-cluster tree: Algorithm 4 (the product through
 * sum-expressions, Def. 3.1, restricted level by level by Algorithm 3), each
 * admissible leaf compressed by the scheme chosen in opts (Section 4), each
 * inadmissible leaf evaluated exactly (evaluate() in Algorithm 4; the
 * nearfield is S applied to the identity, as in the proof of Theorem 5.4).
 * For every farfield leaf the stored
 * rank-k factors satisfy ||(AB)[t,s] - L R^T||_F <= ~eps ||(AB)[t,s]||_F with k
 * close to the epsilon-rank; nearfield leaves are exact up to rounding.
 *  A, B   unmodified; they must share one tree (HMAT_ERR_TREE_MISMATCH).
 *  eps    in (0, 1), else HMAT_ERR_ARG.
 *  opts   nullable (defaults).
 *  C      receives a new H-matrix on the same tree.
 * If farfield blocks exhaust max_growth, C is still returned, their best
 * available factors are stored, stats->n_not_converged counts them,
 * hmat_block_get reports them with converged = 0, and the call returns
 * HMAT_ERR_NOT_CONVERGED.
 */
hmat_status hmat_multiply(hmat A, hmat B, double eps, const hmat_opts* opts, hmat* C);

/*
 * count independent products C[i] = A[i] B[i] (each pair on its own tree).
 * status (host int32[count], nullable) receives the per-product status; the
 * return value is the first non-OK status (HMAT_OK if all succeeded) and
 * hmat_last_error names the first failing product.
 * Products run concurrently: opts->streams host threads, each with its own
 * HIP stream (created and destroyed inside the call; opts->stream is not
 * used), take products in index order. With streams = 0 the count is
 * autotuned: the first products are run with 1, 2 and 4 streams (2 x
 * streams products each), the rate (algorithmic flops / wall time) of each
 * trial is compared, the best count runs the rest and is remembered for
 * later batches of the same size class (rounded mean log2 n). If
 * opts->stats is set it receives the sums over all products, with t_total
 * the wall time of the call and streams_used the count that ran the rest.
 * Each product in flight gets an equal share of the device memory for its
 * workspaces; a product that still runs out of memory next to others is run
 * again alone after the others (its status then reflects that run).
 * Known problem: on a batch of 64 products of 4096 to 65536 points, the call
 * after a first complete call has stopped making progress, for a reason not
 * yet found. Batches of a few products are tested.
 */
hmat_status hmat_multiply_batched(const hmat* A, const hmat* B, int32_t count, double eps,
                                  const hmat_opts* opts, hmat* C, int32_t* status);

/* ------------------------------------------------------------------------ */
/* H-matrix times vectors                                                   */
/* ------------------------------------------------------------------------ */

/*
 * y = M x (trans = 0) or y = M^T x (trans = 1) for a block of nvec vectors:
 * Algorithm 2 (HtimesV) run over the leaves of the block-cluster tree; every
 * farfield leaf contributes L (R^T x[sigma]), every nearfield leaf D x[sigma].
 * x and y are DEVICE memory, column-major n x nvec with leading dimensions
 * ldx, ldy >= n, rows in original point order (order = 0) or cluster order
 * (order = 1); y is overwritten and must not overlap x. The work is enqueued on
 * `stream` (hipStream_t, NULL = null stream) and the call returns without
 * waiting; y is complete when the stream passes this point. Each output entry
 * is summed by one thread in a fixed order, so results are deterministic.
 * Device scratch (one int64 per block plus nvec doubles per farfield rank
 * unit) comes from the library's allocator and is reused once the stream has
 * passed the call.
 * Errors: HMAT_ERR_ARG for NULL pointers, trans/order outside {0, 1},
 * nvec < 1, ldx or ldy < n, overlapping x and y, or a current device other
 * than the one M lives on.
 */
hmat_status hmat_matvec(hmat M, int32_t trans, int32_t order, int32_t nvec, const double* x, int64_t ldx,
                        double* y, int64_t ldy, void* stream);

/*
 * hmat_matvec for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments, results bit-identical to hmat_matvec, but the scratch lives in a
 * static device array of HMAT_MATVEC_NOALLOC_BYTES that each GPU the library
 * runs on holds until the process ends; no hipMalloc, hipFree or allocating
 * library routine is called. Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (on different streams, or from several host
 * threads without ordering) race and give wrong results. The tree's device copy
 * must already exist (any product, assembly or hmat_matvec on M creates it).
 * Errors: those of hmat_matvec, and HMAT_ERR_ARG when the scratch (8 bytes per
 * block of the tree plus 8 nvec bytes per farfield rank unit) exceeds
 * HMAT_MATVEC_NOALLOC_BYTES.
 */
#define HMAT_MATVEC_NOALLOC_BYTES (64LL << 20)
hmat_status hmat_matvec_noalloc(hmat M, int32_t trans, int32_t order, int32_t nvec, const double* x, int64_t ldx,
                                double* y, int64_t ldy, void* stream);

/*
 * Accuracy estimate of a product C ~ A B (the error estimator of the paper's
 * numerical examples): subspace iteration on E v = C v - A (B v), whose
 * products are three calls of Algorithm 2. From the start block X0 (DEVICE
 * memory, n x p column-major, cluster order, p in [1, n]; the caller draws it,
 * for instance Gaussian): repeat iters times Y = orth(E X), X = orth(E^T Y);
 * *err = ||E X||_F. *norm_ab is the same estimate for v -> A (B v) from the same
 * X0, so *err / *norm_ab estimates the relative error ||C - A B||_F / ||A B||_F
 * on the dominant p-dimensional subspaces. Runs on `stream` and returns when
 * both values are on the host. Device scratch: 4 n p doubles plus one matvec
 * scratch, from the library's allocator.
 * Errors: HMAT_ERR_ARG for NULL pointers, p outside [1, n], iters outside
 * [0, 100] or a current device other than the matrices'; HMAT_ERR_TREE_MISMATCH
 * unless C, A and B share one tree.
 */
hmat_status hmat_error_estimate(hmat C, hmat A, hmat B, const double* X0, int32_t p, int32_t iters, void* stream,
                                double* err, double* norm_ab);

/*
 * The Gaussian test matrix Omega of the randomized scheme (Section 4.3): entry
 * (i, j) is Box-Muller of one Philox4x32-10 block with counter (i mod 2^32, j,
 * i div 2^32, 0x0A11CE5) and key (seed mod 2^32, seed div 2^32), output words
 * w0..w3: a = (w0 2^21 xor w1 div 2^11) mod 2^53, b likewise from w2, w3,
 * u1 = (a + 1) 2^-53, u2 = b 2^-53, Omega(i, j) = sqrt(-2 ln u1) cos(2 pi u2).
 * Writes Omega(i, j) for i < n, j < ncol
 * into DEVICE memory out (n x ncol, column-major, leading dimension n) on `stream`
 * and returns when it is written. A product sketches the target block tau x sigma
 * with the rows of sigma's positions (cluster order) of this matrix, seeded by
 * opts.seed, so callers can reproduce its test vectors (for an error estimate on
 * the same stream, or to check the generator).
 * Errors: HMAT_ERR_ARG for a NULL out, negative sizes or n >= 2^38.
 */
hmat_status hmat_gaussian_panel(int64_t n, int32_t ncol, uint64_t seed, double* out, void* stream);

/* ------------------------------------------------------------------------ */
/* Export                                                                   */
/* ------------------------------------------------------------------------ */

/*
 * Dense n x n copy of M into host memory out (column-major, leading dimension
 * ld >= n); order 0 = original point order, 1 = cluster order. The leaves
 * (low-rank L R^T or dense, Def. 2.6) are expanded on the device in column
 * slabs of at most 1 GiB, then copied to out.
 * Errors: HMAT_ERR_ARG for NULL pointers, ld < n or an unknown order.
 */
hmat_status hmat_to_dense(hmat M, double* out, int64_t ld, int32_t order);

typedef struct {
  int64_t row_begin, rows, col_begin, cols;  /* positions in cluster order */
  int32_t level;
  int32_t kind;   /* 1 = farfield (low rank), 2 = nearfield (dense) */
  int32_t rank;   /* farfield rank, 0 for nearfield */
  int32_t block;  /* id in hmat_tree_blocks order */
  int32_t converged;  /* 0 for a farfield block of a product whose growth budget ran out, else 1 */
  int32_t pad;
} hmat_block_desc;

/* Number of leaf blocks (farfield + nearfield), breadth-first leaf order. */
hmat_status hmat_block_count(hmat M, int64_t* count);
/*
 * Leaf i: descriptor, and (if not NULL) its data in host memory: farfield
 * U (rows x rank) and V (cols x rank) with block = U V^T; nearfield the dense
 * rows x cols block in V_or_dense (U unused).
 */
hmat_status hmat_block_get(hmat M, int64_t i, hmat_block_desc* d, double* U, double* V_or_dense);
/*
 * Bulk export: ranks (host int32[count]), offsets (host int64[count], element
 * offsets into the pool) and, if pool is not NULL, the pool itself (host
 * float64[*pool_len]). Call first with pool = NULL to get *pool_len.
 */
hmat_status hmat_export(hmat M, int32_t* ranks, int64_t* offsets, double* pool, int64_t* pool_len);

/*
 * Algorithmic flops the product that computed M charged to each leaf as a
 * target (the work model of the cost analysis in Section 5, at the final ranks:
 * one forward and one transposed pass per farfield leaf plus its core
 * factorisation, S applied to the identity per nearfield leaf; the creation of
 * the low-rank terms is not charged to leaves). flops: host double[count] in
 * hmat_block_get order; all zero for a matrix that no product computed.
 */
hmat_status hmat_product_block_flops(hmat M, double* flops);

/* ------------------------------------------------------------------------ */
/* Learned rank predictor (multi-layer perceptron 6-64-64-64-1, ReLU, fp32) */
/* ------------------------------------------------------------------------ */

enum { HMAT_N_FEATURES = 6 };

typedef struct {
  int32_t epochs;      /* passes over the data (default 200) */
  int32_t batch;       /* minibatch size (default 256) */
  float lr;            /* Adam step size (default 1e-3) */
  float weight_decay;  /* default 0 */
  uint64_t seed;       /* init and shuffling (default 1) */
  void* stream;
  float* loss_out;     /* host float[epochs], nullable: mean loss per epoch */
} hmat_train_opts;

void hmat_train_opts_default(hmat_train_opts* o);

/* New model with seeded random weights (on the current device). */
hmat_status hmat_rank_model_create(uint64_t seed, hmat_rank_model* out);
hmat_status hmat_rank_model_destroy(hmat_rank_model m);
/*
 * Trains on m samples: feats host float[m * 6] row-major (level, log diam tau,
 * log diam sigma, log dist, input-rank sum, term count; raw, the model
 * standardises them), ranks host float[m]. Loss: mean squared error in the
 * rank. Forward, backward and Adam run on the device.
 */
hmat_status hmat_rank_model_train(hmat_rank_model model, const float* feats, const float* ranks,
                                  int64_t m, const hmat_train_opts* opts);
/* Inference: pred host float[m]. */
hmat_status hmat_rank_model_predict(hmat_rank_model model, const float* feats, int64_t m,
                                    float* pred, void* stream);
/* Model file (parameters and standardisation, little-endian float32 with a header). */
hmat_status hmat_rank_model_save(hmat_rank_model model, const char* path);
hmat_status hmat_rank_model_load(const char* path, hmat_rank_model* out);
/* Parameters as host floats (count via *len when params is NULL). */
hmat_status hmat_rank_model_get(hmat_rank_model model, float* params, int64_t* len);
hmat_status hmat_rank_model_set(hmat_rank_model model, const float* params, int64_t len);
/*
 * One forward+backward of the loss on a batch without updating: grads host
 * float[len] (same layout as hmat_rank_model_get), loss host float[1].
 */
hmat_status hmat_rank_model_grad(hmat_rank_model model, const float* feats, const float* ranks,
                                 int64_t m, float* grads, float* loss);
/*
 * Features and ranks of the farfield blocks of the last product computed with
 * a stats pointer into C (HMAT_RANK_ADAPTIVE): feats host float[n_far*6],
 * ranks host float[n_far]; *count receives n_far (call with NULL outputs to
 * query it).
 */
hmat_status hmat_product_features(hmat C, float* feats, float* ranks, int64_t* count);
/*
 * Sketch widths of the same blocks (same order as hmat_product_features): the
 * number of orthonormal sketch columns at which the residual check passed, the
 * width a first sketch must have to need no growth round. widths: host
 * float[n_far]; *count as above.
 */
hmat_status hmat_product_widths(hmat C, float* widths, int64_t* count);

#ifdef __cplusplus
}
#endif

#endif /* HMAT_H */
