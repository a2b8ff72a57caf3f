// Learned rank predictor: a multi-layer perceptron 6 -> 64 -> 64 -> 64 -> 1 with
// ReLU, in float32, with forward, backward and Adam kernels of its own. It maps a
// farfield target's features (level, log diam tau, log diam sigma, log dist,
// input-rank sum, term count) to its epsilon-rank, so that the randomized
// compression starts with a sketch of about the right width; the a-posteriori
// residual check of the compression stays in force and grows the sketch when a
// prediction is too small.
//
// Parameter layout (floats): W1 (64x6), b1 (64), W2 (64x64), b2 (64), W3 (64x64),
// b3 (64), W4 (1x64), b4 (1); W row-major (out x in). The model also keeps the
// feature means / standard deviations and the rank scale used in training.
#include <cmath>
#include <cstring>
#include <random>

#include "device_common.h"
#include "hmat_internal.h"

namespace hm {

constexpr int NF = HMAT_N_FEATURES, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH, OFF_W4 = OFF_B3 + NH, OFF_B4 = OFF_W4 + NH,
              NPARAM = OFF_B4 + 1;
constexpr int NNORM = 2 * NF + 2;  // feature mean, feature std, rank mean, rank std

struct RankModel {
  DevBuf<float> p, m, v, g;  // parameters, Adam moments, gradient
  std::vector<float> norm;   // NNORM floats
  int64_t step = 0;
};

// ---------------------------------------------------------------- kernels
// Y (n x NO) = act(X (n x NI) W^T + b), row-major rows = samples; act = ReLU if relu.
__global__ void k_dense_fwd(const float* __restrict__ X, int n, int ni, const float* __restrict__ W,
                            const float* __restrict__ b, int no, int relu, float* __restrict__ Y) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(n) * no) return;
  const int r = int(idx / no), o = int(idx % no);
  float acc = b[o];
  const float* x = X + int64_t(r) * ni;
  const float* wr = W + int64_t(o) * ni;
  for (int k = 0; k < ni; ++k) acc += wr[k] * x[k];
  Y[idx] = relu ? fmaxf(acc, 0.f) : acc;
}

// dX (n x ni) = (dY (n x no) W) masked by X > 0 when mask (ReLU of the previous layer)
__global__ void k_dense_bwd_x(const float* __restrict__ dY, int n, int no, const float* __restrict__ W, int ni,
                              const float* __restrict__ Xact, int mask, float* __restrict__ dX) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(n) * ni) return;
  const int r = int(idx / ni), k = int(idx % ni);
  float acc = 0.f;
  const float* dy = dY + int64_t(r) * no;
  for (int o = 0; o < no; ++o) acc += dy[o] * W[int64_t(o) * ni + k];
  if (mask && !(Xact[idx] > 0.f)) acc = 0.f;
  dX[idx] = acc;
}

// dW (no x ni) = dY^T X * scale, db (no) = column sums of dY * scale: one wave per
// output entry, lanes stride over the samples, fixed-order butterfly sum
__global__ void __launch_bounds__(256) k_dense_bwd_w(const float* __restrict__ dY, int n, int no,
                                                     const float* __restrict__ X, int ni, float scale,
                                                     float* __restrict__ dW, float* __restrict__ db) {
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int total = no * ni + no;
  if (idx >= total) return;
  float acc = 0.f;
  if (idx < no * ni) {
    const int o = idx / ni, k = idx % ni;
    for (int r = lane; r < n; r += 64) acc += dY[int64_t(r) * no + o] * X[int64_t(r) * ni + k];
  } else {
    const int o = idx - no * ni;
    for (int r = lane; r < n; r += 64) acc += dY[int64_t(r) * no + o];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) {
    if (idx < no * ni) dW[idx] = acc * scale;
    else db[idx - no * ni] = acc * scale;
  }
}

// standardised features: Z = (F - mean) / std
__global__ void k_standardise(const float* __restrict__ F, int n, const float* __restrict__ norm,
                              float* __restrict__ Z) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(n) * NF) return;
  const int k = int(idx % NF);
  Z[idx] = (F[idx] - norm[k]) / norm[NF + k];
}

// loss = mean (out - t)^2 on standardised ranks; dOut = 2 (out - t); per-sample squared error
__global__ void k_mse(const float* __restrict__ out, const float* __restrict__ t, int n,
                      const float* __restrict__ norm, float* __restrict__ dout, float* __restrict__ se) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float ts = (t[i] - norm[2 * NF]) / norm[2 * NF + 1];
  const float e = out[i] - ts;
  dout[i] = 2.f * e;
  se[i] = e * e;
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float c1, float c2,
                       float wd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i] + wd * p[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// prediction in rank units: out * std + mean
__global__ void k_unscale(const float* __restrict__ out, int n, const float* __restrict__ norm,
                          float* __restrict__ pred) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pred[i] = out[i] * norm[2 * NF + 1] + norm[2 * NF];
}

static unsigned nblk(int64_t n) { return unsigned((n + 255) / 256); }
static unsigned wblk(int64_t n) { return unsigned((n + 3) / 4); }  // one wave per item, 4 per block

// ---------------------------------------------------------------- host helpers
struct Work {
  DevBuf<float> Z, H1, H2, H3, O, dO, dH1, dH2, dH3, se, normd;
  int cap = 0;
  void ensure(int n) {
    if (n <= cap) return;
    cap = n;
    Z.alloc(size_t(n) * NF);
    H1.alloc(size_t(n) * NH);
    H2.alloc(size_t(n) * NH);
    H3.alloc(size_t(n) * NH);
    O.alloc(n);
    dO.alloc(n);
    dH1.alloc(size_t(n) * NH);
    dH2.alloc(size_t(n) * NH);
    dH3.alloc(size_t(n) * NH);
    se.alloc(n);
  }
};

static void forward(RankModel& M, Work& W, const float* F, int n, hipStream_t s) {
  const float* P = M.p.p;
  hipLaunchKernelGGL(k_standardise, dim3(nblk(int64_t(n) * NF)), dim3(256), 0, s, F, n, W.normd.p, W.Z.p);
  hipLaunchKernelGGL(k_dense_fwd, dim3(nblk(int64_t(n) * NH)), dim3(256), 0, s, W.Z.p, n, NF, P + OFF_W1, P + OFF_B1,
                     NH, 1, W.H1.p);
  hipLaunchKernelGGL(k_dense_fwd, dim3(nblk(int64_t(n) * NH)), dim3(256), 0, s, W.H1.p, n, NH, P + OFF_W2, P + OFF_B2,
                     NH, 1, W.H2.p);
  hipLaunchKernelGGL(k_dense_fwd, dim3(nblk(int64_t(n) * NH)), dim3(256), 0, s, W.H2.p, n, NH, P + OFF_W3, P + OFF_B3,
                     NH, 1, W.H3.p);
  hipLaunchKernelGGL(k_dense_fwd, dim3(nblk(n)), dim3(256), 0, s, W.H3.p, n, NH, P + OFF_W4, P + OFF_B4, 1, 0, W.O.p);
  HM_CHECK_HIP(hipGetLastError());
}

// gradient of the mean squared error over n samples into M.g; the samples' squared errors
// go to se
static void backward(RankModel& M, Work& W, const float* ranks, int n, float* se, hipStream_t s) {
  const float* P = M.p.p;
  float* G = M.g.p;
  const float sc = 1.f / float(n);
  hipLaunchKernelGGL(k_mse, dim3(nblk(n)), dim3(256), 0, s, W.O.p, ranks, n, W.normd.p, W.dO.p, se);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(wblk(NH + 1)), dim3(256), 0, s, W.dO.p, n, 1, W.H3.p, NH, sc, G + OFF_W4,
                     G + OFF_B4);
  hipLaunchKernelGGL(k_dense_bwd_x, dim3(nblk(int64_t(n) * NH)), dim3(256), 0, s, W.dO.p, n, 1, P + OFF_W4, NH, W.H3.p,
                     1, W.dH3.p);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(wblk(NH * NH + NH)), dim3(256), 0, s, W.dH3.p, n, NH, W.H2.p, NH, sc,
                     G + OFF_W3, G + OFF_B3);
  hipLaunchKernelGGL(k_dense_bwd_x, dim3(nblk(int64_t(n) * NH)), dim3(256), 0, s, W.dH3.p, n, NH, P + OFF_W3, NH,
                     W.H2.p, 1, W.dH2.p);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(wblk(NH * NH + NH)), dim3(256), 0, s, W.dH2.p, n, NH, W.H1.p, NH, sc,
                     G + OFF_W2, G + OFF_B2);
  hipLaunchKernelGGL(k_dense_bwd_x, dim3(nblk(int64_t(n) * NH)), dim3(256), 0, s, W.dH2.p, n, NH, P + OFF_W2, NH,
                     W.H1.p, 1, W.dH1.p);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(wblk(NH * NF + NH)), dim3(256), 0, s, W.dH1.p, n, NH, W.Z.p, NF, sc,
                     G + OFF_W1, G + OFF_B1);
  HM_CHECK_HIP(hipGetLastError());
}

static void init_model(RankModel& M, uint64_t seed) {
  std::vector<float> p(NPARAM, 0.f);
  std::mt19937_64 rng(seed);
  auto fill = [&](int off, int fan_in, int count) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.f / float(fan_in)));  // He initialisation
    for (int i = 0; i < count; ++i) p[off + i] = nd(rng);
  };
  fill(OFF_W1, NF, NH * NF);
  fill(OFF_W2, NH, NH * NH);
  fill(OFF_W3, NH, NH * NH);
  fill(OFF_W4, NH, NH);
  M.p.upload(p, 0);
  std::vector<float> z(NPARAM, 0.f);
  M.m.upload(z, 0);
  M.v.upload(z, 0);
  M.g.upload(z, 0);
  M.norm.assign(NNORM, 0.f);
  for (int k = 0; k < NF; ++k) M.norm[NF + k] = 1.f;
  M.norm[2 * NF + 1] = 1.f;
}

// inference for the product: widths from features (host in / host out)
void predict_ranks(hmat_rank_model model, const std::vector<float>& feats, std::vector<float>& out, hipStream_t s) {
  RankModel& M = *reinterpret_cast<RankModel*>(model);
  set_current_stream(s);
  const int n = int(feats.size() / NF);
  out.assign(n, 0.f);
  if (n == 0) return;
  Work W;
  W.ensure(n);
  W.normd.upload(M.norm, s);
  DevBuf<float> F;
  F.upload(feats, s);
  forward(M, W, F.p, n, s);
  DevBuf<float> pred(n);
  hipLaunchKernelGGL(k_unscale, dim3(nblk(n)), dim3(256), 0, s, W.O.p, n, W.normd.p, pred.p);
  HM_CHECK_HIP(hipGetLastError());
  HM_CHECK_HIP(hipMemcpyAsync(out.data(), pred.p, 4 * n, hipMemcpyDeviceToHost, s));
  HM_CHECK_HIP(hipStreamSynchronize(s));
}

}  // namespace hm

using namespace hm;

#define API_BEGIN try {
#define API_END                                  \
  }                                              \
  catch (const hm::Error& e) {                   \
    set_last_error(e.what());                    \
    return e.code;                               \
  }                                              \
  catch (const std::exception& e) {              \
    set_last_error(e.what());                    \
    return HMAT_ERR_INTERNAL;                    \
  }                                              \
  set_last_error("");                            \
  return HMAT_OK;

extern "C" {

void hmat_train_opts_default(hmat_train_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->epochs = 200;
  o->batch = 256;
  o->lr = 1e-3f;
  o->weight_decay = 0.f;
  o->seed = 1;
}

hmat_status hmat_rank_model_create(uint64_t seed, hmat_rank_model* out) {
  API_BEGIN
  HM_REQUIRE(out, HMAT_ERR_ARG, "out is NULL");
  set_current_stream(0);
  RankModel* M = new RankModel();
  M->p.alloc(NPARAM);
  M->m.alloc(NPARAM);
  M->v.alloc(NPARAM);
  M->g.alloc(NPARAM);
  init_model(*M, seed);
  HM_CHECK_HIP(hipDeviceSynchronize());
  *out = reinterpret_cast<hmat_rank_model>(M);
  API_END
}

hmat_status hmat_rank_model_destroy(hmat_rank_model m) {
  API_BEGIN
  delete reinterpret_cast<RankModel*>(m);
  API_END
}

hmat_status hmat_rank_model_get(hmat_rank_model m, float* params, int64_t* len) {
  API_BEGIN
  HM_REQUIRE(m && len, HMAT_ERR_ARG, "NULL argument");
  RankModel& M = *reinterpret_cast<RankModel*>(m);
  const int64_t total = NPARAM + NNORM;
  if (params) {
    HM_REQUIRE(*len >= total, HMAT_ERR_ARG, "params buffer too small");
    HM_CHECK_HIP(hipMemcpy(params, M.p.p, 4 * NPARAM, hipMemcpyDeviceToHost));
    std::memcpy(params + NPARAM, M.norm.data(), 4 * NNORM);
  }
  *len = total;
  API_END
}

hmat_status hmat_rank_model_set(hmat_rank_model m, const float* params, int64_t len) {
  API_BEGIN
  HM_REQUIRE(m && params, HMAT_ERR_ARG, "NULL argument");
  HM_REQUIRE(len == NPARAM + NNORM, HMAT_ERR_ARG, "wrong parameter count");
  RankModel& M = *reinterpret_cast<RankModel*>(m);
  M.p.upload(params, NPARAM, 0);
  M.norm.assign(params + NPARAM, params + NPARAM + NNORM);
  API_END
}

hmat_status hmat_rank_model_grad(hmat_rank_model m, const float* feats, const float* ranks, int64_t n, float* grads,
                                 float* loss) {
  API_BEGIN
  HM_REQUIRE(m && feats && ranks && grads && loss && n > 0, HMAT_ERR_ARG, "bad argument");
  RankModel& M = *reinterpret_cast<RankModel*>(m);
  hipStream_t s = 0;
  set_current_stream(s);
  Work W;
  W.ensure(int(n));
  W.normd.upload(M.norm, s);
  DevBuf<float> F, R;
  F.upload(feats, size_t(n) * NF, s);
  R.upload(ranks, size_t(n), s);
  forward(M, W, F.p, int(n), s);
  backward(M, W, R.p, int(n), W.se.p, s);
  std::vector<float> se(n);
  HM_CHECK_HIP(hipMemcpy(grads, M.g.p, 4 * NPARAM, hipMemcpyDeviceToHost));
  HM_CHECK_HIP(hipMemcpy(se.data(), W.se.p, 4 * n, hipMemcpyDeviceToHost));
  double acc = 0;
  for (float e : se) acc += e;
  *loss = float(acc / double(n));
  for (int i = NPARAM; i < NPARAM + NNORM; ++i) grads[i] = 0.f;
  API_END
}

hmat_status hmat_rank_model_train(hmat_rank_model m, const float* feats, const float* ranks, int64_t n,
                                  const hmat_train_opts* opts) {
  API_BEGIN
  HM_REQUIRE(m && feats && ranks && n > 0, HMAT_ERR_ARG, "bad argument");
  hmat_train_opts o;
  hmat_train_opts_default(&o);
  if (opts) o = *opts;
  HM_REQUIRE(o.epochs >= 0 && o.batch >= 1, HMAT_ERR_ARG, "bad training options");
  RankModel& M = *reinterpret_cast<RankModel*>(m);
  hipStream_t s = reinterpret_cast<hipStream_t>(o.stream);
  set_current_stream(s);
  // standardisation from the training data
  std::vector<double> mean(NF, 0), var(NF, 0);
  double rm = 0, rv = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < NF; ++k) mean[k] += feats[i * NF + k];
    rm += ranks[i];
  }
  for (int k = 0; k < NF; ++k) mean[k] /= double(n);
  rm /= double(n);
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < NF; ++k) var[k] += (feats[i * NF + k] - mean[k]) * (feats[i * NF + k] - mean[k]);
    rv += (ranks[i] - rm) * (ranks[i] - rm);
  }
  for (int k = 0; k < NF; ++k) {
    M.norm[k] = float(mean[k]);
    M.norm[NF + k] = float(std::max(1e-6, std::sqrt(var[k] / double(n))));
  }
  M.norm[2 * NF] = float(rm);
  M.norm[2 * NF + 1] = float(std::max(1e-6, std::sqrt(rv / double(n))));
  const int B = int(std::min<int64_t>(o.batch, n));
  Work W;
  W.ensure(B);
  W.normd.upload(M.norm, s);
  // Shuffled minibatches (deterministic for a seed): an epoch's samples are gathered on the
  // host in shuffled order and uploaded once, and its per-sample squared errors are read back
  // once, so the minibatches' launches run back to back with no synchronisation between them.
  std::mt19937_64 rng(o.seed);
  std::vector<int64_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  const size_t ns = static_cast<size_t>(n);
  std::vector<float> fe(ns * NF), re(ns), see(ns);
  DevBuf<float> Fe(ns * NF), Re(ns), Se(ns);
  const float b1 = 0.9f, b2 = 0.999f;
  for (int ep = 0; ep < o.epochs; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    for (int64_t i = 0; i < n; ++i) {
      std::memcpy(&fe[size_t(i) * NF], feats + perm[i] * NF, 4 * NF);
      re[size_t(i)] = ranks[perm[i]];
    }
    // synchronous copies: the previous epoch's kernels, which read these buffers, come
    // before them on the stream
    Fe.upload(fe.data(), size_t(n) * NF, s);
    Re.upload(re.data(), size_t(n), s);
    int64_t ep_cnt = 0;
    for (int64_t st = 0; st + B <= n || (st < n && st == 0); st += B) {
      const int nb = int(std::min<int64_t>(B, n - st));
      forward(M, W, Fe.p + st * NF, nb, s);
      backward(M, W, Re.p + st, nb, Se.p + st, s);
      ++M.step;
      const float c1 = 1.f - std::pow(b1, float(M.step)), c2 = 1.f - std::pow(b2, float(M.step));
      hipLaunchKernelGGL(k_adam, dim3(nblk(NPARAM)), dim3(256), 0, s, M.p.p, M.m.p, M.v.p, M.g.p, NPARAM, o.lr, b1,
                         b2, c1, c2, o.weight_decay);
      HM_CHECK_HIP(hipGetLastError());
      ep_cnt += nb;
    }
    if (o.loss_out) {
      HM_CHECK_HIP(hipMemcpyAsync(see.data(), Se.p, 4 * size_t(ep_cnt), hipMemcpyDeviceToHost, s));
      HM_CHECK_HIP(hipStreamSynchronize(s));
      double ep_loss = 0;
      for (int64_t i = 0; i < ep_cnt; ++i) ep_loss += see[size_t(i)];  // minibatch order, as they ran
      o.loss_out[ep] = float(ep_loss / double(std::max<int64_t>(ep_cnt, 1)));
    }
  }
  HM_CHECK_HIP(hipStreamSynchronize(s));
  API_END
}

hmat_status hmat_rank_model_predict(hmat_rank_model m, const float* feats, int64_t n, float* pred, void* stream) {
  API_BEGIN
  HM_REQUIRE(m && feats && pred && n >= 0, HMAT_ERR_ARG, "bad argument");
  std::vector<float> f(feats, feats + n * NF), out;
  predict_ranks(m, f, out, reinterpret_cast<hipStream_t>(stream));
  std::memcpy(pred, out.data(), 4 * n);
  API_END
}

static const char kModelMagic[8] = {'H', 'M', 'R', 'K', 'M', 'L', 'P', '1'};

hmat_status hmat_rank_model_save(hmat_rank_model m, const char* path) {
  API_BEGIN
  HM_REQUIRE(m && path, HMAT_ERR_ARG, "NULL argument");
  RankModel& M = *reinterpret_cast<RankModel*>(m);
  std::vector<float> p(NPARAM + NNORM);
  HM_CHECK_HIP(hipMemcpy(p.data(), M.p.p, 4 * NPARAM, hipMemcpyDeviceToHost));
  std::memcpy(p.data() + NPARAM, M.norm.data(), 4 * NNORM);
  FILE* f = std::fopen(path, "wb");
  HM_REQUIRE(f, HMAT_ERR_ARG, std::string("cannot open ") + path);
  const int32_t cnt = NPARAM + NNORM;
  const bool ok = std::fwrite(kModelMagic, 1, 8, f) == 8 && std::fwrite(&cnt, 4, 1, f) == 1 &&
                  std::fwrite(p.data(), 4, p.size(), f) == p.size();
  std::fclose(f);
  HM_REQUIRE(ok, HMAT_ERR_ARG, std::string("write failed: ") + path);
  API_END
}

hmat_status hmat_rank_model_load(const char* path, hmat_rank_model* out) {
  API_BEGIN
  HM_REQUIRE(path && out, HMAT_ERR_ARG, "NULL argument");
  FILE* f = std::fopen(path, "rb");
  HM_REQUIRE(f, HMAT_ERR_ARG, std::string("cannot open ") + path);
  char magic[8] = {};
  int32_t cnt = 0;
  std::vector<float> p(NPARAM + NNORM);
  const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kModelMagic, 8) == 0 &&
                  std::fread(&cnt, 4, 1, f) == 1 && cnt == NPARAM + NNORM &&
                  std::fread(p.data(), 4, p.size(), f) == p.size();
  std::fclose(f);
  HM_REQUIRE(ok, HMAT_ERR_ARG, std::string("not a rank model file: ") + path);
  hmat_rank_model m = nullptr;
  const hmat_status st = hmat_rank_model_create(0, &m);
  if (st != HMAT_OK) return st;
  RankModel& M = *reinterpret_cast<RankModel*>(m);
  M.p.upload(p.data(), NPARAM, 0);
  M.norm.assign(p.begin() + NPARAM, p.end());
  *out = m;
  API_END
}

hmat_status hmat_product_features(hmat C, float* feats, float* ranks, int64_t* count) {
  API_BEGIN
  HM_REQUIRE(C && count, HMAT_ERR_ARG, "NULL argument");
  const ProductFeatures& pf = reinterpret_cast<HMat*>(C)->features;
  const int64_t nf = int64_t(pf.ranks.size());
  if (feats) std::memcpy(feats, pf.feats.data(), 4 * pf.feats.size());
  if (ranks) std::memcpy(ranks, pf.ranks.data(), 4 * nf);
  *count = nf;
  API_END
}

hmat_status hmat_product_widths(hmat C, float* widths, int64_t* count) {
  API_BEGIN
  HM_REQUIRE(C && count, HMAT_ERR_ARG, "NULL argument");
  const ProductFeatures& pf = reinterpret_cast<HMat*>(C)->features;
  const int64_t nf = int64_t(pf.widths.size());
  if (widths) std::memcpy(widths, pf.widths.data(), 4 * nf);
  *count = nf;
  API_END
}

}  // extern "C"
