// Per-target step kernels of ACA (Algorithm 6), Lanczos bidiagonalization
// (Algorithm 7) and the randomized rank-k scheme (Algorithm 9), and their final
// recompression. One workgroup of 256 threads per target; vectors and panels
// stay in global memory (a target's panels are a few hundred KB at most and stay
// in L2 while its workgroup runs). The operator passes between these kernels are
// the product's apply kernels.
#include <algorithm>
#include <climits>

#include "device_common.h"
#include "schemes.h"

namespace hm {

namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;

struct Best {
  double a;  // |value|
  int i;     // index (smallest on ties)
  double v;  // signed value
};

__device__ __forceinline__ Best better(Best x, Best y) { return (y.a > x.a || (y.a == x.a && y.i < x.i)) ? y : x; }

__device__ Best block_argmax(Best b, Best* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    Best y;
    y.a = __shfl_xor(b.a, o, WAVE);
    y.i = __shfl_xor(b.i, o, WAVE);
    y.v = __shfl_xor(b.v, o, WAVE);
    b = better(b, y);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = b;
  __syncthreads();
  Best r = sh[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) r = better(r, sh[k]);
  return r;
}

// h[j] = Q[:, j] . v for j < r (Q with ld rows), one wave per column.
__device__ void dots(const double* Q, int rows, int r, const double* v, double* h) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = w; j < r; j += NW) {
    const double* q = Q + int64_t(j) * rows;
    double acc = 0.0;
    for (int i = lane; i < rows; i += 64) acc += q[i] * v[i];
    acc = wave_sum(acc);
    if (lane == 0) h[j] = acc;
  }
  __syncthreads();
}

// v -= Q[:, :r] h
__device__ void subtract(const double* Q, int rows, int r, const double* h, double* v) {
  for (int i = threadIdx.x; i < rows; i += NT) {
    double acc = v[i];
    for (int j = 0; j < r; ++j) acc -= Q[int64_t(j) * rows + i] * h[j];
    v[i] = acc;
  }
  __syncthreads();
}

__device__ double sumsq(const double* v, int rows, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < rows; i += NT) acc += v[i] * v[i];
  return block_sum<NT>(acc, red);
}

// two passes of classical Gram-Schmidt of v against Q[:, :r]
__device__ void reorth(const double* Q, int rows, int r, double* v, double* h) {
  for (int pass = 0; pass < 2; ++pass) {
    dots(Q, rows, r, v, h);
    subtract(Q, rows, r, h, v);
  }
}

__device__ __forceinline__ double* core_of(const ITarget& T) { return T.work; }
__device__ __forceinline__ double* jrot_of(const ITarget& T, int cap) { return T.work + cap * cap; }
__device__ __forceinline__ double* sigma_of(const ITarget& T, int cap) { return T.work + 2 * cap * cap; }
__device__ __forceinline__ double* alpha_of(const ITarget& T, int cap) { return T.work + 2 * cap * cap + cap; }
__device__ __forceinline__ double* beta_of(const ITarget& T, int cap) { return T.work + 2 * cap * cap + 2 * cap; }

// ---------------------------------------------------------------- ACA
__global__ void __launch_bounds__(NT) k_aca_init(ITarget* __restrict__ tg) {
  ITarget& T = tg[blockIdx.x];
  for (int i = threadIdx.x; i < T.n; i += NT) T.xf[i] = 0.0;
  for (int i = threadIdx.x; i < T.m; i += NT) {
    T.xt[i] = i == 0 ? 1.0 : 0.0;
    T.used[i] = 0;
  }
  if (threadIdx.x == 0) {
    T.r = 0;
    T.state = T.lim == 0 ? 1 : 0;
    T.pi = 0;
    T.pj = -1;
    T.nrm2 = 0.0;
    T.e2 = 0.0;
  }
}

__global__ void __launch_bounds__(NT) k_aca_row(ITarget* __restrict__ tg, int cap) {
  __shared__ double h[ISCHEME_CAP];
  __shared__ Best sh[NW];
  ITarget& T = tg[blockIdx.x];
  if (T.state != 0) return;
  const int m = T.m, n = T.n, r = T.r, pi = T.pi;
  double* u = T.U + int64_t(r) * n;
  for (int j = threadIdx.x; j < r; j += NT) h[j] = T.L[int64_t(j) * m + pi];
  __syncthreads();
  Best b{-1.0, INT_MAX, 0.0};
  for (int c = threadIdx.x; c < n; c += NT) {
    double v = T.yt[c];
    for (int j = 0; j < r; ++j) v -= h[j] * T.U[int64_t(j) * n + c];
    u[c] = v;
    b = better(b, Best{fabs(v), c, v});
  }
  b = block_argmax(b, sh);
  if (threadIdx.x == 0) T.used[pi] = 1;
  if (b.v == 0.0 || b.i >= n) {  // the residual row is zero: no pivot left
    if (threadIdx.x == 0) T.state = 1;
    return;
  }
  const double piv = b.v;
  for (int c = threadIdx.x; c < n; c += NT) u[c] = u[c] / piv;
  const int old = T.pj;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (old >= 0) T.xf[old] = 0.0;
    T.xf[b.i] = 1.0;
    T.pj = b.i;
  }
}

__global__ void __launch_bounds__(NT) k_aca_col(ITarget* __restrict__ tg, int cap, int fixed, double eps,
                                                int32_t* __restrict__ state_out) {
  __shared__ double h[ISCHEME_CAP];
  __shared__ double dl[ISCHEME_CAP], du[ISCHEME_CAP];
  __shared__ double red[NW];
  __shared__ Best sh[NW];
  ITarget& T = tg[blockIdx.x];
  if (T.state != 0) {
    if (threadIdx.x == 0) state_out[blockIdx.x] = T.state;
    return;
  }
  const int m = T.m, n = T.n, r = T.r, pj = T.pj;
  double* l = T.L + int64_t(r) * m;
  const double* u = T.U + int64_t(r) * n;
  for (int j = threadIdx.x; j < r; j += NT) h[j] = T.U[int64_t(j) * n + pj];
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += NT) {
    double v = T.yf[i];
    for (int j = 0; j < r; ++j) v -= h[j] * T.L[int64_t(j) * m + i];
    l[i] = v;
  }
  __syncthreads();
  const double nl = sumsq(l, m, red);
  const double nu = sumsq(u, n, red);
  if (!fixed && nl * nu <= eps * eps * T.nrm2) {
    if (threadIdx.x == 0) {
      T.e2 = nl * nu;
      T.state = 1;
      state_out[blockIdx.x] = 1;
    }
    return;
  }
  dots(T.L, m, r, l, dl);
  dots(T.U, n, r, u, du);
  double cross = 0.0;
  for (int j = 0; j < r; ++j) cross += dl[j] * du[j];
  const int r1 = r + 1;
  int st = 0;
  if (r1 == T.lim) st = (fixed || r1 == min(m, n)) ? 1 : 2;
  // next row pivot: largest |l_i| among the rows not used yet
  Best b{-1.0, INT_MAX, 0.0};
  if (st == 0)
    for (int i = threadIdx.x; i < m; i += NT)
      if (!T.used[i]) b = better(b, Best{fabs(l[i]), i, l[i]});
  b = block_argmax(b, sh);
  if (threadIdx.x == 0) {
    T.nrm2 += 2.0 * cross + nl * nu;
    T.r = r1;
    if (st == 0 && b.i < m) {
      T.xt[T.pi] = 0.0;
      T.xt[b.i] = 1.0;
      T.pi = b.i;
    } else if (st == 0) {
      st = 1;  // every row used
    }
    T.state = st;
    state_out[blockIdx.x] = st;
  }
}

// CGS2 QR of the r columns of P (rows x r) in place; R (upper, r x r) into R with ld ldr.
__device__ void qr_inplace(double* P, int rows, int r, double* R, int ldr, double* h, double* red) {
  for (int j = 0; j < r; ++j) {
    double* v = P + int64_t(j) * rows;
    for (int i = threadIdx.x; i < r; i += NT) R[int64_t(j) * ldr + i] = 0.0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      dots(P, rows, j, v, h);
      if (threadIdx.x < j) R[int64_t(j) * ldr + threadIdx.x] += h[threadIdx.x];
      __syncthreads();
      subtract(P, rows, j, h, v);
    }
    const double d2 = sumsq(v, rows, red);
    const double d = sqrt(d2);
    const double inv = d > 0.0 ? 1.0 / d : 0.0;
    for (int i = threadIdx.x; i < rows; i += NT) v[i] *= inv;
    if (threadIdx.x == 0) R[int64_t(j) * ldr + j] = d;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(NT) k_aca_core(ITarget* __restrict__ tg, int cap) {
  __shared__ double h[ISCHEME_CAP];
  __shared__ double red[NW];
  __shared__ double Ms[ISCHEME_CAP * ISCHEME_CAP];
  ITarget& T = tg[blockIdx.x];
  const int r = T.r;
  if (r == 0) return;
  // R_L into the J area and R_U into the core area (both r x r, ld r), then the core
  // M = R_L R_U^T through LDS into the core area
  double* RL = jrot_of(T, cap);
  double* RU = core_of(T);
  qr_inplace(T.L, T.m, r, RL, r, h, red);
  qr_inplace(T.U, T.n, r, RU, r, h, red);
  for (int idx = threadIdx.x; idx < r * r; idx += NT) {
    const int i = idx % r, j = idx / r;
    double acc = 0.0;  // (R_L R_U^T)(i, j) = sum_c R_L(i, c) R_U(j, c), both upper triangular
    for (int c = max(i, j); c < r; ++c) acc += RL[int64_t(c) * r + i] * RU[int64_t(c) * r + j];
    Ms[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < r * r; idx += NT) RU[idx] = Ms[idx];
}

// ---------------------------------------------------------------- Lanczos
__global__ void __launch_bounds__(NT) k_gkl_init(ITarget* __restrict__ tg, const double* __restrict__ om) {
  __shared__ double red[NW];
  ITarget& T = tg[blockIdx.x];
  const int n = T.n;
  const double* w = om + T.col0;
  const double s2 = sumsq(w, n, red);
  const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double v = w[i] * inv;
    T.U[i] = v;
    T.xf[i] = v;
  }
  if (threadIdx.x == 0) {
    T.r = 0;
    T.state = (T.lim == 0 || s2 == 0.0) ? 1 : 0;
    T.nrm2 = 0.0;
    T.e2 = 0.0;
    T.beta_prev = 0.0;
  }
}

__global__ void __launch_bounds__(NT) k_gkl_fwd(ITarget* __restrict__ tg, int cap, int fixed, double eps) {
  __shared__ double h[ISCHEME_CAP];
  __shared__ double red[NW];
  ITarget& T = tg[blockIdx.x];
  if (T.state != 0) return;
  const int m = T.m, r = T.r;
  double* q = T.L + int64_t(r) * m;  // candidate column (kept only if the step is)
  const double bp = T.beta_prev;
  for (int i = threadIdx.x; i < m; i += NT) q[i] = T.yf[i] - (r > 0 ? bp * T.L[int64_t(r - 1) * m + i] : 0.0);
  __syncthreads();
  reorth(T.L, m, r, q, h);
  const double a2 = sumsq(q, m, red);
  const double a = sqrt(a2);
  const double upd2 = a2 + bp * bp;
  if ((!fixed && upd2 <= eps * eps * T.nrm2) || a == 0.0) {
    if (threadIdx.x == 0) {
      T.e2 = upd2;
      T.state = 1;
    }
    return;
  }
  const double inv = 1.0 / a;
  for (int i = threadIdx.x; i < m; i += NT) {
    const double v = q[i] * inv;
    q[i] = v;
    T.xt[i] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    alpha_of(T, cap)[r] = a;
    T.nrm2 += upd2;
    T.r = r + 1;
    if (fixed && r + 1 == T.lim) T.state = 1;
  }
}

__global__ void __launch_bounds__(NT) k_gkl_bwd(ITarget* __restrict__ tg, int cap, int fixed,
                                                int32_t* __restrict__ state_out) {
  __shared__ double h[ISCHEME_CAP + 1];
  __shared__ double red[NW];
  ITarget& T = tg[blockIdx.x];
  if (T.state != 0) {
    if (threadIdx.x == 0) state_out[blockIdx.x] = T.state;
    return;
  }
  const int n = T.n, r = T.r;  // r >= 1: the forward step of this round was kept
  double* w = T.U + int64_t(r) * n;
  const double a = alpha_of(T, cap)[r - 1];
  for (int i = threadIdx.x; i < n; i += NT) w[i] = T.yt[i] - a * T.U[int64_t(r - 1) * n + i];
  __syncthreads();
  reorth(T.U, n, r, w, h);
  const double b2 = sumsq(w, n, red);
  const double b = sqrt(b2);
  if (r == T.lim) {
    if (threadIdx.x == 0) {
      T.e2 = fixed ? 0.0 : b2;
      T.state = (fixed || r == min(T.m, n)) ? 1 : 2;
      state_out[blockIdx.x] = T.state;
    }
    return;
  }
  if (b == 0.0) {
    if (threadIdx.x == 0) {
      T.state = 1;
      state_out[blockIdx.x] = 1;
    }
    return;
  }
  const double inv = 1.0 / b;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double v = w[i] * inv;
    w[i] = v;
    T.xf[i] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    beta_of(T, cap)[r - 1] = b;
    T.beta_prev = b;
    state_out[blockIdx.x] = 0;
  }
}

__global__ void __launch_bounds__(NT) k_gkl_core(ITarget* __restrict__ tg, int cap) {
  ITarget& T = tg[blockIdx.x];
  const int r = T.r;
  double* M = core_of(T);
  for (int idx = threadIdx.x; idx < r * r; idx += NT) {
    const int i = idx % r, j = idx / r;
    M[idx] = i == j ? alpha_of(T, cap)[i] : (j == i + 1 ? beta_of(T, cap)[i] : 0.0);
  }
}

// ---------------------------------------------------------------- final SVD and output
constexpr int JACOBI_SWEEPS = 60;

// One-sided Jacobi on the columns of the r x r core M (ld r): M J = W with orthogonal
// columns, their norms the singular values. Columns are sorted by norm, and the rank
// is the smallest k with tail(k)^2 <= eps^2 sum sigma^2 - e2 (fixed mode: k = r).
// W (sorted) replaces the core, J (sorted) goes to the J area, sigma to the sigma area.
// M and J live in dynamic LDS of 2 LD^2 doubles, LD = the launch's largest r.
__global__ void __launch_bounds__(NT) k_iter_svd(ITarget* __restrict__ tg, int cap, int fixed, double eps, int LD) {
  extern __shared__ double dyn[];
  double* M = dyn;
  double* J = dyn + LD * LD;
  __shared__ double sig[ISCHEME_CAP];
  __shared__ int order[ISCHEME_CAP];
  ITarget& T = tg[blockIdx.x];
  const int r = min(T.r, LD);  // the host sizes LD as the largest r
  if (r == 0) {
    if (threadIdx.x == 0) {
      T.k = 0;
      T.svd_sweeps = 0;
    }
    return;
  }
  const double* src = core_of(T);
  for (int idx = threadIdx.x; idx < r * r; idx += NT) {
    M[idx] = src[idx];
    J[idx] = (idx % r) == (idx / r) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double total = 0.0;
    for (int j = 0; j < r; ++j) {
      const double x = lane < r ? M[j * r + lane] : 0.0;
      total += wave_uniform(wave_sum(x * x));
    }
    int sweeps = -1;
    for (int sweep = 0; sweep < JACOBI_SWEEPS; ++sweep) {
      int rotated = 0;
      for (int p = 0; p < r - 1; ++p)
        for (int q = p + 1; q < r; ++q) {
          const double mp = lane < r ? M[p * r + lane] : 0.0;
          const double mq = lane < r ? M[q * r + lane] : 0.0;
          // one rotation for the whole wave: the angle must not differ between lanes
          const double a = wave_uniform(wave_sum(mp * mp)), b = wave_uniform(wave_sum(mq * mq)),
                       c = wave_uniform(wave_sum(mp * mq));
          // converged pair: orthogonal to working precision, or both columns at the
          // rounding level of the whole core
          if (c == 0.0 || fabs(c) <= 1e-15 * sqrt(a * b) || fabs(c) <= 1e-32 * total) continue;
          rotated = 1;
          const double zeta = (b - a) / (2.0 * c);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          if (lane < r) {
            M[p * r + lane] = cs * mp - sn * mq;
            M[q * r + lane] = sn * mp + cs * mq;
            const double jp = J[p * r + lane], jq = J[q * r + lane];
            J[p * r + lane] = cs * jp - sn * jq;
            J[q * r + lane] = sn * jp + cs * jq;
          }
        }
      if (!rotated) {
        sweeps = sweep + 1;
        break;
      }
    }
    for (int j = 0; j < r; ++j) {
      const double x = lane < r ? M[j * r + lane] : 0.0;
      const double s2 = wave_sum(x * x);
      if (lane == 0) sig[j] = sqrt(s2);
    }
    if (lane == 0) {
      for (int j = 0; j < r; ++j) order[j] = j;
      for (int a = 1; a < r; ++a) {  // insertion sort, descending
        const int x = order[a];
        int b = a - 1;
        while (b >= 0 && sig[order[b]] < sig[x]) {
          order[b + 1] = order[b];
          --b;
        }
        order[b + 1] = x;
      }
      double s2 = 0.0;
      for (int j = 0; j < r; ++j) s2 += sig[j] * sig[j];
      int k = r;
      if (!fixed) {
        const double budget = eps * eps * s2 - T.e2;
        double tail = 0.0;
        for (int kk = r; kk >= 0; --kk) {
          if (kk < r) tail += sig[order[kk]] * sig[order[kk]];
          if (budget >= 0.0 && tail <= budget) k = kk;
          else break;
        }
      }
      T.k = k;
      T.svd_sweeps = sweeps;
    }
  }
  __syncthreads();
  double* W = core_of(T);
  double* Jo = jrot_of(T, cap);
  double* so = sigma_of(T, cap);
  for (int idx = threadIdx.x; idx < r * r; idx += NT) {
    const int j = idx / r, i = idx % r;
    const int s = order[j];
    W[idx] = M[s * r + i];
    Jo[idx] = J[s * r + i];
  }
  for (int j = threadIdx.x; j < r; j += NT) so[j] = sig[order[j]];
}

__global__ void __launch_bounds__(NT) k_iter_write(const ITarget* __restrict__ tg, int cap,
                                                   double* __restrict__ pool) {
  const ITarget& T = tg[blockIdx.x];
  const int m = T.m, n = T.n, r = T.r, k = T.k;
  if (k == 0) return;
  const double* W = T.work;
  const double* J = T.work + cap * cap;
  double* L = pool + T.out_off;
  double* R = L + int64_t(m) * k;
  for (int i = threadIdx.x; i < m; i += NT)
    for (int c = 0; c < k; ++c) {
      double acc = 0.0;
      for (int j = 0; j < r; ++j) acc += T.L[int64_t(j) * m + i] * W[c * r + j];
      L[int64_t(c) * m + i] = acc;
    }
  for (int i = threadIdx.x; i < n; i += NT)
    for (int c = 0; c < k; ++c) {
      double acc = 0.0;
      for (int j = 0; j < r; ++j) acc += T.U[int64_t(j) * n + i] * J[c * r + j];
      R[int64_t(c) * n + i] = acc;
    }
}

// ---------------------------------------------------------------- Algorithm 9
__global__ void __launch_bounds__(NT) k_orth_cols(ITarget* __restrict__ tg, int side, int cnt,
                                                  int32_t* __restrict__ counts_out) {
  __shared__ double h[ISCHEME_CAP];
  __shared__ double red[NW];
  ITarget& T = tg[blockIdx.x];
  const int rows = side == 0 ? T.m : T.n;
  double* P = side == 0 ? T.L : T.U;
  const int c_in = cnt > 0 ? cnt : (side == 0 ? T.rz : T.r);  // input count: the other side's
  int r = 0;
  for (int c = 0; c < c_in; ++c) {
    double* v = P + int64_t(c) * rows;
    const double n0 = sumsq(v, rows, red);
    reorth(P, rows, r, v, h);
    const double n1 = sumsq(v, rows, red);
    const bool keep = r < ISCHEME_CAP && n1 > 0.0 && n1 > 1e-26 * n0;  // relative residual > 1e-13
    if (keep) {
      const double inv = 1.0 / sqrt(n1);
      double* dst = P + int64_t(r) * rows;
      for (int i = threadIdx.x; i < rows; i += NT) dst[i] = v[i] * inv;
      __syncthreads();
      ++r;
    }
  }
  if (threadIdx.x == 0) {
    if (side == 0) T.r = r;
    else T.rz = r;
    counts_out[blockIdx.x] = r;
  }
}

__global__ void __launch_bounds__(NT) k_copy_out(ITarget* __restrict__ tg, double* __restrict__ pool) {
  ITarget& T = tg[blockIdx.x];
  const int m = T.m, n = T.n, k = T.r;
  double* L = pool + T.out_off;
  double* R = L + int64_t(m) * k;
  for (int64_t i = threadIdx.x; i < int64_t(m) * k; i += NT) L[i] = T.L[i];
  for (int64_t i = threadIdx.x; i < int64_t(n) * k; i += NT) R[i] = T.U[i];
}

}  // namespace

#define LAUNCH(kern, nt, ...)                                                     \
  do {                                                                            \
    if ((nt) <= 0) return;                                                        \
    hipLaunchKernelGGL(kern, dim3(unsigned(nt)), dim3(NT), 0, s, __VA_ARGS__);    \
    HM_CHECK_HIP(hipGetLastError());                                              \
  } while (0)

void launch_aca_init(ITarget* t, int nt, hipStream_t s) { LAUNCH(k_aca_init, nt, t); }
void launch_aca_row(ITarget* t, int nt, const IParams& p, hipStream_t s) { LAUNCH(k_aca_row, nt, t, p.cap); }
void launch_aca_col(ITarget* t, int nt, const IParams& p, int32_t* state_out, hipStream_t s) {
  LAUNCH(k_aca_col, nt, t, p.cap, p.fixed, p.eps, state_out);
}
void launch_aca_core(ITarget* t, int nt, const IParams& p, hipStream_t s) { LAUNCH(k_aca_core, nt, t, p.cap); }
void launch_gkl_init(ITarget* t, int nt, const double* omega, hipStream_t s) {
  LAUNCH(k_gkl_init, nt, t, omega);
}
void launch_gkl_fwd(ITarget* t, int nt, const IParams& p, hipStream_t s) { LAUNCH(k_gkl_fwd, nt, t, p.cap, p.fixed, p.eps); }
void launch_gkl_bwd(ITarget* t, int nt, const IParams& p, int32_t* state_out, hipStream_t s) {
  LAUNCH(k_gkl_bwd, nt, t, p.cap, p.fixed, state_out);
}
void launch_gkl_core(ITarget* t, int nt, const IParams& p, hipStream_t s) { LAUNCH(k_gkl_core, nt, t, p.cap); }
void launch_iter_svd(ITarget* t, int nt, const IParams& p, int rmax, hipStream_t s) {
  if (nt <= 0) return;
  const int ld = std::max(1, std::min(rmax, int(ISCHEME_CAP)));
  hipLaunchKernelGGL(k_iter_svd, dim3(unsigned(nt)), dim3(NT), size_t(2) * ld * ld * sizeof(double), s, t, p.cap,
                     p.fixed, p.eps, ld);
  HM_CHECK_HIP(hipGetLastError());
}
void launch_iter_write(ITarget* t, int nt, const IParams& p, double* pool, hipStream_t s) {
  LAUNCH(k_iter_write, nt, t, p.cap, pool);
}
void launch_orth_cols(ITarget* t, int nt, int side, int cnt, int32_t* counts_out, hipStream_t s) {
  LAUNCH(k_orth_cols, nt, t, side, cnt, counts_out);
}
void launch_copy_out(ITarget* t, int nt, double* pool, hipStream_t s) { LAUNCH(k_copy_out, nt, t, pool); }

}  // namespace hm
