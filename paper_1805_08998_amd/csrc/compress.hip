// Per-target kernels of the randomized compression (orthogonalisation, probe
// residual, residual check, core SVD and truncation, factor output). One
// workgroup of 256 threads per target; panels stay in global memory (they are
// small enough to live in L2 while a workgroup works on them).
#include "compress.h"
#include "device_common.h"

namespace hm {

constexpr int NT = 256;

// ---------------------------------------------------------------- Gaussian matrix
__global__ void k_fill_gaussian(double* __restrict__ om, int64_t n, int64_t i0, int32_t ncol, uint32_t k0,
                                uint32_t k1) {
  int64_t i = i0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int32_t j = blockIdx.y;
  if (i >= n || j >= ncol) return;
  U4 c{uint32_t(i), uint32_t(j), uint32_t(i >> 32), 0x0A11CE5u};
  om[int64_t(j) * n + i] = gaussian_from(philox4x32_10(c, k0, k1));
}

void launch_fill_gaussian(double* omega, int64_t n, int32_t ncol, uint64_t seed, hipStream_t s) {
  if (n <= 0 || ncol <= 0) return;
  // rows in launches of fewer than 2^32 work-items per grid row
  const int64_t rows = 256 * max_groups(256);
  for (int64_t i0 = 0; i0 < n; i0 += rows) {
    const int64_t cnt = std::min(rows, n - i0);
    dim3 grid(unsigned((cnt + 255) / 256), unsigned(ncol));
    hipLaunchKernelGGL(k_fill_gaussian, grid, dim3(256), 0, s, omega, n, i0, ncol, uint32_t(seed),
                       uint32_t(seed >> 32));
    HM_CHECK_HIP(hipGetLastError());
  }
}

// ---------------------------------------------------------------- helpers
// h[j] = Q[:, j] . v for j < r (Q ld m), computed wave-per-column.
__device__ void dots_against(const double* Q, int m, int r, const double* v, double* h) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = w; j < r; j += NT / 64) {
    const double* q = Q + int64_t(j) * m;
    double acc = 0.0;
    for (int i = lane; i < m; i += 64) acc += q[i] * v[i];
    acc = wave_sum(acc);
    if (lane == 0) h[j] = acc;
  }
  __syncthreads();
}

// v -= Q[:, :r] h
__device__ void sub_combination(const double* Q, int m, int r, const double* h, double* v) {
  for (int i = threadIdx.x; i < m; i += NT) {
    double acc = v[i];
    for (int j = 0; j < r; ++j) acc -= Q[int64_t(j) * m + i] * h[j];
    v[i] = acc;
  }
  __syncthreads();
}

__device__ double norm2_col(const double* v, int m, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += NT) acc += v[i] * v[i];
  return block_sum<NT>(acc, red);
}

// Targets of at most SMALL_M rows take the one-wave kernels below (four targets per
// workgroup, lane l owning rows l and l + 64): their Gram-Schmidt steps are wave sums with
// no barriers, where a workgroup of NT threads would leave most of its threads idle and
// wait at a barrier several times per column. Larger targets take the NT-thread kernels.
constexpr int SMALL_M = 128;
constexpr int HMAX = 128;  // Gram-Schmidt coefficients per column: r < cap + probes

// v -= Q[:, :r] (Q[:, :r]^T v) for a vector v held as (v0, v1) = rows (lane, lane + 64):
// all r coefficients from the same v (classical Gram-Schmidt), kept in the wave's LDS row.
__device__ __forceinline__ void project_out_wave(const double* __restrict__ Q, int m, int r, double& v0, double& v1,
                                                 int lane, bool in0, bool in1, double* hs) {
  for (int j = 0; j < r; ++j) {
    const double* q = Q + int64_t(j) * m;
    const double q0 = in0 ? q[lane] : 0.0, q1 = in1 ? q[lane + 64] : 0.0;
    const double hj = wave_sum(q0 * v0 + q1 * v1);
    if (lane == 0) hs[j] = hj;
  }
  // one wave: its LDS accesses complete in issue order; keep the compiler from moving them
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  for (int j = 0; j < r; ++j) {
    const double* q = Q + int64_t(j) * m;
    const double hj = hs[j];
    if (in0) v0 -= q[lane] * hj;
    if (in1) v1 -= q[lane + 64] * hj;
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(NT) k_orth_append_w(CTarget* __restrict__ tg, int nt, int src, int cnt, int cap) {
  __shared__ double hsh[NT / 64][HMAX];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * (NT / 64) + wv;
  if (t >= nt) return;
  CTarget& T = tg[t];
  if (!T.active || T.m > SMALL_M) return;
  double* hs = hsh[wv];
  const int m = T.m;
  double* Y = T.Y;
  int r = T.r;
  const int cnt_t = (src == 0 && T.w0 > 0 && T.w0 < cnt) ? T.w0 : cnt;
  const bool in0 = lane < m, in1 = lane + 64 < m;
  for (int c = src; c < src + cnt_t; ++c) {
    const double* v = Y + int64_t(c) * m;
    double v0 = in0 ? v[lane] : 0.0, v1 = in1 ? v[lane + 64] : 0.0;
    const double n0 = wave_uniform(wave_sum(v0 * v0 + v1 * v1));
    for (int pass = 0; pass < 2; ++pass) project_out_wave(Y, m, r, v0, v1, lane, in0, in1, hs);
    const double n1 = wave_uniform(wave_sum(v0 * v0 + v1 * v1));
    const bool keep = (r < cap) && n1 > 0.0 && n1 > 1e-26 * n0;  // relative residual > 1e-13
    if (keep) {
      const double inv = 1.0 / sqrt(n1);
      double* dst = Y + int64_t(r) * m;
      if (in0) dst[lane] = v0 * inv;
      if (in1) dst[lane + 64] = v1 * inv;
      ++r;
    }
  }
  if (lane == 0) T.r = r;
}

__global__ void __launch_bounds__(NT) k_probe_residual_w(CTarget* __restrict__ tg, int nt, int cap, int g) {
  __shared__ double hsh[NT / 64][HMAX];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * (NT / 64) + wv;
  if (t >= nt) return;
  CTarget& T = tg[t];
  if (!T.active || T.m > SMALL_M) return;
  double* hs = hsh[wv];
  const int m = T.m, r = T.r;
  double* Y = T.Y;
  const bool in0 = lane < m, in1 = lane + 64 < m;
  double e2 = 0.0;
  for (int c = cap; c < cap + g; ++c) {
    double* v = Y + int64_t(c) * m;
    double v0 = in0 ? v[lane] : 0.0, v1 = in1 ? v[lane + 64] : 0.0;
    for (int pass = 0; pass < 2; ++pass) project_out_wave(Y, m, r, v0, v1, lane, in0, in1, hs);
    e2 += wave_uniform(wave_sum(v0 * v0 + v1 * v1));
    if (in0) v[lane] = v0;
    if (in1) v[lane + 64] = v1;
  }
  if (lane == 0) T.E2 = e2 / double(g);
}

// Probe residual of targets above SMALL_M rows, in blocks: the g <= 16 probe columns P are
// projected against Q = Y[:, :r] (r <= 64) twice, each time as H = Q^T P and P -= Q H on
// v_mfma_f64_16x16x4f64 (classical Gram-Schmidt on the whole block: the same arithmetic per
// column as projecting the columns one by one, with Q read four times in all rather than
// four times per column). Row tiles of 16 go round-robin to the four waves; the waves' partial
// H are summed in LDS in wave order, so the result does not depend on scheduling.
// MFMA operand layouts: A[i][k] at lane i + 16k, B[k][j] at lane j + 16k, accumulator
// register v of lane l holds D[l/16 + 4v][l%16].
typedef double cdbl4 __attribute__((ext_vector_type(4)));
static __device__ __forceinline__ cdbl4 cmfma(double a, double b, cdbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
constexpr int PBLK_R = 64, PBLK_G = 16;

__global__ void __launch_bounds__(NT) k_probe_residual_blk(CTarget* __restrict__ tg, int nt, int cap, int g) {
  __shared__ double hp[NT / 64][PBLK_R][PBLK_G];  // per-wave partial H, then H in hp[0]
  __shared__ double red[NT / 64];
  CTarget& T = tg[blockIdx.x];
  if (!T.active || T.m <= SMALL_M) return;
  const int m = T.m, r = T.r;
  const double* Q = T.Y;
  double* P = T.Y + int64_t(cap) * m;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int ntile = (m + 15) >> 4, nrt = (r + 15) >> 4;
  const bool gok = li < g;
  const int gc = min(li, g - 1);
  for (int pass = 0; pass < 2; ++pass) {
    if (r > 0) {
      // H_w = Q[rows of wave w]^T P[rows of wave w]: rows are the K dimension
      cdbl4 acc[PBLK_R / 16];
#pragma unroll
      for (int jt = 0; jt < PBLK_R / 16; ++jt) acc[jt] = cdbl4{0.0, 0.0, 0.0, 0.0};
      for (int t = wv; t < ntile; t += NT / 64) {
#pragma unroll 1
        for (int s4 = 0; s4 < 4; ++s4) {
          const int row = 16 * t + 4 * s4 + lk;
          const bool rok = row < m;
          const int rc = min(row, m - 1);
          const double b = rok && gok ? P[int64_t(gc) * m + rc] : 0.0;
#pragma unroll
          for (int jt = 0; jt < PBLK_R / 16; ++jt) {
            if (jt < nrt) {
              const int j = 16 * jt + li;
              const double a = rok && j < r ? Q[int64_t(min(j, r - 1)) * m + rc] : 0.0;
              acc[jt] = cmfma(a, b, acc[jt]);
            }
          }
        }
      }
#pragma unroll
      for (int jt = 0; jt < PBLK_R / 16; ++jt)
        if (jt < nrt)
#pragma unroll
          for (int v = 0; v < 4; ++v) hp[wv][16 * jt + lk + 4 * v][li] = acc[jt][v];
      __syncthreads();
      // H = sum of the waves' partials, in wave order
      for (int e = threadIdx.x; e < 16 * nrt * PBLK_G; e += NT) {
        const int j = e / PBLK_G, c = e % PBLK_G;
        double h = 0.0;
        for (int w = 0; w < NT / 64; ++w) h += hp[w][j][c];
        hp[0][j][c] = (j < r && c < g) ? h : 0.0;
      }
      __syncthreads();
      // P -= Q H, 16 rows at a time: A = Q[rows, j] (16 consecutive rows per lane group),
      // B = H[j, c]
      for (int t = wv; t < ntile; t += NT / 64) {
        const int row0 = 16 * t;
        const int rowa = min(row0 + li, m - 1);
        cdbl4 d = cdbl4{0.0, 0.0, 0.0, 0.0};
        for (int j0 = 0; j0 < 16 * nrt; j0 += 4) {
          const int j = j0 + lk;
          const double a = j < r ? Q[int64_t(min(j, r - 1)) * m + rowa] : 0.0;
          d = cmfma(a, hp[0][j][li], d);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + lk + 4 * v;
          if (row < m && gok) P[int64_t(li) * m + row] -= d[v];
        }
      }
    }
    __syncthreads();
  }
  // E2 = sum of the projected probes' squared norms over g
  double e2 = 0.0;
  for (int64_t i = threadIdx.x; i < int64_t(g) * m; i += NT) e2 += P[i] * P[i];
  e2 = block_sum<NT>(e2, red);
  if (threadIdx.x == 0) T.E2 = e2 / double(g);
}

// ---------------------------------------------------------------- orthogonalisation
__global__ void __launch_bounds__(NT) k_orth_append(CTarget* __restrict__ tg, int nt, int src, int cnt,
                                                    int cap) {
  __shared__ double h[128];
  __shared__ double red[NT / 64];
  CTarget& T = tg[blockIdx.x];
  if (!T.active || T.m <= SMALL_M) return;
  const int m = T.m;
  double* Y = T.Y;
  int r = T.r;
  // the first sketch block has a per-target width (w0 <= cnt)
  const int cnt_t = (src == 0 && T.w0 > 0 && T.w0 < cnt) ? T.w0 : cnt;
  for (int c = src; c < src + cnt_t; ++c) {
    double* v = Y + int64_t(c) * m;
    double n0 = norm2_col(v, m, red);
    for (int pass = 0; pass < 2; ++pass) {
      dots_against(Y, m, r, v, h);
      sub_combination(Y, m, r, h, v);
    }
    double n1 = norm2_col(v, m, red);
    bool keep = (r < cap) && n1 > 0.0 && n1 > 1e-26 * n0;  // relative residual > 1e-13
    if (keep) {
      double inv = 1.0 / sqrt(n1);
      double* dst = Y + int64_t(r) * m;
      for (int i = threadIdx.x; i < m; i += NT) dst[i] = v[i] * inv;
      __syncthreads();
      ++r;
    }
  }
  if (threadIdx.x == 0) T.r = r;
}

void launch_orth_append(CTarget* t, int nt, int src, int cnt, const CParams& p, hipStream_t s) {
  if (nt <= 0) return;
  if (p.cap > HMAX) throw Error(HMAT_ERR_INTERNAL, "column capacity above the Gram-Schmidt buffer");
  hipLaunchKernelGGL(k_orth_append_w, dim3((nt + NT / 64 - 1) / (NT / 64)), dim3(NT), 0, s, t, nt, src, cnt, p.cap);
  HM_CHECK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_orth_append, dim3(nt), dim3(NT), 0, s, t, nt, src, cnt, p.cap);
  HM_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- probe residual
__global__ void __launch_bounds__(NT) k_probe_residual(CTarget* __restrict__ tg, int nt, int cap, int g) {
  __shared__ double h[128];
  __shared__ double red[NT / 64];
  CTarget& T = tg[blockIdx.x];
  if (!T.active || T.m <= SMALL_M) return;
  const int m = T.m, r = T.r;
  double* Y = T.Y;
  double e2 = 0.0;
  for (int c = cap; c < cap + g; ++c) {
    double* v = Y + int64_t(c) * m;
    for (int pass = 0; pass < 2; ++pass) {
      dots_against(Y, m, r, v, h);
      sub_combination(Y, m, r, h, v);
    }
    e2 += norm2_col(v, m, red);
  }
  if (threadIdx.x == 0) T.E2 = e2 / double(g);
}

void launch_probe_residual(CTarget* t, int nt, const CParams& p, hipStream_t s) {
  if (nt <= 0) return;
  if (p.cap > HMAX) throw Error(HMAT_ERR_INTERNAL, "column capacity above the Gram-Schmidt buffer");
  hipLaunchKernelGGL(k_probe_residual_w, dim3((nt + NT / 64 - 1) / (NT / 64)), dim3(NT), 0, s, t, nt, p.cap, p.g);
  HM_CHECK_HIP(hipGetLastError());
  if (p.g <= PBLK_G && p.cap <= PBLK_R)
    hipLaunchKernelGGL(k_probe_residual_blk, dim3(nt), dim3(NT), 0, s, t, nt, p.cap, p.g);
  else
    hipLaunchKernelGGL(k_probe_residual, dim3(nt), dim3(NT), 0, s, t, nt, p.cap, p.g);
  HM_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- residual check
__global__ void __launch_bounds__(NT) k_check(CTarget* __restrict__ tg, int nt, int cap, int g, double eps,
                                              double delta, int32_t* __restrict__ pending) {
  __shared__ double red[NT / 64];
  CTarget& T = tg[blockIdx.x];
  if (!T.active) {
    if (threadIdx.x == 0) pending[blockIdx.x] = 0;
    return;
  }
  const int64_t len = int64_t(T.n) * T.rz;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += NT) acc += T.Z[i] * T.Z[i];
  acc = block_sum<NT>(acc, red);
  if (threadIdx.x == 0) {
    T.nB2 = acc;
    double lim = delta * eps;
    bool ok = T.E2 <= lim * lim * (acc + T.E2);
    // a zero sketch of a zero operator passes (E2 = 0)
    T.done = ok ? 1 : 0;
    int more = (!ok && T.r + g <= cap) ? 1 : 0;
    pending[blockIdx.x] = more;
  }
}

void launch_check(CTarget* t, int nt, const CParams& p, int32_t* pending, hipStream_t s) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(k_check, dim3(nt), dim3(NT), 0, s, t, nt, p.cap, p.g, p.eps, p.delta, pending);
  HM_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- core SVD + truncation
constexpr int CAPMAX = 64;

// One-sided Jacobi SVD of the r x r matrix M (columns of stride LD, in LDS) by one wave
// (lane 0..63): the rotations accumulate in J; then the column norms sigma, their descending
// order and the truncation rank k (T.k, T.nB2 and T.svd_capped, from lane 0). The pairs are
// taken in parallel (round-robin) order: a sweep is nr - 1 rounds of nr / 2 disjoint pairs
// (nr = r rounded up to even; pairs with the padding index are skipped), and each pair is
// rotated by a group of G lanes at once. A group's rotation angle is taken from its first
// lane, so the lanes of a group apply the same rotation.
__device__ void core_jacobi_wave(CTarget& T, double* M, double* J, double* sig, int* order, int r, int LD,
                                 double eps, double kappa, int lane) {
  for (int i = 0; i < r; ++i)
    if (lane < r) J[i * LD + lane] = (lane == i) ? 1.0 : 0.0;
  const int nr = (r + 1) & ~1;
  int npair = 1;
  while (npair < nr / 2) npair <<= 1;         // groups: a power of two, at most 32
  const int G = 64 / npair;                   // lanes per group
  const int grp = lane / G, gl = lane % G;    // group and lane within it
  const int leader = grp * G;
  int capped = 1;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int t = 0; t + 1 < nr; ++t) {
      // round t of the circle schedule: position 0 holds index 0, position k >= 1 holds
      // 1 + (k - 1 + t) mod (nr - 1); pair k joins positions k and nr - 1 - k
      int p = -1, q = -1;
      if (grp < nr / 2) {
        const int k0 = grp, k1 = nr - 1 - grp;
        const int i0 = k0 == 0 ? 0 : 1 + (k0 - 1 + t) % (nr - 1);
        const int i1 = 1 + (k1 - 1 + t) % (nr - 1);
        p = min(i0, i1);
        q = max(i0, i1);
      }
      const bool live = p >= 0 && q < r;
      double a = 0.0, b = 0.0, c = 0.0;
      if (live)
        for (int e = gl; e < r; e += G) {
          const double mp = M[p * LD + e], mq = M[q * LD + e];
          a += mp * mp;
          b += mq * mq;
          c += mp * mq;
        }
      for (int o = 1; o < G; o <<= 1) {  // within the group (G divides 64, groups aligned)
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
      }
      a = __shfl(a, leader, 64);
      b = __shfl(b, leader, 64);
      c = __shfl(c, leader, 64);
      const bool rot = live && !(fabs(c) <= 1e-15 * sqrt(a * b) || c == 0.0);
      if (rot) {
        const double zeta = (b - a) / (2.0 * c);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        for (int e = gl; e < r; e += G) {
          const double mp = M[p * LD + e], mq = M[q * LD + e];
          M[p * LD + e] = cs * mp - sn * mq;
          M[q * LD + e] = sn * mp + cs * mq;
          const double jp = J[p * LD + e], jq = J[q * LD + e];
          J[p * LD + e] = cs * jp - sn * jq;
          J[q * LD + e] = sn * jp + cs * jq;
        }
      }
      rotated |= __ballot(rot) != 0 ? 1 : 0;
      // the next round reads columns other groups wrote: keep the LDS accesses in order
      // (one wave: its LDS instructions complete in issue order)
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_wave_barrier();
    }
    if (!rotated) {
      capped = 0;
      break;
    }
  }
  if (lane == 0) T.svd_capped = capped;
  for (int j = 0; j < r; ++j) {
    double mj = lane < r ? M[j * LD + lane] : 0.0;
    double s2 = wave_sum(mj * mj);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  if (lane == 0) {
    for (int j = 0; j < r; ++j) order[j] = j;
    for (int a = 1; a < r; ++a) {  // insertion sort, descending
      int x = order[a];
      int b = a - 1;
      while (b >= 0 && sig[order[b]] < sig[x]) {
        order[b + 1] = order[b];
        --b;
      }
      order[b + 1] = x;
    }
    double total = 0.0;
    for (int j = 0; j < r; ++j) total += sig[j] * sig[j];
    double thr = eps * eps * (total + T.E2) - kappa * T.E2;
    int k = r;
    double tail = 0.0;  // tail(k) = sum_{i >= k} sigma_i^2 in sorted order
    for (int kk = r; kk >= 0; --kk) {
      if (kk < r) tail += sig[order[kk]] * sig[order[kk]];
      if (tail <= thr) k = kk;
      else break;
    }
    T.k = k;
    T.nB2 = total;
  }
}

// LD (<= CAPMAX) is the largest column count rz of the launch's targets: the two LD x LD
// work arrays live in dynamic LDS, so small cores leave room for more workgroups per CU.
__global__ void __launch_bounds__(NT) k_core(CTarget* __restrict__ tg, int nt, int cap, double eps,
                                             double kappa, int LD, int skip_n, int skip_r) {
  __shared__ double h[CAPMAX];
  __shared__ double red[NT / 64];
  extern __shared__ double dyn[];
  double* M = dyn;            // Rz^T, column-major, ld LD
  double* J = dyn + LD * LD;  // right rotations, ld LD
  __shared__ double sig[CAPMAX];
  __shared__ int order[CAPMAX];
  CTarget& T = tg[blockIdx.x];
  if (T.n <= skip_n && T.rz <= skip_r) return;  // done by k_core_w
  const int n = T.n, r = min(T.rz, LD);  // the host sizes LD as the maximum rz
  double* Z = T.Z;
  for (int i = threadIdx.x; i < LD * LD; i += NT) {
    M[i] = 0.0;
    J[i] = 0.0;
  }
  __syncthreads();
  // CGS2 QR of Z (n x r) in place; R(i, j) goes to M(j, i)
  for (int j = 0; j < r; ++j) {
    double* v = Z + int64_t(j) * n;
    double n0 = norm2_col(v, n, red);
    for (int pass = 0; pass < 2; ++pass) {
      dots_against(Z, n, j, v, h);
      if (threadIdx.x < j) M[threadIdx.x * LD + j] += h[threadIdx.x];  // M(j, i) = R(i, j)
      __syncthreads();
      sub_combination(Z, n, j, h, v);
    }
    double n1 = norm2_col(v, n, red);
    bool keep = n1 > 0.0 && n1 > 1e-28 * n0;
    double d = keep ? sqrt(n1) : 0.0;
    double inv = keep ? 1.0 / d : 0.0;
    for (int i = threadIdx.x; i < n; i += NT) v[i] *= inv;
    if (threadIdx.x == 0) M[j * LD + j] = d;
    __syncthreads();
  }
  // One-sided Jacobi on the columns of M (r x r), accumulating J; wave 0 only
  if (threadIdx.x < 64) core_jacobi_wave(T, M, J, sig, order, r, LD, eps, kappa, threadIdx.x);
  __syncthreads();
  // store the sorted W (= M) and J columns plus sigma in core
  double* core = T.core;
  for (int idx = threadIdx.x; idx < r * r; idx += NT) {
    int j = idx / r, i = idx % r;
    int src = order[j];
    core[idx] = M[src * LD + i];
    core[cap * cap + idx] = J[src * LD + i];
  }
  for (int j = threadIdx.x; j < r; j += NT) core[2 * cap * cap + j] = sig[order[j]];
}

// k_core for targets whose Z has at most SMALL_M rows and at most LD (<= CORE_W_LD) columns:
// one wave per target (four per workgroup), lane l owning rows l and l + 64 of Z, so the QR
// of Z needs wave sums only; then the same Jacobi stage. Each wave's LDS: M and J (LD x LD
// each), sigma (64), the coefficients of the current column (64) and the sort order (64 ints).
// k_core takes the other targets of the launch.
constexpr int CORE_W_LD = 24;  // four waves of LDS stay within 64 KiB per workgroup
__host__ __device__ constexpr int core_w_lds(int LD) { return 2 * LD * LD + 64 + 64 + 32; }  // doubles

__global__ void __launch_bounds__(NT) k_core_w(CTarget* __restrict__ tg, int nt, int cap, double eps, double kappa,
                                               int LD) {
  extern __shared__ double dyn[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * (NT / 64) + wv;
  if (t >= nt) return;
  CTarget& T = tg[t];
  if (T.n > SMALL_M || T.rz > LD) return;
  double* M = dyn + wv * core_w_lds(LD);
  double* J = M + LD * LD;
  double* sig = J + LD * LD;
  double* hs = sig + 64;
  int* order = reinterpret_cast<int*>(hs + 64);
  const int n = T.n, r = min(T.rz, LD);
  double* Z = T.Z;
  for (int i = lane; i < LD * LD; i += 64) {
    M[i] = 0.0;
    J[i] = 0.0;
  }
  const bool in0 = lane < n, in1 = lane + 64 < n;
  // CGS2 QR of Z (n x r) in place; R(i, j) goes to M(j, i)
  for (int j = 0; j < r; ++j) {
    double* v = Z + int64_t(j) * n;
    double v0 = in0 ? v[lane] : 0.0, v1 = in1 ? v[lane + 64] : 0.0;
    const double n0 = wave_uniform(wave_sum(v0 * v0 + v1 * v1));
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < j; ++i) {
        const double* q = Z + int64_t(i) * n;
        const double h = wave_uniform(wave_sum((in0 ? q[lane] : 0.0) * v0 + (in1 ? q[lane + 64] : 0.0) * v1));
        if (lane == 0) {
          hs[i] = h;
          M[i * LD + j] += h;  // M(j, i) = R(i, j)
        }
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_wave_barrier();
      for (int i = 0; i < j; ++i) {
        const double* q = Z + int64_t(i) * n;
        const double h = hs[i];
        if (in0) v0 -= q[lane] * h;
        if (in1) v1 -= q[lane + 64] * h;
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_wave_barrier();
    }
    const double n1 = wave_uniform(wave_sum(v0 * v0 + v1 * v1));
    const bool keep = n1 > 0.0 && n1 > 1e-28 * n0;
    const double d = keep ? sqrt(n1) : 0.0;
    const double inv = keep ? 1.0 / d : 0.0;
    if (in0) v[lane] = v0 * inv;
    if (in1) v[lane + 64] = v1 * inv;
    if (lane == 0) M[j * LD + j] = d;
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  core_jacobi_wave(T, M, J, sig, order, r, LD, eps, kappa, lane);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  // store the sorted W (= M) and J columns plus sigma in core
  double* core = T.core;
  for (int idx = lane; idx < r * r; idx += 64) {
    const int jj = idx / r, i = idx % r;
    const int src = order[jj];
    core[idx] = M[src * LD + i];
    core[cap * cap + idx] = J[src * LD + i];
  }
  for (int jj = lane; jj < r; jj += 64) core[2 * cap * cap + jj] = sig[order[jj]];
}

void launch_core(CTarget* t, int nt, const CParams& p, hipStream_t s, int rmax) {
  if (nt <= 0) return;
  if (p.cap > CAPMAX) throw Error(HMAT_ERR_INTERNAL, "column capacity above 64");
  const int ld = std::max(1, std::min(rmax > 0 ? rmax : p.cap, CAPMAX));
  // small targets (n <= SMALL_M, rz <= ldw) in one wave each, the others in k_core
  const int ldw = std::min(ld, CORE_W_LD);
  hipLaunchKernelGGL(k_core_w, dim3((nt + NT / 64 - 1) / (NT / 64)), dim3(NT),
                     size_t(NT / 64) * core_w_lds(ldw) * sizeof(double), s, t, nt, p.cap, p.eps, p.kappa, ldw);
  HM_CHECK_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_core, dim3(nt), dim3(NT), size_t(2) * ld * ld * sizeof(double), s, t, nt, p.cap, p.eps,
                     p.kappa, ld, SMALL_M, ldw);
  HM_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- stacked term columns
__global__ void __launch_bounds__(NT) k_term_columns(CTarget* __restrict__ tg, TreeView tv, int c0, int cnt, int cap) {
  __shared__ int sel_term, sel_col;
  CTarget& T = tg[blockIdx.x];
  const int m = T.m;
  for (int j = 0; j < cnt; ++j) {
    double* dst = T.Y + int64_t(cap + j) * m;
    if (threadIdx.x == 0) {
      // find the term holding stacked column c0 + j: terms of the block, then of its ancestors
      int gc = c0 + j, term = -1, col = 0;
      for (int a = T.block; a >= 0 && term < 0; a = tv.b_parent[a])
        for (int it = tv.group_ptr[a]; it < tv.group_ptr[a + 1]; ++it) {
          const int kr = tv.terms[it].kr;
          if (gc < kr) {
            term = it;
            col = gc;
            break;
          }
          gc -= kr;
        }
      sel_term = term;
      sel_col = col;
    }
    __syncthreads();
    const int it = sel_term, lc = sel_col;
    if (it < 0) {
      for (int i = threadIdx.x; i < m; i += NT) dst[i] = 0.0;
    } else {
      const Term tm = tv.terms[it];
      const int64_t r0 = int64_t(T.row0) - tm.lrow0;  // panel row of the target's first row
      for (int i = threadIdx.x; i < m; i += NT) {
        double v;
        if (tm.core) {
          v = 0.0;
          for (int c = 0; c < tm.kl; ++c) v += tm.L[r0 + i + int64_t(c) * tm.ldl] * tm.core[c + int64_t(lc) * tm.kl];
        } else {
          v = tm.L[r0 + i + int64_t(lc) * tm.ldl];
        }
        dst[i] = v;
      }
    }
    __syncthreads();
  }
}

void launch_term_columns(CTarget* t, int nt, const TreeView& tv, int c0, int cnt, int cap, hipStream_t s) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(k_term_columns, dim3(nt), dim3(NT), 0, s, t, tv, c0, cnt, cap);
  HM_CHECK_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- factor output
// out (rows x k, ld rows) = P (rows x r, ld rows) C[:, :k] with C(j, c) at C[c * r + j],
// on v_mfma_f64_16x16x4f64: 16-row tiles round-robin over the workgroup's waves, each tile
// with all (at most four) 16-column blocks of the output, K-steps of 4 over j. Rows at or past
// `rows`, columns at or past k and steps at or past r are clamped in the loads and masked.
__device__ __forceinline__ void small_gemm_out(const double* __restrict__ P, const double* __restrict__ C,
                                               double* __restrict__ out, int rows, int r, int k) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int ntile = (rows + 15) >> 4, nct = (k + 15) >> 4;
  for (int t = wv; t < ntile; t += NT / 64) {
    const int row0 = 16 * t;
    const int ra = min(row0 + li, rows - 1);
    cdbl4 d[CAPMAX_CORE / 16];
#pragma unroll
    for (int ct = 0; ct < CAPMAX_CORE / 16; ++ct) d[ct] = cdbl4{0.0, 0.0, 0.0, 0.0};
    for (int j0 = 0; j0 < r; j0 += 4) {
      const int j = j0 + lk;
      const bool jok = j < r;
      const int jc = min(j, r - 1);
      const double a = jok && row0 + li < rows ? P[int64_t(jc) * rows + ra] : 0.0;
#pragma unroll
      for (int ct = 0; ct < CAPMAX_CORE / 16; ++ct) {
        if (ct < nct) {
          const int c = 16 * ct + li;
          const double b = jok && c < k ? C[min(c, k - 1) * r + jc] : 0.0;
          d[ct] = cmfma(a, b, d[ct]);
        }
      }
    }
#pragma unroll
    for (int ct = 0; ct < CAPMAX_CORE / 16; ++ct) {
      if (ct < nct) {
        const int c = 16 * ct + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row0 + lk + 4 * v;
          if (row < rows && c < k) out[int64_t(c) * rows + row] = d[ct][v];
        }
      }
    }
  }
}

__global__ void __launch_bounds__(NT) k_write_factors(const CTarget* __restrict__ tg, int nt, int cap,
                                                      double* __restrict__ pool) {
  const CTarget& T = tg[blockIdx.x];
  const int m = T.m, n = T.n, r = T.rz, k = T.k;
  if (k == 0) return;
  const double* W = T.core;
  const double* J = T.core + cap * cap;
  double* L = pool + T.out_off;
  double* R = L + int64_t(m) * k;
  small_gemm_out(T.Y, W, L, m, r, k);  // L = Q W
  small_gemm_out(T.Z, J, R, n, r, k);  // R = Q_Z J
}

void launch_write_factors(CTarget* t, int nt, const CParams& p, double* pool, hipStream_t s) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(k_write_factors, dim3(nt), dim3(NT), 0, s, t, nt, p.cap, pool);
  HM_CHECK_HIP(hipGetLastError());
}

}  // namespace hm
