// Device helpers shared by the HIP translation units (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

// A dispatch holds fewer than 2^32 work-items (the grid size of an AQL dispatch packet is a
// 32-bit count of work-items): the most workgroups of `threads` work-items one launch takes.
constexpr int64_t max_groups(int threads) { return ((int64_t(1) << 32) - 1) / threads; }

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Lane 0's value of v in every lane. A wave_sum result can differ in its last bits from
// lane to lane (measured on gfx950 for operands spanning many orders of magnitude), so a
// value that steers per-lane work which must agree across the wave (a rotation angle, a
// skip test) is taken from one lane.
__device__ __forceinline__ double wave_uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Sum over a workgroup of NT threads (NT multiple of 64); `red` holds NT/64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    U4 n;
    n.x = hi1 ^ c.y ^ k0;
    n.y = lo1;
    n.z = hi0 ^ c.w ^ k1;
    n.w = lo0;
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// Standard normal from 64 random bits pairs via Box-Muller (first of the pair).
__device__ __forceinline__ double gaussian_from(U4 r) {
  const double inv53 = 1.0 / 9007199254740992.0;  // 2^-53
  uint64_t a = (uint64_t(r.x) << 21) ^ uint64_t(r.y >> 11);
  uint64_t b = (uint64_t(r.z) << 21) ^ uint64_t(r.w >> 11);
  double u1 = (double(a & ((uint64_t(1) << 53) - 1)) + 1.0) * inv53;  // (0, 1]
  double u2 = double(b & ((uint64_t(1) << 53) - 1)) * inv53;          // [0, 1)
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

}  // namespace hm
