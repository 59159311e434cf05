// Device helpers: hashes, SplitMix64, deterministic wave/block reductions and
// the strict edge order of the heavy-edge matching.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fv_internal.h"

namespace fv {

// MurmurHash3 32-bit finaliser (Appleby, public domain).
__host__ __device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6BU;
  h ^= h >> 13;
  h *= 0xC2B2AE35U;
  h ^= h >> 16;
  return h;
}

// Tie-break hash of an undirected vertex pair a < b.
__host__ __device__ inline uint32_t pair_hash(int a, int b) {
  return fmix32(fmix32((uint32_t)a) ^ (uint32_t)b);
}

// Colouring seed of level `level` and a vertex's colouring priority.
__host__ __device__ inline uint32_t level_seed(unsigned long long colour_seed, int level) {
  uint32_t lo = (uint32_t)colour_seed, hi = (uint32_t)(colour_seed >> 32);
  return fmix32(lo ^ fmix32(hi + (uint32_t)level));
}
__host__ __device__ inline uint32_t colour_priority(int v, uint32_t seed) {
  return fmix32((uint32_t)v ^ seed);
}

// SplitMix64 (Steele, Lea & Flood 2014), counter form: draw k >= 1 of the
// stream seeded s is mix(s + k * 0x9E3779B97F4A7C15).
__device__ inline double splitmix_uniform(unsigned long long seed, unsigned long long k) {
  unsigned long long z = seed + k * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// Strict total order on undirected edges: heavier first, then smaller pair
// hash, then smaller first endpoint, then smaller second endpoint.
__device__ inline bool edge_before(double w1, int u1, int v1, double w2, int u2, int v2) {
  if (w1 != w2) return w1 > w2;
  int a1 = u1 < v1 ? u1 : v1, b1 = u1 < v1 ? v1 : u1;
  int a2 = u2 < v2 ? u2 : v2, b2 = u2 < v2 ? v2 : u2;
  uint32_t h1 = pair_hash(a1, b1), h2 = pair_hash(a2, b2);
  if (h1 != h2) return h1 < h2;
  if (a1 != a2) return a1 < a2;
  return b1 < b2;
}

// XCD-aware block order: workgroups are dealt to the 8 dies round-robin, so
// logical block k of die d is the d-th contiguous chunk; neighbouring rows then
// share one die's L2.
__device__ inline int xcd_block(int b, int nb) {
  int d = b % kXCD, k = b / kXCD;
  int per = nb / kXCD, rem = nb % kXCD;
  return d * per + (d < rem ? d : rem) + k;
}

// ---- deterministic reductions (fixed order; lane 0 / wave order) ----

// DPP move of a double (both 32-bit halves) with a constant control word.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over a full wave of 64 lanes, the same value in every lane.  Butterfly
// inside each row of 16 lanes with DPP (quad permutes, half-row and row
// mirrors: each step adds a lane to its partner, so partners stay equal), then
// the four row sums are read out and added in a fixed order.  Every lane must
// be active.
__device__ inline double row_sum16(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}

__device__ inline double wave_sum(double v) {
  v = row_sum16(v);
  auto lane_val = [&](int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
  };
  return (lane_val(0) + lane_val(16)) + (lane_val(32) + lane_val(48));
}

__device__ inline long long wave_sum_ll(long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Doubles of LDS that block_sum<kNP> needs for a block of `threads`.
__host__ __device__ constexpr int block_sum_lds(int threads) { return (4 * (threads / 64) + 1) * kNP; }

// Sum of NP values over the block; every thread receives the same totals.
// Each wave sums its rows of 16 lanes with DPP and stores the 4 row sums;
// wave 0 sums those (at most 64, one per lane) and publishes the totals.  The
// order is fixed, so the result is reproducible.  lds must hold
// (4 * blockDim/64 + 1) * NP doubles; every thread must call.
template <int NP>
__device__ inline void block_sum(double (&v)[NP], double* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NP; ++k) v[k] = row_sum16(v[k]);
  if ((lane & 15) == 0)
#pragma unroll
    for (int k = 0; k < NP; ++k) lds[(wid * 4 + (lane >> 4)) * NP + k] = v[k];
  __syncthreads();
  const int nr = nw * 4;
  if (wid == 0) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      double t = lane < nr ? lds[lane * NP + k] : 0.0;
      t = wave_sum(t);
      if (lane == 0) lds[nr * NP + k] = t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NP; ++k) v[k] = lds[nr * NP + k];
  __syncthreads();
}

// The same totals as block_sum, bit for bit, with one barrier: every wave
// (instead of wave 0 alone) reads the row sums and adds them with the same
// wave_sum.  buf holds two regions of block_sum_lds(blockDim.x) doubles used
// alternately (flip toggles on every call, and every thread makes the same
// calls), so a call never overwrites row sums that a slower wave may still be
// reading from the previous call; two calls on one region are separated by
// the barrier of the call between them.  Every thread must call.
template <int NP>
__device__ inline void block_allsum(double (&v)[NP], __attribute__((address_space(3))) double* buf,
                                    int& flip) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __attribute__((address_space(3))) double* lds = buf + flip * block_sum_lds((int)blockDim.x);
  flip ^= 1;
#pragma unroll
  for (int k = 0; k < NP; ++k) v[k] = row_sum16(v[k]);
  if ((lane & 15) == 0)
#pragma unroll
    for (int k = 0; k < NP; ++k) lds[(wid * 4 + (lane >> 4)) * NP + k] = v[k];
  __syncthreads();
  const int nr = nw * 4;
#pragma unroll
  for (int k = 0; k < NP; ++k) v[k] = wave_sum(lane < nr ? lds[lane * NP + k] : 0.0);
}

// Sum of NP values over the block for a single consumer: thread k < NP
// returns the block total of value k (other threads return 0).  Rows of 16
// lanes are summed with DPP as in block_sum; thread k then adds the block's
// row sums of value k in row order.  One barrier instead of three.
template <int NP>
__device__ inline double block_sum_spread(double (&v)[NP], double* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NP; ++k) v[k] = row_sum16(v[k]);
  if ((lane & 15) == 0)
#pragma unroll
    for (int k = 0; k < NP; ++k) lds[(wid * 4 + (lane >> 4)) * NP + k] = v[k];
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < NP)
    for (int r = 0; r < nw * 4; ++r) t += lds[r * NP + threadIdx.x];
  return t;
}

// Lanes 0 .. NP-1 of wave 0 hold one value each (block_sum_spread's result);
// every lane of wave 0 receives all NP.  Call from all of wave 0.
template <int NP>
__device__ inline void wave0_collect(double t, double (&out)[NP]) {
#pragma unroll
  for (int k = 0; k < NP; ++k)
    out[k] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(t), k),
                              __builtin_amdgcn_readlane(__double2loint(t), k));
}

__device__ inline long long block_sum_ll(long long v, long long* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum_ll(v);
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  long long t = 0;
  for (int w = 0; w < nw; ++w) t += lds[w];
  __syncthreads();
  return t;
}

__device__ inline double block_max(double v, double* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double t = lds[0];
  for (int w = 1; w < nw; ++w) t = fmax(t, lds[w]);
  __syncthreads();
  return t;
}

__device__ inline int block_min_int(int v, int* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  int t = lds[0];
  for (int w = 1; w < nw; ++w) t = min(t, lds[w]);
  __syncthreads();
  return t;
}

__device__ inline int block_max_int(int v, int* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  int t = lds[0];
  for (int w = 1; w < nw; ++w) t = max(t, lds[w]);
  __syncthreads();
  return t;
}

// Inclusive scan over a wave of 64 lanes.
__device__ inline int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

}  // namespace fv
