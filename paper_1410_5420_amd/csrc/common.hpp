// Device-side building blocks shared by the gfx950 kernels of the k-d tree
// builder: wave64 lane masks and scans, block scans, the implicit shape of the
// balanced tree and the layout of the rank records.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kd {

constexpr int kWave = 64;

// ---- wave helpers -------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below_mask() {
  const uint32_t l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

// Inclusive prefix sum across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, d, kWave);
    if ((int)lane_id() >= d) v += o;
  }
  return v;
}

// Exclusive block-wide prefix sum of one value per thread (NT threads, a
// multiple of 64).  `s_tmp` holds NT/64 + 1 words of LDS.  Returns the
// exclusive prefix; *total receives the block sum.  Contains barriers.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* s_tmp, T* total) {
  constexpr int kWaves = NT / kWave;
  const int w = threadIdx.x / kWave;
  T inc = wave_inclusive_sum(v);
  if (lane_id() == kWave - 1) s_tmp[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
      T c = s_tmp[i];
      s_tmp[i] = run;
      run += c;
    }
    s_tmp[kWaves] = run;
  }
  __syncthreads();
  T res = s_tmp[w] + inc - v;
  *total = s_tmp[kWaves];
  __syncthreads();
  return res;
}

// ---- XCD-aware tile order ------------------------------------------------------
// Workgroups are handed to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8), and each XCD has its own L2.  For a launch of `grid` workgroups
// (a multiple of 8) this bijection gives XCD x the contiguous tile range
// [x * grid/8, (x+1) * grid/8), walked in dispatch order, so partial cache
// lines written by neighbouring tiles meet in the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int grid) {
  return (b % kXcds) * (grid / kXcds) + b / kXcds;
}
__host__ __device__ __forceinline__ int xcd_grid(int tiles) {
  return (tiles + kXcds - 1) / kXcds * kXcds;
}

// ---- implicit shape of the balanced tree --------------------------------------
// The node of [s, e] sits at its lower median; its children cover [s, m-1] and
// [m+1, e].  At depth L the largest subarray holds floor(n / 2^L) elements.

__device__ __forceinline__ int64_t median_of(int64_t s, int64_t e) { return s + ((e - s) >> 1); }

// Subarray at depth `depth` that contains position pos, or e < s when pos is
// the node of a shallower subarray (64- and 32-bit forms).
__device__ __forceinline__ void subarray_at(int64_t pos, int64_t nu, int depth, int64_t* s_out,
                                            int64_t* e_out) {
  int64_t s = 0, e = nu - 1;
  for (int l = 0; l < depth; ++l) {
    int64_t m = median_of(s, e);
    if (pos < m) {
      e = m - 1;
    } else if (pos > m) {
      s = m + 1;
    } else {
      s = 1;
      e = 0;
      break;
    }
  }
  *s_out = s;
  *e_out = e;
}

__device__ __forceinline__ void subarray_at(int pos, int nu, int depth, int* s_out, int* e_out) {
  int s = 0, e = nu - 1;
  for (int l = 0; l < depth; ++l) {
    const int m = s + ((e - s) >> 1);
    if (pos < m) {
      e = m - 1;
    } else if (pos > m) {
      s = m + 1;
    } else {
      s = 1;
      e = 0;
      break;
    }
  }
  *s_out = s;
  *e_out = e;
}

// First depth at which every subarray holds at most `cutover` elements.
__device__ __host__ __forceinline__ int cutover_depth(int64_t nu, int64_t cutover) {
  int d = 0;
  while ((nu >> d) > cutover) ++d;
  return d;
}

// ---- rank-record layout ------------------------------------------------------------
// Array j (0 <= j < k) stores one record per position: k-1 ranks (plane c =
// rank in order (j + 1 + c) mod k), plus the row id for array 0.  Arrays are
// laid out one after another, array 0 first.
__device__ __host__ __forceinline__ int record_width(int j, int k) { return k - 1 + (j == 0); }
__device__ __host__ __forceinline__ int64_t record_offset(int j, int k, int64_t n) {
  return j == 0 ? 0 : (int64_t)k * n + (int64_t)(j - 1) * (k - 1) * n;
}
__device__ __host__ __forceinline__ int64_t record_words(int k, int64_t n) {
  return (int64_t)k * n + (int64_t)(k - 1) * (k - 1) * n;
}

}  // namespace kd
