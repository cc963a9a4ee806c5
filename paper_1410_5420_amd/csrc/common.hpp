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

// Set lanes of m below this lane (two mbcnt steps, no mask of lanes below).
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes of `among` whose digit (the low `bits` bits of d) equals this lane's.
// A compare per bit gives the lanes having that bit set; where that set
// disagrees with this lane's own bit (taken as 0 or all ones), a lane holds
// another digit, so the disagreements ORed over the bits mark every lane to
// drop: two 32-bit logic ops per bit and half besides the compare.  All 64
// lanes must be active.  kMax bounds `bits` (a compile-time count unrolls
// fully; a smaller run-time count skips the later bits).
template <int kMax>
__device__ __forceinline__ uint64_t same_digit_lanes(uint32_t d, int bits, uint64_t among) {
  uint32_t lo = 0u, hi = 0u;
#pragma unroll
  for (int b = 0; b < kMax; ++b) {
    if (b < bits) {
      const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
      const uint64_t bb = __builtin_amdgcn_uicmp(s, 0u, 33);  // lanes where s != 0
      lo |= (uint32_t)bb ^ s;
      hi |= (uint32_t)(bb >> 32) ^ s;
    }
  }
  return among & ~(((uint64_t)hi << 32) | lo);
}

// ---- hand-off between workgroups of one launch ---------------------------------
// Each XCD has its own L2, and a device-scope fence on gfx950 writes back and
// invalidates the whole L2, which costs about a microsecond per fence and
// serialises per XCD.  Values that one workgroup hands to another within a
// launch therefore travel by device-scope atomic loads and stores, which the
// L2s keep coherent, and the waits below only order them around the
// counter that signals the hand-off; no cache is flushed.
__device__ __forceinline__ void store_dev(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_dev(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// This thread's memory operations have completed (vmcnt 0) before any later
// one: after the stores of a hand-off, before the signal.
__device__ __forceinline__ void wait_memory_ops() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt 0; expcnt and lgkmcnt not waited on
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Inclusive prefix sum across the 64 lanes of a wave through DPP lane moves:
// shifts by 1, 2, 4 and 8 within each row of 16 lanes, then the last lane of
// row r added to row r+1 and the last lane of row 1 to rows 2 and 3.  All 64
// lanes must be active.
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t v) {
  v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// Inclusive max across the 64 lanes of a wave (all lanes active; 0 is the
// identity), by the same DPP lane moves.
__device__ __forceinline__ uint32_t wave_max_dpp(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x111, 0xF, 0xF, false));  // row_shr:1
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x112, 0xF, 0xF, false));  // row_shr:2
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x114, 0xF, 0xF, false));  // row_shr:4
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x118, 0xF, 0xF, false));  // row_shr:8
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return v;
}

// Inclusive prefix sum across the 64 lanes of a wave (all lanes active):
// DPP lane moves for 32-bit values, shuffles otherwise.
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
  if constexpr (sizeof(T) == 4) {
    return (T)wave_scan_dpp((uint32_t)v);
  } else {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      T o = __shfl_up(v, d, kWave);
      if ((int)lane_id() >= d) v += o;
    }
    return v;
  }
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

// ---- rolling schedule of the index arrays ----------------------------------
// One tree, level form 4 (Appendix, "Deferred Merge Sort and Partitioning",
// carried through every level): an array is partitioned only right before
// the level that splits it.  At level L the array p = L mod k is brought from
// the layout it had after it last split (depth roll_depth(L, p)) to depth L in
// one stable multi-way split, by the medians of the levels in between; no
// other array moves.  After the last global level D the arrays the on-chip
// finish reads get one last split to depth D.

// Depth of array j's layout before level L's split (L <= D): one below the
// last level < L that split with it, 0 before the first.
__host__ __device__ __forceinline__ int roll_depth(int L, int j, int k) {
  return L > j ? j + k * ((L - 1 - j) / k) + 1 : 0;
}
// Splits of array j at the levels 1 .. L-1 (level 0 splits presorted array 0
// in place).
__host__ __device__ __forceinline__ int roll_moves(int L, int j, int k) {
  if (j == 0) return L >= 1 ? (L - 1) / k : 0;
  return L > j ? (L - 1 - j) / k + 1 : 0;
}
// Record plane of array j that holds the rank in order o (o != j).
__host__ __device__ __forceinline__ int plane_of(int j, int o, int k) { return (o - j - 1 + 2 * k) % k; }

// ---- learned CDF model ------------------------------------------------------
// A monotone piecewise-linear estimate F of the cumulative distribution of one
// coordinate, used by the learned presort to send a key straight to its
// bucket.  K segments split the value range [lo, hi] evenly; c[i] is F at the
// start of segment i (c[0] = 0, c[K] = 1, non-decreasing).  Keys are
// canonical (order-preserving) 32-bit words; at or below kmin F is 0, at or
// above kmax it is 1.  The model changes only where keys land, never the
// sorted result.
constexpr int kCdfSegments = 4096;
struct CdfModel {
  float lo, hi;      // value range of the training sample (finite values)
  float scale;       // K / (hi - lo), or 0 for a degenerate range
  uint32_t kmin;     // canonical key of lo
  uint32_t kmax;     // canonical key of hi
  int32_t is_float;  // coordinate type the model was trained on
  int32_t segments;  // K
  float loss;        // training loss at the last step
  float c[kCdfSegments + 1];
  float theta[kCdfSegments];  // trained parameters (segment-mass logits)
  float pad[55];
};
static_assert(sizeof(CdfModel) == 33024, "model size is part of the ABI");

// Order-preserving 32-bit key of a coordinate: int32 with the sign bit
// flipped (signed order); float32 under IEEE totalOrder (negative encodings
// complemented, non-negative ones with the sign bit set).
__device__ __forceinline__ uint32_t canon_word(uint32_t b, bool is_float) {
  return is_float ? (b ^ ((b >> 31) ? 0xFFFFFFFFu : 0x80000000u)) : (b ^ 0x80000000u);
}

// Coordinate value of a canonical key (monotone non-decreasing in the key).
__device__ __forceinline__ float cdf_key_value(uint32_t key, int is_float) {
  if (!is_float) return (float)(int32_t)(key ^ 0x80000000u);
  const uint32_t bits = (key & 0x80000000u) ? (key ^ 0x80000000u) : ~key;
  return __uint_as_float(bits);
}

// Segment index and fraction of a key strictly inside (kmin, kmax).
// Every operation is a separately rounded single-precision step: contraction
// into fused multiply-adds is switched off here (the library is built with
// -ffp-contract=fast-honor-pragmas), so every kernel that evaluates the model
// gets the same bits.
__device__ __forceinline__ int cdf_segment(float v, float lo, float scale, float* frac) {
#pragma clang fp contract(off)
  const float t = (v - lo) * scale;
  int i = t < (float)kCdfSegments ? (int)t : kCdfSegments - 1;
  if (i < 0) i = 0;
  float f = t - (float)i;
  f = f < 0.f ? 0.f : (f > 1.f ? 1.f : f);
  *frac = f;
  return i;
}

// F(key).  Monotone: inside a segment F grows with the fraction, and F never
// exceeds the next segment's start c[i+1].
__device__ __forceinline__ float cdf_eval(const float* c, float lo, float scale, uint32_t kmin,
                                          uint32_t kmax, int is_float, uint32_t key) {
#pragma clang fp contract(off)
  if (key <= kmin) return 0.f;
  if (key >= kmax) return 1.f;
  float f;
  const int i = cdf_segment(cdf_key_value(key, is_float), lo, scale, &f);
  const float a = c[i], b = c[i + 1];
  return fminf(a + f * (b - a), b);
}

// Bucket of a key among 2^nb_bits buckets.
__device__ __forceinline__ uint32_t cdf_bucket(float F, int nb_bits) {
#pragma clang fp contract(off)
  const uint32_t nb = 1u << nb_bits;
  const uint32_t b = (uint32_t)(F * (float)nb);
  return b < nb ? b : nb - 1;
}

// ---- rank-record layout ------------------------------------------------------------
// Array j (0 <= j < k) stores one record per position: k-1 ranks (plane c =
// rank in order (j + 1 + c) mod k).  Arrays are laid out one after another,
// array 0 first.  (Row ids are read from the order-0 sorted id array, at the
// order-0 rank.)
__device__ __host__ __forceinline__ int record_width(int, int k) { return k - 1; }
__device__ __host__ __forceinline__ int64_t record_offset(int j, int k, int64_t n) {
  return (int64_t)j * (k - 1) * n;
}
__device__ __host__ __forceinline__ int64_t record_words(int k, int64_t n) {
  return (int64_t)k * (k - 1) * n;
}

}  // namespace kd
