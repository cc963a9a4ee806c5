// Host-side launchers of the gfx950 kernels.  Each one enqueues work on the
// given stream and returns the launch status; none of them synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kd {

constexpr int kMaxK = 8;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kPassesPerWord = 32 / kRadixBits;
constexpr int kSortTile = 4096;   // elements per onesweep tile
constexpr int kLevelTile = 4096;  // elements per level-partition tile

// Ping-pong look-back state: the kernel that uses buffer `cur` clears its
// entries of buffer `other` (left by the previous launch of the same kind).
struct LookBack {
  uint32_t* cur;
  uint32_t* other;
  uint32_t* counter;
  uint32_t* counter_other;
};
struct LookBack64 {
  uint64_t* cur;
  uint64_t* other;
  uint32_t* counter;
  uint32_t* counter_other;
};

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t st);
hipError_t launch_store_i64(int64_t* dst, const int64_t* src, hipStream_t st);

// Order-preserving unsigned keys, one column per dimension (keys[d * n + i]).
hipError_t launch_canon(const void* tuples, int64_t n, int k, int is_float, uint32_t* keys,
                        hipStream_t st);

// Digit histograms of all four 8-bit digits of one 32-bit word.
//   gather == 0: key = col[i];  gather == 1: key = col[ids[i]]
// over i < (n_dev ? *n_dev : n).  hist must be zero beforehand (4*256 words).
hipError_t launch_digit_hist(const uint32_t* col, const uint32_t* ids, int64_t n,
                             const int64_t* n_dev, int gather, uint32_t* hist, hipStream_t st);

// One stable onesweep scatter pass on 8-bit digit `shift`.
//   mode 0: key = keys_in[i], val = vals_in[i]
//   mode 1: key = col[vals_in[i]], val = vals_in[i]
//   mode 2: key = col[i], val = i
// keys_out may be null (keys not needed afterwards).
hipError_t launch_onesweep(int mode, const uint32_t* keys_in, const uint32_t* vals_in,
                           const uint32_t* col, uint32_t* keys_out, uint32_t* vals_out, int64_t n,
                           const int64_t* n_dev, int shift, const uint32_t* hist_pass,
                           const LookBack& lb, hipStream_t st);

// Duplicate removal over the fully sorted order: ids[i] sorted, w0[i] its
// first key word.  Writes the kept ids compacted to out_ids and their count
// to *nu.
hipError_t launch_dedup(const uint32_t* ids, const uint32_t* w0, const uint32_t* keys, int64_t n,
                        int k, uint32_t* out_ids, int64_t* nu, const LookBack& lb, hipStream_t st);

// rank[d][S[d][i]] = i for i < nu, every d.
hipError_t launch_invert(const uint32_t* S, int64_t n, int k, const int64_t* nu, uint32_t* rank,
                         hipStream_t st);

// Level-0 rank records: rec[(j * k + q) * n + i] = rank of S[j][i] in order q.
hipError_t launch_records(const uint32_t* S, const uint32_t* rank, int64_t n, int k,
                          const int64_t* nu, uint32_t* rec, hipStream_t st);

// One global partition level (depth) of every array but the split one.
hipError_t launch_level(const uint32_t* buf0, const uint32_t* buf1, int64_t n, int k, int depth,
                        int64_t cutover, const int64_t* nu, const uint32_t* S, int32_t* perm,
                        const LookBack64& lb, hipStream_t st);

// On-chip finish of every subarray at the cutover depth.
hipError_t launch_leaf(const uint32_t* buf0, const uint32_t* buf1, int64_t n, int k,
                       int64_t cutover, const int64_t* nu, const uint32_t* S, int32_t* perm,
                       int grid_bound_depth, hipStream_t st);

// k == 1: the in-order layout is the sorted unique order.
hipError_t launch_copy_k1(const uint32_t* S0, const int64_t* nu, int64_t n, int32_t* perm,
                          hipStream_t st);

// Child positions from the implicit shape.
hipError_t launch_children(const int64_t* nu, int64_t n, int32_t* lo, int32_t* hi, hipStream_t st);

}  // namespace kd
