// Presort half of the build (Sec. 2.1 of Brown's paper): the k index arrays
// sorted by the cyclic super keys, and duplicate removal.
//
// The paper merge-sorts each index array by its super key.  Here every sort is
// a stable LSD radix sort over 32-bit key words (8-bit digits, onesweep passes
// with decoupled look-back).  The first array, sorted by x:y:z:..., is built
// word by word from the least significant word.  Duplicate rows are then
// adjacent, and one pass keeps the first of each run (Sec. 2.1).  The other
// arrays follow by a chain: the array for super key d is the stable sort of
// the array for super key d+1 (mod k) by word d alone, because ties on word d
// are then already in the order d+1 : d+2 : ... requires.
#include "common.hpp"
#include "launch.hpp"

namespace kd {

// ---- small utility kernels --------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, uint32_t value, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_store_i64(int64_t* dst, const int64_t* src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, value, count);
  return hipGetLastError();
}

hipError_t launch_store_i64(int64_t* dst, const int64_t* src, hipStream_t st) {
  hipLaunchKernelGGL(k_store_i64, dim3(1), dim3(64), 0, st, dst, src);
  return hipGetLastError();
}

// ---- key canonicalisation ----------------------------------------------------
// int32: flipping the sign bit turns signed order into unsigned order.
// float32: IEEE totalOrder becomes unsigned order when negative encodings are
// complemented and non-negative ones get the sign bit set.

__global__ __launch_bounds__(256) void k_canon(const uint32_t* __restrict__ t, int64_t n, int k,
                                              int is_float, uint32_t* __restrict__ keys) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int d = 0; d < k; ++d) {
      uint32_t b = t[i * k + d];
      uint32_t c = is_float ? (b ^ ((b >> 31) ? 0xFFFFFFFFu : 0x80000000u)) : (b ^ 0x80000000u);
      keys[(int64_t)d * n + i] = c;
    }
  }
}

hipError_t launch_canon(const void* tuples, int64_t n, int k, int is_float, uint32_t* keys,
                        hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_canon, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const uint32_t*>(tuples), n, k, is_float, keys);
  return hipGetLastError();
}

// ---- digit histograms ---------------------------------------------------------

template <bool kGather>
__global__ __launch_bounds__(256) void k_digit_hist(const uint32_t* __restrict__ col,
                                                   const uint32_t* __restrict__ ids, int64_t n_host,
                                                   const int64_t* n_dev, uint32_t* hist) {
  __shared__ uint32_t s[4 * kRadix];
  for (int i = threadIdx.x; i < 4 * kRadix; i += blockDim.x) s[i] = 0;
  __syncthreads();
  const int64_t n = n_dev ? *n_dev : n_host;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t key = kGather ? col[ids[i]] : col[i];
    atomicAdd(&s[0 * kRadix + (key & 0xFF)], 1u);
    atomicAdd(&s[1 * kRadix + ((key >> 8) & 0xFF)], 1u);
    atomicAdd(&s[2 * kRadix + ((key >> 16) & 0xFF)], 1u);
    atomicAdd(&s[3 * kRadix + (key >> 24)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 4 * kRadix; i += blockDim.x)
    if (s[i]) atomicAdd(&hist[i], s[i]);
}

hipError_t launch_digit_hist(const uint32_t* col, const uint32_t* ids, int64_t n,
                             const int64_t* n_dev, int gather, uint32_t* hist, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 4095) / 4096;
  if (blocks > 2048) blocks = 2048;
  if (gather)
    hipLaunchKernelGGL(k_digit_hist<true>, dim3((unsigned)blocks), dim3(256), 0, st, col, ids, n,
                       n_dev, hist);
  else
    hipLaunchKernelGGL(k_digit_hist<false>, dim3((unsigned)blocks), dim3(256), 0, st, col, ids, n,
                       n_dev, hist);
  return hipGetLastError();
}

// ---- onesweep scatter pass ------------------------------------------------------
// One workgroup = one tile of kSortTile elements, claimed in order from an
// atomic counter so that a tile only ever waits on tiles that started before
// it.  Ranking inside a wave is stable: items are taken in element order and
// lanes with equal digits are found with 8 ballots.  Each tile publishes its
// 256 digit counts, looks back for the counts of all earlier tiles, stages its
// elements in LDS in output order and writes them out in runs.

constexpr int kOsThreads = 256;
constexpr int kOsItems = kSortTile / kOsThreads;  // 16
constexpr int kOsWaves = kOsThreads / kWave;

template <int kMode, bool kWriteKeys>
__global__ __launch_bounds__(kOsThreads) void k_onesweep(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    const uint32_t* __restrict__ col, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, int64_t n_host, const int64_t* n_dev, int shift,
    const uint32_t* __restrict__ hist, uint32_t* lb, uint32_t* lb_other, uint32_t* counter,
    uint32_t* counter_other) {
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  __shared__ uint32_t s_wcnt[kOsWaves][kRadix];
  __shared__ uint32_t s_tile_excl[kRadix];
  __shared__ uint32_t s_gbase[kRadix];
  __shared__ uint32_t s_tmp[kOsWaves + 1];
  __shared__ uint32_t s_tile;

  const int tid = threadIdx.x;
  const int w = tid / kWave;
  const int lane = tid % kWave;
  if (tid == 0) s_tile = next_tile(counter);
#pragma unroll
  for (int q = 0; q < kOsWaves; ++q) s_wcnt[q][tid] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  lb_other[(int64_t)tile * kRadix + tid] = 0;
  if (tile == 0 && tid == 0) *counter_other = 0;

  const int64_t n = n_dev ? *n_dev : n_host;
  const int64_t base = (int64_t)tile * kSortTile;
  if (base >= n) return;

  uint32_t key[kOsItems], val[kOsItems], rank[kOsItems];
  const int64_t wbase = base + (int64_t)w * (kWave * kOsItems) + lane;
#pragma unroll
  for (int j = 0; j < kOsItems; ++j) {
    const int64_t i = wbase + j * kWave;
    if (i < n) {
      if (kMode == 0) {
        key[j] = keys_in[i];
        val[j] = vals_in[i];
      } else if (kMode == 1) {
        val[j] = vals_in[i];
        key[j] = col[val[j]];
      } else {
        val[j] = (uint32_t)i;
        key[j] = col[i];
      }
    } else {
      key[j] = 0;
      val[j] = 0xFFFFFFFFu;  // marks an empty slot
    }
  }

  const uint64_t below = lanes_below_mask();
#pragma unroll
  for (int j = 0; j < kOsItems; ++j) {
    const int64_t i = wbase + j * kWave;
    const bool valid = i < n;
    const uint32_t d = (key[j] >> shift) & 0xFF;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    uint32_t pre = 0;
    if (valid) pre = s_wcnt[w][d];
    __builtin_amdgcn_wave_barrier();
    const uint32_t before = popc64(m & below);
    if (valid && before == 0) s_wcnt[w][d] = pre + popc64(m);
    __builtin_amdgcn_wave_barrier();
    rank[j] = pre + before;
  }
  __syncthreads();

  // thread tid owns digit tid: wave bases and the tile count
  uint32_t tile_cnt = 0;
#pragma unroll
  for (int q = 0; q < kOsWaves; ++q) {
    const uint32_t c = s_wcnt[q][tid];
    s_wcnt[q][tid] = tile_cnt;
    tile_cnt += c;
  }

  // decoupled look-back on digit tid
  uint32_t* mine = lb + (int64_t)tile * kRadix + tid;
  uint32_t excl = 0;
  if (tile == 0) {
    st_flag(mine, kLbInc | tile_cnt);
  } else {
    st_flag(mine, kLbAgg | tile_cnt);
    int64_t t = (int64_t)tile - 1;
    uint32_t spins = 0;
    while (t >= 0) {
      const uint32_t v = ld_flag(lb + t * kRadix + tid);
      const uint32_t status = v >> 30;
      if (status == 0) {
        if (++spins > kSpinLimit) break;
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += v & kLbMask;
      if (status == 2) break;
      --t;
    }
    st_flag(mine, kLbInc | (excl + tile_cnt));
  }

  uint32_t total;
  const uint32_t hexcl = block_exclusive_sum<kOsThreads>(hist[tid], s_tmp, &total);
  s_gbase[tid] = hexcl + excl;
  const uint32_t texcl = block_exclusive_sum<kOsThreads>(tile_cnt, s_tmp, &total);
  s_tile_excl[tid] = texcl;
  __syncthreads();

#pragma unroll
  for (int j = 0; j < kOsItems; ++j) {
    const int64_t i = wbase + j * kWave;
    if (i < n) {
      const uint32_t d = (key[j] >> shift) & 0xFF;
      const uint32_t lpos = s_tile_excl[d] + s_wcnt[w][d] + rank[j];
      s_keys[lpos] = key[j];
      s_vals[lpos] = val[j];
    }
  }
  __syncthreads();

  const int tile_n = (int)((n - base) < kSortTile ? (n - base) : kSortTile);
  for (int i = tid; i < tile_n; i += kOsThreads) {
    const uint32_t kk = s_keys[i];
    const uint32_t d = (kk >> shift) & 0xFF;
    const int64_t g = (int64_t)s_gbase[d] + (i - (int64_t)s_tile_excl[d]);
    if (g < 0 || g >= n) continue;  // only reachable if the counts were inconsistent
    if (kWriteKeys) keys_out[g] = kk;
    vals_out[g] = s_vals[i];
  }
}

hipError_t launch_onesweep(int mode, const uint32_t* keys_in, const uint32_t* vals_in,
                           const uint32_t* col, uint32_t* keys_out, uint32_t* vals_out, int64_t n,
                           const int64_t* n_dev, int shift, const uint32_t* hist_pass,
                           const LookBack& lb, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned tiles = (unsigned)((n + kSortTile - 1) / kSortTile);
#define KD_OS(MODE, WK)                                                                       \
  hipLaunchKernelGGL((k_onesweep<MODE, WK>), dim3(tiles), dim3(kOsThreads), 0, st, keys_in,   \
                     vals_in, col, keys_out, vals_out, n, n_dev, shift, hist_pass, lb.cur,    \
                     lb.other, lb.counter, lb.counter_other)
  const bool wk = keys_out != nullptr;
  if (mode == 0) {
    if (wk) KD_OS(0, true); else KD_OS(0, false);
  } else if (mode == 1) {
    if (wk) KD_OS(1, true); else KD_OS(1, false);
  } else {
    if (wk) KD_OS(2, true); else KD_OS(2, false);
  }
#undef KD_OS
  return hipGetLastError();
}

// ---- duplicate removal --------------------------------------------------------
// Sec. 2.1: after the sort by x:y:z:..., identical rows are contiguous; keep
// the first of each run (the smallest row, the sort being stable).  The first
// key word arrives sorted alongside, so the other words are fetched only when
// it ties with the predecessor.  Kept ids are compacted with a single-word
// decoupled look-back per tile.

constexpr int kDdThreads = 256;
constexpr int kDdItems = kSortTile / kDdThreads;

__global__ __launch_bounds__(kDdThreads) void k_dedup(const uint32_t* __restrict__ ids,
                                                     const uint32_t* __restrict__ w0,
                                                     const uint32_t* __restrict__ keys, int64_t n,
                                                     int k, uint32_t* __restrict__ out_ids,
                                                     int64_t* nu, uint32_t* lb, uint32_t* lb_other,
                                                     uint32_t* counter, uint32_t* counter_other) {
  __shared__ uint32_t s_chunk[kDdItems * (kDdThreads / kWave)];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_base;
  const int tid = threadIdx.x;
  const int w = tid / kWave;
  if (tid == 0) s_tile = next_tile(counter);
  __syncthreads();
  const uint32_t tile = s_tile;
  if (tid == 0) {
    lb_other[tile] = 0;
    if (tile == 0) *counter_other = 0;
  }
  const int64_t base = (int64_t)tile * kSortTile;
  if (base >= n) return;

  uint32_t keep[kDdItems], id[kDdItems], within[kDdItems];
#pragma unroll
  for (int j = 0; j < kDdItems; ++j) {
    const int64_t i = base + j * kDdThreads + tid;
    keep[j] = 0;
    if (i < n) {
      id[j] = ids[i];
      keep[j] = 1;
      if (i > 0) {
        const uint32_t a = w0[i], b = w0[i - 1];
        if (a == b) {
          const uint32_t prev = ids[i - 1];
          bool same = true;
          for (int d = 1; d < k; ++d) {
            if (keys[(int64_t)d * n + id[j]] != keys[(int64_t)d * n + prev]) {
              same = false;
              break;
            }
          }
          keep[j] = same ? 0 : 1;
        }
      }
    }
    const uint32_t inc = wave_inclusive_sum(keep[j]);
    within[j] = inc - keep[j];
    if (lane_id() == kWave - 1) s_chunk[j * (kDdThreads / kWave) + w] = inc;
  }
  __syncthreads();
  // chunks are in element order (item-major, then wave): scan them in one wave
  constexpr int kChunks = kDdItems * (kDdThreads / kWave);
  static_assert(kChunks == kWave, "one wave scans the chunk totals");
  if (w == 0) {
    const uint32_t c = s_chunk[tid];
    const uint32_t inc = wave_inclusive_sum(c);
    s_chunk[tid] = inc - c;
    if (tid == kWave - 1) {
      const uint32_t tile_total = inc;
      uint32_t excl = 0;
      if (tile == 0) {
        st_flag(lb + tile, kLbInc | tile_total);
      } else {
        st_flag(lb + tile, kLbAgg | tile_total);
        int64_t t = (int64_t)tile - 1;
        uint32_t spins = 0;
        while (t >= 0) {
          const uint32_t v = ld_flag(lb + t);
          const uint32_t status = v >> 30;
          if (status == 0) {
            if (++spins > kSpinLimit) break;
            __builtin_amdgcn_s_sleep(1);
            continue;
          }
          excl += v & kLbMask;
          if (status == 2) break;
          --t;
        }
        st_flag(lb + tile, kLbInc | (excl + tile_total));
      }
      s_base = excl;
      if (base + kSortTile >= n) *nu = (int64_t)(excl + tile_total);
    }
  }
  __syncthreads();
  const uint32_t gb = s_base;
#pragma unroll
  for (int j = 0; j < kDdItems; ++j) {
    const int64_t o = (int64_t)gb + s_chunk[j * (kDdThreads / kWave) + w] + within[j];
    if (keep[j] && o < n) out_ids[o] = id[j];
  }
}

hipError_t launch_dedup(const uint32_t* ids, const uint32_t* w0, const uint32_t* keys, int64_t n,
                        int k, uint32_t* out_ids, int64_t* nu, const LookBack& lb, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned tiles = (unsigned)((n + kSortTile - 1) / kSortTile);
  hipLaunchKernelGGL(k_dedup, dim3(tiles), dim3(kDdThreads), 0, st, ids, w0, keys, n, k, out_ids,
                     nu, lb.cur, lb.other, lb.counter, lb.counter_other);
  return hipGetLastError();
}

// ---- rank records ----------------------------------------------------------------
// The tree phase compares ranks instead of tuples: the rank of a row in order
// q is its position in the deduplicated array sorted by super key q, and
// comparing two rows' super keys q is the same as comparing those ranks.

__global__ __launch_bounds__(256) void k_invert(const uint32_t* __restrict__ S, int64_t n, int k,
                                               const int64_t* nu_ptr, uint32_t* __restrict__ rank) {
  const int64_t nu = *nu_ptr;
  const int d = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nu;
       i += (int64_t)gridDim.x * blockDim.x)
    rank[(int64_t)d * n + S[(int64_t)d * n + i]] = (uint32_t)i;
}

hipError_t launch_invert(const uint32_t* S, int64_t n, int k, const int64_t* nu, uint32_t* rank,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_invert, dim3((unsigned)blocks, (unsigned)k), dim3(256), 0, st, S, n, k, nu,
                     rank);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_records(const uint32_t* __restrict__ S,
                                                const uint32_t* __restrict__ rank, int64_t n, int k,
                                                const int64_t* nu_ptr, uint32_t* __restrict__ rec) {
  const int64_t nu = *nu_ptr;
  const int j = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nu;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t id = S[(int64_t)j * n + i];
    for (int q = 0; q < k; ++q) {
      const uint32_t r = (q == j) ? (uint32_t)i : rank[(int64_t)q * n + id];
      rec[((int64_t)j * k + q) * n + i] = r;
    }
  }
}

hipError_t launch_records(const uint32_t* S, const uint32_t* rank, int64_t n, int k,
                          const int64_t* nu, uint32_t* rec, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_records, dim3((unsigned)blocks, (unsigned)k), dim3(256), 0, st, S, rank, n,
                     k, nu, rec);
  return hipGetLastError();
}

}  // namespace kd
