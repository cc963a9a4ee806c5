// Tree half of the build (Sec. 2.1 of Brown's paper): split every subarray at
// the median of the array sorted by the current dimension and partition the
// other k-1 arrays about it, keeping their order, level by level.
//
// Arrays hold rank records instead of row indices: element x of array j is
// stored as its ranks in all k presorted orders (plane q = rank in order q).
// "super key p of x is below the median's" is then simply rank_p(x) <
// rank_p(median), so a level needs no access to the tuples at all, and every
// read and write is a coalesced stream.
//
// Global levels run while a subarray can exceed the cutover C; every array but
// the split one is partitioned by a stable segmented partition with one
// decoupled look-back per tile.  The split array itself is not moved
// (Appendix, "Optimized Partitioning": only k-1 arrays need partitioning);
// each array ping-pongs between two buffers, so its current buffer is a
// function of the depth and is recomputed on the device.  Subarrays of at
// most C elements are then finished in LDS by one workgroup each.
#include "common.hpp"
#include "launch.hpp"

namespace kd {

// number of levels below `depth` at which array j was moved (not the split array)
__device__ __host__ __forceinline__ int moves_before(int depth, int j, int k) {
  const int as_split = depth > j ? (depth - j + k - 1) / k : 0;
  return depth - as_split;
}

// ---- global level -------------------------------------------------------------

constexpr int kLvThreads = 256;
constexpr int kLvItems = kLevelTile / kLvThreads;  // 16
constexpr int kLvWaves = kLvThreads / kWave;
constexpr int kLvChunks = kLvItems * kLvWaves;     // 64

// 64-bit look-back word: [63:62] status, [61] segment head seen, [47:32] node
// count, [31:0] lower count.
constexpr uint64_t kLb64Agg = 1ull << 62;
constexpr uint64_t kLb64Inc = 2ull << 62;
constexpr uint64_t kLb64Head = 1ull << 61;

__device__ __forceinline__ uint64_t pack_counts(uint64_t lower, uint64_t node) {
  return (lower & 0xFFFFFFFFull) | ((node & 0xFFFFull) << 32);
}

// A global level only runs while every subarray holds at least C >= 1024
// elements, so a tile of 4096 positions meets at most kMaxSeg of them.
constexpr int kMaxSeg = 8;

template <int R>
__global__ __launch_bounds__(kLvThreads) void k_level(const uint32_t* __restrict__ buf0,
                                                     const uint32_t* __restrict__ buf1, int64_t n,
                                                     int k, int depth, int64_t cutover,
                                                     const int64_t* nu_ptr,
                                                     const uint32_t* __restrict__ S,
                                                     int32_t* __restrict__ perm, uint64_t* lb,
                                                     uint64_t* lb_other, uint32_t* counter,
                                                     uint32_t* counter_other, int tiles_per_array) {
  __shared__ uint32_t s_chunk[kLvChunks];
  __shared__ uint32_t s_pre[kLevelTile];
  __shared__ int64_t s_seg_s[kMaxSeg], s_seg_e[kMaxSeg];
  __shared__ uint32_t s_med[kMaxSeg];
  __shared__ uint32_t s_seg_pre[kMaxSeg];
  __shared__ int s_nseg;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_total;
  __shared__ uint64_t s_carry;

  const int tid = threadIdx.x;
  const int w = tid / kWave;
  if (tid == 0) s_tile = next_tile(counter);
  __syncthreads();
  const uint32_t tile_g = s_tile;
  if (tid == 0) {
    lb_other[tile_g] = 0;
    if (tile_g == 0) *counter_other = 0;
  }
  const int64_t nu = *nu_ptr;
  if (depth >= cutover_depth(nu, cutover)) return;
  const int p = depth % k;
  const int a = (int)(tile_g / (uint32_t)tiles_per_array);
  const int64_t t = tile_g % (uint32_t)tiles_per_array;
  const int j = (p + 1 + a) % k;
  const int64_t t0 = t * kLevelTile;
  if (t0 >= nu) return;
  const int64_t t1 = (t0 + kLevelTile < nu) ? t0 + kLevelTile : nu;

  const int64_t arr_stride = (int64_t)R * n;
  const bool odd_j = moves_before(depth, j, k) & 1;
  const uint32_t* src = (odd_j ? buf1 : buf0) + j * arr_stride;
  uint32_t* dst = const_cast<uint32_t*>(odd_j ? buf0 : buf1) + j * arr_stride;
  const uint32_t* split = ((moves_before(depth, p, k) & 1) ? buf1 : buf0) + p * arr_stride;

  if (tid == 0) {
    int ns = 0;
    int64_t pos = t0;
    while (pos < t1 && ns < kMaxSeg) {
      int64_t s, e;
      subarray_at(pos, nu, depth, &s, &e);
      if (e < s) {
        ++pos;  // node of a shallower level: no element lives here
        continue;
      }
      s_seg_s[ns] = s;
      s_seg_e[ns] = e;
      const int64_t m = median_of(s, e);
      const uint32_t r = split[(int64_t)p * n + m];  // the median's rank in order p
      s_med[ns] = r;
      if (a == 0 && m >= t0 && m < t1) perm[m] = (int32_t)S[(int64_t)p * n + r];
      ++ns;
      pos = e + 1;
    }
    s_nseg = ns;
  }
  __syncthreads();
  const int nseg = s_nseg;

  uint32_t v[R][kLvItems];
  uint32_t flag[kLvItems];
  int8_t sg[kLvItems];
  uint32_t within[kLvItems];
#pragma unroll
  for (int it = 0; it < kLvItems; ++it) {
    const int64_t i = t0 + it * kLvThreads + tid;
    sg[it] = -1;
    if (i < t1) {
      for (int q = 0; q < nseg; ++q) {
        if (i >= s_seg_s[q] && i <= s_seg_e[q]) {
          sg[it] = (int8_t)q;
          break;
        }
      }
    }
    if (sg[it] >= 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[q][it] = src[(int64_t)q * n + i];
    }
  }
#pragma unroll
  for (int it = 0; it < kLvItems; ++it) {
    uint32_t f = 0;
    if (sg[it] >= 0) {
      uint32_t rp = 0;
#pragma unroll
      for (int q = 0; q < R; ++q)
        if (q == p) rp = v[q][it];
      const uint32_t med = s_med[sg[it]];
      f = rp < med ? 1u : (rp == med ? 0x10000u : 0u);
    }
    flag[it] = f;
    const uint32_t inc = wave_inclusive_sum(f);
    within[it] = inc - f;
    if (lane_id() == kWave - 1) s_chunk[it * kLvWaves + w] = inc;
  }
  __syncthreads();
  if (w == 0) {
    const uint32_t c = s_chunk[tid];
    const uint32_t inc = wave_inclusive_sum(c);
    s_chunk[tid] = inc - c;
    if (tid == kWave - 1) s_total = inc;
  }
  __syncthreads();
  // exclusive in-tile prefix of every position, packed as lower | node << 16
#pragma unroll
  for (int it = 0; it < kLvItems; ++it) {
    const int64_t i = t0 + it * kLvThreads + tid;
    if (i < t1) s_pre[i - t0] = s_chunk[it * kLvWaves + w] + within[it];
  }
  __syncthreads();

  if (tid == 0) {
    const uint32_t tot = s_total;
    for (int q = 0; q < nseg; ++q) s_seg_pre[q] = s_seg_s[q] >= t0 ? s_pre[s_seg_s[q] - t0] : 0u;
    // counts of the tile's last subarray inside this tile
    const bool head = nseg == 0 || s_seg_s[nseg - 1] >= t0;
    const uint32_t lastv = nseg == 0 ? 0u : tot - s_seg_pre[nseg - 1];
    const bool need_carry = nseg > 0 && s_seg_s[0] < t0;
    uint64_t* mine = lb + tile_g;
    if (head)
      st_flag64(mine, kLb64Inc | kLb64Head | pack_counts(lastv & 0xFFFF, lastv >> 16));
    else
      st_flag64(mine, kLb64Agg | pack_counts(lastv & 0xFFFF, lastv >> 16));
    uint64_t lower = 0, node = 0;
    if (need_carry) {
      // counts of the first subarray in all earlier tiles
      int64_t tt = (int64_t)tile_g - 1;
      const int64_t first_tile = (int64_t)a * tiles_per_array;
      uint32_t spins = 0;
      while (tt >= first_tile) {
        const uint64_t x = ld_flag64(lb + tt);
        const uint64_t status = x >> 62;
        if (status == 0) {
          if (++spins > kSpinLimit) break;
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        lower += x & 0xFFFFFFFFull;
        node += (x >> 32) & 0xFFFFull;
        if (status == 2 || (x & kLb64Head)) break;
        --tt;
      }
      if (!head)
        st_flag64(mine, kLb64Inc | pack_counts(lower + (lastv & 0xFFFF), node + (lastv >> 16)));
    }
    s_carry = pack_counts(lower, node);
  }
  __syncthreads();
  const uint64_t carry = s_carry;
  const int64_t carry_lower = (int64_t)(carry & 0xFFFFFFFFull);
  const int64_t carry_node = (int64_t)((carry >> 32) & 0xFFFF);

#pragma unroll
  for (int it = 0; it < kLvItems; ++it) {
    if (sg[it] < 0 || flag[it] == 0x10000u) continue;
    const int q = sg[it];
    const int64_t i = t0 + it * kLvThreads + tid;
    const uint32_t pre = s_pre[i - t0];
    const int64_t s = s_seg_s[q], e = s_seg_e[q];
    const uint32_t base = s_seg_pre[q];
    int64_t low = (int64_t)(pre & 0xFFFF) - (base & 0xFFFF);
    int64_t nd = (int64_t)(pre >> 16) - (base >> 16);
    if (s < t0) {  // only the first subarray can start before the tile
      low += carry_lower;
      nd += carry_node;
    }
    const int64_t m = median_of(s, e);
    const int64_t dest = (flag[it] == 1u) ? s + low : m + 1 + (i - s - low - nd);
    if (dest < s || dest > e || dest == m) continue;  // only reachable if the counts were inconsistent
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(int64_t)r * n + dest] = v[r][it];
  }
}

hipError_t launch_level(const uint32_t* buf0, const uint32_t* buf1, int64_t n, int k, int depth,
                        int64_t cutover, const int64_t* nu, const uint32_t* S, int32_t* perm,
                        const LookBack64& lb, hipStream_t st) {
  if (n <= 0 || k < 2) return hipSuccess;
  const int tiles = (int)((n + kLevelTile - 1) / kLevelTile);
  const unsigned grid = (unsigned)(tiles * (k - 1));
#define KD_LV(RR)                                                                              \
  hipLaunchKernelGGL(k_level<RR>, dim3(grid), dim3(kLvThreads), 0, st, buf0, buf1, n, k, depth, \
                     cutover, nu, S, perm, lb.cur, lb.other, lb.counter, lb.counter_other, tiles)
  switch (k) {
    case 2: KD_LV(2); break;
    case 3: KD_LV(3); break;
    case 4: KD_LV(4); break;
    case 5: KD_LV(5); break;
    case 6: KD_LV(6); break;
    case 7: KD_LV(7); break;
    case 8: KD_LV(8); break;
    default: return hipErrorInvalidValue;
  }
#undef KD_LV
  return hipGetLastError();
}

// ---- on-chip finish (leaf phase) -----------------------------------------------------
// One workgroup takes one subarray of at most C elements at the cutover depth
// and runs all remaining levels in LDS.  Elements get local ids (their position
// in the array sorted by order 0), each array becomes a list of 16-bit local
// ids, and a level needs only "where does this id sit in the split array":
// the element goes to the lower half iff that position is below the median.

constexpr int kLfThreads = 256;

template <int kItems>
__global__ __launch_bounds__(kLfThreads) void k_leaf(const uint32_t* __restrict__ buf0,
                                                    const uint32_t* __restrict__ buf1, int64_t n,
                                                    int k, const int64_t* nu_ptr,
                                                    const uint32_t* __restrict__ S0,
                                                    int32_t* __restrict__ perm) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  constexpr int C = kItems * kLfThreads;
  const int64_t cutover = C;
  uint32_t* s_r0 = reinterpret_cast<uint32_t*>(s_raw);         // [C] rank in order 0 of each local id
  uint32_t* s_pre = s_r0 + C;                                  // [C] prefix counts
  uint16_t* s_segs = reinterpret_cast<uint16_t*>(s_pre + C);   // [C] subarray start per position
  uint16_t* s_sege = s_segs + C;                               // [C] subarray end per position
  uint16_t* s_pos = s_sege + C;                                // [C] position in split array per id
  uint16_t* s_out = s_pos + C;                                 // [C] node id per position
  uint16_t* s_tmp = s_out + C;                                 // [C]
  uint16_t* s_arr = s_tmp + C;                                 // [k][C]
  __shared__ uint32_t s_chunk[kWave + 1];

  const int tid = threadIdx.x;
  const int64_t nu = *nu_ptr;
  const int lc = cutover_depth(nu, cutover);
  const int64_t g = blockIdx.x;
  if (lc < 62 && g >= ((int64_t)1 << lc)) return;
  int64_t s = 0, e = nu - 1;
  for (int l = 0; l < lc; ++l) {
    const int64_t m = median_of(s, e);
    if ((g >> (lc - 1 - l)) & 1)
      s = m + 1;
    else
      e = m - 1;
  }
  const int N = (int)(e - s + 1);
  if (N <= 0) return;

  const int R = k;
  const int64_t arr_stride = (int64_t)R * n;
  // order-0 ranks of the subarray, ascending (array 0 is sorted by order 0)
  {
    const uint32_t* a0 = ((moves_before(lc, 0, k) & 1) ? buf1 : buf0);
    for (int i = tid; i < N; i += kLfThreads) {
      s_r0[i] = a0[0 * n + s + i];
      s_arr[i] = (uint16_t)i;
      s_segs[i] = 0;
      s_sege[i] = (uint16_t)(N - 1);
      s_out[i] = 0xFFFF;
    }
  }
  __syncthreads();
  for (int j = 1; j < k; ++j) {
    const uint32_t* aj = ((moves_before(lc, j, k) & 1) ? buf1 : buf0) + j * arr_stride;
    for (int i = tid; i < N; i += kLfThreads) {
      const uint32_t x = aj[0 * n + s + i];
      int lo = 0, hi = N;  // lower_bound
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_r0[mid] < x)
          lo = mid + 1;
        else
          hi = mid;
      }
      s_arr[j * C + i] = (uint16_t)(lo < N ? lo : N - 1);
    }
  }
  __syncthreads();

  constexpr int items = kItems;
  const int w = tid / kWave;
  constexpr int kWaves = kLfThreads / kWave;
  for (int depth = lc; (N >> (depth - lc)) > 0; ++depth) {
    const int p = depth % k;
    uint16_t* ap = s_arr + p * C;
    // where each live id sits in the split array; record the medians
    for (int i = tid; i < N; i += kLfThreads) {
      const int ss = s_segs[i], ee = s_sege[i];
      if (ss > ee) continue;
      const uint16_t id = ap[i];
      s_pos[id] = (uint16_t)i;
      if (i == ss + ((ee - ss) >> 1)) s_out[i] = id;
    }
    __syncthreads();
    for (int jj = 1; jj < k; ++jj) {
      const int j = (p + jj) % k;
      uint16_t* aj = s_arr + j * C;
      // flags and chunked prefix (chunk = 64 consecutive positions)
      uint32_t flag_reg[kItems], within_reg[kItems];
#pragma unroll
      for (int it = 0; it < items; ++it) {
        const int i = it * kLfThreads + tid;
        uint32_t f = 0;
        if (i < N) {
          const int ss = s_segs[i], ee = s_sege[i];
          if (ss <= ee) {
            const int m = ss + ((ee - ss) >> 1);
            const int pp = s_pos[aj[i]];
            f = pp < m ? 1u : (pp == m ? 0x10000u : 0u);
          }
        }
        const uint32_t inc = wave_inclusive_sum(f);
        flag_reg[it] = f;
        within_reg[it] = inc - f;
        if (lane_id() == kWave - 1) s_chunk[it * kWaves + w] = inc;
      }
      __syncthreads();
      if (w == 0) {
        const int nchunks = items * kWaves;
        const uint32_t c = tid < nchunks ? s_chunk[tid] : 0;
        const uint32_t inc = wave_inclusive_sum(c);
        if (tid < nchunks) s_chunk[tid] = inc - c;
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < items; ++it) {
        const int i = it * kLfThreads + tid;
        if (i < N) s_pre[i] = s_chunk[it * kWaves + w] + within_reg[it];
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < items; ++it) {
        const int i = it * kLfThreads + tid;
        if (i >= N) continue;
        const int ss = s_segs[i], ee = s_sege[i];
        if (ss > ee) continue;
        const uint32_t f = flag_reg[it];
        if (f == 0x10000u) continue;
        const int m = ss + ((ee - ss) >> 1);
        const uint32_t pre = s_pre[i], ps = s_pre[ss];
        const int low = (int)((pre & 0xFFFF) - (ps & 0xFFFF));
        const int nd = (int)((pre >> 16) - (ps >> 16));
        const int dest = (f == 1u) ? ss + low : m + 1 + (i - ss - low - nd);
        if (dest >= ss && dest <= ee) s_tmp[dest] = aj[i];
      }
      __syncthreads();
      // the partitioned list replaces array j (copy back keeps the layout fixed)
      for (int i = tid; i < N; i += kLfThreads) aj[i] = s_tmp[i];
      __syncthreads();
    }
    // next depth's subarrays
    for (int i = tid; i < N; i += kLfThreads) {
      const int ss = s_segs[i], ee = s_sege[i];
      if (ss > ee) continue;
      const int m = ss + ((ee - ss) >> 1);
      if (i < m) {
        s_sege[i] = (uint16_t)(m - 1);
      } else if (i > m) {
        s_segs[i] = (uint16_t)(m + 1);
      } else {
        s_segs[i] = 1;
        s_sege[i] = 0;
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < N; i += kLfThreads) {
    const int id = s_out[i];
    if (id >= N) continue;  // every position receives a node; kept as a guard
    const uint32_t r0 = s_r0[id];
    if (r0 < (uint64_t)nu) perm[s + i] = (int32_t)S0[r0];
  }
}

hipError_t launch_leaf(const uint32_t* buf0, const uint32_t* buf1, int64_t n, int k,
                       int64_t cutover, const int64_t* nu, const uint32_t* S, int32_t* perm,
                       int grid_bound_depth, hipStream_t st) {
  if (n <= 0 || k < 2) return hipSuccess;
  const size_t lds = (size_t)cutover * (4 + 4 + 2 * 5 + 2 * k);
  const unsigned grid = 1u << grid_bound_depth;
#define KD_LF(IT)                                                                              \
  do {                                                                                         \
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_leaf<IT>),              \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);  \
    if (e != hipSuccess) return e;                                                             \
    hipLaunchKernelGGL(k_leaf<IT>, dim3(grid), dim3(kLfThreads), lds, st, buf0, buf1, n, k, nu, \
                       S, perm);                                                               \
  } while (0)
  switch (cutover) {
    case 1024: KD_LF(4); break;
    case 2048: KD_LF(8); break;
    case 4096: KD_LF(16); break;
    default: return hipErrorInvalidValue;
  }
#undef KD_LF
  return hipGetLastError();
}

// ---- shape helpers ---------------------------------------------------------------

__global__ __launch_bounds__(256) void k_copy_k1(const uint32_t* __restrict__ S0,
                                                const int64_t* nu_ptr, int32_t* __restrict__ perm) {
  const int64_t nu = *nu_ptr;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nu;
       i += (int64_t)gridDim.x * blockDim.x)
    perm[i] = (int32_t)S0[i];
}

hipError_t launch_copy_k1(const uint32_t* S0, const int64_t* nu, int64_t n, int32_t* perm,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_copy_k1, dim3((unsigned)blocks), dim3(256), 0, st, S0, nu, perm);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_children(const int64_t* nu_ptr, int32_t* __restrict__ lo,
                                                 int32_t* __restrict__ hi) {
  const int64_t nu = *nu_ptr;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nu;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t s = 0, e = nu - 1;
    while (true) {
      const int64_t m = median_of(s, e);
      if (i < m) {
        e = m - 1;
      } else if (i > m) {
        s = m + 1;
      } else {
        lo[i] = (m - 1 >= s) ? (int32_t)median_of(s, m - 1) : -1;
        hi[i] = (e >= m + 1) ? (int32_t)median_of(m + 1, e) : -1;
        break;
      }
    }
  }
}

hipError_t launch_children(const int64_t* nu, int64_t n, int32_t* lo, int32_t* hi, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_children, dim3((unsigned)blocks), dim3(256), 0, st, nu, lo, hi);
  return hipGetLastError();
}

}  // namespace kd
