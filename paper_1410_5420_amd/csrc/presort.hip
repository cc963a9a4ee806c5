// Presort half of the build (Sec. 2.1 of Brown's paper): the k index arrays
// sorted by the cyclic super keys, and duplicate removal.
//
// The paper merge-sorts each index array by its super key.  Here every sort is
// a stable LSD radix sort over 32-bit key words (8-bit digits; each pass is a
// per-tile count, a scan and a scatter).  The first array, sorted by x:y:z:..., is built
// word by word from the least significant word.  Duplicate rows are then
// adjacent, and one pass keeps the first of each run (Sec. 2.1).  The other
// arrays follow by a chain: the array for super key d is the stable sort of
// the array for super key d+1 (mod k) by word d alone, because ties on word d
// are then already in the order d+1 : d+2 : ... requires.
//
// No pass reads anything out of order: every value a pass needs (the row id,
// the key words of later passes, the ranks known so far) travels with the key
// as a payload plane and is staged through LDS, so all global traffic is in
// coalesced runs.
#include <type_traits>

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

// Run r of the list is written by the workgroups with blockIdx.y == r.
__global__ __launch_bounds__(256) void k_fills(const FillList f) {
  const int r = blockIdx.y;
  uint32_t* p = f.p[r];
  const uint32_t v = f.value[r];
  const int c = f.count[r];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < c; i += gridDim.x * 256) p[i] = v;
}

hipError_t launch_fills(const FillList& f, hipStream_t st) {
  if (f.n < 0 || f.n > kMaxFills) return hipErrorInvalidValue;
  int32_t most = 0;
  for (int r = 0; r < f.n; ++r) {
    if (f.count[r] > 0 && f.p[r] == nullptr) return hipErrorInvalidValue;
    most = f.count[r] > most ? f.count[r] : most;
  }
  if (f.n == 0 || most <= 0) return hipSuccess;
  const int gx = (int)((most + 255) / 256 < 64 ? (most + 255) / 256 : 64);
  hipLaunchKernelGGL(k_fills, dim3(gx, f.n), dim3(256), 0, st, f);
  return hipGetLastError();
}

hipError_t launch_store_i64(int64_t* dst, const int64_t* src, hipStream_t st) {
  hipLaunchKernelGGL(k_store_i64, dim3(1), dim3(64), 0, st, dst, src);
  return hipGetLastError();
}

// ---- key canonicalisation ----------------------------------------------------
// canon_word (common.hpp) turns int32 signed order and float32 IEEE totalOrder
// into unsigned order; it is applied as the tuples are read.

// ---- tuple rows to planes -------------------------------------------------------
// A pass that reads one word of every row straight from the rows fetches the
// rows' cache lines once per word it reads; the words are therefore
// canonicalised into planes once, before the first sort.
__global__ __launch_bounds__(256) void k_rows_to_planes(const TupleSrc ts, int64_t n,
                                                       const PlaneOut out) {
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t* r = ts.t + i * ts.k;
    for (int d = 0; d < ts.k; ++d) out.p[d][i] = canon_word(r[d], ts.is_float);
  }
}

hipError_t launch_rows_to_planes(const TupleSrc& ts, int64_t n, const PlaneOut& out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  for (int d = 0; d < ts.k; ++d)
    if (out.p[d] == nullptr) return hipErrorInvalidValue;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_rows_to_planes, dim3((unsigned)blocks), dim3(256), 0, st, ts, n, out);
  return hipGetLastError();
}

// ---- radix passes: per-tile counts, a two-level scan, then the scatter ----------
// Every pass is three steps, with no workgroup waiting on another:
//   1. count:   tile t (512 * items elements) counts its digits (256, or 2048
//               for 11-bit digits) into cnt[t][d];
//   2. scan:    blocks of 64 tiles turn those into exclusive prefixes per digit
//               (plus per-block totals), one block then scans the block
//               totals and adds each digit's global start (two launches);
//               in a gated pass (one that usually does nothing) the count's
//               last workgroups do this instead, to save the two launches;
//   3. scatter: tile t ranks its elements stably (wave ballots), adds the
//               offsets, stages keys and payload planes through LDS in output
//               order and writes them out in runs.

constexpr int kOsThreads = 512;
constexpr int kOsWaves = kOsThreads / kWave;
constexpr int kScanGroup = 64;                      // tiles per first-level scan block
constexpr int kGatedGrid = 256;                     // workgroups of a gated pass (a multiple of 8)

// Geometry of a pass: digit width (8 or 11 bits: 4 or 3 passes per 32-bit
// word) and keys per thread (a tile of 512 * kItems keys).  Per-wave digit
// counters are 16-bit for 11-bit digits (a wave counts at most 64 * kItems
// keys), so that 2048 bins fit in LDS beside the tile.
template <int kB, int kI>
struct Geom {
  static constexpr int bits = kB;
  static constexpr int bins = 1 << kB;
  static constexpr uint32_t mask = (uint32_t)bins - 1u;
  static constexpr int items = kI;
  static constexpr int tile = kOsThreads * kI;
  using WCnt = typename std::conditional<(kB > 8), uint16_t, uint32_t>::type;
  // the threads that own digits for the tile scan own dpt consecutive ones
  static constexpr int dpt = bins > kOsThreads ? bins / kOsThreads : 1;
  static constexpr int owners = bins / dpt;
  static_assert(bins <= kMaxBins && tile >= kSortTile, "geometry within the workspace's sizing");
};

// Positions fit in 31 bits (n <= 2^30 - 1); only tuple rows are addressed in
// 64-bit, since row * k can exceed that.
__device__ __forceinline__ uint32_t plane_value(const Plane& pl, const TupleSrc& ts, int i) {
  if (pl.kind == kPlaneArray) return pl.in[i];
  if (pl.kind == kPlaneIndex) return (uint32_t)i;
  return canon_word(ts.t[(int64_t)i * ts.k + pl.word], ts.is_float);
}

// Learned digit source: the key's bucket under a CDF model (table in LDS).
struct ModelView {
  const float* c;
  float lo, scale;
  uint32_t kmin, kmax;
  int is_float, nb_bits;
};

// The level table (16 KiB) is copied to LDS (s_c, kCdfSegments + 1 floats):
// the keys of a tile look up segments all over it, which LDS serves far
// faster than the caches.  The copy is complete after the caller's next
// barrier.
__device__ __forceinline__ ModelView load_model(const RadixExtra& ex, float* s_c) {
  ModelView m;
  for (int i = threadIdx.x; i <= kCdfSegments; i += blockDim.x) s_c[i] = ex.model->c[i];
  m.c = s_c;
  m.lo = ex.model->lo;
  m.scale = ex.model->scale;
  m.kmin = ex.model->kmin;
  m.kmax = ex.model->kmax;
  m.is_float = ex.model->is_float;
  m.nb_bits = ex.nb_bits;
  return m;
}

__device__ __forceinline__ uint32_t model_bucket(const ModelView& m, uint32_t key) {
  return cdf_bucket(cdf_eval(m.c, m.lo, m.scale, m.kmin, m.kmax, m.is_float, key), m.nb_bits);
}

__device__ __forceinline__ bool gated_off(const RadixExtra& ex) {
  return ex.gate != nullptr && *ex.gate == 0;
}

// First level: exclusive prefix over the tiles of one group, per digit (256
// digits per block; blockIdx.y picks them).
template <int kBins>
__global__ __launch_bounds__(256) void k_radix_scan_tiles(uint32_t* __restrict__ cnt,
                                                         uint32_t* __restrict__ group_tot,
                                                         int tiles, const RadixExtra ex) {
  if (gated_off(ex)) return;
  const int d = blockIdx.y * 256 + threadIdx.x;
  const int t0 = blockIdx.x * kScanGroup;
  const int t1 = min(t0 + kScanGroup, tiles);
  uint32_t run = 0;
  for (int t = t0; t < t1; t += 8) {
    uint32_t c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = (t + q < t1) ? cnt[(int64_t)(t + q) * kBins + d] : 0u;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (t + q < t1) cnt[(int64_t)(t + q) * kBins + d] = run;
      run += c[q];
    }
  }
  group_tot[(int64_t)blockIdx.x * kBins + d] = run;
}

// Second level: one block turns group totals into group starts that already
// include every digit's global start.  256 digits: four threads per digit
// each take a quarter of the groups; 2048 digits: each thread takes two
// consecutive digits over all groups.  Loads are batched.
constexpr int kSgBatch = 16;
template <int kBins>
__global__ __launch_bounds__(1024) void k_radix_scan_groups(uint32_t* __restrict__ group_tot,
                                                           int groups, const RadixExtra ex) {
  constexpr int kSub = kBins <= 1024 ? 1024 / kBins : 1;  // threads per digit
  constexpr int kDpt = kBins <= 1024 ? 1 : kBins / 1024;  // digits per thread
  __shared__ uint32_t s_part[kSub][kBins <= 1024 ? kBins : 1];
  __shared__ uint32_t s_tmp[1024 / kWave + 1];
  if (gated_off(ex)) return;
  if constexpr (kDpt == 1) {
    const int d = threadIdx.x % kBins;
    const int sub = threadIdx.x / kBins;
    const int per = (groups + kSub - 1) / kSub;
    const int g0 = sub * per, g1 = min(groups, g0 + per);
    uint32_t sum = 0;
    for (int g = g0; g < g1; g += kSgBatch) {
      uint32_t c[kSgBatch];
#pragma unroll
      for (int q = 0; q < kSgBatch; ++q)
        c[q] = g + q < g1 ? group_tot[(int64_t)(g + q) * kBins + d] : 0u;
#pragma unroll
      for (int q = 0; q < kSgBatch; ++q) sum += c[q];
    }
    s_part[sub][d] = sum;
    __syncthreads();
    uint32_t digit_total = 0;
    if (sub == 0)
      for (int q = 0; q < kSub; ++q) digit_total += s_part[q][d];
    uint32_t all;
    const uint32_t digit_start = block_exclusive_sum<1024>(digit_total, s_tmp, &all);
    __syncthreads();
    if (sub == 0) {
      uint32_t run = digit_start;
      for (int q = 0; q < kSub; ++q) {
        const uint32_t c = s_part[q][d];
        s_part[q][d] = run;
        run += c;
      }
    }
    __syncthreads();
    uint32_t run = s_part[sub][d];
    for (int g = g0; g < g1; g += kSgBatch) {
      uint32_t c[kSgBatch];
#pragma unroll
      for (int q = 0; q < kSgBatch; ++q)
        c[q] = g + q < g1 ? group_tot[(int64_t)(g + q) * kBins + d] : 0u;
#pragma unroll
      for (int q = 0; q < kSgBatch; ++q) {
        if (g + q < g1) group_tot[(int64_t)(g + q) * kBins + d] = run;
        run += c[q];
      }
    }
  } else {
    const int d0 = threadIdx.x * kDpt;
    uint32_t tot[kDpt];
#pragma unroll
    for (int q = 0; q < kDpt; ++q) tot[q] = 0;
    for (int g = 0; g < groups; ++g)
#pragma unroll
      for (int q = 0; q < kDpt; ++q) tot[q] += group_tot[(int64_t)g * kBins + d0 + q];
    uint32_t mine = 0;
#pragma unroll
    for (int q = 0; q < kDpt; ++q) mine += tot[q];
    uint32_t all;
    uint32_t run0 = block_exclusive_sum<1024>(mine, s_tmp, &all);
    uint32_t run[kDpt];
#pragma unroll
    for (int q = 0; q < kDpt; ++q) {
      run[q] = run0;
      run0 += tot[q];
    }
    for (int g = 0; g < groups; ++g)
#pragma unroll
      for (int q = 0; q < kDpt; ++q) {
        uint32_t* p = group_tot + (int64_t)g * kBins + d0 + q;
        const uint32_t c = *p;
        *p = run[q];
        run[q] += c;
      }
  }
}

// How a count workgroup shares the scans: kSub threads split a digit's tiles
// (or groups), or each thread takes kDpt digits.  256 digits: 2 and 1; 2048
// digits: 1 and 4.
template <class G>
struct ScanShape {
  static constexpr int sub = G::bins >= kOsThreads ? 1 : kOsThreads / G::bins;
  static constexpr int dpt = G::bins >= kOsThreads ? G::bins / kOsThreads : 1;
  static constexpr int per = kScanGroup / sub;  // tiles of a group per thread
};

// Exclusive prefix over the tg tiles of group g, per digit, in place; the
// group's totals go to group_tot[g].  Called by the whole workgroup.
template <class G>
__device__ void scan_group(uint32_t* __restrict__ cnt, uint32_t* __restrict__ group_tot, int g,
                           int tg, uint32_t* s_part) {
  using S = ScanShape<G>;
  const int tid = threadIdx.x;
  const int sub = S::sub > 1 ? tid / G::bins : 0;
  const int lo = sub * S::per;
  const int64_t t0 = (int64_t)g * kScanGroup + lo;
  for (int q = 0; q < S::dpt; ++q) {
    const int d = S::sub > 1 ? tid % G::bins : q * kOsThreads + tid;
    uint32_t c[S::per];
#pragma unroll
    for (int u = 0; u < S::per; ++u) c[u] = lo + u < tg ? load_dev(cnt + (t0 + u) * G::bins + d) : 0u;
    uint32_t run = 0;
    if constexpr (S::sub > 1) {
      uint32_t sum = 0;
#pragma unroll
      for (int u = 0; u < S::per; ++u) sum += c[u];
      s_part[sub * G::bins + d] = sum;
      __syncthreads();
      for (int v = 0; v < sub; ++v) run += s_part[v * G::bins + d];
    }
#pragma unroll
    for (int u = 0; u < S::per; ++u) {
      if (lo + u < tg) cnt[(t0 + u) * G::bins + d] = run;
      run += c[u];
    }
    if (sub == S::sub - 1) store_dev(group_tot + (int64_t)g * G::bins + d, run);
  }
}

// Group totals to group starts that include every digit's global start, in
// place.  Called by the whole workgroup; s_start holds G::bins words.
template <class G>
__device__ void scan_groups(uint32_t* __restrict__ group_tot, int groups, uint32_t* s_part,
                            uint32_t* s_start, uint32_t* s_tmp) {
  using S = ScanShape<G>;
  const int tid = threadIdx.x;
  const int sub = S::sub > 1 ? tid / G::bins : 0;
  const int per = (groups + S::sub - 1) / S::sub;
  const int g0 = min(groups, sub * per), g1 = min(groups, g0 + per);
  auto digit = [&](int q) { return S::sub > 1 ? tid % G::bins : q * kOsThreads + tid; };
  uint32_t run[S::dpt];
  uint32_t base = 0;  // digits of the earlier q rounds
#pragma unroll
  for (int q = 0; q < S::dpt; ++q) {
    const int d = digit(q);
    uint32_t part = 0;
    for (int g = g0; g < g1; g += kSgBatch) {
      uint32_t c[kSgBatch];
#pragma unroll
      for (int u = 0; u < kSgBatch; ++u)
        c[u] = g + u < g1 ? load_dev(group_tot + (int64_t)(g + u) * G::bins + d) : 0u;
#pragma unroll
      for (int u = 0; u < kSgBatch; ++u) part += c[u];
    }
    // the digit's total, held by the thread of its first sub-range (those
    // threads come first and hold the digits in order), and the part of the
    // sub-ranges before this thread's
    uint32_t tot = part, before = 0;
    if constexpr (S::sub > 1) {
      s_part[sub * G::bins + d] = part;
      __syncthreads();
      tot = 0;
      if (sub == 0)
        for (int v = 0; v < S::sub; ++v) tot += s_part[v * G::bins + d];
      for (int v = 0; v < sub; ++v) before += s_part[v * G::bins + d];
    }
    uint32_t all;
    const uint32_t ds = base + block_exclusive_sum<kOsThreads>(tot, s_tmp, &all);
    base += all;
    if constexpr (S::sub > 1) {
      if (sub == 0) s_start[d] = ds;
      __syncthreads();
      run[q] = s_start[d] + before;
    } else {
      run[q] = ds;
    }
  }
#pragma unroll
  for (int q = 0; q < S::dpt; ++q) {
    const int d = digit(q);
    for (int g = g0; g < g1; g += kSgBatch) {
      uint32_t c[kSgBatch];
#pragma unroll
      for (int u = 0; u < kSgBatch; ++u)
        c[u] = g + u < g1 ? load_dev(group_tot + (int64_t)(g + u) * G::bins + d) : 0u;
#pragma unroll
      for (int u = 0; u < kSgBatch; ++u) {
        if (g + u < g1) group_tot[(int64_t)(g + u) * G::bins + d] = run[q];
        run[q] += c[u];
      }
    }
  }
}

// Workgroup b counts tiles b, b + grid, ... (one tile each in an ordinary
// pass), loading the next tile's keys while it counts the current one.
// kFused (gated passes): after a tile's counts are written, the last tile of
// its group to complete scans the group, and the last group to complete
// scans the groups, as the two scan launches would.  sync[0] counts
// completed groups and sync[1 + g] completed tiles of group g; atomicInc
// wraps each back to zero on its last arrival, so a pass leaves the counters
// as it found them.
template <class G, bool kFromTuples, bool kModel, bool kFused>
__global__ __launch_bounds__(kOsThreads) void k_radix_count(const uint32_t* __restrict__ keys_in,
                                                           const TupleSrc ts, int key_word,
                                                           int64_t n_host, const int32_t* n_dev,
                                                           int shift, uint32_t* __restrict__ cnt,
                                                           uint32_t* __restrict__ group_tot,
                                                           uint32_t* __restrict__ sync,
                                                           const RadixExtra ex) {
  __shared__ uint32_t s_h[G::bins];
  __shared__ uint32_t s_part[kFused && ScanShape<G>::sub > 1 ? kOsThreads : 1];
  __shared__ uint32_t s_tmp[kFused ? kOsWaves + 1 : 1];
  __shared__ float s_c[kModel ? kCdfSegments + 1 : 1];
  __shared__ int s_last;
  if (gated_off(ex)) return;
  const int tid = threadIdx.x;
  ModelView mv{};
  if constexpr (kModel) mv = load_model(ex, s_c);
  const int n = (int)(n_dev ? *n_dev : n_host);
  // every tile of the launch bound gets its row (zeros beyond the device count)
  const int tiles = (int)((n_host + G::tile - 1) / G::tile);
  const int groups = (tiles + kScanGroup - 1) / kScanGroup;
  uint32_t key[G::items];
  auto load = [&](int tile) {
    const int base = tile * G::tile;
#pragma unroll
    for (int j = 0; j < G::items; ++j) {
      const int i = base + j * kOsThreads + tid;
      key[j] = 0u;
      if (i < n)
        key[j] = kFromTuples ? canon_word(ts.t[(int64_t)i * ts.k + key_word], ts.is_float) : keys_in[i];
    }
  };
  int tile = blockIdx.x;
  if (tile < tiles) load(tile);
  for (; tile < tiles; tile += gridDim.x) {
    for (int d = tid; d < G::bins; d += kOsThreads) s_h[d] = 0;
    __syncthreads();
    const int base = tile * G::tile;
#pragma unroll
    for (int j = 0; j < G::items; ++j) {
      const int i = base + j * kOsThreads + tid;
      if (i < n) {
        const uint32_t kk = kModel ? model_bucket(mv, key[j]) : key[j];
        atomicAdd(&s_h[(kk >> shift) & G::mask], 1u);
      }
    }
    if (tile + (int)gridDim.x < tiles) load(tile + gridDim.x);
    __syncthreads();
    if constexpr (!kFused) {
      for (int d = tid; d < G::bins; d += kOsThreads) cnt[(int64_t)tile * G::bins + d] = s_h[d];
    } else {
      for (int d = tid; d < G::bins; d += kOsThreads) store_dev(cnt + (int64_t)tile * G::bins + d, s_h[d]);
      // every thread's counts have reached the device before the group's
      // counter moves
      wait_memory_ops();
      __syncthreads();
      const int g = tile / kScanGroup;
      const unsigned tg = (unsigned)min(kScanGroup, tiles - g * kScanGroup);
      if (tid == 0) s_last = atomicInc(&sync[1 + g], tg - 1u) == tg - 1u;
      __syncthreads();
      if (s_last) {
        wait_memory_ops();  // the counter was read before the other tiles' counts
        scan_group<G>(cnt, group_tot, g, (int)tg, s_part);
        wait_memory_ops();
        __syncthreads();
        if (tid == 0) s_last = atomicInc(&sync[0], (unsigned)groups - 1u) == (unsigned)groups - 1u;
        __syncthreads();
        if (s_last) {
          wait_memory_ops();  // the counter was read before the other groups' totals
          scan_groups<G>(group_tot, groups, s_part, s_h, s_tmp);
        }
      }
    }
    __syncthreads();  // s_h and s_last are reused by the next tile
  }
}

// XCD-aware: the padded tiles are split into 8 contiguous ranges, one per
// XCD, and workgroup b (on XCD b mod 8) walks its XCD's range with a stride of
// grid / 8 (one tile each in an ordinary pass), loading the next tile's keys
// while it writes the current tile's planes.
template <class G, bool kFromTuples, bool kWriteKeys, bool kModel, bool kLoop>
__global__ __launch_bounds__(kOsThreads) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const TupleSrc ts, int key_word,
    uint32_t* __restrict__ keys_out, const Payload pay, int64_t n_host, const int32_t* n_dev,
    int shift, const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ group_start,
    int tiles_pad, const RadixExtra ex) {
  constexpr int kItems = G::items;
  constexpr int kTile = G::tile;
  using WCnt = typename G::WCnt;
  // keys and staging; before the keys are placed, the model table lives here
  __shared__ uint32_t s_buf[2 * kTile];
  static_assert(2 * kTile >= kCdfSegments + 1, "model table fits the tile buffers");
  uint32_t* s_keys = s_buf;
  uint32_t* s_stage = s_buf + kTile;
  __shared__ WCnt s_wcnt[kOsWaves][G::bins];
  __shared__ uint32_t s_tile_excl[G::bins];
  __shared__ uint32_t s_gbase[G::bins];
  __shared__ uint32_t s_tmp[kOsWaves + 1];
  if (gated_off(ex)) return;

  const int tid = threadIdx.x;
  const int w = tid / kWave;
  const int lane = tid % kWave;
  const int n = (int)(n_dev ? *n_dev : n_host);
  ModelView mv{};
  const int range = tiles_pad / kXcds;
  const int xcd = blockIdx.x % kXcds, step = gridDim.x / kXcds;
  uint32_t key[kItems], rank[kItems];
  auto load_keys = [&](int tile) {
    const int wb = tile * kTile + w * (kWave * kItems) + lane;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int i = wb + j * kWave;
      key[j] = 0;
      if (i < n)
        key[j] = kFromTuples ? canon_word(ts.t[(int64_t)i * ts.k + key_word], ts.is_float)
                             : keys_in[i];
    }
  };
  int lt = blockIdx.x / kXcds;
  if (lt < range && (xcd * range + lt) * kTile < n) load_keys(xcd * range + lt);
  for (; lt < range; lt += step) {
  const int tile = xcd * range + lt;
  const int base = tile * kTile;
  if (base >= n) break;  // the XCD's later tiles lie further on
  for (int q = tid; q < kOsWaves * G::bins; q += kOsThreads) (&s_wcnt[0][0])[q] = 0;
  if constexpr (kModel) mv = load_model(ex, reinterpret_cast<float*>(s_buf));
  // global start of this tile's run of every digit
  for (int d = tid; d < G::bins; d += kOsThreads)
    s_gbase[d] = cnt[(int64_t)tile * G::bins + d] +
                 group_start[(int64_t)(tile / kScanGroup) * G::bins + d];
  const int wbase = base + w * (kWave * kItems) + lane;
  __syncthreads();
  // learned digits: rank by bucket (the raw key travels as a payload plane)
  if (kModel) {
#pragma unroll
    for (int j = 0; j < kItems; ++j) key[j] = model_bucket(mv, key[j]);
  }

  const uint64_t below = lanes_below_mask();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int i = wbase + j * kWave;
    const bool valid = i < n;
    const uint32_t d = (key[j] >> shift) & G::mask;
    const uint64_t m = same_digit_lanes<G::bits>(d, G::bits, __ballot(valid));
    uint32_t pre = 0;
    if (valid) pre = s_wcnt[w][d];
    __builtin_amdgcn_wave_barrier();
    const uint32_t before = lanes_below(m);
    if (valid && before == 0) s_wcnt[w][d] = (WCnt)(pre + popc64(m));
    __builtin_amdgcn_wave_barrier();
    rank[j] = pre + before;
  }
  __syncthreads();

  // the first G::owners threads own G::dpt consecutive digits each: wave
  // bases (exclusive over the waves, in place) and the tile's counts
  uint32_t own[G::dpt];
  uint32_t tile_cnt = 0;
  if (tid < G::owners) {
#pragma unroll
    for (int q = 0; q < G::dpt; ++q) {
      const int d = tid * G::dpt + q;
      uint32_t c_d = 0;
#pragma unroll
      for (int v = 0; v < kOsWaves; ++v) {
        const uint32_t c = s_wcnt[v][d];
        s_wcnt[v][d] = (WCnt)c_d;
        c_d += c;
      }
      own[q] = c_d;
      tile_cnt += c_d;
    }
  }
  uint32_t total;
  uint32_t texcl = block_exclusive_sum<kOsThreads>(tile_cnt, s_tmp, &total);
  if (tid < G::owners) {
#pragma unroll
    for (int q = 0; q < G::dpt; ++q) {
      s_tile_excl[tid * G::dpt + q] = texcl;
      texcl += own[q];
    }
  }
  __syncthreads();

  // local (tile-sorted) slot of every item
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int i = wbase + j * kWave;
    if (i < n) {
      const uint32_t d = (key[j] >> shift) & G::mask;
      rank[j] = s_tile_excl[d] + s_wcnt[w][d] + rank[j];
      s_keys[rank[j]] = key[j];
    }
  }
  __syncthreads();

  // global destination of every tile-sorted slot this thread writes out.  A
  // full tile (every tile but the last) writes every slot, so its stores and
  // loads need no guard: the compiler can then count them and wait for the
  // next plane's loads alone, not for the stores issued after them.
  const int tile_n = min(n - base, kTile);
  const bool full = tile_n == kTile;
  int dest[kItems];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int i = tid + j * kOsThreads;
    const uint32_t kk = s_keys[i];  // (a stale key beyond tile_n: its slot is not written)
    const uint32_t d = (kk >> shift) & G::mask;
    const int g = (int)s_gbase[d] + (i - (int)s_tile_excl[d]);
    // out of range only if the counts were inconsistent: flagged, and kept
    // inside the array
    bad = bad || (i < tile_n && (g < 0 || g >= n));
    dest[j] = i < tile_n ? min(max(g, 0), n - 1) : -1;
    if (kWriteKeys) {
      if (full)
        keys_out[dest[j]] = kk;
      else if (dest[j] >= 0)
        keys_out[dest[j]] = kk;
    }
  }
  // the next tile's keys load while this tile's planes are written
  if constexpr (kLoop)
    if (lt + step < range && (xcd * range + lt + step) * kTile < n) load_keys(xcd * range + lt + step);

  // payload planes: the next plane's values are loaded before the current
  // one is written out
  auto planes = [&](auto full_tag) {
    constexpr bool kFull = decltype(full_tag)::value;
    uint32_t nxt[kItems];
    auto load_plane = [&](const Plane& pl) {
      if (pl.kind == kPlaneArray) {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
          const int i = wbase + j * kWave;
          nxt[j] = (kFull || i < n) ? pl.in[i] : 0u;
        }
      } else {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
          const int i = wbase + j * kWave;
          nxt[j] = (kFull || i < n) ? plane_value(pl, ts, i) : 0u;
        }
      }
    };
    if (pay.count > 0) load_plane(pay.p[0]);
    for (int q = 0; q < pay.count; ++q) {
#pragma unroll
      for (int j = 0; j < kItems; ++j) {
        const int i = wbase + j * kWave;
        if (kFull || i < n) s_stage[rank[j]] = nxt[j];
      }
      if (q + 1 < pay.count) load_plane(pay.p[q + 1]);
      __syncthreads();
      uint32_t* out = pay.p[q].out;
#pragma unroll
      for (int j = 0; j < kItems; ++j) {
        if (kFull)
          out[dest[j]] = s_stage[tid + j * kOsThreads];
        else if (dest[j] >= 0)
          out[dest[j]] = s_stage[tid + j * kOsThreads];
      }
      __syncthreads();
    }
  };
  if (full)
    planes(std::true_type{});
  else
    planes(std::false_type{});
  if (bad && ex.status) atomicOr(ex.status, kStatusRadix);
  if constexpr (!kLoop) break;  // one tile per workgroup
  __syncthreads();  // LDS is reused by the next tile
  }
}

template <class G>
hipError_t radix_pass_g(const uint32_t* keys_in, const TupleSrc& ts, int key_word,
                        uint32_t* keys_out, const Payload& pay_in, int64_t n,
                        const int32_t* n_dev, int shift, uint32_t* cnt, uint32_t* group_tot,
                        hipStream_t st, const RadixExtra& ex) {
  const int tiles = (int)((n + G::tile - 1) / G::tile);
  const int groups = (tiles + kScanGroup - 1) / kScanGroup;
  const bool ft = keys_in == nullptr;
  const bool md = ex.model != nullptr;
  Payload pay = pay_in;
  if (md && keys_out) {
    // the kernel ranks by bucket; the raw key is moved like any payload plane
    if (pay.count >= kMaxPlanes) return hipErrorInvalidValue;
    Plane& pl = pay.p[pay.count++];
    pl.in = keys_in;
    pl.out = keys_out;
    pl.kind = ft ? kPlaneTupleWord : kPlaneArray;
    pl.word = key_word;
    keys_out = nullptr;
  }
  // one tile per workgroup; a gated pass (which usually does nothing) is
  // launched with a small persistent grid so that skipping it costs little
  const bool gated = ex.gate != nullptr;
  const int cgrid = gated && tiles > kGatedGrid ? kGatedGrid : tiles;
  const int tiles_pad = xcd_grid(tiles);
  const int sgrid = gated && tiles_pad > kGatedGrid ? kGatedGrid : tiles_pad;
  if (gated && ex.sync == nullptr) return hipErrorInvalidValue;
#define KD_RC(FT, MD)                                                                          \
  do {                                                                                         \
    if (gated)                                                                                 \
      hipLaunchKernelGGL((k_radix_count<G, FT, MD, true>), dim3(cgrid), dim3(kOsThreads), 0, st, \
                         keys_in, ts, key_word, n, n_dev, shift, cnt, group_tot, ex.sync, ex); \
    else                                                                                       \
      hipLaunchKernelGGL((k_radix_count<G, FT, MD, false>), dim3(cgrid), dim3(kOsThreads), 0,  \
                         st, keys_in, ts, key_word, n, n_dev, shift, cnt, group_tot, nullptr, ex); \
  } while (0)
  if (ft) {
    if (md) KD_RC(true, true); else KD_RC(true, false);
  } else {
    if (md) KD_RC(false, true); else KD_RC(false, false);
  }
#undef KD_RC
  if (!gated) {
    hipLaunchKernelGGL(k_radix_scan_tiles<G::bins>, dim3(groups, G::bins / 256), dim3(256), 0, st,
                       cnt, group_tot, tiles, ex);
    hipLaunchKernelGGL(k_radix_scan_groups<G::bins>, dim3(1), dim3(1024), 0, st, group_tot, groups, ex);
  }
#define KD_RS(FT, WK, MD)                                                                        \
  do {                                                                                           \
    if (gated)                                                                                   \
      hipLaunchKernelGGL((k_radix_scatter<G, FT, WK, MD, true>), dim3(sgrid), dim3(kOsThreads), 0, \
                         st, keys_in, ts, key_word, keys_out, pay, n, n_dev, shift, cnt,         \
                         group_tot, tiles_pad, ex);                                              \
    else                                                                                         \
      hipLaunchKernelGGL((k_radix_scatter<G, FT, WK, MD, false>), dim3(sgrid), dim3(kOsThreads), \
                         0, st, keys_in, ts, key_word, keys_out, pay, n, n_dev, shift, cnt,      \
                         group_tot, tiles_pad, ex);                                              \
  } while (0)
  const bool wk = keys_out != nullptr;
  if (md) {
    if (ft) KD_RS(true, false, true); else KD_RS(false, false, true);
  } else if (ft) {
    if (wk) KD_RS(true, true, false); else KD_RS(true, false, false);
  } else {
    if (wk) KD_RS(false, true, false); else KD_RS(false, false, false);
  }
#undef KD_RS
  return hipGetLastError();
}

hipError_t launch_radix_pass(const uint32_t* keys_in, const TupleSrc& ts, int key_word,
                             uint32_t* keys_out, const Payload& pay_in, int64_t n,
                             const int32_t* n_dev, int shift, uint32_t* cnt, uint32_t* group_tot,
                             hipStream_t st, const RadixExtra& ex) {
  if (n <= 0) return hipSuccess;
  // learned (model) passes rank by the bucket's 8-bit digits; every pass
  // takes the build's tile size
  const int bits = ex.model ? 8 : ex.bits;
  const int items = ex.items;
  if (bits == 8 && items == 8)
    return radix_pass_g<Geom<8, 8>>(keys_in, ts, key_word, keys_out, pay_in, n, n_dev, shift, cnt,
                                    group_tot, st, ex);
  if (bits == 8 && items == 16)
    return radix_pass_g<Geom<8, 16>>(keys_in, ts, key_word, keys_out, pay_in, n, n_dev, shift, cnt,
                                     group_tot, st, ex);
  if (bits == 11 && items == 8)
    return radix_pass_g<Geom<11, 8>>(keys_in, ts, key_word, keys_out, pay_in, n, n_dev, shift, cnt,
                                     group_tot, st, ex);
  if (bits == 11 && items == 16)
    return radix_pass_g<Geom<11, 16>>(keys_in, ts, key_word, keys_out, pay_in, n, n_dev, shift, cnt,
                                      group_tot, st, ex);
  return hipErrorInvalidValue;
}

// ---- word-0-first order of array 0 ------------------------------------------
// Appendix, "Optimized Super Key Comparison": compare word 0 first and look at
// the other words only on a tie.  Array 0 is radix-sorted by word 0 (then
// tree) alone, which leaves it in (tree, word 0, row) order; then every run of
// equal (tree, word 0) -- rare for most inputs -- is put in (word 1, ...,
// word k-1, row) order.  Runs of up to kSmallRun are ranked in LDS by the
// workgroup of their tile; longer ones are listed and ranked by a workgroup each,
// unless they are already in order (runs of identical rows).  A listed run longer than
// kBigRun, or a full list, raises the flag, and the complete radix sort then
// runs instead (gated on the flag).

constexpr int kSmallRun = 64;
constexpr int kBigRun = 4096;
constexpr int kTieTile = 1024;               // positions per workgroup
constexpr int kTieSpan = kTieTile + kSmallRun;  // plus the longest run crossing its end

__device__ __forceinline__ bool same_w0(const TieArgs& ta, int i, int j) {
  if (ta.tree && ta.tree[i] != ta.tree[j]) return false;
  return ta.w0[i] == ta.w0[j];
}

// (words 1 .. k-1, then row id) of position x before position y?
__device__ __forceinline__ bool tie_less(const TieArgs& ta, int64_t n, int x, int y) {
  for (int d = 1; d < ta.k; ++d) {
    const uint32_t* w = ta.planes + (int64_t)d * n;
    const uint32_t a = w[x], b = w[y];
    if (a != b) return a < b;
  }
  return ta.planes[x] < ta.planes[y];
}

constexpr int kTileThreads = 256;
constexpr int kTileItems = (kTieSpan + kTileThreads - 1) / kTileThreads;  // positions per thread
constexpr int kTileGrid = 1280;  // resident workgroups walking the tiles (5 per CU)

// Exclusive max over the threads of a kTileThreads workgroup (-1 for thread
// 0); s_tmp holds kTileThreads/64 words.  Contains barriers.
__device__ __forceinline__ int block_exclusive_max(int v, int* s_tmp) {
  const int lane = (int)lane_id(), w = threadIdx.x / kWave;
  const int inc = (int)wave_max_dpp((uint32_t)(v + 1)) - 1;  // values >= -1
  const int below = __shfl_up(inc, 1, kWave);
  if (lane == kWave - 1) s_tmp[w] = inc;
  __syncthreads();
  int res = lane > 0 ? below : -1;
  for (int i = 0; i < w; ++i) res = max(res, s_tmp[i]);
  __syncthreads();
  return res;
}

// Staged values of one tile: thread t holds local positions t - 1 + m * kTileThreads
// (position -1 is the one before the tile).
constexpr int kTileLoads = (kTieSpan + 1 + kTileThreads - 1) / kTileThreads;
struct TileRegs {
  uint32_t w0[kTileLoads], tr[kTileLoads], a[kTileLoads], b[kTileLoads], id[kTileLoads];
};

__device__ __forceinline__ int tile_span(int t0, int n) {
  return min(n, min(n, t0 + kTieTile) + kSmallRun) - t0;
}

__device__ __forceinline__ void tile_load(const TieArgs& ta, int n, int t0, TileRegs& r) {
  const int span = tile_span(t0, n);
  const uint32_t* w1 = ta.k > 1 ? ta.planes + (int64_t)n : nullptr;
  const uint32_t* w2 = ta.k > 2 ? ta.planes + 2 * (int64_t)n : nullptr;
#pragma unroll
  for (int m = 0; m < kTileLoads; ++m) {
    const int x = (int)threadIdx.x - 1 + m * kTileThreads;
    const int i = t0 + x;
    r.w0[m] = 0;
    r.tr[m] = 0xFFFFFFFFu;  // no predecessor: never equal (tree ids are small)
    r.a[m] = r.b[m] = r.id[m] = 0;
    if (x < span && i >= 0) {
      r.w0[m] = ta.w0[i];
      r.tr[m] = ta.tree ? ta.tree[i] : 0u;
      if (x >= 0) {
        if (w1) r.a[m] = w1[i];
        if (w2) r.b[m] = w2[i];
        r.id[m] = ta.planes[i];
      }
    }
  }
}

// Runs that start in a tile of kTieTile positions and hold at most kSmallRun
// elements are ordered in LDS.  The place of an element in its run is the
// number of the run's elements that precede it; the element-by-element
// comparisons this takes (the sum of the squared run lengths) are dealt out
// evenly to the threads, whatever the mix of run lengths.  Words 1 and 2 and
// the row id are staged; later words are read on ties of those.  The planes
// are then rewritten at the positions that moved.  Longer runs are listed for
// k_ties_big.  Each workgroup walks tiles with a grid stride and loads the
// next tile's planes into registers while it orders the current one.  Other
// workgroups rewrite only positions of runs that start in their own tiles, so
// values staged here for positions of such runs may be stale but are never
// used; word 0 and the tree ids are not written at all.
__global__ __launch_bounds__(kTileThreads) void k_ties_tile(const TieArgs ta, int64_t n_host,
                                                           int32_t* __restrict__ list,
                                                           int32_t* __restrict__ count,
                                                           int32_t* __restrict__ flag) {
  __shared__ uint32_t s_w0[kTieSpan + 1], s_tr[kTieSpan + 1];  // later: pair offsets, ranks
  __shared__ uint32_t s_a[kTieSpan], s_b[kTieSpan], s_id[kTieSpan];
  __shared__ int16_t s_start[kTieSpan];
  __shared__ uint16_t s_end[kTieSpan], s_perm[kTieSpan];
  __shared__ int s_tmp[kTileThreads / kWave + 1];
  const int n = (int)n_host;
  const int tid = threadIdx.x;
  const int tiles = (n + kTieTile - 1) / kTieTile;
  TileRegs r;
  if ((int)blockIdx.x < tiles) tile_load(ta, n, blockIdx.x * kTieTile, r);
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int t0 = tile * kTieTile;
    const int own = min(n, t0 + kTieTile) - t0;  // runs starting at local [0, own) are this tile's
    const int t2 = min(n, t0 + own + kSmallRun);
    const int span = t2 - t0;                     // staged local positions [0, span)
    // s_w0[x + 1] holds local position x, s_w0[0] the position before the tile
#pragma unroll
    for (int m = 0; m < kTileLoads; ++m) {
      const int x = tid - 1 + m * kTileThreads;
      if (x < span) {
        s_w0[x + 1] = r.w0[m];
        s_tr[x + 1] = r.tr[m];
        if (x >= 0) {
          s_a[x] = r.a[m];
          s_b[x] = r.b[m];
          s_id[x] = r.id[m];
          s_perm[x] = (uint16_t)x;
        }
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < tiles) tile_load(ta, n, (tile + gridDim.x) * kTieTile, r);
    auto same = [&](int x, int y) {  // local positions, -1 = the one before
      return s_w0[x + 1] == s_w0[y + 1] && s_tr[x + 1] == s_tr[y + 1];
    };
    // run starts: thread t holds positions [t * kTileItems, (t + 1) * kTileItems);
    // a position continuing the run before the tile gets start -1
    const int p0 = tid * kTileItems;
    int last = -1;
    for (int q = 0; q < kTileItems; ++q) {
      const int x = p0 + q;
      if (x < span && !same(x - 1, x)) last = x;
    }
    int st = block_exclusive_max(last, s_tmp);
    for (int q = 0; q < kTileItems; ++q) {
      const int x = p0 + q;
      if (x >= span) break;
      if (!same(x - 1, x)) st = x;
      s_start[x] = (int16_t)st;
      if (st >= 0 && (x + 1 == span || !same(x, x + 1))) s_end[st] = (uint16_t)(x + 1);
    }
    __syncthreads();
    // comparisons per element: its run's length, for runs of 2 .. kSmallRun
    // that start in the tile and end inside the staged span
    int len[kTileItems];
    int mine = 0;
    for (int q = 0; q < kTileItems; ++q) {
      const int x = p0 + q;
      len[q] = 0;
      if (x >= span) continue;
      const int s = s_start[x];
      if (s < 0 || s >= own) continue;
      const int e = s_end[s];
      if (e - s < 2) continue;
      const bool longer = (e - s > kSmallRun) || (e == span && t2 < n && same_w0(ta, t0 + s, t2));
      if (longer) {
        if (x == s) {
          const int idx = atomicAdd(count, 1);
          if (idx < kMaxTieRuns)
            list[idx] = t0 + s;
          else
            atomicOr(flag, 1);
        }
        continue;
      }
      len[q] = e - s;
      mine += len[q];
    }
    int total;
    int off = block_exclusive_sum<kTileThreads>(mine, s_tmp, &total);
    int* s_off = reinterpret_cast<int*>(s_w0);   // s_off[x]: first comparison of x; s_off[span] = total
    int* s_rank = reinterpret_cast<int*>(s_tr);  // elements of the run before x
    for (int q = 0; q < kTileItems; ++q) {
      const int x = p0 + q;
      if (x >= span) break;
      s_off[x] = off;
      s_rank[x] = 0;
      off += len[q];
    }
    if (tid == 0) s_off[span] = total;
    __syncthreads();
    auto less = [&](int x, int y) {  // local positions
      if (s_a[x] != s_a[y]) return s_a[x] < s_a[y];
      if (s_b[x] != s_b[y]) return s_b[x] < s_b[y];
      for (int d = 3; d < ta.k; ++d) {
        const uint32_t* w = ta.planes + (int64_t)d * n;
        const uint32_t a = w[t0 + x], b = w[t0 + y];
        if (a != b) return a < b;
      }
      return s_id[x] < s_id[y];
    };
    if (total > 0) {
      const int chunk = (total + kTileThreads - 1) / kTileThreads;
      const int c0 = min(total, tid * chunk), c1 = min(total, c0 + chunk);
      if (c0 < c1) {
        int lo = 0, hi = span - 1;  // the last x with s_off[x] <= c0 (it has len > 0)
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= c0)
            lo = mid;
          else
            hi = mid - 1;
        }
        int x = lo, ox = s_off[x], ex = s_off[x + 1], sx = s_start[x], c = 0;
        for (int w = c0; w < c1; ++w) {
          while (w >= ex) {  // next element with comparisons
            if (c) atomicAdd(&s_rank[x], c);
            c = 0;
            ++x;
            ox = s_off[x];
            ex = s_off[x + 1];
            sx = s_start[x];
          }
          c += less(sx + (w - ox), x) ? 1 : 0;
        }
        if (c) atomicAdd(&s_rank[x], c);
      }
      __syncthreads();
      for (int q = 0; q < kTileItems; ++q) {
        const int x = p0 + q;
        if (len[q]) s_perm[s_start[x] + s_rank[x]] = (uint16_t)x;
      }
      __syncthreads();
      // rewrite the planes where an element moved; planes 0..2 come from LDS,
      // later ones are staged through s_w0 (free once the places are known)
      for (int d = 0; d < ta.k; ++d) {
        uint32_t* w = ta.planes + (int64_t)d * n + t0;
        const uint32_t* src = d == 0 ? s_id : d == 1 ? s_a : d == 2 ? s_b : s_w0;
        if (d >= 3) {
          for (int x = tid; x < span; x += kTileThreads) s_w0[x] = w[x];
          __syncthreads();
        }
        for (int x = tid; x < span; x += kTileThreads)
          if (s_perm[x] != x) w[x] = src[s_perm[x]];
        if (d >= 3) __syncthreads();
      }
    }
    __syncthreads();  // LDS is refilled for the next tile
  }
}

// One workgroup per listed run: its length, whether it is already in order,
// every element's rank (the number of smaller elements in the run), then the
// planes permuted in place (every plane is read whole before it is written).
constexpr int kTieThreads = 256;
constexpr int kTieItems = kBigRun / kTieThreads;

__global__ __launch_bounds__(kTieThreads) void k_ties_big(const TieArgs ta, int64_t n_host,
                                                         const int32_t* __restrict__ list,
                                                         const int32_t* __restrict__ count,
                                                         int32_t* __restrict__ flag) {
  __shared__ int s_len, s_unsorted;
  const int n = (int)n_host;
  const int tid = threadIdx.x;
  const int runs = min(*count, kMaxTieRuns);
  for (int r = blockIdx.x; r < runs; r += gridDim.x) {
    const int s = list[r];
    if (tid == 0) {
      s_len = kBigRun + 1;
      s_unsorted = 0;
    }
    __syncthreads();
    // run length (at most kBigRun is looked at): the first position that differs
    for (int j = tid + 1; j <= kBigRun; j += kTieThreads)
      if (s + j >= n || !same_w0(ta, s, s + j)) atomicMin(&s_len, j);
    __syncthreads();
    const int L = s_len;
    if (L > kBigRun) {  // longer than a workgroup sorts: the full sort runs instead
      if (tid == 0) atomicOr(flag, 2);
      __syncthreads();
      continue;
    }
    for (int j = tid + 1; j < L; j += kTieThreads)
      if (tie_less(ta, n, s + j, s + j - 1)) s_unsorted = 1;
    __syncthreads();
    if (s_unsorted) {
      int rank[kTieItems];
#pragma unroll
      for (int q = 0; q < kTieItems; ++q) {
        const int j = tid + q * kTieThreads;
        rank[q] = 0;
        if (j < L) {
          int c = 0;
          for (int b = 0; b < L; ++b) c += tie_less(ta, n, s + b, s + j) ? 1 : 0;
          rank[q] = c;
        }
      }
      for (int d = 0; d < ta.k; ++d) {
        uint32_t* w = ta.planes + (int64_t)d * n + s;
        uint32_t v[kTieItems];
#pragma unroll
        for (int q = 0; q < kTieItems; ++q) {
          const int j = tid + q * kTieThreads;
          v[q] = j < L ? w[j] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kTieItems; ++q) {
          const int j = tid + q * kTieThreads;
          if (j < L) w[rank[q]] = v[q];
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

hipError_t launch_ties(const TieArgs& ta, int64_t n, int32_t* list, int32_t* count, int32_t* flag,
                       hipStream_t st) {
  if (n <= 1) return hipSuccess;
  const int64_t tiles = (n + kTieTile - 1) / kTieTile;
  const int64_t blocks = tiles < kTileGrid ? tiles : kTileGrid;
  hipLaunchKernelGGL(k_ties_tile, dim3((unsigned)blocks), dim3(kTileThreads), 0, st, ta, n, list, count, flag);
  hipLaunchKernelGGL(k_ties_big, dim3(1024), dim3(kTieThreads), 0, st, ta, n, list, count, flag);
  return hipGetLastError();
}

// ---- duplicate removal --------------------------------------------------------
// Sec. 2.1: after the sort by x:y:z:..., identical rows are contiguous; keep
// the first of each run (the smallest row, the sort being stable).  The sorted
// key words arrive as coalesced planes: w0 (the last sort key) and the
// payload planes [id, w1, ..., w_{k-1}], plus the tree id of every row when
// several trees are built at once (rows are then grouped by tree, and rows of
// different trees are never duplicates).  Three launches: per-tile counts of
// kept rows, one scan block, then the compaction, which writes the kept ids,
// their words w1..w_{k-1} (and tree ids) for the chain of sorts, and the
// start of every tree in the compacted order.

constexpr int kDdThreads = 512;
constexpr int kDdItems = kSortTile / kDdThreads;
constexpr int kDdWaves = kDdThreads / kWave;

__device__ __forceinline__ bool keep_row(const uint32_t* __restrict__ w0,
                                         const uint32_t* __restrict__ planes,
                                         const uint32_t* __restrict__ tree, int n, int k, int i) {
  if (i == 0) return true;
  if (tree && tree[i] != tree[i - 1]) return true;
  if (w0[i] != w0[i - 1]) return true;
  for (int d = 1; d < k; ++d) {
    const uint32_t* wd = planes + (int64_t)d * n;
    if (wd[i] != wd[i - 1]) return true;
  }
  return false;
}

__global__ __launch_bounds__(kDdThreads) void k_dedup_count(const uint32_t* __restrict__ w0,
                                                           const uint32_t* __restrict__ planes,
                                                           const uint32_t* __restrict__ tree,
                                                           int n, int k,
                                                           uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_part[kDdWaves];
  const int tid = threadIdx.x;
  const int base = blockIdx.x * kSortTile;
  // every position's first word and its predecessor's, loaded together
  // (clamped into the array); the other words only where they are equal
  uint32_t cur[kDdItems], prv[kDdItems];
#pragma unroll
  for (int j = 0; j < kDdItems; ++j) {
    const int i = min(base + j * kDdThreads + tid, n - 1);
    cur[j] = w0[i];
    prv[j] = w0[max(i - 1, 0)];
  }
  uint32_t c = 0;
#pragma unroll
  for (int j = 0; j < kDdItems; ++j) {
    const int i = base + j * kDdThreads + tid;
    if (i >= n) continue;
    if (i == 0 || cur[j] != prv[j] || keep_row(w0, planes, tree, n, k, i)) ++c;
  }
  c = wave_inclusive_sum(c);
  if (lane_id() == kWave - 1) s_part[tid / kWave] = c;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
    for (int q = 0; q < kDdWaves; ++q) t += s_part[q];
    cnt[blockIdx.x] = t;
  }
}

// One block: exclusive scan of the per-tile counts; the total goes to
// uoff[B] (the number of distinct rows over all trees).
__global__ __launch_bounds__(1024) void k_scan_counts(uint32_t* __restrict__ cnt, int tiles,
                                                     int32_t* total) {
  __shared__ uint32_t s_tmp[1024 / kWave + 1];
  __shared__ uint32_t s_carry;
  const int tid = threadIdx.x;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int t0 = 0; t0 < tiles; t0 += 1024) {
    const int t = t0 + tid;
    const uint32_t c = t < tiles ? cnt[t] : 0u;
    uint32_t all;
    const uint32_t ex = block_exclusive_sum<1024>(c, s_tmp, &all);
    const uint32_t carry = s_carry;
    if (t < tiles) cnt[t] = carry + ex;
    __syncthreads();
    if (tid == 0) s_carry = carry + all;
    __syncthreads();
  }
  if (tid == 0) *total = (int32_t)s_carry;
}

// K = k at compile time: every plane of a thread's positions is loaded once,
// together, and the same registers decide the kept rows and are written out.
template <int K>
__global__ __launch_bounds__(kDdThreads) void k_dedup_write(
    const uint32_t* __restrict__ w0, const uint32_t* __restrict__ planes,
    const uint32_t* __restrict__ tree, int n, const uint32_t* __restrict__ cnt,
    uint32_t* __restrict__ out_ids, uint32_t* __restrict__ out_words, int64_t out_stride,
    uint32_t* __restrict__ out_tree, int32_t* __restrict__ uoff) {
  __shared__ uint32_t s_chunk[kDdItems * kDdWaves];
  const int tid = threadIdx.x;
  const int wv = tid / kWave;
  const int lane = tid % kWave;
  const int base = blockIdx.x * kSortTile;
  if (base >= n) return;
  uint32_t id[kDdItems], key[kDdItems], prev[kDdItems];
  uint32_t wd[K > 1 ? K - 1 : 1][kDdItems];
#pragma unroll
  for (int j = 0; j < kDdItems; ++j) {
    const int i = base + j * kDdThreads + tid;
    const bool in = i < n;
    id[j] = in ? planes[i] : 0u;
    key[j] = in ? w0[i] : 0u;
    prev[j] = in && i > 0 ? w0[i - 1] : ~key[j];
#pragma unroll
    for (int d = 1; d < K; ++d) wd[d - 1][j] = in ? planes[(int64_t)d * n + i] : 0u;
  }
  uint32_t keep[kDdItems], within[kDdItems];
#pragma unroll
  for (int j = 0; j < kDdItems; ++j) {
    const int i = base + j * kDdThreads + tid;
    bool k1 = false;
    if (i < n) {
      k1 = i == 0 || key[j] != prev[j];
      if (!k1 && tree) k1 = tree[i] != tree[i - 1];
      if (!k1) {  // equal first words (rare): compare the others with the row before
#pragma unroll
        for (int d = 1; d < K; ++d) k1 = k1 || wd[d - 1][j] != planes[(int64_t)d * n + i - 1];
      }
    }
    keep[j] = k1 ? 1u : 0u;
    const uint32_t inc = wave_inclusive_sum(keep[j]);
    within[j] = inc - keep[j];
    if (lane == kWave - 1) s_chunk[j * kDdWaves + wv] = inc;
  }
  __syncthreads();
  static_assert(kDdItems * kDdWaves == kWave, "one wave scans the chunk totals");
  if (wv == 0) {
    const uint32_t c = s_chunk[lane];
    s_chunk[lane] = wave_inclusive_sum(c) - c;
  }
  __syncthreads();
  const uint32_t gb = cnt[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kDdItems; ++j) {
    const int i = base + j * kDdThreads + tid;
    const int o = (int)(gb + s_chunk[j * kDdWaves + wv] + within[j]);
    if (!keep[j] || o >= n) continue;
    out_ids[o] = id[j];
#pragma unroll
    for (int d = 1; d < K; ++d) out_words[(d - 1) * out_stride + o] = wd[d - 1][j];
    if (tree) {
      const uint32_t b = tree[i];
      out_tree[o] = b;
      if (i == 0 || tree[i - 1] != b) uoff[b] = o;  // first distinct row of tree b
    } else if (i == 0) {
      uoff[0] = 0;
    }
  }
}

hipError_t launch_dedup(const uint32_t* w0, const uint32_t* planes, const uint32_t* tree, int64_t n,
                        int k, uint32_t* out_ids, uint32_t* out_words, int64_t out_stride,
                        uint32_t* out_tree, uint32_t* cnt, int32_t* uoff, int num_trees,
                        hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int tiles = (int)((n + kSortTile - 1) / kSortTile);
  hipLaunchKernelGGL(k_dedup_count, dim3(tiles), dim3(kDdThreads), 0, st, w0, planes, tree, (int)n,
                     k, cnt);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, cnt, tiles, uoff + num_trees);
#define KD_DW(KK)                                                                                \
  hipLaunchKernelGGL(k_dedup_write<KK>, dim3(tiles), dim3(kDdThreads), 0, st, w0, planes, tree,    \
                     (int)n, cnt, out_ids, out_words, out_stride, out_tree, uoff)
  switch (k) {
    case 1: KD_DW(1); break;
    case 2: KD_DW(2); break;
    case 3: KD_DW(3); break;
    case 4: KD_DW(4); break;
    case 5: KD_DW(5); break;
    case 6: KD_DW(6); break;
    case 7: KD_DW(7); break;
    case 8: KD_DW(8); break;
    default: return hipErrorInvalidValue;
  }
#undef KD_DW
  return hipGetLastError();
}

// ---- forest bookkeeping ----------------------------------------------------------

// tree[r] = b for every row r of tree b (rows of tree b: off[b] .. off[b+1]-1).
__global__ __launch_bounds__(256) void k_tree_ids(const int64_t* __restrict__ off,
                                                 uint32_t* __restrict__ tree) {
  const int b = blockIdx.x;
  const int64_t s = off[b], e = off[b + 1];
  for (int64_t r = s + threadIdx.x; r < e; r += blockDim.x) tree[r] = (uint32_t)b;
}

hipError_t launch_tree_ids(const int64_t* off, int num_trees, uint32_t* tree, hipStream_t st) {
  if (num_trees <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tree_ids, dim3(num_trees), dim3(256), 0, st, off, tree);
  return hipGetLastError();
}

// After duplicate removal: trees with no rows start where the next tree
// starts; per-tree distinct counts go to n_unique[b]; lmax = deepest global
// level any tree needs; wgbase[b] = exclusive prefix of the on-chip finish
// items (2^(cutover depth)) of the trees, wgbase[B] their total.
__global__ __launch_bounds__(1024) void k_forest_finish(int32_t* __restrict__ uoff, int B,
                                                       int64_t cutover, int64_t* n_unique,
                                                       int32_t* lmax, int32_t* wgbase,
                                                       int32_t* queue) {
  __shared__ int32_t s_wmin[1024 / kWave];
  __shared__ uint32_t s_tmp[1024 / kWave + 1];
  __shared__ int32_t s_lmax[1024 / kWave];
  __shared__ uint32_t s_carry;
  const int tid = threadIdx.x;
  const int lane = (int)lane_id(), w = tid / kWave;
  // Empty trees (still marked INT32_MAX) start where the next tree starts:
  // every start becomes the minimum over itself and all later trees (starts of
  // non-empty trees increase with the tree index).  Thread t owns a range of
  // `per` trees: local minima, a suffix minimum over the ranges (lanes, then
  // waves), then local suffix minima.
  const int per = (B + 1023) / 1024;
  const int r0 = tid * per, r1 = min(B, r0 + per);
  int32_t m = INT32_MAX;
  for (int b = r1 - 1; b >= r0; --b) m = min(m, uoff[b]);
  int32_t incl = m;  // minimum over the ranges of this lane and the lanes above it
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t o = __shfl_down(incl, d, kWave);
    if (lane + d < kWave) incl = min(incl, o);
  }
  if (lane == 0) s_wmin[w] = incl;
  __syncthreads();
  int32_t after = uoff[B];  // minimum over every range after this thread's
  for (int q = w + 1; q < 1024 / kWave; ++q) after = min(after, s_wmin[q]);
  const int32_t above = __shfl_down(incl, 1, kWave);
  if (lane + 1 < kWave) after = min(after, above);
  {
    int32_t run = after;
    for (int b = r1 - 1; b >= r0; --b) {
      run = min(run, uoff[b]);
      uoff[b] = run;
    }
  }
  __syncthreads();
  int32_t lm = 0;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < B; c0 += 1024) {
    const int b = c0 + tid;
    uint32_t items = 0;
    if (b < B) {
      const int32_t nb = uoff[b + 1] - uoff[b];
      if (n_unique) n_unique[b] = nb;
      const int lc = cutover_depth(nb, cutover);
      lm = max(lm, lc);
      items = nb > 0 ? (1u << lc) : 0u;
    }
    uint32_t all;
    const uint32_t ex = block_exclusive_sum<1024>(items, s_tmp, &all);
    const uint32_t carry = s_carry;
    if (b < B) wgbase[b] = (int32_t)(carry + ex);
    __syncthreads();
    if (tid == 0) s_carry = carry + all;
    __syncthreads();
  }
  // block max of the deepest level
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) lm = max(lm, __shfl_xor(lm, d, kWave));
  if (lane_id() == 0) s_lmax[tid / kWave] = lm;
  __syncthreads();
  if (tid == 0) {
    int32_t m = 0;
    for (int q = 0; q < 1024 / kWave; ++q) m = max(m, s_lmax[q]);
    *lmax = m;
    wgbase[B] = (int32_t)s_carry;
    *queue = 0;
  }
}

hipError_t launch_forest_finish(int32_t* uoff, int num_trees, int64_t cutover, int64_t* n_unique,
                                int32_t* lmax, int32_t* wgbase, int32_t* queue, hipStream_t st) {
  hipLaunchKernelGGL(k_forest_finish, dim3(1), dim3(1024), 0, st, uoff, num_trees, cutover,
                     n_unique, lmax, wgbase, queue);
  return hipGetLastError();
}

// ---- rank records ----------------------------------------------------------------
// The tree phase compares ranks instead of tuples: the rank of a row in order
// q is its position in the deduplicated array sorted by super key q, and
// comparing two rows' super keys q is the same as comparing those ranks.
//
// Array j's record holds the k-1 ranks of the other orders, plane c being the
// rank in order (j + 1 + c) mod k (row ids are read from the order-0 sorted id
// array at the order-0 rank).  Planes are stored as separate columns (plane c of array j at
// record_offset(j) + c * n).  The chain of sorts fills most planes: the sort producing array
// d carries the ranks already known (its input position is the rank in order
// d+1).  Array 1 comes out complete; this kernel reads it and scatters the
// planes still missing: all of array 0's and, for d >= 2, the ranks in orders
// 1 .. d-1 of array d.

__global__ __launch_bounds__(256) void k_complete_records(uint32_t* __restrict__ rec, int64_t n,
                                                         int k, const int32_t* total) {
  const int64_t nu = *total;
  const int R = k - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nu;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t rv[kMaxK];
    rv[1 % k] = (uint32_t)i;
    const uint32_t* a1 = rec + record_offset(1, k, n);
    for (int c = 0; c < R; ++c) rv[(2 + c) % k] = a1[c * n + i];
    uint32_t* a0 = rec + record_offset(0, k, n);
    for (int c = 0; c < R; ++c) a0[c * n + rv[0]] = rv[(1 + c) % k];
    for (int j = 2; j < k; ++j) {
      uint32_t* aj = rec + record_offset(j, k, n);
      for (int c = k - j; c <= k - 2; ++c) aj[c * n + rv[j]] = rv[(j + 1 + c) % k];
    }
  }
}

// Placement: once the elements are grouped by key >> kPlaceBits (radix
// passes on those digits), the elements at positions [b * 4096, (b+1) * 4096)
// are exactly those whose keys -- a permutation of 0 .. nu-1 -- lie in that
// same range.  Workgroup b therefore gathers its values in LDS at key - base
// and writes the block out in order: every global write is coalesced.
constexpr int kPlaceBits = 12;
constexpr int kPlaceTile = 1 << kPlaceBits;

__global__ __launch_bounds__(512) void k_place(const uint32_t* __restrict__ key, const PlaceArgs pa,
                                              const int32_t* total, uint32_t* status) {
  constexpr int kItems = kPlaceTile / 512;
  extern __shared__ uint32_t s_val[];  // [nv][kPlaceTile]
  const int nu = *total;
  const int base = blockIdx.x * kPlaceTile;
  if (base >= nu) return;
  const int cnt = min(nu - base, kPlaceTile);
  // every position's slot, then each plane's values, loaded for all of a
  // thread's positions at once
  uint32_t slot[kItems];
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const int p = (int)threadIdx.x + q * 512;
    slot[q] = p < cnt ? key[base + p] - (uint32_t)base : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const int p = (int)threadIdx.x + q * 512;
    if (p < cnt && slot[q] >= (uint32_t)cnt) {  // not a permutation: the counts were inconsistent
      atomicOr(status, kStatusPlace);
      slot[q] = 0xFFFFFFFFu;
    }
  }
  for (int v = 0; v < pa.nv; ++v) {
    const uint32_t* src = pa.val[v] + base;
    uint32_t val[kItems];
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int p = (int)threadIdx.x + q * 512;
      val[q] = p < cnt ? src[p] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kItems; ++q)
      if (slot[q] < (uint32_t)cnt) s_val[v * kPlaceTile + slot[q]] = val[q];
  }
  __syncthreads();
  for (int v = 0; v < pa.nv; ++v) {
    uint32_t* d = pa.dst[v] + base;
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int p = (int)threadIdx.x + q * 512;
      if (p < cnt) d[p] = s_val[v * kPlaceTile + p];
    }
  }
}

int place_passes(int64_t n) {
  int bits = 1;
  while (((int64_t)1 << bits) < n) ++bits;
  const int rest = bits - kPlaceBits;
  return rest <= 0 ? 1 : (rest + kRadixBits - 1) / kRadixBits;
}
int place_shift(int pass) { return kPlaceBits + pass * kRadixBits; }

hipError_t launch_place(const uint32_t* key, const PlaceArgs& pa, int64_t n, const int32_t* total,
                        uint32_t* status, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = (size_t)pa.nv * kPlaceTile * 4;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_place),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int blocks = (int)((n + kPlaceTile - 1) / kPlaceTile);
  hipLaunchKernelGGL(k_place, dim3(blocks), dim3(512), lds, st, key, pa, total, status);
  return hipGetLastError();
}

hipError_t launch_complete_records(uint32_t* rec, int64_t n, int k, const int32_t* nu,
                                   hipStream_t st) {
  if (n <= 0 || k < 2) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_complete_records, dim3((unsigned)blocks), dim3(256), 0, st, rec, n, k, nu);
  return hipGetLastError();
}

}  // namespace kd
