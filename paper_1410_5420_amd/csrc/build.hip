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

// Record buffers: level-0 records stay untouched in rec0 (they double as the
// rank-translation tables); moved arrays alternate between b1 and b2.  rows:
// the row id of every order-0 rank (the deduplicated order-0 id array).
// Deferred partitioning (Appendix, "Deferred Merge Sort and Partitioning",
// in the form that suits radix sorts; one tree only): every array j >= 2
// keeps its presorted order until depth j and then reaches its depth-j
// layout in one stable split (one write into b1), which stands for its
// first j moves.
struct RecBufs {
  const uint32_t* rec0;
  const uint32_t* rows;
  uint32_t* b1;
  uint32_t* b2;
};
__device__ __forceinline__ const uint32_t* buf_after(const RecBufs& B, int moves) {
  return moves == 0 ? B.rec0 : ((moves & 1) ? B.b1 : B.b2);
}
// Writes into array j's records before `depth`.  Deferred, an array j >= 2
// is only read from depth j on, or by the on-chip finish of a tree whose
// global levels end above depth j; its split output counts as one write.
__device__ __host__ __forceinline__ int array_moves(int defer, int depth, int j, int k) {
  if (!defer || j < 2) return moves_before(depth, j, k);
  return depth >= j ? moves_before(depth, j, k) - (j - 1) : 1;
}
// Array j's records as they are at `depth` (kDefer: deferred partitioning;
// a template argument, so that the plain build carries no test of it).
template <bool kDefer>
__device__ __forceinline__ const uint32_t* rec_array(const RecBufs& B, int depth, int j, int k,
                                                     int64_t n) {
  return buf_after(B, array_moves(kDefer ? 1 : 0, depth, j, k)) + record_offset(j, k, n);
}

// The on-chip finish's view of array j at the cutover depth: form 0 (levels
// of form 1/2), 1 (deferred partitioning) or 2 (one split per level, whose
// last split of each array the finish reads brought it to that depth).
template <int kForm>
__device__ __forceinline__ const uint32_t* leaf_array(const RecBufs& B, int depth, int j, int k,
                                                      int64_t n) {
  int moves;
  if constexpr (kForm == 2)
    moves = roll_moves(depth, j, k) + (depth >= 1 && roll_depth(depth, j, k) < depth ? 1 : 0);
  else
    moves = array_moves(kForm, depth, j, k);
  return buf_after(B, moves) + record_offset(j, k, n);
}

// ---- forests ------------------------------------------------------------------
// Several independent trees are built at once as a forest.  In the sorted
// orders the distinct rows of tree b occupy positions uoff[b] .. uoff[b+1]-1
// (ranks are global positions, consistent within each tree); in the input and
// in perm, tree b owns rows off[b] .. off[b+1]-1.  A single build is a forest
// of one tree.
struct Forest {
  int B;
  const int64_t* off;
  const int32_t* uoff;
  const int32_t* lmax;    // deepest global level any tree needs
  const int32_t* wgbase;  // on-chip finish items of tree b: wgbase[b] .. wgbase[b+1]-1
  int32_t* queue;         // work counter of the on-chip finish (zero before it runs)
  uint32_t* status;       // the build's status word
};

// Largest b < B with v[b] <= x (v non-decreasing, v[0] <= x).
__device__ __forceinline__ int upper_index(const int32_t* v, int B, int x) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (v[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Subarray of the forest at `depth` that contains position pos, or e < s when
// pos is the node of a shallower level or its tree is finished on-chip from
// a shallower depth.  *tree receives the tree.
__device__ __forceinline__ void forest_subarray(const Forest& F, int64_t cutover, int pos,
                                                int depth, int* s_out, int* e_out, int* tree) {
  const int b = F.B == 1 ? 0 : upper_index(F.uoff, F.B, pos);
  const int base = F.uoff[b];
  const int nb = F.uoff[b + 1] - base;
  *tree = b;
  if (depth >= cutover_depth(nb, cutover)) {
    *s_out = 1;
    *e_out = 0;
    return;
  }
  int s, e;
  subarray_at(pos - base, nb, depth, &s, &e);
  *s_out = s + base;
  *e_out = e + base;
}

// ---- global level -------------------------------------------------------------
// A level is three launches with no waiting between workgroups:
//   1. seg:   one workgroup per tile finds the subarrays that meet it and
//      their medians' ranks (and records the medians' row ids), and counts,
//      in every moving array, the elements of the tile's last subarray piece
//      that go to the lower half and whether the median itself is there;
//   2. scan:  one block per array chains those counts from tile to tile
//      along each subarray (a segmented scan);
//   3. move:  tile t recomputes its elements' sides, adds the in-tile prefix
//      to the carried counts and writes every rank plane to its new place.
// (A look-back form that chains the counts inside the move launch follows
// the move kernel.)

constexpr int kLvThreads = 512;
constexpr int kLvItems = kLevelTile / kLvThreads;  // 8
constexpr int kLvWaves = kLvThreads / kWave;
constexpr int kLvChunks = kLvItems * kLvWaves;     // 64

// A global level only runs while every subarray holds at least C >= 1024
// elements, so a tile of 4096 positions meets at most kMaxSeg of them and
// every one of them contains one of the sample positions t0, t0+512, ...,
// t0+3584, t1-1 (or the position after it, when the sample is a node).
constexpr int kMaxSeg = 8;
constexpr int kSamples = kLevelTile / 512 + 1;

// Subarrays meeting a tile, shared by the count and move launches.
struct SegInfo {
  int32_t s[kMaxSeg];
  int32_t e[kMaxSeg];
  uint32_t med[kMaxSeg];  // the median's rank in the split order
  int32_t nseg;
  int32_t pad;
};

// Sum over a wave (all lanes active), the same in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  if constexpr (sizeof(T) == 4) {
    return (T)__builtin_amdgcn_readlane((int)wave_scan_dpp((uint32_t)v), kWave - 1);
  } else {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
  }
}

// Wave 0 of a block: subarrays meeting [t0, t1) at `depth`, their medians'
// ranks in order p, and (write_perm) the row id of every median in the tile.
template <bool kDefer>
__device__ void find_subarrays(const RecBufs& B, const Forest& F, int64_t n, int k, int depth,
                               int64_t cutover, int t0, int t1, bool write_perm, int32_t* perm,
                               SegInfo* out) {
  const int lane = lane_id();
  const int p = depth % k;
  int s = INT32_MAX, e = -1, tr = 0;
  if (lane < kSamples) {
    int pos = t0 + lane * 512;
    if (pos > t1 - 1) pos = t1 - 1;
    forest_subarray(F, cutover, pos, depth, &s, &e, &tr);
    if (e < s && pos + 1 < t1) forest_subarray(F, cutover, pos + 1, depth, &s, &e, &tr);
    if (e < s) {
      s = INT32_MAX;
      e = -1;
    }
  }
  const int prev_s = __shfl_up(s, 1, kWave);
  const bool keep = lane < kSamples && s != INT32_MAX && (lane == 0 || prev_s != s);
  const uint64_t km = __ballot(keep);
  if (keep) {
    const int idx = (int)popc64(km & lanes_below_mask());
    if (idx < kMaxSeg) {
      out->s[idx] = s;
      out->e[idx] = e;
      // The median's rank in order p: the split array's record holds its rank
      // in order p+1 (plane 0), and the level-0 records of array p+1 translate
      // that (their plane k-2 is order p).
      const int m = s + ((e - s) >> 1);
      const uint32_t* split = rec_array<kDefer>(B, depth, p, k, n);
      const uint32_t r1 = split[m];
      const int p1 = (p + 1) % k;
      const uint32_t rp = B.rec0[record_offset(p1, k, n) + (int64_t)(k - 2) * n + r1];
      out->med[idx] = rp;
      if (write_perm && m >= t0 && m < t1) {
        // the row id is found at the median's rank in order 0: that is rp
        // itself when p == 0, otherwise plane (k - p - 1) of its record
        const uint32_t r0 = p == 0 ? rp : split[(int64_t)((k - p - 1) % k) * n + m];
        const int64_t row = B.rows[r0];
        const int64_t ob = F.off[tr];
        perm[ob + (m - F.uoff[tr])] = (int32_t)(row - ob);
      }
    }
  }
  if (lane == 0) {
    const int ns = (int)popc64(km);
    if (ns > kMaxSeg) atomicOr(F.status, kStatusLevelSeg);  // subarrays below C elements
    out->nseg = min(ns, kMaxSeg);
  }
}

// Subarrays meeting every tile, their medians' ranks, and the row ids of the
// medians inside the tile (wave 0 of a workgroup per tile); then, for every
// moving array, the counts of the tile's last subarray piece (lower | node <<
// 32), whether that subarray starts inside the tile (bit 48) and whether the
// tile's first subarray started before it (bit 49).  The rank planes are
// loaded before the subarrays are known, so the loads overlap that search.
constexpr int kSegThreads = 256;
constexpr int kSegItems = kLevelTile / kSegThreads;
// R: moving arrays counted (k - 1, or 0 when only the subarrays are wanted)
template <int R, bool kDefer>
__global__ __launch_bounds__(kSegThreads) void k_level_seg(const RecBufs B, const Forest F, int64_t n,
                                                          int k, int depth, int64_t cutover,
                                                          int32_t* __restrict__ perm,
                                                          SegInfo* __restrict__ seginfo,
                                                          uint64_t* __restrict__ tval, int tiles,
                                                          uint64_t wmasks) {
  __shared__ SegInfo s_si;
  __shared__ uint32_t s_c[kMaxK];
  const int tid = threadIdx.x;
  const int t = blockIdx.x;
  const int t0 = t * kLevelTile;
  if (t >= tiles) return;
  // The rank planes are loaded first, bounded by the rows (every plane holds
  // n entries); the device counts decide afterwards what is used.
  const int tl = (int)min((int64_t)t0 + kLevelTile, n);
  const int p = depth % k;
  constexpr int arrays = R;
  uint32_t rp[R > 0 ? R : 1][kSegItems];
#pragma unroll
  for (int a = 0; a < R; ++a) {
    const int j = (p + 1 + a) % k;
    const int cp = (p - j - 1 + 2 * k) % k;  // the plane holding the rank in order p
    const uint32_t* plane = rec_array<kDefer>(B, depth, j, k, n) + (int64_t)cp * n;
    // an array that writes no plane at this level stays put: no counts
    const bool need = ((wmasks >> (8 * j)) & 0xFFu) != 0;
#pragma unroll
    for (int it = 0; it < kSegItems; ++it) {
      const int i = t0 + it * kSegThreads + tid;
      rp[a][it] = need && i < tl ? plane[i] : 0u;
    }
  }
  const int nu = F.uoff[F.B];
  if (depth >= *F.lmax || t0 >= nu) return;
  const int t1 = min(t0 + kLevelTile, nu);
  if (tid < kWave)
    find_subarrays<kDefer>(B, F, n, k, depth, cutover, t0, t1, true, perm, &s_si);
  if (tid < kMaxK) s_c[tid] = 0;
  __syncthreads();
  if (tid < kMaxSeg) {
    seginfo[t].s[tid] = s_si.s[tid];
    seginfo[t].e[tid] = s_si.e[tid];
    seginfo[t].med[tid] = s_si.med[tid];
    if (tid == 0) seginfo[t].nseg = s_si.nseg;
  }
  if (R == 0) return;
  const int ns = s_si.nseg;
  int from = t1, to = t1;
  uint32_t med = 0;
  if (ns > 0) {
    from = max(s_si.s[ns - 1], t0);
    to = min(s_si.e[ns - 1] + 1, t1);
    med = s_si.med[ns - 1];
  }
#pragma unroll
  for (int a = 0; a < R; ++a) {
    uint32_t c = 0;
#pragma unroll
    for (int it = 0; it < kSegItems; ++it) {
      const int i = t0 + it * kSegThreads + tid;
      if (i >= from && i < to) c += rp[a][it] < med ? 1u : (rp[a][it] == med ? 0x10000u : 0u);
    }
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(&s_c[a], c);
  }
  __syncthreads();
  if (tid < arrays) {
    const uint32_t c = s_c[tid];
    uint64_t v = (uint64_t)(c & 0xFFFF) | ((uint64_t)(c >> 16) << 32);
    const bool head = ns == 0 || s_si.s[ns - 1] >= t0;
    const bool cont = ns > 0 && s_si.s[0] < t0;
    v |= ((uint64_t)head << 48) | ((uint64_t)cont << 49);
    tval[(int64_t)tid * tiles + t] = v;
  }
}

// Chains the counts along every subarray: carry[a][t] = counts of tile t's
// first subarray in all earlier tiles (lower in bits 0-31, node in 32-47).
// Tile t contributes (v, h): v = the counts of its last subarray, h = that
// subarray starts inside the tile; the chained value is the segmented
// inclusive scan I_t = h ? v : I_{t-1} + v, and carry[t] = I_{t-1} when the
// tile's first subarray started before it.  One block per moving array:
// every thread scans a run of consecutive tiles, and the runs are joined by
// a segmented scan over the block.
__device__ __forceinline__ void seg_combine(uint64_t& v, int& h, uint64_t v_prev, int h_prev) {
  if (!h) v += v_prev;
  h = h || h_prev;
}

__global__ __launch_bounds__(1024) void k_level_scan(const Forest F, int depth,
                                                    const uint64_t* __restrict__ tval,
                                                    uint64_t* __restrict__ carry,
                                                    int tiles_per_array) {
  constexpr int kThreads = 1024, kWaves = kThreads / kWave;
  __shared__ uint64_t s_v[kWaves];
  __shared__ int s_h[kWaves];
  const int tid = threadIdx.x;
  const int nu = F.uoff[F.B];
  if (depth >= *F.lmax) return;
  const int a = blockIdx.x;
  const int tiles = (int)((nu + kLevelTile - 1) / kLevelTile);
  const int per = (tiles + kThreads - 1) / kThreads;
  const int c0 = min(tiles, tid * per), c1 = min(tiles, c0 + per);
  auto tile_value = [&](int t, uint64_t* v, int* h, bool* cont) {
    const uint64_t x = tval[(int64_t)a * tiles_per_array + t];
    *v = x & ((1ull << 48) - 1);
    *h = (int)((x >> 48) & 1);
    *cont = ((x >> 49) & 1) != 0;
  };
  // aggregate of this thread's run
  uint64_t av = 0;
  int ah = 0;
  for (int t = c0; t < c1; ++t) {
    uint64_t v;
    int h;
    bool cont;
    tile_value(t, &v, &h, &cont);
    seg_combine(v, h, av, ah);
    av = v;
    ah = h;
  }
  // inclusive segmented scan of the run aggregates over the block
  uint64_t iv = av;
  int ih = ah;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint64_t ov = __shfl_up(iv, d, kWave);
    const int oh = __shfl_up(ih, d, kWave);
    if ((int)lane_id() >= d) seg_combine(iv, ih, ov, oh);
  }
  const int w = tid / kWave;
  if (lane_id() == kWave - 1) {
    s_v[w] = iv;
    s_h[w] = ih;
  }
  __syncthreads();
  if (tid == 0) {
    uint64_t rv = 0;
    int rh = 0;
    for (int q = 0; q < kWaves; ++q) {  // exclusive prefix of the wave totals
      const uint64_t qv = s_v[q];
      const int qh = s_h[q];
      s_v[q] = rv;
      s_h[q] = rh;
      uint64_t nv = qv;
      int nh = qh;
      seg_combine(nv, nh, rv, rh);
      rv = nv;
      rh = nh;
    }
  }
  __syncthreads();
  // exclusive value before this thread's run: the wave prefix joined with
  // the lanes below
  uint64_t ev = __shfl_up(iv, 1, kWave);
  int eh = __shfl_up(ih, 1, kWave);
  if (lane_id() == 0) {
    ev = 0;
    eh = 0;
  }
  seg_combine(ev, eh, s_v[w], s_h[w]);
  // walk the run again, writing every tile's carry
  uint64_t run = ev;
  for (int t = c0; t < c1; ++t) {
    uint64_t v;
    int h;
    bool cont;
    tile_value(t, &v, &h, &cont);
    carry[(int64_t)a * tiles_per_array + t] = cont ? run : 0ull;
    run = h ? v : run + v;
  }
}

template <int W>
struct Rec {
  uint32_t v[W];
};

// ---- single-pass level: decoupled look-back --------------------------------------
// The count and chain steps can instead run inside the move launch: tiles are
// taken in launch order from a counter, every tile publishes the counts of its
// last subarray (and whether that subarray starts inside it) as soon as it has
// them, and a tile whose first subarray started earlier sums its
// predecessors' published values backwards until it meets a subarray start or
// a predecessor that already published its inclusive value.  A tile only ever
// waits for tiles that took their numbers before it and publish before they
// wait themselves, so the waits always end.
// Status word of (tile, array): bits 0-31 lower count, 32-47 median count,
// bit 48 head (the last subarray starts inside the tile), bits 56-62 the
// level's epoch (depth + 1), bit 63 inclusive (the value runs from the
// subarray's start).
constexpr uint64_t kStValue = (1ull << 48) - 1;
constexpr int kStHead = 48, kStEpoch = 56, kStIncl = 63;
constexpr int kLookbackSpin = 1 << 24;  // polls before giving up (never reached when consistent)

struct LookBack {
  uint64_t* status;
  int stride;  // moving arrays per tile
  int a, t;
  uint32_t epoch;
};

__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_load(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave 0: publish this tile's value, then (cont) gather the carry of its
// first subarray; returns it in every lane.
__device__ uint64_t level_lookback(const LookBack& lb, uint64_t agg, bool head, bool cont) {
  const int lane = lane_id();
  uint64_t* me = lb.status + (int64_t)lb.t * lb.stride + lb.a;
  const uint64_t tag = ((uint64_t)lb.epoch << kStEpoch) | ((uint64_t)head << kStHead);
  if (lane == 0) status_store(me, tag | agg | (head ? 1ull << kStIncl : 0ull));
  uint64_t carry = 0;
  if (cont) {
    int pos = lb.t - 1;
    for (int spin = 0; spin < kLookbackSpin; ++spin) {
      const int q = pos - lane;  // lane l looks at tile pos - l
      uint64_t sv = 0;
      bool ready = true, stop = true;
      if (q >= 0) {
        sv = status_load(lb.status + (int64_t)q * lb.stride + lb.a);
        ready = (uint32_t)((sv >> kStEpoch) & 0x7F) == lb.epoch;
        stop = ready && (((sv >> kStIncl) & 1) || ((sv >> kStHead) & 1));
      }
      const uint64_t nr = __ballot(!ready), sp = __ballot(stop);
      const int fnr = nr ? __ffsll((unsigned long long)nr) - 1 : kWave;
      const int fsp = sp ? __ffsll((unsigned long long)sp) - 1 : kWave;
      // consume the ready lanes below the first unready one, up to the first stop
      const int take = fsp < fnr ? fsp + 1 : fnr;
      carry += wave_sum(lane < take ? (sv & kStValue) : 0ull);
      if (fsp < fnr) break;
      pos -= take;
    }
    if (!head && lane == 0) status_store(me, tag | ((carry + agg) & kStValue) | (1ull << kStIncl));
  }
  return carry;
}

// Move one tile of one array: its W = k-1 rank planes.
// kFused: the carry comes from the look-back instead of `carry`.
// The tile's subarrays (gsi, global) are copied to si (LDS) while the planes
// are in flight.
// wmask: the planes to write (bit c: plane c); the others are not read again.
template <int W, bool kFused>
__device__ __forceinline__ void level_move_tile(const uint32_t* __restrict__ src,
                                               uint32_t* __restrict__ dst, int64_t n, int cp,
                                               int t0, int t1, const SegInfo* __restrict__ gsi,
                                               SegInfo& si, uint64_t carry, uint32_t* s_chunk,
                                               uint32_t* s_pre, const LookBack& lb,
                                               uint64_t* s_carry, uint32_t wmask,
                                               uint32_t* status) {
  const int tid = threadIdx.x;
  const int w = tid / kWave;
  const int lane = tid % kWave;

  uint32_t v[W][kLvItems];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const uint32_t* sp = src + (int64_t)c * n;
    const bool need = ((wmask >> c) & 1u) || c == cp;  // written, or decides the side
#pragma unroll
    for (int it = 0; it < kLvItems; ++it) {
      const int i = t0 + it * kLvThreads + tid;
      v[c][it] = need && i < t1 ? sp[i] : 0u;
    }
  }
  if (tid < kMaxSeg) {
    si.s[tid] = gsi->s[tid];
    si.e[tid] = gsi->e[tid];
    si.med[tid] = gsi->med[tid];
    if (tid == 0) si.nseg = gsi->nseg;
  }
  __syncthreads();
  const int nseg = si.nseg;
  uint32_t flag[kLvItems];
  int8_t sg[kLvItems];
  uint32_t within[kLvItems];
#pragma unroll
  for (int it = 0; it < kLvItems; ++it) {
    const int i = t0 + it * kLvThreads + tid;
    sg[it] = -1;
    if (i < t1) {
      for (int q = 0; q < nseg; ++q) {
        if (i >= si.s[q] && i <= si.e[q]) {
          sg[it] = (int8_t)q;
          break;
        }
      }
    }
    uint32_t f = 0;
    if (sg[it] >= 0) {
      uint32_t rp = 0;
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (c == cp) rp = v[c][it];
      const uint32_t med = si.med[sg[it]];
      f = rp < med ? 1u : (rp == med ? 0x10000u : 0u);
    }
    flag[it] = f;
    const uint32_t inc = wave_inclusive_sum(f);
    within[it] = inc - f;
    if (lane == kWave - 1) s_chunk[it * kLvWaves + w] = inc;
  }
  __syncthreads();
  uint32_t tile_total = 0;  // wave 0: the tile's packed total
  if (w == 0) {
    const uint32_t c = s_chunk[tid];
    const uint32_t inc = wave_inclusive_sum(c);
    s_chunk[tid] = inc - c;
    tile_total = __shfl(inc, kWave - 1, kWave);
  }
  __syncthreads();
  // exclusive in-tile prefix of every position, packed as lower | node << 16
#pragma unroll
  for (int it = 0; it < kLvItems; ++it) {
    const int i = t0 + it * kLvThreads + tid;
    if (i < t1) s_pre[i - t0] = s_chunk[it * kLvWaves + w] + within[it];
  }
  __syncthreads();
  if constexpr (kFused) {
    if (w == 0) {
      // value for the next tiles: the counts of the last subarray in this tile
      uint64_t agg = 0;
      bool head = true, cont = false;
      if (nseg > 0) {
        const int sl = si.s[nseg - 1];
        head = sl >= t0;
        cont = si.s[0] < t0;
        const uint32_t part = tile_total - (head ? s_pre[sl - t0] : 0u);
        agg = (uint64_t)(part & 0xFFFF) | ((uint64_t)(part >> 16) << 32);
      }
      const uint64_t c = level_lookback(lb, agg, head, cont);
      if (tid == 0) *s_carry = c;
    }
    __syncthreads();
    carry = *s_carry;
  }
  const int carry_lower = (int)(carry & 0xFFFFFFFFull);
  const int carry_node = (int)((carry >> 32) & 0xFFFF);
  int dest[kLvItems];
#pragma unroll
  for (int it = 0; it < kLvItems; ++it) {
    dest[it] = -1;
    if (sg[it] < 0 || flag[it] == 0x10000u) continue;
    const int q = sg[it];
    const int i = t0 + it * kLvThreads + tid;
    const uint32_t pre = s_pre[i - t0];
    const int s = si.s[q], e = si.e[q];
    const uint32_t base = s >= t0 ? s_pre[s - t0] : 0u;
    int low = (int)(pre & 0xFFFF) - (int)(base & 0xFFFF);
    int nd = (int)(pre >> 16) - (int)(base >> 16);
    if (s < t0) {  // only the first subarray can start before the tile
      low += carry_lower;
      nd += carry_node;
    }
    const int m = s + ((e - s) >> 1);
    const int d = (flag[it] == 1u) ? s + low : m + 1 + (i - s - low - nd);
    if (d >= s && d <= e && d != m)
      dest[it] = d;
    else  // only if the counts were inconsistent
      atomicOr(status, kStatusLevelMove);
  }
#pragma unroll
  for (int c = 0; c < W; ++c) {
    if (!((wmask >> c) & 1u)) continue;
    uint32_t* dp = dst + (int64_t)c * n;
#pragma unroll
    for (int it = 0; it < kLvItems; ++it)
      if (dest[it] >= 0) dp[dest[it]] = v[c][it];
  }
}

template <int R, bool kDefer>
__global__ __launch_bounds__(kLvThreads) void k_level_move(const RecBufs B, const Forest F,
                                                          int64_t n, int k, int depth,
                                                          const SegInfo* __restrict__ seginfo,
                                                          const uint64_t* __restrict__ carry,
                                                          int tiles_per_array, uint32_t arows,
                                                          uint64_t wmasks) {
  __shared__ uint32_t s_chunk[kLvChunks];
  __shared__ uint32_t s_pre[kLevelTile];
  __shared__ SegInfo s_si;
  const int nu = F.uoff[F.B];
  const int lmax = *F.lmax;
  if (depth >= lmax) return;
  const int p = depth % k;
  // XCD-aware: each XCD takes a contiguous range of (array, tile) numbers.
  // The grid covers only the moving arrays that write anything (the others
  // stay put), so no XCD is handed only idle tiles: grid row r moves array
  // (p + 1 + a) mod k with a = bits 4r .. 4r+3 of `arows` (15: no array).
  const int bt = xcd_tile(blockIdx.x, gridDim.x);
  const int r = bt / tiles_per_array;
  const int t = bt % tiles_per_array;
  if (r >= 8) return;
  const int a = (int)((arows >> (4 * r)) & 0xFu);
  if (a >= k - 1) return;
  const int j = (p + 1 + a) % k;
  // The deepest global level (the last one for every tree still at global
  // levels) is followed by the on-chip finish, which reads only the order-0
  // plane of arrays 1 .. k-1 and nothing of array 0: array 0 stays put and
  // the others write that one plane.
  // wmasks (8 bits per array: the planes later levels and the finish read),
  // or all ones when the caller does not know the levels ahead (a batch):
  // then only the deepest level is trimmed, to what the finish reads
  uint32_t wmask = (uint32_t)(wmasks >> (8 * j)) & 0xFFu;
  if (wmasks == ~0ull) wmask = depth == lmax - 1 ? (j == 0 ? 0u : 1u << (k - 1 - j)) : ~0u;
  if (wmask == 0) return;
  const int t0 = t * kLevelTile;
  if (t0 >= nu) return;
  const int t1 = min(t0 + kLevelTile, nu);
  const uint64_t cy = carry[(int64_t)a * tiles_per_array + t];
  const int mj = array_moves(kDefer ? 1 : 0, depth, j, k);
  const uint32_t* src = buf_after(B, mj) + record_offset(j, k, n);
  uint32_t* dst = const_cast<uint32_t*>(buf_after(B, mj + 1)) + record_offset(j, k, n);
  const int cp = (p - j - 1 + 2 * k) % k;
  const LookBack lb{};
  level_move_tile<R, false>(src, dst, n, cp, t0, t1, seginfo + t, s_si, cy, s_chunk, s_pre, lb,
                            nullptr, wmask, F.status);
}

// Count, chain and move in one launch (look-back).  Tile numbers come from
// tickets[depth], cleared before the first level; tile t of array a is
// ticket t * (k - 1) + a, so the arrays advance together.
template <int R>
__global__ __launch_bounds__(kLvThreads) void k_level_fused(const RecBufs B, const Forest F,
                                                           int64_t n, int k, int depth,
                                                           const SegInfo* __restrict__ seginfo,
                                                           uint64_t* __restrict__ status,
                                                           int32_t* __restrict__ tickets) {
  __shared__ uint32_t s_chunk[kLvChunks];
  __shared__ uint32_t s_pre[kLevelTile];
  __shared__ SegInfo s_si;
  __shared__ int s_ticket;
  __shared__ uint64_t s_carry;
  const int tid = threadIdx.x;
  const int nu = F.uoff[F.B];
  if (depth >= *F.lmax) return;  // the same for every workgroup of the launch
  if (tid == 0) s_ticket = atomicAdd(tickets + depth, 1);
  __syncthreads();
  const int a = s_ticket % (k - 1);
  const int t = s_ticket / (k - 1);
  const int p = depth % k;
  const int j = (p + 1 + a) % k;
  const int t0 = t * kLevelTile;
  if (t0 >= nu) return;
  const int t1 = min(t0 + kLevelTile, nu);
  const int mj = moves_before(depth, j, k);
  const uint32_t* src = buf_after(B, mj) + record_offset(j, k, n);
  uint32_t* dst = const_cast<uint32_t*>(buf_after(B, mj + 1)) + record_offset(j, k, n);
  const int cp = (p - j - 1 + 2 * k) % k;
  const LookBack lb{status, k - 1, a, t, (uint32_t)depth + 1};
  level_move_tile<R, true>(src, dst, n, cp, t0, t1, seginfo + t, s_si, 0, s_chunk, s_pre, lb,
                           &s_carry, ~0u, F.status);
}

hipError_t launch_level(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1, uint32_t* b2,
                        int64_t n, int k,
                        int depth, int64_t cutover, const ForestArgs& fa, int32_t* perm,
                        void* seginfo, uint32_t* cnt, uint64_t* carry, uint64_t* status,
                        int32_t* tickets, uint64_t wmasks, int defer, hipStream_t st) {
  if (n <= 0 || k < 2) return hipSuccess;
  const int tiles = (int)((n + kLevelTile - 1) / kLevelTile);
  const unsigned grid = (unsigned)(tiles * (k - 1));
  RecBufs B{rec0, rows, b1, b2};
  Forest F{fa.B, fa.off, fa.uoff, fa.lmax, fa.wgbase, fa.queue, fa.status};
  SegInfo* si = static_cast<SegInfo*>(seginfo);
  if (defer && status) return hipErrorInvalidValue;  // deferred: three-launch levels only
  uint64_t* tval = status ? nullptr : reinterpret_cast<uint64_t*>(cnt);
  const uint64_t seg_masks = status == nullptr ? wmasks : ~0ull;
#define KD_SEG(RR)                                                                                \
  do {                                                                                            \
    if (defer)                                                                                    \
      hipLaunchKernelGGL((k_level_seg<RR, true>), dim3(tiles), dim3(kSegThreads), 0, st, B, F, n, k, \
                         depth, cutover, perm, si, tval, tiles, seg_masks);                       \
    else                                                                                          \
      hipLaunchKernelGGL((k_level_seg<RR, false>), dim3(tiles), dim3(kSegThreads), 0, st, B, F, n, \
                         k, depth, cutover, perm, si, tval, tiles, seg_masks);                    \
  } while (0)
  switch (status ? 0 : k - 1) {
    case 0: KD_SEG(0); break;
    case 1: KD_SEG(1); break;
    case 2: KD_SEG(2); break;
    case 3: KD_SEG(3); break;
    case 4: KD_SEG(4); break;
    case 5: KD_SEG(5); break;
    case 6: KD_SEG(6); break;
    case 7: KD_SEG(7); break;
    default: return hipErrorInvalidValue;
  }
#undef KD_SEG
  if (status) {
    if (depth >= kMaxLevels) return hipErrorInvalidValue;
#define KD_LF(RR)                                                                                \
  hipLaunchKernelGGL(k_level_fused<RR>, dim3(grid), dim3(kLvThreads), 0, st, B, F, n, k, depth, si, \
                     status, tickets)
    switch (k - 1) {
      case 1: KD_LF(1); break;
      case 2: KD_LF(2); break;
      case 3: KD_LF(3); break;
      case 4: KD_LF(4); break;
      case 5: KD_LF(5); break;
      case 6: KD_LF(6); break;
      case 7: KD_LF(7); break;
      default: return hipErrorInvalidValue;
    }
#undef KD_LF
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_level_scan, dim3(k - 1), dim3(1024), 0, st, F, depth, tval, carry, tiles);
  // arrays staying put at this level (they write no plane) are left out of
  // the grid
  const int p = depth % k;
  uint32_t arows = ~0u;
  int nact = 0;
  for (int a = 0; a < k - 1; ++a)
    if (wmasks == ~0ull || ((wmasks >> (8 * ((p + 1 + a) % k))) & 0xFFu) != 0) {
      arows = (arows & ~(0xFu << (4 * nact))) | ((uint32_t)a << (4 * nact));
      ++nact;
    }
  const unsigned mgrid = (unsigned)(tiles * nact);
  if (mgrid == 0) return hipGetLastError();
#define KD_LV(RR)                                                                               \
  do {                                                                                          \
    if (defer)                                                                                  \
      hipLaunchKernelGGL((k_level_move<RR, true>), dim3(xcd_grid(mgrid)), dim3(kLvThreads), 0, st, \
                         B, F, n, k, depth, si, carry, tiles, arows, wmasks);                   \
    else                                                                                        \
      hipLaunchKernelGGL((k_level_move<RR, false>), dim3(xcd_grid(mgrid)), dim3(kLvThreads), 0, \
                         st, B, F, n, k, depth, si, carry, tiles, arows, wmasks);               \
  } while (0)
  switch (k - 1) {
    case 1: KD_LV(1); break;
    case 2: KD_LV(2); break;
    case 3: KD_LV(3); break;
    case 4: KD_LV(4); break;
    case 5: KD_LV(5); break;
    case 6: KD_LV(6); break;
    case 7: KD_LV(7); break;
    default: return hipErrorInvalidValue;
  }
#undef KD_LV
  return hipGetLastError();
}

size_t level_seginfo_bytes() { return sizeof(SegInfo); }

// Walking back from the on-chip finish (which reads the order-0 plane of
// arrays 1 .. k-1 and nothing of array 0): a level's move writes exactly the
// planes that later levels or the finish read.  A level reads, of its split
// array p, plane 0 (the median's rank in order p+1) and, when p != 0, the
// order-0 plane (the median's row id); of every array it moves, the plane
// deciding the side and every plane it writes.  An array with nothing to
// write stays put and is not read.  Deferred, arrays j >= 2 write nothing
// above depth j (their split writes every plane).
int level_array_moves(int defer, int depth, int j, int k) { return array_moves(defer, depth, j, k); }

void level_write_masks(int k, int levels, uint64_t* masks, int defer) {
  uint32_t need[kMaxK] = {};
  for (int j = 1; j < k; ++j) need[j] = 1u << (k - 1 - j);
  for (int d = levels - 1; d >= 0; --d) {
    const int p = d % k;
    uint64_t m = 0;
    for (int j = 0; j < k; ++j)
      if (j != p && !(defer && j >= 2 && d < j)) m |= (uint64_t)need[j] << (8 * j);
    masks[d] = m;
    for (int j = 0; j < k; ++j) {
      if (j == p) {
        need[j] |= 1u;
        if (p != 0) need[j] |= 1u << ((k - p - 1) % k);
      } else if (need[j] != 0) {
        need[j] |= 1u << ((p - j - 1 + 2 * k) % k);
      }
    }
  }
}

// ---- deferred partitioning: the split of array j ----------------------------------
// One tree only.  node_rank[(1 << d) - 1 + q] is the rank in order d of the
// node of subarray q at depth d (subarrays numbered left to right), taken
// once array d has its depth-d layout: the median sits at the middle of the
// subarray in array d, and the level-0 records of array d+1 translate its
// rank in order d+1 (plane 0) to order d, as at a global level.
__global__ __launch_bounds__(64) void k_node_ranks(const RecBufs B, const Forest F, int64_t n,
                                                   int k, int depth,
                                                   uint32_t* __restrict__ node_rank) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (1 << depth) || depth >= *F.lmax) return;
  const int base = F.uoff[0];
  int s = 0, e = F.uoff[1] - base - 1;
  for (int l = 0; l < depth; ++l) {
    const int m = s + ((e - s) >> 1);
    if ((q >> (depth - 1 - l)) & 1)
      s = m + 1;
    else
      e = m - 1;
  }
  if (e < s) {  // not reached: global-level subarrays hold at least C rows
    atomicOr(F.status, kStatusNode);
    return;
  }
  const int p = depth % k;
  const int m = base + s + ((e - s) >> 1);
  const uint32_t r1 = rec_array<true>(B, depth, p, k, n)[m];
  if (r1 >= (uint32_t)n) {  // not reached: a rank
    atomicOr(F.status, kStatusNode);
    return;
  }
  node_rank[(1 << depth) - 1 + q] = B.rec0[record_offset((p + 1) % k, k, n) + (int64_t)(k - 2) * n + r1];
}

// Bucket of every element of array j (level-0 records, presorted order j)
// among the subarrays and nodes of depth D = min(j, deepest global level),
// numbered in order (subarray q is 2q; the node of subarray q at depth d < D
// sits between the halves below it, at q * 2^(D-d+1) + 2^(D-d) - 1).  The
// element walks down from the root comparing its rank in order d with the
// node's.  A stable sort by bucket then gives array j's layout at depth D.
__global__ __launch_bounds__(256) void k_defer_bucket(const RecBufs B, const Forest F, int64_t n,
                                                      int k, int j,
                                                      const uint32_t* __restrict__ node_rank,
                                                      uint32_t* __restrict__ key) {
  __shared__ uint32_t s_nr[1 << (kMaxK - 1)];
  const int lmax = *F.lmax;
  const int D = j < lmax ? j : lmax;
  for (int i = threadIdx.x; i < (1 << D) - 1; i += blockDim.x) s_nr[i] = node_rank[i];
  __syncthreads();
  const int base = F.uoff[0];
  const int nu = F.uoff[1] - base;
  const uint32_t* rec = B.rec0 + record_offset(j, k, n);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nu; i += gridDim.x * blockDim.x) {
    uint32_t q = 0, b = 0xFFFFFFFFu;
    for (int d = 0; d < D; ++d) {
      const int c = (d - j - 1 + 2 * k) % k;  // the plane holding the rank in order d
      const uint32_t r = rec[(int64_t)c * n + base + i];
      const uint32_t nr = s_nr[(1 << d) - 1 + q];
      if (r == nr) {
        b = q * (2u << (D - d)) + (1u << (D - d)) - 1u;
        break;
      }
      q = 2 * q + (r > nr ? 1u : 0u);
    }
    key[base + i] = b != 0xFFFFFFFFu ? b : 2 * q;
  }
}

hipError_t launch_node_ranks(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1,
                             uint32_t* b2, int64_t n, int k, int depth, const ForestArgs& fa,
                             uint32_t* node_rank, hipStream_t st) {
  if (n <= 0 || k < 2 || fa.B != 1 || depth < 0 || depth > kMaxK - 2) return hipErrorInvalidValue;
  RecBufs B{rec0, rows, b1, b2};
  Forest F{fa.B, fa.off, fa.uoff, fa.lmax, fa.wgbase, fa.queue, fa.status};
  const int nodes = 1 << depth;
  hipLaunchKernelGGL(k_node_ranks, dim3((nodes + 63) / 64), dim3(64), 0, st, B, F, n, k, depth,
                     node_rank);
  return hipGetLastError();
}

hipError_t launch_defer_bucket(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1,
                               uint32_t* b2, int64_t n, int k, int j, const ForestArgs& fa,
                               const uint32_t* node_rank, uint32_t* key, hipStream_t st) {
  if (n <= 0 || k < 3 || fa.B != 1 || j < 2 || j >= k) return hipErrorInvalidValue;
  RecBufs B{rec0, rows, b1, b2};
  Forest F{fa.B, fa.off, fa.uoff, fa.lmax, fa.wgbase, fa.queue, fa.status};
  const int64_t want = (n + 255) / 256;
  const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(k_defer_bucket, dim3(grid), dim3(256), 0, st, B, F, n, k, j, node_rank, key);
  return hipGetLastError();
}

// ---- on-chip finish (leaf phase) -----------------------------------------------------
// One workgroup takes one subarray of at most C elements at the cutover depth
// and runs all remaining levels in LDS.  Elements get local ids -- their
// position in the array sorted by order 0 -- and each array becomes a list of
// 16-bit local ids.  A level then needs only "where does this id sit in the
// split array": the element goes to the lower half iff that position is below
// the median.  The k-1 arrays that move are partitioned together with
// segmented scans (4 barriers per level).

constexpr int kLfThreads = 256;
constexpr int kLfWaves = kLfThreads / kWave;
constexpr uint32_t kHole = 0xFFFFFFFFu;
constexpr uint32_t kHeadBit = 0x80000000u;

// Inclusive segmented sum across a wave (all lanes active): a lane with
// `head` starts a new run.  On return v is the sum from the latest head at or
// before the lane (from lane 0 when there is none) and h tells whether there
// is such a head.  An unsegmented DPP sum S and a DPP max-scan of the head
// lanes give it: v = S[lane] - S[latest head - 1].
__device__ __forceinline__ void wave_seg_scan(uint32_t& v, bool& h) {
  const uint32_t sum = wave_scan_dpp(v);
  const uint32_t hl = wave_max_dpp(h ? lane_id() + 1u : 0u);  // latest head lane + 1, 0 if none
  const uint32_t before = __shfl(sum, hl > 1u ? (int)hl - 2 : 0, kWave);
  v = sum - (hl > 1u ? before : 0u);
  h = hl != 0u;
}

// Stable LSD radix sort of up to C keys in LDS (8-bit digits): keys and 16-bit
// values move between (ka, va) and (kb, vb); returns true when the result ended
// in (kb, vb).  Element e is owned by wave e / (64 * kItems).
template <int kItems>
__device__ bool lds_radix_sort(uint32_t* ka, uint16_t* va, uint32_t* kb, uint16_t* vb, int N,
                               int passes, uint32_t (*s_cnt)[kRadix], uint32_t* s_dbase,
                               uint32_t* s_tmp) {
  const int tid = threadIdx.x;
  const int w = tid / kWave;
  const int lane = tid % kWave;
  bool flipped = false;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = ps * kRadixBits;
#pragma unroll
    for (int q = 0; q < kLfWaves; ++q) s_cnt[q][tid] = 0;
    __syncthreads();
    uint32_t key[kItems], rank[kItems];
    uint16_t val[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int e = w * (kWave * kItems) + j * kWave + lane;
      const bool valid = e < N;
      key[j] = valid ? ka[e] : 0u;
      val[j] = valid ? va[e] : (uint16_t)0;
      const uint32_t d = (key[j] >> shift) & 0xFF;
      const uint64_t m = same_digit_lanes<kRadixBits>(d, kRadixBits, __ballot(valid));
      uint32_t pre = 0;
      if (valid) pre = s_cnt[w][d];
      __builtin_amdgcn_wave_barrier();
      const uint32_t before = lanes_below(m);
      if (valid && before == 0) s_cnt[w][d] = pre + popc64(m);
      __builtin_amdgcn_wave_barrier();
      rank[j] = pre + before;
    }
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int q = 0; q < kLfWaves; ++q) {
      const uint32_t c = s_cnt[q][tid];
      s_cnt[q][tid] = tot;
      tot += c;
    }
    uint32_t all;
    s_dbase[tid] = block_exclusive_sum<kLfThreads>(tot, s_tmp, &all);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int e = w * (kWave * kItems) + j * kWave + lane;
      if (e < N) {
        const uint32_t d = (key[j] >> shift) & 0xFF;
        const uint32_t dest = s_dbase[d] + s_cnt[w][d] + rank[j];
        kb[dest] = key[j];
        vb[dest] = val[j];
      }
    }
    __syncthreads();
    uint32_t* tk = ka; ka = kb; kb = tk;
    uint16_t* tv = va; va = vb; vb = tv;
    flipped = !flipped;
  }
  return flipped;
}

// Local ids of the subarray of N elements at s0 (cutover depth lc): an
// element's local id is its position in array 0 (sorted by order 0).
// Array 1 stores the order-0 rank of each of its elements (plane k-2);
// sorting those ranks gives array 0's order, hence every array-1 element's
// local id, and the sorted list lets the other arrays find theirs by binary
// search.  On return s_r0[id] is the order-0 rank of id and s_lid[j * C + i]
// the id at position i of array j (the row ids are read at the end at the
// order-0 ranks).  No barrier after the last writes.
template <int kItems, int R, int kForm>
__device__ void leaf_local_ids(const RecBufs& B, const Forest& F, int64_t n, int lc, int N, int s0,
                               uint32_t* s_r0, uint16_t* s_lid, uint32_t (*s_cnt)[kRadix],
                               uint32_t* s_dbase, uint32_t* s_tmp) {
  constexpr int k = R + 1;
  constexpr int C = kItems * kLfThreads;
  const int tid = threadIdx.x;
  const uint32_t* a1 = leaf_array<kForm>(B, lc, 1, k, n);
  uint32_t* sk = reinterpret_cast<uint32_t*>(s_lid);        // sort scratch (aliases s_lid)
  uint16_t* sv = reinterpret_cast<uint16_t*>(sk + C);
  uint16_t* sv2 = sv + C;
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int i = it * kLfThreads + tid;
    if (i < N) {
      s_r0[i] = a1[(int64_t)(k - 2) * n + s0 + i];
      sv2[i] = (uint16_t)i;
    }
  }
  __syncthreads();
  int passes = 1;
  const uint32_t total = (uint32_t)F.uoff[F.B];
  while (passes < 4 && ((uint64_t)(total - 1) >> (8 * passes)) != 0) ++passes;
  const bool in_b = lds_radix_sort<kItems>(s_r0, sv2, sk, sv, N, passes, s_cnt, s_dbase, s_tmp);
  // sorted ranks must end in s_r0; the array-1 positions they came from in regs
  uint16_t from[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int i = it * kLfThreads + tid;
    if (i < N) {
      from[it] = in_b ? sv[i] : sv2[i];
      if (in_b) s_r0[i] = sk[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int i = it * kLfThreads + tid;
    if (i < N) {
      s_lid[i] = (uint16_t)i;                 // array 0
      s_lid[1 * C + from[it]] = (uint16_t)i;  // array 1
    }
  }
  // the other arrays: lower bound of each order-0 rank among the sorted ones,
  // by halving steps taken for all of a thread's items at once
  int top = 1;
  while (2 * top <= N) top *= 2;
  for (int j = 2; j < k; ++j) {
    const uint32_t* aj = leaf_array<kForm>(B, lc, j, k, n);
    const int c0 = k - 1 - j;  // plane of order 0 in array j
    uint32_t x[kItems];
    int pos[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const int i = it * kLfThreads + tid;
      x[it] = i < N ? aj[(int64_t)c0 * n + s0 + i] : 0u;
      pos[it] = 0;
    }
    for (int step = top; step > 0; step >>= 1) {
#pragma unroll
      for (int it = 0; it < kItems; ++it) {
        const int cand = pos[it] + step;  // ranks at 0 .. cand-1 all below x?
        if (cand <= N && s_r0[cand - 1] < x[it]) pos[it] = cand;
      }
    }
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const int i = it * kLfThreads + tid;
      if (i < N) s_lid[j * C + i] = (uint16_t)(pos[it] < N ? pos[it] : N - 1);
    }
  }
}

template <int kItems, int R, int kForm>
__global__ __launch_bounds__(kLfThreads) void k_leaf(const RecBufs B, const Forest F, int64_t n,
                                                    int /* k: R + 1 */, int32_t* __restrict__ perm) {
  constexpr int k = R + 1;  // known at compile time: index arithmetic mod k folds
  constexpr int C = kItems * kLfThreads;
  constexpr int kChunks = kItems * kLfWaves;
  static_assert(kChunks <= kWave, "one wave scans the chunk totals of an array");
  extern __shared__ __align__(16) unsigned char s_raw[];
  uint32_t* s_r0 = reinterpret_cast<uint32_t*>(s_raw);       // [C] sorted order-0 ranks
  uint8_t* s_side = reinterpret_cast<uint8_t*>(s_r0 + C);    // [C] side of each local id this level
  uint16_t* s_out = reinterpret_cast<uint16_t*>(s_side + 2 * C);  // [C] node id of each position
  uint16_t* s_lid = s_out + C;                               // [2][k][C] local-id arrays
  __shared__ uint32_t s_chunk[R][kWave];
  __shared__ uint32_t s_cnt[kLfWaves][kRadix];
  __shared__ uint32_t s_dbase[kRadix];
  __shared__ uint32_t s_tmp[kLfWaves + 1];
  __shared__ int s_item;

  const int tid = threadIdx.x;
  const int w = tid / kWave;
  const int lane = tid % kWave;
  const int items_total = F.wgbase[F.B];
  // Persistent: every workgroup takes (tree, subarray) items from a counter
  // until none are left; items never wait on each other.
  for (;;) {
  if (tid == 0) s_item = atomicAdd(F.queue, 1);
  __syncthreads();
  const int item = s_item;
  __syncthreads();
  if (item >= items_total) break;
  const int tree = F.B == 1 ? 0 : upper_index(F.wgbase, F.B, item);
  const int g = item - F.wgbase[tree];
  const int tbase = F.uoff[tree];
  const int nb = F.uoff[tree + 1] - tbase;
  const int lc = cutover_depth(nb, C);
  int s0 = 0, e0 = nb - 1;
  for (int l = 0; l < lc; ++l) {
    const int m = s0 + ((e0 - s0) >> 1);
    if ((g >> (lc - 1 - l)) & 1)
      s0 = m + 1;
    else
      e0 = m - 1;
  }
  const int N = e0 - s0 + 1;
  if (N <= 0) continue;
  s0 += tbase;

  leaf_local_ids<kItems, R, kForm>(B, F, n, lc, N, s0, s_r0, s_lid, s_cnt, s_dbase, s_tmp);

  // Position i = it * kLfThreads + tid is owned by one thread for the whole
  // phase, so its subarray (s | e << 16, or a hole) lives in registers.
  uint32_t seg[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it)
    seg[it] = (it * kLfThreads + tid) < N ? ((uint32_t)(N - 1) << 16) : kHole;
  uint32_t curmask = 0;  // bit j: which of the two buffers holds array j
  __syncthreads();

  for (int depth = lc, rel = 0; (N >> rel) > 0; ++depth, ++rel) {
    const int p = depth % k;
    const uint16_t* ap = s_lid + ((((curmask >> p) & 1) * k) + p) * C;
    // The largest subarray at this level holds N >> rel elements.  Once that
    // is at most 3, every child holds at most one element, and the split
    // array, which this level does not move, already has each child's
    // element in the child's position: every remaining node is the split
    // array's element in place.
    const bool last = (N >> rel) <= 3;
    // phase 1: step down one level (the parent's node becomes a hole), then
    // record the side of each id (from its place in the split array) and
    // each subarray's node
    // (every LDS read of a phase is issued before its first write: the reads
    // then overlap instead of each waiting behind the writes before it)
    uint16_t idv[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) idv[it] = ap[it * kLfThreads + tid];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const int i = it * kLfThreads + tid;
      const bool was = seg[it] != kHole;
      int ss = (int)(seg[it] & 0xFFFF), ee = (int)(seg[it] >> 16);
      bool live = was;
      if (rel > 0) {
        const int pm = ss + ((ee - ss) >> 1);
        live = was && i != pm;
        ee = i < pm ? pm - 1 : ee;
        ss = i > pm ? pm + 1 : ss;
      }
      seg[it] = live ? ((uint32_t)ss | ((uint32_t)ee << 16)) : kHole;
      const uint16_t id = idv[it];
      const int m = ss + ((ee - ss) >> 1);
      if (live && (last || i == m)) s_out[i] = id;
      if (live && !last) s_side[id] = i < m ? 1 : (i > m ? 2 : 0);  // lower, upper, node
    }
    __syncthreads();
    if (last) break;
    // phase 2: side of every element of the k-1 moving arrays, counted as
    // lower (bits 0-15) | upper << 16 by a plain scan over each wave chunk;
    // an element whose subarray starts in the same chunk takes its count
    // relative to that start right away, the others add the chunk's carry in
    // phase 4.  Each chunk's last subarray piece goes to s_chunk (with
    // kHeadBit when the piece starts inside the chunk).
    // per element and array: count of the same side before it (bits 0-28),
    // side << 29 (1 lower, 2 upper, 0 node), head in this chunk << 31
    uint32_t pref[R][kItems];
    uint32_t sdv[R][kItems];
    {
      uint16_t idr[R][kItems];
#pragma unroll
      for (int it = 0; it < kItems; ++it)
#pragma unroll
        for (int a2 = 0; a2 < R; ++a2) {
          const int j = (p + 1 + a2) % k;
          idr[a2][it] = s_lid[((((curmask >> j) & 1) * k) + j) * C + it * kLfThreads + tid];
        }
#pragma unroll
      for (int it = 0; it < kItems; ++it)
#pragma unroll
        for (int a2 = 0; a2 < R; ++a2) sdv[a2][it] = s_side[idr[a2][it] & (C - 1)];
    }
    // the scans of all items and arrays together, so that their lane moves
    // interleave
    uint32_t incv[R][kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it)
#pragma unroll
      for (int a2 = 0; a2 < R; ++a2) {
        if (seg[it] == kHole) sdv[a2][it] = 0u;
        const uint32_t side = sdv[a2][it];
        incv[a2][it] = wave_scan_dpp((side & 1u) | ((side & 2u) << 15));
      }
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const bool live = seg[it] != kHole;
      const int ss = (int)(seg[it] & 0xFFFF);
      const int cbase = it * kLfThreads + w * kWave;
      const bool hin = live && ss >= cbase;
      const int hlane = hin ? ss - cbase : 0;
#pragma unroll
      for (int a2 = 0; a2 < R; ++a2) {
        const uint32_t side = sdv[a2][it];
        const uint32_t f = (side & 1u) | ((side & 2u) << 15);
        const uint32_t inc = incv[a2][it];
        const uint32_t exc = inc - f;
        const uint32_t hexc = __shfl(exc, hlane, kWave);
        pref[a2][it] = (hin ? exc - hexc : exc) | (side << 29) | (hin ? 1u << 31 : 0u);
        if (lane == kWave - 1)
          s_chunk[a2][it * kLfWaves + w] = !live ? kHeadBit : (hin ? (inc - hexc) | kHeadBit : inc);
      }
    }
    __syncthreads();
    // phase 3: segmented exclusive scan over each array's chunk pieces
    for (int a2 = w; a2 < R; a2 += kLfWaves) {
      const uint32_t c = lane < kChunks ? s_chunk[a2][lane] : kHeadBit;
      uint32_t v = c & ~kHeadBit;
      bool h = (c & kHeadBit) != 0;
      wave_seg_scan(v, h);
      const uint32_t prev = __shfl_up(v, 1, kWave);
      if (lane < kChunks) s_chunk[a2][lane] = lane == 0 ? 0u : prev;
    }
    __syncthreads();
    // phase 4: move every element of the k-1 arrays to its new position
    uint16_t vv[R][kItems];
    uint32_t cyv[R][kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it)
#pragma unroll
      for (int a2 = 0; a2 < R; ++a2) {
        const int j = (p + 1 + a2) % k;
        vv[a2][it] = s_lid[(((curmask >> j) & 1) * k + j) * C + it * kLfThreads + tid];
        cyv[a2][it] = s_chunk[a2][it * kLfWaves + w];
      }
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const int ss = (int)(seg[it] & 0xFFFF), ee = (int)(seg[it] >> 16);
      const int m = ss + ((ee - ss) >> 1);
#pragma unroll
      for (int a2 = 0; a2 < R; ++a2) {
        const uint32_t x = pref[a2][it];
        const uint32_t side = (x >> 29) & 3u;  // 0: a hole, or the node (not copied)
        const int j = (p + 1 + a2) % k;
        const uint32_t pre = (x & 0x1FFFFFFFu) + ((x >> 31) ? 0u : cyv[a2][it]);
        const int dest = side == 1u ? ss + (int)(pre & 0xFFFF) : m + 1 + (int)(pre >> 16);
        const int cb = (curmask >> j) & 1;
        const uint16_t v = vv[a2][it];
        if (side != 0u) {
          if (dest >= ss && dest <= ee)
            s_lid[((cb ^ 1) * k + j) * C + dest] = v;
          else  // only if the counts were inconsistent
            atomicOr(F.status, kStatusLeaf);
        }
      }
    }
    curmask ^= ((1u << k) - 1) & ~(1u << p);  // every array but the split one moved
    __syncthreads();
  }
  {
    const int64_t ob = F.off[tree];
    int32_t* out = perm + ob + (s0 - tbase);
    const uint32_t* rows = B.rows;
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const int i = it * kLfThreads + tid;
      if (i < N) {
        const int id = s_out[i];
        // the row id of order-0 rank r is rows[r]
        if (id < N) out[i] = (int32_t)((int64_t)rows[s_r0[id]] - ob);
      }
    }
  }
  __syncthreads();  // LDS is reused by the next item
  }
}

hipError_t launch_leaf(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1, uint32_t* b2,
                       int64_t n, int k,
                       int64_t cutover, const ForestArgs& fa, int32_t* perm, int64_t items_bound,
                       int blocks, int form, hipStream_t st) {
  if (n <= 0 || k < 2) return hipSuccess;
  if (form < 0 || form > 2) return hipErrorInvalidValue;
  const size_t lds = leaf_lds_bytes(cutover, k);
  RecBufs B{rec0, rows, b1, b2};
  Forest F{fa.B, fa.off, fa.uoff, fa.lmax, fa.wgbase, fa.queue, fa.status};
  const void* fn = nullptr;
#define KD_LF_F(IT, RR)                                                          \
  fn = form == 2   ? reinterpret_cast<const void*>(k_leaf<IT, RR, 2>)           \
       : form == 1 ? reinterpret_cast<const void*>(k_leaf<IT, RR, 1>)           \
                   : reinterpret_cast<const void*>(k_leaf<IT, RR, 0>)
#define KD_LF_R(IT)                                  \
  switch (k - 1) {                                   \
    case 1: KD_LF_F(IT, 1); break;                   \
    case 2: KD_LF_F(IT, 2); break;                   \
    case 3: KD_LF_F(IT, 3); break;                   \
    case 4: KD_LF_F(IT, 4); break;                   \
    case 5: KD_LF_F(IT, 5); break;                   \
    case 6: KD_LF_F(IT, 6); break;                   \
    case 7: KD_LF_F(IT, 7); break;                   \
    default: return hipErrorInvalidValue;            \
  }
  switch (cutover) {
    case 1024: KD_LF_R(4); break;
    case 2048: KD_LF_R(8); break;
    case 4096: KD_LF_R(16); break;
    default: return hipErrorInvalidValue;
  }
#undef KD_LF_R
#undef KD_LF_F
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  // persistent grid: enough workgroups to fill the chip, never more than items
  int64_t grid = blocks;
  if (items_bound < grid) grid = items_bound;
  if (grid < 1) grid = 1;
  void* args[] = {&B, &F, &n, &k, &perm};
  return hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kLfThreads), args, lds, st);
}

// ---- shape helpers ---------------------------------------------------------------

// k == 1: every tree's in-order layout is its sorted distinct rows.
__global__ __launch_bounds__(256) void k_copy_k1(const uint32_t* __restrict__ S0, const Forest F,
                                                int32_t* __restrict__ perm) {
  const int total = F.uoff[F.B];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int b = F.B == 1 ? 0 : upper_index(F.uoff, F.B, i);
    const int64_t ob = F.off[b];
    perm[ob + (i - F.uoff[b])] = (int32_t)((int64_t)S0[i] - ob);
  }
}

hipError_t launch_copy_k1(const uint32_t* S0, const ForestArgs& fa, int64_t n, int32_t* perm,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  Forest F{fa.B, fa.off, fa.uoff, fa.lmax, fa.wgbase, fa.queue, fa.status};
  hipLaunchKernelGGL(k_copy_k1, dim3((unsigned)blocks), dim3(256), 0, st, S0, F, perm);
  return hipGetLastError();
}

// Child positions of a single tree's in-order layout.
__global__ __launch_bounds__(256) void k_children(const int32_t* __restrict__ uoff,
                                                 int32_t* __restrict__ lo, int32_t* __restrict__ hi) {
  const int64_t nu = uoff[1];
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

hipError_t launch_children(const int32_t* uoff, int64_t n, int32_t* lo, int32_t* hi,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_children, dim3((unsigned)blocks), dim3(256), 0, st, uoff, lo, hi);
  return hipGetLastError();
}

}  // namespace kd
