// Level form 4 of the tree half of the build (one tree): every global level
// moves one array instead of k-1.
//
// The paper partitions k-1 arrays about every median (Sec. 2.1) and notes
// that partitioning an array can be put off until its dimension is needed
// (Appendix, "Deferred Merge Sort and Partitioning").  Carried through every
// level: the array sorted by dimension p is only needed at the levels that
// split in p, so it is partitioned right before such a level, about all the
// medians found since it was last split (k-1 levels), in one stable
// multi-way split.  Each element walks down from its subarray through the
// medians of those levels -- a compare of its own rank with the median's, as
// at a global level -- and lands in its subarray k-1 levels further down, in
// the array's order.  The tree is the same: a stable split of a sorted
// subarray by subtree yields every subtree in sorted order.
//
// A split is three launches (count, chain, move) as a level of the other
// forms; a fourth small launch per level records the medians' ranks (the
// walks of later splits read them) and writes the nodes into perm.
#include "common.hpp"
#include "launch.hpp"

namespace kd {

namespace {

constexpr int kSpThreads = 512;
constexpr int kSpItems = kLevelTile / kSpThreads;  // 8 positions per thread
constexpr int kSpWaves = kSpThreads / kWave;
constexpr int kSpMaxPieces = 8;   // subarrays of the source depth meeting a tile
constexpr int kSpSamples = kLevelTile / 512 + 1;
constexpr int kSpKeys = 256;      // (piece, bucket) pairs of a tile
constexpr int kSpMaxBuckets = 1 << (kMaxK - 1);
constexpr uint32_t kDrop = 0xFFFFFFFFu;

struct Bufs {
  const uint32_t* rec0;
  const uint32_t* rows;
  uint32_t* b1;
  uint32_t* b2;
};
__device__ __forceinline__ const uint32_t* buf_of(const Bufs& B, int moves) {
  return moves == 0 ? B.rec0 : ((moves & 1) ? B.b1 : B.b2);
}

// What a split launch does, decided on the device from the deepest global
// level D (the host enqueues every level a tree of n rows could need).
struct Plan {
  int q;         // the array split
  int from, to;  // its layout's depth before and after
  int moves;     // splits of the array before this one
  bool active;
};
__device__ __forceinline__ Plan split_plan(const SplitJob& J) {
  Plan P;
  const int D = *J.lmax;
  if (J.final_j < 0) {
    const int L = J.level;
    P.q = L % J.k;
    P.to = L;
    P.from = roll_depth(L, P.q, J.k);
    P.moves = roll_moves(L, P.q, J.k);
    P.active = L >= 1 && L < D;
  } else {
    P.q = J.final_j;
    P.to = D;
    P.from = roll_depth(D, P.q, J.k);
    P.moves = roll_moves(D, P.q, J.k);
    P.active = D >= 1 && P.from < D;
  }
  return P;
}

// Planes holding the ranks the walk from depth `from` to `to` compares.
__device__ __forceinline__ uint32_t deciding_planes(int q, int from, int to, int k) {
  uint32_t m = 0;
  for (int l = from; l < to; ++l) m |= 1u << plane_of(q, l % k, k);
  return m;
}

// Subarray of depth `depth` holding position pos of a tree of nu positions:
// its range and index (left to right), or e < s when pos is the node of a
// shallower subarray.
__device__ __forceinline__ void subarray_index(int pos, int nu, int depth, int* s_out, int* e_out,
                                               int* c_out) {
  int s = 0, e = nu - 1, c = 0;
  for (int l = 0; l < depth; ++l) {
    const int m = s + ((e - s) >> 1);
    if (pos < m) {
      e = m - 1;
      c = 2 * c;
    } else if (pos > m) {
      s = m + 1;
      c = 2 * c + 1;
    } else {
      s = 1;
      e = 0;
      c = -1;
      break;
    }
  }
  *s_out = s;
  *e_out = e;
  *c_out = c;
}

// Wave 0: the subarrays of depth `depth` meeting positions [t0, t1).  Every
// such subarray holds at least 1024 positions, so one of the positions t0,
// t0 + 512, ..., t1 - 1 (or the one after it, if that one is a node) lies in
// it.  Returns the count in every lane of wave 0 (more than kSpMaxPieces is
// an inconsistency: only the first kSpMaxPieces are kept).
__device__ int find_pieces(int nu, int depth, int t0, int t1, SplitInfo* out, uint32_t* status) {
  const int lane = lane_id();
  int s = INT32_MAX, e = -1, c = -1;
  if (lane < kSpSamples) {
    int pos = t0 + lane * 512;
    if (pos > t1 - 1) pos = t1 - 1;
    subarray_index(pos, nu, depth, &s, &e, &c);
    if (e < s && pos + 1 < t1) subarray_index(pos + 1, nu, depth, &s, &e, &c);
    if (e < s) {
      s = INT32_MAX;
      e = -1;
    }
  }
  const int prev_s = __shfl_up(s, 1, kWave);
  const bool keep = lane < kSpSamples && s != INT32_MAX && (lane == 0 || prev_s != s);
  const uint64_t km = __ballot(keep);
  if (keep) {
    const int idx = (int)popc64(km & lanes_below_mask());
    if (idx < kSpMaxPieces) {
      out->s[idx] = s;
      out->e[idx] = e;
      out->c[idx] = c;
    }
  }
  const int np = (int)popc64(km);
  if (lane == 0) {
    if (np > kSpMaxPieces) atomicOr(status, kStatusSplit);
    out->np = min(np, kSpMaxPieces);
  }
  return min(np, kSpMaxPieces);
}

// Ranks (in the orders of the levels walked) of the nodes below every piece,
// in heap order: s_med[piece * kSpMaxBuckets + h], h = 1 for the piece's own
// node, 2h / 2h+1 for the nodes of its lower / upper half.  The table
// med[(1 << l) - 1 + c] holds the rank in order l mod k of subarray c's node
// at depth l.
__device__ __forceinline__ void stage_medians(const SplitInfo& si, int from, int s_levels,
                                              const uint32_t* __restrict__ med, uint32_t* s_med) {
  const int B = 1 << s_levels;
  for (int t = threadIdx.x; t < si.np * B; t += blockDim.x) {
    const int pc = t / B, h = t % B;
    if (h == 0) continue;
    const int lr = 31 - __clz(h);  // level below the piece
    const int c = (si.c[pc] << lr) + (h - (1 << lr));
    s_med[pc * kSpMaxBuckets + h] = med[((1 << (from + lr)) - 1) + c];
  }
}

// Bucket of an element (its subtree k-1 levels down, 0 .. 2^s - 1), or kDrop
// when it is one of the nodes passed on the way.  v: its record planes.
template <int W>
__device__ __forceinline__ uint32_t walk(const uint32_t (&v)[W], const uint32_t* s_med_piece, int q,
                                         int from, int s_levels, int k) {
  uint32_t h = 1;
  for (int l = 0; l < s_levels; ++l) {
    const int pl = plane_of(q, (from + l) % k, k);
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < W; ++c)
      if (c == pl) r = v[c];
    const uint32_t nr = s_med_piece[h];
    if (r == nr) return kDrop;
    h = 2 * h + (r > nr ? 1u : 0u);
  }
  return h - (1u << s_levels);
}

// Range of the subtree reached from [s, e] by the bucket's bits (most
// significant first, s_levels of them).
__device__ __forceinline__ void descend(int& s, int& e, uint32_t b, int s_levels) {
  for (int l = s_levels - 1; l >= 0; --l) {
    const int m = s + ((e - s) >> 1);
    if ((b >> l) & 1u)
      s = m + 1;
    else
      e = m - 1;
  }
}

// Counts of every bucket among the tile's last piece (tval[b][t]) and the
// tile's flags (bit 0: that piece starts inside the tile; bit 1: the first
// piece started before it), with the pieces kept for the move (info[t]).
template <int W>
__global__ __launch_bounds__(kSpThreads) void k_split_count(const Bufs Bf, const SplitJob J,
                                                           SplitInfo* __restrict__ info,
                                                           uint32_t* __restrict__ tval,
                                                           uint32_t* __restrict__ tflag,
                                                           int tiles_stride) {
  __shared__ SplitInfo s_si;
  __shared__ uint32_t s_med[kSpMaxPieces * kSpMaxBuckets];
  __shared__ uint32_t s_hist[kSpMaxBuckets];
  const Plan P = split_plan(J);
  if (!P.active) return;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int nu = J.uoff[1];
  const int t = blockIdx.x;
  const int t0 = t * kLevelTile;
  if (t0 >= nu) return;
  const int t1 = min(t0 + kLevelTile, nu);
  const int sl = P.to - P.from;
  const int B = 1 << sl;
  const int k = J.k;
  const uint32_t dmask = deciding_planes(P.q, P.from, P.to, k);
  const uint32_t* src = buf_of(Bf, P.moves) + record_offset(P.q, k, J.n);
  // planes first: their loads overlap the piece search
  uint32_t v[W][kSpItems];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const bool need = (dmask >> c) & 1u;
#pragma unroll
    for (int it = 0; it < kSpItems; ++it) {
      const int i = t0 + w * (kWave * kSpItems) + it * kWave + lane;
      v[c][it] = need && i < t1 ? src[(int64_t)c * J.n + i] : 0u;
    }
  }
  if (tid < kWave) find_pieces(nu, P.from, t0, t1, &s_si, J.status);
  if (tid < kSpMaxBuckets) s_hist[tid] = 0;
  __syncthreads();
  stage_medians(s_si, P.from, sl, J.med, s_med);
  if (tid < kSpMaxPieces) {
    info[t].s[tid] = s_si.s[tid];
    info[t].e[tid] = s_si.e[tid];
    info[t].c[tid] = s_si.c[tid];
    if (tid == 0) info[t].np = s_si.np;
  }
  __syncthreads();
  const int np = s_si.np;
  const int ls = np > 0 ? max(s_si.s[np - 1], t0) : t1;
  const int le = np > 0 ? min(s_si.e[np - 1] + 1, t1) : t1;
  const uint64_t below = lanes_below_mask();
#pragma unroll
  for (int it = 0; it < kSpItems; ++it) {
    const int i = t0 + w * (kWave * kSpItems) + it * kWave + lane;
    uint32_t b = kDrop;
    if (i >= ls && i < le) {
      uint32_t x[W];
#pragma unroll
      for (int c = 0; c < W; ++c) x[c] = v[c][it];
      b = walk<W>(x, s_med + (np - 1) * kSpMaxBuckets, P.q, P.from, sl, k);
    }
    // lanes with the same bucket: one LDS add per distinct bucket
    const bool valid = b != kDrop;
    uint64_t m = __ballot(valid);
    for (int bit = 0; bit < sl; ++bit) {
      const bool on = (b >> bit) & 1u;
      const uint64_t bb = __ballot(on);
      m &= on ? bb : ~bb;
    }
    if (valid && popc64(m & below) == 0) atomicAdd(&s_hist[b], popc64(m));
  }
  __syncthreads();
  if (tid < B) tval[(int64_t)tid * tiles_stride + t] = s_hist[tid];
  if (tid == 0) {
    const bool head = np == 0 || s_si.s[np - 1] >= t0;
    const bool cont = np > 0 && s_si.s[0] < t0;
    tflag[t] = (head ? 1u : 0u) | (cont ? 2u : 0u);
  }
}

// Chains the counts along every piece, one block per bucket: carry[b][t] =
// the elements of bucket b of tile t's first piece in the tiles before t
// (when that piece started before t).  A segmented scan: tile t contributes
// (v, h) = (its count, its last piece starts inside it).
__global__ __launch_bounds__(1024) void k_split_scan(const SplitJob J,
                                                    const uint32_t* __restrict__ tval,
                                                    const uint32_t* __restrict__ tflag,
                                                    uint32_t* __restrict__ carry,
                                                    int tiles_stride) {
  constexpr int kThreads = 1024, kWaves = kThreads / kWave;
  __shared__ uint32_t s_v[kWaves];
  __shared__ int s_h[kWaves];
  const Plan P = split_plan(J);
  if (!P.active) return;
  const int b = blockIdx.x;
  if (b >= (1 << (P.to - P.from))) return;
  const int tid = threadIdx.x;
  const int nu = J.uoff[1];
  const int tiles = (nu + kLevelTile - 1) / kLevelTile;
  const int per = (tiles + kThreads - 1) / kThreads;
  const int c0 = min(tiles, tid * per), c1 = min(tiles, c0 + per);
  const uint32_t* tv = tval + (int64_t)b * tiles_stride;
  uint32_t av = 0;
  int ah = 0;
  for (int t = c0; t < c1; ++t) {
    const int h = (int)(tflag[t] & 1u);
    av = h ? tv[t] : av + tv[t];
    ah |= h;
  }
  uint32_t iv = av;
  int ih = ah;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t ov = __shfl_up(iv, d, kWave);
    const int oh = __shfl_up(ih, d, kWave);
    if ((int)lane_id() >= d) {
      if (!ih) iv += ov;
      ih |= oh;
    }
  }
  const int w = tid / kWave;
  if (lane_id() == kWave - 1) {
    s_v[w] = iv;
    s_h[w] = ih;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t rv = 0;
    int rh = 0;
    for (int q = 0; q < kWaves; ++q) {
      const uint32_t qv = s_v[q];
      const int qh = s_h[q];
      s_v[q] = rv;
      s_h[q] = rh;
      rv = qh ? qv : rv + qv;
      rh |= qh;
    }
  }
  __syncthreads();
  uint32_t ev = __shfl_up(iv, 1, kWave);
  int eh = __shfl_up(ih, 1, kWave);
  if (lane_id() == 0) {
    ev = 0;
    eh = 0;
  }
  if (!eh) ev += s_v[w];
  uint32_t run = ev;
  uint32_t* cy = carry + (int64_t)b * tiles_stride;
  for (int t = c0; t < c1; ++t) {
    const uint32_t f = tflag[t];
    cy[t] = (f & 2u) ? run : 0u;
    run = (f & 1u) ? tv[t] : run + tv[t];
  }
}

// Moves one tile: every element's (piece, bucket) key, its stable rank among
// the tile's elements of that key (wave ballots, as in a radix pass), and the
// start of its subtree plus the carried count give its new position; the
// planes in wmask are written there.
template <int W>
__global__ __launch_bounds__(kSpThreads) void k_split_move(const Bufs Bf, const SplitJob J,
                                                          const SplitInfo* __restrict__ info,
                                                          const uint32_t* __restrict__ tflag,
                                                          const uint32_t* __restrict__ carry,
                                                          int tiles_stride) {
  __shared__ SplitInfo s_si;
  __shared__ uint32_t s_med[kSpMaxPieces * kSpMaxBuckets];
  __shared__ uint32_t s_wcnt[kSpWaves][kSpKeys];
  __shared__ int32_t s_base[kSpKeys];
  __shared__ int32_t s_end[kSpKeys];
  const Plan P = split_plan(J);
  if (!P.active) return;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int nu = J.uoff[1];
  const int tiles = (nu + kLevelTile - 1) / kLevelTile;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= tiles) return;
  const int t0 = t * kLevelTile;
  const int t1 = min(t0 + kLevelTile, nu);
  const int sl = P.to - P.from;
  const int B = 1 << sl;
  const int k = J.k;
  const uint32_t dmask = deciding_planes(P.q, P.from, P.to, k);
  const uint32_t wmask = J.wmask;
  const uint32_t* src = buf_of(Bf, P.moves) + record_offset(P.q, k, J.n);
  uint32_t* dst = const_cast<uint32_t*>(buf_of(Bf, P.moves + 1)) + record_offset(P.q, k, J.n);
  uint32_t v[W][kSpItems];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const bool need = ((dmask | wmask) >> c) & 1u;
#pragma unroll
    for (int it = 0; it < kSpItems; ++it) {
      const int i = t0 + w * (kWave * kSpItems) + it * kWave + lane;
      v[c][it] = need && i < t1 ? src[(int64_t)c * J.n + i] : 0u;
    }
  }
  if (tid < kSpMaxPieces) {
    s_si.s[tid] = info[t].s[tid];
    s_si.e[tid] = info[t].e[tid];
    s_si.c[tid] = info[t].c[tid];
    if (tid == 0) s_si.np = info[t].np;
  }
  for (int q = tid; q < kSpWaves * kSpKeys; q += kSpThreads) (&s_wcnt[0][0])[q] = 0;
  __syncthreads();
  const int np = s_si.np;
  if (np * B > kSpKeys) {  // not reached: pieces are large when buckets are many
    if (tid == 0) atomicOr(J.status, kStatusSplit);
    return;
  }
  stage_medians(s_si, P.from, sl, J.med, s_med);
  const uint32_t f = tflag[t];
  if (tid < np * B) {
    const int pc = tid / B;
    const uint32_t b = (uint32_t)(tid % B);
    int s = s_si.s[pc], e = s_si.e[pc];
    descend(s, e, b, sl);
    const int cy = (pc == 0 && (f & 2u)) ? (int)carry[(int64_t)b * tiles_stride + t] : 0;
    s_base[tid] = s + cy;
    s_end[tid] = e;
  }
  __syncthreads();
  // key of every element: piece * B + bucket, or kDrop (a node passed on the
  // way, or a position that is a node of a shallower depth)
  uint32_t key[kSpItems], rank[kSpItems];
  const uint64_t below = lanes_below_mask();
#pragma unroll
  for (int it = 0; it < kSpItems; ++it) {
    const int i = t0 + w * (kWave * kSpItems) + it * kWave + lane;
    uint32_t kk = kDrop;
    if (i < t1) {
      int pc = -1;
      for (int q = 0; q < np; ++q)
        if (i >= s_si.s[q] && i <= s_si.e[q]) {
          pc = q;
          break;
        }
      if (pc >= 0) {
        uint32_t x[W];
#pragma unroll
        for (int c = 0; c < W; ++c) x[c] = v[c][it];
        const uint32_t b = walk<W>(x, s_med + pc * kSpMaxBuckets, P.q, P.from, sl, k);
        if (b != kDrop) kk = (uint32_t)pc * (uint32_t)B + b;
      }
    }
    key[it] = kk;
    const bool valid = kk != kDrop;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (kk >> bit) & 1u;
      const uint64_t bb = __ballot(on);
      m &= on ? bb : ~bb;
    }
    uint32_t pre = 0;
    if (valid) pre = s_wcnt[w][kk & 0xFF];
    __builtin_amdgcn_wave_barrier();
    const uint32_t before = popc64(m & below);
    if (valid && before == 0) s_wcnt[w][kk] = pre + popc64(m);
    __builtin_amdgcn_wave_barrier();
    rank[it] = pre + before;
  }
  __syncthreads();
  // waves before this one, per key
  if (tid < kSpKeys) {
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < kSpWaves; ++q) {
      const uint32_t c = s_wcnt[q][tid];
      s_wcnt[q][tid] = run;
      run += c;
    }
  }
  __syncthreads();
  int dest[kSpItems];
#pragma unroll
  for (int it = 0; it < kSpItems; ++it) {
    dest[it] = -1;
    const uint32_t kk = key[it];
    if (kk == kDrop) continue;
    const int d = s_base[kk] + (int)(s_wcnt[w][kk] + rank[it]);
    if (d <= s_end[kk])
      dest[it] = d;
    else  // only if the counts were inconsistent
      atomicOr(J.status, kStatusSplit);
  }
#pragma unroll
  for (int c = 0; c < W; ++c) {
    if (!((wmask >> c) & 1u)) continue;
    uint32_t* dp = dst + (int64_t)c * J.n;
#pragma unroll
    for (int it = 0; it < kSpItems; ++it)
      if (dest[it] >= 0) dp[dest[it]] = v[c][it];
  }
}

// The nodes of depth L: array p = L mod k has its depth-L layout (after its
// split at L, or presorted for L = 0), so subarray c's node is its middle
// element there.  Its rank in order p (plane 0 holds order p+1, which the
// level-0 records of array p+1 translate) goes to the median table, and its
// row (the order-0 id array at its order-0 rank) to perm.
__global__ __launch_bounds__(256) void k_split_medians(const Bufs Bf, const SplitJob J,
                                                      uint32_t* __restrict__ med,
                                                      int32_t* __restrict__ perm) {
  const int L = J.level;
  if (L >= *J.lmax) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (1 << L)) return;
  const int k = J.k;
  const int nu = J.uoff[1];
  int s = 0, e = nu - 1;
  for (int l = L - 1; l >= 0; --l) {
    const int m = s + ((e - s) >> 1);
    if ((c >> l) & 1)
      s = m + 1;
    else
      e = m - 1;
  }
  if (e < s) {  // not reached: global-level subarrays hold at least C rows
    atomicOr(J.status, kStatusNode);
    return;
  }
  const int p = L % k;
  const int m = s + ((e - s) >> 1);
  const uint32_t* arr =
      buf_of(Bf, roll_moves(L, p, k) + (L >= 1 ? 1 : 0)) + record_offset(p, k, J.n);
  const uint32_t r1 = arr[m];
  if (r1 >= (uint32_t)nu) {  // not reached: a rank
    atomicOr(J.status, kStatusNode);
    return;
  }
  const uint32_t rp = Bf.rec0[record_offset((p + 1) % k, k, J.n) + (int64_t)(k - 2) * J.n + r1];
  med[(1 << L) - 1 + c] = rp;
  const uint32_t r0 = p == 0 ? rp : arr[(int64_t)plane_of(p, 0, k) * J.n + m];
  if (r0 >= (uint32_t)nu) {  // not reached: a rank
    atomicOr(J.status, kStatusNode);
    return;
  }
  perm[m] = (int32_t)Bf.rows[r0];
}

}  // namespace

size_t split_info_bytes() { return sizeof(SplitInfo); }

hipError_t launch_split(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1, uint32_t* b2,
                        const SplitJob& J, SplitInfo* info, uint32_t* tval, uint32_t* tflag,
                        uint32_t* carry, hipStream_t st) {
  if (J.n <= 0 || J.k < 2 || J.k > kMaxK) return hipSuccess;
  const int tiles = (int)level_tiles(J.n);
  const Bufs Bf{rec0, rows, b1, b2};
#define KD_SP(WW)                                                                              \
  do {                                                                                         \
    hipLaunchKernelGGL(k_split_count<WW>, dim3(tiles), dim3(kSpThreads), 0, st, Bf, J, info,  \
                       tval, tflag, tiles);                                                    \
    hipLaunchKernelGGL(k_split_scan, dim3(1 << (J.k - 1)), dim3(1024), 0, st, J, tval, tflag, \
                       carry, tiles);                                                          \
    hipLaunchKernelGGL(k_split_move<WW>, dim3(xcd_grid(tiles)), dim3(kSpThreads), 0, st, Bf, J, \
                       info, tflag, carry, tiles);                                             \
  } while (0)
  switch (J.k - 1) {
    case 1: KD_SP(1); break;
    case 2: KD_SP(2); break;
    case 3: KD_SP(3); break;
    case 4: KD_SP(4); break;
    case 5: KD_SP(5); break;
    case 6: KD_SP(6); break;
    case 7: KD_SP(7); break;
    default: return hipErrorInvalidValue;
  }
#undef KD_SP
  return hipGetLastError();
}

hipError_t launch_split_medians(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1,
                                uint32_t* b2, const SplitJob& J, uint32_t* med, int32_t* perm,
                                hipStream_t st) {
  if (J.n <= 0 || J.k < 2 || J.level < 0 || J.level > 30) return hipErrorInvalidValue;
  const Bufs Bf{rec0, rows, b1, b2};
  const int nodes = 1 << J.level;
  hipLaunchKernelGGL(k_split_medians, dim3((nodes + 255) / 256), dim3(256), 0, st, Bf, J, med, perm);
  return hipGetLastError();
}

// Planes each split writes, walking back from the on-chip finish exactly as
// the launches run: the finish reads the order-0 plane of arrays 1 .. k-1; a
// final split of array j writes what the finish reads and reads the planes
// its walk compares; the medians of level L read plane 0 of array p and, for
// p != 0, its order-0 plane; the split at level L writes what later reads of
// array p need and reads the planes its walk compares.
// A final split always writes just the order-0 plane: the device runs one
// for every array whose layout is above its own deepest level, which for a
// tree that duplicates made shallower can be an array the host's count says
// needs none.  Trimming the earlier splits by the host's count is safe: with
// fewer levels, each array's last split is followed by a final split that
// compares a subset of the levels the host's schedule compares after it.
void rolling_masks(int k, int levels, uint32_t* level_mask, uint32_t* final_mask) {
  uint32_t need[kMaxK] = {};
  final_mask[0] = 0;
  for (int j = 1; j < k; ++j) final_mask[j] = need[j] = 1u << plane_of(j, 0, k);
  if (levels >= 1)
    for (int j = 1; j < k; ++j) {
      const int a = roll_depth(levels, j, k);
      if (a >= levels) continue;
      for (int l = a; l < levels; ++l) need[j] |= 1u << plane_of(j, l % k, k);
    }
  for (int L = levels - 1; L >= 0; --L) {
    const int p = L % k;
    need[p] |= 1u;
    if (p != 0) need[p] |= 1u << plane_of(p, 0, k);
    level_mask[L] = 0;
    if (L >= 1) {
      level_mask[L] = need[p];
      for (int l = roll_depth(L, p, k); l < L; ++l) need[p] |= 1u << plane_of(p, l % k, k);
    }
  }
}

}  // namespace kd
