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
// A split is three launches as a level of the other forms: the count walks
// every element once (its key goes to a byte array the move reads instead of
// walking again), the chain scans the counts along every piece, the move
// ranks and writes.  A fourth small launch per level records the medians'
// ranks (the walks of later splits read them) and writes the nodes to perm.
#include "common.hpp"
#include "launch.hpp"

namespace kd {

namespace {

constexpr int kSpThreads = 512;
constexpr int kSpItems = kLevelTile / kSpThreads;  // 8 positions per thread
constexpr int kSpWaves = kSpThreads / kWave;
constexpr int kSpMaxPieces = 8;   // subarrays of the source depth meeting a tile
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

// The subarrays of depth `depth` meeting positions [t0, t1) are the
// consecutive ones c_lo .. c_hi: those holding the first and the last
// position of the range that is not a node of a shallower depth (such a node
// has subarray positions on both sides, and subarrays here hold at least 1024
// positions).  Every thread computes the same two indices.
__device__ __forceinline__ void tile_pieces(int nu, int depth, int t0, int t1, int* c_lo, int* c_hi) {
  int s, e, c;
  subarray_index(t0, nu, depth, &s, &e, &c);
  if (c < 0) subarray_index(t0 + 1, nu, depth, &s, &e, &c);
  *c_lo = c;
  subarray_index(t1 - 1, nu, depth, &s, &e, &c);
  if (c < 0) subarray_index(t1 - 2, nu, depth, &s, &e, &c);
  *c_hi = c;
}

// Range of subarray c at `depth` (one tree of nu positions).
__device__ __forceinline__ void subarray_range(int nu, int depth, int c, int* s_out, int* e_out) {
  int s = 0, e = nu - 1;
  for (int l = depth - 1; l >= 0; --l) {
    const int m = s + ((e - s) >> 1);
    if ((c >> l) & 1)
      s = m + 1;
    else
      e = m - 1;
  }
  *s_out = s;
  *e_out = e;
}

// Record plane compared at each level of the walk from depth `from`, three
// bits per level (the same for every element of a split).
template <int K>
__device__ __forceinline__ uint32_t walk_planes(int q, int from, int s_levels) {
  uint32_t packed = 0;
  for (int l = 0; l < s_levels; ++l) packed |= (uint32_t)plane_of(q, (from + l) % K, K) << (3 * l);
  return packed;
}

// Bucket of an element (its subtree sl levels down, 0 .. 2^sl - 1), or kDrop
// when it is one of the nodes passed on the way.  xv[l]: its rank in the order
// compared at level l of the walk.  Branch-free, so the walks of a thread's
// elements interleave: after a node is met the remaining steps run on
// harmlessly.
template <int W>
__device__ __forceinline__ uint32_t walk(const uint32_t (&xv)[W], const uint32_t* s_med_piece, int sl) {
  uint32_t h = 1;
  bool node = false;
#pragma unroll
  for (int l = 0; l < W; ++l) {
    if (l < sl) {
      const uint32_t r = xv[l];
      const uint32_t nr = s_med_piece[h];
      node = node || r == nr;
      h = 2 * h + (r > nr ? 1u : 0u);
    }
  }
  return node ? kDrop : h - (1u << sl);
}

// Range of the subtree reached from [s, e] by the bucket's bits (most
// significant first, sl of them).
__device__ __forceinline__ void descend(int& s, int& e, uint32_t b, int sl) {
  for (int l = sl - 1; l >= 0; --l) {
    const int m = s + ((e - s) >> 1);
    if ((b >> l) & 1u)
      s = m + 1;
    else
      e = m - 1;
  }
}

// The same walk for a tile inside one piece, kSl <= 3 levels deep: the
// seven node ranks below the piece are the same for every element (m[h],
// heap order), so they sit in registers and each step picks one of them.
template <int W, int kSl>
__device__ __forceinline__ uint32_t walk3(const uint32_t (&xv)[W], const uint32_t (&m)[8]) {
  uint32_t h = 1;
  bool node = false;
#pragma unroll
  for (int l = 0; l < kSl; ++l) {
    const uint32_t r = xv[l];
    uint32_t nr;
    if (l == 0)
      nr = m[1];
    else if (l == 1)
      nr = h == 2 ? m[2] : m[3];
    else
      nr = h == 4 ? m[4] : (h == 5 ? m[5] : (h == 6 ? m[6] : m[7]));
    node = node || r == nr;
    h = 2 * h + (r > nr ? 1u : 0u);
  }
  return node ? kDrop : h - (1u << kSl);
}

// The elements of a tile inside one piece, walked kSl levels: keys packed
// into kw, bucket counts by wave ballots summed in scalar registers and added
// to s_hist once per wave.
template <int W, int kSl, int kBits, int kPerWord, int kWords>
__device__ __forceinline__ void count_single(const uint32_t (&x)[W][kSpItems], const uint32_t* s_med,
                                             int t0, int t1, int ps0, int pe0, int w, int lane,
                                             uint32_t (&kw)[kWords], uint32_t* s_hist) {
  constexpr int kB = 1 << kSl;
  constexpr uint32_t kNone = (1u << kBits) - 1u;
  uint32_t m1[8];
#pragma unroll
  for (int h = 0; h < 8; ++h) m1[h] = h >= 1 && h < kB ? s_med[h] : 0u;
  // a tile wholly inside the piece needs no per-element test; otherwise a
  // node of a shallower depth may open or close the tile
  const bool whole = ps0 <= t0 && pe0 >= t1 - 1;
  uint32_t hc[kB];
#pragma unroll
  for (int bb = 0; bb < kB; ++bb) hc[bb] = 0u;
#pragma unroll
  for (int it = 0; it < kSpItems; ++it) {
    const int i = t0 + w * (kWave * kSpItems) + it * kWave + lane;
    uint32_t xv[W];
#pragma unroll
    for (int l = 0; l < W; ++l) xv[l] = x[l][it];
    const bool in = i < t1 && (whole || (i >= ps0 && i <= pe0));
    const uint32_t b = in ? walk3<W, kSl>(xv, m1) : kDrop;
    kw[it / kPerWord] |= (b == kDrop ? kNone : b) << (kBits * (it % kPerWord));
#pragma unroll
    for (int bb = 0; bb < kB; ++bb) hc[bb] += popc64(__ballot(b == (uint32_t)bb));
  }
  if (lane == 0) {
#pragma unroll
    for (int bb = 0; bb < kB; ++bb)
      if (hc[bb] != 0u) atomicAdd(&s_hist[bb], hc[bb]);
  }
}

// Key of an element for the move: piece << sl | bucket, below 256 (pieces
// are few where buckets are many); 8 bits, or 16 at k = 8 where all 256
// values occur.  The largest value marks an element that does not move.
// A thread's keys are packed into 32-bit words, stored where only the same
// thread of the move reads them: word j of thread (tile t, wave w, lane) at
// ((t * kSpWaves + w) * KeyWords + j) * 64 + lane, so every store and load is
// a whole 256-byte run.
template <int W>
struct SplitKeys {
  static constexpr int kBits = W >= 7 ? 16 : 8;
  static constexpr uint32_t kNone = (1u << kBits) - 1u;
  static constexpr int kPerWord = 32 / kBits;
  static constexpr int kWords = kSpItems / kPerWord;
};

// Piece of position i among the tile's pieces (bounds in registers), or -1.
__device__ __forceinline__ int piece_of(int i, const int (&ps)[kSpMaxPieces],
                                        const int (&pe)[kSpMaxPieces], int np) {
  int pc = -1;
#pragma unroll
  for (int q = 0; q < kSpMaxPieces; ++q)
    if (q < np && i >= ps[q]) pc = q;
  int e = -1;
#pragma unroll
  for (int q = 0; q < kSpMaxPieces; ++q)
    if (q == pc) e = pe[q];
  return (pc >= 0 && i <= e) ? pc : -1;
}

// Walks every element of the tile once: its key for the move (keys[i]), the
// counts of every bucket among the tile's last piece (tval[b][t]) and the
// tile's flags (bit 0: that piece starts inside the tile; bit 1: the first
// piece started before it), with the pieces kept for the move (info[t]).
// The usual tile lies inside one piece and walks at most three levels: its
// node ranks sit in registers and its bucket counts are wave ballots summed in
// scalar registers; other tiles search each element's piece and count with a
// digit match.
template <int W>
__global__ __launch_bounds__(kSpThreads) void k_split_count(const Bufs Bf, const SplitJob J,
                                                           SplitInfo* __restrict__ info,
                                                           uint32_t* __restrict__ tval,
                                                           uint32_t* __restrict__ tflag,
                                                           int tiles_stride,
                                                           uint32_t* __restrict__ keys) {
  using K = SplitKeys<W>;
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
  constexpr int k = W + 1;
  const uint32_t planes = walk_planes<k>(P.q, P.from, sl);
  const uint32_t* src = buf_of(Bf, P.moves) + record_offset(P.q, k, J.n);
  // the compared planes, in walk order, first: their loads overlap the piece search
  uint32_t x[W][kSpItems];
#pragma unroll
  for (int l = 0; l < W; ++l) {
    const bool need = l < sl;
    const int pl = (int)((planes >> (3 * l)) & 7u);
#pragma unroll
    for (int it = 0; it < kSpItems; ++it) {
      const int i = t0 + w * (kWave * kSpItems) + it * kWave + lane;
      x[l][it] = need && i < t1 ? src[(int64_t)pl * J.n + i] : 0u;
    }
  }
  // the pieces and the medians below them, without waiting for the planes
  int c_lo, c_hi;
  tile_pieces(nu, P.from, t0, t1, &c_lo, &c_hi);
  int np = c_hi - c_lo + 1;
  if (np > kSpMaxPieces || np < 1) {  // not reached: pieces hold at least 1024 positions
    if (tid == 0) atomicOr(J.status, kStatusSplit);
    np = max(1, min(np, kSpMaxPieces));
  }
  if (tid < kSpMaxPieces) {
    int ss = 1, ee = 0;
    if (tid < np) subarray_range(nu, P.from, c_lo + tid, &ss, &ee);
    s_si.s[tid] = ss;
    s_si.e[tid] = ee;
    info[t].s[tid] = ss;
    info[t].e[tid] = ee;
    info[t].c[tid] = c_lo + tid;
    if (tid == 0) info[t].np = np;
  }
  for (int q = tid; q < np * B; q += kSpThreads) {
    const int pc = q >> sl, h = q & (B - 1);
    if (h == 0) continue;
    const int lr = 31 - __clz(h);  // level below the piece
    const int c = ((c_lo + pc) << lr) + (h - (1 << lr));
    s_med[pc * kSpMaxBuckets + h] = J.med[((1 << (P.from + lr)) - 1) + c];
  }
  if (tid < kSpMaxBuckets) s_hist[tid] = 0;
  __syncthreads();
  int ps[kSpMaxPieces], pe[kSpMaxPieces];
#pragma unroll
  for (int q = 0; q < kSpMaxPieces; ++q) {
    ps[q] = s_si.s[q];
    pe[q] = s_si.e[q];
  }
  uint32_t kw[K::kWords];
#pragma unroll
  for (int j = 0; j < K::kWords; ++j) kw[j] = 0u;
  if (np == 1 && sl <= 3) {
    if (sl == 1)
      count_single<W, 1, K::kBits, K::kPerWord, K::kWords>(x, s_med, t0, t1, ps[0], pe[0], w, lane, kw, s_hist);
    else if constexpr (W >= 2) {
      if (sl == 2)
        count_single<W, 2, K::kBits, K::kPerWord, K::kWords>(x, s_med, t0, t1, ps[0], pe[0], w, lane, kw, s_hist);
      else if constexpr (W >= 3)
        count_single<W, 3, K::kBits, K::kPerWord, K::kWords>(x, s_med, t0, t1, ps[0], pe[0], w, lane, kw, s_hist);
    }
  } else {
#pragma unroll
    for (int it = 0; it < kSpItems; ++it) {
      const int i = t0 + w * (kWave * kSpItems) + it * kWave + lane;
      uint32_t xv[W];
#pragma unroll
      for (int l = 0; l < W; ++l) xv[l] = x[l][it];
      const int pc = i < t1 ? piece_of(i, ps, pe, np) : -1;
      const uint32_t b = pc >= 0 ? walk<W>(xv, s_med + pc * kSpMaxBuckets, sl) : kDrop;
      const uint32_t kk = b == kDrop ? K::kNone : (((uint32_t)pc << sl) | b);
      kw[it / K::kPerWord] |= kk << (K::kBits * (it % K::kPerWord));
      // the last piece's buckets: one LDS add per distinct bucket of a wave
      const bool last = b != kDrop && pc == np - 1;
      const uint64_t m = same_digit_lanes<W>(b, sl, __ballot(last));
      if (last && lanes_below(m) == 0) atomicAdd(&s_hist[b], popc64(m));
    }
  }
  {
    uint32_t* kp = keys + ((int64_t)t * kSpWaves + w) * K::kWords * kWave + lane;
#pragma unroll
    for (int j = 0; j < K::kWords; ++j) kp[j * kWave] = kw[j];
  }
  __syncthreads();
  if (tid < B) tval[(int64_t)tid * tiles_stride + t] = s_hist[tid];
  if (tid == 0) {
    const bool head = ps[np - 1] >= t0;
    const bool cont = ps[0] < t0;
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

// Stable rank of every element of a wave among the wave's elements of its
// key, for keys below kNk: one ballot per key value and item, the wave's
// running count per key in scalar registers, written to wcnt[0 .. kNk) once.
// Elements whose key is kNk or more (not moving) get no rank.
template <int kNk>
__device__ __forceinline__ void rank_few_keys(const uint32_t (&key)[kSpItems], int lane,
                                              uint32_t (&rank)[kSpItems], uint32_t* wcnt) {
  uint32_t run[kNk];
#pragma unroll
  for (int q = 0; q < kNk; ++q) run[q] = 0u;
#pragma unroll
  for (int it = 0; it < kSpItems; ++it) {
    const uint32_t kk = key[it];
    uint64_t mine = 0;
    uint32_t base = 0;
#pragma unroll
    for (int q = 0; q < kNk; ++q) {
      const uint64_t mq = __ballot(kk == (uint32_t)q);
      if (kk == (uint32_t)q) {
        mine = mq;
        base = run[q];
      }
      run[q] += popc64(mq);
    }
    rank[it] = base + lanes_below(mine);
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < kNk; ++q) wcnt[q] = run[q];
  }
}

// Moves one tile: every element's key (from the count), its stable rank
// among the tile's elements of that key (wave ballots, as in a radix pass),
// and the start of its subtree plus the carried count give its new position;
// the planes in wmask are written there.
template <int W>
__global__ __launch_bounds__(kSpThreads) void k_split_move(const Bufs Bf, const SplitJob J,
                                                          const SplitInfo* __restrict__ info,
                                                          const uint32_t* __restrict__ tflag,
                                                          const uint32_t* __restrict__ carry,
                                                          int tiles_stride,
                                                          const uint32_t* __restrict__ keys) {
  using K = SplitKeys<W>;
  constexpr uint32_t kNoKey = K::kNone;
  __shared__ SplitInfo s_si;
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
  constexpr int k = W + 1;
  const uint32_t wmask = J.wmask;
  const uint32_t* src = buf_of(Bf, P.moves) + record_offset(P.q, k, J.n);
  uint32_t* dst = const_cast<uint32_t*>(buf_of(Bf, P.moves + 1)) + record_offset(P.q, k, J.n);
  uint32_t key[kSpItems];
  {
    const uint32_t* kp = keys + ((int64_t)t * kSpWaves + w) * K::kWords * kWave + lane;
    uint32_t kw[K::kWords];
#pragma unroll
    for (int j = 0; j < K::kWords; ++j) kw[j] = kp[j * kWave];
#pragma unroll
    for (int it = 0; it < kSpItems; ++it)
      key[it] = (kw[it / K::kPerWord] >> (K::kBits * (it % K::kPerWord))) & K::kNone;
  }
  uint32_t v[W][kSpItems];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const bool need = (wmask >> c) & 1u;
#pragma unroll
    for (int it = 0; it < kSpItems; ++it) {
      const int i = t0 + w * (kWave * kSpItems) + it * kWave + lane;
      v[c][it] = need && i < t1 ? src[(int64_t)c * J.n + i] : 0u;
    }
  }
  // the carry of the first piece's buckets, loaded with the planes
  const uint32_t f = tflag[t];
  const uint32_t cy0 = tid < B ? carry[(int64_t)tid * tiles_stride + t] : 0u;
  if (tid < kSpMaxPieces) {
    s_si.s[tid] = info[t].s[tid];
    s_si.e[tid] = info[t].e[tid];
    if (tid == 0) s_si.np = info[t].np;
  }
  if (tid < B) s_end[tid] = (f & 2u) ? (int32_t)cy0 : 0;  // staged in s_end for a moment
  for (int q = tid; q < kSpWaves * kSpKeys; q += kSpThreads) (&s_wcnt[0][0])[q] = 0;
  __syncthreads();
  const int np = s_si.np;
  if (np * B > kSpKeys) {  // not reached: pieces are large when buckets are many
    if (tid == 0) atomicOr(J.status, kStatusSplit);
    return;
  }
  int base_q = 0, end_q = 0;
  if (tid < np * B) {
    const int pc = tid >> sl;
    const uint32_t b = (uint32_t)(tid & (B - 1));
    int s = s_si.s[pc], e = s_si.e[pc];
    descend(s, e, b, sl);
    base_q = s + (pc == 0 ? s_end[b] : 0);
    end_q = e;
  }
  __syncthreads();
  if (tid < np * B) {
    s_base[tid] = base_q;
    s_end[tid] = end_q;
  }
  uint32_t rank[kSpItems];
  if (np * B <= 4) {
    rank_few_keys<4>(key, lane, rank, s_wcnt[w]);
  } else if (np * B <= 8) {
    rank_few_keys<8>(key, lane, rank, s_wcnt[w]);
  } else {
    const int kbits = 32 - __clz((uint32_t)(np * B) - 1u);  // bits of the largest key
#pragma unroll
    for (int it = 0; it < kSpItems; ++it) {
      const uint32_t kk = key[it];
      const bool valid = kk != kNoKey;
      const uint64_t m = same_digit_lanes<8>(kk, kbits, __ballot(valid));
      uint32_t pre = 0;
      if (valid) pre = s_wcnt[w][kk & 0xFF];
      __builtin_amdgcn_wave_barrier();
      const uint32_t before = lanes_below(m);
      if (valid && before == 0) s_wcnt[w][kk & 0xFF] = pre + popc64(m);
      __builtin_amdgcn_wave_barrier();
      rank[it] = pre + before;
    }
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
    if (kk == kNoKey) continue;
    if (kk >= (uint32_t)(np * B)) {  // not reached: a key of this tile
      atomicOr(J.status, kStatusSplit);
      continue;
    }
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
                        uint32_t* carry, void* keys, hipStream_t st) {
  if (J.n <= 0 || J.k < 2 || J.k > kMaxK) return hipSuccess;
  const int tiles = (int)level_tiles(J.n);
  const Bufs Bf{rec0, rows, b1, b2};
#define KD_SP(WW)                                                                              \
  do {                                                                                         \
    hipLaunchKernelGGL(k_split_count<WW>, dim3(tiles), dim3(kSpThreads), 0, st, Bf, J, info,  \
                       tval, tflag, tiles, static_cast<uint32_t*>(keys));                      \
    hipLaunchKernelGGL(k_split_scan, dim3(1 << (J.k - 1)), dim3(1024), 0, st, J, tval, tflag, \
                       carry, tiles);                                                          \
    hipLaunchKernelGGL(k_split_move<WW>, dim3(xcd_grid(tiles)), dim3(kSpThreads), 0, st, Bf, J, \
                       info, tflag, carry, tiles, static_cast<const uint32_t*>(keys));         \
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
