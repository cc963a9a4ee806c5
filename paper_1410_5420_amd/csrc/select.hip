// The comparison builder (Sec. 3): an O(n log n) method that, at every level,
// selects each subarray's median by the level's super key afresh and
// partitions the subarray about it during the search; only the first array is
// sorted (for duplicate removal, Sec. 2.1).  No other presort, no rank records.
//
// The rows travel with their k key words (canonical, order-preserving) as
// k + 1 planes.  A global level (subarrays of more than kSelLeaf rows):
//   1. hist:  per subarray, a histogram of the top digit of word p (p = depth
//             mod k) -- the most significant digit of the super key;
//   2. pick:  the bucket that holds the median's rank (len - 1) / 2;
//   3. partition (count, chain, move): a stable 3-way split of every subarray
//             by that digit: smaller, equal (the candidates), larger;
//   4. zone:  one workgroup per subarray finishes its candidates: more digit
//             rounds over them while they are many, then a sort of the few
//             left by the super key in LDS, which puts the median at the node
//             position and the smaller and larger candidates on its sides.
// The lower zone holds every row below the median and the upper zone every
// row above it, so after step 4 the subarray is partitioned about its node.
// Subarrays of at most kSelLeaf rows are finished by one workgroup each, level
// by level: a sort of every subrange by its super key in LDS (median in the
// middle), then the subranges split.
#include "common.hpp"
#include "launch.hpp"

namespace kd {

namespace {

constexpr int kSelThreads = 512;
constexpr int kSelItems = kLevelTile / kSelThreads;  // 8
constexpr int kSelWaves = kSelThreads / kWave;
constexpr int kSelChunk = 4096;   // rows sorted in LDS at once
constexpr int kSelLeaf = 2048;    // subarrays finished on-chip
constexpr int kSelPieces = 4;     // subarrays (> kSelLeaf rows) meeting a tile
constexpr int kSelRun = 32;       // longest tie run sorted by insertion
constexpr int kSelCount = 256;    // ranges up to this many rows are ranked by counting

// Planes: 0 = row id, 1 + j = canonical word j; plane c at P + c * n.
__device__ __forceinline__ uint32_t word_of(const uint32_t* P, int64_t n, int j, int i) {
  return P[(int64_t)(1 + j) * n + i];
}

// Deepest global level of a tree of nu rows (subarrays above kSelLeaf rows).
__device__ __forceinline__ int sel_levels(int nu) { return cutover_depth(nu, kSelLeaf); }

// Range of subarray c at `depth` (one tree of nu rows).
__device__ __forceinline__ void sel_range(int nu, int depth, int c, int* s_out, int* e_out) {
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

// Subarray index at `depth` of position pos, or -1 for a shallower node.
__device__ __forceinline__ int sel_index(int pos, int nu, int depth) {
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
      return -1;
    }
  }
  return c;
}

// The subarrays meeting positions [t0, t1) at `depth` are consecutive: those
// of the first and the last position that is not a shallower node.
__device__ __forceinline__ void sel_pieces(int nu, int depth, int t0, int t1, int* c_lo, int* c_hi) {
  int c = sel_index(t0, nu, depth);
  if (c < 0) c = sel_index(t0 + 1, nu, depth);
  *c_lo = c;
  c = sel_index(t1 - 1, nu, depth);
  if (c < 0) c = sel_index(t1 - 2, nu, depth);
  *c_hi = c;
}

struct Pieces {
  int np;
  int c0;
  int s[kSelPieces], e[kSelPieces];
};

__device__ __forceinline__ Pieces load_pieces(int nu, int depth, int t0, int t1, uint32_t* status) {
  Pieces pc;
  int c_lo, c_hi;
  sel_pieces(nu, depth, t0, t1, &c_lo, &c_hi);
  pc.c0 = c_lo;
  pc.np = c_hi - c_lo + 1;
  if (pc.np < 1 || pc.np > kSelPieces) {  // not reached: subarrays hold more than kSelLeaf rows
    if (threadIdx.x == 0) atomicOr(status, kStatusSplit);
    pc.np = max(1, min(pc.np, kSelPieces));
  }
#pragma unroll
  for (int q = 0; q < kSelPieces; ++q) {
    pc.s[q] = 1;
    pc.e[q] = 0;
    if (q < pc.np) sel_range(nu, depth, c_lo + q, &pc.s[q], &pc.e[q]);
  }
  return pc;
}

__device__ __forceinline__ int piece_at(const Pieces& pc, int i) {
  int q = -1;
#pragma unroll
  for (int r = 0; r < kSelPieces; ++r)
    if (r < pc.np && i >= pc.s[r] && i <= pc.e[r]) q = r;
  return q;
}

// ---- global level: digit histogram, bucket pick ------------------------------

__global__ __launch_bounds__(kSelThreads) void k_sel_hist(const SelJob J, const uint32_t* __restrict__ P,
                                                         uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[kSelPieces][256];
  const int nu = *J.nu;
  if (J.depth >= sel_levels(nu)) return;
  const int t0 = blockIdx.x * kLevelTile;
  if (t0 >= nu) return;
  const int t1 = min(t0 + kLevelTile, nu);
  const int tid = threadIdx.x;
  const int p = J.depth % J.k;
  uint32_t w[kSelItems];
#pragma unroll
  for (int it = 0; it < kSelItems; ++it) {
    const int i = t0 + it * kSelThreads + tid;
    w[it] = i < t1 ? word_of(P, J.n, p, i) : 0u;
  }
  for (int q = tid; q < kSelPieces * 256; q += kSelThreads) (&s_h[0][0])[q] = 0;
  const Pieces pc = load_pieces(nu, J.depth, t0, t1, J.status);
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kSelItems; ++it) {
    const int i = t0 + it * kSelThreads + tid;
    if (i >= t1) continue;
    const int q = piece_at(pc, i);
    if (q >= 0) atomicAdd(&s_h[q][w[it] >> 24], 1u);
  }
  __syncthreads();
  for (int q = tid; q < pc.np * 256; q += kSelThreads) {
    const uint32_t v = s_h[q >> 8][q & 255];
    if (v) atomicAdd(&hist[(int64_t)(pc.c0 + (q >> 8)) * 256 + (q & 255)], v);
  }
}

// One wave per subarray: the bucket holding the median's rank, the counts
// below it and in it; the histogram is cleared for the next level.
__global__ __launch_bounds__(256) void k_sel_pick(const SelJob J, uint32_t* __restrict__ hist,
                                                 SelState* __restrict__ state) {
  const int nu = *J.nu;
  if (J.depth >= sel_levels(nu)) return;
  const int c = blockIdx.x * 4 + (int)(threadIdx.x / kWave);
  if (c >= (1 << J.depth)) return;
  const int lane = lane_id();
  int s, e;
  sel_range(nu, J.depth, c, &s, &e);
  const uint32_t len = (uint32_t)(e - s + 1);
  const uint32_t r = (len - 1) / 2;
  uint32_t* h = hist + (int64_t)c * 256;
  uint32_t b4[4];
  uint32_t sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    b4[q] = h[lane * 4 + q];
    sum += b4[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) h[lane * 4 + q] = 0u;
  const uint32_t inc = wave_scan_dpp(sum);
  const uint32_t exc = inc - sum;
  const bool here = exc <= r && r < inc;
  if (here) {
    uint32_t run = exc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (r >= run && r < run + b4[q]) {
        SelState st;
        st.lo = run;
        st.cnt = b4[q];
        st.digit = (uint32_t)(lane * 4 + q);
        st.rank = r;
        state[c] = st;
      }
      run += b4[q];
    }
  }
  if (__ballot(here) == 0 && lane == 0) atomicOr(J.status, kStatusSplit);  // counts do not add up
}

// ---- global level: stable 3-way partition by the picked digit --------------
// Category of a row: 0 below the bucket, 1 in it, 2 above.  The counts of a
// tile's last piece (below | in << 32) are chained along every subarray as at
// a level of the presort builder.

__device__ __forceinline__ uint32_t sel_cat(uint32_t w, uint32_t digit) {
  const uint32_t d = w >> 24;
  return d < digit ? 0u : (d == digit ? 1u : 2u);
}

__global__ __launch_bounds__(kSelThreads) void k_sel_count(const SelJob J, const uint32_t* __restrict__ P,
                                                          const SelState* __restrict__ state,
                                                          uint64_t* __restrict__ tval,
                                                          uint32_t* __restrict__ tflag) {
  __shared__ uint32_t s_c[2];
  const int nu = *J.nu;
  if (J.depth >= sel_levels(nu)) return;
  const int t = blockIdx.x;
  const int t0 = t * kLevelTile;
  if (t0 >= nu) return;
  const int t1 = min(t0 + kLevelTile, nu);
  const int tid = threadIdx.x;
  const int p = J.depth % J.k;
  uint32_t w[kSelItems];
#pragma unroll
  for (int it = 0; it < kSelItems; ++it) {
    const int i = t0 + it * kSelThreads + tid;
    w[it] = i < t1 ? word_of(P, J.n, p, i) : 0u;
  }
  if (tid < 2) s_c[tid] = 0;
  const Pieces pc = load_pieces(nu, J.depth, t0, t1, J.status);
  const uint32_t digit = state[pc.c0 + pc.np - 1].digit;
  const int ls = max(pc.s[pc.np - 1], t0), le = min(pc.e[pc.np - 1] + 1, t1);
  __syncthreads();
  uint32_t lo = 0, eq = 0;
#pragma unroll
  for (int it = 0; it < kSelItems; ++it) {
    const int i = t0 + it * kSelThreads + tid;
    if (i >= ls && i < le) {
      const uint32_t ct = sel_cat(w[it], digit);
      lo += ct == 0u;
      eq += ct == 1u;
    }
  }
  const uint32_t v = lo | (eq << 16);
  const uint32_t ws = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_dpp(v), kWave - 1);
  if (lane_id() == 0 && ws) {
    atomicAdd(&s_c[0], ws & 0xFFFFu);
    atomicAdd(&s_c[1], ws >> 16);
  }
  __syncthreads();
  if (tid == 0) {
    tval[t] = (uint64_t)s_c[0] | ((uint64_t)s_c[1] << 32);
    const bool head = pc.s[pc.np - 1] >= t0;
    const bool cont = pc.s[0] < t0;
    tflag[t] = (head ? 1u : 0u) | (cont ? 2u : 0u);
  }
}

// Segmented scan of the tile counts along every subarray (one block):
// carry[t] = counts of tile t's first subarray in the tiles before it.
__global__ __launch_bounds__(1024) void k_sel_scan(const SelJob J, const uint64_t* __restrict__ tval,
                                                  const uint32_t* __restrict__ tflag,
                                                  uint64_t* __restrict__ carry) {
  constexpr int kThreads = 1024, kWaves = kThreads / kWave;
  __shared__ uint64_t s_v[kWaves];
  __shared__ int s_h[kWaves];
  const int nu = *J.nu;
  if (J.depth >= sel_levels(nu)) return;
  const int tid = threadIdx.x;
  const int tiles = (nu + kLevelTile - 1) / kLevelTile;
  const int per = (tiles + kThreads - 1) / kThreads;
  const int c0 = min(tiles, tid * per), c1 = min(tiles, c0 + per);
  uint64_t av = 0;
  int ah = 0;
  for (int t = c0; t < c1; ++t) {
    const int h = (int)(tflag[t] & 1u);
    av = h ? tval[t] : av + tval[t];
    ah |= h;
  }
  uint64_t iv = av;
  int ih = ah;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint64_t ov = __shfl_up(iv, d, kWave);
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
    uint64_t rv = 0;
    int rh = 0;
    for (int q = 0; q < kWaves; ++q) {
      const uint64_t qv = s_v[q];
      const int qh = s_h[q];
      s_v[q] = rv;
      s_h[q] = rh;
      rv = qh ? qv : rv + qv;
      rh |= qh;
    }
  }
  __syncthreads();
  uint64_t ev = __shfl_up(iv, 1, kWave);
  int eh = __shfl_up(ih, 1, kWave);
  if (lane_id() == 0) {
    ev = 0;
    eh = 0;
  }
  if (!eh) ev += s_v[w];
  uint64_t run = ev;
  for (int t = c0; t < c1; ++t) {
    const uint32_t f = tflag[t];
    carry[t] = (f & 2u) ? run : 0ull;
    run = (f & 1u) ? tval[t] : run + tval[t];
  }
}

// Moves one tile: every row's category and its rank among the rows of its
// piece and category before it (packed wave scans: below | in << 16, within
// the tile; the carry for the first piece) give its place in the lower zone,
// the candidate zone or the upper zone of its subarray.
__global__ __launch_bounds__(kSelThreads) void k_sel_move(const SelJob J, const uint32_t* __restrict__ P,
                                                         uint32_t* __restrict__ Q,
                                                         const SelState* __restrict__ state,
                                                         const uint64_t* __restrict__ carry) {
  __shared__ uint32_t s_chunk[kSelItems * kSelWaves];
  __shared__ uint32_t s_pre[kLevelTile];
  const int nu = *J.nu;
  if (J.depth >= sel_levels(nu)) return;
  const int tiles = (nu + kLevelTile - 1) / kLevelTile;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= tiles) return;
  const int t0 = t * kLevelTile;
  const int t1 = min(t0 + kLevelTile, nu);
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int k = J.k;
  const int p = J.depth % k;
  uint32_t wp[kSelItems];
#pragma unroll
  for (int it = 0; it < kSelItems; ++it) {
    const int i = t0 + it * kSelThreads + tid;
    wp[it] = i < t1 ? word_of(P, J.n, p, i) : 0u;
  }
  const Pieces pc = load_pieces(nu, J.depth, t0, t1, J.status);
  const uint64_t cy = carry[t];
  uint32_t dig[kSelPieces], slo[kSelPieces], scnt[kSelPieces];
#pragma unroll
  for (int q = 0; q < kSelPieces; ++q) {
    dig[q] = slo[q] = scnt[q] = 0;
    if (q < pc.np) {
      const SelState st = state[pc.c0 + q];
      dig[q] = st.digit;
      slo[q] = st.lo;
      scnt[q] = st.cnt;
    }
  }
  int pq[kSelItems];
  uint32_t cat[kSelItems], within[kSelItems];
#pragma unroll
  for (int it = 0; it < kSelItems; ++it) {
    const int i = t0 + it * kSelThreads + tid;
    pq[it] = i < t1 ? piece_at(pc, i) : -1;
    uint32_t d = 0;
#pragma unroll
    for (int q = 0; q < kSelPieces; ++q)
      if (q == pq[it]) d = dig[q];
    cat[it] = pq[it] >= 0 ? sel_cat(wp[it], d) : 3u;
    const uint32_t f = cat[it] == 0u ? 1u : (cat[it] == 1u ? 0x10000u : 0u);
    const uint32_t inc = wave_scan_dpp(f);
    within[it] = inc - f;
    if (lane == kWave - 1) s_chunk[it * kSelWaves + w] = inc;
  }
  __syncthreads();
  if (w == 0) {
    const uint32_t c = s_chunk[tid];
    const uint32_t inc = wave_scan_dpp(c);
    s_chunk[tid] = inc - c;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kSelItems; ++it) {
    const int i = t0 + it * kSelThreads + tid;
    if (i < t1) s_pre[i - t0] = s_chunk[it * kSelWaves + w] + within[it];
  }
  __syncthreads();
  int dest[kSelItems];
#pragma unroll
  for (int it = 0; it < kSelItems; ++it) {
    dest[it] = -1;
    const int q = pq[it];
    if (q < 0) continue;
    const int i = t0 + it * kSelThreads + tid;
    int s = 0, e = 0;
    uint32_t lo = 0, cnt = 0;
#pragma unroll
    for (int r = 0; r < kSelPieces; ++r)
      if (r == q) {
        s = pc.s[r];
        e = pc.e[r];
        lo = slo[r];
        cnt = scnt[r];
      }
    const uint32_t pre = s_pre[i - t0];
    const uint32_t base = s >= t0 ? s_pre[s - t0] : 0u;
    int nlo = (int)(pre & 0xFFFF) - (int)(base & 0xFFFF);
    int neq = (int)(pre >> 16) - (int)(base >> 16);
    if (s < t0) {  // only the first piece starts before the tile
      nlo += (int)(cy & 0xFFFFFFFFull);
      neq += (int)(cy >> 32);
    }
    int d;
    if (cat[it] == 0u)
      d = s + nlo;
    else if (cat[it] == 1u)
      d = s + (int)lo + neq;
    else
      d = s + (int)(lo + cnt) + ((i - s) - nlo - neq);
    if (d >= s && d <= e)
      dest[it] = d;
    else  // only if the counts were inconsistent
      atomicOr(J.status, kStatusSplit);
  }
  for (int c = 0; c <= k; ++c) {
    const uint32_t* src = P + (int64_t)c * J.n;
    uint32_t* dst = Q + (int64_t)c * J.n;
#pragma unroll
    for (int it = 0; it < kSelItems; ++it) {
      const int i = t0 + it * kSelThreads + tid;
      if (dest[it] >= 0) dst[dest[it]] = src[i];
    }
  }
}

// ---- sorting a chunk of rows in LDS by (range, super key) ----------------------
// rows base .. base + N - 1 of the planes P (N <= kSelChunk), each with a
// relative range start rs[i] (equal for the rows of one range); afterwards
// every range holds its rows in super-key order (words p, p+1, ..., p+k-1;
// rows are distinct, so the order is strict) and the planes are permuted in
// place.  512 threads.

struct ChunkLds {
  uint32_t ka[kSelChunk];
  uint32_t kb[kSelChunk];
  uint16_t va[kSelChunk];
  uint16_t vb[kSelChunk];
  uint16_t rs[kSelChunk];
  uint32_t cnt[kSelWaves][256];
  uint32_t dbase[256];
  uint32_t tmp[kSelWaves + 1];
  int flag;
};

// One stable LSD pass of 8-bit digit `shift` over (ka, va) -> (kb, vb).
__device__ void chunk_pass(ChunkLds& L, int N, int shift) {
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  for (int q = tid; q < kSelWaves * 256; q += kSelThreads) (&L.cnt[0][0])[q] = 0;
  __syncthreads();
  uint32_t key[kSelItems], rank[kSelItems];
  uint16_t val[kSelItems];
#pragma unroll
  for (int j = 0; j < kSelItems; ++j) {
    const int e = w * (kWave * kSelItems) + j * kWave + lane;
    const bool valid = e < N;
    key[j] = valid ? L.ka[e] : 0u;
    val[j] = valid ? L.va[e] : (uint16_t)0;
    const uint32_t d = (key[j] >> shift) & 0xFF;
    const uint64_t m = same_digit_lanes<8>(d, 8, __ballot(valid));
    uint32_t pre = 0;
    if (valid) pre = L.cnt[w][d];
    __builtin_amdgcn_wave_barrier();
    const uint32_t before = lanes_below(m);
    if (valid && before == 0) L.cnt[w][d] = pre + popc64(m);
    __builtin_amdgcn_wave_barrier();
    rank[j] = pre + before;
  }
  __syncthreads();
  uint32_t tot = 0;
  if (tid < 256) {
#pragma unroll
    for (int q = 0; q < kSelWaves; ++q) {
      const uint32_t c = L.cnt[q][tid];
      L.cnt[q][tid] = tot;
      tot += c;
    }
  }
  uint32_t all;
  const uint32_t ex = block_exclusive_sum<kSelThreads>(tot, L.tmp, &all);
  if (tid < 256) L.dbase[tid] = ex;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSelItems; ++j) {
    const int e = w * (kWave * kSelItems) + j * kWave + lane;
    if (e < N) {
      const uint32_t d = (key[j] >> shift) & 0xFF;
      const uint32_t dst = L.dbase[d] + L.cnt[w][d] + rank[j];
      L.kb[dst] = key[j];
      L.vb[dst] = val[j];
    }
  }
  __syncthreads();
  for (int e = tid; e < N; e += kSelThreads) {
    L.ka[e] = L.kb[e];
    L.va[e] = L.vb[e];
  }
  __syncthreads();
}

// Sort by one key word: ka[e] = that word of row va[e] (the current order),
// then four passes.
__device__ void chunk_sort_word(ChunkLds& L, const uint32_t* P, int64_t n, int base, int N, int word) {
  for (int e = threadIdx.x; e < N; e += kSelThreads) L.ka[e] = word_of(P, n, word, base + L.va[e]);
  __syncthreads();
  for (int sh = 0; sh < 32; sh += 8) chunk_pass(L, N, sh);
}

// Lexicographic compare of rows a and b by words p+1, ..., p+k-1.
__device__ __forceinline__ bool rest_less(const uint32_t* P, int64_t n, int k, int p, int a, int b) {
  for (int j = 1; j < k; ++j) {
    const int wd = (p + j) % k;
    const uint32_t x = word_of(P, n, wd, a), y = word_of(P, n, wd, b);
    if (x != y) return x < y;
  }
  return false;
}

__device__ void chunk_sort(ChunkLds& L, uint32_t* P, int64_t n, int k, int p, int base, int N,
                           bool ranges, uint32_t* status) {
  const int tid = threadIdx.x;
  for (int e = tid; e < N; e += kSelThreads) L.va[e] = (uint16_t)e;
  if (tid == 0) L.flag = 0;
  __syncthreads();
  chunk_sort_word(L, P, n, base, N, p);
  if (ranges) {
    for (int e = tid; e < N; e += kSelThreads) L.ka[e] = L.rs[L.va[e]];
    __syncthreads();
    chunk_pass(L, N, 0);
    chunk_pass(L, N, 8);
  }
  // ties on word p inside a range: a run of equal (range, word p) is ordered
  // by the later words -- by insertion while runs are short, else by
  // sorting the whole chunk by every word (rare)
  for (int e = tid; e < N; e += kSelThreads) {
    const bool start = e == 0 || L.rs[L.va[e]] != L.rs[L.va[e - 1]] ||
                       word_of(P, n, p, base + L.va[e]) != word_of(P, n, p, base + L.va[e - 1]);
    if (!start) continue;
    int end = e + 1;
    while (end < N && end - e <= kSelRun && L.rs[L.va[end]] == L.rs[L.va[e]] &&
           word_of(P, n, p, base + L.va[end]) == word_of(P, n, p, base + L.va[e]))
      ++end;
    if (end - e > kSelRun) {
      atomicOr(reinterpret_cast<uint32_t*>(&L.flag), 1u);
      continue;
    }
    for (int a = e + 1; a < end; ++a) {
      const uint16_t x = L.va[a];
      int b = a - 1;
      while (b >= e && rest_less(P, n, k, p, base + x, base + L.va[b])) {
        L.va[b + 1] = L.va[b];
        --b;
      }
      L.va[b + 1] = x;
    }
  }
  __syncthreads();
  if (L.flag) {
    // long runs: LSD over every word of the super key, then the ranges
    for (int e = tid; e < N; e += kSelThreads) L.va[e] = (uint16_t)e;
    __syncthreads();
    for (int j = k - 1; j >= 0; --j) chunk_sort_word(L, P, n, base, N, (p + j) % k);
    if (ranges) {
      for (int e = tid; e < N; e += kSelThreads) L.ka[e] = L.rs[L.va[e]];
      __syncthreads();
      chunk_pass(L, N, 0);
      chunk_pass(L, N, 8);
    }
  }
  // permute the planes in place: position e takes row va[e]
  for (int c = 0; c <= k; ++c) {
    uint32_t* pl = P + (int64_t)c * n + base;
    uint32_t tmp[kSelItems];
#pragma unroll
    for (int j = 0; j < kSelItems; ++j) {
      const int e = j * kSelThreads + tid;
      tmp[j] = e < N ? pl[L.va[e]] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSelItems; ++j) {
      const int e = j * kSelThreads + tid;
      if (e < N) pl[e] = tmp[j];
    }
    __syncthreads();
  }
  (void)status;
}

// ---- ranking small ranges by counting ----------------------------------------
// Rows base .. base + N - 1 (N <= kSelChunk) in ranges: range(i) = [rs[i],
// re[i]] (relative), every range at most kSelCount rows.  A row's place in
// its range is the number of rows of the range with a smaller super key p
// (words p, p+1, ..., compared in that order; rows are distinct, so the
// ranks are a permutation of the range).  s_wp caches word p of every row;
// later words are read from the planes only on a tie.  Then the planes are
// permuted in place.
struct CountLds {
  uint32_t wp[kSelChunk];
  uint16_t dst[kSelChunk];
};

__device__ __forceinline__ bool key_less(const uint32_t* P, int64_t n, int k, int p, const uint32_t* wp,
                                         int base, int a, int b) {
  if (wp[a] != wp[b]) return wp[a] < wp[b];
  return rest_less(P, n, k, p, base + a, base + b);
}

template <int kPer>
__device__ void count_rank(CountLds& C, uint32_t* P, int64_t n, int k, int p, int base, int N,
                           const int (&rs)[kPer], const int (&re)[kPer]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int i = j * kSelThreads + tid;
    if (i < N) C.wp[i] = word_of(P, n, p, base + i);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int i = j * kSelThreads + tid;
    if (i >= N) continue;
    if (rs[j] < 0) {  // a node: stays
      C.dst[i] = (uint16_t)i;
      continue;
    }
    int r = 0;
    for (int q = rs[j]; q <= re[j]; ++q)
      if (q != i && key_less(P, n, k, p, C.wp, base, q, i)) ++r;
    C.dst[i] = (uint16_t)(rs[j] + r);
  }
  __syncthreads();
  for (int c = 0; c <= k; ++c) {
    uint32_t* pl = P + (int64_t)c * n + base;
    uint32_t tmp[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i = j * kSelThreads + tid;
      tmp[j] = i < N ? pl[i] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i = j * kSelThreads + tid;
      if (i < N) pl[C.dst[i]] = tmp[j];
    }
    __syncthreads();
  }
}

// ---- global level: finish the candidate zone of every subarray -------------

__global__ __launch_bounds__(kSelThreads) void k_sel_zone(const SelJob J, uint32_t* __restrict__ Q,
                                                         uint32_t* __restrict__ scratch,
                                                         const SelState* __restrict__ state,
                                                         int32_t* __restrict__ perm) {
  __shared__ union {
    ChunkLds L;
    CountLds C;
  } u;
  ChunkLds& L = u.L;
  __shared__ uint32_t s_h[256];
  __shared__ uint32_t s_pick[3];
  __shared__ uint32_t s_tmp[kSelWaves + 1];
  const int nu = *J.nu;
  if (J.depth >= sel_levels(nu)) return;
  const int c = blockIdx.x;
  if (c >= (1 << J.depth)) return;
  const int tid = threadIdx.x;
  const int k = J.k;
  const int p = J.depth % k;
  int s, e;
  sel_range(nu, J.depth, c, &s, &e);
  const SelState st = state[c];
  int zs = s + (int)st.lo;
  int cnt = (int)st.cnt;
  int rz = (int)st.rank - (int)st.lo;  // the median's rank among the candidates
  // more digit rounds while the candidates are many: digit q of the super
  // key (q = 0 was the global pass); a stable 3-way split of the zone into
  // the scratch planes, copied back
  for (int q = 1; cnt > kSelChunk && q < 4 * k; ++q) {
    const int wd = (p + q / 4) % k;
    const int sh = 24 - 8 * (q % 4);
    if (tid < 256) s_h[tid] = 0;
    __syncthreads();
    for (int i = tid; i < cnt; i += kSelThreads)
      atomicAdd(&s_h[(word_of(Q, J.n, wd, zs + i) >> sh) & 0xFF], 1u);
    __syncthreads();
    if (tid < kWave) {
      uint32_t b4[4], sum = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        b4[r] = s_h[tid * 4 + r];
        sum += b4[r];
      }
      const uint32_t inc = wave_scan_dpp(sum);
      uint32_t run = inc - sum;
      if (run <= (uint32_t)rz && (uint32_t)rz < inc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if ((uint32_t)rz >= run && (uint32_t)rz < run + b4[r]) {
            s_pick[0] = (uint32_t)(tid * 4 + r);
            s_pick[1] = run;
            s_pick[2] = b4[r];
          }
          run += b4[r];
        }
      }
    }
    __syncthreads();
    const uint32_t b = s_pick[0], lo = s_pick[1], in = s_pick[2];
    // stable split in chunks of kSelThreads rows: every row's category and
    // its rank among the earlier rows of that category
    uint32_t run_lo = 0, run_in = 0, run_hi = 0;
    for (int c0 = 0; c0 < cnt; c0 += kSelThreads) {
      const int i = c0 + tid;
      uint32_t ct = 3;
      if (i < cnt) {
        const uint32_t d = (word_of(Q, J.n, wd, zs + i) >> sh) & 0xFF;
        ct = d < b ? 0u : (d == b ? 1u : 2u);
      }
      uint32_t tl, tin;
      const uint32_t f = ct == 0u ? 1u : (ct == 1u ? 0x10000u : 0u);
      uint32_t tot;
      const uint32_t ex = block_exclusive_sum<kSelThreads>(f, s_tmp, &tot);
      tl = tot & 0xFFFF;
      tin = tot >> 16;
      const uint32_t elo = ex & 0xFFFF, ein = ex >> 16;
      if (i < cnt) {
        int d;
        if (ct == 0u)
          d = (int)(run_lo + elo);
        else if (ct == 1u)
          d = (int)(lo + run_in + ein);
        else
          d = (int)(lo + in + run_hi + ((uint32_t)tid - elo - ein));
        for (int pl = 0; pl <= k; ++pl)
          scratch[(int64_t)pl * J.n + zs + d] = Q[(int64_t)pl * J.n + zs + i];
      }
      const uint32_t chunk_n = (uint32_t)min(kSelThreads, cnt - c0);
      run_lo += tl;
      run_in += tin;
      run_hi += chunk_n - tl - tin;
      __syncthreads();
    }
    __syncthreads();
    for (int pl = 0; pl <= k; ++pl)
      for (int i = tid; i < cnt; i += kSelThreads)
        Q[(int64_t)pl * J.n + zs + i] = scratch[(int64_t)pl * J.n + zs + i];
    __syncthreads();
    zs += (int)lo;
    rz -= (int)lo;
    cnt = (int)in;
  }
  if (cnt > kSelChunk) {  // not reached: distinct rows differ in some digit
    if (tid == 0) atomicOr(J.status, kStatusSplit);
    return;
  }
  // the few candidates left: sorted by the super key, which puts the median
  // at rank rz of the zone, its node position (by counting when very few)
  if (cnt <= kSelCount) {
    int rs1[1] = {0}, re1[1] = {cnt - 1};
    count_rank<1>(u.C, Q, J.n, k, p, zs, cnt, rs1, re1);
  } else {
    for (int i = tid; i < cnt; i += kSelThreads) L.rs[i] = 0;
    __syncthreads();
    chunk_sort(L, Q, J.n, k, p, zs, cnt, false, J.status);
  }
  const int m = s + ((e - s) >> 1);
  if (tid == 0) {
    if (zs + rz != m) atomicOr(J.status, kStatusSplit);  // not reached: rank and shape agree
    perm[m] = (int32_t)Q[m];
  }
}

// ---- on-chip finish: every subarray of at most kSelLeaf rows -----------------

// P0 / P1: the two plane buffers; the global levels the device ran (its own
// count, which duplicate removal can make smaller than the host's) decide
// which one holds the rows.
__global__ __launch_bounds__(kSelThreads) void k_sel_leaf(const SelJob J, uint32_t* __restrict__ P0,
                                                         uint32_t* __restrict__ P1,
                                                         int32_t* __restrict__ perm,
                                                         int32_t* __restrict__ queue) {
  __shared__ union {
    ChunkLds L;
    CountLds C;
  } u;
  ChunkLds& L = u.L;
  __shared__ int s_item;
  __shared__ int s_more;
  __shared__ int s_big;
  const int nu = *J.nu;
  const int D = sel_levels(nu);
  uint32_t* Q = (D & 1) ? P1 : P0;
  const int items = nu > 0 ? (1 << D) : 0;
  const int tid = threadIdx.x;
  const int k = J.k;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= items) break;
    int s0, e0;
    sel_range(nu, D, item, &s0, &e0);
    const int N = e0 - s0 + 1;
    if (N <= 0) continue;
    // every position's range, relative to s0 (s | e << 16), or a node
    uint32_t seg[kSelItems];
#pragma unroll
    for (int j = 0; j < kSelItems; ++j) {
      const int i = j * kSelThreads + tid;
      seg[j] = i < N ? ((uint32_t)(N - 1) << 16) : 0xFFFFFFFFu;
    }
    for (int depth = D;; ++depth) {
      const int p = depth % k;
      if (tid == 0) {
        s_more = 0;
        s_big = 0;
      }
      __syncthreads();
      int rsv[kSelItems], rev[kSelItems];
#pragma unroll
      for (int j = 0; j < kSelItems; ++j) {
        const int i = j * kSelThreads + tid;
        rsv[j] = -1;
        rev[j] = -1;
        if (i >= N || seg[j] == 0xFFFFFFFFu) continue;
        rsv[j] = (int)(seg[j] & 0xFFFF);
        rev[j] = (int)(seg[j] >> 16);
        if (rev[j] > rsv[j]) s_more = 1;
        if (rev[j] - rsv[j] + 1 > kSelCount) s_big = 1;
      }
      __syncthreads();
      if (s_more && !s_big) {
        count_rank<kSelItems>(u.C, Q, J.n, k, p, s0, N, rsv, rev);
      } else if (s_more) {
#pragma unroll
        for (int j = 0; j < kSelItems; ++j) {
          const int i = j * kSelThreads + tid;
          if (i < N) L.rs[i] = (uint16_t)(rsv[j] < 0 ? i : rsv[j]);  // a node: a range of its own
        }
        __syncthreads();
        chunk_sort(L, Q, J.n, k, p, s0, N, true, J.status);
      }
      // the middle of every range is its node; the halves become ranges
      int any = 0;
#pragma unroll
      for (int j = 0; j < kSelItems; ++j) {
        const int i = j * kSelThreads + tid;
        if (i >= N || seg[j] == 0xFFFFFFFFu) continue;
        const int ss = (int)(seg[j] & 0xFFFF), ee = (int)(seg[j] >> 16);
        const int m = ss + ((ee - ss) >> 1);
        if (i == m) {
          perm[s0 + m] = (int32_t)Q[s0 + m];
          seg[j] = 0xFFFFFFFFu;
        } else if (i < m) {
          seg[j] = (uint32_t)ss | ((uint32_t)(m - 1) << 16);
          any = 1;
        } else {
          seg[j] = (uint32_t)(m + 1) | ((uint32_t)ee << 16);
          any = 1;
        }
      }
      if (!__syncthreads_or(any)) break;
    }
  }
}

// Rows and canonical words of the order-0 array: P[0][i] = S[i], P[1 + j][i]
// = word j of row S[i].
__global__ __launch_bounds__(256) void k_sel_init(const uint32_t* __restrict__ tuples, int k,
                                                 int is_float, const uint32_t* __restrict__ S,
                                                 const int32_t* __restrict__ nu, int64_t n,
                                                 uint32_t* __restrict__ P) {
  const int64_t total = *nu;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = S[i];
    P[i] = (uint32_t)r;
    for (int j = 0; j < k; ++j) P[(int64_t)(1 + j) * n + i] = canon_word(tuples[r * k + j], is_float);
  }
}

}  // namespace

int select_levels_host(int64_t n) { return cutover_depth(n, kSelLeaf); }

hipError_t launch_sel_init(const uint32_t* tuples, int k, int is_float, const uint32_t* S,
                           const int32_t* nu, int64_t n, uint32_t* P, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_sel_init, dim3((unsigned)blocks), dim3(256), 0, st, tuples, k, is_float, S, nu,
                     n, P);
  return hipGetLastError();
}

hipError_t launch_sel_level(const SelJob& J, uint32_t* P, uint32_t* Q, uint32_t* hist,
                            SelState* state, uint64_t* tval, uint32_t* tflag, uint64_t* carry,
                            int32_t* perm, hipStream_t st) {
  if (J.n <= 0 || J.k < 2 || J.depth < 0 || J.depth > 30) return hipErrorInvalidValue;
  const int tiles = (int)level_tiles(J.n);
  const int subs = 1 << J.depth;
  hipLaunchKernelGGL(k_sel_hist, dim3(tiles), dim3(kSelThreads), 0, st, J, P, hist);
  hipLaunchKernelGGL(k_sel_pick, dim3((subs + 3) / 4), dim3(256), 0, st, J, hist, state);
  hipLaunchKernelGGL(k_sel_count, dim3(tiles), dim3(kSelThreads), 0, st, J, P, state, tval, tflag);
  hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, st, J, tval, tflag, carry);
  hipLaunchKernelGGL(k_sel_move, dim3(xcd_grid(tiles)), dim3(kSelThreads), 0, st, J, P, Q, state,
                     carry);
  // the zone kernel uses the previous layout's planes as its scratch
  hipLaunchKernelGGL(k_sel_zone, dim3(subs), dim3(kSelThreads), 0, st, J, Q, P, state, perm);
  return hipGetLastError();
}

hipError_t launch_sel_leaf(const SelJob& J, uint32_t* P0, uint32_t* P1, int32_t* perm,
                           int32_t* queue, int64_t items_bound, hipStream_t st) {
  if (J.n <= 0 || J.k < 2) return hipSuccess;
  int64_t grid = 2048;
  if (items_bound < grid) grid = items_bound;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_sel_leaf, dim3((unsigned)grid), dim3(kSelThreads), 0, st, J, P0, P1, perm,
                     queue);
  return hipGetLastError();
}

}  // namespace kd
