// Searches over a built tree (the paper's Appendix: the hyper-rectangle
// region search of "Source Code for Optimized Algorithms" and the m nearest
// neighbours of "Nearest Neighbors"), batched: one query per thread.
//
// The tree is implicit in the in-order layout: the node of positions [s, e]
// is at s + (e - s) / 2 and splits on dimension depth mod k.  Its "less than"
// subtree holds super keys below the node's, so their coordinate in the split
// dimension is <= the node's; the "greater than" subtree's is >= (equal
// coordinates are possible when a later portion of the super key decides).
// Both searches prune with those non-strict bounds, so they return exactly
// what a linear scan over the nodes returns.
//
// The searches read the nodes' coordinates in tree-position order (written
// once per tree by k_gather_nodes), so a visit is one read at the node's own
// position and a subtree's nodes are contiguous; perm is read only to report
// a row.  A balanced tree of at most 2^30 nodes is at most 30 levels deep, so
// a walk's path fits in two 32-bit masks.
#include "common.hpp"
#include "launch.hpp"

namespace kd {

constexpr int kQThreads = 256;
constexpr int kQStack = 32;

// Coordinates of the node at position m.  int32: signed values; float32:
// IEEE values (a NaN compares false, -0.0 == +0.0).
template <typename T, int K>
__device__ __forceinline__ void load_point(const T* __restrict__ nodes, int m, T* x) {
#pragma unroll
  for (int d = 0; d < K; ++d) x[d] = nodes[(int64_t)m * K + d];
}

// nodes[pos][d] = tuples[perm[pos]][d] for pos < the node count (zeros for a
// perm entry that is not a row below n).
template <typename T, int K>
__global__ __launch_bounds__(256) void k_gather_nodes(const T* __restrict__ tuples, int64_t n,
                                                     const int32_t* __restrict__ perm,
                                                     const int64_t* __restrict__ n_nodes,
                                                     T* __restrict__ nodes) {
  const int64_t nn = *n_nodes < 0 ? 0 : (*n_nodes > n ? n : *n_nodes);
  for (int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < nn;
       pos += (int64_t)gridDim.x * blockDim.x) {
    const int32_t row = perm[pos];
    const bool ok = (uint64_t)row < (uint64_t)n;
#pragma unroll
    for (int d = 0; d < K; ++d) nodes[pos * K + d] = ok ? tuples[(int64_t)row * K + d] : (T)0;
  }
}

// Squared distances: exact 128-bit integers for int32 coordinates (a
// component is below 2^64, k of them below 2^67), float64 sums in dimension
// order for float32 coordinates (each difference, square and sum rounded
// once; no fused multiply-add).
template <typename T>
struct DistOf;
template <>
struct DistOf<int32_t> {
  using type = unsigned __int128;
  static constexpr type kMax = ~(type)0;
  __device__ static __forceinline__ type comp(int32_t a, int32_t b) {
    const int64_t d = (int64_t)a - (int64_t)b;
    const uint64_t u = (uint64_t)(d < 0 ? -d : d);  // < 2^32
    return (type)(u * u);
  }
};
template <>
struct DistOf<float> {
  using type = double;
  static constexpr type kMax = __builtin_huge_val();
  __device__ static __forceinline__ type comp(float a, float b) {
#pragma clang fp contract(off)
    const double d = (double)a - (double)b;
    return d * d;
  }
};

template <typename T, int K>
__device__ __forceinline__ typename DistOf<T>::type sq_dist(const T* x, const T* q) {
#pragma clang fp contract(off)
  typename DistOf<T>::type acc = 0;
#pragma unroll
  for (int d = 0; d < K; ++d) acc = acc + DistOf<T>::comp(x[d], q[d]);
  return acc;
}

// Node visits of a wave added to one counter (every lane of the wave calls
// this: the launches have no early exits).
__device__ __forceinline__ void add_visits(unsigned long long* visits, uint32_t seen) {
  uint64_t v = seen;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  if (lane_id() == 0 && v) atomicAdd(visits, (unsigned long long)v);
}

// The tree's node count, clamped to the rows.
__device__ __forceinline__ int node_count(const int64_t* n_nodes, int64_t n) {
  const int64_t v = *n_nodes;
  return (int)(v < 0 ? 0 : (v > n ? n : v));
}

// Bounding box of every subtree, stored at the subtree's node position:
// bounds[pos][d] = smallest, bounds[pos][K + d] = largest coordinate d in the
// subtree (a float subtree holding a NaN gets NaN bounds, which no test
// passes, so the search walks it).  One launch per depth, deepest first: the
// g-th subarray of `depth` (its path from the root spelled by the bits of g)
// joins its node's point with its children's boxes.
template <typename T>
__device__ __forceinline__ T bound_lo(T a, T b) {
  if constexpr (sizeof(T) == 4 && (T)0.5 != (T)0) {
    if (a != a || b != b) return a != a ? a : b;
  }
  return b < a ? b : a;
}
template <typename T>
__device__ __forceinline__ T bound_hi(T a, T b) {
  if constexpr (sizeof(T) == 4 && (T)0.5 != (T)0) {
    if (a != a || b != b) return a != a ? a : b;
  }
  return a < b ? b : a;
}

template <typename T, int K>
__global__ __launch_bounds__(256) void k_subtree_bounds(const T* __restrict__ nodes, int64_t n,
                                                       const int64_t* __restrict__ n_nodes,
                                                       int depth, T* __restrict__ bounds) {
  const int nn = node_count(n_nodes, n);
  const int64_t count = (int64_t)1 << depth;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < count;
       g += (int64_t)gridDim.x * blockDim.x) {
    int s = 0, e = nn - 1;
    for (int l = depth - 1; l >= 0 && s <= e; --l) {
      const int m = s + ((e - s) >> 1);
      if ((g >> l) & 1)
        s = m + 1;
      else
        e = m - 1;
    }
    if (s > e) continue;
    const int m = s + ((e - s) >> 1);
    T lo[K], hi[K];
#pragma unroll
    for (int d = 0; d < K; ++d) lo[d] = hi[d] = nodes[(int64_t)m * K + d];
    const int cl[2] = {s + ((m - 1 - s) >> 1), (m + 1) + ((e - m - 1) >> 1)};
    const bool has[2] = {m - 1 >= s, e >= m + 1};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (!has[c]) continue;
      const T* cb = bounds + (int64_t)cl[c] * 2 * K;
#pragma unroll
      for (int d = 0; d < K; ++d) {
        lo[d] = bound_lo(lo[d], cb[d]);
        hi[d] = bound_hi(hi[d], cb[K + d]);
      }
    }
    T* ob = bounds + (int64_t)m * 2 * K;
#pragma unroll
    for (int d = 0; d < K; ++d) {
      ob[d] = lo[d];
      ob[K + d] = hi[d];
    }
  }
}

// ---- region search ---------------------------------------------------------------
// In-order walk (lower subtree, node, upper subtree), so the rows of a query
// come out in increasing tree position.  No stack: the path from the root is
// two bit masks, dirs (bit i: the walk went to the upper child at depth i)
// and pend (bit i: the node at depth i waits for its test and its upper
// subtree).  When a subtree is done the walk climbs to the deepest pending
// node, recomputes its range from the root along dirs (arithmetic only),
// tests it and enters its upper subtree.  kRows: write the rows from
// offsets[q] (no write at or past cap); otherwise count them.
template <typename T, int K>
__device__ __forceinline__ bool in_box(const T* x, const T* lo, const T* hi) {
  bool in = true;
#pragma unroll
  for (int d = 0; d < K; ++d) in = in && lo[d] <= x[d] && x[d] <= hi[d];
  return in;
}

template <typename T, int K, bool kRows>
__global__ __launch_bounds__(kQThreads) void k_region(
    const T* __restrict__ nodes, const T* __restrict__ bounds, int64_t n,
    const int32_t* __restrict__ perm, const int64_t* __restrict__ n_nodes, const T* __restrict__ lower,
    const T* __restrict__ upper, int64_t nq, int32_t* __restrict__ counts,
    const int64_t* __restrict__ offsets, int32_t* __restrict__ rows, int64_t cap,
    unsigned long long* __restrict__ visits) {
  const int64_t q = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
  const int nn = node_count(n_nodes, n);
  uint32_t seen = 0;
  if (q < nq) {
    T lo[K], hi[K];
#pragma unroll
    for (int d = 0; d < K; ++d) {
      lo[d] = lower[q * K + d];
      hi[d] = upper[q * K + d];
    }
    int32_t found = 0;
    int64_t out_pos = kRows ? offsets[q] : 0;
    auto take = [&](int m) {
      if (kRows) {
        if (out_pos < cap) rows[out_pos] = perm[m];
        ++out_pos;
      }
      ++found;
    };
    uint32_t dirs = 0, pend = 0;
    int s = 0, e = nn - 1, depth = 0;
    for (;;) {
      // down the lower spine while the box reaches below the node
      while (s <= e) {
        const int m = s + ((e - s) >> 1);
        ++seen;
        if (bounds) {
          // a subtree outside the box is skipped, one inside it is taken whole
          const T* bb = bounds + (int64_t)m * 2 * K;
          bool out = false, inside = true;
#pragma unroll
          for (int d = 0; d < K; ++d) {
            const T bl = bb[d], bh = bb[K + d];
            out = out || hi[d] < bl || bh < lo[d];
            inside = inside && lo[d] <= bl && bh <= hi[d];
          }
          if (out) break;
          if (inside) {
            found += e - s + 1;
            if (kRows)
              for (int i = s; i <= e; ++i) {
                if (out_pos < cap) rows[out_pos] = perm[i];
                ++out_pos;
              }
            break;
          }
        }
        const int p = depth % K;
        const T xp = nodes[(int64_t)m * K + p];
        // a side is skipped only when the split value proves the box misses
        // it (a NaN split value proves nothing)
        if (!(lo[p] > xp)) {
          pend |= 1u << depth;
          dirs &= ~(1u << depth);
          e = m - 1;
          ++depth;
          continue;
        }
        // nothing below: test the node now and go up it
        T x[K];
        load_point<T, K>(nodes, m, x);
        if (in_box<T, K>(x, lo, hi)) take(m);
        if (hi[p] < xp) break;
        dirs |= 1u << depth;
        pend &= ~(1u << depth);
        s = m + 1;
        ++depth;
      }
      // climb to the deepest node still waiting
      const uint32_t wait = pend & (depth >= 32 ? ~0u : ((1u << depth) - 1u));
      if (wait == 0) break;
      const int a = 31 - __builtin_clz(wait);
      pend &= ~(1u << a);
      s = 0;
      e = nn - 1;
      for (int i = 0; i < a; ++i) {
        const int m = s + ((e - s) >> 1);
        if ((dirs >> i) & 1u)
          s = m + 1;
        else
          e = m - 1;
      }
      const int m = s + ((e - s) >> 1);
      T x[K];
      load_point<T, K>(nodes, m, x);
      if (in_box<T, K>(x, lo, hi)) take(m);
      const int p = a % K;
      dirs |= 1u << a;
      depth = a + 1;
      if (!(hi[p] < x[p])) {
        s = m + 1;  // e stays: the upper subtree of [s, e]
      } else {
        s = 1;  // nothing above
        e = 0;
      }
    }
    if (!kRows) counts[q] = found;
  }
  if (visits) add_visits(visits, seen);
}

// ---- m nearest neighbours -----------------------------------------------------------
// Depth-first, nearer child first.  As in the region walk the path is two bit
// masks: dirs (bit i: the child taken at depth i is the upper one) and pend
// (bit i: the farther child at depth i is still to be considered), plus, per
// depth, a lower bound of the squared distance to that node's splitting plane
// (rounded toward zero to float, so pruning on it is never wrong).  A farther
// child is entered only while fewer than kM candidates are held or its bound
// does not exceed the kM-th best distance.  The best kM (distance, row) pairs
// are kept sorted in registers (every index static), so ties go to the
// smaller row and the first m of them are the answer whatever the walk
// (m <= kM).
__device__ __forceinline__ float plane_bound(int32_t a, int32_t b) {
  const int64_t d = (int64_t)a - (int64_t)b;
  const uint64_t u = (uint64_t)(d < 0 ? -d : d);  // < 2^32, so u * u fits
  return __ull2float_rz(u * u);
}
__device__ __forceinline__ float plane_bound(float a, float b) {
  return __double2float_rz(DistOf<float>::comp(a, b));
}
// bound > dist, exactly, for a bound that is a non-negative float
__device__ __forceinline__ bool bound_above(float b, unsigned __int128 dist) {
  return (unsigned __int128)(uint64_t)b > dist;
}
__device__ __forceinline__ bool bound_above(float b, double dist) { return (double)b > dist; }

// kSelf: the queries are the tree's own nodes (query q is the node at
// position q < the node count), and a node is not its own neighbour.
template <typename T, int K, int kM, bool kSelf>
__global__ __launch_bounds__(kQThreads) void k_nearest(
    const T* __restrict__ nodes, int64_t n, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ n_nodes, const T* __restrict__ points, int64_t nq,
    int32_t m_want, int32_t* __restrict__ out_rows, unsigned long long* __restrict__ visits) {
  using D = typename DistOf<T>::type;
  const int64_t q = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
  const int nn = node_count(n_nodes, n);
  uint32_t seen = 0;
  if (q < nq && (!kSelf || q < nn)) {
    T qp[K];
#pragma unroll
    for (int d = 0; d < K; ++d) qp[d] = points[q * K + d];
    // best[0 .. kM-1] ascending; unused slots hold (max, INT32_MAX)
    D bd[kM];
    int32_t br[kM];
#pragma unroll
    for (int i = 0; i < kM; ++i) {
      bd[i] = DistOf<T>::kMax;
      br[i] = INT32_MAX;
    }
    int held = 0;
    float fb[kQStack];
    uint32_t dirs = 0, pend = 0;
    int s = 0, e = nn - 1, depth = 0;
    for (;;) {
      while (s <= e && depth < kQStack) {
        const int mid = s + ((e - s) >> 1);
        ++seen;
        T x[K];
        load_point<T, K>(nodes, mid, x);
        const D dist = sq_dist<T, K>(x, qp);
        // the row (the tie-break) is read only for a possible candidate
        const bool cand = dist <= bd[kM - 1] && (!kSelf || mid != q);
        const int32_t row = cand ? perm[mid] : INT32_MAX;
        if (cand && (dist < bd[kM - 1] || (dist == bd[kM - 1] && row < br[kM - 1]))) {
          // insert, keeping the list sorted (static indices only)
#pragma unroll
          for (int i = kM - 1; i >= 0; --i) {
            const int j = i > 0 ? i - 1 : 0;
            const bool here = dist < bd[i] || (dist == bd[i] && row < br[i]);
            const bool before = i > 0 && (dist < bd[j] || (dist == bd[j] && row < br[j]));
            if (here) {
              bd[i] = before ? bd[j] : dist;
              br[i] = before ? br[j] : row;
            }
          }
          held += held < kM ? 1 : 0;
        }
        const int p = depth % K;
        const bool upper_near = qp[p] > x[p];  // the query above the plane
        fb[depth] = plane_bound(qp[p], x[p]);
        pend |= 1u << depth;
        if (upper_near) {
          dirs |= 1u << depth;
          s = mid + 1;
        } else {
          dirs &= ~(1u << depth);
          e = mid - 1;
        }
        ++depth;
      }
      // climb to the deepest farther child that can still hold a better one
      bool next = false;
      for (;;) {
        const uint32_t wait = pend & (depth >= 32 ? ~0u : ((1u << depth) - 1u));
        if (wait == 0) break;
        const int a = 31 - __builtin_clz(wait);
        pend &= ~(1u << a);
        depth = a + 1;
        if (held == kM && bound_above(fb[a], bd[kM - 1])) continue;
        s = 0;
        e = nn - 1;
        for (int i = 0; i < a; ++i) {
          const int m = s + ((e - s) >> 1);
          if ((dirs >> i) & 1u)
            s = m + 1;
          else
            e = m - 1;
        }
        const int m = s + ((e - s) >> 1);
        if ((dirs >> a) & 1u) {  // the upper child was nearer: the lower one now
          e = m - 1;
          dirs &= ~(1u << a);
        } else {
          s = m + 1;
          dirs |= 1u << a;
        }
        if (s <= e) {
          next = true;
          break;
        }
      }
      if (!next) break;
    }
    int32_t* o = out_rows + q * m_want;
#pragma unroll
    for (int i = 0; i < kM; ++i)
      if (i < m_want) o[i] = i < held ? br[i] : -1;
  }
  if (visits) add_visits(visits, seen);
}

namespace {
inline unsigned query_blocks(int64_t nq) { return (unsigned)((nq + kQThreads - 1) / kQThreads); }
}  // namespace

#define KD_FOR_K(MACRO) \
  switch (k) {          \
    case 1: MACRO(1); break; \
    case 2: MACRO(2); break; \
    case 3: MACRO(3); break; \
    case 4: MACRO(4); break; \
    case 5: MACRO(5); break; \
    case 6: MACRO(6); break; \
    case 7: MACRO(7); break; \
    case 8: MACRO(8); break; \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_gather_nodes(const void* tuples, int64_t n, int k, int is_float,
                               const int32_t* perm, const int64_t* nn, void* nodes, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
#define KD_GN_T(T, KK)                                                                         \
  hipLaunchKernelGGL((k_gather_nodes<T, KK>), dim3((unsigned)blocks), dim3(256), 0, st,        \
                     static_cast<const T*>(tuples), n, perm, nn, static_cast<T*>(nodes))
#define KD_GN_I(KK) KD_GN_T(int32_t, KK)
#define KD_GN_F(KK) KD_GN_T(float, KK)
  if (is_float) {
    KD_FOR_K(KD_GN_F)
  } else {
    KD_FOR_K(KD_GN_I)
  }
#undef KD_GN_F
#undef KD_GN_I
#undef KD_GN_T
  return hipGetLastError();
}

hipError_t launch_subtree_bounds(const void* nodes, int64_t n, int k, int is_float,
                                 const int64_t* nn, void* bounds, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int top = 0;  // deepest depth with a node: floor(log2 n)
  while (((int64_t)2 << top) <= n) ++top;
  for (int depth = top; depth >= 0; --depth) {
    int64_t blocks = (((int64_t)1 << depth) + 255) / 256;
    if (blocks > 8192) blocks = 8192;
#define KD_SB_T(T, KK)                                                                          \
  hipLaunchKernelGGL((k_subtree_bounds<T, KK>), dim3((unsigned)blocks), dim3(256), 0, st,       \
                     static_cast<const T*>(nodes), n, nn, depth, static_cast<T*>(bounds))
#define KD_SB_I(KK) KD_SB_T(int32_t, KK)
#define KD_SB_F(KK) KD_SB_T(float, KK)
    if (is_float) {
      KD_FOR_K(KD_SB_F)
    } else {
      KD_FOR_K(KD_SB_I)
    }
#undef KD_SB_F
#undef KD_SB_I
#undef KD_SB_T
  }
  return hipGetLastError();
}

hipError_t launch_region(const void* nodes, const void* bounds, int64_t n, int k, int is_float,
                         const int32_t* perm, const int64_t* nn, const void* lower,
                         const void* upper, int64_t nq, int32_t* counts, const int64_t* offsets,
                         int32_t* rows, int64_t cap, unsigned long long* visits, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  const bool want_rows = offsets != nullptr;
#define KD_RG_T(T, KK)                                                                          \
  do {                                                                                          \
    if (want_rows)                                                                              \
      hipLaunchKernelGGL((k_region<T, KK, true>), dim3(query_blocks(nq)), dim3(kQThreads), 0, st, \
                         static_cast<const T*>(nodes), static_cast<const T*>(bounds), n, perm, nn, \
                         static_cast<const T*>(lower),                                          \
                         static_cast<const T*>(upper), nq, counts, offsets, rows, cap, visits);  \
    else                                                                                        \
      hipLaunchKernelGGL((k_region<T, KK, false>), dim3(query_blocks(nq)), dim3(kQThreads), 0, st, \
                         static_cast<const T*>(nodes), static_cast<const T*>(bounds), n, perm, nn, \
                         static_cast<const T*>(lower),                                          \
                         static_cast<const T*>(upper), nq, counts, offsets, rows, cap, visits);  \
  } while (0)
#define KD_RG_I(KK) KD_RG_T(int32_t, KK)
#define KD_RG_F(KK) KD_RG_T(float, KK)
  if (is_float) {
    KD_FOR_K(KD_RG_F)
  } else {
    KD_FOR_K(KD_RG_I)
  }
#undef KD_RG_F
#undef KD_RG_I
#undef KD_RG_T
  return hipGetLastError();
}

hipError_t launch_nearest(const void* nodes, int64_t n, int k, int is_float, const int32_t* perm,
                          const int64_t* nn, const void* points, int64_t nq, int32_t m, int32_t* rows,
                          unsigned long long* visits, hipStream_t st) {
  const bool self = points == nullptr;  // every node of the tree as a query (nq = n)
  if (nq <= 0) return hipSuccess;
  if (m < 1 || m > kMaxNeighbors) return hipErrorInvalidValue;
#define KD_NN_M(T, KK, MM)                                                                    \
  do {                                                                                        \
    if (self)                                                                                 \
      hipLaunchKernelGGL((k_nearest<T, KK, MM, true>), dim3(query_blocks(nq)), dim3(kQThreads), \
                         0, st, static_cast<const T*>(nodes), n, perm, nn,                    \
                         static_cast<const T*>(nodes), nq, m, rows, visits);                  \
    else                                                                                      \
      hipLaunchKernelGGL((k_nearest<T, KK, MM, false>), dim3(query_blocks(nq)), dim3(kQThreads), \
                         0, st, static_cast<const T*>(nodes), n, perm, nn,                    \
                         static_cast<const T*>(points), nq, m, rows, visits);                 \
  } while (0)
#define KD_NN_T(T, KK)                         \
  do {                                         \
    if (m <= 1)                                \
      KD_NN_M(T, KK, 1);                       \
    else if (m <= 4)                           \
      KD_NN_M(T, KK, 4);                       \
    else if (m <= 8)                           \
      KD_NN_M(T, KK, 8);                       \
    else if (m <= 16)                          \
      KD_NN_M(T, KK, 16);                      \
    else if (m <= 32)                          \
      KD_NN_M(T, KK, 32);                      \
    else                                       \
      KD_NN_M(T, KK, kMaxNeighbors);           \
  } while (0)
#define KD_NN_I(KK) KD_NN_T(int32_t, KK)
#define KD_NN_F(KK) KD_NN_T(float, KK)
  if (is_float) {
    KD_FOR_K(KD_NN_F)
  } else {
    KD_FOR_K(KD_NN_I)
  }
#undef KD_NN_F
#undef KD_NN_I
#undef KD_NN_T
#undef KD_NN_M
  return hipGetLastError();
}

#undef KD_FOR_K


// ---- reverse nearest neighbours ---------------------------------------------------
// From every node's m nearest (rows[pos * m + i], -1 past the count), the
// reverse list of every row r: the rows of the nodes that have r among their
// m nearest, as compressed lists (offsets over row ids 0 .. n-1), each in
// ascending row order.  Counts, a scan of the counts, a fill that claims list
// slots with atomics, then a sort of every list (they are short: m on
// average), so the output does not depend on the order of the atomics.
constexpr int kRevChunk = 4096;  // rows per scan block (256 threads x 16)

__global__ __launch_bounds__(256) void k_rev_count(const int32_t* __restrict__ rows, int64_t n,
                                                  const int64_t* __restrict__ n_nodes, int m,
                                                  uint32_t* __restrict__ cnt) {
  const int64_t total = (int64_t)node_count(n_nodes, n) * m;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = rows[i];
    if ((uint64_t)r < (uint64_t)n) atomicAdd(&cnt[r], 1u);
  }
}

// per-chunk sums of the counts
__global__ __launch_bounds__(256) void k_rev_sums(const uint32_t* __restrict__ cnt, int64_t n,
                                                 uint64_t* __restrict__ sums) {
  __shared__ uint64_t s_tmp[256 / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kRevChunk;
  uint64_t v = 0;
  for (int i = threadIdx.x; i < kRevChunk; i += 256)
    if (base + i < n) v += cnt[base + i];
  uint64_t all;
  block_exclusive_sum<256>(v, s_tmp, &all);
  if (threadIdx.x == 0) sums[blockIdx.x] = all;
}

// one block: exclusive scan of the chunk sums, in place
__global__ __launch_bounds__(1024) void k_rev_scan_sums(uint64_t* __restrict__ sums, int64_t nb) {
  __shared__ uint64_t s_tmp[1024 / kWave + 1];
  __shared__ uint64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t b = b0 + threadIdx.x;
    const uint64_t v = b < nb ? sums[b] : 0;
    uint64_t all;
    const uint64_t ex = block_exclusive_sum<1024>(v, s_tmp, &all);
    const uint64_t carry = s_carry;
    if (b < nb) sums[b] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + all;
    __syncthreads();
  }
}

// offsets[r] = chunk start + the counts before r in its chunk; offsets[n] =
// the total.  Each thread owns 16 consecutive rows of the chunk.
__global__ __launch_bounds__(256) void k_rev_offsets(const uint32_t* __restrict__ cnt, int64_t n,
                                                    const uint64_t* __restrict__ sums,
                                                    int64_t* __restrict__ offsets) {
  __shared__ uint64_t s_tmp[256 / kWave + 1];
  constexpr int kPer = kRevChunk / 256;
  const int64_t r0 = (int64_t)blockIdx.x * kRevChunk + (int64_t)threadIdx.x * kPer;
  uint32_t c[kPer];
  uint64_t v = 0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    c[j] = r0 + j < n ? cnt[r0 + j] : 0u;
    v += c[j];
  }
  uint64_t all;
  uint64_t run = sums[blockIdx.x] + block_exclusive_sum<256>(v, s_tmp, &all);
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (r0 + j < n) offsets[r0 + j] = (int64_t)run;
    run += c[j];
  }
  if (r0 < n && r0 + kPer >= n) offsets[n] = (int64_t)run;  // the thread holding the last row
}

__global__ __launch_bounds__(256) void k_rev_fill(const int32_t* __restrict__ rows, int64_t n,
                                                 const int32_t* __restrict__ perm,
                                                 const int64_t* __restrict__ n_nodes, int m,
                                                 const int64_t* __restrict__ offsets,
                                                 uint32_t* __restrict__ cursor,
                                                 int32_t* __restrict__ lists) {
  const int64_t total = (int64_t)node_count(n_nodes, n) * m;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = rows[i];
    if ((uint64_t)r >= (uint64_t)n) continue;
    const uint32_t slot = atomicAdd(&cursor[r], 1u);
    const int64_t at = offsets[r] + slot;
    if (at < offsets[r + 1]) lists[at] = perm[i / m];  // the querying node's row
  }
}

// every list in ascending order, by one thread: insertion sort for the usual
// short lists, heapsort (L log L at worst) once a list is longer than 32 (a
// row that is among the nearest of very many nodes has a long list)
__device__ __forceinline__ void rev_sift(int32_t* __restrict__ v, int64_t i, int64_t len) {
  for (;;) {
    const int64_t l = 2 * i + 1;
    if (l >= len) return;
    int64_t c = l;
    if (l + 1 < len && v[l + 1] > v[l]) c = l + 1;
    if (!(v[c] > v[i])) return;
    const int32_t t = v[i];
    v[i] = v[c];
    v[c] = t;
    i = c;
  }
}

__global__ __launch_bounds__(256) void k_rev_sort(int64_t n, const int64_t* __restrict__ offsets,
                                                 int32_t* __restrict__ lists) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = offsets[r], len = offsets[r + 1] - a;
    int32_t* v = lists + a;
    if (len <= 32) {
      for (int64_t i = 1; i < len; ++i) {
        const int32_t x = v[i];
        int64_t j = i - 1;
        while (j >= 0 && v[j] > x) {
          v[j + 1] = v[j];
          --j;
        }
        v[j + 1] = x;
      }
      continue;
    }
    for (int64_t i = len / 2 - 1; i >= 0; --i) rev_sift(v, i, len);
    for (int64_t end = len - 1; end > 0; --end) {
      const int32_t t = v[0];
      v[0] = v[end];
      v[end] = t;
      rev_sift(v, 0, end);
    }
  }
}

size_t reverse_workspace_bytes(int64_t n) {
  const int64_t nb = (n + kRevChunk - 1) / kRevChunk;
  return (size_t)(4 * n + 255) / 256 * 256 + (size_t)8 * (nb > 0 ? nb : 1);
}

hipError_t launch_reverse_nearest(const int32_t* perm, const int64_t* nn, int64_t n, int m,
                                  const int32_t* rows, int64_t* offsets, int32_t* lists, void* ws,
                                  hipStream_t st) {
  if (n <= 0) return hipSuccess;
  uint32_t* cnt = static_cast<uint32_t*>(ws);
  uint64_t* sums = reinterpret_cast<uint64_t*>(static_cast<char*>(ws) + (4 * n + 255) / 256 * 256);
  const int64_t nb = (n + kRevChunk - 1) / kRevChunk;
  int64_t g = (n * m + 255) / 256;
  if (g > 16384) g = 16384;
  int64_t gs = (n + 255) / 256;
  if (gs > 16384) gs = 16384;
  hipError_t e = launch_fill_u32(cnt, 0u, n, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rev_count, dim3((unsigned)g), dim3(256), 0, st, rows, n, nn, m, cnt);
  hipLaunchKernelGGL(k_rev_sums, dim3((unsigned)nb), dim3(256), 0, st, cnt, n, sums);
  hipLaunchKernelGGL(k_rev_scan_sums, dim3(1), dim3(1024), 0, st, sums, nb);
  hipLaunchKernelGGL(k_rev_offsets, dim3((unsigned)nb), dim3(256), 0, st, cnt, n, sums, offsets);
  e = launch_fill_u32(cnt, 0u, n, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rev_fill, dim3((unsigned)g), dim3(256), 0, st, rows, n, perm, nn, m, offsets,
                     cnt, lists);
  hipLaunchKernelGGL(k_rev_sort, dim3((unsigned)gs), dim3(256), 0, st, n, offsets, lists);
  return hipGetLastError();
}

}  // namespace kd
