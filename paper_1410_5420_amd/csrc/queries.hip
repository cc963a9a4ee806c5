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
    const T* __restrict__ nodes, int64_t n, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ n_nodes, const T* __restrict__ lower,
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
    int64_t out = kRows ? offsets[q] : 0;
    auto take = [&](int m) {
      if (kRows) {
        if (out < cap) rows[out] = perm[m];
        ++out;
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
        const int p = depth % K;
        const T xp = nodes[(int64_t)m * K + p];
        if (lo[p] <= xp) {
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
        if (!(hi[p] >= xp)) break;
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
      if (hi[p] >= x[p]) {
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

template <typename T, int K, int kM>
__global__ __launch_bounds__(kQThreads) void k_nearest(
    const T* __restrict__ nodes, int64_t n, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ n_nodes, const T* __restrict__ points, int64_t nq,
    int32_t m_want, int32_t* __restrict__ out_rows, unsigned long long* __restrict__ visits) {
  using D = typename DistOf<T>::type;
  const int64_t q = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
  const int nn = node_count(n_nodes, n);
  uint32_t seen = 0;
  if (q < nq) {
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
        const int32_t row = dist <= bd[kM - 1] ? perm[mid] : INT32_MAX;
        if (dist < bd[kM - 1] || (dist == bd[kM - 1] && row < br[kM - 1])) {
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

hipError_t launch_region(const void* nodes, int64_t n, int k, int is_float, const int32_t* perm,
                         const int64_t* nn, const void* lower, const void* upper, int64_t nq,
                         int32_t* counts, const int64_t* offsets, int32_t* rows, int64_t cap,
                         unsigned long long* visits, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  const bool want_rows = offsets != nullptr;
#define KD_RG_T(T, KK)                                                                          \
  do {                                                                                          \
    if (want_rows)                                                                              \
      hipLaunchKernelGGL((k_region<T, KK, true>), dim3(query_blocks(nq)), dim3(kQThreads), 0, st, \
                         static_cast<const T*>(nodes), n, perm, nn, static_cast<const T*>(lower), \
                         static_cast<const T*>(upper), nq, counts, offsets, rows, cap, visits);  \
    else                                                                                        \
      hipLaunchKernelGGL((k_region<T, KK, false>), dim3(query_blocks(nq)), dim3(kQThreads), 0, st, \
                         static_cast<const T*>(nodes), n, perm, nn, static_cast<const T*>(lower), \
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
  if (nq <= 0) return hipSuccess;
  if (m < 1 || m > kMaxNeighbors) return hipErrorInvalidValue;
#define KD_NN_M(T, KK, MM)                                                                    \
  hipLaunchKernelGGL((k_nearest<T, KK, MM>), dim3(query_blocks(nq)), dim3(kQThreads), 0, st,  \
                     static_cast<const T*>(nodes), n, perm, nn, static_cast<const T*>(points), \
                     nq, m, rows, visits)
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

}  // namespace kd
