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
// A thread walks its query's tree with a small stack in private memory (a
// balanced tree of at most 2^30 nodes is at most 30 levels deep); the loads of
// a node's row id and coordinates are the whole memory traffic.
#include "common.hpp"
#include "launch.hpp"

namespace kd {

constexpr int kQThreads = 256;
constexpr int kQStack = 32;

// Coordinates of one row.  int32: signed values; float32: IEEE values (a NaN
// compares false, -0.0 == +0.0).
template <typename T, int K>
__device__ __forceinline__ void load_point(const T* __restrict__ tuples, int64_t row, T* x) {
#pragma unroll
  for (int d = 0; d < K; ++d) x[d] = tuples[row * K + d];
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
  __device__ static __forceinline__ type comp(int32_t a, int32_t b) {
    const int64_t d = (int64_t)a - (int64_t)b;
    const uint64_t u = (uint64_t)(d < 0 ? -d : d);  // < 2^32
    return (type)(u * u);
  }
};
template <>
struct DistOf<float> {
  using type = double;
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
// come out in increasing tree position.  The stack holds nodes whose lower
// subtree is being walked: when one is popped it is tested against the box
// and its upper subtree is entered.  kRows: write the rows from offsets[q]
// (at most cap rows in all); otherwise count them.
template <typename T, int K, bool kRows>
__global__ __launch_bounds__(kQThreads) void k_region(
    const T* __restrict__ tuples, int64_t n, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ n_nodes, const T* __restrict__ lower, const T* __restrict__ upper, int64_t nq,
    int32_t* __restrict__ counts, const int64_t* __restrict__ offsets, int32_t* __restrict__ rows,
    int64_t cap, unsigned long long* __restrict__ visits) {
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
  int32_t st_s[kQStack], st_e[kQStack], st_r[kQStack];
  uint8_t st_d[kQStack];
  int sp = 0;
  int s = 0, e = nn - 1, depth = 0;
  int32_t found = 0;
  int64_t out = kRows ? offsets[q] : 0;
  for (;;) {
    // down the lower spine while the box reaches below the node
    while (s <= e && sp < kQStack) {
      const int m = s + ((e - s) >> 1);
      const int32_t row = perm[m];
      ++seen;
      st_s[sp] = s;
      st_e[sp] = e;
      st_r[sp] = row;
      st_d[sp] = (uint8_t)depth;
      ++sp;
      if ((uint64_t)row >= (uint64_t)n) break;  // not a valid layout: skip the subtree
      const int p = depth % K;
      const T xp = tuples[(int64_t)row * K + p];
      if (!(lo[p] <= xp)) break;
      e = m - 1;
      ++depth;
    }
    if (sp == 0) break;
    --sp;
    s = st_s[sp];
    e = st_e[sp];
    depth = st_d[sp];
    const int m = s + ((e - s) >> 1);
    const int32_t row = st_r[sp];
    if ((uint64_t)row >= (uint64_t)n) {
      s = 1;
      e = 0;
      continue;
    }
    T x[K];
    load_point<T, K>(tuples, row, x);
    bool in = true;
#pragma unroll
    for (int d = 0; d < K; ++d) in = in && lo[d] <= x[d] && x[d] <= hi[d];
    if (in) {
      if (kRows) {
        if (out < cap) rows[out] = row;
        ++out;
      }
      ++found;
    }
    const int p = depth % K;
    if (hi[p] >= x[p]) {
      s = m + 1;
      ++depth;
    } else {
      s = 1;
      e = 0;
    }
  }
  if (!kRows) counts[q] = found;
  }
  if (visits) add_visits(visits, seen);
}

// ---- m nearest neighbours -----------------------------------------------------------
// Depth-first, nearer child first; the farther child is entered only while
// the heap is not full or its bound (the squared distance to the splitting
// plane) does not exceed the m-th best distance.  The heap keeps the m
// smallest (distance, row) pairs, so ties are resolved by row and the result
// does not depend on the walk.
template <typename T, int K, int kM>  // kM: heap capacity, m_want <= kM
__global__ __launch_bounds__(kQThreads) void k_nearest(
    const T* __restrict__ tuples, int64_t n, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ n_nodes, const T* __restrict__ points, int64_t nq, int32_t m_want, int32_t* __restrict__ out_rows,
    unsigned long long* __restrict__ visits) {
  using D = typename DistOf<T>::type;
  const int64_t q = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
  const int nn = node_count(n_nodes, n);
  uint32_t seen = 0;
  if (q < nq) {
  T qp[K];
#pragma unroll
  for (int d = 0; d < K; ++d) qp[d] = points[q * K + d];
  D hd[kM];
  int32_t hr[kM];
  int hn = 0;
  auto worse = [](D da, int32_t ra, D db, int32_t rb) {  // (da, ra) > (db, rb)
    return da > db || (da == db && ra > rb);
  };
  // max-heap on (distance, row)
  auto sift_down = [&](int i, int cnt) {
    for (;;) {
      const int l = 2 * i + 1;
      if (l >= cnt) break;
      int c = l;
      if (l + 1 < cnt && worse(hd[l + 1], hr[l + 1], hd[l], hr[l])) c = l + 1;
      if (!worse(hd[c], hr[c], hd[i], hr[i])) break;
      const D td = hd[i];
      const int32_t tr = hr[i];
      hd[i] = hd[c];
      hr[i] = hr[c];
      hd[c] = td;
      hr[c] = tr;
      i = c;
    }
  };
  int32_t st_s[kQStack], st_e[kQStack];
  uint8_t st_d[kQStack];
  D st_b[kQStack];
  int sp = 0;
  st_s[0] = 0;
  st_e[0] = nn - 1;
  st_d[0] = 0;
  st_b[0] = 0;
  sp = 1;
  while (sp > 0) {
    --sp;
    const int s = st_s[sp], e = st_e[sp], depth = st_d[sp];
    if (e < s) continue;
    if (hn == m_want && st_b[sp] > hd[0]) continue;
    const int mid = s + ((e - s) >> 1);
    const int32_t row = perm[mid];
    ++seen;
    if ((uint64_t)row >= (uint64_t)n) continue;  // not a valid layout: skip the subtree
    T x[K];
    load_point<T, K>(tuples, row, x);
    const D dist = sq_dist<T, K>(x, qp);
    if (hn < m_want) {
      // append and sift up
      int i = hn++;
      hd[i] = dist;
      hr[i] = row;
      while (i > 0) {
        const int pa = (i - 1) >> 1;
        if (!worse(hd[i], hr[i], hd[pa], hr[pa])) break;
        const D td = hd[i];
        const int32_t tr = hr[i];
        hd[i] = hd[pa];
        hr[i] = hr[pa];
        hd[pa] = td;
        hr[pa] = tr;
        i = pa;
      }
    } else if (worse(hd[0], hr[0], dist, row)) {
      hd[0] = dist;
      hr[0] = row;
      sift_down(0, hn);
    }
    const int p = depth % K;
    const bool lower_near = !(qp[p] > x[p]);  // the query at or below the plane
    const D bound = DistOf<T>::comp(qp[p], x[p]);
    if (sp + 2 > kQStack) continue;  // cannot happen for <= 2^30 nodes
    // farther child first on the stack, so the nearer one is walked first
    st_s[sp] = lower_near ? mid + 1 : s;
    st_e[sp] = lower_near ? e : mid - 1;
    st_d[sp] = (uint8_t)(depth + 1);
    st_b[sp] = bound;
    ++sp;
    st_s[sp] = lower_near ? s : mid + 1;
    st_e[sp] = lower_near ? mid - 1 : e;
    st_d[sp] = (uint8_t)(depth + 1);
    st_b[sp] = 0;
    ++sp;
  }
  // heap sort: ascending (distance, row)
  for (int cnt = hn; cnt > 1; --cnt) {
    const D td = hd[0];
    const int32_t tr = hr[0];
    hd[0] = hd[cnt - 1];
    hr[0] = hr[cnt - 1];
    hd[cnt - 1] = td;
    hr[cnt - 1] = tr;
    sift_down(0, cnt - 1);
  }
  int32_t* o = out_rows + q * m_want;
  for (int i = 0; i < m_want; ++i) o[i] = i < hn ? hr[i] : -1;
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

hipError_t launch_region(const void* tuples, int64_t n, int k, int is_float, const int32_t* perm,
                         const int64_t* nn, const void* lower, const void* upper, int64_t nq,
                         int32_t* counts, const int64_t* offsets, int32_t* rows, int64_t cap,
                         unsigned long long* visits, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  const bool want_rows = offsets != nullptr;
#define KD_RG_T(T, KK)                                                                          \
  do {                                                                                          \
    if (want_rows)                                                                              \
      hipLaunchKernelGGL((k_region<T, KK, true>), dim3(query_blocks(nq)), dim3(kQThreads), 0, st, \
                         static_cast<const T*>(tuples), n, perm, nn, static_cast<const T*>(lower), \
                         static_cast<const T*>(upper), nq, counts, offsets, rows, cap, visits);  \
    else                                                                                        \
      hipLaunchKernelGGL((k_region<T, KK, false>), dim3(query_blocks(nq)), dim3(kQThreads), 0, st, \
                         static_cast<const T*>(tuples), n, perm, nn, static_cast<const T*>(lower), \
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

hipError_t launch_nearest(const void* tuples, int64_t n, int k, int is_float, const int32_t* perm,
                          const int64_t* nn, const void* points, int64_t nq, int32_t m, int32_t* rows,
                          unsigned long long* visits, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  if (m < 1 || m > kMaxNeighbors) return hipErrorInvalidValue;
#define KD_NN_M(T, KK, MM)                                                                    \
  hipLaunchKernelGGL((k_nearest<T, KK, MM>), dim3(query_blocks(nq)), dim3(kQThreads), 0, st,  \
                     static_cast<const T*>(tuples), n, perm, nn, static_cast<const T*>(points), \
                     nq, m, rows, visits)
#define KD_NN_T(T, KK)                         \
  do {                                         \
    if (m <= 8)                                \
      KD_NN_M(T, KK, 8);                       \
    else if (m <= 16)                          \
      KD_NN_M(T, KK, 16);                      \
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
