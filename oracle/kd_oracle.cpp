// CPU oracle for the presorting balanced k-d tree build
// (R. A. Brown, "Building a Balanced k-d Tree in O(kn log n) Time").
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
// calls this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark load it.  It shares no code, header, table or helper
// with the HIP path.
//
// It is deliberately plain: top-down merge sorts with a super-key comparator,
// a one-pass duplicate removal per index array and the recursive partition
// with the cyclic index-array rotation, all in the order the paper gives
// them.  Every function names the passage it follows.
//
// Readings of points the paper leaves open (each is exercised by a test):
//   * median of an even-sized subarray: the lower one, m = s + (e - s) / 2
//     (the two-element rule of Sec. 3.1 makes the first element the node);
//   * which duplicate survives: the first of each run in the stable sort
//     order, i.e. the smallest input row;
//   * sorts are stable, so identical tuples stay in row order;
//   * int32 coordinates compare as signed integers;
//   * float32 coordinates compare under the IEEE-754 totalOrder relation
//     (-0.0 < +0.0, NaN ordered by its bits); duplicates are bit-identical
//     rows;
//   * split dimension at depth L is L mod k and the super key that starts at
//     dimension p is p : p+1 : ... : p+k-1 (mod k).
#include <cstdint>
#include <cstring>
#include <chrono>
#include <thread>
#include <vector>

namespace {

enum { DT_I32 = 0, DT_F32 = 1 };

// One coordinate turned into a signed 64-bit integer with the same order.
// int32: the value.  float32: IEEE totalOrder, obtained by reversing the
// magnitude bits of negative encodings so that larger-magnitude negatives sort
// lower (IEEE 754-2008 Sec. 5.10).
struct Tuples {
  const void* data;
  int64_t n;
  int k;
  int dtype;
  inline int64_t coord(int64_t row, int d) const {
    int32_t raw;
    std::memcpy(&raw, static_cast<const char*>(data) + 4 * (row * k + d), 4);
    if (dtype == DT_F32 && raw < 0) raw ^= 0x7FFFFFFF;
    return static_cast<int64_t>(raw);
  }
};

// Super-key comparison (Sec. 2.1; Appendix "Optimized Super Key Comparison"):
// compare the most significant portion (dimension p) first and only enter the
// loop over the remaining portions p+1, ..., p+k-1 (mod k) when it ties.
inline int super_key_compare(const Tuples& T, int64_t a, int64_t b, int p) {
  int64_t va = T.coord(a, p), vb = T.coord(b, p);
  if (va != vb) return va < vb ? -1 : 1;
  for (int i = 1; i < T.k; ++i) {
    int d = (p + i) % T.k;
    va = T.coord(a, d);
    vb = T.coord(b, d);
    if (va != vb) return va < vb ? -1 : 1;
  }
  return 0;
}

// Top-down merge sort of an index array by the super key that starts at p
// (Sec. 2.1 presort; Sec. 2.2 parent/child threads: the parent hands the lower
// half to a child thread while `thread_levels` allows it).  Stable: on ties
// the element from the lower half is taken first.
void merge_sort(const Tuples& T, int32_t* a, int32_t* tmp, int64_t lo, int64_t hi, int p,
                int thread_levels) {
  if (hi - lo < 2) return;
  int64_t mid = lo + (hi - lo) / 2;
  if (thread_levels > 0) {
    std::thread child(merge_sort, std::cref(T), a, tmp, lo, mid, p, thread_levels - 1);
    merge_sort(T, a, tmp, mid, hi, p, thread_levels - 1);
    child.join();
  } else {
    merge_sort(T, a, tmp, lo, mid, p, 0);
    merge_sort(T, a, tmp, mid, hi, p, 0);
  }
  int64_t i = lo, j = mid, o = lo;
  while (i < mid && j < hi) {
    if (super_key_compare(T, a[j], a[i], p) < 0)
      tmp[o++] = a[j++];
    else
      tmp[o++] = a[i++];
  }
  while (i < mid) tmp[o++] = a[i++];
  while (j < hi) tmp[o++] = a[j++];
  std::memcpy(a + lo, tmp + lo, sizeof(int32_t) * (hi - lo));
}

// Duplicate removal (Sec. 2.1): one pass through a sorted index array that
// keeps an index only when its tuple differs from the last one kept.
int64_t remove_duplicates(const Tuples& T, int32_t* a, int64_t n, int p) {
  if (n == 0) return 0;
  int64_t kept = 1;
  for (int64_t i = 1; i < n; ++i) {
    if (super_key_compare(T, a[i], a[kept - 1], p) != 0) a[kept++] = a[i];
  }
  return kept;
}

struct Builder {
  const Tuples& T;
  std::vector<int32_t*> A;  // A[0..k-1]: index arrays; A[0] is sorted in the split dimension
  int32_t* temp;
  int32_t* perm;
  int32_t* lo;
  int32_t* hi;
  int max_depth;  // < 0: build the whole tree; otherwise stop before partitioning at this depth

  // Sec. 2.1: the node of subarray [s, e] is the median of the index array
  // that is sorted by the current split dimension; the other k-1 arrays are
  // partitioned about it, keeping their order, and the median itself is
  // dropped.  The single temporary array makes the k arrays rotate by one
  // role per level, so the array that is sorted in the split dimension is
  // always A[0].  Returns the position of the node, or -1 for an empty range.
  int64_t build(int64_t s, int64_t e, int depth, int thread_levels) {
    if (e < s) return -1;
    if (max_depth >= 0 && depth >= max_depth) return -1;
    const int k = T.k;
    const int p = depth % k;
    const int64_t m = s + (e - s) / 2;
    const int32_t node = A[0][m];
    perm[m] = node;
    // Sec. 2.1: recursion ends at one, two or three elements, whose order in
    // A[0] already decides the node and its children (two elements: the first
    // is the node, the second its "greater than" child -- Sec. 3.1).
    int64_t n_here = e - s + 1;
    if (n_here <= 3 && max_depth < 0) {
      const bool kids = lo && hi;
      if (kids) lo[m] = hi[m] = -1;
      if (n_here == 2) {
        perm[s + 1] = A[0][s + 1];
        if (kids) {
          hi[m] = static_cast<int32_t>(s + 1);
          lo[s + 1] = hi[s + 1] = -1;
        }
      } else if (n_here == 3) {
        perm[s] = A[0][s];
        perm[s + 2] = A[0][s + 2];
        if (kids) {
          lo[m] = static_cast<int32_t>(s);
          hi[m] = static_cast<int32_t>(s + 2);
          lo[s] = hi[s] = lo[s + 2] = hi[s + 2] = -1;
        }
      }
      return m;
    }
    if (k > 1) {
      // Copy A[0] to the temporary array, partition A[j] into the two halves
      // of A[j-1] for j = 1..k-1, then copy the temporary array into A[k-1].
      std::memcpy(temp + s, A[0] + s, sizeof(int32_t) * n_here);
      for (int j = 1; j < k; ++j) {
        int64_t lower = s, upper = m + 1;
        for (int64_t i = s; i <= e; ++i) {
          int c = super_key_compare(T, A[j][i], node, p);
          if (c < 0)
            A[j - 1][lower++] = A[j][i];
          else if (c > 0)
            A[j - 1][upper++] = A[j][i];
          // c == 0: the median itself, which is not copied
        }
      }
      std::memcpy(A[k - 1] + s, temp + s, sizeof(int32_t) * n_here);
    }
    // With k == 1 the single array is already sorted and needs no partition.
    int64_t l, h;
    if (thread_levels > 0) {
      // Sec. 2.2: a child thread builds the lower half while the parent builds
      // the upper half.
      int64_t lres = -1;
      std::thread child([&] { lres = build(s, m - 1, depth + 1, thread_levels - 1); });
      h = build(m + 1, e, depth + 1, thread_levels - 1);
      child.join();
      l = lres;
    } else {
      l = build(s, m - 1, depth + 1, 0);
      h = build(m + 1, e, depth + 1, 0);
    }
    if (lo && hi) {
      lo[m] = static_cast<int32_t>(l);
      hi[m] = static_cast<int32_t>(h);
    }
    return m;
  }
};

int thread_levels_for(int threads) {
  // Sec. 2.2: only powers of two; q threads allow child threads at the first
  // log2(q) levels of recursion.
  int lv = 0;
  while ((2 << lv) <= threads) ++lv;
  return threads > 1 ? lv : 0;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

// Presort + duplicate removal (Sec. 2.1): fills out_arrays[d*n + i], i < n_unique,
// with the deduplicated index array sorted by the super key that starts at d.
int kdo_presort(const void* tuples, int64_t n, int32_t k, int32_t dtype, int32_t threads,
                int32_t* out_arrays, int64_t* out_nu) {
  if (n < 0 || k < 1 || (dtype != DT_I32 && dtype != DT_F32)) return -1;
  Tuples T{tuples, n, k, dtype};
  std::vector<int32_t> tmp(n > 0 ? n : 1);
  int tl = thread_levels_for(threads);
  int64_t nu = 0;
  for (int d = 0; d < k; ++d) {
    int32_t* a = out_arrays + d * n;
    for (int64_t i = 0; i < n; ++i) a[i] = static_cast<int32_t>(i);
    merge_sort(T, a, tmp.data(), 0, n, d, tl);
    int64_t u = remove_duplicates(T, a, n, d);
    if (d > 0 && u != nu) return -2;  // every array must keep the same tuples
    nu = u;
  }
  *out_nu = nu;
  return 0;
}

// Whole build (Sec. 2.1 / 2.2).  perm[pos] receives the input row of the node
// stored at in-order position pos (pos < n_unique); lo/hi (optional, may be
// NULL) the positions of its "less than" / "greater than" children or -1.
// max_depth >= 0 stops before partitioning at that depth and leaves the index
// arrays, in their rotated roles, in out_arrays (k*n, optional).
// times (optional): [0] presort + dedup seconds, [1] build seconds.
int kdo_build(const void* tuples, int64_t n, int32_t k, int32_t dtype, int32_t threads,
              int32_t max_depth, int32_t* perm, int32_t* lo, int32_t* hi, int64_t* out_nu,
              int32_t* out_arrays, double* times) {
  if (n < 0 || k < 1 || (dtype != DT_I32 && dtype != DT_F32)) return -1;
  std::vector<int32_t> arrays(static_cast<size_t>(k) * (n > 0 ? n : 1));
  double t0 = now_s();
  int64_t nu = 0;
  int rc = kdo_presort(tuples, n, k, dtype, threads, arrays.data(), &nu);
  if (rc != 0) return rc;
  double t1 = now_s();
  Tuples T{tuples, n, k, dtype};
  std::vector<int32_t> temp(n > 0 ? n : 1);
  Builder B{T, {}, temp.data(), perm, lo, hi, max_depth};
  for (int d = 0; d < k; ++d) B.A.push_back(arrays.data() + d * n);
  B.build(0, nu - 1, 0, thread_levels_for(threads));
  double t2 = now_s();
  if (out_arrays) {
    // The arrays rotate once per level: after `depth` levels the storage of
    // A[r] holds the array sorted by super key (depth + r) mod k.
    std::memcpy(out_arrays, arrays.data(), sizeof(int32_t) * k * n);
  }
  *out_nu = nu;
  if (times) {
    times[0] = t1 - t0;
    times[1] = t2 - t1;
  }
  return 0;
}

}  // extern "C"
