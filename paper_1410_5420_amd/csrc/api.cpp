// Host orchestration and C ABI of the k-d tree builder (see include/kdtree.h).
//
// A build is a fixed sequence of kernel launches on the caller's stream with
// no host synchronisation: the number of distinct rows stays on the device,
// and every launch sized by n (a bound on it) lets surplus workgroups exit.
// The whole sequence can therefore be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "../../include/kdtree.h"
#include "common.hpp"
#include "launch.hpp"

namespace kd {
namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout for n rows in k dimensions.  Everything from `hist` to the
// end is cleared at the start of every build.
struct Layout {
  size_t keys, rka, rkb, rva, rvb, S, rank, rec0, rec1;
  size_t hist, rlb0, rlb1, dlb0, dlb1, llb0, llb1, counters, nu, end;
};

Layout plan(int64_t n, int k) {
  Layout L{};
  const size_t un = (size_t)(n > 0 ? n : 1);
  const size_t tiles = (un + kSortTile - 1) / kSortTile;
  const size_t ltiles = (un + kLevelTile - 1) / kLevelTile;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.keys = take(4 * un * k);
  L.rka = take(4 * un);
  L.rkb = take(4 * un);
  L.rva = take(4 * un);
  L.rvb = take(4 * un);
  L.S = take(4 * un * k);
  L.rank = take(4 * un * k);
  L.rec0 = take(4 * un * k * k);
  L.rec1 = take(4 * un * k * k);
  L.hist = take(4 * (size_t)kPassesPerWord * kRadix * 2 * k);
  L.rlb0 = take(4 * tiles * kRadix);
  L.rlb1 = take(4 * tiles * kRadix);
  L.dlb0 = take(4 * tiles);
  L.dlb1 = take(4 * tiles);
  L.llb0 = take(8 * ltiles * (k > 1 ? k - 1 : 1));
  L.llb1 = take(8 * ltiles * (k > 1 ? k - 1 : 1));
  L.counters = take(4 * 8);
  L.nu = take(8);
  L.end = o;
  return L;
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

int check_common(const void* tuples, int64_t n, int32_t k, int32_t dtype, void* ws,
                 size_t ws_bytes, const kd_options* opts, int64_t* cutover) {
  if (n < 0 || k < 1 || (dtype != KD_I32 && dtype != KD_F32)) return KD_EINVAL;
  if (n > KD_MAX_N || k > KD_MAX_K) return KD_EUNSUPPORTED;
  if ((n > 0 && !tuples) || !ws) return KD_EINVAL;
  if (!aligned4(tuples) || !aligned4(ws)) return KD_EINVAL;
  if (ws_bytes < plan(n, k).end) return KD_ENOMEM;
  *cutover = 2048;
  if (opts) {
    for (int i = 0; i < 7; ++i)
      if (opts->reserved[i] != 0) return KD_EINVAL;
    if (opts->cutover != 0) {
      if (opts->cutover != 1024 && opts->cutover != 2048 && opts->cutover != 4096)
        return KD_EINVAL;
      *cutover = opts->cutover;
    }
  }
  return KD_OK;
}

#define KD_TRY(expr)                         \
  do {                                       \
    if ((expr) != hipSuccess) return KD_EHIP; \
  } while (0)

// ---- kernel probe (diagnostics) ---------------------------------------------
struct Probe {
  int cls = 0;
  int capacity = 0;
  int count = 0;
  std::vector<hipEvent_t> begin, end;
};
Probe g_probe;

void probe_begin(int cls, hipStream_t st) {
  if (g_probe.cls == cls && g_probe.count < g_probe.capacity)
    (void)hipEventRecord(g_probe.begin[g_probe.count], st);
}
void probe_end(int cls, hipStream_t st) {
  if (g_probe.cls == cls && g_probe.count < g_probe.capacity)
    (void)hipEventRecord(g_probe.end[g_probe.count++], st);
}

// launch `expr` (a hipError_t expression) bracketed by the probe for class `cls`
#define KD_LAUNCH(cls, expr)      \
  do {                            \
    probe_begin((cls), st);       \
    hipError_t e__ = (expr);      \
    probe_end((cls), st);         \
    if (e__ != hipSuccess) return KD_EHIP; \
  } while (0)

int presort_impl(const void* tuples, int64_t n, int k, int dtype, void* ws, hipStream_t st) {
  const Layout L = plan(n, k);
  uint32_t* keys = at<uint32_t>(ws, L.keys);
  uint32_t* kbuf[2] = {at<uint32_t>(ws, L.rka), at<uint32_t>(ws, L.rkb)};
  uint32_t* vbuf[2] = {at<uint32_t>(ws, L.rva), at<uint32_t>(ws, L.rvb)};
  uint32_t* S = at<uint32_t>(ws, L.S);
  uint32_t* hist = at<uint32_t>(ws, L.hist);
  uint32_t* rlb[2] = {at<uint32_t>(ws, L.rlb0), at<uint32_t>(ws, L.rlb1)};
  uint32_t* counters = at<uint32_t>(ws, L.counters);
  int64_t* nu = at<int64_t>(ws, L.nu);
  const size_t un = (size_t)n;

  KD_TRY(launch_fill_u32(hist, 0u, (int64_t)((L.end - L.hist) / 4), st));
  if (n == 0) return KD_OK;
  KD_LAUNCH(KD_K_CANON, launch_canon(tuples, n, k, dtype == KD_F32, keys, st));

  int pass = 0;
  auto lookback = [&](int ps) {
    LookBack lb;
    lb.cur = rlb[ps & 1];
    lb.other = rlb[(ps + 1) & 1];
    lb.counter = counters + (ps & 1);
    lb.counter_other = counters + ((ps + 1) & 1);
    return lb;
  };
  constexpr int kHist = kPassesPerWord * kRadix;
  // array 0: LSD over the words of x:y:z:..., least significant word first
  int cur = 0;
  for (int w = k - 1; w >= 0; --w) {
    uint32_t* h = hist + (size_t)(k - 1 - w) * kHist;
    const uint32_t* col = keys + (size_t)w * un;
    const bool first = w == k - 1;
    // every row takes part, so the digit counts need no particular order
    KD_LAUNCH(KD_K_HIST, launch_digit_hist(col, nullptr, n, nullptr, 0, h, st));
    for (int ps = 0; ps < kPassesPerWord; ++ps) {
      const int mode = ps > 0 ? 0 : (first ? 2 : 1);
      const bool last_of_word = ps == kPassesPerWord - 1;
      uint32_t* kout = (!last_of_word || w == 0) ? kbuf[cur ^ 1] : nullptr;
      KD_LAUNCH(KD_K_ONESWEEP, launch_onesweep(mode, kbuf[cur], vbuf[cur], col, kout, vbuf[cur ^ 1], n, nullptr,
                             ps * kRadixBits, h + ps * kRadix, lookback(pass++), st));
      cur ^= 1;
    }
  }
  // Sec. 2.1 duplicate removal on the fully sorted order
  {
    LookBack lb;
    lb.cur = at<uint32_t>(ws, L.dlb0);
    lb.other = at<uint32_t>(ws, L.dlb1);
    lb.counter = counters + 2;
    lb.counter_other = counters + 3;
    KD_LAUNCH(KD_K_DEDUP, launch_dedup(vbuf[cur], kbuf[cur], keys, n, k, S, nu, lb, st));
  }
  // chain: the array for super key d is the stable sort by word d of the
  // array for super key d+1
  for (int d = k - 1; d >= 1; --d) {
    uint32_t* h = hist + (size_t)(k + (k - 1 - d)) * kHist;
    const uint32_t* col = keys + (size_t)d * un;
    const uint32_t* in = S + (size_t)((d + 1) % k) * un;
    KD_LAUNCH(KD_K_HIST, launch_digit_hist(col, in, n, nu, 1, h, st));
    int c = 0;
    for (int ps = 0; ps < kPassesPerWord; ++ps) {
      const bool last = ps == kPassesPerWord - 1;
      const int mode = ps == 0 ? 1 : 0;
      const uint32_t* vin = ps == 0 ? in : vbuf[c];
      uint32_t* vout = last ? S + (size_t)d * un : vbuf[c ^ 1];
      uint32_t* kout = last ? nullptr : kbuf[c ^ 1];
      KD_LAUNCH(KD_K_ONESWEEP, launch_onesweep(mode, kbuf[c], vin, col, kout, vout, n, nu, ps * kRadixBits,
                             h + ps * kRadix, lookback(pass++), st));
      c ^= 1;
    }
  }
  if (k > 1) {
    KD_LAUNCH(KD_K_RECORDS, launch_invert(S, n, k, nu, at<uint32_t>(ws, L.rank), st));
    KD_LAUNCH(KD_K_RECORDS, launch_records(S, at<uint32_t>(ws, L.rank), n, k, nu, at<uint32_t>(ws, L.rec0), st));
  }
  return KD_OK;
}

int partition_impl(int64_t n, int k, int32_t* perm, int32_t* lo, int32_t* hi, int64_t* n_unique,
                   void* ws, int64_t cutover, hipStream_t st) {
  const Layout L = plan(n, k);
  const int64_t* nu = at<int64_t>(ws, L.nu);
  uint32_t* S = at<uint32_t>(ws, L.S);
  uint32_t* counters = at<uint32_t>(ws, L.counters);
  if (n > 0) {
    if (k == 1) {
      KD_TRY(launch_copy_k1(S, nu, n, perm, st));
    } else {
      const uint32_t* b0 = at<uint32_t>(ws, L.rec0);
      const uint32_t* b1 = at<uint32_t>(ws, L.rec1);
      uint64_t* llb[2] = {at<uint64_t>(ws, L.llb0), at<uint64_t>(ws, L.llb1)};
      const int levels = cutover_depth(n, cutover);
      for (int d = 0; d < levels; ++d) {
        LookBack64 lb;
        lb.cur = llb[d & 1];
        lb.other = llb[(d + 1) & 1];
        lb.counter = counters + 4 + (d & 1);
        lb.counter_other = counters + 4 + ((d + 1) & 1);
        KD_LAUNCH(KD_K_LEVEL, launch_level(b0, b1, n, k, d, cutover, nu, S, perm, lb, st));
      }
      KD_LAUNCH(KD_K_LEAF, launch_leaf(b0, b1, n, k, cutover, nu, S, perm, levels, st));
    }
    if (lo && hi) KD_TRY(launch_children(nu, n, lo, hi, st));
  }
  KD_TRY(launch_store_i64(n_unique, nu, st));
  return KD_OK;
}

}  // namespace
}  // namespace kd

extern "C" {

const char* kd_strerror(int code) {
  switch (code) {
    case KD_OK: return "ok";
    case KD_EINVAL: return "invalid argument";
    case KD_ENOMEM: return "workspace too small";
    case KD_EHIP: return "HIP runtime error";
    case KD_EUNSUPPORTED: return "unsupported size (n or k beyond the limits)";
    default: return "unknown status";
  }
}

int kdtree_workspace_bytes(int64_t n, int32_t k, int32_t dtype, size_t* h_bytes) {
  if (!h_bytes || n < 0 || k < 1 || (dtype != KD_I32 && dtype != KD_F32)) return KD_EINVAL;
  if (n > KD_MAX_N || k > KD_MAX_K) return KD_EUNSUPPORTED;
  *h_bytes = kd::plan(n, k).end;
  return KD_OK;
}

int kdtree_presort(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int64_t* d_n_unique,
                   void* d_workspace, size_t workspace_bytes, const kd_options* opts,
                   void* stream) {
  int64_t cutover;
  int rc = kd::check_common(d_tuples, n, k, dtype, d_workspace, workspace_bytes, opts, &cutover);
  if (rc != KD_OK) return rc;
  if (!d_n_unique || (reinterpret_cast<uintptr_t>(d_n_unique) & 7u)) return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = kd::presort_impl(d_tuples, n, k, dtype, d_workspace, st);
  if (rc != KD_OK) return rc;
  if (kd::launch_store_i64(d_n_unique, kd::at<int64_t>(d_workspace, kd::plan(n, k).nu), st) !=
      hipSuccess)
    return KD_EHIP;
  return KD_OK;
}

int kdtree_partition(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                     int32_t* d_lo, int32_t* d_hi, int64_t* d_n_unique, void* d_workspace,
                     size_t workspace_bytes, const kd_options* opts, void* stream) {
  int64_t cutover;
  int rc = kd::check_common(d_tuples, n, k, dtype, d_workspace, workspace_bytes, opts, &cutover);
  if (rc != KD_OK) return rc;
  if (!d_n_unique || (reinterpret_cast<uintptr_t>(d_n_unique) & 7u)) return KD_EINVAL;
  if ((n > 0 && !d_perm) || !kd::aligned4(d_perm)) return KD_EINVAL;
  if ((d_lo == nullptr) != (d_hi == nullptr)) return KD_EINVAL;
  if (!kd::aligned4(d_lo) || !kd::aligned4(d_hi)) return KD_EINVAL;
  return kd::partition_impl(n, k, d_perm, d_lo, d_hi, d_n_unique, d_workspace, cutover,
                            static_cast<hipStream_t>(stream));
}

int kdtree_build(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                 int32_t* d_lo, int32_t* d_hi, int64_t* d_n_unique, void* d_workspace,
                 size_t workspace_bytes, const kd_options* opts, void* stream) {
  int64_t cutover;
  int rc = kd::check_common(d_tuples, n, k, dtype, d_workspace, workspace_bytes, opts, &cutover);
  if (rc != KD_OK) return rc;
  if (!d_n_unique || (reinterpret_cast<uintptr_t>(d_n_unique) & 7u)) return KD_EINVAL;
  if ((n > 0 && !d_perm) || !kd::aligned4(d_perm)) return KD_EINVAL;
  if ((d_lo == nullptr) != (d_hi == nullptr)) return KD_EINVAL;
  if (!kd::aligned4(d_lo) || !kd::aligned4(d_hi)) return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = kd::presort_impl(d_tuples, n, k, dtype, d_workspace, st);
  if (rc != KD_OK) return rc;
  return kd::partition_impl(n, k, d_perm, d_lo, d_hi, d_n_unique, d_workspace, cutover, st);
}

int kd_probe_start(int32_t kernel_class, int32_t capacity) {
  if (kernel_class < KD_K_ONESWEEP || kernel_class > KD_K_RECORDS || capacity < 1 ||
      capacity > (1 << 20))
    return KD_EINVAL;
  kd::Probe& p = kd::g_probe;
  p.cls = 0;
  while ((int)p.begin.size() < capacity) {
    hipEvent_t b, e;
    if (hipEventCreate(&b) != hipSuccess) return KD_EHIP;
    if (hipEventCreate(&e) != hipSuccess) return KD_EHIP;
    p.begin.push_back(b);
    p.end.push_back(e);
  }
  p.capacity = capacity;
  p.count = 0;
  p.cls = kernel_class;
  return KD_OK;
}

int kd_probe_stop(float* h_ms, int32_t* h_count) {
  kd::Probe& p = kd::g_probe;
  if (!h_ms || !h_count) return KD_EINVAL;
  const int n = p.count;
  p.cls = 0;
  for (int i = 0; i < n; ++i) {
    if (hipEventSynchronize(p.end[i]) != hipSuccess) return KD_EHIP;
    if (hipEventElapsedTime(&h_ms[i], p.begin[i], p.end[i]) != hipSuccess) return KD_EHIP;
  }
  *h_count = n;
  p.count = 0;
  return KD_OK;
}

}  // extern "C"
