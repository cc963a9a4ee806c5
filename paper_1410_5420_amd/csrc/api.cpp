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

// Workspace layout for n rows in k dimensions.  Every region is fully written
// before it is read within a build, so nothing needs clearing.
struct Layout {
  size_t vbuf, carry, S, rec0, rec1, rec2;
  size_t rcnt, rgrp, dcnt, seginfo, lcnt, lcarry, nu, end;
};

Layout plan(int64_t n, int k) {
  Layout L{};
  const int64_t nn = n > 0 ? n : 1;
  const size_t un = (size_t)nn;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.vbuf = take(4 * un * (k + 1) * 2);  // radix passes: two sets of key + k payload planes
  L.carry = take(4 * un * k);           // key words handed from one sort to the next
  L.S = take(4 * un * k);               // the k deduplicated sorted id arrays
  const size_t rw = 4 * (size_t)record_words(k, nn);
  L.rec0 = take(k > 1 ? rw : 4);        // level-0 rank records (kept)
  L.rec1 = take(k > 1 ? rw : 4);        // moved records, odd number of moves
  L.rec2 = take(k > 1 ? rw : 4);        // moved records, even number of moves
  L.rcnt = take(4 * (size_t)radix_count_words(nn));
  L.rgrp = take(4 * (size_t)radix_group_words(nn));
  L.dcnt = take(4 * (size_t)radix_tiles(nn));
  const size_t lt = (size_t)level_tiles(nn);
  L.seginfo = take(lt * level_seginfo_bytes());
  L.lcnt = take(4 * lt * 8 * (k > 1 ? k - 1 : 1));
  L.lcarry = take(8 * lt * (k > 1 ? k - 1 : 1));
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
  *cutover = 1024;
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
  uint32_t* vb = at<uint32_t>(ws, L.vbuf);
  uint32_t* carry = at<uint32_t>(ws, L.carry);
  uint32_t* S = at<uint32_t>(ws, L.S);
  uint32_t* rec0 = at<uint32_t>(ws, L.rec0);
  uint32_t* rcnt = at<uint32_t>(ws, L.rcnt);
  uint32_t* rgrp = at<uint32_t>(ws, L.rgrp);
  int64_t* nu = at<int64_t>(ws, L.nu);
  const size_t un = (size_t)n;
  // slot q of set `set`: radix pass buffers
  auto slot = [&](int set, int q) { return vb + ((size_t)set * (k + 1) + q) * un; };
  const TupleSrc ts{static_cast<const uint32_t*>(tuples), k, dtype == KD_F32 ? 1 : 0};

  if (n == 0) {
    KD_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(nu), 0u, 2, st));
    return KD_OK;
  }

  // Array 0: LSD over the words of x:y:z:..., least significant word first.
  // Slots: 0 = row id, d = word d (1 <= d < k), k = word 0.  Every pass moves
  // the sort word as its key and all other slots as payload; the first pass
  // reads the tuple rows themselves.
  auto word_slot = [&](int d) { return d == 0 ? k : d; };
  int cur = 0;
  for (int w = k - 1; w >= 0; --w) {
    for (int ps = 0; ps < kPassesPerWord; ++ps) {
      const bool from_tuples = (w == k - 1 && ps == 0);
      Payload pay{};
      int q = 0;
      for (int sl = 0; sl <= k; ++sl) {
        if (sl == word_slot(w)) continue;
        Plane& pl = pay.p[q++];
        pl.out = slot(cur ^ 1, sl);
        if (from_tuples) {
          pl.kind = sl == 0 ? kPlaneIndex : kPlaneTupleWord;
          pl.word = sl == k ? 0 : sl;
        } else {
          pl.kind = kPlaneArray;
          pl.in = slot(cur, sl);
        }
      }
      pay.count = q;
      KD_LAUNCH(KD_K_ONESWEEP,
                launch_radix_pass(from_tuples ? nullptr : slot(cur, word_slot(w)), ts, w,
                                  slot(cur ^ 1, word_slot(w)), pay, n, nullptr, ps * kRadixBits,
                                  rcnt, rgrp, st));
      cur ^= 1;
    }
  }
  // Sec. 2.1 duplicate removal on the fully sorted order; hands the words
  // w1..w_{k-1} of the kept rows to the chain
  KD_LAUNCH(KD_K_DEDUP, launch_dedup(slot(cur, k), slot(cur, 0), n, k, S, carry, (int64_t)un,
                                     at<uint32_t>(ws, L.dcnt), nu, st));
  // carry slot d-1 holds word d of the current order
  auto carried = [&](int d) { return carry + (size_t)(d - 1) * un; };
  // Chain: the array for super key d is the stable sort by word d of the
  // array for super key d+1.  Besides the row id, each sort carries the ranks
  // already known -- the input position is the rank in order d+1 -- straight
  // into array d's level-0 rank planes (plane c = rank in order d+1+c), and
  // the key words of the sorts still to come.
  for (int d = k - 1; d >= 1; --d) {
    const uint32_t* in_ids = S + (size_t)((d + 1) % k) * un;
    const uint32_t* in_rec = rec0 + record_offset((d + 1) % k, k, n);
    uint32_t* out_rec = rec0 + record_offset(d, k, n);
    const int known = k - d;  // record planes 0 .. k-d-1
    int c = 0;
    for (int ps = 0; ps < kPassesPerWord; ++ps) {
      const bool first = ps == 0, last = ps == kPassesPerWord - 1;
      Payload pay{};
      int q = 0;
      {  // slot 0: row id
        Plane& pl = pay.p[q++];
        pl.kind = kPlaneArray;
        pl.in = first ? in_ids : slot(c, 0);
        pl.out = last ? S + (size_t)d * un : slot(c ^ 1, 0);
      }
      for (int cc = 0; cc < known; ++cc) {  // slots 1 .. known: rank planes
        Plane& pl = pay.p[q++];
        if (first) {
          pl.kind = cc == 0 ? kPlaneIndex : kPlaneArray;
          pl.in = cc == 0 ? nullptr : in_rec + (size_t)(cc - 1) * un;
        } else {
          pl.kind = kPlaneArray;
          pl.in = slot(c, 1 + cc);
        }
        pl.out = last ? out_rec + (size_t)cc * un : slot(c ^ 1, 1 + cc);
      }
      for (int dd = d - 1; dd >= 1; --dd) {  // key words of the later sorts
        const int sl = known + (d - dd);
        Plane& pl = pay.p[q++];
        pl.kind = kPlaneArray;
        pl.in = first ? carried(dd) : slot(c, sl);
        pl.out = last ? carried(dd) : slot(c ^ 1, sl);
      }
      pay.count = q;
      const uint32_t* kin = first ? carried(d) : slot(c, k);
      uint32_t* kout = last ? nullptr : slot(c ^ 1, k);
      KD_LAUNCH(KD_K_ONESWEEP, launch_radix_pass(kin, ts, 0, kout, pay, n, nu, ps * kRadixBits,
                                                 rcnt, rgrp, st));
      c ^= 1;
    }
  }
  if (k > 1)
    KD_LAUNCH(KD_K_RECORDS, launch_complete_records(rec0, S + (size_t)1 * un, n, k, nu, st));
  return KD_OK;
}

int partition_impl(int64_t n, int k, int32_t* perm, int32_t* lo, int32_t* hi, int64_t* n_unique,
                   void* ws, int64_t cutover, hipStream_t st) {
  const Layout L = plan(n, k);
  const int64_t* nu = at<int64_t>(ws, L.nu);
  uint32_t* S = at<uint32_t>(ws, L.S);
  if (n > 0) {
    if (k == 1) {
      KD_TRY(launch_copy_k1(S, nu, n, perm, st));
    } else {
      // keep the on-chip finish within the 160 KiB of LDS of a workgroup
      while (cutover > 1024 && leaf_lds_bytes(cutover, k) + 8192 > 160 * 1024) cutover /= 2;
      const uint32_t* r0 = at<uint32_t>(ws, L.rec0);
      uint32_t* r1 = at<uint32_t>(ws, L.rec1);
      uint32_t* r2 = at<uint32_t>(ws, L.rec2);
      const int levels = cutover_depth(n, cutover);
      for (int d = 0; d < levels; ++d)
        KD_LAUNCH(KD_K_LEVEL, launch_level(r0, r1, r2, n, k, d, cutover, nu, perm,
                                           at<void>(ws, L.seginfo), at<uint32_t>(ws, L.lcnt),
                                           at<uint64_t>(ws, L.lcarry), st));
      KD_LAUNCH(KD_K_LEAF, launch_leaf(r0, r1, r2, n, k, cutover, nu, perm, levels, st));
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
