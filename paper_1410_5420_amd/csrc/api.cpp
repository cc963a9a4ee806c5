// Host orchestration and C ABI of the k-d tree builder (see include/kdtree.h).
//
// A build is a fixed sequence of kernel launches on the caller's stream with
// no host synchronisation: the number of distinct rows stays on the device,
// and every launch sized by n (a bound on it) lets surplus workgroups exit.
// The whole sequence can therefore be captured into a HIP graph.  A single
// build is a forest of one tree; the batched entry point builds many trees
// with the same sequence of launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/kdtree.h"
#include "common.hpp"
#include "launch.hpp"

namespace kd {
namespace {

constexpr size_t kAlign = 256;
constexpr int kStatusWords = 4;  // the status word and spare words at the workspace start

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int tree_digit_passes(int B) {
  int bits = 0;
  while (B > 1 && ((int64_t)(B - 1) >> bits) != 0) ++bits;
  return (bits + kRadixBits - 1) / kRadixBits;
}

// Workspace layout for N rows in k dimensions and B trees.  Every region is
// fully written before it is read within a build, so nothing needs clearing.
// The learned presort appends its own regions, so the regions shared with the
// plain build sit at the same offsets in both layouts.
struct Layout {
  size_t status, rsync, vbuf, carry, S, rec0, rec1, rec2;
  size_t rcnt, rgrp, dcnt, seginfo, lcnt, lcarry, lstat, ltick;
  size_t uoff, wgbase, lmax, queue, offs, ties, nodes;
  size_t med, sinfo, stval, stflag, scarry, skeys;  // level form 4
  size_t starts, flags, lkey, carry2;  // learned presort only
  size_t end;
};

constexpr int kMaxBucketBits = 16;

// Buckets of the learned presort: about 1024 keys each, at most 2^16.
int bucket_bits(int64_t n) {
  int b = 1;
  while (b < kMaxBucketBits && ((int64_t)1024 << b) < n) ++b;
  return b;
}

Layout plan(int64_t n, int k, int B, bool learned = false) {
  Layout L{};
  const int64_t nn = n > 0 ? n : 1;
  const size_t un = (size_t)nn;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.status = take(4 * kStatusWords);    // device status word, always at offset 0
  L.rsync = take(4 * (size_t)radix_sync_words(nn));  // counters of the gated radix passes
  L.vbuf = take(4 * un * (k + 2) * 2);  // radix passes: two sets of k+2 quantity slots
  L.carry = take(4 * un * (k + 1));     // key words (and tree ids) handed between sorts
  L.S = take(4 * un);                   // row ids in order 0 (the deduplicated order-0 array)
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
  L.lstat = take(8 * lt * (k > 1 ? k - 1 : 1));
  L.ltick = take(4 * kMaxLevels);
  L.uoff = take(4 * ((size_t)B + 1));
  L.wgbase = take(4 * ((size_t)B + 1));
  L.lmax = take(4);
  L.queue = take(4);
  L.offs = take(16);
  L.ties = take(4 * ((size_t)kMaxTieRuns + 2));  // run list, count, flag
  L.nodes = take(4 * ((size_t)1 << (kMaxK - 1)));  // node ranks of deferred partitioning
  // level form 4: median table (every depth above the smallest cutover),
  // per-tile pieces, bucket counts, flags and carries
  L.med = take(4 * ((size_t)2 << cutover_depth(nn, 1024)));
  L.sinfo = take(lt * split_info_bytes());
  L.stval = take(4 * (lt << (k > 1 ? k - 1 : 0)));
  L.stflag = take(4 * lt);
  L.scarry = take(4 * (lt << (k > 1 ? k - 1 : 0)));
  L.skeys = take(2 * lt * kLevelTile);  // 2 bytes per position of every tile
  if (learned) {
    L.starts = take(4 * (((size_t)1 << kMaxBucketBits) + 1));
    L.flags = take(4 * kMaxK);
    L.lkey = take(4 * un);
    L.carry2 = take(4 * un * (k + 1));
  }
  L.end = o;
  return L;
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

int check_opts(const kd_options* opts, int64_t* cutover, int* leaf_blocks, int* records,
               int* learned_sorts, int* level, int* digit_bits, int* sort_items) {
  *cutover = 1024;
  *leaf_blocks = 2048;
  *records = 0;
  *learned_sorts = 0;
  *level = 0;
  *digit_bits = 8;
  *sort_items = 8;
  if (opts) {
    if (opts->reserved[0] != 0) return KD_EINVAL;
    if (opts->digit_bits != 0 && opts->digit_bits != 8 && opts->digit_bits != 11) return KD_EINVAL;
    if (opts->digit_bits != 0) *digit_bits = opts->digit_bits;
    if (opts->sort_tile != 0 && opts->sort_tile != 4096 && opts->sort_tile != 8192) return KD_EINVAL;
    if (opts->sort_tile != 0) *sort_items = opts->sort_tile / 512;
    if (opts->level < 0 || opts->level > 4) return KD_EINVAL;
    *level = opts->level;
    if (opts->learned_sorts < 0 || opts->learned_sorts > 0xFF) return KD_EINVAL;
    *learned_sorts = opts->learned_sorts;
    if (opts->records < 0 || opts->records > 2) return KD_EINVAL;
    *records = opts->records;
    if (opts->cutover != 0) {
      if (opts->cutover != 1024 && opts->cutover != 2048 && opts->cutover != 4096)
        return KD_EINVAL;
      *cutover = opts->cutover;
    }
    if (opts->leaf_blocks != 0) {
      if (opts->leaf_blocks < 256 || opts->leaf_blocks > 16384) return KD_EINVAL;
      *leaf_blocks = opts->leaf_blocks;
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
#define KD_LAUNCH(cls, expr)                   \
  do {                                         \
    probe_begin((cls), st);                    \
    hipError_t e__ = (expr);                   \
    probe_end((cls), st);                      \
    if (e__ != hipSuccess) return KD_EHIP;     \
  } while (0)

// ---- stable multi-pass sorts ----------------------------------------------------
// A sort moves a set of quantities (row id, key words, tree id, ranks) through
// a list of radix passes, each keyed on one quantity's digit.  Between passes
// quantity i lives in slot i of one of two buffer sets; after its last use a
// quantity is dropped, and the last pass writes the survivors to their
// destinations.
struct Quant {
  int kind;             // kPlaneArray / kPlaneIndex / kPlaneTupleWord
  const uint32_t* in;   // current location (kPlaneArray)
  int word;             // tuple word (kPlaneTupleWord)
  uint32_t* dst;        // destination after the sort, or null when not needed
};

struct Pass {
  int key;       // quantity index
  int shift;     // digit
  int bits = 8;  // digit width
};

// The status word of the build being enqueued (set by every entry point that
// enqueues a build before its first launch; null outside builds).
thread_local uint32_t* t_status = nullptr;
// Its counters of the gated radix passes (cleared with the status word).
thread_local uint32_t* t_sync = nullptr;

int run_sort(std::vector<Quant>& q, const std::vector<Pass>& passes, const TupleSrc& ts, int64_t n,
             const int32_t* n_dev, uint32_t* vb, int slots, uint32_t* rcnt, uint32_t* rgrp,
             hipStream_t st, const int32_t* gate = nullptr, int items = 8) {
  RadixExtra ex;
  ex.gate = gate;
  ex.status = t_status;
  ex.sync = t_sync;
  ex.items = items;
  const size_t un = (size_t)n;
  auto slot = [&](int set, int i) { return vb + ((size_t)set * slots + i) * un; };
  const int np = (int)passes.size();
  auto needed_after = [&](int i, int p) {
    for (int p2 = p + 1; p2 < np; ++p2)
      if (passes[p2].key == i) return true;
    return q[i].dst != nullptr;
  };
  int set = 0;
  for (int p = 0; p < np; ++p) {
    const bool last = p == np - 1;
    const int kq = passes[p].key;
    const uint32_t* kin = q[kq].kind == kPlaneArray ? q[kq].in : nullptr;
    uint32_t* kout = nullptr;
    if (needed_after(kq, p)) kout = last ? q[kq].dst : slot(set ^ 1, kq);
    Payload pay{};
    int c = 0;
    std::vector<int> moved;
    for (int i = 0; i < (int)q.size(); ++i) {
      if (i == kq || q[i].kind < 0 || !needed_after(i, p)) continue;
      Plane& pl = pay.p[c++];
      pl.kind = q[i].kind;
      pl.in = q[i].in;
      pl.word = q[i].word;
      pl.out = last ? q[i].dst : slot(set ^ 1, i);
      moved.push_back(i);
    }
    pay.count = c;
    ex.bits = passes[p].bits;
    KD_LAUNCH(KD_K_ONESWEEP, launch_radix_pass(kin, ts, q[kq].word, kout, pay, n, n_dev,
                                               passes[p].shift, rcnt, rgrp, st, ex));
    for (int i = 0; i < (int)q.size(); ++i) {
      if (q[i].kind < 0) continue;
      const bool written = i == kq ? kout != nullptr
                                   : std::find(moved.begin(), moved.end(), i) != moved.end();
      if (written) {
        q[i].kind = kPlaneArray;
        q[i].in = i == kq ? kout : (last ? q[i].dst : slot(set ^ 1, i));
      } else {
        q[i].kind = -1;  // dropped
      }
    }
    set ^= 1;
  }
  return KD_OK;
}

// Learned sort of the quantities q (every one with a destination) by the
// key words sortq (least significant first), bucketed on quantity keyq under
// `model`.  Sets *flag when a bucket overflows LDS or the certificate (words
// certq most significant first, then tieq, strictly increasing) fails; the
// caller then runs the radix sort gated on the flag.
struct LearnedSort {
  const CdfModel* model;
  int nb_bits;
  int keyq;
  std::vector<int> sortq, certq;
  int tieq;
  int32_t* starts;
  int32_t* flag;
  int items = 8;  // keys per thread of the bucket passes
};

int learned_sort(std::vector<Quant> q, const LearnedSort& ls, const TupleSrc& ts, int64_t n,
                 const int32_t* n_dev, uint32_t* vb, int slots, uint32_t* rcnt, uint32_t* rgrp,
                 hipStream_t st) {
  const size_t un = (size_t)n;
  auto slot = [&](int set, int i) { return vb + ((size_t)set * slots + i) * un; };
  KD_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ls.flag), 0u, 1, st));
  RadixExtra ex;
  ex.status = t_status;
  ex.sync = t_sync;
  ex.model = ls.model;
  ex.nb_bits = ls.nb_bits;
  ex.items = ls.items;
  // bucket passes: stable, keyed by the bucket's 8-bit digits, moving everything
  const int bpasses = ls.nb_bits > kRadixBits ? 2 : 1;
  int set = 0;
  for (int p = 0; p < bpasses; ++p) {
    const Quant& kqq = q[ls.keyq];
    const uint32_t* kin = kqq.kind == kPlaneArray ? kqq.in : nullptr;
    Payload pay{};
    for (int i = 0; i < (int)q.size(); ++i) {
      if (i == ls.keyq) continue;
      Plane& pl = pay.p[pay.count++];
      pl.kind = q[i].kind;
      pl.in = q[i].in;
      pl.word = q[i].word;
      pl.out = slot(set ^ 1, i);
    }
    KD_LAUNCH(KD_K_ONESWEEP, launch_radix_pass(kin, ts, kqq.word, slot(set ^ 1, ls.keyq), pay, n,
                                               n_dev, p * kRadixBits, rcnt, rgrp, st, ex));
    for (int i = 0; i < (int)q.size(); ++i) {
      q[i].kind = kPlaneArray;
      q[i].in = slot(set ^ 1, i);
    }
    set ^= 1;
  }
  KD_TRY(launch_bucket_bounds(q[ls.keyq].in, n, n_dev, ls.model, ls.nb_bits, ls.starts, ls.flag, st));
  LocalSort lso{};
  lso.nq = (int)q.size();
  for (int i = 0; i < lso.nq; ++i) {
    lso.in[i] = q[i].in;
    lso.out[i] = q[i].dst;
  }
  lso.nkeys = (int)ls.sortq.size();
  for (int w = 0; w < lso.nkeys; ++w) lso.keyq[w] = ls.sortq[w];
  lso.model = ls.model;
  lso.nb_bits = ls.nb_bits;
  KD_LAUNCH(KD_K_BUCKET, launch_bucket_sort(ls.starts, ls.nb_bits, n, n_dev, ls.flag, lso, st));
  CertArgs ca{};
  ca.nw = (int)ls.certq.size();
  for (int w = 0; w < ca.nw; ++w) ca.w[w] = q[ls.certq[w]].dst;
  ca.tie = q[ls.tieq].dst;
  KD_TRY(launch_certify(ca, n, n_dev, ls.flag, st));
  return KD_OK;
}

// ---- the build ---------------------------------------------------------------------

struct Job {
  const void* tuples;
  int64_t n;      // rows over all trees
  int B;          // trees
  const int64_t* d_off;
  const int64_t* h_off;
  int k;
  int dtype;
  int32_t* perm;
  int32_t* lo;
  int32_t* hi;
  int64_t* n_unique;  // [B]
  void* ws;
  int64_t cutover;
  int leaf_blocks = 2048;
  int records = 0;  // 0: by size, 1: direct scatter, 2: radix pass + placement
  int learned_sorts = 0;  // learned presort: bit d = sort d uses the buckets; 0 = all
  int level = 0;          // 0/1: seg + chain + move launches per level, 2: look-back launch
  int digit_bits = 8;     // digit width of the presort's key-word passes (8 or 11)
  int sort_items = 8;     // keys per thread of every radix pass (tiles of 512 * this)
  const CdfModel* models = nullptr;  // learned presort: one model per dimension
  int32_t* fell_back = nullptr;      // learned presort: per-sort fallback flags (device)
};

ForestArgs forest_args(const Job& J, const Layout& L) {
  ForestArgs fa;
  fa.B = J.B;
  fa.off = J.d_off;
  fa.uoff = at<int32_t>(J.ws, L.uoff);
  fa.lmax = at<int32_t>(J.ws, L.lmax);
  fa.wgbase = at<int32_t>(J.ws, L.wgbase);
  fa.queue = at<int32_t>(J.ws, L.queue);
  fa.status = at<uint32_t>(J.ws, L.status);
  return fa;
}

// Up to this many rows the level-0 records are completed by one direct
// scatter; above it by radix passes plus a placement through LDS (measured
// faster from 2^24 rows on: 0.79 against 1.27 ms at 2^24, 2.6 against 9 ms
// at 2^26).
constexpr int64_t kDirectRecordsRows = (int64_t)1 << 16;

bool learned_sort_on(const Job& J, int d) {
  return J.learned_sorts == 0 || ((J.learned_sorts >> d) & 1) != 0;
}

int presort_impl(const Job& J, hipStream_t st, bool first_only = false) {
  const int64_t n = J.n;
  const int k = J.k;
  const int B = J.B;
  const bool learned = J.models != nullptr;
  const Layout L = plan(n, k, B, learned);
  void* ws = J.ws;
  uint32_t* vb = at<uint32_t>(ws, L.vbuf);
  uint32_t* carry = at<uint32_t>(ws, L.carry);
  uint32_t* S = at<uint32_t>(ws, L.S);
  uint32_t* rec0 = at<uint32_t>(ws, L.rec0);
  uint32_t* rcnt = at<uint32_t>(ws, L.rcnt);
  uint32_t* rgrp = at<uint32_t>(ws, L.rgrp);
  int32_t* uoff = at<int32_t>(ws, L.uoff);
  const size_t un = (size_t)n;
  const int slots = k + 2;
  const int tp = tree_digit_passes(B);
  const TupleSrc ts{static_cast<const uint32_t*>(J.tuples), k, J.dtype == KD_F32 ? 1 : 0};

  t_status = at<uint32_t>(ws, L.status);
  t_sync = at<uint32_t>(ws, L.rsync);
  {
    // the status word, the learned sorts' fallback flags, the tree starts
    // (empty until duplicate removal writes them) and the distinct count,
    // the tie step's run count and fallback flag, and the counters of the
    // gated radix passes
    FillList init;
    init.add(t_status, 0u, kStatusWords);
    if (learned) init.add(at<uint32_t>(ws, L.flags), 0u, k);
    init.add(reinterpret_cast<uint32_t*>(uoff), 0x7FFFFFFFu, B);
    init.add(reinterpret_cast<uint32_t*>(uoff + B), 0u, 1);
    init.add(at<uint32_t>(ws, L.ties) + kMaxTieRuns, 0u, 2);
    init.add(t_sync, 0u, (int32_t)radix_sync_words(n > 0 ? n : 1));
    KD_TRY(launch_fills(init, st));
  }
  if (n > 0) {
    // Array 0: LSD over the words of x:y:z:..., least significant word first,
    // then (several trees) the tree id, which groups the rows by tree.
    // Quantities: 0 = row id, d = word d (1 <= d < k), k = word 0, k+1 = tree.
    uint32_t* tree_in = carry + (size_t)(k - 1) * un;
    if (B > 1) KD_TRY(launch_tree_ids(J.d_off, B, tree_in, st));
    // The rows' words as planes of canonical words: carry's planes 0 .. k-2
    // take words 1 .. k-1 and its plane k word 0 (plane k-1 holds the tree
    // ids); duplicate removal overwrites them only after both sorts of
    // array 0.
    PlaneOut rp{};
    for (int d = 0; d < k; ++d) rp.p[d] = carry + (size_t)(d == 0 ? k : d - 1) * un;
    KD_LAUNCH(KD_K_CANON, launch_rows_to_planes(ts, n, rp, st));
    std::vector<Quant> q(k + 2);
    // word 0 at the chosen digit width in both sorts of array 0, the other
    // words of the complete sort at 8 bits: the two sorts then differ by
    // 4 (k - 1) passes, so they end in the same buffer set
    const int r = J.digit_bits;
    const int P0 = passes_per_word(r);
    const int fs = (P0 + 4 * (k - 1) + tp) & 1;  // buffer set holding the sorted result
    auto final_slot = [&](int i) { return vb + ((size_t)fs * slots + i) * un; };
    q[0] = Quant{kPlaneIndex, nullptr, 0, final_slot(0)};
    for (int d = 1; d < k; ++d) q[d] = Quant{kPlaneArray, rp.p[d], 0, final_slot(d)};
    q[k] = Quant{kPlaneArray, rp.p[0], 0, final_slot(k)};
    q[k + 1] = B > 1 ? Quant{kPlaneArray, tree_in, 0, final_slot(k + 1)}
                     : Quant{-1, nullptr, 0, nullptr};
    std::vector<Pass> passes;
    for (int w = k - 1; w >= 1; --w)
      for (int ps = 0; ps < kPassesPerWord; ++ps) passes.push_back({w, ps * kRadixBits, 8});
    for (int ps = 0; ps < P0; ++ps) passes.push_back({k, ps * r, r});
    for (int ps = 0; ps < tp; ++ps) passes.push_back({k + 1, ps * kRadixBits, 8});
    const int32_t* gate = nullptr;
    if (k > 1 && !(learned && learned_sort_on(J, 0))) {
      // word 0 first (then tree), then the runs of equal word 0 by the other
      // words and row; the complete sort above runs only if a run is too
      // long for the tie step
      std::vector<Pass> first;
      for (int ps = 0; ps < P0; ++ps) first.push_back({k, ps * r, r});
      for (int ps = 0; ps < tp; ++ps) first.push_back({k + 1, ps * kRadixBits, 8});
      std::vector<Quant> qf = q;
      int rc = run_sort(qf, first, ts, n, nullptr, vb, slots, rcnt, rgrp, st, nullptr,
                        J.sort_items);
      if (rc != KD_OK) return rc;
      int32_t* tl = at<int32_t>(ws, L.ties);
      int32_t* tcount = tl + kMaxTieRuns;  // count, flag (cleared above)
      TieArgs ta{final_slot(k), B > 1 ? final_slot(k + 1) : nullptr, final_slot(0), k};
      KD_LAUNCH(KD_K_TIES, launch_ties(ta, n, tl, tcount, tcount + 1, st));
      gate = tcount + 1;
    } else if (learned && learned_sort_on(J, 0)) {
      // bucket on word 0; finish by words k-1 .. 1, then word 0; ties by row
      LearnedSort ls;
      ls.model = J.models;
      ls.nb_bits = bucket_bits(n);
      ls.keyq = k;
      for (int d = k - 1; d >= 1; --d) ls.sortq.push_back(d);
      ls.sortq.push_back(k);
      ls.certq.push_back(k);
      for (int d = 1; d < k; ++d) ls.certq.push_back(d);
      ls.tieq = 0;
      ls.starts = at<int32_t>(ws, L.starts);
      ls.flag = at<int32_t>(ws, L.flags);
      ls.items = J.sort_items;
      std::vector<Quant> ql(q.begin(), q.begin() + k + 1);
      int rc = learned_sort(ql, ls, ts, n, nullptr, vb, slots, rcnt, rgrp, st);
      if (rc != KD_OK) return rc;
      gate = ls.flag;
    }
    int rc = run_sort(q, passes, ts, n, nullptr, vb, slots, rcnt, rgrp, st, gate, J.sort_items);
    if (rc != KD_OK) return rc;
    // Sec. 2.1 duplicate removal on the fully sorted order; hands the words
    // w1..w_{k-1} (and tree ids) of the kept rows to the chain
    KD_LAUNCH(KD_K_DEDUP, launch_dedup(final_slot(k), final_slot(0), B > 1 ? final_slot(k + 1) : nullptr,
                                       n, k, S, carry, (int64_t)un, B > 1 ? tree_in : nullptr,
                                       at<uint32_t>(ws, L.dcnt), uoff, B, st));
  }
  KD_TRY(launch_forest_finish(uoff, B, J.cutover, J.n_unique, at<int32_t>(ws, L.lmax),
                              at<int32_t>(ws, L.wgbase), at<int32_t>(ws, L.queue), st));
  if (n == 0 || first_only) return KD_OK;  // first_only: array 0 and the duplicate removal
  const int32_t* total = uoff + B;
  // Chain: the array for super key d is the stable sort by word d (then tree)
  // of the array for super key d+1.  Each sort carries the ranks already
  // known -- the input position is the rank in order d+1 --
  // straight into array d's level-0 rank planes (plane c = rank in order
  // d+1+c), the key words of the sorts still to come, and the tree ids.
  // The plain build rewrites the carried key words in place.  The learned
  // sort must leave its inputs intact for a fallback, so it alternates
  // between two carry buffers.
  uint32_t* cin = carry;
  uint32_t* cout = learned ? at<uint32_t>(ws, L.carry2) : carry;
  uint32_t* tree_c = carry + (size_t)(k - 1) * un;
  for (int d = k - 1; d >= 1; --d) {
    auto carried_in = [&](int dd) { return cin + (size_t)(dd - 1) * un; };
    auto carried_out = [&](int dd) { return cout + (size_t)(dd - 1) * un; };
    const uint32_t* in_rec = rec0 + record_offset((d + 1) % k, k, n);
    uint32_t* out_rec = rec0 + record_offset(d, k, n);
    const int known = k - d;  // record planes 0 .. k-d-1
    std::vector<Quant> q;  // (row ids are needed in order 0 only: none travel here)
    for (int cc = 0; cc < known; ++cc)
      q.push_back(cc == 0 ? Quant{kPlaneIndex, nullptr, 0, out_rec}
                          : Quant{kPlaneArray, in_rec + (size_t)(cc - 1) * un, 0,
                                  out_rec + (size_t)cc * un});
    for (int dd = d - 1; dd >= 1; --dd)
      q.push_back(Quant{kPlaneArray, carried_in(dd), 0, carried_out(dd)});
    const int keyq = (int)q.size();
    q.push_back(Quant{kPlaneArray, carried_in(d), 0, nullptr});
    int treeq = -1;
    if (B > 1) {
      treeq = (int)q.size();
      q.push_back(Quant{kPlaneArray, tree_c, 0, tree_c});
    }
    std::vector<Pass> passes;
    const int r = J.digit_bits;
    for (int ps = 0; ps < passes_per_word(r); ++ps) passes.push_back({keyq, ps * r, r});
    for (int ps = 0; ps < tp; ++ps) passes.push_back({treeq, ps * kRadixBits, 8});
    const int32_t* gate = nullptr;
    if (learned && learned_sort_on(J, d)) {
      // bucket on word d and finish by it; ties keep the order of array d+1,
      // whose position is the quantity-1 rank plane
      LearnedSort ls;
      ls.model = J.models + d;
      ls.nb_bits = bucket_bits(n);
      ls.keyq = keyq;
      ls.sortq.push_back(keyq);
      ls.certq.push_back(keyq);
      ls.tieq = 0;
      ls.starts = at<int32_t>(ws, L.starts);
      ls.flag = at<int32_t>(ws, L.flags) + d;
      ls.items = J.sort_items;
      std::vector<Quant> ql = q;
      ql[keyq].dst = at<uint32_t>(ws, L.lkey);
      int rc = learned_sort(ql, ls, ts, n, total, vb, slots, rcnt, rgrp, st);
      if (rc != KD_OK) return rc;
      gate = ls.flag;
    }
    int rc = run_sort(q, passes, ts, n, total, vb, slots, rcnt, rgrp, st, gate, J.sort_items);
    if (rc != KD_OK) return rc;
    if (learned) std::swap(cin, cout);
  }
  const bool direct = J.records == 1 || (J.records == 0 && n <= kDirectRecordsRows);
  if (k > 1 && direct) {
    // small: one direct scatter
    KD_LAUNCH(KD_K_RECORDS, launch_complete_records(rec0, n, k, total, st));
  } else if (k > 1) {
    // The record planes the chain could not fill (array 0's, and the ranks
    // in orders 1 .. j-1 of array j >= 2) are scattered from array 1: the
    // element at position i of array 1 has rank rv[1] = i in order 1 and
    // rv[m] = plane (m - 2) mod k of its record in the other orders.  For
    // each target array t the scatter key is rv[t]; radix passes on its
    // digits above the low 12 bring every element to the 4096-position
    // block holding its destination, and a placement pass writes each
    // block out through LDS.
    const uint32_t* a1 = rec0 + record_offset(1, k, n);
    auto rv_plane = [&](int m) -> Quant {
      if (m == 1) return Quant{kPlaneIndex, nullptr, 0, nullptr};
      return Quant{kPlaneArray, a1 + (size_t)((m - 2 + k) % k) * un, 0, nullptr};
    };
    const int passes = place_passes(n);
    for (int tgt = 0; tgt < k; ++tgt) {
      if (tgt == 1) continue;
      uint32_t* at_rec = rec0 + record_offset(tgt, k, n);
      std::vector<std::pair<Quant, uint32_t*>> vals;  // source, destination plane
      if (tgt == 0) {
        for (int c = 0; c <= k - 2; ++c) vals.push_back({rv_plane((1 + c) % k), at_rec + (size_t)c * un});
      } else {
        for (int c = k - tgt; c <= k - 2; ++c)
          vals.push_back({rv_plane((tgt + 1 + c) % k), at_rec + (size_t)c * un});
      }
      const int nv = (int)vals.size();
      auto slot = [&](int set, int i) { return vb + ((size_t)set * (k + 2) + i) * un; };
      const uint32_t* kin = rv_plane(tgt).in;
      int set = 0;
      for (int p = 0; p < passes; ++p) {
        Payload pay{};
        for (int v = 0; v < nv; ++v) {
          Plane& pl = pay.p[pay.count++];
          pl.kind = p == 0 ? vals[v].first.kind : kPlaneArray;
          pl.in = p == 0 ? vals[v].first.in : slot(set, v + 1);
          pl.word = 0;
          pl.out = slot(set ^ 1, v + 1);
        }
        RadixExtra rx;
        rx.status = t_status;
        KD_LAUNCH(KD_K_RECORDS, launch_radix_pass(kin, ts, 0, slot(set ^ 1, 0), pay, n, total,
                                                  place_shift(p), rcnt, rgrp, st, rx));
        set ^= 1;
        kin = slot(set, 0);
      }
      PlaceArgs pa{};
      pa.nv = nv;
      for (int v = 0; v < nv; ++v) {
        pa.val[v] = slot(set, v + 1);
        pa.dst[v] = vals[v].second;
      }
      KD_LAUNCH(KD_K_RECORDS, launch_place(slot(set, 0), pa, n, total, t_status, st));
    }
  }
  return KD_OK;
}

int partition_impl(const Job& J, hipStream_t st) {
  const int64_t n = J.n;
  const int k = J.k;
  const Layout L = plan(n, k, J.B);
  void* ws = J.ws;
  const ForestArgs fa = forest_args(J, L);
  uint32_t* S = at<uint32_t>(ws, L.S);
  if (n > 0) {
    if (k == 1) {
      KD_TRY(launch_copy_k1(S, fa, n, J.perm, st));
    } else {
      int64_t cutover = J.cutover;
      const uint32_t* r0 = at<uint32_t>(ws, L.rec0);
      uint32_t* r1 = at<uint32_t>(ws, L.rec1);
      uint32_t* r2 = at<uint32_t>(ws, L.rec2);
      // host bounds from the row counts: deepest global level, finish items
      int levels = 0;
      int64_t items = 0;
      for (int b = 0; b < J.B; ++b) {
        const int64_t nb = J.h_off[b + 1] - J.h_off[b];
        const int lc = cutover_depth(nb, cutover);
        levels = lc > levels ? lc : levels;
        items += nb > 0 ? ((int64_t)1 << lc) : 0;
      }
      // the default level form: one split per level (form 4) for a single
      // tree of k >= 3 (measured faster from k = 3 on), else form 1
      const int level = J.level != 0 ? J.level : (J.B == 1 && k >= 3 ? 4 : 1);
      // look-back levels: status words and tile counters start from zero
      const bool lookback = level == 2;
      uint64_t* lstat = lookback ? at<uint64_t>(ws, L.lstat) : nullptr;
      int32_t* ltick = at<int32_t>(ws, L.ltick);
      if (lookback && levels > 0) {
        KD_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(lstat), 0u,
                               2 * level_tiles(n) * (k - 1), st));
        KD_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ltick), 0u, kMaxLevels, st));
      }
      // one tree: every level moves only the planes later levels and the
      // on-chip finish read (a batch's trees end at different depths)
      const int defer = level == 3 && J.B == 1 && k >= 3 ? 1 : 0;
      if (level == 4 && J.B == 1) {
        // level form 4: at level L only array L mod k moves (one multi-level
        // split), then the nodes of depth L are recorded; the arrays the
        // on-chip finish reads get their last split after the last level
        std::vector<uint32_t> lm(levels > 0 ? levels : 1, 0u), fm(kMaxK, 0u);
        rolling_masks(k, levels, lm.data(), fm.data());
        SplitJob sj{};
        sj.n = n;
        sj.k = k;
        sj.uoff = fa.uoff;
        sj.lmax = fa.lmax;
        sj.status = fa.status;
        uint32_t* med = at<uint32_t>(ws, L.med);
        sj.med = med;
        SplitInfo* info = at<SplitInfo>(ws, L.sinfo);
        uint32_t* tval = at<uint32_t>(ws, L.stval);
        uint32_t* tflag = at<uint32_t>(ws, L.stflag);
        uint32_t* scarry = at<uint32_t>(ws, L.scarry);
        void* skeys = at<void>(ws, L.skeys);
        for (int d = 0; d < levels; ++d) {
          sj.level = d;
          sj.final_j = -1;
          sj.wmask = lm[d];
          if (d >= 1)
            KD_LAUNCH(KD_K_LEVEL, launch_split(r0, S, r1, r2, sj, info, tval, tflag, scarry, skeys, st));
          KD_LAUNCH(KD_K_LEVEL, launch_split_medians(r0, S, r1, r2, sj, med, J.perm, st));
        }
        for (int j = 1; j < k && levels > 0; ++j) {
          sj.level = -1;
          sj.final_j = j;
          sj.wmask = fm[j];
          KD_LAUNCH(KD_K_LEVEL, launch_split(r0, S, r1, r2, sj, info, tval, tflag, scarry, skeys, st));
        }
        KD_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(fa.queue), 0u, 1, st));
        KD_LAUNCH(KD_K_LEAF, launch_leaf(r0, S, r1, r2, n, k, cutover, fa, J.perm, items,
                                         J.leaf_blocks, 2, st));
        if (J.lo && J.hi) KD_TRY(launch_children(fa.uoff, n, J.lo, J.hi, st));
        return KD_OK;
      }
      std::vector<uint64_t> wm(levels > 0 ? levels : 1, ~0ull);
      if (J.B == 1 && !lookback && levels > 0) level_write_masks(k, levels, wm.data(), defer);
      // Deferred partitioning: array j >= 2 reaches its layout at depth
      // min(j, deepest global level) in one stable radix pass by bucket
      // (keys in the radix slots, which the partition does not use), right
      // before the level that splits it, or before the finish when no such
      // level runs; the node ranks of depth d are taken while array d has its
      // depth-d layout.
      uint32_t* nodes = at<uint32_t>(ws, L.nodes);
      uint32_t* dkey = at<uint32_t>(ws, L.vbuf);
      const int32_t* nu_dev = fa.uoff + 1;
      auto split = [&](int j) -> int {
        KD_LAUNCH(KD_K_LEVEL, launch_defer_bucket(r0, S, r1, r2, n, k, j, fa, nodes, dkey, st));
        Payload pay{};
        pay.count = k - 1;
        for (int c = 0; c < k - 1; ++c) {
          const int64_t o = record_offset(j, k, n) + (int64_t)c * n;
          pay.p[c].in = r0 + o;
          pay.p[c].out = r1 + o;  // one write: the first moved-record buffer
          pay.p[c].kind = kPlaneArray;
          pay.p[c].word = 0;
        }
        const TupleSrc none{nullptr, k, 0};
        RadixExtra rx;
        rx.status = fa.status;
        KD_LAUNCH(KD_K_LEVEL, launch_radix_pass(dkey, none, 0, nullptr, pay, n, nu_dev, 0,
                                                at<uint32_t>(ws, L.rcnt), at<uint32_t>(ws, L.rgrp),
                                                st, rx));
        return KD_OK;
      };
      for (int d = 0; d < levels; ++d) {
        if (defer && d >= 2 && d < k) {
          const int rc = split(d);
          if (rc != KD_OK) return rc;
        }
        if (defer && d <= k - 2)
          KD_LAUNCH(KD_K_LEVEL, launch_node_ranks(r0, S, r1, r2, n, k, d, fa, nodes, st));
        KD_LAUNCH(KD_K_LEVEL, launch_level(r0, S, r1, r2, n, k, d, cutover, fa, J.perm,
                                           at<void>(ws, L.seginfo), at<uint32_t>(ws, L.lcnt),
                                           at<uint64_t>(ws, L.lcarry), lstat, ltick, wm[d],
                                           defer, st));
      }
      if (defer)
        for (int j = levels > 2 ? levels : 2; j < k; ++j) {
          const int rc = split(j);
          if (rc != KD_OK) return rc;
        }
      // the finish takes its items from a counter; partition may run again
      // after one presort, so the counter is cleared here
      KD_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(fa.queue), 0u, 1, st));
      KD_LAUNCH(KD_K_LEAF, launch_leaf(r0, S, r1, r2, n, k, cutover, fa, J.perm, items, J.leaf_blocks,
                                       defer, st));
    }
    if (J.lo && J.hi) KD_TRY(launch_children(fa.uoff, n, J.lo, J.hi, st));
  }
  return KD_OK;
}

// Validation shared by every entry point; `cutover` may be lowered so that the
// on-chip finish fits the 160 KiB of LDS of a workgroup.
int check_job(Job& J, size_t ws_bytes, const kd_options* opts) {
  if (J.n < 0 || J.k < 1 || J.B < 1 || (J.dtype != KD_I32 && J.dtype != KD_F32)) return KD_EINVAL;
  if (J.n > KD_MAX_N || J.k > KD_MAX_K) return KD_EUNSUPPORTED;
  if ((J.n > 0 && !J.tuples) || !J.ws || !J.n_unique) return KD_EINVAL;
  if (!aligned4(J.tuples) || !aligned4(J.ws)) return KD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(J.n_unique) & 7u) != 0) return KD_EINVAL;
  if (ws_bytes < plan(J.n, J.k, J.B, J.models != nullptr).end) return KD_ENOMEM;
  int rc = check_opts(opts, &J.cutover, &J.leaf_blocks, &J.records, &J.learned_sorts, &J.level,
                      &J.digit_bits, &J.sort_items);
  if (rc != KD_OK) return rc;
  while (J.cutover > 1024 && leaf_lds_bytes(J.cutover, J.k) + 8192 > 160 * 1024) J.cutover /= 2;
  return KD_OK;
}

// The comparison builder (Sec. 3: an O(n log n) method that selects each
// subarray's median afresh at every level and partitions about it): array 0
// and duplicate removal as in the presort (so the nodes are the same distinct
// rows), then the rows with their k key words go through the global levels of
// select.hip (a radix-select of every subarray's median by the level's super
// key and a partition about it) and the on-chip finish below 2048 rows.
// Uses the build's workspace: the row planes in the radix slots, the
// histograms and per-subarray state in the record space.
int select_impl(const Job& J, hipStream_t st) {
  const int64_t n = J.n;
  const int k = J.k;
  int rc = presort_impl(J, st, true);
  if (rc != KD_OK) return rc;
  if (n == 0) return KD_OK;
  void* ws = J.ws;
  const Layout L = plan(n, k, J.B);
  const size_t un = (size_t)n;
  uint32_t* S = at<uint32_t>(ws, L.S);
  int32_t* uoff = at<int32_t>(ws, L.uoff);
  const ForestArgs fa = forest_args(J, L);
  if (k == 1) {
    KD_TRY(launch_copy_k1(S, fa, n, J.perm, st));
    return KD_OK;
  }
  uint32_t* P = at<uint32_t>(ws, L.vbuf);
  uint32_t* Q = P + (size_t)(k + 1) * un;
  uint32_t* hist = at<uint32_t>(ws, L.rec0);
  SelState* state = at<SelState>(ws, L.rec1);
  const int levels = select_levels_host(n);
  KD_TRY(launch_fill_u32(hist, 0u, (int64_t)256 << levels, st));
  const TupleSrc ts{static_cast<const uint32_t*>(J.tuples), k, J.dtype == KD_F32 ? 1 : 0};
  KD_TRY(launch_sel_init(ts.t, k, ts.is_float, S, uoff + 1, n, P, st));
  SelJob sj{n, k, 0, uoff + 1, fa.status};
  for (int d = 0; d < levels; ++d) {  // levels past the device's own count do nothing
    sj.depth = d;
    uint32_t* in = (d & 1) ? Q : P;
    uint32_t* out = (d & 1) ? P : Q;
    KD_LAUNCH(KD_K_LEVEL, launch_sel_level(sj, in, out, hist, state, at<uint64_t>(ws, L.lstat),
                                           at<uint32_t>(ws, L.stflag), at<uint64_t>(ws, L.lcarry),
                                           J.perm, st));
  }
  KD_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(fa.queue), 0u, 1, st));
  KD_LAUNCH(KD_K_LEAF, launch_sel_leaf(sj, P, Q, J.perm, fa.queue, (int64_t)1 << levels, st));
  return KD_OK;
}

int check_outputs(const Job& J) {
  if ((J.n > 0 && !J.perm) || !aligned4(J.perm)) return KD_EINVAL;
  if ((J.lo == nullptr) != (J.hi == nullptr)) return KD_EINVAL;
  if (!aligned4(J.lo) || !aligned4(J.hi)) return KD_EINVAL;
  return KD_OK;
}

// single tree: offsets {0, n} live in the workspace
int single_job(Job& J, const void* tuples, int64_t n, int32_t k, int32_t dtype, int64_t* nu,
               void* ws, size_t ws_bytes, const kd_options* opts, int64_t* h_off, hipStream_t st,
               bool upload, const void* models = nullptr) {
  J = Job{};
  J.models = static_cast<const CdfModel*>(models);
  if (models && (reinterpret_cast<uintptr_t>(models) & 3u) != 0) return KD_EINVAL;
  J.tuples = tuples;
  J.n = n;
  J.B = 1;
  J.k = k;
  J.dtype = dtype;
  J.n_unique = nu;
  J.ws = ws;
  h_off[0] = 0;
  h_off[1] = n;
  J.h_off = h_off;
  int rc = check_job(J, ws_bytes, opts);
  if (rc != KD_OK) return rc;
  int64_t* d_off = at<int64_t>(ws, plan(n, k, 1).offs);
  J.d_off = d_off;
  if (upload) {
    // {0, n} as 64-bit words
    FillList f;
    f.add(reinterpret_cast<uint32_t*>(d_off), 0u, 2);
    f.add(reinterpret_cast<uint32_t*>(d_off) + 2, (uint32_t)(n & 0xFFFFFFFF), 1);
    f.add(reinterpret_cast<uint32_t*>(d_off) + 3, (uint32_t)(n >> 32), 1);
    KD_TRY(launch_fills(f, st));
  }
  return KD_OK;
}

int presort_learned(const Job& J, hipStream_t st) {
  int rc = presort_impl(J, st);
  if (rc != KD_OK) return rc;
  if (J.fell_back) {
    const Layout L = plan(J.n, J.k, 1, true);
    KD_TRY(launch_copy_i32(at<int32_t>(J.ws, L.flags), J.k, J.fell_back, st));
  }
  return KD_OK;
}

// ---- model training (host side) -----------------------------------------------------
struct TrainLayout {
  size_t a, b, cnt, grp, range, end;
};
TrainLayout train_plan(int k, int S) {
  TrainLayout T{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at2 = o;
    o = align_up(o + bytes);
    return at2;
  };
  T.a = take(4 * (size_t)k * S);
  T.b = take(4 * (size_t)k * S);
  T.cnt = take(4 * (size_t)radix_count_words(S));
  T.grp = take(4 * (size_t)radix_group_words(S));
  T.range = take(4 * 2 * (size_t)k);
  T.end = o;
  return T;
}

}  // namespace
}  // namespace kd

namespace kd {
namespace {
// Shared checks of the tree searches; on success *is_float is set.  perm may
// be null only where the caller says so.
int check_query(const void* d_nodes, int64_t n, int32_t k, int32_t dtype, const int32_t* d_perm,
                bool need_perm, const int64_t* d_n_nodes, int64_t nq, uint64_t* d_visits,
                int* is_float) {
  if (n < 0 || k < 1 || nq < 0 || (dtype != KD_I32 && dtype != KD_F32)) return KD_EINVAL;
  if (n > KD_MAX_N || k > KD_MAX_K || nq > KD_MAX_QUERIES) return KD_EUNSUPPORTED;
  if (!d_nodes || !d_n_nodes || (need_perm && !d_perm)) return KD_EINVAL;
  if (!kd::aligned4(d_nodes) || !kd::aligned4(d_perm) ||
      (reinterpret_cast<uintptr_t>(d_n_nodes) & 7u) || (reinterpret_cast<uintptr_t>(d_visits) & 7u))
    return KD_EINVAL;
  *is_float = dtype == KD_F32;
  return KD_OK;
}
}  // namespace
}  // namespace kd

// ---- builds without allocation: the library's own workspace --------------------
// kdtree_build_noalloc() builds with a workspace that is a file-scope device
// array of KD_NOALLOC_WORKSPACE_BYTES bytes instead of one the caller passes.
// Each device holds its own copy at its own address, taken once per device
// (with that device current) and kept; host code uses that address, never the
// array's name, which on the host is only a stand-in.
__device__ __align__(256) unsigned char scratch[KD_NOALLOC_WORKSPACE_BYTES];

namespace kd {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch[kMaxDevices] = {};

// The current device's copy of `scratch` (null on failure).
void* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
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
    case KD_EUNSUPPORTED: return "unsupported size (n or k beyond the limits) or model kind";
    case KD_EINTERNAL: return "internal inconsistency found by a kernel (see kd_status)";
    default: return "unknown status";
  }
}

int kd_level_plan(int32_t k, int32_t levels, uint32_t* h_level_mask, uint32_t* h_final_mask) {
  if (k < 2 || levels < 0 || !h_final_mask || (levels > 0 && !h_level_mask)) return KD_EINVAL;
  if (k > KD_MAX_K || levels > 30) return KD_EUNSUPPORTED;
  std::vector<uint32_t> lm(levels > 0 ? levels : 1, 0u), fm(kd::kMaxK, 0u);
  kd::rolling_masks(k, levels, lm.data(), fm.data());
  for (int l = 0; l < levels; ++l) h_level_mask[l] = lm[l];
  for (int j = 0; j < k; ++j) h_final_mask[j] = fm[j];
  return KD_OK;
}

int kd_level_masks(int32_t k, int32_t levels, int32_t defer, uint64_t* h_masks, int32_t* h_moves) {
  if (k < 2 || levels < 0 || !h_moves || (levels > 0 && !h_masks) || (defer != 0 && defer != 1))
    return KD_EINVAL;
  if (k > KD_MAX_K || levels > 30) return KD_EUNSUPPORTED;
  if (levels > 0) kd::level_write_masks(k, levels, h_masks, defer);
  for (int d = 0; d <= levels; ++d)
    for (int j = 0; j < k; ++j) h_moves[d * k + j] = kd::level_array_moves(defer, d, j, k);
  return KD_OK;
}

int kd_status(const void* d_workspace, size_t workspace_bytes, uint32_t* h_bits, void* stream) {
  if (!d_workspace || !h_bits || !kd::aligned4(d_workspace)) return KD_EINVAL;
  if (workspace_bytes < 4 * (size_t)kd::kStatusWords) return KD_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t bits = 0;
  if (hipMemcpyAsync(&bits, d_workspace, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return KD_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return KD_EHIP;
  *h_bits = bits;
  return bits ? KD_EINTERNAL : KD_OK;
}

int kdtree_workspace_bytes(int64_t n, int32_t k, int32_t dtype, size_t* h_bytes) {
  if (!h_bytes || n < 0 || k < 1 || (dtype != KD_I32 && dtype != KD_F32)) return KD_EINVAL;
  if (n > KD_MAX_N || k > KD_MAX_K) return KD_EUNSUPPORTED;
  *h_bytes = kd::plan(n, k, 1).end;
  return KD_OK;
}

int kdtree_workspace_bytes_batched(int64_t total_rows, int32_t num_trees, int32_t k, int32_t dtype,
                                   size_t* h_bytes) {
  if (!h_bytes || total_rows < 0 || num_trees < 1 || k < 1 ||
      (dtype != KD_I32 && dtype != KD_F32))
    return KD_EINVAL;
  if (total_rows > KD_MAX_N || k > KD_MAX_K || num_trees > KD_MAX_TREES) return KD_EUNSUPPORTED;
  *h_bytes = kd::plan(total_rows, k, num_trees).end;
  return KD_OK;
}

int kdtree_presort(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int64_t* d_n_unique,
                   void* d_workspace, size_t workspace_bytes, const kd_options* opts,
                   void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  kd::Job J;
  int64_t h_off[2];
  int rc = kd::single_job(J, d_tuples, n, k, dtype, d_n_unique, d_workspace, workspace_bytes, opts,
                          h_off, st, true);
  if (rc != KD_OK) return rc;
  return kd::presort_impl(J, st);
}

int kdtree_partition(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                     int32_t* d_lo, int32_t* d_hi, int64_t* d_n_unique, void* d_workspace,
                     size_t workspace_bytes, const kd_options* opts, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  kd::Job J;
  int64_t h_off[2];
  int rc = kd::single_job(J, d_tuples, n, k, dtype, d_n_unique, d_workspace, workspace_bytes, opts,
                          h_off, st, false);
  if (rc != KD_OK) return rc;
  J.perm = d_perm;
  J.lo = d_lo;
  J.hi = d_hi;
  rc = kd::check_outputs(J);
  if (rc != KD_OK) return rc;
  return kd::partition_impl(J, st);
}

int kdtree_build(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                 int32_t* d_lo, int32_t* d_hi, int64_t* d_n_unique, void* d_workspace,
                 size_t workspace_bytes, const kd_options* opts, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  kd::Job J;
  int64_t h_off[2];
  // validate everything before the first launch
  {
    kd::Job V;
    int64_t h2[2];
    int rc = kd::single_job(V, d_tuples, n, k, dtype, d_n_unique, d_workspace, workspace_bytes,
                            opts, h2, st, false);
    if (rc != KD_OK) return rc;
    V.perm = d_perm;
    V.lo = d_lo;
    V.hi = d_hi;
    rc = kd::check_outputs(V);
    if (rc != KD_OK) return rc;
  }
  int rc = kd::single_job(J, d_tuples, n, k, dtype, d_n_unique, d_workspace, workspace_bytes, opts,
                          h_off, st, true);
  if (rc != KD_OK) return rc;
  J.perm = d_perm;
  J.lo = d_lo;
  J.hi = d_hi;
  rc = kd::presort_impl(J, st);
  if (rc != KD_OK) return rc;
  return kd::partition_impl(J, st);
}

int kdtree_build_noalloc(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                         int32_t* d_lo, int32_t* d_hi, int64_t* d_n_unique,
                         const kd_options* opts, void* stream) {
  // the same validation as kdtree_build, with the workspace's size checked
  // against the array before anything touches the device
  if (n < 0 || k < 1 || (dtype != KD_I32 && dtype != KD_F32)) return KD_EINVAL;
  if (n > KD_MAX_N || k > KD_MAX_K) return KD_EUNSUPPORTED;
  if (kd::plan(n, k, 1).end > (size_t)KD_NOALLOC_WORKSPACE_BYTES) return KD_ENOMEM;
  {
    kd::Job V;
    int64_t h2[2];
    // any aligned non-null stand-in: single_job only checks it
    int rc = kd::single_job(V, d_tuples, n, k, dtype, d_n_unique, reinterpret_cast<void*>(256),
                            KD_NOALLOC_WORKSPACE_BYTES, opts, h2, nullptr, false);
    if (rc != KD_OK) return rc;
    V.perm = d_perm;
    V.lo = d_lo;
    V.hi = d_hi;
    rc = kd::check_outputs(V);
    if (rc != KD_OK) return rc;
  }
  void* ws = kd::scratch_on_current_device();
  if (!ws) return KD_EHIP;
  return kdtree_build(d_tuples, n, k, dtype, d_perm, d_lo, d_hi, d_n_unique, ws,
                      KD_NOALLOC_WORKSPACE_BYTES, opts, stream);
}

int kdtree_build_select(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                        int64_t* d_n_unique, void* d_workspace, size_t workspace_bytes,
                        const kd_options* opts, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  {
    kd::Job V;
    int64_t h2[2];
    int rc = kd::single_job(V, d_tuples, n, k, dtype, d_n_unique, d_workspace, workspace_bytes,
                            opts, h2, st, false);
    if (rc != KD_OK) return rc;
    V.perm = d_perm;
    rc = kd::check_outputs(V);
    if (rc != KD_OK) return rc;
  }
  kd::Job J;
  int64_t h_off[2];
  int rc = kd::single_job(J, d_tuples, n, k, dtype, d_n_unique, d_workspace, workspace_bytes, opts,
                          h_off, st, true);
  if (rc != KD_OK) return rc;
  J.perm = d_perm;
  return kd::select_impl(J, st);
}

int kdtree_build_batched(const void* d_tuples, const int64_t* d_offsets, const int64_t* h_offsets,
                         int32_t num_trees, int32_t k, int32_t dtype, int32_t* d_perm,
                         int64_t* d_n_unique, void* d_workspace, size_t workspace_bytes,
                         const kd_options* opts, void* stream) {
  if (num_trees < 1 || !d_offsets || !h_offsets) return KD_EINVAL;
  if (num_trees > KD_MAX_TREES) return KD_EUNSUPPORTED;
  if ((reinterpret_cast<uintptr_t>(d_offsets) & 7u) != 0) return KD_EINVAL;
  if (h_offsets[0] != 0) return KD_EINVAL;
  for (int b = 0; b < num_trees; ++b)
    if (h_offsets[b + 1] < h_offsets[b]) return KD_EINVAL;
  kd::Job J{};
  J.tuples = d_tuples;
  J.n = h_offsets[num_trees];
  J.B = num_trees;
  J.d_off = d_offsets;
  J.h_off = h_offsets;
  J.k = k;
  J.dtype = dtype;
  J.perm = d_perm;
  J.n_unique = d_n_unique;
  J.ws = d_workspace;
  int rc = kd::check_job(J, workspace_bytes, opts);
  if (rc != KD_OK) return rc;
  rc = kd::check_outputs(J);
  if (rc != KD_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = kd::presort_impl(J, st);
  if (rc != KD_OK) return rc;
  return kd::partition_impl(J, st);
}

int kdtree_workspace_bytes_learned(int64_t n, int32_t k, int32_t dtype, size_t* h_bytes) {
  if (!h_bytes || n < 0 || k < 1 || (dtype != KD_I32 && dtype != KD_F32)) return KD_EINVAL;
  if (n > KD_MAX_N || k > KD_MAX_K) return KD_EUNSUPPORTED;
  *h_bytes = kd::plan(n, k, 1, true).end;
  return KD_OK;
}

int kd_cdf_model_bytes(int32_t k, size_t* h_bytes) {
  if (!h_bytes || k < 1) return KD_EINVAL;
  if (k > KD_MAX_K) return KD_EUNSUPPORTED;
  *h_bytes = (size_t)k * sizeof(kd::CdfModel);
  return KD_OK;
}

int kd_cdf_train_workspace_bytes(int32_t k, int32_t n_samples, size_t* h_bytes) {
  if (!h_bytes || k < 1 || n_samples < 1) return KD_EINVAL;
  if (k > KD_MAX_K || n_samples > KD_CDF_MAX_SAMPLES) return KD_EUNSUPPORTED;
  *h_bytes = kd::train_plan(k, n_samples).end;
  return KD_OK;
}

int kd_cdf_train(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t kind,
                 int32_t n_samples, int32_t steps, float lr, void* d_models, void* d_workspace,
                 size_t workspace_bytes, void* stream) {
  if (n < 1 || k < 1 || n_samples < 1 || steps < 0 || (dtype != KD_I32 && dtype != KD_F32))
    return KD_EINVAL;
  if (kind != KD_CDF_PWL) return KD_EUNSUPPORTED;
  if (!(lr > 0.f) || !std::isfinite(lr)) return KD_EINVAL;
  if (n > KD_MAX_N || k > KD_MAX_K || n_samples > KD_CDF_MAX_SAMPLES || steps > KD_CDF_MAX_STEPS)
    return KD_EUNSUPPORTED;
  if (!d_tuples || !d_models || !d_workspace) return KD_EINVAL;
  if (!kd::aligned4(d_tuples) || !kd::aligned4(d_models) || !kd::aligned4(d_workspace))
    return KD_EINVAL;
  const kd::TrainLayout T = kd::train_plan(k, n_samples);
  if (workspace_bytes < T.end) return KD_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t* a = kd::at<uint32_t>(d_workspace, T.a);
  uint32_t* b = kd::at<uint32_t>(d_workspace, T.b);
  uint32_t* cnt = kd::at<uint32_t>(d_workspace, T.cnt);
  uint32_t* grp = kd::at<uint32_t>(d_workspace, T.grp);
  const int is_float = dtype == KD_F32 ? 1 : 0;
  KD_TRY(kd::launch_cdf_sample(static_cast<const uint32_t*>(d_tuples), n, k, is_float, n_samples, a,
                               st));
  // the sample of each dimension is presorted by the radix passes (4 passes,
  // so the result is back in a)
  const kd::TupleSrc ts{nullptr, k, is_float};
  const kd::Payload none{};
  for (int d = 0; d < k; ++d) {
    uint32_t* x = a + (size_t)d * n_samples;
    uint32_t* y = b + (size_t)d * n_samples;
    for (int ps = 0; ps < kd::kPassesPerWord; ++ps) {
      KD_TRY(kd::launch_radix_pass(x, ts, 0, y, none, n_samples, nullptr, ps * kd::kRadixBits, cnt,
                                   grp, st));
      std::swap(x, y);
    }
  }
  uint32_t* range = kd::at<uint32_t>(d_workspace, T.range);
  KD_TRY(kd::launch_col_range(static_cast<const uint32_t*>(d_tuples), n, k, is_float, range, st));
  KD_TRY(kd::launch_cdf_fit(a, n_samples, k, is_float, range, steps, lr,
                            static_cast<kd::CdfModel*>(d_models), st));
  return KD_OK;
}

int kd_cdf_loss_grad(const void* d_values, int32_t m, int32_t dtype, uint32_t lo_bits,
                     uint32_t hi_bits, const float* d_theta, float* d_loss, float* d_grad,
                     void* d_scratch, void* stream) {
  if (m < 1 || (dtype != KD_I32 && dtype != KD_F32)) return KD_EINVAL;
  if (m > KD_CDF_MAX_SAMPLES) return KD_EUNSUPPORTED;
  if (!d_values || !d_theta || !d_loss || !d_grad || !d_scratch) return KD_EINVAL;
  if (!kd::aligned4(d_values) || !kd::aligned4(d_theta) || !kd::aligned4(d_loss) ||
      !kd::aligned4(d_grad) || !kd::aligned4(d_scratch))
    return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KD_TRY(kd::launch_cdf_loss_grad(static_cast<const uint32_t*>(d_values), m, dtype == KD_F32 ? 1 : 0,
                                  lo_bits, hi_bits, d_theta, static_cast<uint32_t*>(d_scratch),
                                  d_loss, d_grad, st));
  return KD_OK;
}

int kd_cdf_eval(const void* d_model, const void* d_values, int32_t m, int32_t nb_bits, float* d_F,
                int32_t* d_bucket, void* stream) {
  if (m < 0 || nb_bits < 1 || nb_bits > 16) return KD_EINVAL;
  if (m == 0) return KD_OK;
  if (!d_model || !d_values || !d_F || !d_bucket) return KD_EINVAL;
  if (!kd::aligned4(d_model) || !kd::aligned4(d_values) || !kd::aligned4(d_F) ||
      !kd::aligned4(d_bucket))
    return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KD_TRY(kd::launch_cdf_eval(static_cast<const kd::CdfModel*>(d_model),
                             static_cast<const uint32_t*>(d_values), m, nb_bits, d_F, d_bucket, st));
  return KD_OK;
}

int kdtree_presort_learned(const void* d_tuples, int64_t n, int32_t k, int32_t dtype,
                           const void* d_models, int64_t* d_n_unique, int32_t* d_fell_back,
                           void* d_workspace, size_t workspace_bytes, const kd_options* opts,
                           void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!d_models) return KD_EINVAL;
  if (!kd::aligned4(d_fell_back)) return KD_EINVAL;
  kd::Job J;
  int64_t h_off[2];
  int rc = kd::single_job(J, d_tuples, n, k, dtype, d_n_unique, d_workspace, workspace_bytes, opts,
                          h_off, st, true, d_models);
  if (rc != KD_OK) return rc;
  J.fell_back = d_fell_back;
  return kd::presort_learned(J, st);
}

int kdtree_build_learned(const void* d_tuples, int64_t n, int32_t k, int32_t dtype,
                         const void* d_models, int32_t* d_perm, int32_t* d_lo, int32_t* d_hi,
                         int64_t* d_n_unique, int32_t* d_fell_back, void* d_workspace,
                         size_t workspace_bytes, const kd_options* opts, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!d_models) return KD_EINVAL;
  if (!kd::aligned4(d_fell_back)) return KD_EINVAL;
  {
    kd::Job V;
    int64_t h2[2];
    int rc = kd::single_job(V, d_tuples, n, k, dtype, d_n_unique, d_workspace, workspace_bytes,
                            opts, h2, st, false, d_models);
    if (rc != KD_OK) return rc;
    V.perm = d_perm;
    V.lo = d_lo;
    V.hi = d_hi;
    rc = kd::check_outputs(V);
    if (rc != KD_OK) return rc;
  }
  kd::Job J;
  int64_t h_off[2];
  int rc = kd::single_job(J, d_tuples, n, k, dtype, d_n_unique, d_workspace, workspace_bytes, opts,
                          h_off, st, true, d_models);
  if (rc != KD_OK) return rc;
  J.perm = d_perm;
  J.lo = d_lo;
  J.hi = d_hi;
  J.fell_back = d_fell_back;
  rc = kd::presort_learned(J, st);
  if (rc != KD_OK) return rc;
  return kd::partition_impl(J, st);
}

#define KD_QLAUNCH(expr)                              \
  do {                                                \
    kd::probe_begin(KD_K_QUERY, st);                  \
    hipError_t e__ = (expr);                          \
    kd::probe_end(KD_K_QUERY, st);                    \
    if (e__ != hipSuccess) return KD_EHIP;            \
  } while (0)


int kd_gather_nodes(const void* d_tuples, int64_t n, int32_t k, int32_t dtype,
                    const int32_t* d_perm, const int64_t* d_n_nodes, void* d_nodes, void* stream) {
  int fl = 0;
  int rc = kd::check_query(d_tuples, n, k, dtype, d_perm, true, d_n_nodes, 0, nullptr, &fl);
  if (rc != KD_OK) return rc;
  if (n == 0) return KD_OK;
  if (!d_nodes || !kd::aligned4(d_nodes)) return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KD_QLAUNCH(kd::launch_gather_nodes(d_tuples, n, k, fl, d_perm, d_n_nodes, d_nodes, st));
  return KD_OK;
}

int kd_subtree_bounds(const void* d_nodes, int64_t n, int32_t k, int32_t dtype,
                      const int64_t* d_n_nodes, void* d_bounds, void* stream) {
  int fl = 0;
  int rc = kd::check_query(d_nodes, n, k, dtype, nullptr, false, d_n_nodes, 0, nullptr, &fl);
  if (rc != KD_OK) return rc;
  if (n == 0) return KD_OK;
  if (!d_bounds || !kd::aligned4(d_bounds)) return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KD_QLAUNCH(kd::launch_subtree_bounds(d_nodes, n, k, fl, d_n_nodes, d_bounds, st));
  return KD_OK;
}

int kd_region_count(const void* d_nodes, const void* d_bounds, int64_t n, int32_t k, int32_t dtype,
                    const int64_t* d_n_nodes, const void* d_lower, const void* d_upper, int64_t nq,
                    int32_t* d_counts, uint64_t* d_visits, void* stream) {
  int fl = 0;
  int rc = kd::check_query(d_nodes, n, k, dtype, nullptr, false, d_n_nodes, nq, d_visits, &fl);
  if (rc != KD_OK) return rc;
  if (!kd::aligned4(d_bounds)) return KD_EINVAL;
  if (nq == 0) return KD_OK;
  if (!d_lower || !d_upper || !d_counts) return KD_EINVAL;
  if (!kd::aligned4(d_lower) || !kd::aligned4(d_upper) || !kd::aligned4(d_counts)) return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KD_QLAUNCH(kd::launch_region(d_nodes, d_bounds, n, k, fl, nullptr, d_n_nodes, d_lower, d_upper, nq,
                               d_counts, nullptr, nullptr, 0,
                               reinterpret_cast<unsigned long long*>(d_visits), st));
  return KD_OK;
}

int kd_region_rows(const void* d_nodes, const void* d_bounds, int64_t n, int32_t k, int32_t dtype,
                   const int32_t* d_perm, const int64_t* d_n_nodes, const void* d_lower,
                   const void* d_upper, int64_t nq, const int64_t* d_offsets, int32_t* d_rows,
                   int64_t rows_capacity, uint64_t* d_visits, void* stream) {
  int fl = 0;
  int rc = kd::check_query(d_nodes, n, k, dtype, d_perm, true, d_n_nodes, nq, d_visits, &fl);
  if (rc != KD_OK) return rc;
  if (rows_capacity < 0 || !kd::aligned4(d_bounds)) return KD_EINVAL;
  if (nq == 0) return KD_OK;
  if (!d_lower || !d_upper || !d_offsets || (!d_rows && rows_capacity > 0)) return KD_EINVAL;
  if (!kd::aligned4(d_lower) || !kd::aligned4(d_upper) || !kd::aligned4(d_rows) ||
      (reinterpret_cast<uintptr_t>(d_offsets) & 7u))
    return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // a null row buffer (capacity 0) still walks: nothing is written
  KD_QLAUNCH(kd::launch_region(d_nodes, d_bounds, n, k, fl, d_perm, d_n_nodes, d_lower, d_upper, nq,
                               nullptr, d_offsets, d_rows, rows_capacity,
                               reinterpret_cast<unsigned long long*>(d_visits), st));
  return KD_OK;
}

int kd_nearest(const void* d_nodes, int64_t n, int32_t k, int32_t dtype, const int32_t* d_perm,
               const int64_t* d_n_nodes, const void* d_points, int64_t nq, int32_t m,
               int32_t* d_rows, uint64_t* d_visits, void* stream) {
  int fl = 0;
  int rc = kd::check_query(d_nodes, n, k, dtype, d_perm, true, d_n_nodes, nq, d_visits, &fl);
  if (rc != KD_OK) return rc;
  if (m < 1 || m > KD_MAX_NEIGHBORS) return KD_EINVAL;
  if (nq == 0) return KD_OK;
  if (!d_points || !d_rows) return KD_EINVAL;
  if (!kd::aligned4(d_points) || !kd::aligned4(d_rows)) return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KD_QLAUNCH(kd::launch_nearest(d_nodes, n, k, fl, d_perm, d_n_nodes, d_points, nq, m, d_rows,
                                reinterpret_cast<unsigned long long*>(d_visits), st));
  return KD_OK;
}

int kd_all_nearest(const void* d_nodes, int64_t n, int32_t k, int32_t dtype, const int32_t* d_perm,
                   const int64_t* d_n_nodes, int32_t m, int32_t* d_rows, uint64_t* d_visits,
                   void* stream) {
  int fl = 0;
  int rc = kd::check_query(d_nodes, n, k, dtype, d_perm, true, d_n_nodes, 0, d_visits, &fl);
  if (rc != KD_OK) return rc;
  if (m < 1 || m > KD_MAX_NEIGHBORS) return KD_EINVAL;
  if (n > KD_MAX_QUERIES) return KD_EUNSUPPORTED;
  if (n == 0) return KD_OK;
  if (!d_rows || !kd::aligned4(d_rows)) return KD_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KD_QLAUNCH(kd::launch_nearest(d_nodes, n, k, fl, d_perm, d_n_nodes, nullptr, n, m, d_rows,
                                reinterpret_cast<unsigned long long*>(d_visits), st));
  return KD_OK;
}

int kd_reverse_workspace_bytes(int64_t n, size_t* h_bytes) {
  if (!h_bytes || n < 0) return KD_EINVAL;
  if (n > KD_MAX_N) return KD_EUNSUPPORTED;
  *h_bytes = kd::reverse_workspace_bytes(n);
  return KD_OK;
}

int kd_reverse_nearest(const int32_t* d_perm, const int64_t* d_n_nodes, int64_t n, int32_t m,
                       const int32_t* d_rows, int64_t* d_offsets, int32_t* d_lists,
                       void* d_workspace, size_t workspace_bytes, void* stream) {
  if (n < 0 || m < 1 || m > KD_MAX_NEIGHBORS) return KD_EINVAL;
  if (n > KD_MAX_N) return KD_EUNSUPPORTED;
  if (n == 0) return KD_OK;
  if (!d_perm || !d_n_nodes || !d_rows || !d_offsets || !d_lists || !d_workspace) return KD_EINVAL;
  if (!kd::aligned4(d_perm) || !kd::aligned4(d_rows) || !kd::aligned4(d_lists) ||
      (reinterpret_cast<uintptr_t>(d_n_nodes) & 7u) || (reinterpret_cast<uintptr_t>(d_offsets) & 7u) ||
      (reinterpret_cast<uintptr_t>(d_workspace) & 7u))
    return KD_EINVAL;
  if (workspace_bytes < kd::reverse_workspace_bytes(n)) return KD_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KD_QLAUNCH(kd::launch_reverse_nearest(d_perm, d_n_nodes, n, m, d_rows, d_offsets, d_lists,
                                        d_workspace, st));
  return KD_OK;
}

int kd_probe_start(int32_t kernel_class, int32_t capacity) {
  if (kernel_class < KD_K_ONESWEEP || kernel_class > KD_K_QUERY || capacity < 1 ||
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
