// Host-side launchers of the gfx950 kernels.  Each one enqueues work on the
// given stream and returns the launch status; none of them synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kd {

constexpr int kMaxK = 8;
constexpr int kRadixBits = 8;      // the default digit width
constexpr int kRadix = 1 << kRadixBits;
constexpr int kPassesPerWord = 32 / kRadixBits;
constexpr int kSortTile = 4096;   // elements per radix tile (the smaller of the two tile sizes)
constexpr int kMaxBins = 1 << 11; // bins of the widest digit (11 bits)
// Digit passes of a 32-bit word at digit width `bits` (8: 4 passes, 11: 3).
inline int passes_per_word(int bits) { return (32 + bits - 1) / bits; }
constexpr int kLevelTile = 4096;  // elements per level-partition tile

// Device view of a forest of independent trees (a single build is one tree):
// rows of tree b are off[b] .. off[b+1]-1; after duplicate removal its distinct
// rows occupy positions uoff[b] .. uoff[b+1]-1 of every sorted order.
struct ForestArgs {
  int B;
  const int64_t* off;
  const int32_t* uoff;
  const int32_t* lmax;
  const int32_t* wgbase;
  int32_t* queue;
  uint32_t* status;  // the build's status word (see kStatus* below)
};

// Bits of a build's device status word (the first word of its workspace,
// cleared when the presort starts).  A kernel that finds counts contradicting
// each other (which a correct build never does) drops the write it cannot
// place and sets its bit; the host then reports KD_EINTERNAL.
enum : uint32_t {
  kStatusRadix = 1u,       // a radix pass computed a destination outside the array
  kStatusLevelSeg = 2u,    // more subarrays meet a level tile than it can hold
  kStatusLevelMove = 4u,   // a level move computed a destination outside its subarray
  kStatusLeaf = 8u,        // the on-chip finish computed a destination outside its subarray
  kStatusSplit = 16u,      // a multi-level split computed a destination outside its subarray
  kStatusPlace = 32u,      // a record placement key was not a permutation
  kStatusNode = 64u,       // a node rank lookup found no subarray or no rank
};

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t st);
hipError_t launch_store_i64(int64_t* dst, const int64_t* src, hipStream_t st);
// Several short runs of equal words written by one launch: the small
// initialisations a build makes before its kernels (one launch instead of
// one per run).
constexpr int kMaxFills = 8;
struct FillList {
  uint32_t* p[kMaxFills];
  uint32_t value[kMaxFills];
  int32_t count[kMaxFills];
  int n = 0;
  void add(uint32_t* ptr, uint32_t v, int32_t c) {
    p[n] = ptr;
    value[n] = v;
    count[n] = c;
    ++n;
  }
};
// Fails (hipErrorInvalidValue) if a run is null with a positive count or the
// list holds more than kMaxFills runs.
hipError_t launch_fills(const FillList& f, hipStream_t st);

// Row-major tuples as a source of canonical (order-preserving unsigned) keys.
struct TupleSrc {
  const uint32_t* t;
  int k;
  int is_float;
};

// Tuple rows (row-major, k words each) to k planes of canonical words (plane
// d at out.p[d]), so that every radix pass reads coalesced planes.
struct PlaneOut {
  uint32_t* p[kMaxK];
};
hipError_t launch_rows_to_planes(const TupleSrc& ts, int64_t n, const PlaneOut& out, hipStream_t st);

// One payload plane of a radix pass.  Element i's value is in[i] (kind
// kPlaneArray), i itself (kPlaneIndex) or the canonical key word `word` of
// tuple row i (kPlaneTupleWord); it is written to out[dest].
enum { kPlaneArray = 0, kPlaneIndex = 1, kPlaneTupleWord = 2 };
struct Plane {
  const uint32_t* in;
  uint32_t* out;
  int kind;
  int word;
};
constexpr int kMaxPlanes = 10;
struct Payload {
  Plane p[kMaxPlanes];
  int count;
};

struct CdfModel;

// Options of a radix pass.  model: rank by the key's bucket under a learned
// CDF model (2^nb_bits buckets) instead of the key itself.  gate: when set,
// every kernel of the pass does nothing unless *gate != 0 (a sort that only
// runs when an earlier attempt failed).
struct RadixExtra {
  const CdfModel* model = nullptr;
  int nb_bits = 0;
  const int32_t* gate = nullptr;
  uint32_t* status = nullptr;  // status word (kStatusRadix), or null
  int bits = 8;                // digit width: 8 or 11 (model passes always 8)
  int items = 8;               // keys per thread: 8 (tiles of 4096) or 16 (8192)
  uint32_t* sync = nullptr;    // gated passes: radix_sync_words(n) counters, zero at first
};

// One stable LSD radix pass on the digit of width ex.bits at bit `shift`
// (tiles of 512 * ex.items keys): per-tile digit counts, a
// two-level scan and the scatter (four launches, no waiting between
// workgroups).  A gated pass, which usually does nothing, is two launches
// instead: the count's last workgroups do the scans, signalled through the
// ex.sync counters (required then: radix_sync_words(n) words, zero before a
// workspace's first gated pass; every pass leaves them zero again, and
// passes sharing them run one after another on one stream).  The key of
// element i is keys_in[i], or (keys_in == nullptr) the canonical word
// `key_word` of tuple row i.  keys_out may be null.  Every payload plane
// travels with its key.  Elements: i < (n_dev ? *n_dev : n).
// cnt: radix_count_words(n) words; group_tot: radix_group_words(n) words.
hipError_t launch_radix_pass(const uint32_t* keys_in, const TupleSrc& ts, int key_word,
                             uint32_t* keys_out, const Payload& pay, int64_t n,
                             const int32_t* n_dev, int shift, uint32_t* cnt, uint32_t* group_tot,
                             hipStream_t st, const RadixExtra& ex = RadixExtra());
inline int64_t radix_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }
// sized for every geometry: the smaller tile and the wider digit
inline int64_t radix_count_words(int64_t n) { return radix_tiles(n) * kMaxBins; }
inline int64_t radix_group_words(int64_t n) { return (radix_tiles(n) + 63) / 64 * kMaxBins; }
inline int64_t radix_sync_words(int64_t n) { return 1 + (radix_tiles(n) + 63) / 64; }

// Duplicate removal over the fully sorted order.  w0: sorted first key word;
// planes: n-strided planes [id, w1, ..., w_{k-1}] in the same order.  Writes
// the kept ids to out_ids, their words w1..w_{k-1} to out_words[(d-1) *
// out_stride + o] and the count to *nu.  cnt: radix_tiles(n) words.
hipError_t launch_dedup(const uint32_t* w0, const uint32_t* planes, const uint32_t* tree, int64_t n,
                        int k, uint32_t* out_ids, uint32_t* out_words, int64_t out_stride,
                        uint32_t* out_tree, uint32_t* cnt, int32_t* uoff, int num_trees,
                        hipStream_t st);

// Word-0-first order of array 0 (after a radix sort by word 0 and tree):
// w0 and tree (null for one tree) are the sorted key planes, planes the
// n-strided planes [row id, w1, ..., w_{k-1}].  list: kMaxTieRuns words;
// count and flag must be zero on entry; a non-zero flag asks for the full
// radix sort instead.
constexpr int kMaxTieRuns = 1 << 20;
struct TieArgs {
  const uint32_t* w0;
  const uint32_t* tree;
  uint32_t* planes;
  int k;
};
hipError_t launch_ties(const TieArgs& ta, int64_t n, int32_t* list, int32_t* count, int32_t* flag,
                       hipStream_t st);

// tree[r] = b for the rows of every tree b.
hipError_t launch_tree_ids(const int64_t* off, int num_trees, uint32_t* tree, hipStream_t st);

// After duplicate removal (uoff[b] = first distinct position of tree b, or
// INT32_MAX when the tree has none; uoff[B] = total): fixes empty trees,
// writes n_unique[b] (may be null), the deepest global level *lmax, the
// on-chip finish item prefix wgbase[0..B], and clears the work counter.
hipError_t launch_forest_finish(int32_t* uoff, int num_trees, int64_t cutover, int64_t* n_unique,
                                int32_t* lmax, int32_t* wgbase, int32_t* queue, hipStream_t st);

// dst[v][key[p]] = val[v][p] for p < *total, where key is a permutation of
// 0 .. *total - 1 already grouped by key >> 12: place_passes(n) radix passes
// on digits place_shift(0), place_shift(1), ... do that.
struct PlaceArgs {
  int nv;
  const uint32_t* val[kMaxK];
  uint32_t* dst[kMaxK];
};
hipError_t launch_place(const uint32_t* key, const PlaceArgs& pa, int64_t n, const int32_t* total,
                        uint32_t* status, hipStream_t st);
int place_passes(int64_t n);
int place_shift(int pass);

// Scatters the record planes the chain of sorts could not fill (see
// presort.hip).
hipError_t launch_complete_records(uint32_t* rec, int64_t n, int k, const int32_t* nu,
                                   hipStream_t st);

// One global partition level (depth) of every array but the split one.
// rec0 holds the level-0 records (never overwritten); b1/b2 the moved ones.
// Scratch: seginfo level_tiles(n) * level_seginfo_bytes() bytes.  With
// `status` null the level runs as count, chain and move launches (cnt
// (k-1) * level_tiles(n) 64-bit words of tile counts, carry (k-1) *
// level_tiles(n) 64-bit words); otherwise the counts are chained by
// look-back inside the move launch (status (k-1) * level_tiles(n) 64-bit
// words and tickets kMaxLevels words, both zeroed before depth 0).
// wmasks: for every array j, bits 8j .. 8j+7 = the record planes its move
// writes (the planes later levels and the on-chip finish read; an array with
// none stays put and is left out of the launch); ~0 when unknown, and then
// only the deepest level is trimmed, to what the finish reads.
constexpr int kMaxLevels = 64;
hipError_t launch_level(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1, uint32_t* b2,
                        int64_t n, int k,
                        int depth, int64_t cutover, const ForestArgs& fa, int32_t* perm,
                        void* seginfo, uint32_t* cnt, uint64_t* carry, uint64_t* status,
                        int32_t* tickets, uint64_t wmasks, int defer, hipStream_t st);
// The write masks of every global level of one tree with `levels` global
// levels (element d for depth d); defer: deferred partitioning.
void level_write_masks(int k, int levels, uint64_t* masks, int defer);
// Moves array j has taken before `depth` (levels of form 1, or 3 with defer).
int level_array_moves(int defer, int depth, int j, int k);
// Deferred partitioning of one tree (defer = 1 in launch_level and
// launch_leaf): node_rank (2^(k-1) - 1 words) receives the ranks of the nodes
// of depth `depth` (<= k-2) once array `depth` has its depth layout; key[i]
// receives the in-order bucket of element i of array j (2 <= j < k) at depth
// min(j, deepest global level), the key of the stable split that gives array
// j that layout.
hipError_t launch_node_ranks(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1,
                             uint32_t* b2, int64_t n, int k, int depth, const ForestArgs& fa,
                             uint32_t* node_rank, hipStream_t st);
hipError_t launch_defer_bucket(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1,
                               uint32_t* b2, int64_t n, int k, int j, const ForestArgs& fa,
                               const uint32_t* node_rank, uint32_t* key, hipStream_t st);
size_t level_seginfo_bytes();

// ---- level form 4: one multi-level split per level (split.hip) -----------------
// A split launch brings one array to a deeper layout (see roll_depth in
// common.hpp): the regular split of level `level` (final_j < 0), or the last
// split of array final_j to the deepest global level before the on-chip
// finish.  What it does is decided on the device from *lmax.
struct SplitJob {
  int64_t n;
  int k;
  int level;
  int final_j;
  const int32_t* uoff;   // uoff[1] = n_unique (one tree)
  const int32_t* lmax;   // deepest global level
  uint32_t* status;
  const uint32_t* med;   // median table: med[(1 << l) - 1 + c] (depth l, subarray c)
  uint32_t wmask;        // record planes the split writes
};
struct SplitInfo {
  int32_t s[8];
  int32_t e[8];
  int32_t c[8];
  int32_t np;
};
size_t split_info_bytes();
// Count, chain and move launches of one split.  info: level_tiles(n)
// SplitInfo; tval, carry: level_tiles(n) << (k - 1) words; tflag:
// level_tiles(n) words; keys: 2 * kLevelTile * level_tiles(n) bytes.
hipError_t launch_split(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1, uint32_t* b2,
                        const SplitJob& J, SplitInfo* info, uint32_t* tval, uint32_t* tflag,
                        uint32_t* carry, void* keys, hipStream_t st);
// The nodes of depth J.level: their ranks into med, their rows into perm.
hipError_t launch_split_medians(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1,
                                uint32_t* b2, const SplitJob& J, uint32_t* med, int32_t* perm,
                                hipStream_t st);
// Planes written by the split of every level (level_mask[L]) and by the final
// split of every array (final_mask[j]) of a tree with `levels` global levels.
void rolling_masks(int k, int levels, uint32_t* level_mask, uint32_t* final_mask);
inline int64_t level_tiles(int64_t n) { return (n + kLevelTile - 1) / kLevelTile; }

// LDS bytes the on-chip finish needs for a cutover C in k dimensions.
inline size_t leaf_lds_bytes(int64_t cutover, int k) {
  return (size_t)cutover * (4 + 2 + 2 + 2 * 2 * k);  // s_r0, s_side (padded to 2), s_out, s_lid
}

// On-chip finish of every subarray at the cutover depth (row ids come from
// array 0's records): a persistent grid of `blocks` workgroups (at most one
// per item).
// form: 0 = levels of form 1/2, 1 = deferred partitioning (form 3), 2 = one
// split per level (form 4); it decides which buffer holds each array.
hipError_t launch_leaf(const uint32_t* rec0, const uint32_t* rows, uint32_t* b1, uint32_t* b2,
                       int64_t n, int k,
                       int64_t cutover, const ForestArgs& fa, int32_t* perm, int64_t items_bound,
                       int blocks, int form, hipStream_t st);

// ---- the comparison builder (select.hip) -------------------------------------
// Planes P: row id, then the k canonical words (plane c at P + c * n).
struct SelJob {
  int64_t n;
  int k;
  int depth;
  const int32_t* nu;  // distinct rows (device)
  uint32_t* status;
};
struct SelState {
  uint32_t lo, cnt, digit, rank;  // rows below / in the picked bucket, its digit, median rank
};
// Global levels: subarrays of more than 2048 rows (a function of n).
int select_levels_host(int64_t n);
hipError_t launch_sel_init(const uint32_t* tuples, int k, int is_float, const uint32_t* S,
                           const int32_t* nu, int64_t n, uint32_t* P, hipStream_t st);
// One global level from planes P into Q (P then serves as scratch).  hist:
// (1 << depth) * 256 words, zero on entry and left zero; state: 1 << depth
// entries; tval, carry: level_tiles(n) 64-bit words; tflag: level_tiles(n).
hipError_t launch_sel_level(const SelJob& J, uint32_t* P, uint32_t* Q, uint32_t* hist,
                            SelState* state, uint64_t* tval, uint32_t* tflag, uint64_t* carry,
                            int32_t* perm, hipStream_t st);
// Every subarray below the global levels, finished on-chip (persistent;
// queue zero on entry).  Level d reads P0 (d even) or P1 and writes the
// other; the finish reads the one the device's last level wrote.
hipError_t launch_sel_leaf(const SelJob& J, uint32_t* P0, uint32_t* P1, int32_t* perm,
                           int32_t* queue, int64_t items_bound, hipStream_t st);

// k == 1: the in-order layout is the sorted unique order.
hipError_t launch_copy_k1(const uint32_t* S0, const ForestArgs& fa, int64_t n, int32_t* perm,
                          hipStream_t st);

// ---- learned presort (learned.hip) ----------------------------------------------

// Sample of S canonical keys per dimension (rows floor(s * n / S)); out [k][S].
hipError_t launch_cdf_sample(const uint32_t* t, int64_t n, int k, int is_float, int S, uint32_t* out,
                             hipStream_t st);
// Finite range of every column: range[2d], range[2d+1] = smallest, largest
// canonical key of dimension d among its finite values.
hipError_t launch_col_range(const uint32_t* t, int64_t n, int k, int is_float, uint32_t* range,
                            hipStream_t st);
// Train k models (one workgroup each) on the sorted samples [k][S] over the
// column ranges.
hipError_t launch_cdf_fit(const uint32_t* sorted, int S, int k, int is_float, const uint32_t* range,
                          int steps, float lr, CdfModel* models, hipStream_t st);
// Loss and gradient of the training objective on a sorted raw sample.
// keys: M words of scratch.
hipError_t launch_cdf_loss_grad(const uint32_t* raw, int M, int is_float, uint32_t lo_bits,
                                uint32_t hi_bits, const float* theta, uint32_t* keys, float* loss,
                                float* grad, hipStream_t st);
hipError_t launch_cdf_eval(const CdfModel* model, const uint32_t* raw, int M, int nb_bits, float* F,
                           int32_t* bucket, hipStream_t st);

// Bucket starts (2^nb_bits + 1 entries) of keys ordered by bucket.
hipError_t launch_bucket_bounds(const uint32_t* keys, int64_t n, const int32_t* n_dev,
                                const CdfModel* model, int nb_bits, int32_t* starts, int32_t* flag,
                                hipStream_t st);

// Planes of one bucket sort: nq planes moved from in[q] to out[q] (out may
// equal in); the sort words are planes keyq[0..nkeys-1], least significant
// first.
struct LocalSort {
  int nq;
  const uint32_t* in[kMaxPlanes];
  uint32_t* out[kMaxPlanes];
  int nkeys;
  int keyq[kMaxK];
  const CdfModel* model;  // the model the buckets were cut with
  int nb_bits;            // 2^nb_bits buckets
};
hipError_t launch_bucket_sort(const int32_t* starts, int nb_bits, int64_t n, const int32_t* n_dev,
                              int32_t* flag, const LocalSort& ls, hipStream_t st);
size_t bucket_sort_lds_bytes();
int bucket_sort_capacity();

// Strict order check of a sorted output: words w[0..nw-1] (most significant
// first), then tie.
struct CertArgs {
  int nw;
  const uint32_t* w[kMaxK];
  const uint32_t* tie;
};
hipError_t launch_certify(const CertArgs& ca, int64_t n, const int32_t* n_dev, int32_t* flag,
                          hipStream_t st);
hipError_t launch_copy_i32(const int32_t* src, int count, int32_t* dst, hipStream_t st);

// ---- queries over a built tree (queries.hip) ---------------------------------------

constexpr int kMaxNeighbors = 64;
// nodes[pos][d] = tuples[perm[pos]][d] for the *nn (device count) nodes.
hipError_t launch_gather_nodes(const void* tuples, int64_t n, int k, int is_float,
                               const int32_t* perm, const int64_t* nn, void* nodes, hipStream_t st);
// Subtree bounding boxes (n * 2k values: smallest k, then largest k) at every
// node position, from the node coordinates.
hipError_t launch_subtree_bounds(const void* nodes, int64_t n, int k, int is_float,
                                 const int64_t* nn, void* bounds, hipStream_t st);
// Box queries over the *nn nodes whose coordinates `nodes` holds in tree
// position order (bounds: their subtree boxes, or null): counts[q] (offsets ==
// null), or the rows (perm entries) of query q written from rows[offsets[q]]
// in increasing tree position (no write at or past cap).  visits: null, or a
// counter that receives the number of nodes visited.
hipError_t launch_region(const void* nodes, const void* bounds, int64_t n, int k, int is_float,
                         const int32_t* perm, const int64_t* nn, const void* lower,
                         const void* upper, int64_t nq, int32_t* counts, const int64_t* offsets,
                         int32_t* rows, int64_t cap, unsigned long long* visits, hipStream_t st);
// The m (1 .. kMaxNeighbors) nodes smallest in (squared distance, row) of
// every query point, ascending, -1 past the node count: rows[q * m + i].
// points == null: the queries are the nodes themselves (nq = n; query q is
// node position q, rows of positions past the count are left alone), and a
// node is not its own neighbour.
hipError_t launch_nearest(const void* nodes, int64_t n, int k, int is_float, const int32_t* perm,
                          const int64_t* nn, const void* points, int64_t nq, int32_t m, int32_t* rows,
                          unsigned long long* visits, hipStream_t st);

// Reverse lists from launch_nearest's all-nodes output (rows, n * m): the
// list of row r is lists[offsets[r] .. offsets[r + 1] - 1], ascending
// (offsets: n + 1 words).  ws: reverse_workspace_bytes(n) bytes.
size_t reverse_workspace_bytes(int64_t n);
hipError_t launch_reverse_nearest(const int32_t* perm, const int64_t* nn, int64_t n, int m,
                                  const int32_t* rows, int64_t* offsets, int32_t* lists, void* ws,
                                  hipStream_t st);

// Child positions from the implicit shape of a single tree (uoff[1] rows).
hipError_t launch_children(const int32_t* uoff, int64_t n, int32_t* lo, int32_t* hi,
                           hipStream_t st);

}  // namespace kd
