/*
 * kdtree.h -- C ABI of the MI355X (gfx950) presorting balanced k-d tree builder.
 *
 * The method is R. A. Brown, "Building a Balanced k-d Tree in O(kn log n)
 * Time": presort the tuples k times by the cyclic super keys (Sec. 2.1: x:y:z,
 * y:z:x, z:x:y, ...; the k = 4 forms in the Appendix, "Deferred Merge Sort and
 * Partitioning"), remove duplicate tuples in one pass (Sec. 2.1), then split
 * each subarray at the median of the array sorted in the current dimension and
 * partition the other k-1 arrays about it, keeping their order (Sec. 2.1;
 * Appendix, "Optimized Partitioning").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Tuples are n rows of k coordinates, row-major, either int32 (signed
 *    order) or float32 (IEEE-754 totalOrder: -0.0 < +0.0, NaN ordered by its
 *    bits).  Two rows are duplicates when they are bit-identical; the row
 *    with the smallest index survives (Sec. 2.1 keeps one index of each run of
 *    identical tuples; the sorts are stable).
 *  - The split dimension at depth L is L mod k; the node of a subarray [s, e]
 *    is its lower median, position s + (e - s) / 2 (the two-element rule of
 *    Sec. 3.1 makes the first element the node).
 *  - Output is the tree's in-order layout: perm[pos] = input row of the node at
 *    position pos, for pos < n_unique; entries at pos >= n_unique are left
 *    untouched.  Optional lo[pos] / hi[pos] receive the positions of the
 *    "less than" / "greater than" children, or -1.  The tree's shape depends
 *    only on n_unique.
 *  - All pointers named d_* are device memory owned by the caller; h_* are
 *    host memory.  The library never frees caller memory and allocates no
 *    device memory inside a build: it uses the caller's workspace.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL is the default
 *    stream).  Outputs are valid once the stream has synchronised.  The
 *    workspace must not be shared by builds that may run concurrently.
 *  - Arguments are validated on the host before anything is enqueued; on an
 *    error return nothing has been enqueued.  Limits: 0 <= n <= KD_MAX_N,
 *    1 <= k <= KD_MAX_K, 4-byte aligned device pointers.
 *  - Return value: KD_OK (0) or a negative KD_E* code; kd_strerror() names it.
 */
#ifndef KDTREE_H_
#define KDTREE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KD_MAX_N (((int64_t)1 << 30) - 1) /* rows per build (and per batch) */
#define KD_MAX_K 8
#define KD_MAX_TREES (1 << 20) /* trees per batched build */

enum kd_dtype { KD_I32 = 0, KD_F32 = 1 };

enum kd_status {
  KD_OK = 0,
  KD_EINVAL = -1,        /* bad argument (null, misaligned, out of range) */
  KD_ENOMEM = -2,        /* workspace smaller than kdtree_workspace_bytes() */
  KD_EHIP = -3,          /* a HIP runtime call failed */
  KD_EUNSUPPORTED = -4,  /* k or n beyond the limits above */
  KD_EINTERNAL = -5      /* kd_status(): a kernel found inconsistent counts */
};

/* Tuning knobs; pass NULL for the defaults.  They change speed only, never the
 * result. */
typedef struct kd_options {
  int32_t cutover;     /* largest subarray finished on-chip by one workgroup:
                          1024, 2048 or 4096; 0 = default (1024) */
  int32_t leaf_blocks; /* workgroups of the persistent on-chip finish:
                          0 = default (2048), else 256 .. 16384 */
  int32_t records;     /* how the level-0 rank records are completed: 0 = by
                          size, 1 = one direct scatter, 2 = radix passes on
                          the destination's high digits, then placement */
  int32_t learned_sorts; /* learned builds only: bit d set = the sort for
                          super key d goes through the learned buckets, the
                          others through the radix passes; 0 = all */
  int32_t level;       /* global partition levels: 0 = default (4 for a
                          single build of k >= 3, else 1), 1 = count,
                          chain and move launches, 2 = one move launch per
                          level whose tiles chain their counts by look-back,
                          3 = form 1 with deferred partitioning (Appendix,
                          "Deferred Merge Sort and Partitioning"): array j
                          >= 2 keeps its presorted order until depth j and
                          then reaches its depth-j layout in one stable
                          radix split by subtree instead of j moves (single
                          builds; a batch runs form 1), 4 = deferred
                          partitioning at every level: at level L only the
                          array sorted by dimension L mod k moves, in one
                          stable split by subtree about the medians of the
                          k-1 levels since it last split (single builds; a
                          batch runs form 1) */
  int32_t digit_bits;  /* radix digit width of the presort's key-word passes:
                          0 = default (8), 8 (four passes per 32-bit word)
                          or 11 (three) */
  int32_t sort_tile;   /* keys per radix tile: 0 = default (4096), 4096 or
                          8192 */
  int32_t reserved[1]; /* must be zero */
} kd_options;

/* Write masks of level form 4 for a tree with `levels` global levels
 * (host only, diagnostic; no device work): h_level_mask[L] (levels words) =
 * the record planes (bit c = plane c) the split at level L writes into the
 * array sorted by dimension L mod k; h_final_mask[j] (k words) = the planes
 * the last split of array j before the on-chip finish writes (0: none).
 * 2 <= k <= KD_MAX_K, 0 <= levels <= 30. */
int kd_level_plan(int32_t k, int32_t levels, uint32_t* h_level_mask, uint32_t* h_final_mask);

/* The plan of level forms 1 and 3 (host only, diagnostic; no device work):
 * h_masks[L] (levels words) = the record planes each array's move writes at
 * global level L, 8 bits per array (bits 8j .. 8j+7 for array j, bit c of
 * them = plane c); h_moves[d * k + j] ((levels + 1) * k words) = the number
 * of moves array j has taken before depth d, which decides the buffer that
 * holds its layout there.  defer = 1 for the deferred partitioning (form 3),
 * 0 for form 1.  2 <= k <= KD_MAX_K, 0 <= levels <= 30; KD_EINVAL on null
 * pointers or a bad defer. */
int kd_level_masks(int32_t k, int32_t levels, int32_t defer, uint64_t* h_masks, int32_t* h_moves);

/* Human-readable name of a status code (static string). */
const char* kd_strerror(int code);

/* Consistency check of the last build enqueued with this workspace (any
 * entry point that takes a build workspace).  The build's kernels clear a
 * device status word at the start of the workspace when the presort starts,
 * and a kernel that finds counts contradicting each other -- which a correct
 * build never does -- drops the write it cannot place and sets a bit there,
 * instead of writing out of bounds.  kd_status() waits for `stream`, copies
 * that word to *h_bits (0 when clean) and returns KD_EINTERNAL when a bit is
 * set, KD_OK otherwise.  Bits: 1 radix pass, 2 level tile subarrays, 4 level
 * move, 8 on-chip finish, 16 multi-level split, 32 record placement, 64 node
 * rank.  Synchronises the stream, so it is not for capture into a graph. */
int kd_status(const void* d_workspace, size_t workspace_bytes, uint32_t* h_bits, void* stream);

/* Bytes of device workspace a build of n rows in k dimensions needs.  Host
 * only; writes *h_bytes.  Returns KD_EINVAL / KD_EUNSUPPORTED on bad sizes. */
int kdtree_workspace_bytes(int64_t n, int32_t k, int32_t dtype, size_t* h_bytes);

/* Whole build (Sec. 2.1): presort by the k cyclic super keys, remove
 * duplicates, partition level by level.
 *   d_tuples    n*k int32 or float32, row-major, read only
 *   d_perm      int32[n]  in-order layout (see above)
 *   d_lo, d_hi  int32[n]  child positions, or both NULL to skip
 *   d_n_unique  int64[1]  number of distinct rows
 *   d_workspace workspace_bytes >= kdtree_workspace_bytes(n, k, dtype)
 *   opts        NULL or tuning knobs                                      */
int kdtree_build(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                 int32_t* d_lo, int32_t* d_hi, int64_t* d_n_unique, void* d_workspace,
                 size_t workspace_bytes, const kd_options* opts, void* stream);

/* kdtree_build for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same build, arguments and result, with no workspace argument.  The
 * workspace is a device array inside the library of
 * KD_NOALLOC_WORKSPACE_BYTES bytes, one per GPU, held until the process ends;
 * inputs whose kdtree_workspace_bytes() exceeds it are refused with
 * KD_ENOMEM before anything is enqueued.  The call allocates nothing and
 * never calls hipMalloc or hipFree.  Every call on a GPU uses that GPU's
 * array, so calls that may overlap on one GPU (two streams, two threads)
 * race and must be serialised by the caller; each build rewrites what it
 * reads, so nothing needs clearing between calls.  With k = 3 the largest
 * accepted n is about 450,000 rows. */
#define KD_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
int kdtree_build_noalloc(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                         int32_t* d_lo, int32_t* d_hi, int64_t* d_n_unique,
                         const kd_options* opts, void* stream);

/* The two halves of kdtree_build, for phase timing.  kdtree_presort() runs the
 * presort and duplicate removal (Sec. 2.1, first half) into the workspace and
 * writes d_n_unique; kdtree_partition() must follow on the same stream with
 * the same workspace and arguments and builds the tree (Sec. 2.1, second
 * half).  Together they do exactly what kdtree_build does. */
int kdtree_presort(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int64_t* d_n_unique,
                   void* d_workspace, size_t workspace_bytes, const kd_options* opts, void* stream);
int kdtree_partition(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                     int32_t* d_lo, int32_t* d_hi, int64_t* d_n_unique, void* d_workspace,
                     size_t workspace_bytes, const kd_options* opts, void* stream);

/* The same tree by the comparison method (Sec. 3.1, "The O(n log n)
 * Algorithm": every subarray's median is found afresh at each level and the
 * subarray partitioned about it, instead of presorting k times): array 0 is
 * sorted by its super key and its duplicates removed as in kdtree_build;
 * then, at each level, an MSD radix-select by that level's super key finds
 * every subarray's median (digit histograms, a stable three-way partition
 * by the median's digit, the candidates finished by one workgroup each) and
 * leaves the subarray partitioned with the median at its middle position;
 * subarrays of at most 2048 rows are finished in LDS.  Arguments and
 * workspace as kdtree_build (no child positions).  The result equals
 * kdtree_build's; it is a cross-check built on none of the rank records or
 * partition kernels, and the timing baseline of the paper's comparison. */
int kdtree_build_select(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t* d_perm,
                        int64_t* d_n_unique, void* d_workspace, size_t workspace_bytes,
                        const kd_options* opts, void* stream);

/* Batched build: num_trees independent trees in one sequence of launches
 * (the rows of tree b are rows offsets[b] .. offsets[b+1]-1 of d_tuples, and
 * each tree is exactly the tree kdtree_build would produce from those rows
 * alone).  The on-chip finish, where every tree of at most the cutover size is
 * built entirely, is one persistent launch whose workgroups take (tree,
 * subarray) items from a work counter.
 *   d_offsets   int64[num_trees + 1] device, non-decreasing, offsets[0] = 0
 *   h_offsets   the same values in host memory (used to size launches)
 *   d_perm      int32[offsets[B]]: tree b's in-order layout in positions
 *               offsets[b] .. offsets[b] + n_unique[b] - 1, as row indices
 *               local to the tree (0 .. n_b - 1); later positions untouched
 *   d_n_unique  int64[num_trees]
 *   d_workspace >= kdtree_workspace_bytes_batched(offsets[B], B, k, dtype)
 * Limits: 1 <= num_trees <= KD_MAX_TREES, offsets[B] <= KD_MAX_N.  Returns
 * KD_EINVAL for decreasing or non-zero-based offsets.  The tuples of all trees
 * must share k and dtype. */
int kdtree_workspace_bytes_batched(int64_t total_rows, int32_t num_trees, int32_t k, int32_t dtype,
                                   size_t* h_bytes);
int kdtree_build_batched(const void* d_tuples, const int64_t* d_offsets, const int64_t* h_offsets,
                         int32_t num_trees, int32_t k, int32_t dtype, int32_t* d_perm,
                         int64_t* d_n_unique, void* d_workspace, size_t workspace_bytes,
                         const kd_options* opts, void* stream);

/* ---- learned presort ---------------------------------------------------------
 * Not in the paper: a faster route to the same presorted arrays (Sec. 2.1).
 * Each sort sends a key straight to one of 2^b buckets through a learned
 * model of the key's cumulative distribution, orders the buckets with one or
 * two stable radix passes on the bucket number, and finishes each bucket in
 * LDS.  Because the model is monotone the result equals the radix presort bit
 * for bit; a bucket larger than the on-chip capacity, or an output that fails
 * the strict-order certificate, makes that sort fall back to the radix sort
 * on the device (no host synchronisation).  The tree is therefore always
 * exactly the tree kdtree_build produces.
 *
 * Model: per dimension, a piecewise-linear CDF over KD_CDF_SEGMENTS equal
 * segments of the column's finite value range, whose segment masses are the
 * softmax of trainable logits.  kd_cdf_train() fits them on the GPU: it
 * takes the finite range of every column, a strided sample of n_samples rows
 * (row floor(s * n / n_samples)), presorts each dimension's sample with the
 * radix passes, reads the mass of every segment off the sample's ranks, and
 * runs `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, step size lr)
 * from all-zero logits on the cross-entropy between the model's masses and
 * the sample's.  The exported levels floor every segment's mass at
 * 1/(4 n_samples) and renormalise.  A model buffer
 * holds k consecutive records of KD_CDF_MODEL_BYTES bytes:
 *   float lo, hi, scale; uint32 kmin, kmax; int32 is_float, segments;
 *   float loss; float c[KD_CDF_SEGMENTS + 1]; float theta[KD_CDF_SEGMENTS];
 *   padding.
 * c[i] is the cumulative distribution at the start of segment i (c[0] = 0,
 * c[K] = 1, non-decreasing); kmin / kmax are the order-preserving keys of lo
 * and hi.  A model trained on one data set may be reused for others of the
 * same dtype: a poor model costs speed (fallbacks), never correctness.      */
#define KD_CDF_SEGMENTS 4096
#define KD_CDF_MODEL_BYTES 33024
#define KD_CDF_MAX_SAMPLES (1 << 20)
#define KD_CDF_MAX_STEPS 100000

/* Bytes of a model buffer for k dimensions (host only). */
int kd_cdf_model_bytes(int32_t k, size_t* h_bytes);
/* Workspace bytes of kd_cdf_train (host only). */
int kd_cdf_train_workspace_bytes(int32_t k, int32_t n_samples, size_t* h_bytes);
/* Train one model per dimension on d_tuples (n >= 1 rows).  Asynchronous on
 * `stream`; writes d_models (kd_cdf_model_bytes(k) bytes, 4-byte aligned).
 * kind selects the model family: KD_CDF_PWL (0), the piecewise-linear model
 * above, is the one built; any other value (KD_CDF_MLP = 1, a small
 * multi-layer perceptron, is not built) returns KD_EUNSUPPORTED before
 * anything is enqueued.  1 <= n_samples <= KD_CDF_MAX_SAMPLES,
 * 0 <= steps <= KD_CDF_MAX_STEPS, lr > 0. */
#define KD_CDF_PWL 0
#define KD_CDF_MLP 1
int kd_cdf_train(const void* d_tuples, int64_t n, int32_t k, int32_t dtype, int32_t kind,
                 int32_t n_samples, int32_t steps, float lr, void* d_models, void* d_workspace,
                 size_t workspace_bytes, void* stream);
/* The training objective for given logits, for checking: d_values holds m
 * coordinates of `dtype` sorted ascending in the order above; lo_bits /
 * hi_bits are the raw bits of the range ends.  Writes the cross-entropy to
 * *d_loss and its gradient with respect to the K logits d_theta to d_grad
 * (K floats).  d_scratch: m words.  1 <= m <= KD_CDF_MAX_SAMPLES. */
int kd_cdf_loss_grad(const void* d_values, int32_t m, int32_t dtype, uint32_t lo_bits,
                     uint32_t hi_bits, const float* d_theta, float* d_loss, float* d_grad,
                     void* d_scratch, void* stream);
/* Evaluate one dimension's model (d_model points at its record) on m raw
 * coordinates of the model's dtype: d_F[i] = F(value i), d_bucket[i] its
 * bucket among 2^nb_bits (1 <= nb_bits <= 16). */
int kd_cdf_eval(const void* d_model, const void* d_values, int32_t m, int32_t nb_bits, float* d_F,
                int32_t* d_bucket, void* stream);

/* Workspace bytes of a learned build (host only). */
int kdtree_workspace_bytes_learned(int64_t n, int32_t k, int32_t dtype, size_t* h_bytes);
/* Build with the learned presort: arguments as kdtree_build, plus
 *   d_models     k model records (kd_cdf_train)
 *   d_fell_back  int32[k] device, or NULL: entry d receives 0 when the sort
 *                for super key d used the learned path, else a non-zero
 *                reason (1: a bucket exceeded the on-chip capacity, 2: the
 *                certificate failed, 4: inconsistent bucket bounds)
 *   d_workspace  >= kdtree_workspace_bytes_learned(n, k, dtype)
 * The output equals kdtree_build's. */
int kdtree_build_learned(const void* d_tuples, int64_t n, int32_t k, int32_t dtype,
                         const void* d_models, int32_t* d_perm, int32_t* d_lo, int32_t* d_hi,
                         int64_t* d_n_unique, int32_t* d_fell_back, void* d_workspace,
                         size_t workspace_bytes, const kd_options* opts, void* stream);
/* Presort half of kdtree_build_learned (for phase timing); follow it with
 * kdtree_partition on the same workspace. */
int kdtree_presort_learned(const void* d_tuples, int64_t n, int32_t k, int32_t dtype,
                           const void* d_models, int64_t* d_n_unique, int32_t* d_fell_back,
                           void* d_workspace, size_t workspace_bytes, const kd_options* opts,
                           void* stream);

/* ---- searches over a built tree ---------------------------------------------
 * The two searches the paper runs on its tree, batched over many queries on
 * the device (one query per thread): all nodes inside a k-dimensional
 * hyper-rectangle (Appendix, "Source Code for Optimized Algorithms": region
 * search) and the m nearest nodes of a point (Appendix, "Nearest Neighbors").
 * Both walk the implicit tree of the in-order layout (the node of [s, e] is
 * position s + (e - s) / 2 and splits on dimension depth mod k) and prune
 * with non-strict bounds: a "less than" subtree's coordinates in the split
 * dimension are <= the node's, a "greater than" subtree's are >= (equal
 * values occur when a later portion of the super key decides), so the
 * results are exactly those of a linear scan over the tree's nodes.
 * Coordinates compare as values of dtype (float32: IEEE comparisons, so
 * -0.0 == +0.0 and a NaN coordinate is never inside a box, while a NaN split
 * value prunes neither side; a node whose distance is NaN is never a
 * neighbour).
 *
 * The searches read the nodes' coordinates in tree-position order, written
 * once per tree by kd_gather_nodes: a visit is one read at the node's own
 * position, and every subtree is contiguous.
 *   d_nodes     n*k of dtype, row-major: node pos at row pos (pos < n_nodes)
 *   d_perm      int32 in-order layout from kdtree_build: the row reported for
 *               node pos is d_perm[pos]
 *   d_n_nodes   int64[1] device: the tree's node count (kdtree_build's
 *               d_n_unique), clamped to 0 .. n
 *   d_visits    uint64[1] device, or NULL: the number of nodes the queries
 *               visited is added to it (for measurement)
 * Queries are nq rows of k values of dtype, row-major; 0 <= nq <=
 * KD_MAX_QUERIES.  Asynchronous on `stream`; validation as for the builds. */
#define KD_MAX_QUERIES ((int64_t)1 << 28)
#define KD_MAX_NEIGHBORS 64

/* Node coordinates in tree-position order: d_nodes[pos][d] =
 * d_tuples[d_perm[pos]][d] for pos < n_nodes (n*k of dtype; a perm entry
 * that is not a row below n gives zeros). */
int kd_gather_nodes(const void* d_tuples, int64_t n, int32_t k, int32_t dtype,
                    const int32_t* d_perm, const int64_t* d_n_nodes, void* d_nodes, void* stream);
/* Bounding box of every subtree, at its node's position: d_bounds[pos][d] is
 * the smallest and d_bounds[pos][k + d] the largest coordinate d of the
 * subtree rooted at pos (n*2k of dtype; float subtrees that hold a NaN get
 * NaN bounds).  Optional input of the box queries: a subtree inside a box is
 * then taken whole and one outside it skipped, without visiting its nodes. */
int kd_subtree_bounds(const void* d_nodes, int64_t n, int32_t k, int32_t dtype,
                      const int64_t* d_n_nodes, void* d_bounds, void* stream);
/* Box queries, counts: d_counts[q] = number of nodes x with
 * d_lower[q][d] <= x[d] <= d_upper[q][d] for every d (int32[nq]).  d_bounds:
 * kd_subtree_bounds' output, or NULL; the result is the same. */
int kd_region_count(const void* d_nodes, const void* d_bounds, int64_t n, int32_t k, int32_t dtype,
                    const int64_t* d_n_nodes, const void* d_lower, const void* d_upper, int64_t nq,
                    int32_t* d_counts, uint64_t* d_visits, void* stream);
/* Box queries, rows: the rows of query q's nodes are written to
 * d_rows[d_offsets[q]], d_rows[d_offsets[q] + 1], ... in increasing tree
 * position (int64 d_offsets[nq], e.g. the exclusive scan of kd_region_count's
 * counts); no write goes at or past rows_capacity.  d_bounds as above. */
int kd_region_rows(const void* d_nodes, const void* d_bounds, int64_t n, int32_t k, int32_t dtype,
                   const int32_t* d_perm, const int64_t* d_n_nodes, const void* d_lower,
                   const void* d_upper, int64_t nq, const int64_t* d_offsets, int32_t* d_rows,
                   int64_t rows_capacity, uint64_t* d_visits, void* stream);
/* m nearest nodes (1 <= m <= KD_MAX_NEIGHBORS) of each query point by squared
 * Euclidean distance: exact integers for int32 coordinates, for float32 the
 * float64 sum over d = 0 .. k-1 of (x[d] - q[d])^2, each difference, square
 * and sum rounded once.  d_rows[q * m + i] (int32[nq * m]) receives the rows
 * of the m nodes smallest in (distance, row), in that order, and -1 past the
 * node count; ties in distance go to the smaller row, so the result does not
 * depend on the walk. */
int kd_nearest(const void* d_nodes, int64_t n, int32_t k, int32_t dtype, const int32_t* d_perm,
               const int64_t* d_n_nodes, const void* d_points, int64_t nq, int32_t m,
               int32_t* d_rows, uint64_t* d_visits, void* stream);

/* All-points nearest neighbours (Appendix, "Nearest Neighbors": every point
 * of the tree taken as a query point): for node position pos < n_nodes,
 * d_rows[pos * m + i] (int32[n * m]) receives the rows of the m other nodes
 * smallest in (distance, row), in that order, and -1 past n_nodes - 1; a node
 * is not its own neighbour.  Rows of positions >= n_nodes are left
 * untouched.  n <= KD_MAX_QUERIES. */
int kd_all_nearest(const void* d_nodes, int64_t n, int32_t k, int32_t dtype, const int32_t* d_perm,
                   const int64_t* d_n_nodes, int32_t m, int32_t* d_rows, uint64_t* d_visits,
                   void* stream);
/* Reverse nearest neighbours (the same Appendix section: the points to which
 * a point is a nearest neighbour) from kd_all_nearest's output: the list of
 * row r is d_lists[d_offsets[r]] .. d_lists[d_offsets[r + 1] - 1], the rows
 * of the nodes that have r among their m nearest, in ascending order.  Any
 * table of that shape is accepted (entries that are not a row below n are
 * ignored); a row may appear in at most 2^32 - 1 entries in all, which
 * kd_all_nearest's output (a row at most once per node) always meets.
 *   d_offsets   int64[n + 1] over row ids 0 .. n-1 (a row that is no node
 *               has an empty list)
 *   d_lists     int32[n * m] (at most n_nodes * m entries are written)
 *   d_workspace >= kd_reverse_workspace_bytes(n), 8-byte aligned        */
int kd_reverse_workspace_bytes(int64_t n, size_t* h_bytes);
int kd_reverse_nearest(const int32_t* d_perm, const int64_t* d_n_nodes, int64_t n, int32_t m,
                       const int32_t* d_rows, int64_t* d_offsets, int32_t* d_lists,
                       void* d_workspace, size_t workspace_bytes, void* stream);

/* ---- diagnostics ------------------------------------------------------------
 * Kernel probe for measurement tools.  kd_probe_start() makes the library
 * record a HIP event pair around every launch of one kernel class (on the
 * stream the kernel runs on) for the next `capacity` launches; kd_probe_stop()
 * waits for those events, writes up to `capacity` durations in milliseconds to
 * h_ms (host), the number recorded to *h_count, and disables the probe.  The
 * probe is process-wide state for single-threaded measurement, not for
 * concurrent builds.  Events are created by the library (host objects, no
 * device memory). */
enum kd_kernel_class {
  KD_K_ONESWEEP = 1, /* one radix scatter pass */
  KD_K_LEVEL = 2,    /* one global partition level */
  KD_K_LEAF = 3,     /* the on-chip finish */
  KD_K_DEDUP = 4,    /* duplicate removal */
  KD_K_HIST = 5,     /* digit histograms */
  KD_K_CANON = 6,    /* key canonicalisation */
  KD_K_RECORDS = 7,  /* rank tables and level-0 records */
  KD_K_BUCKET = 8,   /* learned presort: per-bucket finish */
  KD_K_TIES = 9,     /* array 0: ordering the runs of equal first words */
  KD_K_QUERY = 10    /* one batch of tree searches */
};
int kd_probe_start(int32_t kernel_class, int32_t capacity);
int kd_probe_stop(float* h_ms, int32_t* h_count);

#ifdef __cplusplus
}
#endif

#endif /* KDTREE_H_ */
