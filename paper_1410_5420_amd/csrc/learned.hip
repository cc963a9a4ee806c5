// Learned presort (not in the paper; an alternative way to produce the same
// presorted arrays as Sec. 2.1).
//
// A per-dimension CDF model F sends every key straight to one of 2^b buckets
// (b = F * 2^b, monotone in the key).  A sort then is: one or two stable
// radix passes keyed by the bucket (8-bit digits of the bucket number) that
// move every payload plane, and one workgroup per bucket that finishes the
// order in LDS with a stable LSD sort of the real key words.  Because the
// bucket passes are stable and the bucket is monotone in the key, the result
// is exactly the stable sort by the key words.  A bucket too large for LDS, or
// an output that is not strictly increasing in (key words, tie breaker),
// raises a flag, and the radix sort then runs in its place (gated on the
// flag, so nothing waits on the host).
//
// The model (common.hpp) is a piecewise-linear CDF over K = 4096 equal value
// segments.  Its parameters are logits theta of the segment masses q =
// softmax(theta); it is trained by Adam on the cross-entropy between q and
// the masses that the ranks of a presorted sample of the keys give (the mass
// of segment j is the rank of the first sample beyond it minus the rank of
// its first sample, over the sample size).  The gradient of that loss with
// respect to theta is q - p.
#include "common.hpp"
#include "launch.hpp"

namespace kd {

constexpr int kFitThreads = 1024;
constexpr int kSegPer = kCdfSegments / kFitThreads;  // segments owned by one thread
static_assert(kSegPer * kFitThreads == kCdfSegments, "thread j owns segments j*kSegPer ..");

// ---- block reductions (1024 threads, fixed order, deterministic) --------------

template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, T* s_tmp, Op op) {
  constexpr int kWaves = kFitThreads / kWave;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = op(v, __shfl_xor(v, d, kWave));
  if (lane_id() == 0) s_tmp[threadIdx.x / kWave] = v;
  __syncthreads();
  T r = s_tmp[0];
  for (int i = 1; i < kWaves; ++i) r = op(r, s_tmp[i]);
  __syncthreads();
  return r;
}

struct OpMin {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a < b ? a : b; }
};
struct OpMax {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};
struct OpAdd {
  template <typename T>
  __device__ T operator()(T a, T b) const { return a + b; }
};

__device__ __forceinline__ bool finite_key(uint32_t key, int is_float) {
  if (!is_float) return true;
  const uint32_t bits = (key & 0x80000000u) ? (key ^ 0x80000000u) : ~key;
  return ((bits >> 23) & 0xFF) != 0xFF;
}

// Domain of a model: value range [lo, hi] and their canonical keys.
struct Domain {
  float lo, hi, scale;
  uint32_t kmin, kmax;
};

__device__ __forceinline__ Domain make_domain(uint32_t kmin, uint32_t kmax, int is_float) {
  Domain dm;
  dm.kmin = kmin;
  dm.kmax = kmax;
  dm.lo = cdf_key_value(kmin, is_float);
  dm.hi = cdf_key_value(kmax, is_float);
  // in double, so that a range near the float limit cannot overflow
  dm.scale = dm.hi > dm.lo ? (float)((double)kCdfSegments / ((double)dm.hi - (double)dm.lo)) : 0.f;
  return dm;
}

// Segment of a sample key: keys at or below kmin count in segment 0, keys at
// or above kmax in segment K-1.  Non-decreasing in the key.
__device__ __forceinline__ int sample_segment(const Domain& dm, uint32_t key, int is_float) {
  if (key <= dm.kmin) return 0;
  if (key >= dm.kmax) return kCdfSegments - 1;
  float f;
  return cdf_segment(cdf_key_value(key, is_float), dm.lo, dm.scale, &f);
}

// Segment masses from the ranks of the sorted sample: the rank of the first
// sample in segment >= j is found by binary search (thread j owns segments
// j*kSegPer ..); p_j = (start_{j+1} - start_j) / S.
__device__ void segment_mass(const uint32_t* keys, int S, const Domain& dm, int is_float,
                             int32_t* s_start, float (&p)[kSegPer]) {
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) {
    const int j = threadIdx.x * kSegPer + r;
    int lo = 0, hi = S;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sample_segment(dm, keys[mid], is_float) < j)
        lo = mid + 1;
      else
        hi = mid;
    }
    s_start[j] = lo;
  }
  if (threadIdx.x == 0) s_start[kCdfSegments] = S;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) {
    const int j = threadIdx.x * kSegPer + r;
    p[r] = S > 0 ? (float)(s_start[j + 1] - s_start[j]) / (float)S : 0.f;
  }
  __syncthreads();
}

// q = softmax(theta) over the block's kCdfSegments logits.
__device__ void softmax_mass(const float (&th)[kSegPer], float* s_tmp, float (&q)[kSegPer]) {
  float mx = th[0];
#pragma unroll
  for (int r = 1; r < kSegPer; ++r) mx = fmaxf(mx, th[r]);
  mx = block_reduce(mx, s_tmp, OpMax());
  float e[kSegPer], sum = 0.f;
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) {
    e[r] = expf(th[r] - mx);
    sum += e[r];
  }
  sum = block_reduce(sum, s_tmp, OpAdd());
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) q[r] = e[r] / sum;
}

// Cross-entropy -sum_j p_j log q_j.
__device__ float cross_entropy(const float (&p)[kSegPer], const float (&q)[kSegPer], float* s_tmp) {
  float term = 0.f;
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) term += p[r] > 0.f ? -p[r] * logf(fmaxf(q[r], 1e-30f)) : 0.f;
  return block_reduce(term, s_tmp, OpAdd());
}

// ---- training -------------------------------------------------------------------

// Strided sample: sample s of dimension d is the canonical key of row
// floor(s * n / S).  out: [k][S].
__global__ void k_cdf_sample(const uint32_t* __restrict__ t, int64_t n, int k, int is_float,
                             int S, uint32_t* __restrict__ out) {
  const int64_t total = (int64_t)k * S;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int d = (int)(idx / S);
    const int64_t s = idx % S;
    const int64_t row = s * n / S;
    out[idx] = canon_word(t[row * k + d], is_float != 0);
  }
}

// Finite range of every column: range[2d] = smallest, range[2d + 1] =
// largest canonical key among the finite values of dimension d (ranges
// start as [0xFFFFFFFF, 0], which also marks a column with none).
__global__ void k_col_range(const uint32_t* __restrict__ t, int64_t n, int k, int is_float,
                            uint32_t* __restrict__ range) {
  uint32_t mn[kMaxK], mx[kMaxK];
#pragma unroll
  for (int d = 0; d < kMaxK; ++d) {
    mn[d] = 0xFFFFFFFFu;
    mx[d] = 0u;
  }
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int d = 0; d < kMaxK; ++d) {
      if (d < k) {
        const uint32_t key = canon_word(t[r * k + d], is_float != 0);
        if (finite_key(key, is_float)) {
          mn[d] = min(mn[d], key);
          mx[d] = max(mx[d], key);
        }
      }
    }
  }
#pragma unroll
  for (int d = 0; d < kMaxK; ++d) {
    if (d >= k) continue;
    uint32_t a = mn[d], b = mx[d];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      a = min(a, (uint32_t)__shfl_xor((int)a, o, kWave));
      b = max(b, (uint32_t)__shfl_xor((int)b, o, kWave));
    }
    if (lane_id() == 0) {
      atomicMin(&range[2 * d], a);
      atomicMax(&range[2 * d + 1], b);
    }
  }
}

struct AdamCfg {
  int steps;
  float lr, b1, b2, eps;
};

// One block per dimension: domain from the column's finite range, masses
// from the sorted sample's ranks, Adam from theta = 0 (the untrained model is
// the linear map of [lo, hi]), then the cumulative levels c (with a small
// mass floor).
__global__ __launch_bounds__(kFitThreads) void k_cdf_fit(const uint32_t* __restrict__ sorted,
                                                         int S, int is_float,
                                                         const uint32_t* __restrict__ range,
                                                         AdamCfg cfg,
                                                         CdfModel* __restrict__ models) {
  __shared__ float s_tmp[kFitThreads / kWave];
  __shared__ int32_t s_itmp[kFitThreads / kWave];
  __shared__ int32_t s_start[kCdfSegments + 1];
  __shared__ float s_q[kCdfSegments];
  const int d = blockIdx.x;
  const int j = threadIdx.x;
  const uint32_t* keys = sorted + (int64_t)d * S;
  CdfModel* m = models + d;

  // the domain is the column's finite range (so the tails beyond the
  // sample's extremes stay inside it)
  (void)s_itmp;
  uint32_t kmin = range[2 * d], kmax = range[2 * d + 1];
  if (kmin > kmax) kmin = kmax = 0x80000000u;  // no finite value
  const Domain dm = make_domain(kmin, kmax, is_float);
  float p[kSegPer];
  segment_mass(keys, S, dm, is_float, s_start, p);

  float th[kSegPer], m1[kSegPer], m2[kSegPer], q[kSegPer];
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) th[r] = m1[r] = m2[r] = 0.f;
  float b1t = 1.f, b2t = 1.f;
  for (int step = 0; step < cfg.steps; ++step) {
    softmax_mass(th, s_tmp, q);
    b1t *= cfg.b1;
    b2t *= cfg.b2;
#pragma unroll
    for (int r = 0; r < kSegPer; ++r) {
      const float g = q[r] - p[r];
      m1[r] = cfg.b1 * m1[r] + (1.f - cfg.b1) * g;
      m2[r] = cfg.b2 * m2[r] + (1.f - cfg.b2) * g * g;
      const float mh = m1[r] / (1.f - b1t);
      const float vh = m2[r] / (1.f - b2t);
      th[r] -= cfg.lr * mh / (sqrtf(vh) + cfg.eps);
    }
  }
  softmax_mass(th, s_tmp, q);
  const float loss = cross_entropy(p, q, s_tmp);
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) {
    s_q[j * kSegPer + r] = q[r];
    m->theta[j * kSegPer + r] = th[r];
  }
  __syncthreads();
  if (j == 0) {
    // Levels: every segment keeps a mass of at least 1/(4S) (regions the
    // sample missed still spread over a slice of buckets), renormalised; a
    // sequential cumulative sum is non-decreasing by construction.
    const float floor_mass = S > 0 ? 0.25f / (float)S : 0.f;
    const float norm = 1.f / (1.f + (float)kCdfSegments * floor_mass);
    float run = 0.f;
    for (int i = 0; i < kCdfSegments; ++i) {
      m->c[i] = fminf(run, 1.f);
      run += (s_q[i] + floor_mass) * norm;
    }
    m->c[kCdfSegments] = 1.f;
    m->lo = dm.lo;
    m->hi = dm.hi;
    m->scale = dm.scale;
    m->kmin = dm.kmin;
    m->kmax = dm.kmax;
    m->is_float = is_float;
    m->segments = kCdfSegments;
    m->loss = loss;
  }
}

// Loss and gradient for given parameters on a sorted sample of raw
// coordinates (the functions the training loop uses, exposed for checking).
__global__ __launch_bounds__(kFitThreads) void k_cdf_loss_grad(const uint32_t* __restrict__ raw,
                                                               int M, int is_float,
                                                               uint32_t lo_bits, uint32_t hi_bits,
                                                               const float* __restrict__ theta,
                                                               uint32_t* __restrict__ keys,
                                                               float* __restrict__ loss,
                                                               float* __restrict__ grad) {
  __shared__ float s_tmp[kFitThreads / kWave];
  __shared__ int32_t s_start[kCdfSegments + 1];
  for (int i = threadIdx.x; i < M; i += kFitThreads) keys[i] = canon_word(raw[i], is_float != 0);
  __syncthreads();
  const Domain dm = make_domain(canon_word(lo_bits, is_float != 0), canon_word(hi_bits, is_float != 0),
                                is_float);
  float p[kSegPer], th[kSegPer], q[kSegPer];
  segment_mass(keys, M, dm, is_float, s_start, p);
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) th[r] = theta[threadIdx.x * kSegPer + r];
  softmax_mass(th, s_tmp, q);
  const float L = cross_entropy(p, q, s_tmp);
#pragma unroll
  for (int r = 0; r < kSegPer; ++r) grad[threadIdx.x * kSegPer + r] = q[r] - p[r];
  if (threadIdx.x == 0) *loss = L;
}

// F and bucket of raw coordinates under one dimension's model.
__global__ void k_cdf_eval(const CdfModel* __restrict__ model, const uint32_t* __restrict__ raw,
                           int M, int nb_bits, float* __restrict__ F, int32_t* __restrict__ bucket) {
  __shared__ float s_c[kCdfSegments + 1];
  for (int q = threadIdx.x; q <= kCdfSegments; q += blockDim.x) s_c[q] = model->c[q];
  __syncthreads();
  const int is_float = model->is_float;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) {
    const uint32_t key = canon_word(raw[i], is_float != 0);
    const float f = cdf_eval(s_c, model->lo, model->scale, model->kmin, model->kmax, is_float, key);
    F[i] = f;
    bucket[i] = (int32_t)cdf_bucket(f, nb_bits);
  }
}

hipError_t launch_cdf_sample(const uint32_t* t, int64_t n, int k, int is_float, int S, uint32_t* out,
                             hipStream_t st) {
  const int64_t total = (int64_t)k * S;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_cdf_sample, dim3((unsigned)blocks), dim3(256), 0, st, t, n, k, is_float, S,
                     out);
  return hipGetLastError();
}

hipError_t launch_col_range(const uint32_t* t, int64_t n, int k, int is_float, uint32_t* range,
                            hipStream_t st) {
  hipError_t e = launch_fill_u32(range, 0u, 2 * k, st);  // maxima start at 0
  if (e != hipSuccess) return e;
  for (int d = 0; d < k; ++d) {
    e = launch_fill_u32(range + 2 * d, 0xFFFFFFFFu, 1, st);  // minima at the top
    if (e != hipSuccess) return e;
  }
  int64_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_col_range, dim3((unsigned)blocks), dim3(256), 0, st, t, n, k, is_float, range);
  return hipGetLastError();
}

hipError_t launch_cdf_fit(const uint32_t* sorted, int S, int k, int is_float, const uint32_t* range,
                          int steps, float lr, CdfModel* models, hipStream_t st) {
  AdamCfg cfg{steps, lr, 0.9f, 0.999f, 1e-8f};
  hipLaunchKernelGGL(k_cdf_fit, dim3(k), dim3(kFitThreads), 0, st, sorted, S, is_float, range, cfg,
                     models);
  return hipGetLastError();
}

hipError_t launch_cdf_loss_grad(const uint32_t* raw, int M, int is_float, uint32_t lo_bits,
                                uint32_t hi_bits, const float* theta, uint32_t* keys, float* loss,
                                float* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_cdf_loss_grad, dim3(1), dim3(kFitThreads), 0, st, raw, M, is_float, lo_bits,
                     hi_bits, theta, keys, loss, grad);
  return hipGetLastError();
}

hipError_t launch_cdf_eval(const CdfModel* model, const uint32_t* raw, int M, int nb_bits, float* F,
                           int32_t* bucket, hipStream_t st) {
  int blocks = (M + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_cdf_eval, dim3(blocks), dim3(256), 0, st, model, raw, M, nb_bits, F, bucket);
  return hipGetLastError();
}

// ---- bucket sort ------------------------------------------------------------------

// starts[b] = first position of bucket b in an array already ordered by bucket
// (positions 0 .. nu-1), starts[2^nb_bits] = nu.  Every entry is written
// exactly once: the thread at position i writes the starts of the buckets
// after its predecessor's, up to its own.  A bucket sequence that decreases
// (which the bucket passes rule out) raises flag bit 4.
__global__ void k_bucket_bounds(const uint32_t* __restrict__ keys, int64_t n_host,
                                const int32_t* n_dev, const CdfModel* __restrict__ model,
                                int nb_bits, int32_t* __restrict__ starts,
                                int32_t* __restrict__ flag) {
  __shared__ float s_c[kCdfSegments + 1];
  for (int q = threadIdx.x; q <= kCdfSegments; q += blockDim.x) s_c[q] = model->c[q];
  __syncthreads();
  const int nu = (int)(n_dev ? *n_dev : n_host);
  const int NB = 1 << nb_bits;
  const float lo = model->lo, scale = model->scale;
  const uint32_t kmin = model->kmin, kmax = model->kmax;
  const int is_float = model->is_float;
  const int stride = gridDim.x * blockDim.x;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (nu <= 0) {
    for (int b = gid; b <= NB; b += stride) starts[b] = 0;
    return;
  }
  // kBbBatch positions per thread and round, their keys and their
  // predecessors' loaded together (one round trip per round, not per key)
  constexpr int kBbBatch = 8;
  for (int i0 = gid; i0 < nu; i0 += kBbBatch * stride) {
    uint32_t kc[kBbBatch], kp[kBbBatch];
#pragma unroll
    for (int j = 0; j < kBbBatch; ++j) {
      const int i = min(i0 + j * stride, nu - 1);
      kc[j] = keys[i];
      kp[j] = keys[max(i - 1, 0)];
    }
#pragma unroll
    for (int j = 0; j < kBbBatch; ++j) {
      const int i = i0 + j * stride;
      if (i >= nu) break;
      const int b = (int)cdf_bucket(cdf_eval(s_c, lo, scale, kmin, kmax, is_float, kc[j]), nb_bits);
      const int pb =
          i == 0 ? -1 : (int)cdf_bucket(cdf_eval(s_c, lo, scale, kmin, kmax, is_float, kp[j]), nb_bits);
      if (b < pb) atomicOr(flag, 4);
      for (int bb = pb + 1; bb <= b; ++bb) starts[bb] = i;
      if (i == nu - 1)
        for (int bb = b + 1; bb <= NB; ++bb) starts[bb] = nu;
    }
  }
}

hipError_t launch_bucket_bounds(const uint32_t* keys, int64_t n, const int32_t* n_dev,
                                const CdfModel* model, int nb_bits, int32_t* starts, int32_t* flag,
                                hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_bucket_bounds, dim3((unsigned)blocks), dim3(256), 0, st, keys, n, n_dev, model,
                     nb_bits, starts, flag);
  return hipGetLastError();
}

constexpr int kBsThreads = 512;
constexpr int kBsWaves = kBsThreads / kWave;
constexpr int kBsCap = 4096;      // most keys a workgroup sorts at once (two workgroups per CU)
constexpr int kBsItems = kBsCap / kBsThreads;
constexpr int kBsMaxBins = kBsCap / 2;  // CDF interpolation bins per unit (plus up to half as many tail bins)
constexpr int kBsWorkPerKey = 64;  // most element comparisons per key of a unit (sum of squared bin sizes)
constexpr int kBsPrefetch = 3;    // output planes loaded into registers while the unit sorts
constexpr int kBsLdsTies = 1;     // tie-break words held in LDS (later ones are read from memory)

// primary word and one tie-break word (both reused as output staging), the
// bin order, the sorted order and every slot's bin
size_t bucket_sort_lds_bytes() { return (size_t)kBsCap * (4 * (1 + kBsLdsTies) + 3 * 2); }
int bucket_sort_capacity() { return kBsCap; }
int bucket_sort_target() { return kBsCap * 3 / 4; }

template <typename T, typename Op>
__device__ __forceinline__ T bs_reduce(T v, T* s_red, Op op) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = op(v, __shfl_xor(v, d, kWave));
  if (lane_id() == 0) s_red[threadIdx.x / kWave] = v;
  __syncthreads();
  T r = s_red[0];
  for (int i = 1; i < kBsWaves; ++i) r = op(r, s_red[i]);
  __syncthreads();
  return r;
}

// Element i of a kernel-argument array without dynamic indexing (a chain of
// selects), so the argument block stays in scalar registers.
template <typename T, int N>
__device__ __forceinline__ T pick(const T (&arr)[N], int i) {
  T r = arr[0];
#pragma unroll
  for (int t = 1; t < N; ++t) r = i == t ? arr[t] : r;
  return r;
}

// The model as the bucket sort reads it.
struct ModelLds {
  const float* c;
  float lo, hi, scale;
  uint32_t kmin, kmax;
  int is_float;
  float nbf;  // number of buckets, 2^nb_bits
};

// Interpolation bins of a unit of buckets [b0, b0 + nbk): keys inside the
// model's domain use their position F * 2^nb_bits - b0 in the model's CDF
// space (where the model has spread keys evenly); keys at or below kmin (only
// in bucket 0) and at or above kmax (only in the last bucket) all have F = 0
// or 1, so they get bins of their own, cut by value between the unit's
// extreme and the domain's end.  The layout [low tail | CDF bins | high tail]
// is monotone non-decreasing in the key; NaN keys go to the outermost bins.
struct UnitBins {
  float fb0, fscale;         // CDF bins
  int nlo, nmid, nhi;        // bins per region
  float vmin, lo_scale;      // low tail: (value - vmin) * lo_scale
  float hi, hi_scale;        // high tail: (value - hi) * hi_scale
};

__device__ __forceinline__ int tail_bin(float t, int nt) {
  if (t >= 0.f) return t < (float)nt ? (int)t : nt - 1;
  return t < 0.f ? 0 : nt - 1;  // t is NaN: the last bin
}

__device__ __forceinline__ int interp_bin(const ModelLds& m, const UnitBins& u, uint32_t v) {
#pragma clang fp contract(off)
  if (v <= m.kmin && u.nlo > 0) {
    const float t = (cdf_key_value(v, m.is_float) - u.vmin) * u.lo_scale;
    if (t != t) return 0;  // NaN: the lowest keys
    return tail_bin(t, u.nlo);
  }
  if (v >= m.kmax && u.nhi > 0) return u.nlo + u.nmid + tail_bin((cdf_key_value(v, m.is_float) - u.hi) * u.hi_scale, u.nhi);
  if (v <= m.kmin) return u.nlo;
  if (v >= m.kmax) return u.nlo + u.nmid - 1;
  // the model's F in double precision: a bucket of 2^-16 of the CDF holds
  // only a few hundred single-precision values of F near 1
  const double t = ((double)cdf_key_value(v, m.is_float) - (double)m.lo) * (double)m.scale;
  int i = t < (double)kCdfSegments ? (int)t : kCdfSegments - 1;
  if (i < 0) i = 0;
  double f = t - (double)i;
  f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
  const double a = m.c[i], b = m.c[i + 1];
  double F = a + f * (b - a);
  F = F < b ? F : b;
  const double x = (F * (double)m.nbf - u.fb0) * u.fscale;
  int bin = 0;
  if (x >= 0.0) bin = x < (double)u.nmid ? (int)x : u.nmid - 1;
  return u.nlo + bin;
}

// Sort positions [s, s + N) (N <= kBsCap), which hold the buckets [bk0,
// bk0 + nbk), stably by the sort words and write every plane permuted.
// Elements are placed in bin order first ("slots"), with the primary and
// first tie word copied into slot order so that ranking reads them in
// sequence; s_perm[slot] is the element (its input position, the final tie).
// Returns false (after raising flag bit 8) when the bins are too uneven for
// the ranking step.
__device__ bool sort_unit(const LocalSort& ls, const ModelLds& m, int s, int N, int bk0, int nbk,
                          uint32_t* s_k, uint32_t* s_t1, uint16_t* s_perm, uint16_t* s_ord,
                          uint16_t* s_bin, uint32_t* s_cnt, uint32_t* s_tmp, uint32_t* s_red,
                          int32_t* flag) {
  const int tid = threadIdx.x;
  const int nk = ls.nkeys;
  const uint32_t* k0 = pick(ls.in, pick(ls.keyq, nk - 1)) + s;
  const uint32_t* w1 = nk >= 2 ? pick(ls.in, pick(ls.keyq, nk - 2)) + s : nullptr;
  // the first planes that are not sort words held in LDS are loaded now, so
  // their loads overlap the sort
  int pq[kBsPrefetch] = {-1, -1, -1};
  {
    int r = 0;
    for (int q = 0; q < ls.nq && r < kBsPrefetch; ++q) {
      const uint32_t* in = pick(ls.in, q) + s;
      if (in == k0 || (w1 && in == w1)) continue;
      pq[r++] = q;
    }
  }
  uint32_t pre[kBsPrefetch][kBsItems];
#pragma unroll
  for (int r = 0; r < kBsPrefetch; ++r) {
    const uint32_t* in = pq[r] >= 0 ? pick(ls.in, pq[r]) + s : nullptr;
#pragma unroll
    for (int j = 0; j < kBsItems; ++j) {
      const int i = tid + j * kBsThreads;
      pre[r][j] = (in && i < N) ? in[i] : 0u;
    }
  }
  UnitBins u;
  u.nmid = 1;
  while (u.nmid < kBsMaxBins && 2 * u.nmid < N) u.nmid <<= 1;
  u.fb0 = (float)bk0;
  u.fscale = (float)u.nmid / (float)nbk;
  const bool lowend = bk0 == 0, highend = bk0 + nbk == (int)m.nbf;
  u.nlo = lowend ? max(1, u.nmid / 4) : 0;
  u.nhi = highend ? max(1, u.nmid / 4) : 0;
  u.vmin = u.hi = 0.f;
  u.lo_scale = u.hi_scale = 0.f;
  // every thread owns elements tid + j * kBsThreads: their primary and first
  // tie words, bins and slots stay in registers
  uint32_t kv[kBsItems], tv[kBsItems];
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
#pragma unroll
  for (int j = 0; j < kBsItems; ++j) {
    const int i = tid + j * kBsThreads;
    kv[j] = i < N ? k0[i] : 0u;
    tv[j] = (w1 && i < N) ? w1[i] : 0u;
  }
#pragma unroll
  for (int j = 0; j < kBsItems; ++j) {
    if (tid + j * kBsThreads < N) {
      mn = min(mn, kv[j]);
      mx = max(mx, kv[j]);
    }
  }
  if (lowend || highend) {
    mn = bs_reduce(mn, s_red, OpMin());
    mx = bs_reduce(mx, s_red, OpMax());
    u.vmin = cdf_key_value(mn, m.is_float);
    u.hi = m.hi;
    const float vmax = cdf_key_value(mx, m.is_float);
    if (m.lo > u.vmin) u.lo_scale = (float)((double)u.nlo / (((double)m.lo - (double)u.vmin) * (1.0 + 1e-6)));
    if (vmax > m.hi) u.hi_scale = (float)((double)u.nhi / (((double)vmax - (double)m.hi) * (1.0 + 1e-6)));
  }
  const int nbins = u.nlo + u.nmid + u.nhi;
  for (int b = tid; b < nbins; b += kBsThreads) s_cnt[b] = 0;
  int bin[kBsItems];
#pragma unroll
  for (int j = 0; j < kBsItems; ++j)
    bin[j] = tid + j * kBsThreads < N ? interp_bin(m, u, kv[j]) : 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kBsItems; ++j)
    if (tid + j * kBsThreads < N) atomicAdd(&s_cnt[bin[j]], 1u);
  __syncthreads();
  // exclusive bin starts (each thread scans a run of consecutive bins), and
  // the ranking work: the sum of the squared bin sizes
  const int per = (nbins + kBsThreads - 1) / kBsThreads;
  const int b0 = min(nbins, tid * per), b1 = min(nbins, b0 + per);
  uint32_t run = 0, work = 0;
  for (int b = b0; b < b1; ++b) {
    const uint32_t c = s_cnt[b];
    run += c;
    work += c > 1 ? c * c : 0u;
  }
  uint32_t all, all_work;
  uint32_t off = block_exclusive_sum<kBsThreads>(run, s_tmp, &all);
  block_exclusive_sum<kBsThreads>(work, s_tmp, &all_work);
  if (all_work > (uint32_t)kBsWorkPerKey * (uint32_t)N) {
    if (tid == 0) atomicOr(flag, 8);
    return false;
  }
  for (int b = b0; b < b1; ++b) {
    const uint32_t c = s_cnt[b];
    s_cnt[b] = off;
    off += c;
  }
  __syncthreads();
  int slot[kBsItems];
#pragma unroll
  for (int j = 0; j < kBsItems; ++j) {
    const int i = tid + j * kBsThreads;
    slot[j] = -1;
    if (i >= N) continue;
    const uint32_t pos = atomicAdd(&s_cnt[bin[j]], 1u);
    if (pos < (uint32_t)N) {
      slot[j] = (int)pos;
      s_perm[pos] = (uint16_t)i;
      s_bin[pos] = (uint16_t)bin[j];
      s_k[pos] = kv[j];
      s_t1[pos] = tv[j];
    } else {
      atomicOr(flag, 4);  // inconsistent counts (cannot happen)
    }
  }
  __syncthreads();
  // s_cnt[b] is now the end of bin b.  Every slot ranks its element among its
  // bin's (slots of a bin are neighbours, so a wave's slots mostly share the
  // same few bins and loop about as long as each other): the element goes to
  // bin start + the number of the bin's elements before it in the total order
  // (primary word, tie words, input position).
#pragma unroll
  for (int j = 0; j < kBsItems; ++j) {
    const int p = tid + j * kBsThreads;
    if (p >= N) continue;
    const int b = s_bin[p];
    const int st = b ? (int)s_cnt[b - 1] : 0;
    const int en = (int)s_cnt[b];
    int r = 0;
    if (en - st > 1) {
      const uint32_t kx = s_k[p], tx = s_t1[p];
      const int x = s_perm[p];
      for (int q = st; q < en; ++q) {
        const uint32_t ky = s_k[q], ty = s_t1[q];
        bool lt = ky < kx || (ky == kx && ty < tx);
        if (ky == kx && ty == tx && q != p) {
          const int y = s_perm[q];
          int c = 0;
          for (int t = nk - 3; t >= 0 && c == 0; --t) {
            const uint32_t* w = pick(ls.in, pick(ls.keyq, t)) + s;
            const uint32_t a = w[y], bb = w[x];
            c = a < bb ? -1 : (a > bb ? 1 : 0);
          }
          lt = c < 0 || (c == 0 && y < x);
        }
        r += lt ? 1 : 0;
      }
    }
    s_ord[st + r] = (uint16_t)p;
  }
  // every plane permuted: the sort words straight from LDS, then the
  // prefetched planes, then the rest, two at a time through the LDS arrays
  // (staged in slot order)
  __syncthreads();
  for (int q = 0; q < ls.nq; ++q) {
    const uint32_t* in = pick(ls.in, q) + s;
    const uint32_t* src = in == k0 ? s_k : (w1 && in == w1 ? s_t1 : nullptr);
    if (!src) continue;
    uint32_t* out = pick(ls.out, q) + s;
    for (int i = tid; i < N; i += kBsThreads) out[i] = src[s_ord[i]];
  }
  __syncthreads();
  uint32_t* stage[2] = {s_k, s_t1};
#pragma unroll
  for (int r0 = 0; r0 < kBsPrefetch; r0 += 2) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = r0 + h;
      if (r >= kBsPrefetch || pq[r] < 0) continue;
#pragma unroll
      for (int j = 0; j < kBsItems; ++j)
        if (slot[j] >= 0) stage[h][slot[j]] = pre[r][j];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = r0 + h;
      if (r >= kBsPrefetch || pq[r] < 0) continue;
      uint32_t* out = pick(ls.out, pq[r]) + s;
      for (int i = tid; i < N; i += kBsThreads) out[i] = stage[h][s_ord[i]];
    }
    __syncthreads();
  }
  int r = 0;
  int rest[2];
  for (int q = 0; q <= ls.nq; ++q) {
    bool take = false;
    if (q < ls.nq) {
      const uint32_t* in = pick(ls.in, q) + s;
      const bool in_lds = in == k0 || (w1 && in == w1);
      take = !in_lds && q != pq[0] && q != pq[1] && q != pq[2];
    }
    if (take) rest[r++] = q;
    if (r == 2 || (q == ls.nq && r > 0)) {
      for (int x = 0; x < r; ++x) {
        const uint32_t* in = pick(ls.in, rest[x]) + s;
#pragma unroll
        for (int j = 0; j < kBsItems; ++j) {
          const int i = tid + j * kBsThreads;
          if (slot[j] >= 0) stage[x][slot[j]] = in[i];
        }
      }
      __syncthreads();
      for (int x = 0; x < r; ++x) {
        uint32_t* out = pick(ls.out, rest[x]) + s;
        for (int i = tid; i < N; i += kBsThreads) out[i] = stage[x][s_ord[i]];
      }
      __syncthreads();
      r = 0;
    }
  }
  return true;
}

// Workgroup g takes buckets [g * G, (g + 1) * G).  Buckets are already in
// order, so consecutive buckets sort as one unit; the workgroup packs them
// into units of at most kBsCap keys.  The bucket's elements arrive in stable
// order (the bucket passes are stable), and each unit comes out stably
// sorted by the sort words ls.keyq (least significant first), i.e. by the
// total order (primary word, the other words from most to least significant,
// position):
//   1. the primary word (and two tie words) go to LDS;
//   2. an interpolation step in the model's CDF space, where keys are close
//      to uniform: about two keys per bin, bin = (F * 2^b - first bucket) *
//      bins / buckets (keys outside the model's domain: by value), counted
//      and scattered with LDS atomics;
//   3. the keys are copied into bin order (slots); every slot's key is
//      ranked by counting the keys of its bin that precede it in the total
//      order above (primary and first tie word from LDS, later tie words
//      from memory only on a full tie);
//   4. every plane is written permuted: the sort words straight from LDS,
//      the others staged through LDS (so an output may be its input), the
//      first three of them loaded into registers before the sort.
// A bucket beyond kBsCap raises flag bit 1, and bins so uneven that the
// ranking would exceed kBsWorkPerKey comparisons per key (the sum of the
// squared bin sizes) bit 8: the caller's radix sort then runs instead.
__global__ __launch_bounds__(kBsThreads) void k_bucket_sort(const int32_t* __restrict__ starts,
                                                            int nb, int group, int64_t n_host,
                                                            const int32_t* n_dev,
                                                            int32_t* __restrict__ flag,
                                                            const LocalSort ls) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  uint32_t* s_k = reinterpret_cast<uint32_t*>(s_raw);
  uint32_t* s_t1 = s_k + kBsCap;
  uint16_t* s_perm = reinterpret_cast<uint16_t*>(s_t1 + kBsCap);
  uint16_t* s_ord = s_perm + kBsCap;
  uint16_t* s_bin = s_ord + kBsCap;
  __shared__ uint32_t s_cnt[kBsMaxBins + kBsMaxBins / 2];
  static_assert(kBsMaxBins + kBsMaxBins / 2 <= 65536, "bins fit 16 bits");
  __shared__ uint32_t s_tmp[kBsWaves + 1];
  __shared__ uint32_t s_red[kBsWaves];
  __shared__ int32_t s_flag;

  // Other workgroups of this launch may raise the flag while this one reads
  // it, so one thread reads it and the block follows that one value.
  const int tid = threadIdx.x;
  if (tid == 0) s_flag = *flag;
  __syncthreads();
  if (s_flag != 0) return;
  ModelLds m;
  m.c = ls.model->c;  // read through the caches (the table is 16 KiB)
  m.lo = ls.model->lo;
  m.hi = ls.model->hi;
  m.scale = ls.model->scale;
  m.kmin = ls.model->kmin;
  m.kmax = ls.model->kmax;
  m.is_float = ls.model->is_float;
  m.nbf = (float)(1 << ls.nb_bits);
  const int nu = (int)(n_dev ? *n_dev : n_host);
  const int g0 = blockIdx.x * group, g1 = min(nb, g0 + group);
  int b = g0;
  while (b < g1) {
    // the longest run of buckets from b that fits
    const int s = starts[b];
    int e = starts[b + 1];
    if (s < 0 || e < s || e > nu) {
      if (tid == 0) atomicOr(flag, 4);
      return;
    }
    if (e - s > kBsCap) {
      if (tid == 0) atomicOr(flag, 1);
      return;
    }
    int nb2 = b + 1;
    while (nb2 < g1) {
      const int e2 = starts[nb2 + 1];
      if (e2 < e || e2 > nu || e2 - s > kBsCap) break;
      e = e2;
      ++nb2;
    }
    if (e > s && !sort_unit(ls, m, s, e - s, b, nb2 - b, s_k, s_t1, s_perm, s_ord, s_bin, s_cnt,
                            s_tmp, s_red, flag))
      return;
    b = nb2;
  }
}

hipError_t launch_bucket_sort(const int32_t* starts, int nb_bits, int64_t n, const int32_t* n_dev,
                              int32_t* flag, const LocalSort& ls, hipStream_t st) {
  const size_t lds = bucket_sort_lds_bytes();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bucket_sort),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int nb = 1 << nb_bits;
  // about half the capacity per workgroup on average
  const int64_t mean = n / nb + 1;
  int group = (int)((bucket_sort_target() + mean / 2) / mean);
  if (group < 1) group = 1;
  if (group > nb) group = nb;
  const int grid = (nb + group - 1) / group;
  hipLaunchKernelGGL(k_bucket_sort, dim3(grid), dim3(kBsThreads), lds, st, starts, nb, group, n,
                     n_dev, flag, ls);
  return hipGetLastError();
}

// Certificate: positions i-1, i must be strictly increasing in (words, MSW
// first; then tie).  A violation raises flag bit 2.
__global__ void k_certify(const CertArgs ca, int64_t n_host, const int32_t* n_dev,
                          int32_t* __restrict__ flag) {
  if (*flag != 0) return;  // already falling back
  const int nu = (int)(n_dev ? *n_dev : n_host);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x + 1; i < nu; i += gridDim.x * blockDim.x) {
    int c = 0;
    for (int q = 0; q < ca.nw && c == 0; ++q) {
      const uint32_t* wq = pick(ca.w, q);
      const uint32_t x = wq[i - 1], y = wq[i];
      c = x < y ? -1 : (x > y ? 1 : 0);
    }
    if (c == 0) c = ca.tie[i - 1] < ca.tie[i] ? -1 : 1;
    if (c > 0) atomicOr(flag, 2);
  }
}

hipError_t launch_certify(const CertArgs& ca, int64_t n, const int32_t* n_dev, int32_t* flag,
                          hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_certify, dim3((unsigned)blocks), dim3(256), 0, st, ca, n, n_dev, flag);
  return hipGetLastError();
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int count, int32_t* __restrict__ dst) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = src[i];
}

hipError_t launch_copy_i32(const int32_t* src, int count, int32_t* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_i32, dim3(1), dim3(64), 0, st, src, count, dst);
  return hipGetLastError();
}

}  // namespace kd
