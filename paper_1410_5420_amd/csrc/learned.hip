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
// The model (common.hpp) is a piecewise-linear CDF over K = 1024 equal value
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
static_assert(kFitThreads == kCdfSegments, "thread j owns segment j");

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

// Segment masses from the ranks of the sorted sample: thread j finds the rank
// of the first sample in segment >= j; p_j = (start_{j+1} - start_j) / S.
__device__ float segment_mass(const uint32_t* keys, int S, const Domain& dm, int is_float,
                              int32_t* s_start) {
  const int j = threadIdx.x;
  int lo = 0, hi = S;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sample_segment(dm, keys[mid], is_float) < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  s_start[j] = lo;
  if (j == 0) s_start[kCdfSegments] = S;
  __syncthreads();
  const float p = S > 0 ? (float)(s_start[j + 1] - s_start[j]) / (float)S : 0.f;
  __syncthreads();
  return p;
}

// q_j = softmax(theta)_j over the block (thread j holds theta_j).
__device__ float softmax_mass(float th, float* s_tmp) {
  const float mx = block_reduce(th, s_tmp, OpMax());
  const float e = expf(th - mx);
  const float sum = block_reduce(e, s_tmp, OpAdd());
  return e / sum;
}

// Cross-entropy -sum_j p_j log q_j.
__device__ float cross_entropy(float p, float q, float* s_tmp) {
  const float term = p > 0.f ? -p * logf(fmaxf(q, 1e-30f)) : 0.f;
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

struct AdamCfg {
  int steps;
  float lr, b1, b2, eps;
};

// One block per dimension: domain from the sorted sample, masses from its
// ranks, Adam from theta = 0 (the untrained model is the linear map of
// [lo, hi]), then the cumulative levels c.
__global__ __launch_bounds__(kFitThreads) void k_cdf_fit(const uint32_t* __restrict__ sorted,
                                                         int S, int is_float, AdamCfg cfg,
                                                         CdfModel* __restrict__ models) {
  __shared__ float s_tmp[kFitThreads / kWave];
  __shared__ int32_t s_itmp[kFitThreads / kWave];
  __shared__ int32_t s_start[kCdfSegments + 1];
  __shared__ float s_q[kCdfSegments];
  const int d = blockIdx.x;
  const int j = threadIdx.x;
  const uint32_t* keys = sorted + (int64_t)d * S;
  CdfModel* m = models + d;

  // finite range of the sample (NaN and infinities sit at the two ends)
  int first = S, last = -1;
  for (int i = j; i < S; i += kFitThreads) {
    if (finite_key(keys[i], is_float)) {
      first = min(first, i);
      last = max(last, i);
    }
  }
  first = block_reduce(first, s_itmp, OpMin());
  last = block_reduce(last, s_itmp, OpMax());
  uint32_t kmin = 0x80000000u, kmax = 0x80000000u;
  if (last >= 0) {
    kmin = keys[first];
    kmax = keys[last];
  }
  const Domain dm = make_domain(kmin, kmax, is_float);
  const float p = segment_mass(keys, S, dm, is_float, s_start);

  float th = 0.f, m1 = 0.f, m2 = 0.f, b1t = 1.f, b2t = 1.f;
  for (int step = 0; step < cfg.steps; ++step) {
    const float q = softmax_mass(th, s_tmp);
    const float g = q - p;
    m1 = cfg.b1 * m1 + (1.f - cfg.b1) * g;
    m2 = cfg.b2 * m2 + (1.f - cfg.b2) * g * g;
    b1t *= cfg.b1;
    b2t *= cfg.b2;
    const float mh = m1 / (1.f - b1t);
    const float vh = m2 / (1.f - b2t);
    th -= cfg.lr * mh / (sqrtf(vh) + cfg.eps);
  }
  const float q = softmax_mass(th, s_tmp);
  const float loss = cross_entropy(p, q, s_tmp);
  s_q[j] = q;
  m->theta[j] = th;
  __syncthreads();
  if (j == 0) {
    // sequential cumulative sum: non-decreasing by construction
    float run = 0.f;
    for (int i = 0; i < kCdfSegments; ++i) {
      m->c[i] = fminf(run, 1.f);
      run += s_q[i];
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
  const float p = segment_mass(keys, M, dm, is_float, s_start);
  const float q = softmax_mass(theta[threadIdx.x], s_tmp);
  const float L = cross_entropy(p, q, s_tmp);
  grad[threadIdx.x] = q - p;
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

hipError_t launch_cdf_fit(const uint32_t* sorted, int S, int k, int is_float, int steps, float lr,
                          CdfModel* models, hipStream_t st) {
  AdamCfg cfg{steps, lr, 0.9f, 0.999f, 1e-8f};
  hipLaunchKernelGGL(k_cdf_fit, dim3(k), dim3(kFitThreads), 0, st, sorted, S, is_float, cfg, models);
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
  for (int i = gid; i < nu; i += stride) {
    const int b = (int)cdf_bucket(cdf_eval(s_c, lo, scale, kmin, kmax, is_float, keys[i]), nb_bits);
    const int pb = i == 0 ? -1
                          : (int)cdf_bucket(cdf_eval(s_c, lo, scale, kmin, kmax, is_float, keys[i - 1]),
                                            nb_bits);
    if (b < pb) atomicOr(flag, 4);
    for (int bb = pb + 1; bb <= b; ++bb) starts[bb] = i;
    if (i == nu - 1)
      for (int bb = b + 1; bb <= NB; ++bb) starts[bb] = nu;
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
constexpr int kBsCap = 8192;
constexpr int kBsMaxItems = kBsCap / kBsThreads;  // 16

size_t bucket_sort_lds_bytes() { return (size_t)kBsCap * (4 + 4 + 4 + 2 + 2); }
int bucket_sort_capacity() { return kBsCap; }

// Stable LSD radix sort of N <= kBsCap (key, 16-bit value) pairs in LDS over
// `passes` 8-bit digits.  Wave w owns elements [w * items * 64, (w+1) *
// items * 64), items = ceil(N / kBsThreads).  Returns true when the result is
// in (kb, vb).
__device__ bool bucket_lds_sort(uint32_t* ka, uint16_t* va, uint32_t* kb, uint16_t* vb, int N,
                                int passes, uint32_t (*s_cnt)[kRadix], uint32_t* s_dbase,
                                uint32_t* s_tmp) {
  const int tid = threadIdx.x;
  const int w = tid / kWave;
  const int lane = tid % kWave;
  const uint64_t below = lanes_below_mask();
  const int items = (N + kBsThreads - 1) / kBsThreads;
  const int per_wave = items * kWave;
  bool flipped = false;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = ps * kRadixBits;
    for (int q = tid; q < kBsWaves * kRadix; q += kBsThreads) (&s_cnt[0][0])[q] = 0;
    __syncthreads();
    uint32_t key[kBsMaxItems], rank[kBsMaxItems];
    uint16_t val[kBsMaxItems];
#pragma unroll
    for (int j = 0; j < kBsMaxItems; ++j) {
      if (j < items) {
        const int e = w * per_wave + j * kWave + lane;
        const bool valid = e < N;
        key[j] = valid ? ka[e] : 0u;
        val[j] = valid ? va[e] : (uint16_t)0;
        const uint32_t d = (key[j] >> shift) & 0xFF;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
          const bool bit = (d >> b) & 1;
          const uint64_t bb = __ballot(bit);
          m &= bit ? bb : ~bb;
        }
        uint32_t pre = 0;
        if (valid) pre = s_cnt[w][d];
        __builtin_amdgcn_wave_barrier();
        const uint32_t before = popc64(m & below);
        if (valid && before == 0) s_cnt[w][d] = pre + popc64(m);
        __builtin_amdgcn_wave_barrier();
        rank[j] = pre + before;
      }
    }
    __syncthreads();
    uint32_t tot = 0;
    if (tid < kRadix) {
#pragma unroll
      for (int q = 0; q < kBsWaves; ++q) {
        const uint32_t c = s_cnt[q][tid];
        s_cnt[q][tid] = tot;
        tot += c;
      }
    }
    uint32_t all;
    const uint32_t ex = block_exclusive_sum<kBsThreads>(tot, s_tmp, &all);
    if (tid < kRadix) s_dbase[tid] = ex;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBsMaxItems; ++j) {
      if (j < items) {
        const int e = w * per_wave + j * kWave + lane;
        if (e < N) {
          const uint32_t d = (key[j] >> shift) & 0xFF;
          const uint32_t dest = s_dbase[d] + s_cnt[w][d] + rank[j];
          kb[dest] = key[j];
          vb[dest] = val[j];
        }
      }
    }
    __syncthreads();
    uint32_t* tk = ka;
    ka = kb;
    kb = tk;
    uint16_t* tv = va;
    va = vb;
    vb = tv;
    flipped = !flipped;
  }
  return flipped;
}

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

// One workgroup per bucket: the bucket's elements (in stable bucket-pass
// order) are sorted stably by the key words ls.keyq (least significant
// first; each word's digits are taken relative to its minimum in the bucket,
// so only the digits that vary are sorted), then every plane is written
// permuted.  Planes are staged through LDS, so an output may be its input.
__global__ __launch_bounds__(kBsThreads) void k_bucket_sort(const int32_t* __restrict__ starts,
                                                            int64_t n_host, const int32_t* n_dev,
                                                            int32_t* __restrict__ flag,
                                                            const LocalSort ls) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  uint32_t* ka = reinterpret_cast<uint32_t*>(s_raw);
  uint32_t* kb = ka + kBsCap;
  uint32_t* stage = kb + kBsCap;
  uint16_t* va = reinterpret_cast<uint16_t*>(stage + kBsCap);
  uint16_t* vb = va + kBsCap;
  __shared__ uint32_t s_cnt[kBsWaves][kRadix];
  __shared__ uint32_t s_dbase[kRadix];
  __shared__ uint32_t s_tmp[kBsWaves + 1];
  __shared__ uint32_t s_red[kBsWaves];
  __shared__ int32_t s_flag;

  // Other workgroups of this launch may raise the flag while this one reads
  // it, so one thread reads it and the block follows that one value.
  const int tid = threadIdx.x;
  if (tid == 0) s_flag = *flag;
  __syncthreads();
  if (s_flag != 0) return;
  const int nu = (int)(n_dev ? *n_dev : n_host);
  const int s = starts[blockIdx.x], e = starts[blockIdx.x + 1];
  if (s < 0 || e < s || e > nu) {
    if (tid == 0) atomicOr(flag, 4);
    return;
  }
  const int N = e - s;
  if (N == 0) return;
  if (N > kBsCap) {
    if (tid == 0) atomicOr(flag, 1);
    return;
  }
  for (int i = tid; i < N; i += kBsThreads) va[i] = (uint16_t)i;
  uint32_t* ck = ka;
  uint16_t* cv = va;
  uint32_t* ok = kb;
  uint16_t* ov = vb;
  for (int w = 0; w < ls.nkeys; ++w) {
    const uint32_t* src = pick(ls.in, pick(ls.keyq, w)) + s;
    __syncthreads();
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
    for (int i = tid; i < N; i += kBsThreads) {
      const uint32_t v = src[i];
      stage[i] = v;
      mn = min(mn, v);
      mx = max(mx, v);
    }
    mn = bs_reduce(mn, s_red, OpMin());
    mx = bs_reduce(mx, s_red, OpMax());
    if (mn == mx) continue;
    const int bits = 32 - __clz(mx - mn);
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    for (int i = tid; i < N; i += kBsThreads) ck[i] = stage[cv[i]] - mn;
    __syncthreads();
    if (bucket_lds_sort(ck, cv, ok, ov, N, passes, s_cnt, s_dbase, s_tmp)) {
      uint32_t* tk = ck;
      ck = ok;
      ok = tk;
      uint16_t* tv = cv;
      cv = ov;
      ov = tv;
    }
  }
  for (int q = 0; q < ls.nq; ++q) {
    __syncthreads();
    const uint32_t* in = pick(ls.in, q) + s;
    for (int i = tid; i < N; i += kBsThreads) stage[i] = in[i];
    __syncthreads();
    uint32_t* out = pick(ls.out, q) + s;
    for (int i = tid; i < N; i += kBsThreads) out[i] = stage[cv[i]];
  }
}

hipError_t launch_bucket_sort(const int32_t* starts, int nb_bits, int64_t n, const int32_t* n_dev,
                              int32_t* flag, const LocalSort& ls, hipStream_t st) {
  const size_t lds = bucket_sort_lds_bytes();
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_bucket_sort),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bucket_sort, dim3(1u << nb_bits), dim3(kBsThreads), lds, st, starts, n, n_dev,
                     flag, ls);
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
