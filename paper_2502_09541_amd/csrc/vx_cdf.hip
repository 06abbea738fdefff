// Learned range-partition splitters: sample, GPU radix sort, mid-CDF targets, an FP32
// one-hidden-layer ReLU network trained with Adam by hand-written forward/backward kernels,
// and splitter extraction.
//
// Training is bit-reproducible: every wave owns a fixed contiguous slice of the sample and
// accumulates its gradient in FP64 in sample order; per-wave partials are summed in wave order
// by one thread per parameter.  Lane j of a wave is hidden unit j, so a sample's forward pass
// is one FMA per lane and a fixed butterfly sum across the wave.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "vx_cdf.h"
#include "vx_part.h"

namespace vx {

constexpr unsigned long long kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint32_t kPartialStride = kModelParams + 1;   // gradient components + loss
constexpr uint64_t kTrainMax = 1ull << 16;              // training points taken from the sample

// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ unsigned long long splitmix_out(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------- sample

// Row i is sampled iff the (i+1)-th SplitMix64 output of the stream seeded by `seed` is below thr.
// Only sampled rows are read.  Each wave gathers its sampled keys in LDS and reserves room in
// `out` once per kSampleBuf - 64 keys, so the shared counter sees few atomics.
constexpr uint32_t kSampleBuf = 512;

__global__ void __launch_bounds__(256) k_sample(const void* key, uint32_t ks, uint64_t n, uint64_t seed,
                                                uint64_t thr, long long* out, uint64_t cap,
                                                unsigned long long* count) {
  __shared__ long long buf[4][kSampleBuf];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t first = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x - lane;
  uint32_t held = 0;   // wave-uniform
  auto flush = [&]() {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(count, (unsigned long long)held);
    base = __shfl(base, 0, 64);
    for (uint32_t j = lane; j < held; j += 64)
      if (base + j < cap) out[base + j] = buf[wave][j];
    held = 0;
  };
  for (uint64_t wb = first; wb < n; wb += stride) {
    uint64_t i = wb + lane;
    bool take = i < n && splitmix_out(seed + kGolden * (i + 1)) < thr;
    unsigned long long m = __ballot(take);
    if (!m) continue;
    if (take) {
      uint32_t pos = held + (uint32_t)__popcll(m & ((1ull << lane) - 1));
      buf[wave][pos] = ks == 4 ? (long long)((const int*)key)[i] : ((const long long*)key)[i];
    }
    held += (uint32_t)__popcll(m);
    if (held > kSampleBuf - 64) {
      __builtin_amdgcn_wave_barrier();
      flush();
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (held) {
    __builtin_amdgcn_wave_barrier();
    flush();
  }
}

// min / max of the sign-flipped keys (unsigned order == signed order of the keys)
__global__ void k_minmax(const long long* s, uint64_t m, unsigned long long* mm) {
  unsigned long long lo = ~0ull, hi = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    unsigned long long u = (unsigned long long)s[i] ^ 0x8000000000000000ull;
    lo = u < lo ? u : lo;
    hi = u > hi ? u : hi;
  }
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long a = __shfl_xor(lo, o, 64), b = __shfl_xor(hi, o, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(mm, lo);
    atomicMax(mm + 1, hi);
  }
}

__global__ void k_init_minmax(unsigned long long* mm) {
  mm[0] = ~0ull;
  mm[1] = 0;
}

// ---------------------------------------------------------------- targets and features

__device__ __forceinline__ uint64_t lower_bound_i64(const long long* s, uint64_t m, long long k) {
  uint64_t lo = 0, hi = m;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (s[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t upper_bound_i64(const long long* s, uint64_t m, long long k) {
  uint64_t lo = 0, hi = m;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (s[mid] <= k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Piecewise-linear log2 of the key's offset above the sample minimum (exponent and the next
// 23 bits read as fixed point), saturated at 2^63 - 1, times scale.
__device__ __forceinline__ float key_feature(long long key, long long kmin, float scale) {
  unsigned long long u = key < kmin ? 0ull : (unsigned long long)key - (unsigned long long)kmin;
  if (u > 0x7FFFFFFFFFFFFFFFull) u = 0x7FFFFFFFFFFFFFFFull;
  unsigned long long v = u + 1;
  int l = 63 - __clzll((long long)v);
  unsigned long long mant = l >= 23 ? (v >> (l - 23)) & 0x7FFFFFull : (v << (23 - l)) & 0x7FFFFFull;
  int fixed = (l << 23) | (int)mant;
  return (float)fixed * scale;
}

__global__ void k_targets(const long long* s, uint64_t m, long long kmin, float scale, float* x,
                          float* t) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    long long k = s[i];
    uint64_t lo = lower_bound_i64(s, m, k), hi = upper_bound_i64(s, m, k);
    t[i] = (float)(((double)lo + (double)hi) / (2.0 * (double)m));
    x[i] = key_feature(k, kmin, scale);
  }
}

// ---------------------------------------------------------------- the network

// y = b2 + sum_j w2_j * relu(w1_j * x + b1_j), in FP32, units in order.
__device__ __forceinline__ float mlp_eval(float x, const float* p) {
  float y = p[3 * kHidden];
  for (uint32_t j = 0; j < kHidden; ++j) {
    float z = fmaf(p[j], x, p[kHidden + j]);
    if (z > 0.0f) y = fmaf(p[2 * kHidden + j], z, y);
  }
  return y;
}

__global__ void k_mlp_forward(const float* x, uint64_t n, const float* params, float* y) {
  __shared__ float p[kModelParams];
  for (uint32_t j = threadIdx.x; j < kModelParams; j += blockDim.x) p[j] = params[j];
  __syncthreads();
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    y[i] = mlp_eval(x[i], p);
}

// One forward/backward pass of the mean squared error over the wave's slice of samples.
// partial[w * kPartialStride + c]: gradient component c (w1, b1, w2, b2), then the squared-
// error sum, all FP64.
constexpr int kGradUnroll = 4;

__global__ void __launch_bounds__(256) k_mlp_grad(const float* x, const float* t, uint64_t n,
                                                  const float* params, uint64_t per_wave,
                                                  double* partial) {
  const uint32_t j = threadIdx.x & 63;
  const uint64_t w = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const float w1 = params[j], b1 = params[kHidden + j], w2 = params[2 * kHidden + j];
  const float b2 = params[3 * kHidden];
  const double scale = 2.0 / (double)n;
  double aw1 = 0, ab1 = 0, aw2 = 0, ab2 = 0, al = 0;
  const uint64_t i0 = w * per_wave;
  const uint64_t i1 = i0 + per_wave < n ? i0 + per_wave : n;
  uint64_t i = i0;
  for (; i + kGradUnroll <= i1; i += kGradUnroll) {
    float xs[kGradUnroll], ts[kGradUnroll], z[kGradUnroll], h[kGradUnroll], ps[kGradUnroll];
#pragma unroll
    for (int u = 0; u < kGradUnroll; ++u) {
      xs[u] = x[i + u];
      ts[u] = t[i + u];
      z[u] = fmaf(w1, xs[u], b1);
      h[u] = z[u] > 0.0f ? z[u] : 0.0f;
      ps[u] = w2 * h[u];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int u = 0; u < kGradUnroll; ++u) ps[u] += __shfl_xor(ps[u], o, 64);
#pragma unroll
    for (int u = 0; u < kGradUnroll; ++u) {
      float y = b2 + ps[u];
      double e = (double)y - (double)ts[u];
      double r = e * scale;
      aw2 += r * (double)h[u];
      if (z[u] > 0.0f) {
        double g = r * (double)w2;
        ab1 += g;
        aw1 += g * (double)xs[u];
      }
      ab2 += r;
      al += e * e;
    }
  }
  for (; i < i1; ++i) {
    float xs = x[i], ts = t[i];
    float z = fmaf(w1, xs, b1);
    float h = z > 0.0f ? z : 0.0f;
    float ps = w2 * h;
    for (int o = 32; o > 0; o >>= 1) ps += __shfl_xor(ps, o, 64);
    float y = b2 + ps;
    double e = (double)y - (double)ts;
    double r = e * scale;
    aw2 += r * (double)h;
    if (z > 0.0f) {
      double g = r * (double)w2;
      ab1 += g;
      aw1 += g * (double)xs;
    }
    ab2 += r;
    al += e * e;
  }
  double* out = partial + w * kPartialStride;
  out[j] = aw1;
  out[kHidden + j] = ab1;
  out[2 * kHidden + j] = aw2;
  if (j == 0) {
    out[3 * kHidden] = ab2;
    out[3 * kHidden + 1] = al;
  }
}

// grad[c] = SUM over waves of partial[w][c] in a fixed order (block c: thread t adds waves
// t, t + 256, ... in turn, then a fixed tree over the threads); grad[kModelParams] = loss.
__global__ void __launch_bounds__(256) k_mlp_reduce(const double* partial, uint32_t waves, uint64_t n,
                                                    double* grad) {
  __shared__ double red[256];
  const uint32_t c = blockIdx.x;
  double s = 0;
  for (uint32_t w = threadIdx.x; w < waves; w += blockDim.x) s += partial[(uint64_t)w * kPartialStride + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[c] = c == kModelParams ? red[0] / (double)n : red[0];
}

// One training step's second half: block c reduces gradient component c over the waves (the
// fixed order of k_mlp_reduce) and applies Adam (Kingma and Ba, 2015) to parameter c, on FP32
// parameters and moments evaluated in FP64 (components are independent).
__global__ void __launch_bounds__(256) k_mlp_reduce_adam(const double* partial, uint32_t waves, uint64_t n,
                                                         double* grad, float* params, float* m, float* v,
                                                         double lr, double b1, double b2, double eps, double c1,
                                                         double c2) {
  __shared__ double red[256];
  const uint32_t c = blockIdx.x;
  double s = 0;
  for (uint32_t w = threadIdx.x; w < waves; w += blockDim.x) s += partial[(uint64_t)w * kPartialStride + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (c == kModelParams) {
    grad[c] = red[0] / (double)n;
    return;
  }
  grad[c] = red[0];
  const double g = (double)(float)red[0];
  const double mj = b1 * (double)m[c] + (1.0 - b1) * g;
  const double vj = b2 * (double)v[c] + (1.0 - b2) * g * g;
  m[c] = (float)mj;
  v[c] = (float)vj;
  params[c] = (float)((double)params[c] - lr * (mj / c1) / (sqrt(vj / c2) + eps));
}


// c = the number of quantiles j/P (1 <= j < P) the value reaches; first[c] = min row reaching c
__global__ void k_cross(const float* x, const float* t, uint64_t m, const float* params,
                        uint32_t P, unsigned long long* first) {
  __shared__ float p[kModelParams];
  if (params)
    for (uint32_t j = threadIdx.x; j < kModelParams; j += blockDim.x) p[j] = params[j];
  __syncthreads();
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    double y = params ? (double)mlp_eval(x[i], p) : (double)t[i];
    double yp = y * (double)P;
    long long c = yp >= (double)(P - 1) ? (long long)(P - 1) : (yp < 0.0 ? 0 : (long long)floor(yp));
    while (c < (long long)P - 1 && y >= (double)(c + 1) / (double)P) ++c;
    while (c > 0 && !(y >= (double)c / (double)P)) --c;
    // lanes hold consecutive rows, so only the first lane of each run of equal counts can hold
    // its run's smallest row
    long long cp = __shfl_up(c, 1, 64);
    if (c >= 1 && ((threadIdx.x & 63) == 0 || cp != c)) atomicMin(first + c, (unsigned long long)i);
  }
}

// x_s[i] = x[i * stride], t_s[i] = t[i * stride]: evenly spaced order statistics of the sorted sample
__global__ void k_stride_gather(const float* x, const float* t, uint64_t m_s, uint64_t stride, float* xs,
                                float* ts) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m_s;
       i += (uint64_t)gridDim.x * blockDim.x) {
    xs[i] = x[i * stride];
    ts[i] = t[i * stride];
  }
}

// *out += number of rows i >= 1 with s[i] != s[i - 1] (distinct keys - 1 of a sorted array)
__global__ void k_count_changes(const long long* s, uint64_t m, unsigned long long* out) {
  unsigned long long c = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x + 1; i < m;
       i += (uint64_t)gridDim.x * blockDim.x)
    c += s[i] != s[i - 1];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

__global__ void k_gather_i64(const long long* s, const unsigned long long* idx, uint32_t cnt,
                             long long* out) {
  uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < cnt) out[j] = s[idx[j]];
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- host side

static unsigned grid1(const vx_ctx* ctx, uint64_t n) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, (uint64_t)ctx->cu_count * 8));
}

// LSD radix sort of m int64 keys (signed order) in 8-bit digits over the bits where the keys
// differ; each digit pass is a stable multisplit.  Returns the buffer holding the result.
static vx_status sort_i64(vx_ctx* ctx, long long* a, long long* b, uint64_t m, long long** sorted) {
  *sorted = a;
  if (m < 2) return VX_OK;
  hipStream_t s = ctx->compute;
  unsigned long long* mm = (unsigned long long*)ctx->dev_acc;
  hipLaunchKernelGGL(k_init_minmax, dim3(1), dim3(1), 0, s, mm);
  hipLaunchKernelGGL(k_minmax, dim3(grid1(ctx, m)), dim3(256), 0, s, a, m, mm);
  unsigned long long hm[2];
  VX_HIP(hipMemcpyAsync(hm, mm, 16, hipMemcpyDeviceToHost, s));
  VX_HIP(hipStreamSynchronize(s));
  unsigned long long diff = hm[0] ^ hm[1];
  if (diff == 0) return VX_OK;
  uint32_t top = 63 - (uint32_t)__builtin_clzll(diff);
  PartGeom g = part_geom(ctx, m);
  ArenaBlock scratch;
  scratch.a = &ctx->arena;
  scratch.p = ctx->arena.alloc((uint64_t)256 * g.waves * 12);
  VX_CHECK(scratch.p, VX_EBUDGET, "sort: no room for digit histograms");
  uint32_t* hist = (uint32_t*)scratch.p;
  unsigned long long* offs = (unsigned long long*)(scratch.p + (uint64_t)256 * g.waves * 4);
  long long* src = a;
  long long* dst = b;
  for (uint32_t shift = 0; shift <= top; shift += 8) {
    PartSpec ps{};
    ps.fn = kPartBits;
    ps.n_parts = 256;
    ps.log2p = 8;
    ps.shift = shift;
    ps.flip_sign = 1;
    PartIO io{};
    io.key = src;
    io.key_size = 8;
    io.n = m;
    io.out_key = dst;
    VX_TRY(part_hist(ctx, ps, io, g, hist, nullptr, nullptr, nullptr, s));
    VX_TRY(part_scan(ctx, hist, 256, g.waves, nullptr, offs, nullptr, s));
    VX_TRY(part_scatter(ctx, ps, io, g, offs, s));
    std::swap(src, dst);
  }
  *sorted = src;
  return VX_OK;
}

struct Model {
  float* params;      // device [kModelParams]
  float* m;
  float* v;
  double* grad;       // device [kPartialStride]
  double* partial;    // device [waves * kPartialStride]
  uint32_t waves;
  uint64_t per_wave;
};

static void init_params(float* p) {
  for (uint32_t j = 0; j < kHidden; ++j) {
    p[j] = 1.0f;                                   // w1
    p[kHidden + j] = -(float)j / (float)kHidden;   // b1: hinge knots at j/64
    p[2 * kHidden + j] = 1.0f / (float)kHidden;    // w2
  }
  p[3 * kHidden] = 0.0f;
}

static void model_geometry(const vx_ctx* ctx, uint64_t n, uint32_t* waves, uint64_t* per_wave) {
  uint64_t wv = std::min<uint64_t>((uint64_t)ctx->cu_count * 16, std::max<uint64_t>(1, (n + 255) / 256));
  wv = (wv + 3) / 4 * 4;
  *per_wave = std::max<uint64_t>(1, (n + wv - 1) / wv);
  *waves = (uint32_t)wv;
}

static vx_status grad_pass(vx_ctx* ctx, const Model& md, const float* x, const float* t, uint64_t n) {
  hipStream_t s = ctx->compute;
  hipLaunchKernelGGL(k_mlp_grad, dim3(md.waves / 4), dim3(256), 0, s, x, t, n, md.params, md.per_wave,
                     md.partial);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(kPartialStride), dim3(256), 0, s, md.partial, md.waves, n, md.grad);
  VX_HIP(hipGetLastError());
  return VX_OK;
}

static vx_status train(vx_ctx* ctx, Model& md, const float* x, const float* t, uint64_t n,
                       uint32_t steps, double lr, double* final_loss) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  fill_zero((uint64_t*)md.m, (kModelParams + 1) / 2, ctx->compute);
  fill_zero((uint64_t*)md.v, (kModelParams + 1) / 2, ctx->compute);
  // cosine learning-rate decay: lr at the first step, towards 0 at the last
  for (uint32_t st = 1; st <= steps; ++st) {
    const double lr_t = lr * 0.5 * (1.0 + std::cos(M_PI * (double)(st - 1) / (double)steps));
    double c1 = 1.0 - std::pow(b1, (double)st), c2 = 1.0 - std::pow(b2, (double)st);
    hipLaunchKernelGGL(k_mlp_grad, dim3(md.waves / 4), dim3(256), 0, ctx->compute, x, t, n, md.params,
                       md.per_wave, md.partial);
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3(kPartialStride), dim3(256), 0, ctx->compute, md.partial, md.waves,
                       n, md.grad, md.params, md.m, md.v, lr_t, b1, b2, eps, c1, c2);
  }
  VX_HIP(hipGetLastError());
  VX_TRY(grad_pass(ctx, md, x, t, n));
  double hg[kPartialStride];
  VX_HIP(hipMemcpyAsync(hg, md.grad, sizeof hg, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  *final_loss = hg[kModelParams];
  return VX_OK;
}

// Device scratch for a model over n samples, carved from the arena.
struct ModelMem {
  ArenaBlock blk;
  Model md{};
  vx_status alloc(vx_ctx* ctx, uint64_t n) {
    model_geometry(ctx, n, &md.waves, &md.per_wave);
    uint64_t bytes = 3 * 1024 + 2 * kPartialStride * 8 + (uint64_t)md.waves * kPartialStride * 8;
    blk.a = &ctx->arena;
    blk.p = ctx->arena.alloc(bytes);
    VX_CHECK(blk.p, VX_EBUDGET, "cdf: no room for the model scratch");
    md.params = (float*)blk.p;
    md.m = (float*)(blk.p + 1024);
    md.v = (float*)(blk.p + 2048);
    md.grad = (double*)(blk.p + 3072);
    md.partial = (double*)(blk.p + 3072 + 2 * kPartialStride * 8);
    return VX_OK;
  }
};

static double imbalance_of(const std::vector<unsigned long long>& h) {
  double tot = 0, mx = 0;
  for (auto v : h) {
    tot += (double)v;
    mx = std::max(mx, (double)v);
  }
  return tot > 0 ? mx / (tot / (double)h.size()) : 0.0;
}

vx_status cdf_splitters(vx_ctx* ctx, const ColInfo& key, uint64_t n, const vx_part_opts& o,
                        uint32_t n_parts, std::vector<int64_t>* splitters, CdfReport* rep,
                        float* model_out) {
  splitters->clear();
  VX_CHECK(n_parts >= 1 && n_parts <= kMaxParts, VX_EINVAL, "cdf: %u partitions", n_parts);
  hipStream_t s = ctx->compute;
  double t0 = now_ms();
  const double frac = o.sample_frac > 0 ? (double)o.sample_frac : 0.01;
  VX_CHECK(frac > 0 && frac <= 1.0, VX_EINVAL, "cdf: sample_frac %f outside (0, 1]", frac);
  const uint64_t thr = frac >= 1.0 ? ~0ull : (uint64_t)(frac * 18446744073709551616.0);
  const double mean = frac * (double)n;
  const uint64_t cap = std::min<uint64_t>(n, (uint64_t)(mean + 8.0 * std::sqrt(mean) + 1024));
  // sample buffers (two for the sort), features and targets
  ArenaBlock sb;
  sb.a = &ctx->arena;
  sb.p = ctx->arena.alloc(cap * (8 + 8 + 4 + 4) + 1024);
  VX_CHECK(sb.p, VX_EBUDGET, "cdf: no room for a sample of %llu keys", (unsigned long long)cap);
  long long* sa = (long long*)sb.p;
  long long* sbuf = sa + cap;
  float* fx = (float*)(sbuf + cap);
  float* ft = fx + cap;
  unsigned long long* count = (unsigned long long*)ctx->dev_acc;
  fill_zero((uint64_t*)count, 1, s);
  if (n) {
    unsigned g = (unsigned)std::min<uint64_t>((n + 255) / 256, (uint64_t)ctx->cu_count * 16);
    hipLaunchKernelGGL(k_sample, dim3(g), dim3(256), 0, s, key.dev, (uint32_t)key.elsize, n, o.seed,
                       thr, sa, cap, count);
    VX_HIP(hipGetLastError());
  }
  unsigned long long m = 0;
  VX_HIP(hipMemcpyAsync(&m, count, 8, hipMemcpyDeviceToHost, s));
  VX_HIP(hipStreamSynchronize(s));
  VX_CHECK(m <= cap, VX_ECAPACITY, "cdf: sample of %llu rows exceeds its buffer (%llu)",
           (unsigned long long)m, (unsigned long long)cap);
  rep->sample_rows = m;
  double t1 = now_ms();
  rep->sample_ms = t1 - t0;
  if (m == 0) return VX_OK;   // no splitters: a single partition
  long long* sorted = nullptr;
  VX_TRY(sort_i64(ctx, sa, sbuf, m, &sorted));
  long long ends[2];
  VX_HIP(hipMemcpyAsync(&ends[0], sorted, 8, hipMemcpyDeviceToHost, s));
  VX_HIP(hipMemcpyAsync(&ends[1], sorted + m - 1, 8, hipMemcpyDeviceToHost, s));
  VX_HIP(hipStreamSynchronize(s));
  double t2 = now_ms();
  rep->sort_ms = t2 - t1;
  // feature scale: 1 / (L * 2^23), L = floor(log2(range + 1)) + 1 over the sample's key range
  unsigned long long range = (unsigned long long)ends[1] - (unsigned long long)ends[0];
  if (range > 0x7FFFFFFFFFFFFFFFull) range = 0x7FFFFFFFFFFFFFFFull;
  uint32_t L = 64 - (uint32_t)__builtin_clzll(range + 1);
  const float scale = (float)(1.0 / ((double)L * 8388608.0));
  hipLaunchKernelGGL(k_targets, dim3(grid1(ctx, m)), dim3(256), 0, s, sorted, m, ends[0], scale, fx, ft);
  VX_HIP(hipGetLastError());

  // model, fit to at most kTrainMax evenly spaced points of the sorted sample
  const float* tx = fx;
  const float* tt = ft;
  uint64_t mt = m;
  ArenaBlock tb;
  if (m > kTrainMax) {
    const uint64_t stride = (m + kTrainMax - 1) / kTrainMax;
    mt = (m + stride - 1) / stride;
    tb.a = &ctx->arena;
    tb.p = ctx->arena.alloc(mt * 8 + 256);
    VX_CHECK(tb.p, VX_EBUDGET, "cdf: no room for the training points");
    float* sx = (float*)tb.p;
    float* st = sx + mt;
    hipLaunchKernelGGL(k_stride_gather, dim3(grid1(ctx, mt)), dim3(256), 0, s, fx, ft, mt, stride, sx, st);
    VX_HIP(hipGetLastError());
    tx = sx;
    tt = st;
  }
  ModelMem mm;
  VX_TRY(mm.alloc(ctx, mt));
  float hp[kModelParams];
  init_params(hp);
  VX_HIP(hipMemcpyAsync(mm.md.params, hp, sizeof hp, hipMemcpyHostToDevice, s));
  const bool use_model = o.method != VX_PART_QUANTILE;
  if (o.method == VX_PART_LEARNED || o.method == VX_PART_AUTO) {
    uint32_t steps = o.train_steps ? o.train_steps : 1000;
    double lr = o.lr > 0 ? (double)o.lr : 1e-2;
    VX_TRY(train(ctx, mm.md, tx, tt, mt, steps, lr, &rep->final_loss));
  } else if (use_model) {
    VX_TRY(grad_pass(ctx, mm.md, tx, tt, mt));
    double hg[kPartialStride];
    VX_HIP(hipMemcpyAsync(hg, mm.md.grad, sizeof hg, hipMemcpyDeviceToHost, s));
    VX_HIP(hipStreamSynchronize(s));
    rep->final_loss = hg[kModelParams];
  }
  if (model_out) {
    VX_HIP(hipMemcpyAsync(model_out, mm.md.params, kModelParams * 4, hipMemcpyDeviceToHost, s));
  }
  double t3 = now_ms();
  rep->train_ms = t3 - t2;

  // splitters: idx_j = first sample row whose value reaches j / P, under the model (or, with
  // model == false, under the empirical mid-CDF: the sample quantiles)
  const uint32_t P = n_parts;
  auto make_splitters = [&](bool model, std::vector<int64_t>* out) -> vx_status {
    out->clear();
    if (P > 1) {
      ArenaBlock fb;
      fb.a = &ctx->arena;
      fb.p = ctx->arena.alloc((uint64_t)P * 8 * 3);
      VX_CHECK(fb.p, VX_EBUDGET, "cdf: no room for quantile scratch");
      unsigned long long* first = (unsigned long long*)fb.p;
      unsigned long long* idxd = first + P;
      long long* keysd = (long long*)(idxd + P);
      hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, s, first, (uint64_t)P, ~0ull);
      hipLaunchKernelGGL(k_cross, dim3(grid1(ctx, m)), dim3(256), 0, s, fx, ft, m,
                         model ? mm.md.params : nullptr, P, first);
      std::vector<unsigned long long> fh(P);
      VX_HIP(hipMemcpyAsync(fh.data(), first, P * 8, hipMemcpyDeviceToHost, s));
      VX_HIP(hipStreamSynchronize(s));
      // the first row reaching quantile j is the earliest row reaching any j' >= j
      std::vector<unsigned long long> idx(P, ~0ull);
      unsigned long long run = ~0ull;
      for (int64_t j = (int64_t)P - 1; j >= 1; --j) {
        run = std::min(run, fh[j]);
        idx[j] = run;
      }
      // distinct rows in quantile order, with how many quantiles each carries
      std::vector<unsigned long long> rows;
      std::vector<uint32_t> carried;
      for (uint32_t j = 1; j < P; ++j) {
        if (idx[j] == ~0ull) break;
        if (!rows.empty() && rows.back() == idx[j]) ++carried.back();
        else {
          rows.push_back(idx[j]);
          carried.push_back(1);
        }
      }
      if (!rows.empty()) {
        VX_HIP(hipMemcpyAsync(idxd, rows.data(), rows.size() * 8, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_gather_i64, dim3((unsigned)((rows.size() + 255) / 256)), dim3(256), 0, s,
                           sorted, idxd, (uint32_t)rows.size(), keysd);
        std::vector<long long> ks(rows.size());
        VX_HIP(hipMemcpyAsync(ks.data(), keysd, rows.size() * 8, hipMemcpyDeviceToHost, s));
        VX_HIP(hipStreamSynchronize(s));
        for (size_t r = 0; r < rows.size(); ++r) {
          long long k = ks[r];
          if (out->empty() || out->back() < k) out->push_back(k);
          if (carried[r] > 1 && k < INT64_MAX && out->back() < k + 1) out->push_back(k + 1);
        }
      }
    }
    return VX_OK;
  };
  // the share of the sample in singleton partitions under range splitters sp (a histogram of
  // the sorted sample)
  auto single_share = [&](const std::vector<int64_t>& sp, double* share) -> vx_status {
    const uint32_t np = (uint32_t)sp.size() + 1;
    PartGeom g = part_geom(ctx, m);
    ArenaBlock b;
    b.a = &ctx->arena;
    b.p = ctx->arena.alloc((uint64_t)np * g.waves * 4 + (uint64_t)np * 8 + sp.size() * 8 + 256);
    VX_CHECK(b.p, VX_EBUDGET, "cdf: no room for sample histograms");
    uint32_t* hist = (uint32_t*)b.p;
    unsigned long long* tot = (unsigned long long*)(b.p + (uint64_t)np * g.waves * 4);
    long long* spl = (long long*)(tot + np);
    PartIO io{};
    io.key = sorted;
    io.key_size = 8;
    io.n = m;
    PartSpec ps{};
    ps.fn = kPartRange;
    ps.n_split = np - 1;
    ps.n_parts = np;
    ps.splitters = spl;
    if (ps.n_split) VX_HIP(hipMemcpyAsync(spl, sp.data(), ps.n_split * 8, hipMemcpyHostToDevice, s));
    fill_zero((uint64_t*)tot, np, s);
    VX_TRY(part_hist(ctx, ps, io, g, hist, tot, nullptr, nullptr, s));
    std::vector<unsigned long long> h(np);
    VX_HIP(hipMemcpyAsync(h.data(), tot, np * 8, hipMemcpyDeviceToHost, s));
    VX_HIP(hipStreamSynchronize(s));
    uint64_t one = 0;
    for (uint32_t p = 1; p + 1 < np; ++p)
      if (sp[p] == sp[p - 1] + 1) one += h[p];
    *share = (double)one / (double)m;
    return VX_OK;
  };
  VX_TRY(make_splitters(use_model, splitters));
  // AUTO: the sample quantiles are kept instead when their singleton partitions hold clearly more
  // of the sample (5 points) than the model's: keys whose order carries no skew (scrambled, say)
  // defeat the model's log-scale feature, not the quantiles
  if (o.method == VX_PART_AUTO) {
    std::vector<int64_t> q;
    VX_TRY(make_splitters(false, &q));
    double sm = 0, sq = 0;
    VX_TRY(single_share(*splitters, &sm));
    VX_TRY(single_share(q, &sq));
    if (sq > sm + 0.05) {
      splitters->swap(q);
      rep->auto_quantile = true;
    }
  }
  rep->split_ms = now_ms() - t3;

  // imbalance of both partitioners on the sample
  {
    uint32_t l = 0;
    while ((1u << l) < P) ++l;
    rep->radix_parts = 1u << l;
    uint32_t pr = std::max<uint32_t>(rep->radix_parts, (uint32_t)splitters->size() + 1);
    PartGeom g = part_geom(ctx, m);
    ArenaBlock hb;
    hb.a = &ctx->arena;
    hb.p = ctx->arena.alloc((uint64_t)pr * g.waves * 4 + (uint64_t)pr * 8 + splitters->size() * 8 + 256);
    VX_CHECK(hb.p, VX_EBUDGET, "cdf: no room for sample histograms");
    uint32_t* hist = (uint32_t*)hb.p;
    unsigned long long* tot = (unsigned long long*)(hb.p + (uint64_t)pr * g.waves * 4);
    long long* spl = (long long*)(tot + pr);
    PartIO io{};
    io.key = sorted;
    io.key_size = 8;
    io.n = m;
    PartSpec ps{};
    ps.fn = kPartHash;
    ps.n_parts = rep->radix_parts;
    ps.log2p = l;
    fill_zero((uint64_t*)tot, pr, s);
    VX_TRY(part_hist(ctx, ps, io, g, hist, tot, nullptr, nullptr, s));
    std::vector<unsigned long long> h(ps.n_parts);
    VX_HIP(hipMemcpyAsync(h.data(), tot, h.size() * 8, hipMemcpyDeviceToHost, s));
    VX_HIP(hipStreamSynchronize(s));
    rep->imbalance_radix = imbalance_of(h);
    PartSpec pr2{};
    pr2.fn = kPartRange;
    pr2.n_split = (uint32_t)splitters->size();
    pr2.n_parts = pr2.n_split + 1;
    pr2.splitters = spl;
    if (pr2.n_split)
      VX_HIP(hipMemcpyAsync(spl, splitters->data(), pr2.n_split * 8, hipMemcpyHostToDevice, s));
    fill_zero((uint64_t*)tot, pr, s);
    VX_TRY(part_hist(ctx, pr2, io, g, hist, tot, nullptr, nullptr, s));
    h.assign(pr2.n_parts, 0);
    VX_HIP(hipMemcpyAsync(h.data(), tot, h.size() * 8, hipMemcpyDeviceToHost, s));
    fill_zero((uint64_t*)tot, 1, s);
    hipLaunchKernelGGL(k_count_changes, dim3(grid1(ctx, m)), dim3(256), 0, s, sorted, m, tot);
    unsigned long long changes = 0;
    VX_HIP(hipMemcpyAsync(&changes, tot, 8, hipMemcpyDeviceToHost, s));
    VX_HIP(hipStreamSynchronize(s));
    rep->imbalance_range = imbalance_of(h);
    uint64_t single = 0, mx = 0;
    for (uint32_t p = 0; p < pr2.n_parts; ++p) {
      bool one = p >= 1 && p + 1 < pr2.n_parts && (*splitters)[p] == (*splitters)[p - 1] + 1;
      if (one) single += h[p];
      else mx = std::max<uint64_t>(mx, h[p]);
    }
    rep->single_share = (double)single / (double)m;
    rep->max_share = (double)mx / (double)m;
    rep->distinct_share = (double)(changes + 1) / (double)m;
  }
  return VX_OK;
}

}  // namespace vx

using namespace vx;

// ---------------------------------------------------------------- exported model kernels

static vx_status cdf_inputs(vx_ctx* ctx, const float* x, const float* t, uint64_t n, ColInfo* xi,
                            ColInfo* ti) {
  // float columns are classified as 4-byte columns
  vx_col xc{x, VX_I32, 0}, tc{t, VX_I32, 0};
  VX_TRY(classify(ctx, xc, n, xi, "cdf x"));
  if (t) VX_TRY(classify(ctx, tc, n, ti, "cdf t"));
  return VX_OK;
}

extern "C" {

vx_status vx_cdf_loss_grad(vx_ctx* ctx, const float* x, const float* t, uint64_t n,
                           const float* params, float* grad, double* loss) {
  VX_CHECK(ctx && x && t && params && grad && n, VX_EINVAL, "vx_cdf_loss_grad: bad argument");
  release_cached(ctx);
  VX_HIP(hipSetDevice(ctx->device));
  ColInfo xi, ti;
  VX_TRY(cdf_inputs(ctx, x, t, n, &xi, &ti));
  ModelMem mm;
  VX_TRY(mm.alloc(ctx, n));
  VX_HIP(hipMemcpyAsync(mm.md.params, params, kModelParams * 4, hipMemcpyHostToDevice, ctx->compute));
  VX_TRY(grad_pass(ctx, mm.md, (const float*)xi.dev, (const float*)ti.dev, n));
  double hg[kPartialStride];
  VX_HIP(hipMemcpyAsync(hg, mm.md.grad, sizeof hg, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  for (uint32_t c = 0; c < kModelParams; ++c) grad[c] = (float)hg[c];
  if (loss) *loss = hg[kModelParams];
  return VX_OK;
}

vx_status vx_cdf_forward(vx_ctx* ctx, const float* x, uint64_t n, const float* params, float* y) {
  VX_CHECK(ctx && x && params && y, VX_EINVAL, "vx_cdf_forward: bad argument");
  release_cached(ctx);
  VX_HIP(hipSetDevice(ctx->device));
  if (n == 0) return VX_OK;
  ColInfo xi, ti;
  VX_TRY(cdf_inputs(ctx, x, nullptr, n, &xi, &ti));
  ArenaBlock b;
  b.a = &ctx->arena;
  b.p = ctx->arena.alloc(n * 4 + 1024);
  VX_CHECK(b.p, VX_EBUDGET, "vx_cdf_forward: no room for %llu outputs", (unsigned long long)n);
  float* dp = (float*)b.p;
  float* dy = (float*)(b.p + 1024);
  VX_HIP(hipMemcpyAsync(dp, params, kModelParams * 4, hipMemcpyHostToDevice, ctx->compute));
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid1(ctx, n)), dim3(256), 0, ctx->compute, (const float*)xi.dev,
                     n, dp, dy);
  VX_HIP(hipMemcpyAsync(y, dy, n * 4, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  return VX_OK;
}

vx_status vx_cdf_train(vx_ctx* ctx, const float* x, const float* t, uint64_t n, float* params,
                       uint32_t steps, float lr, double* final_loss) {
  VX_CHECK(ctx && x && t && params && n, VX_EINVAL, "vx_cdf_train: bad argument");
  release_cached(ctx);
  VX_HIP(hipSetDevice(ctx->device));
  ColInfo xi, ti;
  VX_TRY(cdf_inputs(ctx, x, t, n, &xi, &ti));
  ModelMem mm;
  VX_TRY(mm.alloc(ctx, n));
  VX_HIP(hipMemcpyAsync(mm.md.params, params, kModelParams * 4, hipMemcpyHostToDevice, ctx->compute));
  double fl = 0;
  VX_TRY(train(ctx, mm.md, (const float*)xi.dev, (const float*)ti.dev, n, steps,
               lr > 0 ? (double)lr : 1e-2, &fl));
  VX_HIP(hipMemcpyAsync(params, mm.md.params, kModelParams * 4, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  if (final_loss) *final_loss = fl;
  return VX_OK;
}

}  // extern "C"
