// Partitioning: ids, per-wave histograms, scan, stable scatter, and vx_partition.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "vx_cdf.h"
#include "vx_part.h"
#include "vx_pipeline.h"

namespace vx {

// ---------------------------------------------------------------- device side

__device__ __forceinline__ long long load_any(const void* p, uint64_t i, uint32_t size) {
  return size == 4 ? (long long)((const int*)p)[i] : ((const long long*)p)[i];
}

__device__ __forceinline__ void store_any(void* p, uint64_t i, uint32_t size, long long v) {
  if (size == 4) ((int*)p)[i] = (int)v;
  else ((long long*)p)[i] = v;
}

// mask of the active lanes whose id equals this lane's (all lanes must call it together)
__device__ __forceinline__ unsigned long long peers_of(uint32_t pid, bool valid, uint32_t bits) {
  unsigned long long peers = __ballot(valid);
  for (uint32_t b = 0; b < bits; ++b) {
    bool bit = (pid >> b) & 1u;
    unsigned long long m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

__device__ __forceinline__ uint32_t id_bits(uint32_t n_parts) {
  uint32_t b = 0;
  while ((1u << b) < n_parts) ++b;
  return b;
}

__global__ void __launch_bounds__(256) k_part_hist(PartSpec ps, PartIO io, uint64_t tile,
                                                   uint32_t* hist, unsigned long long* totals,
                                                   const int* sum_slot, unsigned long long* sums) {
  __shared__ long long split[kMaxParts];
  __shared__ uint32_t whist[4][kMaxParts];
  __shared__ unsigned long long ssum[kMaxSumSlots][2];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (ps.fn == kPartRange)
    for (uint32_t j = threadIdx.x; j < ps.n_split; j += blockDim.x) split[j] = ps.splitters[j];
  for (uint32_t j = threadIdx.x; j < 4 * kMaxParts; j += blockDim.x) (&whist[0][0])[j] = 0;
  for (uint32_t j = threadIdx.x; j < 2 * kMaxSumSlots; j += blockDim.x) (&ssum[0][0])[j] = 0;
  __syncthreads();
  const uint32_t bits = id_bits(ps.n_parts);
  const uint64_t w = (uint64_t)blockIdx.x * 4 + wave;
  const uint64_t r0 = w * tile;
  const uint64_t r1 = r0 + tile < io.n ? r0 + tile : io.n;
  for (uint64_t base = r0; base < r1; base += 64) {
    uint64_t i = base + lane;
    bool valid = i < r1;
    long long k = valid ? load_any(io.key, i, io.key_size) : 0;
    uint32_t pid = valid ? part_of(ps, k, split) : 0;
    unsigned long long peers = peers_of(pid, valid, bits);
    if (valid && (peers & ((1ull << lane) - 1)) == 0)
      atomicAdd(&whist[wave][pid], (uint32_t)__popcll(peers));
    if (sum_slot && valid) {
      int slot = sum_slot[pid];
      if (slot >= 0) {
        atomicAdd(&ssum[slot][0], 1ull);
        if (io.n_pay) atomicAdd(&ssum[slot][1], (unsigned long long)load_any(io.pay[0], i, io.pay_size[0]));
      }
    }
  }
  __syncthreads();
  const uint64_t W = (uint64_t)gridDim.x * 4;
  for (uint32_t j = threadIdx.x; j < 4 * ps.n_parts; j += blockDim.x) {
    uint32_t wv = j / ps.n_parts, p = j % ps.n_parts;
    uint32_t c = whist[wv][p];
    hist[(uint64_t)p * W + (uint64_t)blockIdx.x * 4 + wv] = c;
    if (totals && c) atomicAdd(totals + p, (unsigned long long)c);
  }
  if (sums)
    for (uint32_t j = threadIdx.x; j < 2 * kMaxSumSlots; j += blockDim.x) {
      unsigned long long v = (&ssum[0][0])[j];
      if (v) atomicAdd(sums + j, v);
    }
}

// single-block exclusive scan over count entries (partition-major hist)
// Exclusive scan of the partition-major histogram, in three launches: per-tile sums, a scan of
// the tile sums, and each tile rescanned from its base.  boundary[p] (optional) receives the
// offset of entry p * waves, i.e. partition p's first row, and boundary[n_parts] the total.
constexpr uint32_t kScanThreads = 256;

// exclusive prefix of v over the block (256 threads); *total receives the block's sum
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long v, unsigned long long* ws,
                                                              unsigned long long* total) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long x = v;
  for (int o = 1; o < 64; o <<= 1) {
    unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == 63) ws[wave] = x;
  __syncthreads();
  unsigned long long base = 0, tot = 0;
  for (uint32_t w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) base += ws[w];
    tot += ws[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const uint32_t* hist, uint64_t count, uint64_t tile,
                                                             unsigned long long* tsum) {
  __shared__ unsigned long long ws[kScanThreads / 64];
  const uint64_t a = blockIdx.x * tile, e = a + tile < count ? a + tile : count;
  unsigned long long s = 0;
  for (uint64_t i = a + threadIdx.x; i < e; i += blockDim.x) s += hist[i];
  unsigned long long tot = 0;
  block_excl_scan(s, ws, &tot);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// tsum[0..nt) becomes its exclusive scan; tsum[nt] the total (nt <= 4 * kScanThreads)
__global__ void __launch_bounds__(kScanThreads) k_scan_top(unsigned long long* tsum, uint32_t nt) {
  __shared__ unsigned long long ws[kScanThreads / 64];
  const uint32_t a = threadIdx.x * 4;
  unsigned long long v[4], s = 0;
  for (uint32_t j = 0; j < 4; ++j) {
    v[j] = a + j < nt ? tsum[a + j] : 0ull;
    s += v[j];
  }
  unsigned long long tot = 0;
  unsigned long long run = block_excl_scan(s, ws, &tot);
  for (uint32_t j = 0; j < 4; ++j)
    if (a + j < nt) {
      tsum[a + j] = run;
      run += v[j];
    }
  if (threadIdx.x == 0) tsum[nt] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const uint32_t* hist, uint64_t count, uint64_t tile,
                                                             const unsigned long long* tsum, uint32_t nt,
                                                             unsigned long long* offs, uint32_t n_parts,
                                                             uint32_t waves, unsigned long long* boundary) {
  __shared__ unsigned long long ws[kScanThreads / 64];
  const uint64_t a = blockIdx.x * tile, e = a + tile < count ? a + tile : count;
  const uint64_t per = (tile + kScanThreads - 1) / kScanThreads;
  const uint64_t ta = a + threadIdx.x * per < e ? a + threadIdx.x * per : e;
  const uint64_t te = ta + per < e ? ta + per : e;
  unsigned long long s = 0;
  for (uint64_t i = ta; i < te; ++i) s += hist[i];
  unsigned long long tot = 0;
  unsigned long long run = tsum[blockIdx.x] + block_excl_scan(s, ws, &tot);
  for (uint64_t i = ta; i < te; ++i) {
    offs[i] = run;
    if (boundary && i % waves == 0) boundary[i / waves] = run;
    run += hist[i];
  }
  if (boundary && blockIdx.x == 0 && threadIdx.x == 0) boundary[n_parts] = tsum[nt];
}

// one block per partition: offs[p*W + w] = base[p] + sum of hist[p*W + w'] for w' < w
__global__ void __launch_bounds__(256) k_scan_seg(const uint32_t* hist, uint32_t waves,
                                                  const unsigned long long* part_base,
                                                  unsigned long long* offs) {
  __shared__ unsigned long long part[256];
  const uint64_t p = blockIdx.x;
  const uint32_t per = (waves + blockDim.x - 1) / blockDim.x;
  const uint32_t a = threadIdx.x * per, b = a + per < waves ? a + per : waves;
  unsigned long long s = 0;
  for (uint32_t i = a; i < b; ++i) s += hist[p * waves + i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = part_base[p];
    for (uint32_t t = 0; t < blockDim.x; ++t) {
      unsigned long long v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  unsigned long long run = part[threadIdx.x];
  for (uint32_t i = a; i < b; ++i) {
    offs[p * waves + i] = run;
    run += hist[p * waves + i];
  }
}

__global__ void __launch_bounds__(256) k_part_scatter(PartSpec ps, PartIO io, uint64_t tile,
                                                      const unsigned long long* offs) {
  __shared__ long long split[kMaxParts];
  __shared__ unsigned long long run[4][kMaxParts];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t W = (uint64_t)gridDim.x * 4;
  const uint64_t w = (uint64_t)blockIdx.x * 4 + wave;
  if (ps.fn == kPartRange)
    for (uint32_t j = threadIdx.x; j < ps.n_split; j += blockDim.x) split[j] = ps.splitters[j];
  for (uint32_t p = lane; p < ps.n_parts; p += 64) run[wave][p] = offs[(uint64_t)p * W + w];
  __syncthreads();
  const uint32_t bits = id_bits(ps.n_parts);
  const uint64_t r0 = w * tile;
  const uint64_t r1 = r0 + tile < io.n ? r0 + tile : io.n;
  for (uint64_t base = r0; base < r1; base += 64) {
    uint64_t i = base + lane;
    bool valid = i < r1;
    long long k = valid ? load_any(io.key, i, io.key_size) : 0;
    uint32_t pid = valid ? part_of(ps, k, split) : 0;
    unsigned long long peers = peers_of(pid, valid, bits);
    if (valid) {
      uint32_t rank = (uint32_t)__popcll(peers & ((1ull << lane) - 1));
      uint64_t pos = io.out_base + run[wave][pid] + rank;
      if (io.out_key) store_any(io.out_key, pos, io.key_size, k);
      for (uint32_t c = 0; c < io.n_pay; ++c)
        if (io.out_pay[c]) store_any(io.out_pay[c], pos, io.pay_size[c], load_any(io.pay[c], i, io.pay_size[c]));
    }
    // every lane has read run[] above; the group leader advances it
    __builtin_amdgcn_wave_barrier();
    if (valid && (peers & ((1ull << lane) - 1)) == 0) run[wave][pid] += (unsigned long long)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
}

// start[p] += add[p]; add[p] = 0
__global__ void k_advance(unsigned long long* start, unsigned long long* add, uint32_t n) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) {
    start[p] += add[p];
    add[p] = 0;
  }
}

// ---------------------------------------------------------------- host wrappers

PartGeom part_geom(const vx_ctx* ctx, uint64_t n) {
  PartGeom g;
  uint64_t waves_wanted = (n + 64 * 16 - 1) / (64 * 16);      // >= 16 steps of 64 rows per wave
  uint64_t blocks = (waves_wanted + 3) / 4;
  uint64_t cap = (uint64_t)ctx->cu_count * 4;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  g.blocks = (uint32_t)blocks;
  g.waves = g.blocks * 4;
  uint64_t tile = (n + g.waves - 1) / g.waves;
  g.tile = (tile + 63) / 64 * 64;
  if (g.tile == 0) g.tile = 64;
  return g;
}

vx_status part_hist(vx_ctx* ctx, const PartSpec& ps, const PartIO& io, const PartGeom& g,
                    uint32_t* hist, unsigned long long* totals, const int* sum_slot,
                    unsigned long long* sums, hipStream_t s) {
  hipLaunchKernelGGL(k_part_hist, dim3(g.blocks), dim3(256), 0, s, ps, io, g.tile, hist, totals,
                     sum_slot, sums);
  VX_HIP(hipGetLastError());
  return VX_OK;
}

vx_status part_scan(vx_ctx* ctx, const uint32_t* hist, uint32_t n_parts, uint32_t waves,
                    const unsigned long long* part_base, unsigned long long* offs,
                    unsigned long long* boundary, hipStream_t s) {
  if (part_base) {
    hipLaunchKernelGGL(k_scan_seg, dim3(n_parts), dim3(256), 0, s, hist, waves, part_base, offs);
  } else {
    const uint64_t count = (uint64_t)n_parts * waves;
    uint64_t tile = 4096;
    while ((count + tile - 1) / tile > kScanTilesMax) tile *= 2;
    const uint32_t nt = (uint32_t)std::max<uint64_t>(1, (count + tile - 1) / tile);
    unsigned long long* tsum = (unsigned long long*)ctx->dev_scan;
    hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(kScanThreads), 0, s, hist, count, tile, tsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, tsum, nt);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kScanThreads), 0, s, hist, count, tile, tsum, nt, offs,
                       n_parts, waves, boundary);
  }
  VX_HIP(hipGetLastError());
  return VX_OK;
}

vx_status part_scatter(vx_ctx* ctx, const PartSpec& ps, const PartIO& io, const PartGeom& g,
                       const unsigned long long* offs, hipStream_t s) {
  (void)ctx;
  hipLaunchKernelGGL(k_part_scatter, dim3(g.blocks), dim3(256), 0, s, ps, io, g.tile, offs);
  VX_HIP(hipGetLastError());
  return VX_OK;
}

// ---------------------------------------------------------------- vx_partition

static uint32_t log2_ceil(uint64_t v) {
  uint32_t r = 0;
  while ((1ull << r) < v) ++r;
  return r;
}

vx_status make_spec(vx_ctx* ctx, const vx_part_opts& o, uint32_t n_parts, const int64_t* host_split,
                    uint32_t n_split, ArenaBlock& split_mem, PartSpec* ps) {
  std::memset(ps, 0, sizeof *ps);
  if (o.method == VX_PART_RADIX_HASH || o.method == VX_PART_RADIX_BITS) {
    uint32_t l = log2_ceil(std::max<uint32_t>(n_parts, 1));
    ps->fn = o.method == VX_PART_RADIX_HASH ? kPartHash : kPartBits;
    ps->n_parts = 1u << l;
    ps->log2p = l;
    ps->shift = o.shift;
    VX_CHECK(o.method == VX_PART_RADIX_HASH || o.shift + l <= 64, VX_EINVAL,
             "partition: shift %u + %u bits exceeds 64", o.shift, l);
  } else {
    ps->fn = kPartRange;
    ps->n_parts = n_split + 1;
    ps->n_split = n_split;
    for (uint32_t i = 1; i < n_split; ++i)
      VX_CHECK(host_split[i - 1] < host_split[i], VX_EINVAL, "partition: splitters not strictly ascending");
    if (n_split) {
      split_mem.a = &ctx->arena;
      split_mem.p = ctx->arena.alloc(n_split * 8);
      VX_CHECK(split_mem.p, VX_EBUDGET, "partition: no room for splitters");
      VX_HIP(hipMemcpyAsync(split_mem.p, host_split, n_split * 8, hipMemcpyHostToDevice, ctx->compute));
      ps->splitters = (const long long*)split_mem.p;
    }
  }
  VX_CHECK(ps->n_parts >= 1 && ps->n_parts <= kMaxParts, VX_EINVAL, "partition: %u partitions (1..%u)",
           ps->n_parts, kMaxParts);
  return VX_OK;
}

static vx_status partition_impl(vx_ctx* ctx, const vx_partition_desc* d, vx_partition_out* out) {
  VX_CHECK(d->n_pay <= 4, VX_EINVAL, "partition: at most 4 payload columns");
  VX_CHECK(d->n_pay == 0 || d->pay, VX_EINVAL, "partition: pay is NULL");
  VX_CHECK(out->hist && out->boundary, VX_EINVAL, "partition: hist and boundary are required");
  const vx_part_opts& o = d->opts;
  VX_CHECK(o.method <= VX_PART_RANGE, VX_EINVAL, "partition: method %u", o.method);
  VX_HIP(hipSetDevice(ctx->device));
  const uint64_t n = d->n;
  ColInfo kc;
  VX_TRY(classify(ctx, d->key, n, &kc, "partition key"));
  ColInfo pc[4];
  for (uint32_t c = 0; c < d->n_pay; ++c) VX_TRY(classify(ctx, d->pay[c], n, &pc[c], "partition payload"));
  uint32_t req = o.n_parts;
  if (req == 0) {
    // planned: a pre-aggregating table sized from each partition's rows fits half the free arena
    uint64_t free_b = ctx->arena.largest_free() / 2;
    uint64_t per = std::max<uint64_t>(free_b / 64, 1);   // 32-byte slots at load factor 0.5
    req = (uint32_t)std::min<uint64_t>(kMaxParts, std::max<uint64_t>(2, (n + per - 1) / per));
  }
  // splitters for range methods
  std::vector<int64_t> split;
  uint32_t method_used = o.method;
  CdfReport rep{};
  if (o.method == VX_PART_RANGE) {
    VX_CHECK(o.n_splitters == 0 || o.splitters, VX_EINVAL, "partition: splitters is NULL");
    split.assign(o.splitters, o.splitters + o.n_splitters);
  } else if (o.method == VX_PART_LEARNED || o.method == VX_PART_QUANTILE ||
             o.method == VX_PART_UNTRAINED || o.method == VX_PART_AUTO) {
    VX_TRY(cdf_splitters(ctx, kc, n, o, req, &split, &rep, out->model));
    method_used = o.method;
    if (o.method == VX_PART_AUTO)
      method_used = rep.imbalance_range < rep.imbalance_radix
                        ? (rep.auto_quantile ? VX_PART_QUANTILE : VX_PART_LEARNED)
                        : VX_PART_RADIX_HASH;
  }
  vx_part_opts eff = o;
  eff.method = method_used == VX_PART_LEARNED || method_used == VX_PART_QUANTILE ||
                       method_used == VX_PART_UNTRAINED
                   ? VX_PART_RANGE
                   : method_used;
  ArenaBlock split_mem;
  PartSpec ps;
  VX_TRY(make_spec(ctx, eff, req, split.data(), (uint32_t)split.size(), split_mem, &ps));
  const uint32_t P = ps.n_parts;
  VX_CHECK(out->n_parts_cap >= P, VX_ECAPACITY, "partition: %u partitions exceed n_parts_cap %u", P,
           out->n_parts_cap);

  // device scratch: totals, base
  ArenaBlock tot_mem;
  tot_mem.a = &ctx->arena;
  tot_mem.p = ctx->arena.alloc(2 * P * 8 + 8 * (P + 1));
  VX_CHECK(tot_mem.p, VX_EBUDGET, "partition: no room for histograms");
  unsigned long long* totals = (unsigned long long*)tot_mem.p;
  unsigned long long* base = totals + P;
  unsigned long long* bnd = base + P;
  fill_zero((uint64_t*)totals, P, ctx->compute);

  const bool scatter = d->out_key != nullptr;
  void* out_key = d->out_key;
  void* out_pay[4] = {};
  if (scatter) {
    // outputs may be device memory or pinned host memory (written by zero-copy stores)
    vx_col oc{d->out_key, d->key.type, 0};
    ColInfo oi;
    VX_TRY(classify(ctx, oc, n, &oi, "partition output key"));
    out_key = const_cast<void*>(oi.dev);
    for (uint32_t c = 0; c < d->n_pay; ++c) {
      VX_CHECK(d->out_pay && d->out_pay[c], VX_EINVAL, "partition: out_pay[%u] is NULL", c);
      vx_col pcol{d->out_pay[c], d->pay[c].type, 0};
      ColInfo pi;
      VX_TRY(classify(ctx, pcol, n, &pi, "partition output payload"));
      out_pay[c] = const_cast<void*>(pi.dev);
    }
  }

  double tp0 = now_ms();
  // pass A: histogram (per chunk when streamed)
  auto run_pass = [&](bool do_scatter) -> vx_status {
    std::vector<PipeCol> cols(1 + (do_scatter ? d->n_pay : 0));
    cols[0].info = kc;
    cols[0].may_copy = cols[0].copy = true;
    for (uint32_t c = 0; do_scatter && c < d->n_pay; ++c) {
      cols[1 + c].info = pc[c];
      cols[1 + c].may_copy = cols[1 + c].copy = true;
    }
    Pipeline pipe;
    VX_TRY(pipe.plan(ctx, n, 0, 0, cols));
    // per-chunk scratch sized for the largest chunk
    PartGeom g0 = part_geom(ctx, pipe.chunk_rows());
    ArenaBlock hmem;
    hmem.a = &ctx->arena;
    hmem.p = ctx->arena.alloc((uint64_t)P * g0.waves * (4 + 8));
    VX_CHECK(hmem.p, VX_EBUDGET, "partition: no room for per-wave histograms");
    uint32_t* hist = (uint32_t*)hmem.p;
    unsigned long long* offs = (unsigned long long*)(hmem.p + (uint64_t)P * g0.waves * 4);
    auto kernel = [&](const ChunkView& v) -> vx_status {
      PartIO io{};
      io.key = (v.global_mask & 1u) ? (const uint8_t*)v.ptr[0] + v.row0 * kc.elsize : v.ptr[0];
      io.key_size = (uint32_t)kc.elsize;
      io.n = v.rows;
      PartGeom g = part_geom(ctx, v.rows);
      if (!do_scatter) return part_hist(ctx, ps, io, g, hist, totals, nullptr, nullptr, ctx->compute);
      io.n_pay = d->n_pay;
      for (uint32_t c = 0; c < d->n_pay; ++c) {
        io.pay[c] = ((v.global_mask >> (1 + c)) & 1u) ? (const uint8_t*)v.ptr[1 + c] + v.row0 * pc[c].elsize
                                                      : v.ptr[1 + c];
        io.pay_size[c] = (uint32_t)pc[c].elsize;
        io.out_pay[c] = out_pay[c];
      }
      io.out_key = out_key;
      io.out_base = 0;
      // global placement: bnd[p] is the running start of partition p (its boundary plus the
      // rows of p in earlier chunks); base receives this chunk's counts and then advances bnd
      VX_TRY(part_hist(ctx, ps, io, g, hist, base, nullptr, nullptr, ctx->compute));
      VX_TRY(part_scan(ctx, hist, P, g.waves, bnd, offs, nullptr, ctx->compute));
      VX_TRY(part_scatter(ctx, ps, io, g, offs, ctx->compute));
      hipLaunchKernelGGL(k_advance, dim3((P + 255) / 256), dim3(256), 0, ctx->compute, bnd, base, P);
      VX_HIP(hipGetLastError());
      return VX_OK;
    };
    VX_TRY(pipe.run(kernel));
    VX_HIP(hipStreamSynchronize(ctx->compute));
    return VX_OK;
  };
  VX_TRY(run_pass(false));
  std::vector<unsigned long long> h(P);
  VX_HIP(hipMemcpy(h.data(), totals, P * 8, hipMemcpyDeviceToHost));
  std::vector<unsigned long long> b(P + 1, 0);
  for (uint32_t p = 0; p < P; ++p) b[p + 1] = b[p] + h[p];
  if (scatter) {
    VX_HIP(hipMemcpy(bnd, b.data(), P * 8, hipMemcpyHostToDevice));
    fill_zero((uint64_t*)base, P, ctx->compute);
    VX_TRY(run_pass(true));
  }
  for (uint32_t p = 0; p < P; ++p) out->hist[p] = h[p];
  for (uint32_t p = 0; p <= P; ++p) out->boundary[p] = b[p];
  out->n_parts = P;
  out->method_used = method_used;
  out->n_splitters = (uint32_t)split.size();
  if (out->splitters && ps.fn == kPartRange)
    for (size_t i = 0; i < split.size() && i < out->n_parts_cap; ++i) out->splitters[i] = split[i];
  double mx = 0;
  for (uint32_t p = 0; p < P; ++p) mx = std::max(mx, (double)h[p]);
  out->imbalance = n ? mx / ((double)n / P) : 0.0;
  out->est_imbalance_radix = rep.imbalance_radix;
  out->est_imbalance_range = rep.imbalance_range;
  out->final_loss = rep.final_loss;
  (void)tp0;
  return VX_OK;
}

}  // namespace vx

extern "C" vx_status vx_partition(vx_ctx* ctx, const vx_partition_desc* d, vx_partition_out* out) {
  VX_CHECK(ctx && d && out, VX_EINVAL, "vx_partition: null argument");
  vx::release_cached(ctx);
  return vx::partition_impl(ctx, d, out);
}
