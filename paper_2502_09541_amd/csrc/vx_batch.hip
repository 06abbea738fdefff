// Many independent device-resident joins, batched into one HIP graph launch.
//
// The work is a list of equal-size tiles: every job's build tiles, then every job's probe
// tiles.  Two queue-draining kernels cover it: the build kernel walks the build tiles
// grid-stride and inserts each tile's rows into its job's table; the probe kernel walks the
// probe tiles and aggregates each tile into its job's result.  The kernel boundary between them
// is the only dependency, so no workgroup ever waits for another.  The tiles are placed by XCD
// (the MI355X has 8, each with its own 4 MB L2): a job whose table fits one L2 is built and
// probed on one XCD only, so its table is cached once instead of in every L2.  Table init,
// result reset, both kernels and the copy of the results are captured once in a HIP graph and
// replayed while the batch is unchanged.  Tile size, workgroup size and load factor come from
// a small autotuner that times candidates on the batch itself and caches the winner per
// workload class (optionally in the file named by VX_TUNE_CACHE).
//
// A job whose build keys fill their value range exactly (n unique keys from min to min + n - 1,
// found by a min/max pass over every job before the graph runs) gets a direct table instead of
// a hash table: the payload of key k sits at k - min, and a bitmap of the keys seen catches a
// duplicate (which would leave a key of the range missing).  The build sets the bits without
// reading them back; a small kernel between the two phases counts each job's bits, and the host
// compares the count with the job's rows.  A probe key outside the range then costs no memory
// access, and one inside reads one payload.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "vx_device.h"

namespace vx {

struct BatchJob {
  const void* bkey;
  const void* bpay;
  const void* pkey;
  uint64_t nb, np;
  uint8_t* slots;         // hash: capacity slots of 8 (int32 key + int32 payload) or 16 bytes;
                          // direct: the key bitmap ((nb + 63) / 64 words), then the payloads
  uint8_t* dpay;          // direct: payload of key kmin + i at index i
  unsigned long long kmin_ord;   // direct: the smallest key, order-preserving unsigned form
  uint32_t direct;        // 1: direct table
  uint64_t mask;
  uint32_t log2cap;
  uint32_t pay_size;      // 0 (no payload), 4 or 8
  uint64_t ctile0;        // first bitmap-count tile of the job (direct tables)
  uint32_t build_tiles, probe_tiles, count_tiles;
  unsigned long long* side;   // sentinel-key record: count, payload sum
};

constexpr uint32_t kMaxBatchJobs = 4096;

template <typename K>
__device__ __forceinline__ void batch_build_rows(const BatchJob& jb, uint64_t r0, uint64_t r1,
                                                 uint32_t slot_shift, unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  for (uint64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    K k = ((const K*)jb.bkey)[i];
    U kb = (U)k;
    long long v = jb.pay_size ? load_signed(jb.bpay, i, jb.pay_size) : 0;
    if (jb.direct) {
      // every build key lies in [kmin, kmin + nb): the range was measured over these keys.  The
      // bit is set without reading it back; k_batch_dupcount counts the bits afterwards, and a
      // job with fewer than nb bits had a repeated key.
      const uint64_t idx = key_ord(k) - jb.kmin_ord;
      atomicOr((unsigned long long*)jb.slots + (idx >> 6), 1ull << (idx & 63));
      if (jb.pay_size == 4) ((int*)jb.dpay)[idx] = (int)v;
      else if (jb.pay_size == 8) ((long long*)jb.dpay)[idx] = v;
      continue;
    }
    if (kb == kEmpty) {
      unsigned long long prev = atomicAdd(jb.side, 1ull);
      if (prev) atomicOr(flags, kFlagDup);
      atomicAdd(jb.side + 1, (unsigned long long)v);
      continue;
    }
    uint64_t h = slot_of(key_bits(k), jb.log2cap);
    bool done = false;
    for (uint64_t step = 0; step <= jb.mask; ++step) {
      uint8_t* slot = jb.slots + (h << slot_shift);
      U prev = atomicCAS((U*)slot, kEmpty, kb);
      if (prev == kEmpty) {
        if (jb.pay_size == 4) *(int*)(slot + sizeof(K)) = (int)v;
        else if (jb.pay_size == 8) *(long long*)(slot + 8) = v;
        done = true;
        break;
      }
      if (prev == kb) {
        atomicOr(flags, kFlagDup);
        done = true;
        break;
      }
      h = (h + 1) & jb.mask;
    }
    if (!done) atomicOr(flags, kFlagFull);
  }
}

template <typename K>
__device__ __forceinline__ void batch_probe_rows(const BatchJob& jb, uint64_t r0, uint64_t r1,
                                                 uint32_t slot_shift, unsigned long long& cnt,
                                                 unsigned long long& sum) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  for (uint64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    K k = __builtin_nontemporal_load(((const K*)jb.pkey) + i);
    U kb = (U)k;
    if (jb.direct) {
      const uint64_t idx = key_ord(k) - jb.kmin_ord;
      if (idx < jb.nb) {   // every key of the range is in the table (no duplicates: checked)
        cnt += 1;
        if (jb.pay_size == 4) sum += (unsigned long long)(long long)((const int*)jb.dpay)[idx];
        else if (jb.pay_size == 8) sum += (unsigned long long)((const long long*)jb.dpay)[idx];
      }
      continue;
    }
    if (kb == kEmpty) {
      unsigned long long c = jb.side[0];
      cnt += c;
      if (c) sum += jb.side[1];
      continue;
    }
    uint64_t h = slot_of(key_bits(k), jb.log2cap);
    for (uint64_t step = 0; step <= jb.mask; ++step) {
      const uint8_t* slot = jb.slots + (h << slot_shift);
      U sk = *(const U*)slot;
      if (sk == kb) {
        cnt += 1;
        if (jb.pay_size == 4) sum += (unsigned long long)(long long)*(const int*)(slot + sizeof(K));
        else if (jb.pay_size == 8) sum += (unsigned long long)*(const long long*)(slot + 8);
        break;
      }
      if (sk == kEmpty) break;
      h = (h + 1) & jb.mask;
    }
  }
}

__device__ __forceinline__ void block_add2(unsigned long long cnt, unsigned long long sum,
                                           unsigned long long* out) {
  __shared__ unsigned long long red[2][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    cnt += __shfl_xor(cnt, o, 64);
    sum += __shfl_xor(sum, o, 64);
  }
  __syncthreads();
  if (lane == 0) {
    red[0][wave] = cnt;
    red[1][wave] = sum;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    unsigned long long s = 0;
    for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
    if (s) atomicAdd(out + threadIdx.x, s);
  }
}

// Tiles of one phase: tile_map[t] holds (job << 32 | the job's own tile index), or ~0 for an
// empty tile.
template <typename K, bool BUILD>
__global__ void __launch_bounds__(512) k_batch_phase(const BatchJob* jobs, uint32_t n_jobs,
                                                     uint64_t phase_tiles, uint32_t tile_rows,
                                                     uint32_t slot_shift, unsigned long long* acc,
                                                     unsigned int* flags,
                                                     const unsigned long long* tile_map) {
  (void)n_jobs;
  for (uint64_t t = blockIdx.x; t < phase_tiles; t += gridDim.x) {
    const unsigned long long e = tile_map[t];
    if (e == ~0ull) continue;     // uniform over the workgroup
    const uint32_t lo = (uint32_t)(e >> 32);
    const uint64_t local = e & 0xffffffffull;
    const BatchJob jb = jobs[lo];
    const uint64_t n = BUILD ? jb.nb : jb.np;
    const uint64_t r0 = local * tile_rows, r1 = r0 + tile_rows < n ? r0 + tile_rows : n;
    if (BUILD) {
      batch_build_rows<K>(jb, r0, r1, slot_shift, flags);
    } else {
      unsigned long long cnt = 0, sum = 0;
      batch_probe_rows<K>(jb, r0, r1, slot_shift, cnt, sum);
      block_add2(cnt, sum, acc + 2 * lo);
    }
  }
}

// Bits set in the direct-table jobs' bitmaps, per job, into cnt[j] (tile order).  Count tile t
// belongs to the job whose first count tile is the largest one <= t; each covers kCountWords
// bitmap words.
constexpr uint32_t kCountWords = 4096;

__global__ void __launch_bounds__(256) k_batch_dupcount(const BatchJob* jobs, uint32_t n_jobs, uint64_t tiles,
                                                        unsigned long long* cnt) {
  __shared__ unsigned long long t0[kMaxBatchJobs];
  __shared__ unsigned long long part[4];
  for (uint32_t j = threadIdx.x; j < n_jobs; j += blockDim.x) t0[j] = jobs[j].ctile0;
  __syncthreads();
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    uint32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (t0[mid] <= t) lo = mid;
      else hi = mid;
    }
    const BatchJob& jb = jobs[lo];
    const uint64_t words = (jb.nb + 63) / 64;
    const uint64_t w0 = (t - jb.ctile0) * kCountWords;
    const uint64_t w1 = w0 + kCountWords < words ? w0 + kCountWords : words;
    unsigned long long c = 0;
    for (uint64_t w = w0 + threadIdx.x; w < w1; w += blockDim.x)
      c += (unsigned long long)__popcll(((const unsigned long long*)jb.slots)[w]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) c += part[w];
      if (c) atomicAdd(cnt + lo, c);
    }
    __syncthreads();   // part is reused by the next tile
  }
}

// one job, two plain launches (the baseline): build kernel over its rows, probe kernel
template <typename K>
__global__ void k_job_build(BatchJob jb, uint32_t slot_shift, unsigned int* flags) {
  uint64_t per = (jb.nb + gridDim.x - 1) / gridDim.x;
  uint64_t r0 = blockIdx.x * per, r1 = r0 + per < jb.nb ? r0 + per : jb.nb;
  if (r0 < r1) batch_build_rows<K>(jb, r0, r1, slot_shift, flags);
}

template <typename K>
__global__ void k_job_probe(BatchJob jb, uint32_t slot_shift, unsigned long long* acc) {
  uint64_t per = (jb.np + gridDim.x - 1) / gridDim.x;
  uint64_t r0 = blockIdx.x * per, r1 = r0 + per < jb.np ? r0 + per : jb.np;
  unsigned long long cnt = 0, sum = 0;
  if (r0 < r1) batch_probe_rows<K>(jb, r0, r1, slot_shift, cnt, sum);
  block_add2(cnt, sum, acc);
}

// Set every slot's key to the empty marker (int32 keys: word 0; int64 keys: word 1) and zero
// the rest, over all jobs' tables (one contiguous region), plus the per-job side records.
__global__ void k_batch_init(uint32_t* slots, uint64_t n_slots, uint32_t slot_words, uint32_t key_size) {
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < n_slots;
       s += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t* w = slots + s * slot_words;
    for (uint32_t i = 0; i < slot_words; ++i) w[i] = 0;
    w[key_size == 4 ? 0 : 1] = 0x80000000u;
  }
}

// Per-job smallest and largest build key (order-preserving unsigned form) over tiles of
// tile_rows rows: mm[2 j] = min, mm[2 j + 1] = max (set to ~0 and 0 beforehand).
struct MmJob {
  const void* key;
  uint64_t n;
  uint64_t tile0;
};

template <typename K>
__global__ void __launch_bounds__(256) k_batch_minmax(const MmJob* jobs, uint32_t n_jobs, uint64_t tiles,
                                                      uint32_t tile_rows, unsigned long long* mm) {
  __shared__ unsigned long long t0[kMaxBatchJobs];
  __shared__ unsigned long long rmin[4], rmax[4];
  for (uint32_t j = threadIdx.x; j < n_jobs; j += blockDim.x) t0[j] = jobs[j].tile0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    uint32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (t0[mid] <= t) lo = mid;
      else hi = mid;
    }
    const MmJob jb = jobs[lo];
    const uint64_t r0 = (t - jb.tile0) * tile_rows, r1 = r0 + tile_rows < jb.n ? r0 + tile_rows : jb.n;
    unsigned long long mn = ~0ull, mx = 0;
    for (uint64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
      const unsigned long long o = key_ord(((const K*)jb.key)[i]);
      mn = o < mn ? o : mn;
      mx = o > mx ? o : mx;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
      mn = a < mn ? a : mn;
      mx = b > mx ? b : mx;
    }
    if (lane == 0) {
      rmin[wave] = mn;
      rmax[wave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < 4; ++w) {
        mn = rmin[w] < mn ? rmin[w] : mn;
        mx = rmax[w] > mx ? rmax[w] : mx;
      }
      atomicMin(mm + 2 * (uint64_t)lo, mn);
      atomicMax(mm + 2 * (uint64_t)lo + 1, mx);
    }
    __syncthreads();
  }
}

__global__ void k_mm_init(unsigned long long* mm, uint32_t n_jobs) {
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_jobs; j += gridDim.x * blockDim.x) {
    mm[2 * (uint64_t)j] = ~0ull;
    mm[2 * (uint64_t)j + 1] = 0;
  }
}

// ---------------------------------------------------------------- host side

struct BatchConfig {
  uint32_t tile_rows = 4096;
  uint32_t block = 256;
  float load_factor = 0.5f;
};

struct BatchPlan {
  std::vector<BatchJob> jobs;      // in tile order (largest probe side first)
  std::vector<uint32_t> job_of;    // caller's job index of jobs[i]
  uint64_t build_tiles = 0, probe_tiles = 0, count_tiles = 0;
  uint64_t total_tiles = 0;
  uint64_t slots = 0;              // hash slots of all hash-table jobs (one region, first)
  // Tile maps of the two phases, kXcds interleaved lists: entry 8 q + x is list x's q-th tile
  // (job << 32 | the job's tile), ~0 when list x is shorter.  Workgroup b runs on XCD b mod 8
  // and a grid of a multiple of 8 workgroups walks tile t on workgroup t mod grid, so list x
  // runs on XCD x.  A job's build and probe tiles go to the same XCD.
  std::vector<unsigned long long> build_map, probe_map;
  uint64_t direct_bytes = 0;       // bitmaps and payloads of the direct-table jobs (after them)
  uint32_t slot_shift = 3;
};

// Which jobs get a direct table: per caller's job, direct[j] and the smallest key kmin[j]
// (order-preserving unsigned form).
struct DirectInfo {
  std::vector<uint8_t> direct;
  std::vector<unsigned long long> kmin;
  bool operator==(const DirectInfo& o) const { return direct == o.direct && kmin == o.kmin; }
};

uint64_t align256(uint64_t v) { return (v + 255) / 256 * 256; }

uint64_t direct_region_bytes(uint64_t nb, uint32_t ps) {
  return align256((nb + 63) / 64 * 8) + align256(nb * ps);
}

// Min and max build key of every job in one launch; a job is direct when its nb keys could be
// exactly the nb values from its min to its max.
static vx_status find_direct(vx_ctx* ctx, const vx_batch_join* d, int ks, DirectInfo* di) {
  const uint32_t J = d->n_jobs;
  const uint32_t tile_rows = 65536;
  std::vector<MmJob> mj(J);
  uint64_t tiles = 0;
  for (uint32_t j = 0; j < J; ++j) {
    mj[j].key = d->build_key[j].data;
    mj[j].n = d->n_build[j];
    mj[j].tile0 = tiles;
    tiles += (d->n_build[j] + tile_rows - 1) / tile_rows;
  }
  di->direct.assign(J, 0);
  di->kmin.assign(J, 0);
  if (!tiles) return VX_OK;
  ArenaBlock blk;
  blk.a = &ctx->arena;
  blk.p = ctx->arena.alloc(align256((uint64_t)J * sizeof(MmJob)) + (uint64_t)J * 16);
  VX_CHECK(blk.p, VX_EBUDGET, "batch: no room for the key ranges");
  MmJob* mjd = (MmJob*)blk.p;
  unsigned long long* mm = (unsigned long long*)(blk.p + align256((uint64_t)J * sizeof(MmJob)));
  VX_HIP(hipMemcpyAsync(mjd, mj.data(), (uint64_t)J * sizeof(MmJob), hipMemcpyHostToDevice, ctx->compute));
  hipLaunchKernelGGL(k_mm_init, dim3((J + 255) / 256), dim3(256), 0, ctx->compute, mm, J);
  const unsigned g = (unsigned)std::min<uint64_t>(tiles, (uint64_t)ctx->cu_count * 8);
  if (ks == 8)
    hipLaunchKernelGGL(k_batch_minmax<int64_t>, dim3(g), dim3(256), 0, ctx->compute, (const MmJob*)mjd, J, tiles,
                       tile_rows, mm);
  else
    hipLaunchKernelGGL(k_batch_minmax<int32_t>, dim3(g), dim3(256), 0, ctx->compute, (const MmJob*)mjd, J, tiles,
                       tile_rows, mm);
  VX_HIP(hipGetLastError());
  std::vector<unsigned long long> h(2 * (uint64_t)J);
  VX_HIP(hipMemcpyAsync(h.data(), mm, h.size() * 8, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  for (uint32_t j = 0; j < J; ++j) {
    const uint64_t nb = d->n_build[j];
    const unsigned long long mn = h[2 * j], mx = h[2 * j + 1];
    di->direct[j] = nb >= 1 && mx >= mn && mx - mn == nb - 1;
    di->kmin[j] = mn;
  }
  return VX_OK;
}

constexpr uint32_t kXcds = 8;   // accelerator complex dies of the MI355X, each with its own L2

// The XCD-aware tile maps.  A job whose table fits in 3/4 of one XCD's L2 gets all of its tiles
// on one XCD (jobs spread over the XCDs longest probe side first, balancing probe tiles), so its
// table is built and read in that L2 only.  Larger jobs spread their tiles over every XCD in
// turn and come first in every list.
static void map_tiles(BatchPlan* pl, uint32_t slot_bytes, uint64_t l2_bytes) {
  const uint32_t J = (uint32_t)pl->jobs.size();
  std::vector<std::vector<unsigned long long>> bl(kXcds), pr(kXcds);
  std::vector<uint32_t> small;
  uint32_t rb = 0, rp = 0;
  auto tiles = [](std::vector<unsigned long long>& l, uint32_t i, uint32_t n) {
    for (uint32_t k = 0; k < n; ++k) l.push_back(((unsigned long long)i << 32) | k);
  };
  for (uint32_t i = 0; i < J; ++i) {
    const BatchJob& b = pl->jobs[i];
    const uint64_t table = b.direct ? b.nb * (uint64_t)b.pay_size : (b.mask + 1) * (uint64_t)slot_bytes;
    if (table <= l2_bytes / 4 * 3) {
      small.push_back(i);
      continue;
    }
    for (uint32_t k = 0; k < b.build_tiles; ++k) bl[rb++ % kXcds].push_back(((unsigned long long)i << 32) | k);
    for (uint32_t k = 0; k < b.probe_tiles; ++k) pr[rp++ % kXcds].push_back(((unsigned long long)i << 32) | k);
  }
  std::stable_sort(small.begin(), small.end(),
                   [&](uint32_t a, uint32_t b) { return pl->jobs[a].probe_tiles > pl->jobs[b].probe_tiles; });
  for (uint32_t i : small) {
    uint32_t x = 0;
    for (uint32_t y = 1; y < kXcds; ++y)
      if (pr[y].size() < pr[x].size()) x = y;
    tiles(bl[x], i, pl->jobs[i].build_tiles);
    tiles(pr[x], i, pl->jobs[i].probe_tiles);
  }
  auto flatten = [](const std::vector<std::vector<unsigned long long>>& lists, std::vector<unsigned long long>* out) {
    size_t len = 0;
    for (const auto& l : lists) len = std::max(len, l.size());
    out->assign(len * kXcds, ~0ull);
    for (uint32_t x = 0; x < kXcds; ++x)
      for (size_t q = 0; q < lists[x].size(); ++q) (*out)[q * kXcds + x] = lists[x][q];
  };
  flatten(bl, &pl->build_map);
  flatten(pr, &pl->probe_map);
}

static vx_status plan_batch(const vx_batch_join* d, const BatchConfig& cfg, int ks, uint32_t ps,
                            const DirectInfo& di, uint64_t l2_bytes, BatchPlan* pl) {
  const uint32_t J = d->n_jobs;
  pl->jobs.resize(J);
  pl->job_of.resize(J);
  for (uint32_t j = 0; j < J; ++j) pl->job_of[j] = j;
  std::stable_sort(pl->job_of.begin(), pl->job_of.end(),
                   [&](uint32_t a, uint32_t b) { return d->n_probe[a] > d->n_probe[b]; });
  uint32_t slot_bytes = 8;
  while (slot_bytes < (uint32_t)ks + ps) slot_bytes <<= 1;
  if (ks == 8 && ps) slot_bytes = 16;
  pl->slot_shift = 0;
  while ((1u << pl->slot_shift) < slot_bytes) ++pl->slot_shift;
  uint64_t bt = 0, pt = 0, ct = 0, slots = 0, dbytes = 0;
  for (uint32_t i = 0; i < J; ++i) {
    const uint32_t j = pl->job_of[i];
    BatchJob& b = pl->jobs[i];
    std::memset(&b, 0, sizeof b);
    b.bkey = d->build_key[j].data;
    b.bpay = d->build_pay ? d->build_pay[j].data : nullptr;
    b.pkey = d->probe_key[j].data;
    b.nb = d->n_build[j];
    b.np = d->n_probe[j];
    b.pay_size = b.bpay ? (uint32_t)ps : 0;
    if (di.direct[j]) {
      // offsets are relocated once memory is carved: direct regions follow the hash slots
      b.direct = 1;
      b.kmin_ord = di.kmin[j];
      b.slots = (uint8_t*)(uintptr_t)dbytes;
      dbytes += direct_region_bytes(b.nb, b.pay_size);
    } else {
      uint64_t want = (uint64_t)std::ceil((double)std::max<uint64_t>(b.nb, 1) / cfg.load_factor);
      uint64_t cap = 64;
      while (cap < want) cap <<= 1;
      b.mask = cap - 1;
      b.log2cap = 0;
      while ((1ull << b.log2cap) < cap) ++b.log2cap;
      b.slots = (uint8_t*)(uintptr_t)slots;
      slots += cap;
    }
    b.ctile0 = ct;
    b.build_tiles = (uint32_t)((b.nb + cfg.tile_rows - 1) / cfg.tile_rows);
    b.probe_tiles = (uint32_t)((b.np + cfg.tile_rows - 1) / cfg.tile_rows);
    b.count_tiles = b.direct ? (uint32_t)(((b.nb + 63) / 64 + kCountWords - 1) / kCountWords) : 0;
    bt += b.build_tiles;
    pt += b.probe_tiles;
    ct += b.count_tiles;
  }
  pl->build_tiles = bt;
  pl->probe_tiles = pt;
  pl->count_tiles = ct;
  pl->total_tiles = bt + pt;
  pl->slots = slots;
  pl->direct_bytes = dbytes;
  map_tiles(pl, slot_bytes, l2_bytes);
  return VX_OK;
}

struct BatchRun {
  ArenaBlock mem;              // slots, side records, descriptors, counters, accumulators
  BatchPlan plan;
  BatchJob* jobs_dev = nullptr;
  unsigned long long* counters = nullptr;   // sides, accumulators, bit counts (cleared together)
  unsigned long long* acc = nullptr;         // per job (tile order): count, sum
  unsigned long long* bits = nullptr;        // per job (tile order): bits set in its direct bitmap
  unsigned long long* probe_map = nullptr;   // the plan's tile maps, in device memory
  unsigned long long* build_map = nullptr;
  uint8_t* slots = nullptr;
  uint64_t counter_words = 0;
};

static vx_status setup_run(vx_ctx* ctx, const vx_batch_join* d, const BatchConfig& cfg, int ks,
                           uint32_t ps, const DirectInfo& di, BatchRun* r) {
  VX_TRY(plan_batch(d, cfg, ks, ps, di, ctx->l2_bytes, &r->plan));
  const uint32_t J = d->n_jobs;
  const uint64_t hash_bytes = align256(r->plan.slots << r->plan.slot_shift);
  uint64_t slot_bytes = hash_bytes + r->plan.direct_bytes;
  uint64_t side_bytes = (uint64_t)J * 16;
  uint64_t desc_bytes = (uint64_t)J * sizeof(BatchJob);
  // side records and accumulators are contiguous so one fill kernel clears them
  r->counter_words = 2 * (uint64_t)J + 2 * (uint64_t)J + (uint64_t)J;
  const uint64_t bmap_bytes = r->plan.build_map.size() * 8, map_bytes = r->plan.probe_map.size() * 8;
  uint64_t bytes = slot_bytes + 256 + desc_bytes + 256 + r->counter_words * 8 + 256 + map_bytes + 256 + bmap_bytes + 256;
  r->mem.a = &ctx->arena;
  r->mem.p = ctx->arena.alloc(bytes);
  VX_CHECK(r->mem.p, VX_EBUDGET, "batch: %llu bytes of tables and descriptors do not fit the arena",
           (unsigned long long)bytes);
  r->slots = r->mem.p;
  uint8_t* q = r->mem.p + ((slot_bytes + 255) / 256) * 256;
  r->jobs_dev = (BatchJob*)q;
  q += ((desc_bytes + 255) / 256) * 256;
  r->counters = (unsigned long long*)q;
  unsigned long long* sides = r->counters;
  r->acc = sides + 2 * (uint64_t)J;
  r->bits = r->acc + 2 * (uint64_t)J;
  r->probe_map = (unsigned long long*)(q + align256(r->counter_words * 8));
  r->build_map = (unsigned long long*)((uint8_t*)r->probe_map + align256(map_bytes));
  (void)side_bytes;
  for (uint32_t j = 0; j < J; ++j) {
    BatchJob& b = r->plan.jobs[j];
    if (b.direct) {
      b.slots = r->slots + hash_bytes + (uint64_t)(uintptr_t)b.slots;
      b.dpay = b.slots + align256((b.nb + 63) / 64 * 8);
    } else {
      b.slots = r->slots + (((uint64_t)(uintptr_t)b.slots) << r->plan.slot_shift);
    }
    b.side = sides + 2 * (uint64_t)j;
  }
  (void)side_bytes;
  VX_HIP(hipMemcpyAsync(r->jobs_dev, r->plan.jobs.data(), desc_bytes, hipMemcpyHostToDevice, ctx->compute));
  if (map_bytes)
    VX_HIP(hipMemcpyAsync(r->probe_map, r->plan.probe_map.data(), map_bytes, hipMemcpyHostToDevice, ctx->compute));
  if (bmap_bytes)
    VX_HIP(hipMemcpyAsync(r->build_map, r->plan.build_map.data(), bmap_bytes, hipMemcpyHostToDevice, ctx->compute));
  return VX_OK;
}

static void launch_dupcount(vx_ctx* ctx, const BatchRun& r, uint32_t J, hipStream_t s) {
  if (!r.plan.count_tiles) return;
  const unsigned g = (unsigned)std::min<uint64_t>(r.plan.count_tiles, (uint64_t)ctx->cu_count * 4);
  hipLaunchKernelGGL(k_batch_dupcount, dim3(g), dim3(256), 0, s, r.jobs_dev, J, r.plan.count_tiles, r.bits);
}

// A direct-table job whose bitmap holds fewer than nb bits had a repeated build key.
static bool direct_dups(const BatchPlan& pl, const unsigned long long* bits) {
  for (size_t i = 0; i < pl.jobs.size(); ++i)
    if (pl.jobs[i].direct && bits[i] != pl.jobs[i].nb) return true;
  return false;
}

// the work of one batch on `s`: init tables, clear results, build phase, probe phase, results
// to the host (accumulators are in tile order; the caller maps them back through job_of)
static vx_status enqueue_batch(vx_ctx* ctx, const BatchRun& r, const BatchConfig& cfg, int ks,
                               uint32_t J, hipStream_t s, uint64_t* host_out) {
  uint32_t sw = (1u << r.plan.slot_shift) / 4;
  unsigned ig = (unsigned)std::min<uint64_t>((r.plan.slots + 255) / 256, (uint64_t)ctx->cu_count * 16);
  if (r.plan.slots)
    hipLaunchKernelGGL(k_batch_init, dim3(std::max(ig, 1u)), dim3(256), 0, s, (uint32_t*)r.slots, r.plan.slots,
                       sw, (uint32_t)ks);
  if (r.plan.direct_bytes)
    fill_zero((uint64_t*)(r.slots + align256(r.plan.slots << r.plan.slot_shift)), r.plan.direct_bytes / 8, s);
  fill_zero((uint64_t*)r.counters, r.counter_words, s);
  fill_zero((uint64_t*)ctx->dev_flags, 1, s);
  const uint64_t per_cu = cfg.block >= 512 ? 4 : 8;
  // the tile maps assume grids of a multiple of kXcds workgroups (see BatchPlan::probe_map)
  const uint64_t bmapped = r.plan.build_map.size(), mapped = r.plan.probe_map.size();
  unsigned gb = (unsigned)std::min<uint64_t>(std::max<uint64_t>(bmapped, 1), ctx->cu_count * per_cu);
  gb = std::max(kXcds, gb / kXcds * kXcds);
  unsigned gp = (unsigned)std::min<uint64_t>(std::max<uint64_t>(mapped, 1), ctx->cu_count * per_cu);
  gp = std::max(kXcds, gp / kXcds * kXcds);
  const unsigned long long* bmap = r.build_map;
  if (ks == 8)
    hipLaunchKernelGGL((k_batch_phase<int64_t, true>), dim3(gb), dim3(cfg.block), 0, s, r.jobs_dev, J,
                       (uint64_t)bmapped, cfg.tile_rows, r.plan.slot_shift, r.acc, ctx->dev_flags, bmap);
  else
    hipLaunchKernelGGL((k_batch_phase<int32_t, true>), dim3(gb), dim3(cfg.block), 0, s, r.jobs_dev, J,
                       (uint64_t)bmapped, cfg.tile_rows, r.plan.slot_shift, r.acc, ctx->dev_flags, bmap);
  launch_dupcount(ctx, r, J, s);
  const unsigned long long* pmap = r.probe_map;
  if (ks == 8)
    hipLaunchKernelGGL((k_batch_phase<int64_t, false>), dim3(gp), dim3(cfg.block), 0, s, r.jobs_dev, J,
                       (uint64_t)mapped, cfg.tile_rows, r.plan.slot_shift, r.acc, ctx->dev_flags, pmap);
  else
    hipLaunchKernelGGL((k_batch_phase<int32_t, false>), dim3(gp), dim3(cfg.block), 0, s, r.jobs_dev, J,
                       (uint64_t)mapped, cfg.tile_rows, r.plan.slot_shift, r.acc, ctx->dev_flags, pmap);
  VX_HIP(hipGetLastError());
  if (host_out) {   // accumulators and bit counts are contiguous: 3 J words, then the flags
    VX_HIP(hipMemcpyAsync(host_out, r.acc, 3 * (uint64_t)J * 8, hipMemcpyDeviceToHost, s));
    VX_HIP(hipMemcpyAsync(host_out + 3 * (uint64_t)J, ctx->dev_flags, 4, hipMemcpyDeviceToHost, s));
  }
  return VX_OK;
}

struct TuneCache {
  std::map<std::string, BatchConfig> m;
};

static TuneCache g_tune;

static std::string class_key(const vx_ctx* ctx, const vx_batch_join* d, int ks) {
  uint64_t nb = 0, np = 0, mb = 0;
  for (uint32_t j = 0; j < d->n_jobs; ++j) {
    nb += d->n_build[j];
    np += d->n_probe[j];
    mb = std::max<uint64_t>(mb, d->n_build[j]);
  }
  auto lg = [](uint64_t v) { int r = 0; while ((1ull << r) < v) ++r; return r; };
  std::ostringstream o;
  o << "cu" << ctx->cu_count << "_k" << ks << "_j" << lg(d->n_jobs) << "_b" << lg(nb) << "_p" << lg(np)
    << "_m" << lg(mb);
  return o.str();
}

static bool load_tuned(const std::string& key, BatchConfig* c) {
  auto it = g_tune.m.find(key);
  if (it != g_tune.m.end()) {
    *c = it->second;
    return true;
  }
  const char* path = getenv("VX_TUNE_CACHE");
  if (!path) return false;
  std::ifstream f(path);
  std::string k;
  BatchConfig v;
  bool found = false;
  while (f >> k >> v.tile_rows >> v.block >> v.load_factor)
    if (k == key) {
      *c = v;
      found = true;
    }
  if (found) g_tune.m[key] = *c;
  return found;
}

static void store_tuned(const std::string& key, const BatchConfig& c) {
  g_tune.m[key] = c;
  const char* path = getenv("VX_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << c.tile_rows << " " << c.block << " " << c.load_factor << "\n";
}

static vx_status time_config(vx_ctx* ctx, const vx_batch_join* d, const BatchConfig& cfg, int ks, uint32_t ps,
                             const DirectInfo& di, float* ms) {
  BatchRun r;
  VX_TRY(setup_run(ctx, d, cfg, ks, ps, di, &r));
  hipEvent_t a = get_event(ctx), b = get_event(ctx);
  VX_TRY(enqueue_batch(ctx, r, cfg, ks, d->n_jobs, ctx->compute, nullptr));   // warm
  VX_HIP(hipEventRecord(a, ctx->compute));
  VX_TRY(enqueue_batch(ctx, r, cfg, ks, d->n_jobs, ctx->compute, nullptr));
  VX_HIP(hipEventRecord(b, ctx->compute));
  VX_HIP(hipEventSynchronize(b));
  VX_HIP(hipEventElapsedTime(ms, a, b));
  put_event(ctx, a);
  put_event(ctx, b);
  return check_flags(ctx, "batch autotune");
}

static vx_status autotune(vx_ctx* ctx, const vx_batch_join* d, int ks, uint32_t ps, const DirectInfo& di,
                          BatchConfig* best) {
  std::string key = class_key(ctx, d, ks);
  uint32_t n_direct = 0;
  for (uint8_t x : di.direct) n_direct += x;
  key += "_d" + std::to_string(n_direct == 0 ? 0 : n_direct == d->n_jobs ? 2 : 1);
  if (load_tuned(key, best)) return VX_OK;
  float best_ms = 1e30f;
  for (uint32_t tile : {2048u, 8192u, 32768u})
    for (uint32_t block : {256u, 512u})
      for (float lf : {0.5f, 0.7f}) {
        BatchConfig c{tile, block, lf};
        float ms = 0;
        VX_TRY(time_config(ctx, d, c, ks, ps, di, &ms));
        if (ms < best_ms) {
          best_ms = ms;
          *best = c;
        }
      }
  store_tuned(key, *best);
  return VX_OK;
}

struct JobKey {
  const void *bkey, *bpay, *pkey;
  uint64_t nb, np;
  bool operator==(const JobKey& o) const {
    return bkey == o.bkey && bpay == o.bpay && pkey == o.pkey && nb == o.nb && np == o.np;
  }
};

static std::vector<JobKey> job_keys(const vx_batch_join* d) {
  std::vector<JobKey> k(d->n_jobs);
  for (uint32_t j = 0; j < d->n_jobs; ++j)
    k[j] = {d->build_key[j].data, d->build_pay ? d->build_pay[j].data : nullptr, d->probe_key[j].data,
            d->n_build[j], d->n_probe[j]};
  return k;
}

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<JobKey> key;
  DirectInfo di;
  BatchConfig cfg;
  BatchRun* run = nullptr;
};

static std::map<const vx_ctx*, GraphCache*> g_graphs;

static void drop_graph(GraphCache* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g->run;
  delete g;
}


void batch_release_ctx(const vx_ctx* ctx) {
  auto it = g_graphs.find(ctx);
  if (it != g_graphs.end()) {
    drop_graph(it->second);
    g_graphs.erase(it);
  }
}

vx_status join_batch(vx_ctx* ctx, const vx_batch_join* d, vx_join_out* out) {
  double t0 = now_ms();
  VX_CHECK(d->n_jobs <= kMaxBatchJobs, VX_EINVAL, "batch: %u jobs (max %u)", d->n_jobs, kMaxBatchJobs);
  VX_CHECK(d->n_jobs == 0 || (d->build_key && d->n_build && d->probe_key && d->n_probe && d->out),
           VX_EINVAL, "batch: null job arrays");
  VX_CHECK(d->mode == 0 || d->mode == 1, VX_EINVAL, "batch: mode %d", d->mode);
  VX_HIP(hipSetDevice(ctx->device));
  if (d->n_jobs == 0) return VX_OK;
  const int32_t kt = d->build_key[0].type;
  const int ks = elsize_of(kt);
  VX_CHECK(ks, VX_EINVAL, "batch: key type %d", kt);
  int32_t pt = 0;
  for (uint32_t j = 0; j < d->n_jobs; ++j) {
    VX_CHECK(d->build_key[j].type == kt && d->probe_key[j].type == kt, VX_EINVAL,
             "batch: every job must use the same key type");
    ColInfo ci;
    VX_TRY(classify(ctx, d->build_key[j], d->n_build[j], &ci, "batch build key"));
    VX_CHECK(ci.where == Where::Device, VX_EINVAL, "batch: job %u build keys must be device-resident", j);
    VX_TRY(classify(ctx, d->probe_key[j], d->n_probe[j], &ci, "batch probe key"));
    VX_CHECK(ci.where == Where::Device, VX_EINVAL, "batch: job %u probe keys must be device-resident", j);
    if (d->build_pay && d->build_pay[j].data) {
      VX_CHECK(pt == 0 || pt == d->build_pay[j].type, VX_EINVAL, "batch: payload types differ");
      pt = d->build_pay[j].type;
      VX_TRY(classify(ctx, d->build_pay[j], d->n_build[j], &ci, "batch build payload"));
      VX_CHECK(ci.where == Where::Device, VX_EINVAL, "batch: job %u payload must be device-resident", j);
    }
  }
  const uint32_t ps = pt ? (uint32_t)elsize_of(pt) : 0;
  const uint32_t J = d->n_jobs;
  // which jobs take a direct table depends on the keys' values: measured on every call
  DirectInfo di;
  VX_CHECK((d->flags & ~(uint32_t)VX_HASHED) == 0, VX_EINVAL, "batch: unknown flags %u", d->flags);
  if (d->flags & VX_HASHED) {   // every job hashed: no key-range pass
    di.direct.assign(J, 0);
    di.kmin.assign(J, 0);
  } else {
    VX_TRY(find_direct(ctx, d, ks, &di));
  }
  const double t_checked = now_ms();
  BatchConfig cfg;
  bool tuned = d->tile_rows == 0 || d->block == 0 || d->load_factor == 0.0f;
  if (tuned && d->mode == 0) VX_TRY(autotune(ctx, d, ks, ps, di, &cfg));
  const double t_tuned = now_ms();
  if (d->tile_rows) cfg.tile_rows = d->tile_rows;
  if (d->block) cfg.block = d->block;
  if (d->load_factor > 0) cfg.load_factor = d->load_factor;
  VX_CHECK(cfg.block == 256 || cfg.block == 512, VX_EINVAL, "batch: block %u (256 or 512)", cfg.block);
  VX_CHECK(cfg.tile_rows >= 64, VX_EINVAL, "batch: tile_rows %u < 64", cfg.tile_rows);
  VX_CHECK(cfg.load_factor > 0.05f && cfg.load_factor <= 0.95f, VX_EINVAL, "batch: load factor");

  std::vector<uint64_t> host(2 * (uint64_t)J + 1, 0);
  std::vector<uint32_t> order;   // baseline: tile order of its plan
  vx_stats& s = out->stats;
  std::memset(&s, 0, sizeof s);
  if (d->mode == 0) {
    GraphCache*& gc = g_graphs[ctx];
    if (!gc || !(gc->key == job_keys(d)) || !(gc->di == di) || gc->cfg.tile_rows != cfg.tile_rows ||
        gc->cfg.block != cfg.block || gc->cfg.load_factor != cfg.load_factor) {
      drop_graph(gc);
      gc = nullptr;
      // the new entry is cached only once its graph is instantiated: a failure part-way leaves
      // no entry, so the next call builds the graph again
      GraphCache* ng = new GraphCache;
      ng->run = new BatchRun;
      ng->cfg = cfg;
      auto build = [&]() -> vx_status {
        VX_TRY(setup_run(ctx, d, cfg, ks, ps, di, ng->run));
        VX_HIP(hipStreamSynchronize(ctx->compute));
        VX_HIP(hipStreamBeginCapture(ctx->compute, hipStreamCaptureModeThreadLocal));
        vx_status cst = enqueue_batch(ctx, *ng->run, cfg, ks, J, ctx->compute, ctx->host_acc);
        hipError_t ce = hipStreamEndCapture(ctx->compute, &ng->graph);
        VX_TRY(cst);
        VX_HIP(ce);
        VX_HIP(hipGraphInstantiate(&ng->exec, ng->graph, nullptr, nullptr, 0));
        return VX_OK;
      };
      const vx_status bst = build();
      if (bst != VX_OK) {
        (void)hipStreamSynchronize(ctx->compute);
        drop_graph(ng);
        return bst;
      }
      ng->key = job_keys(d);
      ng->di = di;
      gc = ng;
    }
    hipEvent_t a = get_event(ctx), b = get_event(ctx);
    VX_HIP(hipEventRecord(a, ctx->compute));
    VX_HIP(hipGraphLaunch(gc->exec, ctx->compute));
    VX_HIP(hipEventRecord(b, ctx->compute));
    VX_HIP(hipStreamSynchronize(ctx->compute));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    put_event(ctx, a);
    put_event(ctx, b);
    std::memcpy(host.data(), ctx->host_acc, (2 * (uint64_t)J) * 8);
    unsigned int f = 0;
    std::memcpy(&f, ctx->host_acc + 3 * (uint64_t)J, 4);
    VX_CHECK(!(f & kFlagDup) && !direct_dups(gc->run->plan, (const unsigned long long*)ctx->host_acc + 2 * (uint64_t)J),
             VX_EDUPKEY, "batch: duplicate build key");
    VX_CHECK(!(f & kFlagFull), VX_ECAPACITY, "batch: table full (internal sizing error)");
    s.kernel_ms = ms;
    s.kernel_launches = gc->run->plan.count_tiles ? 3 : 2;   // build phase, bit count, probe phase
    s.table_bytes = (gc->run->plan.slots << gc->run->plan.slot_shift) + gc->run->plan.direct_bytes;
    s.chunk_rows = cfg.tile_rows;
    s.n_buffers = cfg.block;
    s.imbalance = cfg.load_factor;
  } else {
    BatchRun r;
    VX_TRY(setup_run(ctx, d, cfg, ks, ps, di, &r));
    uint32_t sw = (1u << r.plan.slot_shift) / 4;
    fill_zero((uint64_t*)r.counters, r.counter_words, ctx->compute);
    fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);
    hipEvent_t a = get_event(ctx), b = get_event(ctx);
    VX_HIP(hipEventRecord(a, ctx->compute));
    for (uint32_t j = 0; j < J; ++j) {
      const BatchJob& jb = r.plan.jobs[j];
      if (jb.direct) {
        fill_zero((uint64_t*)jb.slots, direct_region_bytes(jb.nb, jb.pay_size) / 8, ctx->compute);
      } else {
        uint64_t cap = jb.mask + 1;
        unsigned ig = (unsigned)std::min<uint64_t>((cap + 255) / 256, (uint64_t)ctx->cu_count * 16);
        hipLaunchKernelGGL(k_batch_init, dim3(ig), dim3(256), 0, ctx->compute, (uint32_t*)jb.slots, cap, sw,
                           (uint32_t)ks);
      }
      unsigned gb = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((jb.nb + cfg.tile_rows - 1) / cfg.tile_rows,
                                                                       (uint64_t)ctx->cu_count * 8));
      unsigned gp = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((jb.np + cfg.tile_rows - 1) / cfg.tile_rows,
                                                                       (uint64_t)ctx->cu_count * 8));
      if (ks == 8) {
        hipLaunchKernelGGL(k_job_build<int64_t>, dim3(gb), dim3(cfg.block), 0, ctx->compute, jb, r.plan.slot_shift,
                           ctx->dev_flags);
        hipLaunchKernelGGL(k_job_probe<int64_t>, dim3(gp), dim3(cfg.block), 0, ctx->compute, jb, r.plan.slot_shift,
                           r.acc + 2 * (uint64_t)j);
      } else {
        hipLaunchKernelGGL(k_job_build<int32_t>, dim3(gb), dim3(cfg.block), 0, ctx->compute, jb, r.plan.slot_shift,
                           ctx->dev_flags);
        hipLaunchKernelGGL(k_job_probe<int32_t>, dim3(gp), dim3(cfg.block), 0, ctx->compute, jb, r.plan.slot_shift,
                           r.acc + 2 * (uint64_t)j);
      }
    }
    launch_dupcount(ctx, r, J, ctx->compute);
    VX_HIP(hipGetLastError());
    VX_HIP(hipEventRecord(b, ctx->compute));
    std::vector<unsigned long long> bits(J);
    VX_HIP(hipMemcpyAsync(host.data(), r.acc, 2 * (uint64_t)J * 8, hipMemcpyDeviceToHost, ctx->compute));
    VX_HIP(hipMemcpyAsync(bits.data(), r.bits, (uint64_t)J * 8, hipMemcpyDeviceToHost, ctx->compute));
    VX_HIP(hipStreamSynchronize(ctx->compute));
    VX_CHECK(!direct_dups(r.plan, bits.data()), VX_EDUPKEY, "batch: duplicate build key");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    put_event(ctx, a);
    put_event(ctx, b);
    VX_TRY(check_flags(ctx, "batch"));
    order = r.plan.job_of;
    s.kernel_ms = ms;
    s.kernel_launches = 3 * (uint64_t)J + (r.plan.count_tiles ? 1 : 0);
    s.table_bytes = (r.plan.slots << r.plan.slot_shift) + r.plan.direct_bytes;
  }
  // accumulators are in tile order: entry i belongs to the caller's job job_of[i]
  const std::vector<uint32_t>& job_of = d->mode == 0 ? g_graphs[ctx]->run->plan.job_of : order;
  uint64_t rows = 0;
  for (uint32_t i = 0; i < J; ++i) {
    const uint32_t j = job_of[i];
    std::memset(&d->out[j], 0, sizeof(vx_agg));
    d->out[j].match_count = host[2 * i];
    d->out[j].sum[0] = host[2 * i + 1];
    rows += d->n_probe[j];
  }
  s.rows = rows;
  s.total_ms = now_ms() - t0;
  if (getenv("VX_TRACE"))
    fprintf(stderr, "[vx] batch mode %d: checks %.2f ms, tuning %.2f ms, run %.2f ms (kernels %.2f ms)\n", d->mode,
            t_checked - t0, t_tuned - t_checked, now_ms() - t_tuned, s.kernel_ms);
  return VX_OK;
}

}  // namespace vx
