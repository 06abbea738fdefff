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
// a hash table: the payload of key k sits at k - min, and a presence byte per key of the range
// catches a duplicate (which would leave a key of the range missing).  The build sets the bytes
// with plain stores (distinct keys never share a byte, so no atomic is needed); a small kernel
// between the two phases counts each job's set bytes, and the host compares the count with the
// job's rows.  A probe key outside the range then costs no memory access, and one inside reads
// one payload.
//
// Random table reads are what bounds the probe: served by the L2 they reach about half of its
// request rate, and a table larger than one L2 is read from the MALL or HBM.  So the probe phase
// reads every table from LDS instead.  A table of at most 128 KiB is staged whole by each probe
// work item.  A larger one is cut into regions of 128 KiB (key - min for a direct table, the top
// bits of the first slot for a hash table), and the job's probe keys are first partitioned by
// region into one contiguous array per region: a count pass tallies each super-tile's keys per
// region, a per-job scan turns the tallies into positions, and a scatter pass moves the keys.  A
// probe work item (one 1024-thread workgroup per compute unit, its LDS) then stages its region
// and streams its share of the region's keys, about a million.
// Count, scan and scatter run on a second stream, the build phase beside the scatter.  Keys that
// cannot match are dropped: outside the range of a direct table, or outside the smallest and
// largest build key of a hash table (measured with the ranges, on every call).
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
                          // direct: a presence byte per key of the range, then the payloads
  uint8_t* dpay;          // direct: payload of key kmin + i at index i
  unsigned long long kmin_ord;   // direct: the smallest key, order-preserving unsigned form
  uint32_t direct;        // 1: direct table
  uint64_t mask;
  uint32_t log2cap;
  uint32_t pay_size;      // 0 (no payload), 4 or 8
  uint64_t ctile0;        // first presence-count tile of the job (direct tables)
  uint32_t build_tiles, probe_tiles, count_tiles;
  unsigned long long* side;   // sentinel-key record: count, payload sum
  unsigned long long kmax_ord;   // hash: the largest build key (with kmin_ord, the zone a match needs)
  // probe by regions (n_parts 0: the probe tiles read the job's own keys, tables from memory)
  uint32_t n_parts;         // table regions: a key's region is (key - min, or first slot) >> part_shift
  uint32_t part_shift;
  uint32_t in_place;        // 1: one region, probed from the job's own keys (no partitioning)
  uint32_t staged;          // 1: a probe work item holds its region of the table in LDS
  uint32_t ptiles;          // partition tiles of kPartRows probe rows
  uint32_t stiles;          // super-tiles of kSuperTiles partition tiles
  uint32_t items_per_region;   // probe work items per region
  uint64_t cbase;           // the job's tallies: entry cbase + super-tile * n_parts + region
  uint8_t* pbuf;            // partitioned keys: the regions' arrays, in region order, then the sink slots
  unsigned long long* kept; // keys kept by the partitioning (written by the scan)
};

constexpr uint32_t kMaxBatchJobs = 4096;
constexpr uint32_t kXcds = 8;   // accelerator complex dies of the MI355X, each with its own L2

// Device-memory accesses through pointers read from descriptors, as global (not flat) accesses:
// flat loads also count against the LDS counter, so every LDS wait would wait for them too.
#define VX_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gload(const void* base, uint64_t i) {
  return ((const VX_GLOBAL T*)base)[i];
}
template <typename T>
__device__ __forceinline__ T gload_nt(const void* base, uint64_t i) {
  return __builtin_nontemporal_load((const VX_GLOBAL T*)base + i);
}
template <typename T>
__device__ __forceinline__ void gstore(void* base, uint64_t i, T v) {
  ((VX_GLOBAL T*)base)[i] = v;
}
// the same, at a byte offset below 2^32 from a base common to the wave (one address register)
template <typename T>
__device__ __forceinline__ void gstore_at(void* base, uint32_t byte_off, T v) {
  *(VX_GLOBAL T*)((VX_GLOBAL uint8_t*)base + byte_off) = v;
}

// Rows [r0, r1) of a job's build side into its table.
template <typename K>
__device__ __forceinline__ void batch_build_rows(const BatchJob& jb, uint64_t r0, uint64_t r1,
                                                 uint32_t slot_shift, unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  for (uint64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    K k = ((const K*)jb.bkey)[i];
    U kb = (U)k;
    if (jb.direct) {
      // every build key lies in [kmin, kmin + nb): the range was measured over these keys.  The
      // presence byte is set by a plain store; k_batch_dupcount counts the set bytes afterwards,
      // and a job with fewer than nb of them had a repeated key.
      const uint64_t idx = key_ord(k) - jb.kmin_ord;
      const long long v = jb.pay_size ? load_signed(jb.bpay, i, jb.pay_size) : 0;
      jb.slots[idx] = 1;
      if (jb.pay_size == 4) ((int*)jb.dpay)[idx] = (int)v;
      else if (jb.pay_size == 8) ((long long*)jb.dpay)[idx] = v;
      continue;
    }
    const long long v = jb.pay_size ? load_signed(jb.bpay, i, jb.pay_size) : 0;
    if (kb == kEmpty) {
      unsigned long long prev = atomicAdd(jb.side, 1ull);
      if (prev) atomicOr(flags, kFlagDup);
      atomicAdd(jb.side + 1, (unsigned long long)v);
      continue;
    }
    uint64_t h = slot_of(key_bits(k), jb.log2cap);
    bool done = false;
    if constexpr (sizeof(K) == 4) {
      if (jb.pay_size != 8) {
        // an 8-byte slot (int32 key, int32 payload or none): one 64-bit compare-and-swap claims
        // the slot and writes the payload with it.  An empty slot is exactly (empty marker, 0):
        // the init zeroes payloads, and the empty-marker key itself goes to the side record.
        const unsigned long long empty = (unsigned long long)(uint32_t)kEmpty;
        const unsigned long long want = (unsigned long long)(uint32_t)kb | ((unsigned long long)(uint32_t)(int)v << 32);
        for (uint64_t step = 0; step <= jb.mask; ++step) {
          const unsigned long long prev = atomicCAS((unsigned long long*)(jb.slots + (h << slot_shift)), empty, want);
          if (prev == empty) {
            done = true;
            break;
          }
          if ((uint32_t)prev == (uint32_t)kb) {
            atomicOr(flags, kFlagDup);
            done = true;
            break;
          }
          h = (h + 1) & jb.mask;
        }
        if (!done) atomicOr(flags, kFlagFull);
        continue;
      }
    }
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
__device__ __forceinline__ void probe_key(const BatchJob& jb, K k, uint32_t slot_shift, unsigned long long& cnt,
                                          unsigned long long& sum) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  const U kb = (U)k;
  if (jb.direct) {
    const uint64_t idx = key_ord(k) - jb.kmin_ord;
    if (idx < jb.nb) {   // every key of the range is in the table (no duplicates: checked)
      cnt += 1;
      if (jb.pay_size == 4) sum += (unsigned long long)(long long)gload<int>(jb.dpay, idx);
      else if (jb.pay_size == 8) sum += (unsigned long long)gload<long long>(jb.dpay, idx);
    }
    return;
  }
  const unsigned long long ko = key_ord(k);
  if (ko < jb.kmin_ord || ko > jb.kmax_ord) return;   // outside the build keys' range: no match
  if (kb == kEmpty) {
    const unsigned long long c = gload<unsigned long long>(jb.side, 0);
    cnt += c;
    if (c) sum += gload<unsigned long long>(jb.side, 1);
    return;
  }
  uint64_t h = slot_of(key_bits(k), jb.log2cap);
  for (uint64_t step = 0; step <= jb.mask; ++step) {
    const uint8_t* slot = jb.slots + (h << slot_shift);
    const U sk = gload<U>(slot, 0);
    if (sk == kb) {
      cnt += 1;
      if (jb.pay_size == 4) sum += (unsigned long long)(long long)gload<int>(slot + sizeof(K), 0);
      else if (jb.pay_size == 8) sum += (unsigned long long)gload<long long>(slot + 8, 0);
      return;
    }
    if (sk == kEmpty) return;
    h = (h + 1) & jb.mask;
  }
}

template <typename K>
__device__ __forceinline__ void batch_probe_rows(const BatchJob& jb, uint64_t r0, uint64_t r1,
                                                 uint32_t slot_shift, unsigned long long& cnt,
                                                 unsigned long long& sum) {
  for (uint64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x)
    probe_key<K>(jb, gload_nt<K>(jb.pkey, i), slot_shift, cnt, sum);
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

// ---------------------------------------------------------------- probe-side partitioning

// A work-list entry read by the whole workgroup, made provably uniform, so that the descriptor
// it names is read with scalar loads and the code that depends on it does not branch per lane.
__device__ __forceinline__ unsigned long long uniform_entry(const unsigned long long* __restrict__ map, uint64_t i) {
  const unsigned long long e = map[i];
  return (unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)e) |
         ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(e >> 32)) << 32);
}

// A workgroup barrier that orders LDS only: global stores still in flight are not waited for.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr uint32_t kPartThreads = 256, kPartItems = 16, kPartRows = kPartThreads * kPartItems;
constexpr uint32_t kScatterItems = 16;               // keys per lane in a scatter round
constexpr uint32_t kSuperTiles = 16;                 // partition tiles per super-tile (65536 rows)
constexpr uint32_t kMaxTableParts = 1024;
constexpr uint32_t kScanBlock = 1024;
constexpr uint32_t kLdsBytes = 160 << 10;            // LDS per compute unit
constexpr uint32_t kRegionThreads = 1024;
constexpr uint32_t kStageBytes = 128 << 10;          // LDS for one table region
constexpr uint32_t kRunUnroll = 16;                  // keys in flight per lane in the region probe
constexpr uint32_t kSinkGroups = 256;                // scatter sink slots: 64 per group of workgroups

// How a job maps probe keys to table regions, read from its descriptor once (scalar registers).
struct RegionFn {
  unsigned long long kmin, kmax;
  uint64_t nb;
  uint32_t direct, shift, parts, log2cap;
  __device__ __forceinline__ explicit RegionFn(const BatchJob& jb)
      : kmin(jb.kmin_ord), kmax(jb.kmax_ord), nb(jb.nb), direct(jb.direct), shift(jb.part_shift),
        parts(jb.n_parts), log2cap(jb.log2cap) {}
  // the region of probe key k; `parts` for a key that cannot match
  template <typename K>
  __device__ __forceinline__ uint32_t operator()(K k) const {
    const unsigned long long ko = key_ord(k);
    if (direct) {
      const uint64_t idx = ko - kmin;
      return idx < nb ? (uint32_t)(idx >> shift) : parts;
    }
    if (ko < kmin || ko > kmax) return parts;
    return (uint32_t)(slot_of(key_bits(k), log2cap) >> shift);
  }
};

// Tile t's keys, kPartItems per thread: every load is issued (rows past the end reread the last
// row), so that no load sits behind a branch and waits stay exact.
template <typename K>
__device__ __forceinline__ void load_tile(const void* pkey, uint64_t np, uint64_t t, K (&k)[kPartItems]) {
  const uint64_t r0 = t * kPartRows;
  const uint32_t last = (uint32_t)(np - r0 < kPartRows ? np - r0 : kPartRows) - 1;
#pragma unroll
  for (uint32_t it = 0; it < kPartItems; ++it) {
    const uint32_t row = it * kPartThreads + threadIdx.x;
    k[it] = gload_nt<K>(pkey, r0 + (row < last ? row : last));
  }
}

// The regions of this thread's keys of tile t (`parts` for a key that cannot match or a row past
// the end).
template <typename K>
__device__ __forceinline__ void tile_regions(const RegionFn& region, uint64_t np, uint64_t t, const K (&k)[kPartItems],
                                             uint32_t (&r)[kPartItems]) {
  const uint64_t r0 = t * kPartRows;
  const uint32_t n = (uint32_t)(np - r0 < kPartRows ? np - r0 : kPartRows);
#pragma unroll
  for (uint32_t it = 0; it < kPartItems; ++it) {
    const uint32_t row = it * kPartThreads + threadIdx.x;
    r[it] = row < n ? region(k[it]) : region.parts;
  }
}

// Count pass (part_map[g] = job << 32 | super-tile): tally[cbase + st n_parts + r] = the
// super-tile's keys in region r.
template <typename K>
__global__ void __launch_bounds__(kPartThreads) k_batch_count(const BatchJob* __restrict__ jobs,
                                                              const unsigned long long* __restrict__ part_map,
                                                              uint64_t n_super, uint32_t* __restrict__ tally) {
  __shared__ uint32_t cnt[kMaxTableParts];
  for (uint64_t g = blockIdx.x; g < n_super; g += gridDim.x) {
    const unsigned long long e = uniform_entry(part_map, g);
    const BatchJob& jb = jobs[e >> 32];
    const uint64_t st = e & 0xffffffffull;
    const RegionFn region(jb);
    const uint32_t P = region.parts;
    const void* pkey = jb.pkey;
    const uint64_t np = jb.np, t0 = st * kSuperTiles;
    const uint64_t t1 = t0 + kSuperTiles < jb.ptiles ? t0 + kSuperTiles : jb.ptiles;
    for (uint32_t j = threadIdx.x; j < P; j += kPartThreads) cnt[j] = 0;   // each thread rereads its own entries below
    lds_barrier();
    // the waves of the workgroup go through the tiles independently, each reading the next tile
    // while it counts the current one (the loads land in kn, always one tile ahead)
    K k[kPartItems], kn[kPartItems];
    load_tile(pkey, np, t0, kn);
    for (uint64_t t = t0; t < t1; ++t) {
#pragma unroll
      for (uint32_t it = 0; it < kPartItems; ++it) k[it] = kn[it];
      if (t + 1 < t1) load_tile(pkey, np, t + 1, kn);
      uint32_t r[kPartItems];
      tile_regions(region, np, t, k, r);
#pragma unroll
      for (uint32_t it = 0; it < kPartItems; ++it)   // keys that cannot match are not counted: on one
        if (r[it] < P) atomicAdd(&cnt[r[it]], 1u);   // shared counter they would serialize the lanes
    }
    lds_barrier();
    for (uint32_t j = threadIdx.x; j < P; j += kPartThreads) tally[jb.cbase + st * P + j] = cnt[j];
  }
}

// One workgroup per partitioned job: its tallies become exclusive positions in region-major
// order (region r's array starts at the position of (super-tile 0, r)), in place, and *kept the
// job's total.  Thread (g, r) of G = kScanBlock / n_parts groups covers region r over an even
// share of the super-tiles.
__global__ void __launch_bounds__(kScanBlock) k_batch_scan(const BatchJob* __restrict__ jobs, uint32_t* __restrict__ tally) {
  __shared__ uint32_t part[kScanBlock];
  const BatchJob& jb = jobs[blockIdx.x];
  if (!jb.n_parts || jb.in_place) return;
  const uint32_t P = jb.n_parts, G = kScanBlock / P;
  const uint32_t g = threadIdx.x / P, r = threadIdx.x % P;
  const bool active = g < G;
  const uint64_t S = jb.stiles;
  const uint64_t s0 = S * g / G, s1 = S * (g + 1) / G;
  uint32_t* c = tally + jb.cbase;
  uint32_t sum = 0;
  if (active) {
    uint64_t st = s0;
    for (; st + 8 <= s1; st += 8) {   // eight independent loads in flight
      uint32_t v[8];
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) v[u] = c[(st + u) * P + r];
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) sum += v[u];
    }
    for (; st < s1; ++st) sum += c[st * P + r];
  }
  part[threadIdx.x] = active ? sum : 0u;
  __syncthreads();
  {   // exclusive scan of the P * G partial sums in region-major order (entry k = rr * G + gg)
    __shared__ uint32_t wtot[kScanBlock / 64];
    const uint32_t k = threadIdx.x, lane = k & 63, wave = k >> 6;
    const uint32_t at = (k % G) * P + k / G;   // k < P * G: where entry k sits in part
    const uint32_t v = k < P * G ? part[at] : 0u;
    uint32_t incl = v;
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    uint32_t base = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < kScanBlock / 64; ++w) {
      base += w < wave ? wtot[w] : 0u;
      total += wtot[w];
    }
    __syncthreads();   // every entry is read before any is overwritten
    if (k < P * G) part[at] = base + incl - v;
    if (k == 0) *jb.kept = total;
  }
  __syncthreads();
  if (active) {
    uint32_t run = part[threadIdx.x];
    uint64_t st = s0;
    for (; st + 8 <= s1; st += 8) {
      uint32_t v[8];
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) v[u] = c[(st + u) * P + r];
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) {
        c[(st + u) * P + r] = run;
        run += v[u];
      }
    }
    for (; st < s1; ++st) {
      const uint32_t v = c[st * P + r];
      c[st * P + r] = run;
      run += v;
    }
  }
}

// Rows r0 .. r0 + T kScatterItems of a job's probe keys, kScatterItems per thread of T (rows past the
// end reread the last row), and their regions (`parts` for a key that cannot match or a row past
// the end).
template <typename K, uint32_t T>
__device__ __forceinline__ void load_rows(const void* pkey, uint64_t np, uint64_t r0, K (&k)[kScatterItems]) {
  const uint32_t last = (uint32_t)(np - r0 < T * kScatterItems ? np - r0 : T * kScatterItems) - 1;
#pragma unroll
  for (uint32_t it = 0; it < kScatterItems; ++it) {
    const uint32_t row = it * T + threadIdx.x;
    k[it] = gload_nt<K>(pkey, r0 + (row < last ? row : last));
  }
}

template <typename K, uint32_t T>
__device__ __forceinline__ void rows_regions(const RegionFn& region, uint64_t np, uint64_t r0, const K (&k)[kScatterItems],
                                             uint32_t (&r)[kScatterItems]) {
  const uint32_t n = (uint32_t)(np - r0 < T * kScatterItems ? np - r0 : T * kScatterItems);
#pragma unroll
  for (uint32_t it = 0; it < kScatterItems; ++it) {
    const uint32_t row = it * T + threadIdx.x;
    r[it] = row < n ? region(k[it]) : region.parts;
  }
}

// Workgroup size of the scatter: one round sorts T kScatterItems keys in LDS (16384 int32 or 8192
// int64 keys), so that a region's run per round is a line or two on the bench's batch.
template <typename K>
constexpr uint32_t scatter_threads() { return sizeof(K) == 4 ? 1024 : 512; }

// Scatter pass: each kept key of super-tile st to its region's array, at the super-tile's
// position for the region plus its rank.  The super-tile goes in rounds of T kScatterItems keys; each
// round is first sorted by region in LDS (the rank of a key among the round's keys of its region
// comes from an LDS counter), then written out in runs, so that neighbouring lanes store
// neighbouring keys; the order within a region is arbitrary and the aggregates do not depend on
// it.  Every thread issues kScatterItems stores per round (slots past the round's kept keys go to
// sink slots past the partitioned keys), and the next round's loads are issued before them, so
// that waiting for those loads never waits for the stores.  A round takes three barriers: after
// the ranks, after the scan (which also advances the positions for the next round and clears
// the counts), and after the sort; a sorted key's region is recomputed from the key when it is
// stored.
template <typename K, uint32_t T>
__global__ void __launch_bounds__(T) k_batch_scatter(const BatchJob* __restrict__ jobs,
                                                     const unsigned long long* __restrict__ part_map,
                                                     uint64_t n_super, const uint32_t* __restrict__ pos) {
  constexpr uint32_t R = T * kScatterItems;
  constexpr uint64_t kSuperRows = (uint64_t)kPartRows * kSuperTiles;
  // per region: next = where the region's next key goes, cnt = the round's keys, off = the
  // round's first sorted slot, delta = next - off (sorted key i of the region goes to delta + i,
  // modulo 2^32)
  __shared__ uint32_t next[kMaxTableParts + 1], cnt[kMaxTableParts + 1], off[kMaxTableParts + 1],
      delta[kMaxTableParts + 1];
  __shared__ K stage[R];
  const uint32_t lane = threadIdx.x & 63;
  for (uint64_t g = blockIdx.x; g < n_super; g += gridDim.x) {
    const unsigned long long e = uniform_entry(part_map, g);
    const BatchJob& jb = jobs[e >> 32];
    const uint64_t st = e & 0xffffffffull;
    const RegionFn region(jb);
    const uint32_t P = region.parts;
    const void* pkey = jb.pkey;
    void* const dst = jb.pbuf;
    // slots past a round's kept keys store to this workgroup's own 64 sink slots, so that no
    // line is written by many workgroups at once
    const uint64_t np = jb.np, s0 = st * kSuperRows, s1 = s0 + kSuperRows < np ? s0 + kSuperRows : np;
    const uint32_t sink = (uint32_t)np + 64u * (blockIdx.x % kSinkGroups) + lane;   // the planner keeps it below 2^32 / key size
    // the previous super-tile's last stores, which may still be going on, read only stage, delta
    // and off[P]
    for (uint32_t j = threadIdx.x; j <= P; j += T) {
      next[j] = j < P ? pos[jb.cbase + st * P + j] : 0u;
      cnt[j] = 0;
    }
    K k[kScatterItems], kn[kScatterItems];
    load_rows<K, T>(pkey, np, s0, kn);
    lds_barrier();
    for (uint64_t r0 = s0; r0 < s1; r0 += R) {
#pragma unroll
      for (uint32_t it = 0; it < kScatterItems; ++it) k[it] = kn[it];
      // per key: region << 16 | rank among the round's keys of its region (no rank for a key that
      // cannot match: see the count).  cnt was cleared by the previous round's scan; the stores
      // of the previous round, which may still be going on in other waves, do not read it.
      uint32_t rr[kScatterItems];
      rows_regions<K, T>(region, np, r0, k, rr);
#pragma unroll
      for (uint32_t it = 0; it < kScatterItems; ++it)
        rr[it] = rr[it] < P ? rr[it] << 16 | atomicAdd(&cnt[rr[it]], 1u) : P << 16;
      lds_barrier();   // the ranks are taken, and every store of the previous round has read its LDS
      if (threadIdx.x < 64) {   // exclusive scan of cnt[0 .. P) into off; off[P] = the round's kept keys
        const uint32_t per = (P + 63) / 64, j0 = per * lane;
        uint32_t own = 0;
        for (uint32_t u = 0; u < per; ++u)
          if (j0 + u < P) own += cnt[j0 + u];
        uint32_t incl = own;
#pragma unroll
        for (uint32_t o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(incl, o, 64);
          if (lane >= o) incl += y;
        }
        uint32_t run = incl - own;
        for (uint32_t u = 0; u < per; ++u)
          if (j0 + u < P) {
            const uint32_t j = j0 + u, c = cnt[j];
            off[j] = run;
            delta[j] = next[j] - run;
            next[j] += c;
            cnt[j] = 0;
            run += c;
          }
        if (lane == 63) off[P] = incl;
      }
      lds_barrier();
#pragma unroll
      for (uint32_t it = 0; it < kScatterItems; ++it) {
        const uint32_t r = rr[it] >> 16;
        if (r < P) stage[off[r] + (rr[it] & 0xffffu)] = k[it];
      }
      if (r0 + R < s1) load_rows<K, T>(pkey, np, r0 + R, kn);
      lds_barrier();
      const uint32_t total = off[P];
#pragma unroll
      for (uint32_t it = 0; it < kScatterItems; ++it) {
        const uint32_t i = it * T + threadIdx.x;
        const K v = stage[i];
        const uint32_t at = i < total ? delta[region(v)] + i : sink;   // a kept key's region is below P
        gstore_at<K>(dst, at * (uint32_t)sizeof(K), v);
      }
    }
  }
}

// Probe of one key against a table region staged in LDS (stage: region p of the job's table;
// hash chains that leave the region continue in device memory).
template <typename K>
__device__ __forceinline__ void probe_staged(const BatchJob& jb, K k, uint32_t p, const uint8_t* stage,
                                             uint32_t slot_shift, unsigned long long& cnt, unsigned long long& sum) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  const U kb = (U)k;
  const unsigned long long ko = key_ord(k);
  if (jb.direct) {
    const uint64_t idx = ko - jb.kmin_ord;
    if (idx < jb.nb) {
      cnt += 1;
      const uint32_t o = (uint32_t)(idx - ((uint64_t)p << jb.part_shift));
      if (jb.pay_size == 4) sum += (unsigned long long)(long long)((const int*)stage)[o];
      else if (jb.pay_size == 8) sum += (unsigned long long)((const long long*)stage)[o];
    }
    return;
  }
  if (ko < jb.kmin_ord || ko > jb.kmax_ord) return;
  if (kb == kEmpty) {
    const unsigned long long c = gload<unsigned long long>(jb.side, 0);
    cnt += c;
    if (c) sum += gload<unsigned long long>(jb.side, 1);
    return;
  }
  const uint64_t base = (uint64_t)p << jb.part_shift, window = 1ull << jb.part_shift;
  uint64_t h = slot_of(key_bits(k), jb.log2cap);
  for (uint64_t step = 0; step <= jb.mask; ++step) {
    const uint64_t off = (h - base) & jb.mask;
    U sk;
    long long v = 0;
    if (off < window) {   // the staged region
      const uint8_t* slot = stage + (off << slot_shift);
      sk = *(const U*)slot;
      if (sk == kb) v = jb.pay_size == 4 ? (long long)*(const int*)(slot + sizeof(K))
                                         : jb.pay_size == 8 ? *(const long long*)(slot + 8) : 0;
    } else {              // a chain that left the region
      const uint8_t* slot = jb.slots + (h << slot_shift);
      sk = gload<U>(slot, 0);
      if (sk == kb) v = jb.pay_size == 4 ? (long long)gload<int>(slot + sizeof(K), 0)
                                         : jb.pay_size == 8 ? gload<long long>(slot + 8, 0) : 0;
    }
    if (sk == kb) {
      cnt += 1;
      sum += (unsigned long long)v;
      return;
    }
    if (sk == kEmpty) return;
    h = (h + 1) & jb.mask;
  }
}

// Region probe (region_map[t] = job << 44 | region << 32 | item, ~0 for none): item `item` of
// region p takes an even share of the region's keys; with its region staged in LDS when the job's
// regions fit kStageBytes.
template <typename K>
__global__ void __launch_bounds__(kRegionThreads) k_batch_region(const BatchJob* __restrict__ jobs,
                                                                 const unsigned long long* __restrict__ region_map,
                                                                 uint64_t n_items, uint32_t slot_shift,
                                                                 const uint32_t* __restrict__ pos,
                                                                 unsigned long long* __restrict__ acc) {
  __shared__ __attribute__((aligned(16))) uint8_t stage[kStageBytes];
  for (uint64_t t = blockIdx.x; t < n_items; t += gridDim.x) {
    const unsigned long long e = uniform_entry(region_map, t);
    if (e == ~0ull) continue;   // uniform over the workgroup
    const uint32_t lo = (uint32_t)(e >> 44) & 0xfffu, p = (uint32_t)(e >> 32) & 0xfffu, item = (uint32_t)e;
    const BatchJob& jb = jobs[lo];
    uint64_t start = 0, end = jb.np;
    const void* keys = jb.pkey;
    if (!jb.in_place) {
      start = pos[jb.cbase + p];
      end = p + 1 < jb.n_parts ? pos[jb.cbase + p + 1] : gload<unsigned long long>(jb.kept, 0);
      keys = jb.pbuf;
    }
    const uint64_t size = end - start, n = jb.items_per_region;
    const uint64_t q0 = start + size * item / n, q1 = start + size * (item + 1) / n;
    unsigned long long cnt = 0, sum = 0;
    if (jb.staged) {
      // region p of the table: direct payloads of keys min + [p 2^s, (p + 1) 2^s), or hash slots
      // [p 2^s, (p + 1) 2^s), cut at the table's end
      const uint64_t entry = jb.direct ? jb.pay_size : (1ull << slot_shift);
      const uint64_t entries = jb.direct ? jb.nb : jb.mask + 1;
      const uint64_t first = (uint64_t)p << jb.part_shift;
      const uint64_t count = (first + (1ull << jb.part_shift) < entries ? (1ull << jb.part_shift) : entries - first);
      const uint8_t* src = (jb.direct ? jb.dpay : jb.slots) + first * entry;
      const uint32_t words = (uint32_t)(count * entry / 4);
      for (uint32_t w = threadIdx.x; w < words; w += blockDim.x) ((uint32_t*)stage)[w] = gload<uint32_t>(src, w);
      __syncthreads();
      for (uint64_t q = q0 + threadIdx.x; q < q1; q += (uint64_t)blockDim.x * kRunUnroll) {
        K k[kRunUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kRunUnroll; ++u)
          k[u] = q + u * blockDim.x < q1 ? gload_nt<K>(keys, q + u * blockDim.x) : K(0);
#pragma unroll
        for (uint32_t u = 0; u < kRunUnroll; ++u)
          if (q + u * blockDim.x < q1) probe_staged<K>(jb, k[u], p, stage, slot_shift, cnt, sum);
      }
    } else {
      for (uint64_t q = q0 + threadIdx.x; q < q1; q += (uint64_t)blockDim.x * kRunUnroll) {
        K k[kRunUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kRunUnroll; ++u)
          k[u] = q + u * blockDim.x < q1 ? gload_nt<K>(keys, q + u * blockDim.x) : K(0);
#pragma unroll
        for (uint32_t u = 0; u < kRunUnroll; ++u)
          if (q + u * blockDim.x < q1) probe_key<K>(jb, k[u], slot_shift, cnt, sum);
      }
    }
    block_add2(cnt, sum, acc + 2 * lo);   // its barriers also keep the next item's staging behind these reads
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

// Presence bytes set in the direct-table jobs' tables, per job, into cnt[j] (tile order).  Count
// tile t belongs to the job whose first count tile is the largest one <= t; each covers
// kCountWords 8-byte words.  A byte is 0 or 1, so a word's popcount is its set bytes.
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
    const uint64_t words = (jb.nb + 7) / 8;   // the bytes past nb up to the 256-byte alignment are 0
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
  extern __shared__ unsigned long long t0[];   // n_jobs first-tile indices
  __shared__ unsigned long long rmin[4], rmax[4];
  for (uint32_t j = threadIdx.x; j < n_jobs; j += blockDim.x) t0[j] = jobs[j].tile0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr uint32_t kVec = 16 / sizeof(K);   // keys per 16-byte load
  for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    uint32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (t0[mid] <= t) lo = mid;
      else hi = mid;
    }
    const MmJob jb = jobs[lo];
    const uint64_t r0 = (t - jb.tile0) * tile_rows, r1 = r0 + tile_rows < jb.n ? r0 + tile_rows : jb.n;
    const K* key = (const K*)jb.key;
    unsigned long long mn = ~0ull, mx = 0;
    uint64_t i0 = r0;
    if (((uintptr_t)(key + r0) & 15) == 0) {
      // 16-byte loads, four in flight per lane; tile_rows is a multiple of 4 * 256 * kVec
      const uint64_t nv = (r1 - r0) / kVec;
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      const u32x4* v = (const u32x4*)(key + r0);
      uint64_t q = threadIdx.x;
      for (; q + 3 * 256 < nv; q += 4 * 256) {
        u32x4 w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = __builtin_nontemporal_load(v + q + u * 256);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const K* e = (const K*)&w[u];
#pragma unroll
          for (uint32_t c = 0; c < kVec; ++c) {
            const unsigned long long o = key_ord(e[c]);
            mn = o < mn ? o : mn;
            mx = o > mx ? o : mx;
          }
        }
      }
      for (; q < nv; q += 256) {
        const u32x4 w = __builtin_nontemporal_load(v + q);
        const K* e = (const K*)&w;
#pragma unroll
        for (uint32_t c = 0; c < kVec; ++c) {
          const unsigned long long o = key_ord(e[c]);
          mn = o < mn ? o : mn;
          mx = o > mx ? o : mx;
        }
      }
      i0 = r0 + nv * kVec;
    }
    for (uint64_t i = i0 + threadIdx.x; i < r1; i += blockDim.x) {
      const unsigned long long o = key_ord(key[i]);
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
  uint64_t direct_bytes = 0;       // presence bytes and payloads of the direct-table jobs (after them)
  uint32_t slot_shift = 3;
  // probe by regions: the region kernel's work items (kXcds interleaved lists, like the tile
  // maps), the partitioning passes' super-tiles (job << 32 | super-tile), and the bytes of the
  // partitioned keys, tallies and kept totals (a block of their own)
  std::vector<unsigned long long> region_map, part_map;
  uint64_t part_bytes = 0;
  uint64_t pkey_bytes = 0, tally_entries = 0;
  uint32_t part_jobs = 0, region_jobs = 0;
};

// Which jobs get a direct table: per caller's job, direct[j] and the smallest key kmin[j]
// (order-preserving unsigned form).
struct DirectInfo {
  std::vector<uint8_t> direct;
  std::vector<unsigned long long> kmin, kmax;
  bool operator==(const DirectInfo& o) const { return direct == o.direct && kmin == o.kmin && kmax == o.kmax; }
};

uint64_t align256(uint64_t v) { return (v + 255) / 256 * 256; }

uint64_t direct_region_bytes(uint64_t nb, uint32_t ps) {
  return align256(nb) + align256(nb * ps);
}

// Min and max build key of every job in one launch; a job is direct when its nb keys could be
// exactly the nb values from its min to its max.  Hash-table jobs use the range to drop probe
// keys that cannot match.
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
  di->kmin.assign(J, ~0ull);   // no build keys: an empty range
  di->kmax.assign(J, 0);
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
  const size_t lds = (size_t)J * sizeof(unsigned long long);
  if (ks == 8)
    hipLaunchKernelGGL(k_batch_minmax<int64_t>, dim3(g), dim3(256), lds, ctx->compute, (const MmJob*)mjd, J, tiles,
                       tile_rows, mm);
  else
    hipLaunchKernelGGL(k_batch_minmax<int32_t>, dim3(g), dim3(256), lds, ctx->compute, (const MmJob*)mjd, J, tiles,
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
    di->kmax[j] = mx;
  }
  return VX_OK;
}

// The XCD-aware maps.  Work on one table stays on one XCD where the table can stay in that XCD's
// L2: a job probed through the tile map whose table fits in 3/4 of an L2 gets all of its tiles
// there, and each table region of a job probed by regions gets all of its work items on one XCD
// (with the job's build tiles, when the whole table fits).  Such units spread over the XCDs
// largest first, balancing entries; the build tiles of larger tables, and all tiles of a larger
// job probed through the tile map, spread over every XCD in turn and come first in every list.
static uint64_t table_bytes_of(const BatchJob& b, uint32_t slot_bytes) {
  return b.direct ? b.nb * (uint64_t)b.pay_size : (b.mask + 1) * (uint64_t)slot_bytes;
}

static void map_tiles(BatchPlan* pl, uint32_t slot_bytes, uint64_t l2_bytes) {
  const uint32_t J = (uint32_t)pl->jobs.size();
  std::vector<std::vector<unsigned long long>> bl(kXcds), pr(kXcds), rl(kXcds);
  struct Unit {
    uint32_t job, region;   // region ~0: a whole job through the tile map
    uint64_t entries;
  };
  std::vector<Unit> units, regions;
  uint32_t rb = 0, rp = 0;
  for (uint32_t i = 0; i < J; ++i) {
    const BatchJob& b = pl->jobs[i];
    const bool local = table_bytes_of(b, slot_bytes) <= l2_bytes / 4 * 3;
    if (b.n_parts) {
      for (uint32_t p = 0; p < b.n_parts; ++p) regions.push_back({i, p, b.items_per_region});
      if (!local)
        for (uint32_t k = 0; k < b.build_tiles; ++k) bl[rb++ % kXcds].push_back(((unsigned long long)i << 32) | k);
      continue;
    }
    if (local) {
      units.push_back({i, ~0u, b.probe_tiles});
      continue;
    }
    for (uint32_t k = 0; k < b.build_tiles; ++k) bl[rb++ % kXcds].push_back(((unsigned long long)i << 32) | k);
    for (uint32_t k = 0; k < b.probe_tiles; ++k) pr[rp++ % kXcds].push_back(((unsigned long long)i << 32) | k);
  }
  auto by_size = [](const Unit& a, const Unit& b) { return a.entries > b.entries; };
  auto least = [](const std::vector<std::vector<unsigned long long>>& l) {
    uint32_t x = 0;
    for (uint32_t y = 1; y < kXcds; ++y)
      if (l[y].size() < l[x].size()) x = y;
    return x;
  };
  std::stable_sort(units.begin(), units.end(), by_size);
  for (const Unit& u : units) {
    const uint32_t x = least(pr);
    const BatchJob& b = pl->jobs[u.job];
    for (uint32_t k = 0; k < b.build_tiles; ++k) bl[x].push_back(((unsigned long long)u.job << 32) | k);
    for (uint32_t k = 0; k < b.probe_tiles; ++k) pr[x].push_back(((unsigned long long)u.job << 32) | k);
  }
  std::stable_sort(regions.begin(), regions.end(), by_size);
  for (const Unit& u : regions) {
    const uint32_t x = least(rl);
    const BatchJob& b = pl->jobs[u.job];
    if (u.region == 0 && table_bytes_of(b, slot_bytes) <= l2_bytes / 4 * 3)
      for (uint32_t k = 0; k < b.build_tiles; ++k) bl[x].push_back(((unsigned long long)u.job << 32) | k);
    for (uint64_t k = 0; k < u.entries; ++k)
      rl[x].push_back(((unsigned long long)u.job << 44) | ((unsigned long long)u.region << 32) | k);
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
  flatten(rl, &pl->region_map);
}

// Which jobs are probed by regions, and how.  A table of at most `stage` bytes is one region probed
// from the job's own keys.  A larger one is cut into regions of `stage` bytes (at most
// kMaxTableParts; beyond that the regions grow and are read from device memory) and its probe
// side partitioned, largest probe sides first while the buffers fit part_budget bytes; a job left
// over, or one whose partitioned keys would pass 4 GiB, goes through the tile map.  Offsets in the jobs are
// relative to the partition block until setup_run relocates them.
static void plan_regions(BatchPlan* pl, int ks, uint32_t slot_bytes, uint64_t part_budget, uint64_t stage) {
  pl->part_map.clear();
  pl->part_bytes = pl->pkey_bytes = pl->tally_entries = 0;
  pl->part_jobs = pl->region_jobs = 0;
  const uint32_t J = (uint32_t)pl->jobs.size();
  const uint64_t item_keys = 1 << 20;   // probe keys per work item (its region is staged once per item)
  for (uint32_t i = 0; i < J; ++i) {
    BatchJob& b = pl->jobs[i];
    const uint64_t table = table_bytes_of(b, slot_bytes);
    if (table <= stage) {
      b.n_parts = 1;
      b.in_place = 1;
      b.staged = 1;
      uint32_t sh = 0;
      if (b.direct)
        while ((1ull << sh) < b.nb) ++sh;
      else
        sh = b.log2cap;
      b.part_shift = sh;
      b.items_per_region = (uint32_t)std::max<uint64_t>(1, (b.np + item_keys - 1) / item_keys);
      ++pl->region_jobs;
      continue;
    }
    // the scatter addresses a job's partitioned keys (and sink slots) by 32-bit byte offsets
    if (b.np == 0 || (b.np + 64ull * kSinkGroups) * (uint64_t)ks >= (1ull << 32)) continue;
    uint32_t parts, shift;
    bool staged;
    if (b.direct) {
      shift = 0;
      while ((2ull << shift) * b.pay_size <= stage) ++shift;
      while (((b.nb - 1) >> shift) + 1 > kMaxTableParts) ++shift;
      parts = (uint32_t)(((b.nb - 1) >> shift) + 1);
      staged = (1ull << shift) * b.pay_size <= stage;
    } else {
      uint32_t bits = 0;
      const uint32_t max_bits = 10;   // kMaxTableParts regions
      while ((table >> bits) > stage && bits < max_bits && bits < b.log2cap) ++bits;
      parts = 1u << bits;
      shift = b.log2cap - bits;
      staged = (table >> bits) <= stage;
    }
    const uint64_t ptiles = (b.np + kPartRows - 1) / kPartRows;
    const uint64_t stiles = (ptiles + kSuperTiles - 1) / kSuperTiles;
    const uint64_t keys = align256((b.np + 64ull * kSinkGroups) * (uint64_t)ks), tallies = stiles * parts;   // + the sink slots
    const uint64_t need = keys + tallies * 4 + 256 + 8;
    if (pl->part_bytes + need > part_budget) continue;
    b.n_parts = parts;
    b.part_shift = shift;
    b.staged = staged;
    b.ptiles = (uint32_t)ptiles;
    b.stiles = (uint32_t)stiles;
    b.items_per_region = (uint32_t)std::max<uint64_t>(1, (b.np / parts + item_keys - 1) / item_keys);
    b.pbuf = (uint8_t*)(uintptr_t)pl->pkey_bytes;
    b.cbase = pl->tally_entries;
    b.kept = (unsigned long long*)(uintptr_t)(8ull * pl->part_jobs);   // index into the kept totals
    pl->pkey_bytes += keys;
    pl->tally_entries += tallies;
    pl->part_bytes += need;
    ++pl->part_jobs;
    ++pl->region_jobs;
    for (uint64_t t = 0; t < stiles; ++t) pl->part_map.push_back(((unsigned long long)i << 32) | t);
  }
  pl->part_bytes = pl->pkey_bytes + align256(pl->tally_entries * 4) + align256(8ull * pl->part_jobs);
}

static vx_status plan_batch(const vx_batch_join* d, const BatchConfig& cfg, int ks, uint32_t ps,
                            const DirectInfo& di, uint64_t l2_bytes, bool regions, uint64_t part_budget,
                            uint64_t stage, BatchPlan* pl) {
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
    b.kmin_ord = di.kmin[j];
    b.kmax_ord = di.kmax[j];
    if (di.direct[j]) {
      // offsets are relocated once memory is carved: direct regions follow the hash slots
      b.direct = 1;
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
    b.count_tiles = b.direct ? (uint32_t)(((b.nb + 7) / 8 + kCountWords - 1) / kCountWords) : 0;
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
  if (regions) plan_regions(pl, ks, slot_bytes, part_budget, stage);
  map_tiles(pl, slot_bytes, l2_bytes);
  return VX_OK;
}

struct BatchRun {
  ArenaBlock mem;              // slots, side records, descriptors, counters, accumulators
  BatchPlan plan;
  BatchJob* jobs_dev = nullptr;
  unsigned long long* counters = nullptr;   // sides, accumulators, bit counts (cleared together)
  unsigned long long* acc = nullptr;         // per job (tile order): count, sum
  unsigned long long* bits = nullptr;        // per job (tile order): presence bytes set in its direct table
  unsigned long long* probe_map = nullptr;   // the plan's tile maps, in device memory
  unsigned long long* build_map = nullptr;
  unsigned long long* region_map = nullptr;  // the region probe's work items
  unsigned long long* part_map = nullptr;    // the partitioning passes' super-tiles
  uint32_t* tally = nullptr;                 // per partitioned job and super-tile: keys per region, then positions
  uint8_t* slots = nullptr;
  uint64_t counter_words = 0;
};

// Probe by regions unless VX_BATCH_REGIONS=0; VX_BATCH_STAGE_KB (at most 64) lowers the size of a
// region staged in LDS, so that small inputs exercise every path.
static bool regions_enabled() {
  const char* e = getenv("VX_BATCH_REGIONS");
  return !(e && e[0] == '0');
}

static uint64_t stage_bytes() {
  const char* e = getenv("VX_BATCH_STAGE_KB");
  const uint64_t v = e ? strtoull(e, nullptr, 10) << 10 : kStageBytes;
  return std::max<uint64_t>(256, std::min<uint64_t>(v, kStageBytes));
}

// Device bytes of a run's one arena block: tables, descriptors, counters, maps, then the
// partition block.
static uint64_t run_bytes(const BatchPlan& pl, uint32_t J, uint64_t counter_words) {
  return align256(pl.slots << pl.slot_shift) + align256(pl.direct_bytes) + align256((uint64_t)J * sizeof(BatchJob)) +
         align256(counter_words * 8) + align256(pl.probe_map.size() * 8) + align256(pl.build_map.size() * 8) +
         align256(pl.region_map.size() * 8) + align256(pl.part_map.size() * 8) + pl.part_bytes;
}

static vx_status setup_run(vx_ctx* ctx, const vx_batch_join* d, const BatchConfig& cfg, int ks,
                           uint32_t ps, const DirectInfo& di, BatchRun* r, bool regions = true) {
  const uint32_t J = d->n_jobs;
  // side records and accumulators are contiguous so one fill kernel clears them
  r->counter_words = 2 * (uint64_t)J + 2 * (uint64_t)J + (uint64_t)J;
  regions = regions && regions_enabled();
  const uint64_t stage = stage_bytes();
  VX_TRY(plan_batch(d, cfg, ks, ps, di, ctx->l2_bytes, regions, 0, stage, &r->plan));
  const uint64_t base = run_bytes(r->plan, J, r->counter_words), room = ctx->arena.largest_free();
  const char* part_env = getenv("VX_BATCH_PARTITION");   // 0: no probe side is partitioned
  if (regions && !(part_env && part_env[0] == '0') && room > base + (64ull << 20)) {
    // a plan that partitions large probe sides; the margin covers its maps
    BatchPlan pp;
    VX_TRY(plan_batch(d, cfg, ks, ps, di, ctx->l2_bytes, true, room - base - (64ull << 20), stage, &pp));
    if (pp.part_jobs && run_bytes(pp, J, r->counter_words) <= room) r->plan = std::move(pp);
  }
  const BatchPlan& pl = r->plan;
  const uint64_t hash_bytes = align256(pl.slots << pl.slot_shift);
  const uint64_t slot_bytes = hash_bytes + align256(pl.direct_bytes);
  const uint64_t desc_bytes = (uint64_t)J * sizeof(BatchJob);
  const uint64_t map_bytes = pl.probe_map.size() * 8, bmap_bytes = pl.build_map.size() * 8;
  const uint64_t rmap_bytes = pl.region_map.size() * 8, pmap_bytes = pl.part_map.size() * 8;
  const uint64_t bytes = run_bytes(pl, J, r->counter_words);
  r->mem.a = &ctx->arena;
  r->mem.p = ctx->arena.alloc(bytes);
  VX_CHECK(r->mem.p, VX_EBUDGET, "batch: %llu bytes of tables and descriptors do not fit the arena",
           (unsigned long long)bytes);
  r->slots = r->mem.p;
  uint8_t* q = r->mem.p + slot_bytes;
  r->jobs_dev = (BatchJob*)q;
  q += align256(desc_bytes);
  r->counters = (unsigned long long*)q;
  unsigned long long* sides = r->counters;
  r->acc = sides + 2 * (uint64_t)J;
  r->bits = r->acc + 2 * (uint64_t)J;
  q += align256(r->counter_words * 8);
  r->probe_map = (unsigned long long*)q;
  q += align256(map_bytes);
  r->build_map = (unsigned long long*)q;
  q += align256(bmap_bytes);
  r->region_map = (unsigned long long*)q;
  q += align256(rmap_bytes);
  r->part_map = (unsigned long long*)q;
  q += align256(pmap_bytes);
  uint8_t* part_block = q;
  r->tally = (uint32_t*)(part_block + pl.pkey_bytes);
  for (uint32_t j = 0; j < J; ++j) {
    BatchJob& b = r->plan.jobs[j];
    if (b.direct) {
      b.slots = r->slots + hash_bytes + (uint64_t)(uintptr_t)b.slots;
      b.dpay = b.slots + align256(b.nb);
    } else {
      b.slots = r->slots + (((uint64_t)(uintptr_t)b.slots) << pl.slot_shift);
    }
    b.side = sides + 2 * (uint64_t)j;
    if (b.n_parts && !b.in_place) {
      b.pbuf = part_block + (uint64_t)(uintptr_t)b.pbuf;
      b.kept = (unsigned long long*)(part_block + pl.pkey_bytes + align256(pl.tally_entries * 4) +
                                     (uint64_t)(uintptr_t)b.kept);
    }
  }
  VX_HIP(hipMemcpyAsync(r->jobs_dev, pl.jobs.data(), desc_bytes, hipMemcpyHostToDevice, ctx->compute));
  if (map_bytes)
    VX_HIP(hipMemcpyAsync(r->probe_map, pl.probe_map.data(), map_bytes, hipMemcpyHostToDevice, ctx->compute));
  if (bmap_bytes)
    VX_HIP(hipMemcpyAsync(r->build_map, pl.build_map.data(), bmap_bytes, hipMemcpyHostToDevice, ctx->compute));
  if (rmap_bytes)
    VX_HIP(hipMemcpyAsync(r->region_map, pl.region_map.data(), rmap_bytes, hipMemcpyHostToDevice, ctx->compute));
  if (pmap_bytes)
    VX_HIP(hipMemcpyAsync(r->part_map, pl.part_map.data(), pmap_bytes, hipMemcpyHostToDevice, ctx->compute));
  return VX_OK;
}

static void launch_dupcount(vx_ctx* ctx, const BatchRun& r, uint32_t J, hipStream_t s) {
  if (!r.plan.count_tiles) return;
  const unsigned g = (unsigned)std::min<uint64_t>(r.plan.count_tiles, (uint64_t)ctx->cu_count * 4);
  hipLaunchKernelGGL(k_batch_dupcount, dim3(g), dim3(256), 0, s, r.jobs_dev, J, r.plan.count_tiles, r.bits);
}

// A direct-table job with fewer than nb presence bytes set had a repeated build key.
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
  // Streams: the copy stream takes the partitioning (count, scan, scatter) beside the build
  // phase, then, once the tables are built, the region probe beside the tile-map probe.
  const char* fork_env = getenv("VX_BATCH_FORK");   // 0: everything on one stream, in order
  hipStream_t s2 = fork_env && fork_env[0] == '0' ? s : ctx->copy;
  const bool part = !r.plan.part_map.empty(), reg = !r.plan.region_map.empty();
  hipEvent_t ev_built = nullptr, ev_done = nullptr;
  if (reg) {
    hipEvent_t fork = get_event(ctx);
    ev_built = get_event(ctx);
    ev_done = get_event(ctx);
    VX_CHECK(fork && ev_built && ev_done, VX_EHIP, "batch: no events");
    VX_HIP(hipEventRecord(fork, s));
    VX_HIP(hipStreamWaitEvent(s2, fork, 0));
    put_event(ctx, fork);
  }
  if (part) {
    const uint64_t ns = r.plan.part_map.size();
    const unsigned g = (unsigned)std::min<uint64_t>(ns, (uint64_t)ctx->cu_count * 8);
    const unsigned gs = (unsigned)std::min<uint64_t>(ns, (uint64_t)ctx->cu_count);   // one scatter workgroup per CU (its LDS)
    if (ks == 8)
      hipLaunchKernelGGL(k_batch_count<int64_t>, dim3(g), dim3(kPartThreads), 0, s2, r.jobs_dev, r.part_map, ns, r.tally);
    else
      hipLaunchKernelGGL(k_batch_count<int32_t>, dim3(g), dim3(kPartThreads), 0, s2, r.jobs_dev, r.part_map, ns, r.tally);
    hipLaunchKernelGGL(k_batch_scan, dim3(J), dim3(kScanBlock), 0, s2, r.jobs_dev, r.tally);
    // the build phase starts after the count, which reads at the memory's rate: beside the
    // scatter, which does not, the two slow each other less
    if (s2 != s) {
      hipEvent_t counted = get_event(ctx);
      VX_CHECK(counted, VX_EHIP, "batch: no events");
      VX_HIP(hipEventRecord(counted, s2));
      VX_HIP(hipStreamWaitEvent(s, counted, 0));
      put_event(ctx, counted);
    }
    if (ks == 8)
      hipLaunchKernelGGL((k_batch_scatter<int64_t, scatter_threads<int64_t>()>), dim3(gs), dim3(scatter_threads<int64_t>()), 0, s2, r.jobs_dev, r.part_map, ns,
                         (const uint32_t*)r.tally);
    else
      hipLaunchKernelGGL((k_batch_scatter<int32_t, scatter_threads<int32_t>()>), dim3(gs), dim3(scatter_threads<int32_t>()), 0, s2, r.jobs_dev, r.part_map, ns,
                         (const uint32_t*)r.tally);
    VX_HIP(hipGetLastError());
  }
  const unsigned long long* bmap = r.build_map;
  if (ks == 8)
    hipLaunchKernelGGL((k_batch_phase<int64_t, true>), dim3(gb), dim3(cfg.block), 0, s, r.jobs_dev, J,
                       (uint64_t)bmapped, cfg.tile_rows, r.plan.slot_shift, r.acc, ctx->dev_flags, bmap);
  else
    hipLaunchKernelGGL((k_batch_phase<int32_t, true>), dim3(gb), dim3(cfg.block), 0, s, r.jobs_dev, J,
                       (uint64_t)bmapped, cfg.tile_rows, r.plan.slot_shift, r.acc, ctx->dev_flags, bmap);
  launch_dupcount(ctx, r, J, s);
  if (reg) {
    VX_HIP(hipEventRecord(ev_built, s));
    VX_HIP(hipStreamWaitEvent(s2, ev_built, 0));
    put_event(ctx, ev_built);
    const uint64_t items = r.plan.region_map.size();
    unsigned g = (unsigned)std::min<uint64_t>(items, (uint64_t)ctx->cu_count * (kLdsBytes / kStageBytes));   // stages per CU
    g = std::max(kXcds, g / kXcds * kXcds);
    if (ks == 8)
      hipLaunchKernelGGL(k_batch_region<int64_t>, dim3(g), dim3(kRegionThreads), 0, s2, r.jobs_dev, r.region_map, items,
                         r.plan.slot_shift, (const uint32_t*)r.tally, r.acc);
    else
      hipLaunchKernelGGL(k_batch_region<int32_t>, dim3(g), dim3(kRegionThreads), 0, s2, r.jobs_dev, r.region_map, items,
                         r.plan.slot_shift, (const uint32_t*)r.tally, r.acc);
    VX_HIP(hipGetLastError());
    VX_HIP(hipEventRecord(ev_done, s2));
  }
  const unsigned long long* pmap = r.probe_map;
  if (mapped) {
    if (ks == 8)
      hipLaunchKernelGGL((k_batch_phase<int64_t, false>), dim3(gp), dim3(cfg.block), 0, s, r.jobs_dev, J,
                         (uint64_t)mapped, cfg.tile_rows, r.plan.slot_shift, r.acc, ctx->dev_flags, pmap);
    else
      hipLaunchKernelGGL((k_batch_phase<int32_t, false>), dim3(gp), dim3(cfg.block), 0, s, r.jobs_dev, J,
                         (uint64_t)mapped, cfg.tile_rows, r.plan.slot_shift, r.acc, ctx->dev_flags, pmap);
  }
  if (reg) {
    VX_HIP(hipStreamWaitEvent(s, ev_done, 0));
    put_event(ctx, ev_done);
  }
  VX_HIP(hipGetLastError());
  if (host_out) {   // accumulators and presence counts are contiguous: 3 J words, then the flags
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
  VX_TRY(find_direct(ctx, d, ks, &di));
  if (d->flags & VX_HASHED) di.direct.assign(J, 0);   // every job hashed; the ranges still filter probes
  const double t_checked = now_ms();
  if (d->mode == 0) {   // a graph kept for other jobs gives its arena memory back before tuning
    auto it = g_graphs.find(ctx);
    if (it != g_graphs.end() && it->second && !(it->second->key == job_keys(d) && it->second->di == di)) {
      drop_graph(it->second);
      it->second = nullptr;
    }
  }
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
    // build phase, presence count, tile-map probe, count, scan, scatter, region probe
    const BatchPlan& gp = gc->run->plan;
    s.kernel_launches = 1 + (gp.count_tiles ? 1 : 0) + (gp.probe_map.empty() ? 0 : 1) + (gp.part_jobs ? 3 : 0) +
                        (gp.region_map.empty() ? 0 : 1);
    s.n_parts = gp.part_jobs;
    s.survivors = gp.region_jobs;
    s.table_bytes = (gc->run->plan.slots << gc->run->plan.slot_shift) + gc->run->plan.direct_bytes;
    s.chunk_rows = cfg.tile_rows;
    s.n_buffers = cfg.block;
    s.imbalance = cfg.load_factor;
  } else {
    BatchRun r;
    VX_TRY(setup_run(ctx, d, cfg, ks, ps, di, &r, false));   // the baseline reads every job's own keys
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
