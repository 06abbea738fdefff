// Partitioned join for a build side whose table would not fit the device budget.
//
// Pass 1 (the paper's radix-partition step, Sec. 6.2.1): the build side streams through the
// chunk pipeline and each chunk is clustered by partition on the GPU (stable multisplit), with
// its boundary array.  The clustered copy lives in the arena when the range splitters' sample
// predicts that pass 2 fits beside it, otherwise in pinned host memory, written by a kernel that
// stores to mapped memory beside the host-to-device copies.
// Pass 2 (Sec. 6.2.2): each partition's segments of every clustered chunk are located through
// the boundary arrays and read in place; they are pre-aggregated (key -> count, payload sum)
// into a transient table, which is then compacted into a table sized by the partition's
// distinct keys.  The probe side streams once: every key goes to its partition's table.
//
// With range partitioning (learned or sample-quantile splitters) a key that carries several
// quantiles gets a partition of its own.  A singleton partition needs no table: pass 1 counts
// its build rows and sums their payload, the probe stream counts its probe rows, and its
// contribution is count_b * count_p pairs and sum_b * count_p.
//
// The two-table radix join (join_radix, the paper's hash-join case study) uses the same pass 1
// on both tables, by raw key bits or a key hash.  Its pass 2 takes the partitions in turn:
// A's rows of a partition are pre-aggregated into one table (in slices when they exceed it),
// and B's rows of the partition, read in place through their segment list, look it up.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "vx_cdf.h"
#include "vx_device.h"
#include "vx_part.h"
#include "vx_pipeline.h"

namespace vx {

vx_status make_spec(vx_ctx* ctx, const vx_part_opts& o, uint32_t n_parts, const int64_t* host_split,
                    uint32_t n_split, ArenaBlock& split_mem, PartSpec* ps);

constexpr uint32_t kMaxSegs = 1024;

struct SegList {
  const unsigned long long* start;    // first source row of each segment
  const unsigned long long* prefix;   // flattened start of each segment; prefix[nseg] = all rows
  uint32_t nseg;
  uint64_t total;                     // rows taken: flattened indices [base, base + total)
  uint64_t base = 0;
};

// Segment holding flattened index idx: the last segment whose prefix is <= idx.
__device__ __forceinline__ uint32_t seg_find(const unsigned long long* pre, uint32_t nseg, uint64_t idx) {
  uint32_t lo = 0, hi = nseg;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= idx) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The same, searching forward from segment s, which starts at or before idx.  A workgroup
// looks up its tile's first row once; segments span thousands of rows, so a later row of the
// tile is in the same segment or one of the next few.
__device__ __forceinline__ uint32_t seg_advance(const unsigned long long* pre, uint32_t nseg, uint32_t s,
                                                uint64_t idx) {
  while (s + 1 < nseg && pre[s + 1] <= idx) ++s;
  return s;
}

constexpr uint32_t kSideWords = 8;   // per-partition side record: count, payload sum (padded)
constexpr uint32_t kSlotShift = 5;   // 32-byte slots: key, count, payload sum, padding

// Empty every slot of a pre-aggregating table; zero a side record if one is given.
__global__ void k_pj_init(uint32_t* slots, uint64_t capacity, uint32_t key_size, unsigned long long* side) {
  const uint32_t words = 1u << (kSlotShift - 2);
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < capacity;
       s += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t* w = slots + s * words;
    for (uint32_t i = 0; i < words; ++i) w[i] = 0;
    if (key_size == 4) w[0] = 0x80000000u;
    else w[1] = 0x80000000u;
  }
  if (side && blockIdx.x == 0 && threadIdx.x < kSideWords) side[threadIdx.x] = 0;
}

// Add (cnt, sum) to key k's record; returns the slot index when this call claimed a new slot,
// else ~0.
template <typename K>
__device__ __forceinline__ uint64_t preagg_claim_add(const TableView& t, K k, unsigned long long cnt,
                                                     unsigned long long sum, unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  const U kb = (U)k;
  if (kb == kEmpty) {
    atomicAdd(t.side, cnt);
    if (t.n_pay) atomicAdd(t.side + 1, sum);
    return ~0ull;
  }
  uint64_t h = slot_of(key_bits(k), t.log2cap);
  for (uint64_t step = 0; step <= t.mask; ++step) {
    uint8_t* slot = t.slots + (h << kSlotShift);
    U prev = atomicCAS((U*)slot, kEmpty, kb);
    if (prev == kEmpty || prev == kb) {
      unsigned long long* w = (unsigned long long*)(slot + 8);
      atomicAdd(w, cnt);
      if (t.n_pay) atomicAdd(w + 1, sum);
      return prev == kEmpty ? h : ~0ull;
    }
    h = (h + 1) & t.mask;
  }
  atomicOr(flags, kFlagFull);
  return ~0ull;
}

// Appends the slots claimed by the active lanes to the workgroup's LDS claim buffer: one LDS
// atomic per wave.
__device__ __forceinline__ void append_claims(uint64_t slot, uint32_t* lbuf, uint32_t* lcount) {
  const bool c = slot != ~0ull;
  const unsigned long long m = __ballot(c);
  if (!m) return;
  const unsigned long long active = __ballot(true);
  const uint32_t lane = threadIdx.x & 63, leader = (uint32_t)__ffsll((long long)active) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(lcount, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  if (c) lbuf[base + (uint32_t)__popcll(m & ((1ull << lane) - 1))] = (uint32_t)slot;
}

constexpr int kPjLds = 1024;
constexpr int kPjTile = 4096;
constexpr int kPjLdsProbes = 16;  // past this, a row goes straight to the global table

// Pre-aggregate one partition's build segments (read in place: device memory or mapped host
// memory) into the transient table: a per-tile LDS table absorbs repeated keys, its entries are
// then added to the global table.  Every slot claimed in the global table is appended to
// `claims` (*n_claims counts them: the partition's distinct keys), a tile at a time through an
// LDS buffer, so the shared counter sees one atomic per tile; claims may be null (no list).
template <typename K>
__global__ void __launch_bounds__(256) k_pj_build(TableView t, const void* key, const void* pay0,
                                                  uint32_t pay_size, SegList sl, unsigned int* flags,
                                                  uint32_t* claims, unsigned long long* n_claims) {
  __shared__ unsigned long long sst[kMaxSegs], spre[kMaxSegs + 1];
  __shared__ unsigned long long lkey[kPjLds], lcnt[kPjLds], lsum[kPjLds];
  __shared__ uint32_t lclaim[kPjTile + kPjLds];   // a tile claims at most one slot per row + per entry
  __shared__ uint32_t n_lclaim;
  __shared__ unsigned long long claim_base;
  const unsigned long long kFree = ~0ull;
  for (uint32_t j = threadIdx.x; j < sl.nseg; j += blockDim.x) sst[j] = sl.start[j];
  for (uint32_t j = threadIdx.x; j <= sl.nseg; j += blockDim.x) spre[j] = sl.prefix[j];
  __syncthreads();
  for (uint64_t base = (uint64_t)blockIdx.x * kPjTile; base < sl.total;
       base += (uint64_t)gridDim.x * kPjTile) {
    for (int j = threadIdx.x; j < kPjLds; j += blockDim.x) {
      lkey[j] = kFree;
      lcnt[j] = 0;
      lsum[j] = 0;
    }
    if (threadIdx.x == 0) n_lclaim = 0;
    __syncthreads();
    uint64_t end = base + kPjTile < sl.total ? base + kPjTile : sl.total;
    uint32_t sg = seg_find(spre, sl.nseg, sl.base + base);
    for (uint64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
      sg = seg_advance(spre, sl.nseg, sg, sl.base + i);
      uint64_t src = sst[sg] + (sl.base + i - spre[sg]);
      K k = load_key<K>(key, src);
      unsigned long long v = t.n_pay ? (unsigned long long)load_signed(pay0, src, pay_size) : 0ull;
      unsigned long long kb = (unsigned long long)(long long)k;
      bool placed = false;
      if (kb != kFree) {
        uint32_t h = (uint32_t)slot_of(kb, 10);
        for (int s = 0; s < kPjLdsProbes; ++s) {
          uint32_t j = (h + s) & (kPjLds - 1);
          unsigned long long prev = atomicCAS(&lkey[j], kFree, kb);
          if (prev == kFree || prev == kb) {
            atomicAdd(&lcnt[j], 1ull);
            atomicAdd(&lsum[j], v);
            placed = true;
            break;
          }
        }
      }
      append_claims(placed ? ~0ull : preagg_claim_add<K>(t, k, 1ull, v, flags), lclaim, &n_lclaim);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kPjLds; j += blockDim.x)
      append_claims(lkey[j] != kFree ? preagg_claim_add<K>(t, (K)(long long)lkey[j], lcnt[j], lsum[j], flags)
                                     : ~0ull,
                    lclaim, &n_lclaim);
    __syncthreads();
    if (claims) {   // uniform across the workgroup
      if (threadIdx.x == 0) claim_base = n_lclaim ? atomicAdd(n_claims, (unsigned long long)n_lclaim) : 0ull;
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < n_lclaim; j += blockDim.x) claims[claim_base + j] = lclaim[j];
    }
    __syncthreads();
  }
}

// Move every claimed record of the transient table into the partition's compact table (sized
// from its distinct-key count) and empty the transient slot, so the next partition finds it
// clean.
template <typename K>
__global__ void k_pj_compact(uint8_t* tslots, const uint32_t* claims, uint64_t n_claims, TableView c) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n_claims;
       q += (uint64_t)gridDim.x * blockDim.x) {
    uint8_t* src = tslots + ((uint64_t)claims[q] << kSlotShift);
    U k = *(U*)src;
    unsigned long long* w = (unsigned long long*)(src + 8);
    unsigned long long cnt = w[0], sum = w[1];
    *(U*)src = kEmpty;
    w[0] = 0;
    w[1] = 0;
    uint64_t h = slot_of(key_bits((K)k), c.log2cap);
    for (uint64_t step = 0; step <= c.mask; ++step) {
      uint8_t* d = c.slots + (h << kSlotShift);
      if (atomicCAS((U*)d, kEmpty, k) == kEmpty) {
        unsigned long long* dw = (unsigned long long*)(d + 8);
        dw[0] = cnt;
        dw[1] = sum;
        break;
      }
      h = (h + 1) & c.mask;
    }
  }
}

// Streamed probe side: route every key to its partition (the function that clustered the build
// side), count the partition's probe rows (first pass only), and look the key up in the
// partition's compact table when that table is resident in this pass.  Per-partition
// (probe rows, matched build rows, SUM of matched build payloads) accumulate in LDS and are
// added to this block's own row of acc (no atomics: the chunks' kernels run in stream order).
template <typename K>
__global__ void __launch_bounds__(256) k_pj_stream(const void* keys, uint64_t n, PartSpec ps,
                                                   const unsigned long long* tab_slots,
                                                   const uint32_t* tab_log2, const unsigned long long* side,
                                                   uint32_t count_rows, unsigned long long* acc) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  extern __shared__ unsigned long long lds[];
  const uint32_t P = ps.n_parts;
  unsigned long long* lacc = lds;                          // 3 * P
  unsigned long long* lslots = lacc + 3 * P;               // P
  long long* lsplit = (long long*)(lslots + P);            // n_split
  uint32_t* llog2 = (uint32_t*)(lsplit + ps.n_split);      // P
  for (uint32_t j = threadIdx.x; j < 3 * P; j += blockDim.x) lacc[j] = 0;
  for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) {
    lslots[j] = tab_slots[j];
    llog2[j] = tab_log2[j];
  }
  if (ps.fn == kPartRange)
    for (uint32_t j = threadIdx.x; j < ps.n_split; j += blockDim.x) lsplit[j] = ps.splitters[j];
  __syncthreads();
  constexpr int ITEMS = 4;
  const uint64_t tile = (uint64_t)blockDim.x * ITEMS;
  for (uint64_t base = blockIdx.x * tile; base < n; base += (uint64_t)gridDim.x * tile) {
    K kk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      kk[j] = i < n ? ((const K*)keys)[i] : (K)0;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      if (i >= n) continue;
      const uint32_t pid = part_of(ps, (long long)kk[j], lsplit);
      if (count_rows) atomicAdd(&lacc[3 * pid], 1ull);
      const unsigned long long sl = lslots[pid];
      if (!sl) continue;
      const unsigned long long* w;
      if ((U)kk[j] == kEmpty) {
        w = side + (uint64_t)pid * kSideWords;
      } else {
        TableView t{};
        t.slots = (uint8_t*)sl;
        t.log2cap = llog2[pid];
        t.mask = (1ull << t.log2cap) - 1;
        t.slot_shift = kSlotShift;
        const uint8_t* s = find_slot_hashed<K>(t, kk[j]);
        if (!s) continue;
        w = (const unsigned long long*)(s + 8);
      }
      if (w[0]) {
        atomicAdd(&lacc[3 * pid + 1], w[0]);
        atomicAdd(&lacc[3 * pid + 2], w[1]);
      }
    }
  }
  __syncthreads();
  unsigned long long* mine = acc + (uint64_t)blockIdx.x * 3 * P;
  for (uint32_t j = threadIdx.x; j < 3 * P; j += blockDim.x)
    if (lacc[j]) mine[j] += lacc[j];
}

// out[j] = SUM over blocks of acc[b][j]
__global__ void k_pj_reduce(const unsigned long long* acc, uint32_t blocks, uint32_t width,
                            unsigned long long* out) {
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < width; j += gridDim.x * blockDim.x) {
    unsigned long long s = 0;
    for (uint32_t b = 0; b < blocks; ++b) s += acc[(uint64_t)b * width + j];
    out[j] = s;
  }
}

// Copy one clustered chunk from its device staging to its rows of the pinned host copy with
// vector stores.  Kernel stores to host memory run beside the host-to-device copy engine,
// where a device-to-host copy would share it.  Rows of singleton partitions (skip[p] >= 0)
// are never read again and are left out.
__global__ void __launch_bounds__(256) k_pj_writeback(const uint8_t* skey, const uint8_t* spay, uint32_t ks,
                                                      uint32_t psz, uint32_t n_pay, uint64_t rows,
                                                      const unsigned long long* bnd, uint32_t P,
                                                      const int* skip, uint8_t* hkey, uint8_t* hpay) {
  __shared__ unsigned long long sb[kMaxParts + 1];
  __shared__ int sk[kMaxParts];
  if (skip) {
    for (uint32_t j = threadIdx.x; j <= P; j += blockDim.x) sb[j] = bnd[j];
    for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) sk[j] = skip[j];
  }
  __syncthreads();
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < rows;
       r += (uint64_t)gridDim.x * blockDim.x) {
    if (skip) {
      uint32_t lo = 0, hi = P;   // partition p with sb[p] <= r < sb[p + 1]
      while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (sb[mid] <= r) lo = mid;
        else hi = mid;
      }
      if (sk[lo] >= 0) continue;
    }
    if (ks == 8) ((unsigned long long*)hkey)[r] = ((const unsigned long long*)skey)[r];
    else ((unsigned int*)hkey)[r] = ((const unsigned int*)skey)[r];
    if (n_pay) {
      if (psz == 8) ((unsigned long long*)hpay)[r] = ((const unsigned long long*)spay)[r];
      else ((unsigned int*)hpay)[r] = ((const unsigned int*)spay)[r];
    }
  }
}

// Pass 2 probe of the two-table radix join: B's rows of one partition, read in place through
// their segment list, look up the partition's pre-aggregated A table.  A matching row adds A's
// row count for its key to the pair count, A's payload sum for the key to SUM(A), and the count
// times its own payload to SUM(B).  The three sums go to acc[0..2] (one atomic per workgroup).
template <typename K>
__global__ void __launch_bounds__(256) k_rj_probe(TableView t, const void* key, const void* pay,
                                                  uint32_t pay_size, SegList sl, unsigned long long* acc) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  __shared__ unsigned long long sst[kMaxSegs], spre[kMaxSegs + 1];
  for (uint32_t j = threadIdx.x; j < sl.nseg; j += blockDim.x) sst[j] = sl.start[j];
  for (uint32_t j = threadIdx.x; j <= sl.nseg; j += blockDim.x) spre[j] = sl.prefix[j];
  __syncthreads();
  unsigned long long a[3] = {0, 0, 0};
  // 4 rows per lane: 8 rows, or up to 16 workgroups per compute unit, measured the same (the
  // host link bounds the kernel)
  constexpr int ITEMS = 4;
  const uint64_t tile = (uint64_t)blockDim.x * ITEMS;
  for (uint64_t base = blockIdx.x * tile; base < sl.total; base += (uint64_t)gridDim.x * tile) {
    K kk[ITEMS];
    unsigned long long vv[ITEMS];
    uint32_t sg = seg_find(spre, sl.nseg, base);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      kk[j] = (K)0;
      vv[j] = 0;
      if (i < sl.total) {
        sg = seg_advance(spre, sl.nseg, sg, i);
        const uint64_t src = sst[sg] + (i - spre[sg]);
        kk[j] = load_key<K>(key, src);
        if (pay) vv[j] = (unsigned long long)load_signed(pay, src, pay_size);
      }
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      if (i >= sl.total) continue;
      const unsigned long long* w;
      if ((U)kk[j] == kEmpty) {
        w = t.side;
      } else {
        const uint8_t* s = find_slot_hashed<K>(t, kk[j]);
        if (!s) continue;
        w = (const unsigned long long*)(s + 8);
      }
      const unsigned long long c = w[0];
      if (c) {
        a[0] += c;
        a[1] += w[1];
        a[2] += c * vv[j];
      }
    }
  }
  block_flush<3>(a, 3, acc);
}

// ---------------------------------------------------------------- host side

namespace {

struct Side {
  ColInfo key;
  ColInfo pay[kMaxPay];
  uint32_t n_pay = 0;
  uint64_t n = 0;
  // the clustered copy, as device addresses: arena memory, or mapped pinned host memory
  uint8_t* clu_key = nullptr;
  uint8_t* clu_pay[kMaxPay] = {};
  bool on_device = false;               // the clustered copy lives in the arena
  uint64_t chunk_rows = 0, n_chunks = 0;
  std::vector<unsigned long long> bnd;  // n_chunks * (P + 1)
  std::vector<unsigned long long> slot_sums;   // 2 * kMaxSumSlots: count, payload-0 sum
  uint64_t sdma = 0;
};

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// grid-stride launch over n items: at most 8 workgroups per compute unit
unsigned grid_for(const vx_ctx* ctx, uint64_t n) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, (uint64_t)ctx->cu_count * 8));
}

// Pass 1 for one table: stream, cluster each chunk by partition, write it back with its
// boundary array.
// Plans pass 1's pipeline over one side: chunks of 64 MiB of keys (at most kMaxSegs chunks), and
// up to `deep` chunk buffers when the arena can spare a quarter of its free bytes for them.
vx_status plan_pass1(vx_ctx* ctx, Side& sd, uint32_t deep, Pipeline& pipe) {
  std::vector<PipeCol> cols(1 + sd.n_pay);
  cols[0].info = sd.key;
  cols[0].may_copy = cols[0].copy = true;
  uint64_t row_bytes = (uint64_t)sd.key.elsize;
  for (uint32_t c = 0; c < sd.n_pay; ++c) {
    cols[1 + c].info = sd.pay[c];
    cols[1 + c].may_copy = cols[1 + c].copy = true;
    row_bytes += (uint64_t)sd.pay[c].elsize;
  }
  const uint64_t min_rows = (sd.n + kMaxSegs - 1) / kMaxSegs;
  const uint64_t want = env_u64("VX_CHUNK_BYTES", 64ull << 20) / 8;
  const uint64_t rows = std::max(min_rows, std::min<uint64_t>(want, std::max<uint64_t>(sd.n, 1)));
  uint32_t nbuf = 0;
  if (deep > 2) {
    const uint64_t spare = (ctx->arena.capacity() - ctx->arena.used()) / 4;
    nbuf = (uint32_t)std::max<uint64_t>(2, std::min<uint64_t>(deep, spare / (rows * row_bytes + 1024)));
  }
  VX_TRY(pipe.plan(ctx, sd.n, rows, nbuf, cols));
  sd.chunk_rows = pipe.chunk_rows();
  sd.n_chunks = pipe.n_chunks();
  return VX_OK;
}

// Pass 1 over one side through its planned pipeline (whose first copies may already be in
// flight): cluster each chunk and record its boundary array.
vx_status cluster_side(vx_ctx* ctx, const PartSpec& ps, const int* sum_slot_dev, Side& sd, Pipeline& pipe) {
  const uint32_t P = ps.n_parts;
  uint64_t row_bytes = (uint64_t)sd.key.elsize;
  for (uint32_t c = 0; c < sd.n_pay; ++c) row_bytes += (uint64_t)sd.pay[c].elsize;
  // staging for clustered chunks (double-buffered against the write-back), per-wave
  // histograms, offsets, per-chunk boundaries and singleton sums
  PartGeom g0 = part_geom(ctx, sd.chunk_rows);
  // (a device-resident clustered copy is scattered into directly: no staging, no write-back)
  uint64_t stage_bytes = sd.on_device ? 0 : align_up(sd.chunk_rows * row_bytes + 256 * (1 + kMaxPay), 256);
  uint64_t scratch = 2 * stage_bytes + (uint64_t)P * g0.waves * 12 +
                     std::max<uint64_t>(sd.n_chunks, 1) * (P + 1) * 8 + 2 * kMaxSumSlots * 8 + 1024;
  ArenaBlock blk;
  blk.a = &ctx->arena;
  blk.p = ctx->arena.alloc(scratch);
  VX_CHECK(blk.p, VX_EBUDGET, "partitioned join: no room for the partition pass scratch (%llu B)",
           (unsigned long long)scratch);
  uint8_t* stage[2] = {blk.p, blk.p + stage_bytes};
  uint32_t* hist = (uint32_t*)(blk.p + 2 * stage_bytes);
  unsigned long long* offs = (unsigned long long*)((uint8_t*)hist + (uint64_t)P * g0.waves * 4);
  unsigned long long* bnd = offs + (uint64_t)P * g0.waves;
  unsigned long long* sums = bnd + std::max<uint64_t>(sd.n_chunks, 1) * (P + 1);
  fill_zero((uint64_t*)sums, 2 * kMaxSumSlots, ctx->compute);
  hipEvent_t done[2] = {get_event(ctx), get_event(ctx)};
  hipEvent_t wrote[2] = {get_event(ctx), get_event(ctx)};
  bool pending[2] = {false, false};
  const unsigned wb_grid = (unsigned)ctx->cu_count * 8;
  auto kernel = [&](const ChunkView& v) -> vx_status {
    uint32_t b = (uint32_t)(v.index % 2);
    if (pending[b]) VX_HIP(hipStreamWaitEvent(ctx->compute, wrote[b], 0));
    PartIO io{};
    io.key = (v.global_mask & 1u) ? (const uint8_t*)v.ptr[0] + v.row0 * sd.key.elsize : v.ptr[0];
    io.key_size = (uint32_t)sd.key.elsize;
    io.n = v.rows;
    io.n_pay = sd.n_pay;
    uint8_t* out = stage[b];
    io.out_key = sd.on_device ? sd.clu_key + v.row0 * sd.key.elsize : out;
    uint64_t off = align_up(v.rows * sd.key.elsize, 256);
    for (uint32_t c = 0; c < sd.n_pay; ++c) {
      io.pay[c] = ((v.global_mask >> (1 + c)) & 1u)
                      ? (const uint8_t*)v.ptr[1 + c] + v.row0 * sd.pay[c].elsize
                      : v.ptr[1 + c];
      io.pay_size[c] = (uint32_t)sd.pay[c].elsize;
      io.out_pay[c] = sd.on_device ? sd.clu_pay[c] + v.row0 * sd.pay[c].elsize : out + off;
      off += align_up(v.rows * sd.pay[c].elsize, 256);
    }
    PartGeom g = part_geom(ctx, v.rows);
    VX_TRY(part_hist(ctx, ps, io, g, hist, nullptr, sum_slot_dev, sum_slot_dev ? sums : nullptr,
                     ctx->compute));
    VX_TRY(part_scan(ctx, hist, P, g.waves, nullptr, offs, bnd + v.index * (P + 1), ctx->compute));
    VX_TRY(part_scatter(ctx, ps, io, g, offs, ctx->compute));
    if (sd.on_device) return VX_OK;
    VX_HIP(hipEventRecord(done[b], ctx->compute));
    // write the clustered chunk back to host memory at the chunk's own rows
    VX_HIP(hipStreamWaitEvent(ctx->d2h, done[b], 0));
    VX_CHECK(sd.n_pay <= 1, VX_EUNSUPPORTED, "partition pass: at most one payload column");
    hipLaunchKernelGGL(k_pj_writeback, dim3(wb_grid), dim3(256), 0, ctx->d2h, (const uint8_t*)io.out_key,
                       (const uint8_t*)(sd.n_pay ? io.out_pay[0] : nullptr), (uint32_t)sd.key.elsize,
                       sd.n_pay ? (uint32_t)sd.pay[0].elsize : 0u, sd.n_pay, v.rows, bnd + v.index * (P + 1), P,
                       sum_slot_dev, sd.clu_key + v.row0 * sd.key.elsize,
                       sd.n_pay ? sd.clu_pay[0] + v.row0 * sd.pay[0].elsize : nullptr);
    VX_HIP(hipGetLastError());
    VX_HIP(hipEventRecord(wrote[b], ctx->d2h));
    pending[b] = true;
    return VX_OK;
  };
  vx_status st = pipe.run(kernel);
  (void)hipStreamSynchronize(ctx->compute);
  (void)hipStreamSynchronize(ctx->d2h);
  for (int b = 0; b < 2; ++b) {
    put_event(ctx, done[b]);
    put_event(ctx, wrote[b]);
  }
  VX_TRY(st);
  sd.sdma = pipe.sdma_bytes();
  sd.bnd.assign(sd.n_chunks * (P + 1), 0);
  sd.slot_sums.assign(2 * kMaxSumSlots, 0);
  if (sd.n_chunks) VX_HIP(hipMemcpy(sd.bnd.data(), bnd, sd.bnd.size() * 8, hipMemcpyDeviceToHost));
  VX_HIP(hipMemcpy(sd.slot_sums.data(), sums, sd.slot_sums.size() * 8, hipMemcpyDeviceToHost));
  return VX_OK;
}

// segments of partition p across the chunks of one side (row starts in the clustered copy)
uint64_t segments(const Side& sd, uint32_t P, uint32_t p, std::vector<unsigned long long>& start,
                  std::vector<unsigned long long>& prefix) {
  start.clear();
  prefix.clear();
  uint64_t tot = 0;
  for (uint64_t c = 0; c < sd.n_chunks; ++c) {
    const unsigned long long* b = sd.bnd.data() + c * (P + 1);
    uint64_t len = b[p + 1] - b[p];
    if (!len) continue;
    start.push_back(c * sd.chunk_rows + b[p]);
    prefix.push_back(tot);
    tot += len;
  }
  prefix.push_back(tot);
  return tot;
}

}  // namespace

vx_status join_partitioned(vx_ctx* ctx, const vx_partitioned_join* d, vx_join_out* out) {
  double t0 = now_ms();
  const vx_build_desc& B = d->build;
  const vx_probe_desc& Q = d->probe;
  VX_CHECK(B.key.type == Q.key.type, VX_EINVAL, "partitioned join: key types differ");
  VX_CHECK(B.n_pay <= 1, VX_EUNSUPPORTED, "partitioned join: at most one build payload");
  VX_CHECK(B.n_pay == 0 || B.pay, VX_EINVAL, "partitioned join: build pay is NULL");
  VX_CHECK(Q.n_pay == 0, VX_EUNSUPPORTED, "partitioned join: probe payloads are not supported");
  VX_HIP(hipSetDevice(ctx->device));
  Side bs, qs;
  bs.n = B.n;
  qs.n = Q.n;
  VX_TRY(classify(ctx, B.key, B.n, &bs.key, "partitioned build key"));
  bs.n_pay = B.n_pay;
  for (uint32_t c = 0; c < B.n_pay; ++c) VX_TRY(classify(ctx, B.pay[c], B.n, &bs.pay[c], "partitioned build payload"));
  VX_TRY(classify(ctx, Q.key, Q.n, &qs.key, "partitioned probe key"));
  const int ks = bs.key.elsize;

  // partitioner
  vx_part_opts o = d->part;
  uint32_t req = o.n_parts ? o.n_parts : 256;
  std::vector<int64_t> split;
  CdfReport rep{};
  uint32_t method = o.method;
  // pass 1's pipeline is planned first: while the splitters are computed from the key sample,
  // the copies of its first chunks already run (pass 1 needs the splitters only for its kernels)
  const bool sampled = method == VX_PART_LEARNED || method == VX_PART_QUANTILE ||
                       method == VX_PART_UNTRAINED || method == VX_PART_AUTO;
  std::unique_ptr<Pipeline> pipe1(new Pipeline);
  VX_TRY(plan_pass1(ctx, bs, sampled ? 48u : 0u, *pipe1));
  if (sampled) VX_TRY(pipe1->prefetch(pipe1->n_buffers()));
  double tt0 = now_ms();
  if (method == VX_PART_LEARNED || method == VX_PART_QUANTILE || method == VX_PART_UNTRAINED ||
      method == VX_PART_AUTO) {
    VX_TRY(cdf_splitters(ctx, bs.key, B.n, o, req, &split, &rep, nullptr));
    if (method == VX_PART_AUTO) {
      bool singleton = false;
      for (size_t i = 1; i < split.size(); ++i) singleton |= split[i] == split[i - 1] + 1;
      method = singleton ? (rep.auto_quantile ? VX_PART_QUANTILE : VX_PART_LEARNED) : VX_PART_RADIX_HASH;
    }
  }
  double train_ms = now_ms() - tt0;
  const bool trace = getenv("VX_TRACE") != nullptr;
  if (trace && rep.sample_rows)
    fprintf(stderr, "[vx] splitters: sample %llu rows %.1f ms, sort %.1f ms, fit %.1f ms, split %.1f ms, loss %.3g\n",
            (unsigned long long)rep.sample_rows, rep.sample_ms, rep.sort_ms, rep.train_ms, rep.split_ms,
            rep.final_loss);
  vx_part_opts eff = o;
  eff.method = (method == VX_PART_LEARNED || method == VX_PART_QUANTILE || method == VX_PART_UNTRAINED)
                   ? VX_PART_RANGE
                   : method;
  if (eff.method == VX_PART_RANGE && o.method == VX_PART_RANGE) {
    VX_CHECK(o.n_splitters == 0 || o.splitters, VX_EINVAL, "partitioned join: splitters is NULL");
    split.assign(o.splitters, o.splitters + o.n_splitters);
  }
  ArenaBlock split_mem;
  PartSpec ps;
  VX_TRY(make_spec(ctx, eff, req, split.data(), (uint32_t)split.size(), split_mem, &ps));
  const uint32_t P = ps.n_parts;

  // singleton partitions (range methods): [s_{p-1}, s_p) holding exactly one key value
  std::vector<int> slot(P, -1);
  uint32_t n_single = 0;
  if (ps.fn == kPartRange) {
    for (uint32_t p = 1; p + 1 < P && n_single < kMaxSumSlots; ++p)
      if (split[p] == split[p - 1] + 1) slot[p] = (int)n_single++;
  }
  ArenaBlock slot_mem;
  const int* slot_dev = nullptr;
  if (n_single) {
    slot_mem.a = &ctx->arena;
    slot_mem.p = ctx->arena.alloc(P * sizeof(int));
    VX_CHECK(slot_mem.p, VX_EBUDGET, "partitioned join: no room for singleton slots");
    VX_HIP(hipMemcpyAsync(slot_mem.p, slot.data(), P * sizeof(int), hipMemcpyHostToDevice, ctx->compute));
    slot_dev = (const int*)slot_mem.p;
  }

  // Where the clustered build side lives.  In the arena when the range splitters' sample
  // predicts that pass 2 fits beside it: the clustered rows, the transient table of the largest
  // partition, and compact tables sized from the sample's distinct-key share (about 1.8 slots of
  // 32 B per distinct key after power-of-two rounding).  Otherwise in pinned host memory, read
  // back by zero-copy.  Radix-hash partitions come with no size prediction and take the host plan.
  uint64_t hbytes = align_up(B.n * ks, 256);
  for (uint32_t c = 0; c < B.n_pay; ++c) hbytes += align_up(B.n * bs.pay[c].elsize, 256);
  double plan_compact = 0;   // expected bytes of the compact tables (0: no prediction)
  {
    const uint64_t mode = env_u64("VX_PJ_DEVICE", 2);   // 0 host, 1 device, 2 planned
    bool fits = false;
    if (ps.fn == kPartRange && rep.sample_rows > 0) {
      const double ns_rows = (double)B.n * (1.0 - rep.single_share);
      const double part_rows = (double)B.n * rep.max_share * 1.25 + 1024.0;
      const double tbytes = 32.0 * 2.0 * 1.25 * part_rows;
      plan_compact = 32.0 * 1.8 * rep.distinct_share * ns_rows;
      const double pipe_bytes = 3.0 * (64 << 20) * 2.0 + (512 << 20);
      // pass 1 holds the clustered copy beside its own chunk buffers; pass 2 gets those back
      uint64_t row_bytes = (uint64_t)ks;
      for (uint32_t c = 0; c < B.n_pay; ++c) row_bytes += (uint64_t)bs.pay[c].elsize;
      const double pass1_bytes = (double)pipe1->n_buffers() * (double)(bs.chunk_rows * row_bytes);
      const double free_now = (double)(ctx->arena.capacity() - ctx->arena.used());
      fits = (double)hbytes + (64 << 20) <= (double)ctx->arena.largest_free() &&
             free_now + pass1_bytes - (double)hbytes >= tbytes + plan_compact + pipe_bytes;
      if (trace)
        fprintf(stderr, "[vx] plan: clustered %.2f GiB + transient %.2f GiB + compact %.2f GiB (distinct share "
                "%.3f, singleton share %.3f) vs %.2f GiB free: %s\n", hbytes / 1073741824.0, tbytes / 1073741824.0,
                plan_compact / 1073741824.0, rep.distinct_share, rep.single_share,
                ctx->arena.largest_free() / 1073741824.0, fits ? "fits" : "does not fit");
    }
    bs.on_device = mode == 1 || (mode == 2 && fits);
  }
  ArenaBlock cl_mem;
  uint8_t* hs = nullptr;
  if (bs.on_device) {
    cl_mem.a = &ctx->arena;
    cl_mem.p = ctx->arena.alloc(hbytes + 256);
    VX_CHECK(cl_mem.p, VX_EBUDGET, "partitioned join: no room for the clustered build side (%llu B)",
             (unsigned long long)hbytes);
    hs = cl_mem.p;
  } else {
    VX_TRY(host_scratch(ctx, hbytes + 256, &hs));
  }
  void* hs_dev = hs;
  if (!bs.on_device) VX_HIP(hipHostGetDevicePointer(&hs_dev, hs, 0));
  bs.clu_key = (uint8_t*)hs_dev;
  uint64_t off = align_up(B.n * ks, 256);
  for (uint32_t c = 0; c < B.n_pay; ++c) {
    bs.clu_pay[c] = (uint8_t*)hs_dev + off;
    off += align_up(B.n * bs.pay[c].elsize, 256);
  }

  // pass 1: cluster the build side
  double tp0 = now_ms();
  VX_TRY(cluster_side(ctx, ps, slot_dev, bs, *pipe1));
  pipe1.reset();   // pass 1's chunk buffers go back to the arena before pass 2
  double part_ms = now_ms() - tp0;
  std::vector<uint64_t> brows(P, 0);
  for (uint64_t c = 0; c < bs.n_chunks; ++c)
    for (uint32_t p = 0; p < P; ++p) brows[p] += bs.bnd[c * (P + 1) + p + 1] - bs.bnd[c * (P + 1) + p];

  // pass 2 memory: transient table (largest non-singleton partition, worst case all keys
  // distinct at load 0.8), side records, partition directory, per-block accumulators,
  // build segment lists, the probe pipeline's buffers, and the compact tables in the rest
  double tj0 = now_ms();
  uint64_t max_rows = 0;
  for (uint32_t p = 0; p < P; ++p)
    if (slot[p] < 0) max_rows = std::max(max_rows, brows[p]);
  auto pow2_at_least = [](uint64_t v) {
    uint64_t c = 64;
    while (c < v) c <<= 1;
    return c;
  };
  const uint64_t tcap_max = pow2_at_least(max_rows + max_rows / 4);
  const unsigned G = (unsigned)ctx->cu_count * 2;   // probe-stream grid (fixed: accumulator rows)
  const uint64_t seg_stride = 2 * (uint64_t)(kMaxSegs + 1);
  uint8_t* mem_t = nullptr;
  ArenaBlock tmem, aux;
  tmem.a = aux.a = &ctx->arena;
  tmem.p = ctx->arena.alloc((tcap_max << kSlotShift) + 256 + tcap_max * 4);
  VX_CHECK(tmem.p, VX_EBUDGET,
           "partitioned join: the largest partition (%llu build rows, %llu transient slots) does not fit "
           "the arena; use more partitions", (unsigned long long)max_rows, (unsigned long long)tcap_max);
  mem_t = tmem.p;
  uint32_t* claims = (uint32_t*)(mem_t + (tcap_max << kSlotShift) + 256);   // slots claimed by a build
  const uint64_t aux_words = (uint64_t)P * kSideWords + (uint64_t)P + (uint64_t)P +
                             (uint64_t)G * 3 * P + 3ull * P + (uint64_t)P * seg_stride + 8;
  aux.p = ctx->arena.alloc(aux_words * 8);
  VX_CHECK(aux.p, VX_EBUDGET, "partitioned join: no room for the partition directory");
  unsigned long long* side_all = (unsigned long long*)aux.p;
  unsigned long long* tab_slots = side_all + (uint64_t)P * kSideWords;
  uint32_t* tab_log2 = (uint32_t*)(tab_slots + P);
  unsigned long long* accb = tab_slots + 2 * (uint64_t)P;    // tab_log2 takes P/2 words; P words reserved
  unsigned long long* acc_out = accb + (uint64_t)G * 3 * P;
  unsigned long long* segdev = acc_out + 3ull * P;
  unsigned long long* distinct = segdev + (uint64_t)P * seg_stride;   // claims in the transient table
  fill_zero((uint64_t*)aux.p, aux_words, ctx->compute);
  hipLaunchKernelGGL(k_pj_init, dim3(grid_for(ctx, tcap_max)), dim3(256), 0, ctx->compute, (uint32_t*)mem_t,
                     tcap_max, (uint32_t)ks, (unsigned long long*)nullptr);
  fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);
  // build segment lists of every partition: [p][start | prefix]
  std::vector<unsigned long long> hseg((uint64_t)P * seg_stride, 0);
  std::vector<uint64_t> nb_of(P, 0), sb_of(P, 0);
  {
    std::vector<unsigned long long> st, pre;
    for (uint32_t p = 0; p < P; ++p) {
      unsigned long long* h = hseg.data() + (uint64_t)p * seg_stride;
      nb_of[p] = segments(bs, P, p, st, pre);
      sb_of[p] = st.size();
      std::copy(st.begin(), st.end(), h);
      std::copy(pre.begin(), pre.end(), h + (kMaxSegs + 1));
    }
  }
  VX_HIP(hipMemcpyAsync(segdev, hseg.data(), hseg.size() * 8, hipMemcpyHostToDevice, ctx->compute));
  // probe pipeline (keys only).  On the device plan pass 2 reads HBM and leaves the host link
  // idle, so the pipeline takes every chunk buffer the arena spares beside the expected
  // compact tables and starts their copies before the builds.
  std::vector<PipeCol> qcols(1);
  qcols[0].info = qs.key;
  qcols[0].may_copy = qcols[0].copy = true;
  uint32_t qbuf = Q.n_buffers;
  if (bs.on_device && plan_compact > 0 && qs.key.where == Where::Host && Q.n_buffers == 0) {
    const uint64_t chunk_bytes = env_u64("VX_CHUNK_BYTES", 64ull << 20) + 256;
    // buffers fill holes first (first fit); the compact tables then need one contiguous block
    const double spare = (double)(ctx->arena.capacity() - ctx->arena.used()) - 1.05 * plan_compact -
                         (double)(512u << 20);
    qbuf = (uint32_t)std::max<double>(2.0, std::min<double>((double)kMaxBuffers, spare / (double)chunk_bytes));
  }
  Pipeline pipe;
  VX_TRY(pipe.plan(ctx, Q.n, Q.chunk_rows, qbuf, qcols));
  // compact tables: most of what is left
  ArenaBlock cmem;
  cmem.a = &ctx->arena;
  uint64_t cbytes = ctx->arena.largest_free() / 256 * 256;
  cbytes = cbytes > (1u << 20) ? cbytes - (1u << 20) : 0;
  VX_CHECK(cbytes >= 4096, VX_EBUDGET, "partitioned join: no room left for the partition tables");
  cmem.p = ctx->arena.alloc(cbytes);
  VX_CHECK(cmem.p, VX_EBUDGET, "partitioned join: no room left for the partition tables");

  const uint8_t* dk_b = bs.clu_key;
  const uint8_t* dp_b = B.n_pay ? bs.clu_pay[0] : nullptr;
  const uint32_t psz = B.n_pay ? (uint32_t)bs.pay[0].elsize : 8;
  const bool k64 = B.key.type == VX_I64;
  uint64_t launches = 0, stream_passes = 0;
  const size_t lds_bytes = (size_t)(5 * P + ps.n_split) * 8;
  std::vector<unsigned long long> h_slots(P, 0);
  std::vector<uint32_t> h_log2(P, 0);

  // one pass over the probe side against the partitions resident now
  auto stream_probe = [&]() -> vx_status {
    VX_HIP(hipMemcpyAsync(tab_slots, h_slots.data(), P * 8, hipMemcpyHostToDevice, ctx->compute));
    VX_HIP(hipMemcpyAsync(tab_log2, h_log2.data(), P * 4, hipMemcpyHostToDevice, ctx->compute));
    const uint32_t count_rows = stream_passes == 0 ? 1u : 0u;
    auto kern = [&](const ChunkView& v) -> vx_status {
      const void* keys = (v.global_mask & 1u) ? (const uint8_t*)v.ptr[0] + v.row0 * ks : v.ptr[0];
      if (k64)
        hipLaunchKernelGGL(k_pj_stream<int64_t>, dim3(G), dim3(256), lds_bytes, ctx->compute, keys, v.rows, ps,
                           tab_slots, tab_log2, side_all, count_rows, accb);
      else
        hipLaunchKernelGGL(k_pj_stream<int32_t>, dim3(G), dim3(256), lds_bytes, ctx->compute, keys, v.rows, ps,
                           tab_slots, tab_log2, side_all, count_rows, accb);
      VX_HIP(hipGetLastError());
      return VX_OK;
    };
    VX_TRY(pipe.run(kern));
    ++stream_passes;
    return VX_OK;
  };

  // pass 2: per non-singleton partition, pre-aggregate its build segments into the transient
  // table, then compact it into a table sized by its distinct keys; when the compact tables
  // fill their region, stream the probe side against them and start over
  VX_TRY(pipe.prefetch(pipe.n_buffers()));
  uint64_t cused = 0;
  bool any_resident = false;
  double dmx = 0, dtot = 0;   // distinct build keys of the table partitions
  uint32_t dparts = 0;
  for (uint32_t p = 0; p < P; ++p) {
    if (slot[p] >= 0 || brows[p] == 0) continue;
    const uint64_t nb = nb_of[p];
    TableView t{};
    const uint64_t tcap = pow2_at_least(nb + nb / 4);
    t.slots = mem_t;
    t.mask = tcap - 1;
    while ((1ull << t.log2cap) < tcap) ++t.log2cap;
    t.slot_shift = kSlotShift;
    t.side = side_all + (uint64_t)p * kSideWords;
    t.n_pay = B.n_pay;
    t.preagg = 1;
    t.key_size = (uint32_t)ks;
    const unsigned long long* h = segdev + (uint64_t)p * seg_stride;
    SegList lb{h, h + (kMaxSegs + 1), (uint32_t)sb_of[p], nb};
    unsigned gb = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((nb + kPjTile - 1) / kPjTile,
                                                                     (uint64_t)ctx->cu_count * 3));
    fill_zero((uint64_t*)distinct, 1, ctx->compute);
    if (k64)
      hipLaunchKernelGGL(k_pj_build<int64_t>, dim3(gb), dim3(256), 0, ctx->compute, t, dk_b, dp_b, psz, lb,
                         ctx->dev_flags, claims, distinct);
    else
      hipLaunchKernelGGL(k_pj_build<int32_t>, dim3(gb), dim3(256), 0, ctx->compute, t, dk_b, dp_b, psz, lb,
                         ctx->dev_flags, claims, distinct);
    VX_HIP(hipGetLastError());
    unsigned long long nd = 0;
    VX_HIP(hipMemcpyAsync(&nd, distinct, 8, hipMemcpyDeviceToHost, ctx->compute));
    VX_HIP(hipStreamSynchronize(ctx->compute));
    VX_TRY(check_flags(ctx, "partitioned join (build)"));
    dmx = std::max(dmx, (double)nd);
    dtot += (double)nd;
    ++dparts;
    const uint64_t ccap = pow2_at_least(nd + nd / 4);   // load factor 0.4 .. 0.8
    const uint64_t need = ccap << kSlotShift;
    VX_CHECK(need <= cbytes, VX_EBUDGET,
             "partitioned join: partition %u's table (%llu distinct keys) does not fit the arena", p,
             (unsigned long long)nd);
    if (cused + need > cbytes) {
      VX_TRY(stream_probe());
      VX_HIP(hipStreamSynchronize(ctx->compute));
      std::fill(h_slots.begin(), h_slots.end(), 0ull);
      std::fill(h_log2.begin(), h_log2.end(), 0u);
      cused = 0;
      any_resident = false;
    }
    TableView c{};
    c.slots = cmem.p + cused;
    c.mask = ccap - 1;
    while ((1ull << c.log2cap) < ccap) ++c.log2cap;
    c.slot_shift = kSlotShift;
    hipLaunchKernelGGL(k_pj_init, dim3(grid_for(ctx, ccap)), dim3(256), 0, ctx->compute, (uint32_t*)c.slots, ccap,
                       (uint32_t)ks, (unsigned long long*)nullptr);
    if (k64)
      hipLaunchKernelGGL(k_pj_compact<int64_t>, dim3(grid_for(ctx, nd)), dim3(256), 0, ctx->compute, mem_t, claims,
                         (uint64_t)nd, c);
    else
      hipLaunchKernelGGL(k_pj_compact<int32_t>, dim3(grid_for(ctx, nd)), dim3(256), 0, ctx->compute, mem_t, claims,
                         (uint64_t)nd, c);
    VX_HIP(hipGetLastError());
    h_slots[p] = (unsigned long long)(uintptr_t)c.slots;
    h_log2[p] = c.log2cap;
    cused += need;
    any_resident = true;
    launches += 4;
  }
  // the last pass also counts the probe rows of partitions no pass has seen (singletons,
  // empty build partitions) when no earlier pass ran
  const double tb1 = now_ms();
  if (any_resident || stream_passes == 0) VX_TRY(stream_probe());
  launches += pipe.kernel_launches();
  hipLaunchKernelGGL(k_pj_reduce, dim3((3 * P + 255) / 256), dim3(256), 0, ctx->compute, accb, G, 3 * P, acc_out);
  VX_HIP(hipGetLastError());
  std::vector<unsigned long long> accs(3ull * P);
  VX_HIP(hipMemcpyAsync(accs.data(), acc_out, accs.size() * 8, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  VX_TRY(check_flags(ctx, "partitioned join"));
  double join_ms = now_ms() - tj0;
  if (trace)
    fprintf(stderr, "[vx] partitioned join: pass 1 %.1f ms; pass 2 builds until %.1f ms, probe stream %.1f ms, "
            "%llu probe pass(es), transient slots %llu, compact tables %.1f MiB of %.1f MiB, clustered copy in %s\n",
            part_ms, tb1 - tj0, now_ms() - tb1, (unsigned long long)stream_passes, (unsigned long long)tcap_max,
            cused / 1048576.0, cbytes / 1048576.0, bs.on_device ? "device memory" : "host memory");

  // per-partition aggregates: pass 2 results, or the singleton closed form
  std::vector<vx_agg> per(P);
  std::vector<uint64_t> qrows(P, 0);
  uint64_t single_rows = 0;
  for (uint32_t p = 0; p < P; ++p) {
    std::memset(&per[p], 0, sizeof(vx_agg));
    qrows[p] = accs[3 * p];
    if (slot[p] >= 0) {
      uint64_t cb = bs.slot_sums[2 * slot[p]], sb = bs.slot_sums[2 * slot[p] + 1];
      uint64_t cq = qrows[p];
      per[p].match_count = cb * cq;
      per[p].sum[0] = sb * cq;
      single_rows += cb + cq;
    } else {
      per[p].match_count = accs[3 * p + 1];
      if (B.n_pay) per[p].sum[0] = accs[3 * p + 2];
    }
  }
  std::memset(&out->agg, 0, sizeof out->agg);
  for (uint32_t p = 0; p < P; ++p) {
    out->agg.match_count += per[p].match_count;
    for (uint32_t c = 0; c < B.n_pay; ++c) out->agg.sum[c] += per[p].sum[c];
  }
  if (Q.chunk_aggs) {
    VX_CHECK(Q.chunk_aggs_cap >= P, VX_ECAPACITY, "partitioned join: chunk_aggs_cap %llu < %u partitions",
             (unsigned long long)Q.chunk_aggs_cap, P);
    std::copy(per.begin(), per.end(), Q.chunk_aggs);
  }
  double mx = 0, tot = 0;
  for (uint32_t p = 0; p < P; ++p) {
    mx = std::max(mx, (double)(brows[p] + qrows[p]));
    tot += (double)(brows[p] + qrows[p]);
  }
  vx_stats& s = out->stats;
  std::memset(&s, 0, sizeof s);
  s.rows = Q.n;
  s.chunks = pipe.n_chunks();
  s.chunk_rows = pipe.chunk_rows();
  s.n_buffers = pipe.n_buffers();
  s.n_parts = P;
  s.imbalance = tot > 0 ? mx / (tot / P) : 0.0;
  s.part_ms = part_ms;
  s.train_ms = train_ms;
  s.singleton_rows = single_rows;
  double tmx = 0, ttot = 0;
  uint32_t tparts = 0;
  for (uint32_t p = 0; p < P; ++p)
    if (slot[p] < 0) {
      s.survivors += qrows[p];
      tmx = std::max(tmx, (double)(brows[p] + qrows[p]));
      ttot += (double)(brows[p] + qrows[p]);
      ++tparts;
    }
  s.imbalance_tables = ttot > 0 ? tmx / (ttot / tparts) : 0.0;
  s.imbalance_distinct = dtot > 0 ? dmx / (dtot / dparts) : 0.0;
  s.sdma_bytes = bs.sdma + pipe.sdma_bytes();
  uint64_t pass2_bytes = 0;
  for (uint32_t p = 0; p < P; ++p)
    if (slot[p] < 0 && !bs.on_device) pass2_bytes += brows[p] * (ks + (B.n_pay ? bs.pay[0].elsize : 0));
  s.zc_bytes = pass2_bytes;
  s.build_ms = 0;
  s.probe_ms = join_ms;
  s.kernel_ms = pipe.kernel_ms();
  s.kernel_launches = launches;
  s.total_ms = now_ms() - t0;
  out->part_method_used = method;
  return VX_OK;
}


// ---------------------------------------------------------------- two-table radix join

namespace {

uint64_t pow2_ge(uint64_t v) {
  uint64_t c = 64;
  while (c < v) c <<= 1;
  return c;
}

uint64_t side_row_bytes(const Side& sd) {
  uint64_t r = (uint64_t)sd.key.elsize;
  for (uint32_t c = 0; c < sd.n_pay; ++c) r += (uint64_t)sd.pay[c].elsize;
  return r;
}

uint64_t side_clustered_bytes(const Side& sd) {
  uint64_t b = align_up(sd.n * sd.key.elsize, 256);
  for (uint32_t c = 0; c < sd.n_pay; ++c) b += align_up(sd.n * sd.pay[c].elsize, 256);
  return b;
}

// Point a side's clustered copy at `base` (device address): key column, then payloads.
void place_side(Side& sd, uint8_t* base) {
  sd.clu_key = base;
  uint64_t off = align_up(sd.n * sd.key.elsize, 256);
  for (uint32_t c = 0; c < sd.n_pay; ++c) {
    sd.clu_pay[c] = base + off;
    off += align_up(sd.n * sd.pay[c].elsize, 256);
  }
}

// One partition: the input itself, read in place (no clustering pass).
void whole_side(Side& sd) {
  sd.clu_key = (uint8_t*)sd.key.dev;
  for (uint32_t c = 0; c < sd.n_pay; ++c) sd.clu_pay[c] = (uint8_t*)sd.pay[c].dev;
  sd.on_device = sd.key.where == Where::Device;
  sd.chunk_rows = sd.n;
  sd.n_chunks = 1;
  sd.bnd = {0ull, (unsigned long long)sd.n};
}

}  // namespace

vx_status join_radix(vx_ctx* ctx, const vx_radix_join* d, vx_join_out* out) {
  const double t0 = now_ms();
  const vx_build_desc& A = d->a;
  const vx_probe_desc& Bd = d->b;
  VX_CHECK(A.key.type == Bd.key.type, VX_EINVAL, "radix join: key types differ");
  VX_CHECK(A.n_pay <= 1 && Bd.n_pay <= 1, VX_EUNSUPPORTED, "radix join: at most one payload per side");
  VX_CHECK(A.n_pay == 0 || A.pay, VX_EINVAL, "radix join: A pay is NULL");
  VX_CHECK(Bd.n_pay == 0 || Bd.pay, VX_EINVAL, "radix join: B pay is NULL");
  VX_CHECK(d->n_parts == 0 || (d->n_parts <= kMaxParts && (d->n_parts & (d->n_parts - 1)) == 0), VX_EINVAL,
           "radix join: n_parts %u is not a power of two <= %u", d->n_parts, kMaxParts);
  VX_CHECK(d->shift < 64, VX_EINVAL, "radix join: shift %u > 63", d->shift);
  VX_CHECK(d->hash <= 1, VX_EINVAL, "radix join: hash must be 0 or 1");
  VX_CHECK(d->placement >= 0 && d->placement <= 2, VX_EINVAL, "radix join: placement must be 0, 1 or 2");
  VX_HIP(hipSetDevice(ctx->device));
  Side as, bs;
  as.n = A.n;
  bs.n = Bd.n;
  VX_TRY(classify(ctx, A.key, A.n, &as.key, "radix join A key"));
  VX_TRY(classify(ctx, Bd.key, Bd.n, &bs.key, "radix join B key"));
  as.n_pay = A.n_pay;
  bs.n_pay = Bd.n_pay;
  if (A.n_pay) VX_TRY(classify(ctx, A.pay[0], A.n, &as.pay[0], "radix join A payload"));
  if (Bd.n_pay) VX_TRY(classify(ctx, Bd.pay[0], Bd.n, &bs.pay[0], "radix join B payload"));
  const int ks = as.key.elsize;
  const bool k64 = A.key.type == VX_I64;
  std::memset(&out->agg, 0, sizeof out->agg);
  vx_stats& s = out->stats;
  std::memset(&s, 0, sizeof s);
  s.rows = Bd.n;

  // partition count: the fewest whose expected largest table (5% over an even share, at load
  // <= 0.8) takes at most 60% of the free arena
  const uint64_t free0 = ctx->arena.capacity() - ctx->arena.used();
  auto table_bytes = [](uint64_t rows) { return pow2_ge(rows + rows / 4) << kSlotShift; };
  uint32_t P = d->n_parts;
  if (!P) {
    P = 1;
    while (P < kMaxParts && (double)table_bytes((uint64_t)(1.05 * (double)A.n / P) + 64) > 0.6 * (double)free0)
      P <<= 1;
  }
  uint32_t log2p = 0;
  while ((1u << log2p) < P) ++log2p;
  VX_CHECK(d->hash || d->shift + log2p <= 64, VX_EINVAL, "radix join: shift %u + %u bits exceeds 64", d->shift,
           log2p);
  PartSpec ps{};
  ps.fn = d->hash ? kPartHash : kPartBits;
  ps.n_parts = P;
  ps.log2p = log2p;
  ps.shift = d->shift;
  const bool trace = getenv("VX_TRACE") != nullptr;

  // pass 1: cluster both tables (P > 1), into the arena or pinned host scratch
  ArenaBlock cl_mem;
  const double tp0 = now_ms();
  uint64_t pass1_launches = 0;
  if (P > 1 && A.n && Bd.n) {
    const uint64_t hA = side_clustered_bytes(as), hB = side_clustered_bytes(bs);
    const uint64_t rb = std::max(side_row_bytes(as), side_row_bytes(bs));
    const uint64_t exp_rows = (uint64_t)(1.05 * (double)A.n / P) + 64;
    const uint64_t pass1_est = 4 * std::min<uint64_t>(std::max(A.n, Bd.n), 1ull << 23) * rb + (64ull << 20);
    const bool dev = d->placement == 2 ||
                     (d->placement == 0 && hA + hB + 512 + table_bytes(exp_rows) + pass1_est + (256ull << 20) <= free0);
    as.on_device = bs.on_device = dev;
    uint8_t* base = nullptr;
    if (dev) {
      cl_mem.a = &ctx->arena;
      cl_mem.p = ctx->arena.alloc(hA + hB + 512);
      VX_CHECK(cl_mem.p, VX_EBUDGET, "radix join: no room in the arena for the clustered tables (%llu B)",
               (unsigned long long)(hA + hB));
      base = cl_mem.p;
    } else {
      uint8_t* hs = nullptr;
      VX_TRY(host_scratch(ctx, hA + hB + 512, &hs));
      void* hd = nullptr;
      VX_HIP(hipHostGetDevicePointer(&hd, hs, 0));
      base = (uint8_t*)hd;
    }
    place_side(as, base);
    place_side(bs, base + align_up(hA, 256));
    for (Side* sd : {&as, &bs}) {
      std::unique_ptr<Pipeline> pipe(new Pipeline);
      VX_TRY(plan_pass1(ctx, *sd, 4, *pipe));
      VX_TRY(cluster_side(ctx, ps, nullptr, *sd, *pipe));
      pass1_launches += pipe->kernel_launches();
    }
  } else {
    whole_side(as);
    whole_side(bs);
  }
  const double part_ms = now_ms() - tp0;
  std::vector<uint64_t> arows(P, 0), brows(P, 0);
  if (P > 1 && A.n && Bd.n) {
    for (uint64_t c = 0; c < as.n_chunks; ++c)
      for (uint32_t p = 0; p < P; ++p) arows[p] += as.bnd[c * (P + 1) + p + 1] - as.bnd[c * (P + 1) + p];
    for (uint64_t c = 0; c < bs.n_chunks; ++c)
      for (uint32_t p = 0; p < P; ++p) brows[p] += bs.bnd[c * (P + 1) + p + 1] - bs.bnd[c * (P + 1) + p];
  } else {
    arows[0] = A.n;
    brows[0] = Bd.n;
  }

  // pass 2 jobs: slices of A's rows of each partition that has rows on both sides
  const double tj0 = now_ms();
  uint64_t max_a = 0;
  for (uint32_t p = 0; p < P; ++p)
    if (brows[p]) max_a = std::max(max_a, arows[p]);
  const uint64_t seg_stride = 2 * (uint64_t)(kMaxSegs + 1);
  struct Job {
    uint32_t p;
    uint64_t lo, hi;
  };
  std::vector<Job> jobs;
  uint64_t tcap_max = 64;
  std::vector<unsigned long long> hseg;
  ArenaBlock tmem, aux;
  tmem.a = aux.a = &ctx->arena;
  // device memory: [side record | acc (3 P) | A segment lists (P) | B segment lists (P)], then
  // the largest table that fits (no larger than the largest partition needs)
  const uint64_t aux_words = kSideWords + 3ull * P + 2ull * P * seg_stride + 8;
  aux.p = ctx->arena.alloc(aux_words * 8);
  VX_CHECK(aux.p, VX_EBUDGET, "radix join: no room for the partition segment lists");
  unsigned long long* side = (unsigned long long*)aux.p;
  unsigned long long* acc = side + kSideWords;
  unsigned long long* segdev = acc + 3ull * P;
  fill_zero((uint64_t*)aux.p, kSideWords + 3ull * P, ctx->compute);
  if (max_a) {
    const uint64_t need = pow2_ge(max_a + max_a / 4);
    const uint64_t lf = ctx->arena.largest_free();
    const uint64_t room = lf > (1u << 20) ? lf - (1u << 20) : 0;
    while (tcap_max < need && ((tcap_max * 2) << kSlotShift) + 256 <= room) tcap_max <<= 1;
    VX_CHECK((tcap_max << kSlotShift) + 256 <= room, VX_EBUDGET,
             "radix join: no room for a pass-2 table of %llu slots", (unsigned long long)tcap_max);
    // slices of at most 4/5 of the slots: a slice of r rows gets pow2_ge(r + r/4) <= tcap_max slots
    const uint64_t slice = tcap_max / 5 * 4;
    for (uint32_t p = 0; p < P; ++p) {
      if (!arows[p] || !brows[p]) continue;
      for (uint64_t lo = 0; lo < arows[p]; lo += slice) jobs.push_back({p, lo, std::min(arows[p], lo + slice)});
    }
  }
  const uint64_t n_jobs = jobs.size();
  if (n_jobs) {
    tmem.p = ctx->arena.alloc((tcap_max << kSlotShift) + 256);
    VX_CHECK(tmem.p, VX_EBUDGET, "radix join: no room for a pass-2 table of %llu slots",
             (unsigned long long)tcap_max);
  }
  // segment lists of every partition that has a job: A's at [p], B's at [P + p]
  std::vector<uint32_t> a_nseg(P, 0), b_nseg(P, 0);
  if (n_jobs) {
    hseg.assign(2ull * P * seg_stride, 0ull);
    std::vector<unsigned long long> st, pre;
    for (uint32_t p = 0; p < P; ++p) {
      if (!arows[p] || !brows[p]) continue;
      unsigned long long* h = hseg.data() + (uint64_t)p * seg_stride;
      segments(as, P, p, st, pre);
      a_nseg[p] = (uint32_t)st.size();
      std::copy(st.begin(), st.end(), h);
      std::copy(pre.begin(), pre.end(), h + (kMaxSegs + 1));
      h = hseg.data() + (uint64_t)(P + p) * seg_stride;
      segments(bs, P, p, st, pre);
      b_nseg[p] = (uint32_t)st.size();
      std::copy(st.begin(), st.end(), h);
      std::copy(pre.begin(), pre.end(), h + (kMaxSegs + 1));
    }
    VX_HIP(hipMemcpyAsync(segdev, hseg.data(), hseg.size() * 8, hipMemcpyHostToDevice, ctx->compute));
  }
  fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);
  const uint32_t psz_a = A.n_pay ? (uint32_t)as.pay[0].elsize : 8;
  const uint32_t psz_b = Bd.n_pay ? (uint32_t)bs.pay[0].elsize : 8;
  const uint8_t* pay_a = A.n_pay ? as.clu_pay[0] : nullptr;
  const uint8_t* pay_b = Bd.n_pay ? bs.clu_pay[0] : nullptr;
  uint64_t zc_bytes = 0;
  // HIP events around each build and probe launch (on the stream they run on)
  std::vector<hipEvent_t> ev(3 * n_jobs, nullptr);
  for (auto& e : ev) e = get_event(ctx);
  // one job; on an error the stream is still drained before the table goes back to the arena
  auto job = [&](uint64_t j) -> vx_status {
    VX_CHECK(ev[3 * j] && ev[3 * j + 1] && ev[3 * j + 2], VX_EHIP, "radix join: no HIP event");
    const Job& jb = jobs[j];
    const uint64_t na = jb.hi - jb.lo, nbr = brows[jb.p];
    TableView t{};
    const uint64_t tcap = pow2_ge(na + na / 4);
    VX_CHECK(tcap <= tcap_max, VX_EINVAL, "radix join: slice of %llu rows exceeds the table", (unsigned long long)na);
    t.slots = tmem.p;
    t.mask = tcap - 1;
    while ((1ull << t.log2cap) < tcap) ++t.log2cap;
    t.slot_shift = kSlotShift;
    t.side = side;
    t.n_pay = A.n_pay;
    t.preagg = 1;
    t.key_size = (uint32_t)ks;
    const unsigned long long* ha = segdev + (uint64_t)jb.p * seg_stride;
    const unsigned long long* hb = segdev + (uint64_t)(P + jb.p) * seg_stride;
    SegList la{ha, ha + (kMaxSegs + 1), a_nseg[jb.p], na, jb.lo};
    SegList lb{hb, hb + (kMaxSegs + 1), b_nseg[jb.p], nbr};
    hipLaunchKernelGGL(k_pj_init, dim3(grid_for(ctx, tcap)), dim3(256), 0, ctx->compute, (uint32_t*)tmem.p, tcap,
                       (uint32_t)ks, side);
    const unsigned gb = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((na + kPjTile - 1) / kPjTile,
                                                                           (uint64_t)ctx->cu_count * 3));
    const unsigned gp = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((nbr + 1023) / 1024,
                                                                           (uint64_t)ctx->cu_count * 4));
    VX_HIP(hipEventRecord(ev[3 * j], ctx->compute));
    if (k64)
      hipLaunchKernelGGL(k_pj_build<int64_t>, dim3(gb), dim3(256), 0, ctx->compute, t, as.clu_key, pay_a, psz_a, la,
                         ctx->dev_flags, (uint32_t*)nullptr, (unsigned long long*)nullptr);
    else
      hipLaunchKernelGGL(k_pj_build<int32_t>, dim3(gb), dim3(256), 0, ctx->compute, t, as.clu_key, pay_a, psz_a, la,
                         ctx->dev_flags, (uint32_t*)nullptr, (unsigned long long*)nullptr);
    VX_HIP(hipGetLastError());
    VX_HIP(hipEventRecord(ev[3 * j + 1], ctx->compute));
    if (k64)
      hipLaunchKernelGGL(k_rj_probe<int64_t>, dim3(gp), dim3(256), 0, ctx->compute, t, bs.clu_key, pay_b, psz_b, lb,
                         acc + 3ull * jb.p);
    else
      hipLaunchKernelGGL(k_rj_probe<int32_t>, dim3(gp), dim3(256), 0, ctx->compute, t, bs.clu_key, pay_b, psz_b, lb,
                         acc + 3ull * jb.p);
    VX_HIP(hipGetLastError());
    VX_HIP(hipEventRecord(ev[3 * j + 2], ctx->compute));
    if (!as.on_device && as.key.where == Where::Host) zc_bytes += na * side_row_bytes(as);
    if (!bs.on_device && bs.key.where == Where::Host) zc_bytes += nbr * side_row_bytes(bs);
    return VX_OK;
  };
  vx_status rs = VX_OK;
  for (uint64_t j = 0; j < n_jobs && rs == VX_OK; ++j) rs = job(j);
  std::vector<unsigned long long> accs(3ull * P);
  if (rs == VX_OK) {
    const hipError_t ce = hipMemcpyAsync(accs.data(), acc, accs.size() * 8, hipMemcpyDeviceToHost, ctx->compute);
    if (ce != hipSuccess) {
      set_error("radix join: copy of the accumulators: %s", hipGetErrorString(ce));
      rs = VX_EHIP;
    }
  }
  const hipError_t se = hipStreamSynchronize(ctx->compute);
  double build_k_ms = 0, probe_k_ms = 0;
  for (uint64_t j = 0; j < n_jobs && rs == VX_OK; ++j) {
    float a = 0, b = 0;
    if (hipEventElapsedTime(&a, ev[3 * j], ev[3 * j + 1]) == hipSuccess) build_k_ms += a;
    if (hipEventElapsedTime(&b, ev[3 * j + 1], ev[3 * j + 2]) == hipSuccess) probe_k_ms += b;
  }
  for (auto e : ev) put_event(ctx, e);
  VX_TRY(rs);
  VX_HIP(se);
  VX_TRY(check_flags(ctx, "radix join"));
  const double join_ms = now_ms() - tj0;
  if (trace)
    fprintf(stderr, "[vx] radix join: %u partitions, pass 1 %.1f ms (clustered copies in %s), pass 2 %.1f ms, "
            "%llu build slices, table %llu slots\n", P, part_ms, as.on_device ? "device memory" : "host memory",
            join_ms, (unsigned long long)n_jobs, (unsigned long long)tcap_max);

  for (uint32_t p = 0; p < P; ++p) {
    out->agg.match_count += accs[3 * p];
    if (A.n_pay) out->agg.sum[0] += accs[3 * p + 1];
    if (Bd.n_pay) out->agg.sum[A.n_pay] += accs[3 * p + 2];
  }
  if (Bd.chunk_aggs) {
    VX_CHECK(Bd.chunk_aggs_cap >= P, VX_ECAPACITY, "radix join: chunk_aggs_cap %llu < %u partitions",
             (unsigned long long)Bd.chunk_aggs_cap, P);
    for (uint32_t p = 0; p < P; ++p) {
      vx_agg g;
      std::memset(&g, 0, sizeof g);
      g.match_count = accs[3 * p];
      if (A.n_pay) g.sum[0] = accs[3 * p + 1];
      if (Bd.n_pay) g.sum[A.n_pay] = accs[3 * p + 2];
      Bd.chunk_aggs[p] = g;
    }
  }
  double mx = 0, tot = 0;
  for (uint32_t p = 0; p < P; ++p) {
    mx = std::max(mx, (double)(arows[p] + brows[p]));
    tot += (double)(arows[p] + brows[p]);
  }
  s.n_parts = P;
  s.imbalance = tot > 0 ? mx / (tot / P) : 0.0;
  s.part_ms = part_ms;
  s.probe_ms = join_ms;
  s.sdma_bytes = as.sdma + bs.sdma;
  s.zc_bytes = zc_bytes;
  s.table_bytes = n_jobs ? tcap_max << kSlotShift : 0;
  s.chunks = n_jobs;
  s.chunk_rows = as.chunk_rows;
  s.kernel_launches = pass1_launches + 3 * n_jobs;
  s.build_ms = build_k_ms;
  s.kernel_ms = probe_k_ms;
  s.total_ms = now_ms() - t0;
  return VX_OK;
}

}  // namespace vx
