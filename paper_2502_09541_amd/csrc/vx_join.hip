// Hash-table build, probe with fused aggregation, and the streamed probe executor.
//
// Build: open addressing with linear probing.  A lane group of G lanes (G = 1, 4 or 8)
// inspects G consecutive slots at once; __ballot finds the first matching or empty slot
// of the window and the lowest such lane claims it with one compare-and-swap.
// Probe: one lane per probe row, several rows per lane in flight, the streamed key
// column read with non-temporal loads so the table stays in L2 / MALL.  Matches are
// aggregated in registers, reduced across the workgroup in LDS and flushed with one
// 64-bit atomic per accumulator per workgroup.  Probe payload columns are read only for
// matching rows, from the chunk buffer or by zero-copy from pinned host memory.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "vx_device.h"
#include "vx_pipeline.h"

namespace vx {

// ---------------------------------------------------------------- table init

// Every slot gets the empty-marker key and zero payloads.  The slots are written as 16-byte
// stores of four 32-bit words; a slot is 2^k >= 2 words and the capacity is >= 64, so the word
// count is a multiple of 4.  The marker is INT32_MIN in word 0 of an int32 key, and for an int64
// key (little-endian INT64_MIN) word 0 is zero and word 1 holds 0x80000000.
__global__ void k_init_slots(uint32_t* slots, uint64_t capacity, uint32_t slot_words,
                             uint32_t key_size) {
  const uint32_t key_word = key_size == 4 ? 0 : 1;
  const uint64_t quads = capacity * slot_words / 4;
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < quads;
       q += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = ((4 * q + j) & (slot_words - 1)) == key_word ? 0x80000000u : 0u;
    ((uint4*)slots)[q] = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

// ---------------------------------------------------------------- build (unique keys)

struct BuildCols {
  const void* key;
  const void* pay[kMaxPay];
  uint32_t pay_size[kMaxPay];
};

template <typename K>
__device__ __forceinline__ void write_unique_payloads(const TableView& t, uint8_t* slot,
                                                      const BuildCols& c, uint64_t row) {
  for (uint32_t p = 0; p < t.n_pay; ++p) {
    if (t.pay_size[p] == 4) *(int*)(slot + t.pay_off[p]) = ((const int*)c.pay[p])[row];
    else *(long long*)(slot + t.pay_off[p]) = ((const long long*)c.pay[p])[row];
  }
}

template <typename K>
__device__ __forceinline__ void side_add(const TableView& t, const BuildCols& c, uint64_t row,
                                         unsigned int* flags, bool unique) {
  unsigned long long prev = atomicAdd(t.side, 1ull);
  if (unique && prev != 0) atomicOr(flags, kFlagDup);
  for (uint32_t p = 0; p < t.n_pay; ++p)
    atomicAdd(t.side + 1 + p, (unsigned long long)load_signed(c.pay[p], row, c.pay_size[p]));
}

// One lane per row.
template <typename K>
__global__ void k_build_unique_lane(TableView t, BuildCols c, uint64_t n, unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    K k = ((const K*)c.key)[i];
    U kb = (U)k;
    if (kb == kEmpty) {
      side_add<K>(t, c, i, flags, true);
      continue;
    }
    uint64_t h;
    bool done = false;
    // a key outside a direct table's range cannot occur (the range is measured over these keys);
    // if it did, the table is reported full
    if (!first_slot(t, k, h)) {
      atomicOr(flags, kFlagFull);
      continue;
    }
    for (uint64_t step = 0; step <= t.mask; ++step) {
      uint8_t* slot = t.slots + (h << t.slot_shift);
      U prev = atomicCAS((U*)slot, kEmpty, kb);
      if (prev == kEmpty) {
        write_unique_payloads<K>(t, slot, c, i);
        done = true;
        break;
      }
      if (prev == kb) {
        atomicOr(flags, kFlagDup);
        done = true;
        break;
      }
      h = (h + 1) & t.mask;
    }
    if (!done) atomicOr(flags, kFlagFull);
  }
}

// Direct table: each row's slot is fixed (key - min), so key and payloads are written with plain
// stores, no compare-and-swap.  Two rows with one key write the same slot; k_direct_count then
// finds fewer filled slots than rows and raises the duplicate flag.
template <typename K>
__global__ void k_build_direct(TableView t, BuildCols c, uint64_t n, unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const K k = ((const K*)c.key)[i];
    const U kb = (U)k;
    if (kb == kEmpty) {
      side_add<K>(t, c, i, flags, true);
      continue;
    }
    uint64_t h;
    if (!first_slot(t, k, h)) {    // cannot happen: the range was measured over these keys
      atomicOr(flags, kFlagFull);
      continue;
    }
    uint8_t* slot = t.slots + (h << t.slot_shift);
    *(U*)slot = kb;
    write_unique_payloads<K>(t, slot, c, i);
  }
}

// Filled slots of a direct table's range: one atomic per workgroup into cnt[0], then a ticket in
// cnt[1].  The last workgroup to take a ticket compares the total plus the empty-marker key's rows
// (counted in the side record) with the rows inserted: they fall short exactly when two rows
// shared a key.  cnt[0..1] start at zero.
template <typename K>
__global__ void __launch_bounds__(256) k_direct_count(TableView t, unsigned long long* cnt,
                                                      uint64_t n_rows, unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  __shared__ unsigned long long part[4];
  unsigned long long c = 0;
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < t.direct_range;
       s += (uint64_t)gridDim.x * blockDim.x)
    c += *(const U*)(t.slots + (s << t.slot_shift)) != KeyTraits<K>::kEmpty;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) c += part[w];
    atomicAdd(cnt, c);
    __threadfence();
    if (atomicAdd(cnt + 1, 1ull) == gridDim.x - 1) {
      const unsigned long long total = atomicAdd(cnt, 0ull);
      if (total + atomicAdd(t.side, 0ull) != n_rows) atomicOr(flags, kFlagDup);
    }
  }
}

// Dense table: row i's payloads go to slot key - min and its key's presence byte is set, both
// with plain stores.  Every key lies in the measured range and none is the empty marker (the
// layout requires both); k_dense_count then checks that every byte of the range was set.
template <typename K>
__global__ void k_build_dense(TableView t, BuildCols c, uint64_t n, unsigned int* flags) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t h = key_ord(((const K*)c.key)[i]) - t.kmin_ord;
    if (h >= t.direct_range) {    // cannot happen: the range was measured over these keys
      atomicOr(flags, kFlagFull);
      continue;
    }
    if (t.n_pay) write_unique_payloads<K>(t, t.slots + (h << t.slot_shift), c, i);
    t.present[h] = 1;
  }
}

// Set presence bytes of a dense table (four bytes per lane per step), one atomic per workgroup
// into cnt[0], then a ticket in cnt[1]: the last workgroup compares the total with the rows
// inserted.  n rows over a range n wide set every byte exactly when no two rows share a key.
// cnt[0..1] start at zero.
__global__ void __launch_bounds__(256) k_dense_count(const uint8_t* present, uint64_t range, unsigned long long* cnt,
                                                     uint64_t n_rows, unsigned int* flags) {
  __shared__ unsigned long long part[4];
  unsigned long long c = 0;
  const uint64_t words = range / 4;
  for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < words; w += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t v = ((const uint32_t*)present)[w];   // the bytes are 0 or 1
    c += (v & 0xffu) + ((v >> 8) & 0xffu) + ((v >> 16) & 0xffu) + (v >> 24);
  }
  for (uint64_t b = words * 4 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < range;
       b += (uint64_t)gridDim.x * blockDim.x)
    c += present[b];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) c += part[w];
    atomicAdd(cnt, c);
    __threadfence();
    if (atomicAdd(cnt + 1, 1ull) == gridDim.x - 1) {
      if (atomicAdd(cnt, 0ull) != n_rows) atomicOr(flags, kFlagDup);
    }
  }
}

// A group of G lanes per row: the group loads G consecutive slots, ballots for the key
// or an empty slot, and the first empty lane claims it.  Rows of the G lanes of a group
// are handled one after the other.
template <typename K, int G>
__global__ void k_build_unique_group(TableView t, BuildCols c, uint64_t n, unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int gbase = lane - gl;
  const unsigned long long gmask = ((G == 64) ? ~0ull : ((1ull << G) - 1)) << gbase;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  // every lane of a wave runs the same number of outer iterations (ballots stay convergent)
  uint64_t first = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t wave_first = first - lane;
  for (uint64_t wb = wave_first; wb < n; wb += stride) {
    uint64_t i = wb + lane;
    bool valid = i < n;
    // every lane loads its own row (coalesced) before the group works through the rows
    K mykey = valid ? ((const K*)c.key)[i] : (K)0;
    long long mypay[kMaxPay] = {0, 0, 0, 0};
    for (uint32_t p = 0; p < t.n_pay; ++p)
      if (valid) mypay[p] = load_signed(c.pay[p], i, c.pay_size[p]);
    for (int r = 0; r < G; ++r) {
      int src = gbase + r;
      bool v = __shfl(valid ? 1 : 0, src, 64) != 0;
      if (!v) continue;                       // uniform within the group
      K k = __shfl(mykey, src, 64);
      long long pv[kMaxPay];
      for (uint32_t p = 0; p < kMaxPay; ++p) pv[p] = __shfl(mypay[p], src, 64);
      uint64_t row = wb + src;
      U kb = (U)k;
      if (kb == kEmpty) {
        if (gl == 0) side_add<K>(t, c, row, flags, true);
        continue;
      }
      uint64_t h;
      bool done = false;
      if (!first_slot(t, k, h)) {   // uniform within the group; cannot happen (see the lane build)
        if (gl == 0) atomicOr(flags, kFlagFull);
        continue;
      }
      for (uint64_t step = 0; step <= t.mask; step += G) {
        uint64_t pos = (h + gl) & t.mask;
        uint8_t* slot = t.slots + (pos << t.slot_shift);
        U sk = __atomic_load_n((U*)slot, __ATOMIC_RELAXED);
        unsigned long long hit = __ballot(sk == kb) & gmask;
        unsigned long long emp = __ballot(sk == kEmpty) & gmask;
        // the earliest event in probe order decides
        if (hit && (!emp || __ffsll((long long)hit) <= __ffsll((long long)emp))) {
          if (gl == 0) atomicOr(flags, kFlagDup);
          done = true;
          break;
        }
        if (emp) {
          int leader = __ffsll((long long)emp) - 1;
          int won = 0;
          if (lane == leader) {
            U prev = atomicCAS((U*)slot, kEmpty, kb);
            if (prev == kEmpty) {
              for (uint32_t p = 0; p < t.n_pay; ++p) {
                if (t.pay_size[p] == 4) *(int*)(slot + t.pay_off[p]) = (int)pv[p];
                else *(long long*)(slot + t.pay_off[p]) = pv[p];
              }
              won = 1;
            } else if (prev == kb) {
              atomicOr(flags, kFlagDup);
              won = 2;
            }
          }
          won = __shfl(won, leader, 64);
          if (won) {
            done = true;
            break;
          }
          step -= G;          // lost the race: re-read the same window
          continue;
        }
        h = (h + G) & t.mask;
      }
      if (!done && gl == 0) atomicOr(flags, kFlagFull);
    }
  }
}

// ---------------------------------------------------------------- build (pre-aggregated)

// Rows are first combined per workgroup tile in an LDS table (so a hot key costs one
// global update per tile), then flushed into the global table with 64-bit atomics.
constexpr int kPreaggLds = 1024;
constexpr int kPreaggTile = 4096;
constexpr int kPreaggProbe = 32;

template <typename K>
__global__ void __launch_bounds__(256) k_build_preagg(TableView t, BuildCols c, uint64_t n,
                                                      unsigned int* flags) {
  __shared__ unsigned long long lkey[kPreaggLds];
  __shared__ unsigned long long lcnt[kPreaggLds];
  __shared__ unsigned long long lsum[kMaxPay][kPreaggLds];
  const unsigned long long kFree = ~0ull;     // LDS marker; real keys are stored as 64-bit
  const unsigned long long kFreeAlt = ~0ull - 1;
  for (uint64_t base = (uint64_t)blockIdx.x * kPreaggTile; base < n;
       base += (uint64_t)gridDim.x * kPreaggTile) {
    for (int j = threadIdx.x; j < kPreaggLds; j += blockDim.x) {
      lkey[j] = kFree;
      lcnt[j] = 0;
      for (uint32_t p = 0; p < kMaxPay; ++p) lsum[p][j] = 0;
    }
    __syncthreads();
    uint64_t end = base + kPreaggTile < n ? base + kPreaggTile : n;
    for (uint64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
      K k = ((const K*)c.key)[i];
      unsigned long long kb = (unsigned long long)(long long)k;
      unsigned long long vals[kMaxPay];
      for (uint32_t p = 0; p < t.n_pay; ++p)
        vals[p] = (unsigned long long)load_signed(c.pay[p], i, c.pay_size[p]);
      bool placed = false;
      if (kb != kFree && kb != kFreeAlt) {     // those two key values bypass LDS
        uint32_t h = (uint32_t)(slot_of(kb, 10));
        for (int s = 0; s < kPreaggProbe; ++s) {
          uint32_t j = (h + s) & (kPreaggLds - 1);
          unsigned long long prev = atomicCAS(&lkey[j], kFree, kb);
          if (prev == kFree || prev == kb) {
            atomicAdd(&lcnt[j], 1ull);
            for (uint32_t p = 0; p < t.n_pay; ++p) atomicAdd(&lsum[p][j], vals[p]);
            placed = true;
            break;
          }
        }
      }
      if (!placed) global_preagg_add<K>(t, k, 1ull, vals, flags);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kPreaggLds; j += blockDim.x) {
      if (lkey[j] != kFree) {
        unsigned long long sums[kMaxPay];
        for (uint32_t p = 0; p < kMaxPay; ++p) sums[p] = lsum[p][j];
        global_preagg_add<K>(t, (K)(long long)lkey[j], lcnt[j], sums, flags);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- probe

struct ProbeCols {
  const void* key;            // keys of this launch, key[0] is global row row0
  uint64_t n;
  uint64_t row0;
  uint32_t n_pay;
  uint32_t pay_global;        // bit c: pay[c] is indexed by global row (resident / zero-copy)
  const void* pay[kMaxPay];
  uint32_t pay_size[kMaxPay];
  uint32_t zc_count;          // bit c: pay[c] is host memory read by zero-copy; count its granules
  uint32_t zc_shift;          // log2 of the zero-copy granule in bytes
  uint32_t zc_mult[kMaxPay];  // columns whose granules pay[c]'s count stands for (same width and
                              // same offset within a granule: the same granules touched)
};

// Accumulator row of one probe launch: match count, 8 sums, zero-copy granules read.
constexpr int kGranuleWord = 9;
static_assert(kGranuleWord < kAccWords, "the granule count needs its own accumulator word");

// LAYOUT: the table's layout (t.direct: hash, direct or dense), fixed at compile time so that the
// hash loop carries no test of it.
// COUNT: count the zero-copy granules of the gathers (compiled in only when asked for: the count
// slows the gather loop by about 4%).
template <typename K, bool PREAGG, int ITEMS, int LAYOUT, bool COUNT>
__global__ void __launch_bounds__(256) k_probe(TableView t, ProbeCols q, unsigned long long* acc_out) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  constexpr int NACC = kAccWords;
  unsigned long long acc[NACC];
#pragma unroll
  for (int a = 0; a < NACC; ++a) acc[a] = 0;
  const uint32_t nb = t.n_pay;
  const uint64_t tile = (uint64_t)blockDim.x * ITEMS;
  const uint64_t wave_row = threadIdx.x & ~63u;   // row of lane 0 of this wave, within a tile step
  unsigned long long granules = 0;                  // the same in every lane of a wave
  for (uint64_t base = blockIdx.x * tile; base < q.n; base += (uint64_t)gridDim.x * tile) {
    unsigned long long mb[ITEMS];
    K keys[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      keys[j] = i < q.n ? __builtin_nontemporal_load(((const K*)q.key) + i) : (K)0;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      mb[j] = 0;
      if (i >= q.n) continue;
      U kb = (U)keys[j];
      if (kb == kEmpty) {
        unsigned long long c = t.side[0];
        if (c) {
          mb[j] = c;
          acc[0] += c;
          for (uint32_t p = 0; p < nb; ++p) acc[1 + p] += t.side[1 + p];
        }
        continue;
      }
      // the layout is chosen at compile time: the hash instantiation holds no trace of the direct
      // test (a skip that only folds away after inlining still changes the loop's code)
      uint64_t h;
      if constexpr (LAYOUT == kLayoutDense) {
        // every key of the range is in the table: a key in range is a match, its slot holds
        // only the payloads
        h = key_ord(keys[j]) - t.kmin_ord;
        if (h >= t.direct_range) continue;
        const uint8_t* slot = t.slots + (h << t.slot_shift);
        mb[j] = 1;
        acc[0] += 1;
        for (uint32_t p = 0; p < nb; ++p)
          acc[1 + p] += (unsigned long long)slot_signed(slot, t.pay_off[p], t.pay_size[p]);
        continue;
      } else if constexpr (LAYOUT == kLayoutDirect) {
        h = key_ord(keys[j]) - t.kmin_ord;
        if (h >= t.direct_range) continue;   // outside the key range: no slot to read
      } else {
        h = slot_of(key_bits(keys[j]), t.log2cap);
      }
      for (uint64_t step = 0; step <= t.mask; ++step) {
        const uint8_t* slot = t.slots + (h << t.slot_shift);
        U sk = *(const U*)slot;
        if (sk == kb) {
          if (PREAGG) {
            const unsigned long long* w = (const unsigned long long*)(slot + 8);
            mb[j] = w[0];
            acc[0] += w[0];
            for (uint32_t p = 0; p < nb; ++p) acc[1 + p] += w[1 + p];
          } else {
            mb[j] = 1;
            acc[0] += 1;
            for (uint32_t p = 0; p < nb; ++p)
              acc[1 + p] += (unsigned long long)slot_signed(slot, t.pay_off[p], t.pay_size[p]);
          }
          break;
        }
        if (sk == kEmpty) break;
        h = (h + 1) & t.mask;
      }
    }
    // late materialization: probe payloads of matching rows only
    for (uint32_t p = 0; p < q.n_pay; ++p) {
      const bool glob = (q.pay_global >> p) & 1u;
      // the column's base and width, read once per column (the loads below reuse them)
      const void* const col = q.pay[p];
      const uint32_t es = q.pay_size[p];
      long long v[ITEMS];
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
        v[j] = mb[j] ? load_signed(col, glob ? q.row0 + i : i, es) : 0;
      }
      // the granules these loads move, counted while they are in flight
      if (COUNT && ((q.zc_count >> p) & 1u)) {
        const uint64_t a0 = (uint64_t)(uintptr_t)col + ((glob ? q.row0 : 0) + base + wave_row) * es;
        uint32_t g = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) g += wave_granules(mb[j] != 0, a0 + (uint64_t)j * blockDim.x * es, es, q.zc_shift);
        granules += (unsigned long long)g * q.zc_mult[p];
      }
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) acc[1 + nb + p] += mb[j] * (unsigned long long)v[j];
    }
  }
  acc[kGranuleWord] = (threadIdx.x & 63) == 0 ? granules : 0;   // once per wave
  block_flush<NACC>(acc, NACC, acc_out);
}

// Where k_probe_rows writes the join's rows (device-visible addresses: device memory or mapped
// pinned host memory), and the running count of rows.
struct RowsOut {
  unsigned long long* row;
  long long* bpay[kMaxPay];
  long long* ppay[kMaxPay];
  uint64_t cap;
  unsigned long long* count;
};

// k_probe for a unique-key table that also emits one output row per matching probe row:
// (global probe row, build payloads, probe payloads), payloads sign-extended.  A workgroup
// counts its tile's matches, reserves that many rows with one atomic, and its waves write them
// at consecutive positions (coalesced stores, to host memory beside the host-to-device copies).
template <typename K, int ITEMS, int LAYOUT>
__global__ void __launch_bounds__(256) k_probe_rows(TableView t, ProbeCols q, unsigned long long* acc_out,
                                                    RowsOut o) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  constexpr int NACC = kAccWords;
  __shared__ unsigned long long wsum[4];
  __shared__ unsigned long long tile_base;
  unsigned long long acc[NACC];
#pragma unroll
  for (int a = 0; a < NACC; ++a) acc[a] = 0;
  const uint32_t nb = t.n_pay;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t tile = (uint64_t)blockDim.x * ITEMS;
  for (uint64_t base = blockIdx.x * tile; base < q.n; base += (uint64_t)gridDim.x * tile) {
    bool hit[ITEMS];
    long long bv[ITEMS][kMaxPay], pv[ITEMS][kMaxPay];
    K keys[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      keys[j] = i < q.n ? __builtin_nontemporal_load(((const K*)q.key) + i) : (K)0;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      hit[j] = false;
      for (uint32_t p = 0; p < kMaxPay; ++p) bv[j][p] = pv[j][p] = 0;
      if (i >= q.n) continue;
      const U kb = (U)keys[j];
      if (kb == kEmpty) {
        if (t.side[0]) {
          hit[j] = true;
          for (uint32_t p = 0; p < nb; ++p) bv[j][p] = (long long)t.side[1 + p];   // the one row's payload
        }
      } else {
        uint64_t h;
        bool in_range = true;
        if constexpr (LAYOUT == kLayoutDense) {   // compile-time layout, as in k_probe
          h = key_ord(keys[j]) - t.kmin_ord;
          if (h < t.direct_range) {
            hit[j] = true;
            const uint8_t* slot = t.slots + (h << t.slot_shift);
            for (uint32_t p = 0; p < nb; ++p) bv[j][p] = slot_signed(slot, t.pay_off[p], t.pay_size[p]);
          }
          in_range = false;   // no probe loop
        } else if constexpr (LAYOUT == kLayoutDirect) {
          h = key_ord(keys[j]) - t.kmin_ord;
          in_range = h < t.direct_range;
        } else {
          h = slot_of(key_bits(keys[j]), t.log2cap);
        }
        if (in_range) {
          for (uint64_t step = 0; step <= t.mask; ++step) {
            const uint8_t* slot = t.slots + (h << t.slot_shift);
            U sk = *(const U*)slot;
            if (sk == kb) {
              hit[j] = true;
              for (uint32_t p = 0; p < nb; ++p) bv[j][p] = slot_signed(slot, t.pay_off[p], t.pay_size[p]);
              break;
            }
            if (sk == kEmpty) break;
            h = (h + 1) & t.mask;
          }
        }
      }
      if (!hit[j]) continue;
      acc[0] += 1;
      for (uint32_t p = 0; p < nb; ++p) acc[1 + p] += (unsigned long long)bv[j][p];
      // late materialization: probe payloads of matching rows only
      for (uint32_t p = 0; p < q.n_pay; ++p) {
        const bool glob = (q.pay_global >> p) & 1u;
        pv[j][p] = load_signed(q.pay[p], glob ? q.row0 + i : i, q.pay_size[p]);
        acc[1 + nb + p] += (unsigned long long)pv[j][p];
      }
    }
    // zero-copy granules of the payloads just gathered (every lane takes part)
    for (uint32_t p = 0; p < q.n_pay; ++p) {
      if (!((q.zc_count >> p) & 1u)) continue;
      const bool glob = (q.pay_global >> p) & 1u;
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const uint64_t w0 = (glob ? q.row0 : 0) + base + (uint64_t)j * blockDim.x + (threadIdx.x & ~63u);
        const uint32_t g = wave_granules(hit[j], (uint64_t)(uintptr_t)q.pay[p] + w0 * q.pay_size[p],
                                         q.pay_size[p], q.zc_shift);
        if (lane == 0) acc[kGranuleWord] += (unsigned long long)g * q.zc_mult[p];   // for each column it stands for
      }
    }
    // reserve the tile's rows: per-wave counts, one atomic per workgroup
    unsigned long long mine = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) mine += (unsigned long long)__popcll(__ballot(hit[j]));
    if (lane == 0) wsum[wave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long tot = 0;
      for (uint32_t w = 0; w < blockDim.x / 64; ++w) tot += wsum[w];
      tile_base = tot ? atomicAdd(o.count, tot) : 0ull;
    }
    __syncthreads();
    unsigned long long r0 = tile_base;
    for (uint32_t w = 0; w < wave; ++w) r0 += wsum[w];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const unsigned long long m = __ballot(hit[j]);
      if (hit[j]) {
        const uint64_t r = r0 + (uint64_t)__popcll(m & ((1ull << lane) - 1));
        if (r < o.cap) {
          o.row[r] = q.row0 + base + (uint64_t)j * blockDim.x + threadIdx.x;
          for (uint32_t p = 0; p < nb; ++p)
            if (o.bpay[p]) o.bpay[p][r] = bv[j][p];
          for (uint32_t p = 0; p < q.n_pay; ++p)
            if (o.ppay[p]) o.ppay[p][r] = pv[j][p];
        }
      }
      r0 += (unsigned long long)__popcll(m);
    }
    __syncthreads();   // wsum and tile_base are reused by the next tile
  }
  block_flush<NACC>(acc, NACC, acc_out);
}

// ---------------------------------------------------------------- key range

// Min and max of the keys' order-preserving forms, the empty-marker key left out (it lives in
// the side record, not in a slot), and the number of rows with that key.  Workgroup b writes its
// own triple to mm[3b], mm[3b + 1], mm[3b + 2] (~0, 0 and 0 when it saw no key); the host
// reduces the triples.
template <typename K>
__global__ void __launch_bounds__(256) k_key_range(const K* key, uint64_t n, unsigned long long* mm) {
  using U = typename KeyTraits<K>::U;
  __shared__ unsigned long long rmin[4], rmax[4], rempty[4];
  unsigned long long mn = ~0ull, mx = 0, empties = 0;
  auto take = [&](K k) {
    if ((U)k == KeyTraits<K>::kEmpty) {
      ++empties;
      return;
    }
    const unsigned long long o = key_ord(k);
    mn = o < mn ? o : mn;
    mx = o > mx ? o : mx;
  };
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {      // four loads in flight per lane
    const K a = __builtin_nontemporal_load(key + i), b = __builtin_nontemporal_load(key + i + stride);
    const K c = __builtin_nontemporal_load(key + i + 2 * stride), d = __builtin_nontemporal_load(key + i + 3 * stride);
    take(a);
    take(b);
    take(c);
    take(d);
  }
  for (; i < n; i += stride) take(__builtin_nontemporal_load(key + i));
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
    empties += __shfl_xor(empties, o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    rmin[wave] = mn;
    rmax[wave] = mx;
    rempty[wave] = empties;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      mn = rmin[w] < mn ? rmin[w] : mn;
      mx = rmax[w] > mx ? rmax[w] : mx;
      empties += rempty[w];
    }
    mm[3 * blockIdx.x] = mn;
    mm[3 * blockIdx.x + 1] = mx;
    mm[3 * blockIdx.x + 2] = empties;
  }
}

// ---------------------------------------------------------------- host side

static int ilog2(uint64_t v) {
  int r = 0;
  while ((1ull << r) < v) ++r;
  return r;
}

// The table's layout for `expected_rows` rows: capacity (a power of two), slot size and the view's
// fields other than its memory.  Direct when `kr` holds a measured range no wider than the hash
// capacity; dense when, besides, the build is unique, allows it, has no empty-marker key and its
// rows number exactly the range's width (the capacity is then the width itself).
static vx_status plan_table(int32_t key_type, uint32_t flags, const int32_t* pay_types, uint32_t n_pay,
                            uint64_t expected_rows, float load_factor, const KeyRange* kr, TableView* out,
                            uint64_t* cap_out, uint32_t* slot_bytes_out) {
  VX_CHECK(n_pay <= kMaxPay, VX_EINVAL, "build: at most %u payload columns", kMaxPay);
  int ks = elsize_of(key_type);
  VX_CHECK(ks != 0, VX_EINVAL, "build: bad key type %d", key_type);
  bool preagg = (flags & VX_PREAGG) != 0;
  float lf = load_factor > 0 ? load_factor : 0.5f;
  VX_CHECK(lf > 0.05f && lf <= 0.95f, VX_EINVAL, "build: load factor %f outside (0.05, 0.95]", lf);
  uint64_t want = (uint64_t)std::ceil((double)(expected_rows ? expected_rows : 1) / lf);
  uint64_t cap = 64;
  while (cap < want) cap <<= 1;
  TableView v{};
  if (kr && kr->known && kr->max_ord >= kr->min_ord && kr->max_ord - kr->min_ord < cap) {
    const uint64_t range = kr->max_ord - kr->min_ord + 1;
    uint64_t dcap = 64;
    while (dcap < range) dcap <<= 1;
    cap = dcap;
    v.direct = kLayoutDirect;
    v.kmin_ord = kr->min_ord;
    v.direct_range = range;
    if (kr->allow_dense && !preagg && kr->empty_rows == 0 && range == expected_rows) {
      v.direct = kLayoutDense;
      cap = range;
    }
  }
  v.n_pay = n_pay;
  v.preagg = preagg ? 1 : 0;
  v.key_size = (uint32_t)ks;
  uint32_t off;
  if (v.direct == kLayoutDense) {   // payloads only
    off = 0;
    for (uint32_t p = 0; p < n_pay; ++p) {
      int ps = elsize_of(pay_types[p]);
      VX_CHECK(ps != 0, VX_EINVAL, "build: bad payload type %d", pay_types[p]);
      off = (off + ps - 1) / ps * ps;
      v.pay_off[p] = off;
      v.pay_size[p] = (uint32_t)ps;
      off += ps;
    }
    uint32_t slot_bytes = off ? 4 : 0;
    while (slot_bytes && slot_bytes < off) slot_bytes <<= 1;
    v.slot_shift = slot_bytes ? (uint32_t)ilog2(slot_bytes) : 0;
    v.log2cap = (uint32_t)ilog2(cap);
    v.mask = 0;
    *out = v;
    *cap_out = cap;
    *slot_bytes_out = slot_bytes;
    return VX_OK;
  }
  if (preagg) {
    off = 16;   // key (8), count (8)
    for (uint32_t p = 0; p < n_pay; ++p) {
      v.pay_off[p] = off;
      v.pay_size[p] = 8;
      off += 8;
    }
  } else {
    off = (uint32_t)ks;
    for (uint32_t p = 0; p < n_pay; ++p) {
      int ps = elsize_of(pay_types[p]);
      VX_CHECK(ps != 0, VX_EINVAL, "build: bad payload type %d", pay_types[p]);
      off = (off + ps - 1) / ps * ps;
      v.pay_off[p] = off;
      v.pay_size[p] = (uint32_t)ps;
      off += ps;
    }
  }
  uint32_t slot_bytes = 8;
  while (slot_bytes < off) slot_bytes <<= 1;
  v.slot_shift = (uint32_t)ilog2(slot_bytes);
  v.log2cap = (uint32_t)ilog2(cap);
  v.mask = cap - 1;
  *out = v;
  *cap_out = cap;
  *slot_bytes_out = slot_bytes;
  return VX_OK;
}

vx_status make_table(vx_ctx* ctx, int32_t key_type, uint32_t flags, const int32_t* pay_types,
                     uint32_t n_pay, uint64_t expected_rows, float load_factor, vx_table** out,
                     const KeyRange* kr) {
  *out = nullptr;
  TableView v{};
  uint64_t cap = 0;
  uint32_t slot_bytes = 0;
  VX_TRY(plan_table(key_type, flags, pay_types, n_pay, expected_rows, load_factor, kr, &v, &cap, &slot_bytes));
  const int ks = (int)v.key_size;
  const bool dense = v.direct == kLayoutDense;
  // dense: the payload slots, a presence byte per key of the range, the side record; else slots
  // and side record
  const uint64_t slots_bytes = dense ? (cap * slot_bytes + 255) / 256 * 256 : cap * slot_bytes;
  const uint64_t bits_bytes = dense ? (cap + 255) / 256 * 256 : 0;   // presence bytes
  uint64_t bytes = slots_bytes + bits_bytes + 256;
  uint8_t* mem = ctx->arena.alloc(bytes);
  VX_CHECK(mem != nullptr, VX_EBUDGET,
           "build: hash table of %llu slots x %u B = %llu B does not fit the arena (%llu B free, "
           "largest block %llu B)",
           (unsigned long long)cap, slot_bytes, (unsigned long long)bytes,
           (unsigned long long)(ctx->arena.capacity() - ctx->arena.used()),
           (unsigned long long)ctx->arena.largest_free());
  v.slots = mem;
  v.present = dense ? mem + slots_bytes : nullptr;
  v.side = (unsigned long long*)(mem + slots_bytes + bits_bytes);
  vx_table* t = new vx_table;
  t->ctx = ctx;
  t->mem = mem;
  t->bytes = bytes;
  t->capacity = cap;
  t->key_type = key_type;
  t->flags = flags;
  for (uint32_t p = 0; p < n_pay; ++p) t->pay_type[p] = (uint32_t)pay_types[p];
  t->view = v;
  if (dense) {
    // every payload slot is written by the build; the presence bytes and the side record start at zero
    fill_zero((uint64_t*)v.present, (bits_bytes + 256) / 8, ctx->compute);
  } else {
    const uint64_t quads = cap * slot_bytes / 16;   // 16-byte stores of k_init_slots
    uint64_t blocks = std::min<uint64_t>((quads + 255) / 256, 8192);
    hipLaunchKernelGGL(k_init_slots, dim3((unsigned)blocks), dim3(256), 0, ctx->compute,
                       (uint32_t*)mem, cap, slot_bytes / 4, (uint32_t)ks);
    fill_zero((uint64_t*)v.side, 32, ctx->compute);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->arena.release(mem);
    delete t;
    set_error("build: init kernel launch failed: %s", hipGetErrorString(e));
    return VX_EHIP;
  }
  *out = t;
  return VX_OK;
}

vx_status check_flags(vx_ctx* ctx, const char* what) {
  unsigned int f = 0;
  VX_HIP(hipMemcpyAsync(ctx->host_small, ctx->dev_flags, sizeof f, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  std::memcpy(&f, ctx->host_small, sizeof f);
  if (f & kFlagDup) {
    set_error("%s: duplicate key in a build declared unique", what);
    return VX_EDUPKEY;
  }
  if (f & kFlagFull) {
    set_error("%s: hash table full (internal sizing error)", what);
    return VX_ECAPACITY;
  }
  if (f & kFlagGroupOverflow) {
    set_error("%s: group table overflow", what);
    return VX_ECAPACITY;
  }
  return VX_OK;
}

static unsigned grid_for(vx_ctx* ctx, uint64_t work_items, uint64_t per_block, unsigned per_cu) {
  uint64_t blocks = (work_items + per_block - 1) / per_block;
  uint64_t cap = (uint64_t)ctx->cu_count * per_cu;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

vx_status key_range(vx_ctx* ctx, int32_t key_type, const void* dev_keys, uint64_t n, KeyRange* out) {
  *out = KeyRange{};
  if (n == 0) return VX_OK;
  unsigned long long* mm = (unsigned long long*)ctx->dev_acc;   // free between executor steps
  const unsigned g = grid_for(ctx, n, 256 * 16, 2);
  VX_CHECK(3ull * g <= ctx->dev_acc_words, VX_EINVAL, "key range: %u workgroups exceed the scratch", g);
  if (key_type == VX_I64)
    hipLaunchKernelGGL(k_key_range<int64_t>, dim3(g), dim3(256), 0, ctx->compute, (const int64_t*)dev_keys, n, mm);
  else
    hipLaunchKernelGGL(k_key_range<int32_t>, dim3(g), dim3(256), 0, ctx->compute, (const int32_t*)dev_keys, n, mm);
  VX_HIP(hipGetLastError());
  const unsigned long long* h = (const unsigned long long*)ctx->host_acc;   // pinned: a direct copy
  VX_HIP(hipMemcpyAsync(ctx->host_acc, mm, 3 * (uint64_t)g * 8, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  unsigned long long mn = ~0ull, mx = 0, empties = 0;
  for (unsigned b = 0; b < g; ++b) {
    mn = std::min(mn, h[3 * b]);
    mx = std::max(mx, h[3 * b + 1]);
    empties += h[3 * b + 2];
  }
  out->empty_rows = empties;
  if (mn <= mx) {      // at least one key besides the empty marker
    out->known = true;
    out->min_ord = mn;
    out->max_ord = mx;
  }
  return VX_OK;
}

vx_status table_insert(vx_ctx* ctx, vx_table* t, const ColInfo& key, const ColInfo* pays,
                       uint64_t n, hipStream_t s, int group_lanes) {
  if (n == 0) return VX_OK;
  BuildCols c{};
  c.key = key.dev;
  for (uint32_t p = 0; p < t->view.n_pay; ++p) {
    c.pay[p] = pays[p].dev;
    c.pay_size[p] = (uint32_t)pays[p].elsize;
  }
  const bool k64 = t->key_type == VX_I64;
  if (t->view.preagg) {
    unsigned g = grid_for(ctx, n, kPreaggTile, 3);
    if (k64) hipLaunchKernelGGL(k_build_preagg<int64_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
    else hipLaunchKernelGGL(k_build_preagg<int32_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
  } else if (t->view.direct == kLayoutDense) {
    VX_CHECK(t->n_rows == 0, VX_EINVAL, "build: a dense table takes its rows in one insert");
    unsigned long long* cnt = (unsigned long long*)ctx->dev_acc;
    fill_zero((uint64_t*)cnt, 2, s);
    const unsigned g = grid_for(ctx, n, 256, 8);
    const unsigned gc = grid_for(ctx, t->view.direct_range, 256 * 16, 2);
    if (k64) hipLaunchKernelGGL(k_build_dense<int64_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
    else hipLaunchKernelGGL(k_build_dense<int32_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
    hipLaunchKernelGGL(k_dense_count, dim3(gc), dim3(256), 0, s, (const uint8_t*)t->view.present, t->view.direct_range,
                       cnt, n, ctx->dev_flags);
  } else if (t->view.direct) {
    // one insert per direct table: the duplicate check counts every slot against every row
    VX_CHECK(t->n_rows == 0, VX_EINVAL, "build: a direct table takes its rows in one insert");
    unsigned long long* cnt = (unsigned long long*)ctx->dev_acc;
    fill_zero((uint64_t*)cnt, 2, s);
    const unsigned g = grid_for(ctx, n, 256, 8);
    const unsigned gc = grid_for(ctx, t->view.direct_range, 256 * 16, 2);
    if (k64) {
      hipLaunchKernelGGL(k_build_direct<int64_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
      hipLaunchKernelGGL(k_direct_count<int64_t>, dim3(gc), dim3(256), 0, s, t->view, cnt, n, ctx->dev_flags);
    } else {
      hipLaunchKernelGGL(k_build_direct<int32_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
      hipLaunchKernelGGL(k_direct_count<int32_t>, dim3(gc), dim3(256), 0, s, t->view, cnt, n, ctx->dev_flags);
    }
  } else {
    unsigned g = grid_for(ctx, n, 256, 8);
    switch (group_lanes) {
      case 1:
        if (k64) hipLaunchKernelGGL(k_build_unique_lane<int64_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        else hipLaunchKernelGGL(k_build_unique_lane<int32_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        break;
      case 4:
        if (k64) hipLaunchKernelGGL((k_build_unique_group<int64_t, 4>), dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        else hipLaunchKernelGGL((k_build_unique_group<int32_t, 4>), dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        break;
      default:
        if (k64) hipLaunchKernelGGL((k_build_unique_group<int64_t, 8>), dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        else hipLaunchKernelGGL((k_build_unique_group<int32_t, 8>), dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        break;
    }
  }
  VX_HIP(hipGetLastError());
  t->n_rows += n;
  return VX_OK;
}

// Launch one probe kernel over q.n rows, accumulating into acc (kAccWords words).
// rows per lane of the dense-table probe (VX_PROBE_ITEMS = 4, 8 or 16; default 16): its loads have
// no dependent chain, so more rows per lane put more of them in flight (in-memory join, one box:
// 80.7 / 86.4 / 73.8 us per 2^24-row launch)
static int dense_items() {
  const char* e = getenv("VX_PROBE_ITEMS");
  const int v = e ? atoi(e) : 16;
  return v == 4 || v == 8 ? v : 16;
}

template <typename K, int LAYOUT, bool COUNT>
static void launch_probe_count(const vx_table* t, const ProbeCols& q, unsigned long long* acc, hipStream_t s,
                               unsigned g) {
  constexpr int ITEMS = 4;
  if constexpr (LAYOUT == kLayoutDense) {   // dense tables hold unique keys
    switch (dense_items()) {
      case 16:
        hipLaunchKernelGGL((k_probe<K, false, 16, LAYOUT, COUNT>), dim3(g), dim3(256), 0, s, t->view, q, acc);
        break;
      case 4:
        hipLaunchKernelGGL((k_probe<K, false, 4, LAYOUT, COUNT>), dim3(g), dim3(256), 0, s, t->view, q, acc);
        break;
      default:
        hipLaunchKernelGGL((k_probe<K, false, 8, LAYOUT, COUNT>), dim3(g), dim3(256), 0, s, t->view, q, acc);
        break;
    }
  }
  else if (t->view.preagg)
    hipLaunchKernelGGL((k_probe<K, true, ITEMS, LAYOUT, COUNT>), dim3(g), dim3(256), 0, s, t->view, q, acc);
  else
    hipLaunchKernelGGL((k_probe<K, false, ITEMS, LAYOUT, COUNT>), dim3(g), dim3(256), 0, s, t->view, q, acc);
}

template <typename K, int LAYOUT>
static void launch_probe_as(const vx_table* t, const ProbeCols& q, unsigned long long* acc, hipStream_t s,
                            const RowsOut* ro, unsigned g) {
  if (ro)
    hipLaunchKernelGGL((k_probe_rows<K, 4, LAYOUT>), dim3(g), dim3(256), 0, s, t->view, q, acc, *ro);
  else if (q.zc_count)
    launch_probe_count<K, LAYOUT, true>(t, q, acc, s, g);
  else
    launch_probe_count<K, LAYOUT, false>(t, q, acc, s, g);
}

static vx_status launch_probe(vx_ctx* ctx, const vx_table* t, const ProbeCols& q,
                              unsigned long long* acc, hipStream_t s, const RowsOut* ro = nullptr) {
  if (q.n == 0) return VX_OK;
  const unsigned g = grid_for(ctx, q.n, 256 * 4, 8);
  const bool k64 = t->key_type == VX_I64;
  switch (t->view.direct) {
    case kLayoutDense:
      if (k64) launch_probe_as<int64_t, kLayoutDense>(t, q, acc, s, ro, g);
      else launch_probe_as<int32_t, kLayoutDense>(t, q, acc, s, ro, g);
      break;
    case kLayoutDirect:
      if (k64) launch_probe_as<int64_t, kLayoutDirect>(t, q, acc, s, ro, g);
      else launch_probe_as<int32_t, kLayoutDirect>(t, q, acc, s, ro, g);
      break;
    default:
      if (k64) launch_probe_as<int64_t, kLayoutHash>(t, q, acc, s, ro, g);
      else launch_probe_as<int32_t, kLayoutHash>(t, q, acc, s, ro, g);
      break;
  }
  VX_HIP(hipGetLastError());
  return VX_OK;
}

int build_group_lanes() {
  const char* e = getenv("VX_BUILD_LANES");
  int g = e ? atoi(e) : 8;
  return (g == 1 || g == 4 || g == 8) ? g : 8;
}

// ---------------------------------------------------------------- streamed probe executor

// Per probe payload column: read by zero-copy (true) or streamed with the keys (false),
// given the selectivity measured on the first chunk.
static bool choose_zero_copy(int32_t late_mat, double sel, uint64_t rows, uint64_t matches, int es,
                             uint32_t line) {
  if (late_mat == VX_LATE_PAPER) return sel < (double)es / (double)line;  // TH = E/(C_l2 * 1)
  double wire = zc_wire_bytes(rows, std::min(matches, rows), es, line) / (double)std::max<uint64_t>(rows, 1);
  return wire < 0.95 * es;
}

// check_build: the table's build left its error flags unread (build_impl's defer_check); they
// are read back with the results and turned into the build's error.
vx_status probe_impl(vx_ctx* ctx, const vx_table* t, const vx_probe_desc* d, vx_agg* out,
                     vx_stats* st, vx_join_rows* rows, bool check_build = false) {
  double t0 = now_ms();
  VX_CHECK(d->key.type == t->key_type, VX_EINVAL, "probe: key type %d differs from the table's %d",
           d->key.type, t->key_type);
  VX_CHECK(d->n_pay <= kMaxPay, VX_EINVAL, "probe: at most %u payload columns", kMaxPay);
  VX_CHECK(d->n_pay == 0 || d->pay != nullptr, VX_EINVAL, "probe: pay is NULL");
  VX_CHECK(t->view.n_pay + d->n_pay <= 8, VX_EINVAL, "probe: more than 8 aggregate sums");
  VX_CHECK(d->late_mat >= -1 && d->late_mat <= 2, VX_EINVAL, "probe: late_mat %d", d->late_mat);
  VX_CHECK((d->flags & ~(uint32_t)VX_PROBE_COUNT_ZC) == 0, VX_EINVAL, "probe: unknown flags %u", d->flags);
  std::vector<PipeCol> cols(1 + d->n_pay);
  VX_TRY(classify(ctx, d->key, d->n, &cols[0].info, "probe key"));
  cols[0].may_copy = cols[0].copy = true;
  for (uint32_t p = 0; p < d->n_pay; ++p) {
    VX_TRY(classify(ctx, d->pay[p], d->n, &cols[1 + p].info, "probe payload"));
    cols[1 + p].may_copy = d->late_mat != VX_LATE_ZC;
    cols[1 + p].copy = d->late_mat == VX_LATE_SDMA;
  }
  VX_HIP(hipSetDevice(ctx->device));
  const uint64_t n = d->n;
  const uint32_t nacc = 1 + t->view.n_pay + d->n_pay;
  vx_stats s{};
  s.rows = n;
  s.table_bytes = t->bytes;

  Pipeline pipe;
  VX_CHECK(d->n_buffers == 0 || (d->n_buffers >= 2 && d->n_buffers <= 4), VX_EINVAL,
           "probe: n_buffers %u outside 2..4", d->n_buffers);
  VX_TRY(pipe.plan(ctx, n, d->chunk_rows, d->n_buffers, cols));
  const uint64_t n_chunks = pipe.n_chunks();
  const uint64_t acc_rows_cap = ctx->dev_acc_words / kAccWords;
  const uint64_t acc_rows = std::min<uint64_t>(std::max<uint64_t>(n_chunks, 1), acc_rows_cap);
  if (d->chunk_aggs)
    VX_CHECK(n_chunks <= d->chunk_aggs_cap && n_chunks <= acc_rows_cap, VX_ECAPACITY,
             "probe: %llu chunks exceed chunk_aggs_cap %llu", (unsigned long long)n_chunks,
             (unsigned long long)d->chunk_aggs_cap);
  fill_zero((uint64_t*)ctx->dev_acc, acc_rows * kAccWords, ctx->compute);

  // output rows (vx_probe_rows): device-visible addresses of the caller's columns and a counter
  RowsOut ro{};
  ArenaBlock counter;
  if (rows) {
    VX_CHECK(!t->view.preagg, VX_EUNSUPPORTED, "probe rows: the table must have unique keys");
    VX_CHECK(rows->row != nullptr, VX_EINVAL, "probe rows: the row column is NULL");
    ColInfo ci;
    VX_TRY(classify(ctx, vx_col{rows->row, VX_I64, 0}, rows->cap, &ci, "probe rows: row column"));
    ro.row = (unsigned long long*)ci.dev;
    for (uint32_t p = 0; p < t->view.n_pay; ++p)
      if (rows->build_pay[p]) {
        VX_TRY(classify(ctx, vx_col{rows->build_pay[p], VX_I64, 0}, rows->cap, &ci, "probe rows: build payload"));
        ro.bpay[p] = (long long*)ci.dev;
      }
    for (uint32_t p = 0; p < d->n_pay; ++p)
      if (rows->probe_pay[p]) {
        VX_TRY(classify(ctx, vx_col{rows->probe_pay[p], VX_I64, 0}, rows->cap, &ci, "probe rows: probe payload"));
        ro.ppay[p] = (long long*)ci.dev;
      }
    ro.cap = rows->cap;
    counter.a = &ctx->arena;
    counter.p = ctx->arena.alloc(256);
    VX_CHECK(counter.p, VX_EBUDGET, "probe rows: no room for the row counter");
    ro.count = (unsigned long long*)counter.p;
    fill_zero((uint64_t*)ro.count, 1, ctx->compute);
    rows->n_out = 0;
  }

  uint32_t zc_shift = 0;
  while ((2u << zc_shift) <= ctx->zc_line) ++zc_shift;   // log2 of the measured granule
  const bool count_zc = (d->flags & VX_PROBE_COUNT_ZC) != 0;
  auto kernel = [&](const ChunkView& v) -> vx_status {
    ProbeCols q{};
    q.key = v.ptr[0];
    if ((v.global_mask & 1u)) q.key = (const uint8_t*)v.ptr[0] + v.row0 * (uint64_t)cols[0].info.elsize;
    q.n = v.rows;
    q.row0 = v.row0;
    q.n_pay = d->n_pay;
    for (uint32_t p = 0; p < d->n_pay; ++p) {
      q.pay[p] = v.ptr[1 + p];
      q.pay_size[p] = (uint32_t)cols[1 + p].info.elsize;
      if ((v.global_mask >> (1 + p)) & 1u) {
        q.pay_global |= 1u << p;
        if (count_zc && cols[1 + p].info.where == Where::Host) {   // read in place: count its granules, once
          // per group of columns with one width and one offset within a granule
          const uint64_t off = (uint64_t)(uintptr_t)q.pay[p] & (((uint64_t)1 << zc_shift) - 1);
          uint32_t rep = p;
          for (uint32_t o = 0; o < p; ++o)
            if (((q.zc_count >> o) & 1u) && q.pay_size[o] == q.pay_size[p] &&
                ((uint64_t)(uintptr_t)q.pay[o] & (((uint64_t)1 << zc_shift) - 1)) == off)
              rep = o;
          if (rep == p) q.zc_count |= 1u << p;
          q.zc_mult[rep] += 1;
        }
      }
    }
    q.zc_shift = zc_shift;
    return launch_probe(ctx, t, q, (unsigned long long*)ctx->dev_acc + (v.index % acc_rows) * kAccWords,
                        ctx->compute, rows ? &ro : nullptr);
  };
  Pipeline::DecideFn decide = nullptr;
  bool any_host_pay = false;
  for (uint32_t p = 0; p < d->n_pay; ++p) any_host_pay |= cols[1 + p].info.where == Where::Host;
  if ((d->late_mat == VX_LATE_AUTO || d->late_mat == VX_LATE_PAPER) && any_host_pay) {
    decide = [&](std::vector<PipeCol>& cs) -> vx_status {
      unsigned long long first[kAccWords];
      VX_HIP(hipMemcpy(first, ctx->dev_acc, sizeof first, hipMemcpyDeviceToHost));
      uint64_t rows0 = std::min(pipe.chunk_rows(), n);
      double sel = rows0 ? (double)first[0] / (double)rows0 : 0.0;
      for (uint32_t p = 0; p < d->n_pay; ++p)
        if (cs[1 + p].may_copy)
          cs[1 + p].copy = !choose_zero_copy(d->late_mat, sel, rows0, first[0], cs[1 + p].info.elsize,
                                             ctx->zc_line);
      return VX_OK;
    };
  }
  double tk0 = now_ms();
  vx_status status = pipe.run(kernel, decide);
  if (status != VX_OK) return status;   // the pipeline's destructor drains both streams
  VX_HIP(hipMemcpyAsync(ctx->host_acc, ctx->dev_acc, acc_rows * kAccWords * 8, hipMemcpyDeviceToHost,
                        ctx->compute));
  if (rows) VX_HIP(hipMemcpyAsync(&rows->n_out, ro.count, 8, hipMemcpyDeviceToHost, ctx->compute));
  if (check_build)
    VX_HIP(hipMemcpyAsync(ctx->host_small, ctx->dev_flags, 4, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  unsigned int build_flags = 0;
  if (check_build) std::memcpy(&build_flags, ctx->host_small, 4);
  VX_CHECK(!(build_flags & kFlagDup), VX_EDUPKEY, "vx_join_agg: duplicate key in a build declared unique");
  VX_CHECK(!(build_flags & kFlagFull), VX_ECAPACITY, "vx_join_agg: hash table full (internal sizing error)");
  double tk1 = now_ms();
  std::vector<unsigned long long> total(kAccWords, 0);
  for (uint64_t r = 0; r < acc_rows; ++r)
    for (int a = 0; a < kAccWords; ++a) total[a] += ctx->host_acc[r * kAccWords + a];
  if (d->chunk_aggs) {
    for (uint64_t c = 0; c < n_chunks; ++c) {
      vx_agg& ca = d->chunk_aggs[c];
      std::memset(&ca, 0, sizeof ca);
      ca.match_count = ctx->host_acc[c * kAccWords];
      for (uint32_t a = 1; a < nacc; ++a) ca.sum[a - 1] = ctx->host_acc[c * kAccWords + a];
    }
  }
  std::memset(out, 0, sizeof *out);
  out->match_count = total[0];
  for (uint32_t a = 1; a < nacc; ++a) out->sum[a - 1] = total[a];
  uint32_t zc_mask = 0;
  for (uint32_t p = 0; p < d->n_pay; ++p) {
    const PipeCol& c = pipe.cols()[1 + p];
    if (c.info.where != Where::Host || c.copy) continue;
    zc_mask |= 1u << p;
    if (count_zc) continue;
    // not counted: the wire model's estimate from the per-chunk match counts
    for (uint64_t k = 0; k < n_chunks; ++k) {
      const uint64_t crows = std::min(pipe.chunk_rows(), n - k * pipe.chunk_rows());
      const uint64_t m = k < acc_rows ? ctx->host_acc[k * kAccWords] : 0;
      s.zc_bytes += (uint64_t)zc_wire_bytes(crows, std::min(m, crows), c.info.elsize, ctx->zc_line);
    }
  }
  // counted: the granules the probe kernels counted, times the granule
  if (count_zc) s.zc_bytes = total[kGranuleWord] << zc_shift;
  s.zc_counted = count_zc && zc_mask ? 1u : 0u;
  s.zc_mask = zc_mask;
  s.chunk_rows = pipe.chunk_rows();
  s.chunks = pipe.streamed() ? n_chunks : 0;
  s.n_buffers = pipe.streamed() ? pipe.n_buffers() : 0;
  s.sdma_bytes = pipe.sdma_bytes();
  s.kernel_ms = pipe.kernel_ms();
  s.kernel_launches = pipe.kernel_launches();
  s.probe_ms = tk1 - tk0;
  s.total_ms = now_ms() - t0;
  if (st) *st = s;
  VX_CHECK(!rows || rows->n_out <= rows->cap, VX_ECAPACITY,
           "probe rows: %llu output rows exceed cap %llu (n_out holds the count)",
           (unsigned long long)rows->n_out, (unsigned long long)rows->cap);
  return VX_OK;
}

// defer_check: leave the build's error flags for the caller to read with its own results (one
// host round trip less); the table is returned even if they will show a repeated key.
vx_status build_impl(vx_ctx* ctx, const vx_build_desc* d, vx_table** out, double* ms, bool defer_check) {
  double t0 = now_ms();
  VX_CHECK(d != nullptr && out != nullptr, VX_EINVAL, "vx_build: null argument");
  *out = nullptr;
  const uint32_t kind = d->flags & ~(uint32_t)VX_HASHED;
  VX_CHECK(kind == VX_UNIQUE || kind == VX_PREAGG, VX_EINVAL,
           "vx_build: flags must be VX_UNIQUE or VX_PREAGG, optionally with VX_HASHED");
  VX_CHECK(d->n_pay <= kMaxPay, VX_EINVAL, "vx_build: at most %u payload columns", kMaxPay);
  VX_CHECK(d->n_pay == 0 || d->pay != nullptr, VX_EINVAL, "vx_build: pay is NULL");
  ColInfo kc;
  VX_TRY(classify(ctx, d->key, d->n, &kc, "build key"));
  ColInfo pc[kMaxPay];
  int32_t pt[kMaxPay];
  for (uint32_t p = 0; p < d->n_pay; ++p) {
    VX_TRY(classify(ctx, d->pay[p], d->n, &pc[p], "build payload"));
    pt[p] = d->pay[p].type;
  }
  VX_HIP(hipSetDevice(ctx->device));
  // Device-resident keys are measured first: keys that fill a range no wider than the hash
  // table get a direct table.  Host-resident keys are not (the pass would cross the host link).
  KeyRange kr;
  if (!(d->flags & VX_HASHED) && kc.where == Where::Device)
    VX_TRY(key_range(ctx, d->key.type, kc.dev, d->n, &kr));
  kr.allow_dense = kind == VX_UNIQUE;
  vx_table* t = nullptr;
  VX_TRY(make_table(ctx, d->key.type, kind, pt, d->n_pay, d->n, d->load_factor, &t, &kr));
  fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);
  vx_status st = table_insert(ctx, t, kc, pc, d->n, ctx->compute, build_group_lanes());
  if (st == VX_OK && !defer_check) st = check_flags(ctx, "vx_build");
  if (st != VX_OK) {
    ctx->arena.release(t->mem);
    delete t;
    return st;
  }
  *out = t;
  if (ms) *ms = now_ms() - t0;
  return VX_OK;
}

vx_status join_star(vx_ctx* ctx, const vx_star_join* d, vx_join_out* out);
vx_status join_batch(vx_ctx* ctx, const vx_batch_join* d, vx_join_out* out);
vx_status join_partitioned(vx_ctx* ctx, const vx_partitioned_join* d, vx_join_out* out);
vx_status join_radix(vx_ctx* ctx, const vx_radix_join* d, vx_join_out* out);

}  // namespace vx

using namespace vx;

extern "C" {

vx_status vx_build(vx_ctx* ctx, const vx_build_desc* d, vx_table** out) {
  VX_CHECK(ctx != nullptr, VX_EINVAL, "vx_build: ctx is NULL");
  release_cached(ctx);
  return build_impl(ctx, d, out, nullptr, false);
}

vx_status vx_table_destroy(vx_table* t) {
  if (!t) return VX_OK;
  (void)hipStreamSynchronize(t->ctx->compute);
  t->ctx->arena.release(t->mem);
  delete t;
  return VX_OK;
}

vx_status vx_probe_stream(vx_ctx* ctx, const vx_table* t, const vx_probe_desc* d, vx_agg* out,
                          vx_stats* st) {
  VX_CHECK(ctx && t && d && out, VX_EINVAL, "vx_probe_stream: null argument");
  VX_CHECK(t->ctx == ctx, VX_EINVAL, "vx_probe_stream: table belongs to another context");
  release_cached(ctx);
  return probe_impl(ctx, t, d, out, st, nullptr);
}

vx_status vx_probe_rows(vx_ctx* ctx, const vx_table* t, const vx_probe_desc* d, vx_join_rows* rows,
                        vx_agg* out, vx_stats* st) {
  VX_CHECK(ctx && t && d && rows && out, VX_EINVAL, "vx_probe_rows: null argument");
  VX_CHECK(t->ctx == ctx, VX_EINVAL, "vx_probe_rows: table belongs to another context");
  release_cached(ctx);
  return probe_impl(ctx, t, d, out, st, rows);
}

vx_status vx_join_agg(vx_ctx* ctx, const vx_join_desc* d, vx_join_out* out) {
  VX_CHECK(ctx && d && out, VX_EINVAL, "vx_join_agg: null argument");
  std::memset(out, 0, sizeof *out);
  // only the graph-mode batch reuses what an earlier batch call left in the arena
  if (!(d->kind == VX_JOIN_BATCH && d->u.batch.mode == 0)) release_cached(ctx);
  switch (d->kind) {
    case VX_JOIN_PLAIN: {
      double t0 = now_ms(), bms = 0;
      vx_table* t = nullptr;
      // the build's flags are read with the probe's results: one host round trip for both
      VX_TRY(build_impl(ctx, &d->u.plain.build, &t, &bms, true));
      vx_status st = probe_impl(ctx, t, &d->u.plain.probe, &out->agg, &out->stats, nullptr, true);
      vx_table_destroy(t);
      out->stats.build_ms = bms;
      out->stats.total_ms = now_ms() - t0;
      return st;
    }
    case VX_JOIN_STAR: return join_star(ctx, &d->u.star, out);
    case VX_JOIN_BATCH: return join_batch(ctx, &d->u.batch, out);
    case VX_JOIN_PARTITIONED: return join_partitioned(ctx, &d->u.part, out);
    case VX_JOIN_RADIX: return join_radix(ctx, &d->u.radix, out);
    default: break;
  }
  set_error("vx_join_agg: unknown kind %d", d->kind);
  return VX_EINVAL;
}

}  // extern "C"

// ================================================================ no-allocation entry point

namespace vx {

// The device memory of vx_join_plain_noalloc: a fixed array of the library.  Every GPU the library
// runs on holds its own copy until the process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns with that device current: on the host the array's name is a stand-in,
// not a device address.  Layout: [0, 256) the table's side record, [256, end) its slots.
static __device__ __align__(256) uint8_t scratch[VX_NOALLOC_SCRATCH_BYTES];
constexpr uint64_t kNaSlotsOff = 256;
constexpr int kNaMaxDevices = 64;

struct NoAllocDevice {
  std::once_flag once;
  uint8_t* ptr = nullptr;   // device address of `scratch` on this GPU
  int cu_count = 0;
  hipError_t err = hipSuccess;
};
static NoAllocDevice g_noalloc[kNaMaxDevices];

// Once per device, with that device current: the array's address there, and the CU count.
static vx_status noalloc_setup(int dev, NoAllocDevice** out) {
  VX_CHECK(dev >= 0 && dev < kNaMaxDevices, VX_EINVAL, "vx_join_plain_noalloc: device %d", dev);
  NoAllocDevice& d = g_noalloc[dev];
  std::call_once(d.once, [&d, dev]() {
    void* p = nullptr;
    d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (d.err == hipSuccess) d.err = hipDeviceGetAttribute(&d.cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    d.ptr = (uint8_t*)p;
  });
  if (d.err != hipSuccess || d.ptr == nullptr || d.cu_count <= 0) {
    set_error("vx_join_plain_noalloc: no address for the scratch array on device %d (%s)", dev,
              hipGetErrorString(d.err));
    return VX_EHIP;
  }
  *out = &d;
  return VX_OK;
}

// `p` points to device memory of device `dev` (any pointer when bytes == 0).
static vx_status noalloc_device_ptr(const void* p, uint64_t bytes, int dev, const char* what) {
  if (bytes == 0) return VX_OK;
  VX_CHECK(p != nullptr, VX_EINVAL, "vx_join_plain_noalloc: %s is NULL", what);
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof a);
  const hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess || a.type != hipMemoryTypeDevice || a.device != dev) {
    (void)hipGetLastError();
    set_error("vx_join_plain_noalloc: %s must be device memory of device %d", what, dev);
    return VX_EINVAL;
  }
  return VX_OK;
}

static unsigned grid_cu(int cu, uint64_t work_items, uint64_t per_block, unsigned per_cu) {
  uint64_t blocks = (work_items + per_block - 1) / per_block;
  blocks = std::min<uint64_t>(blocks, (uint64_t)cu * per_cu);
  return (unsigned)std::max<uint64_t>(blocks, 1);
}

template <typename K>
static void noalloc_launch(const TableView& v, uint64_t cap, uint32_t slot_bytes, const BuildCols& bc, uint64_t nb,
                           const ProbeCols& q, int cu, unsigned long long* out, hipStream_t s) {
  unsigned int* flags = (unsigned int*)(out + 9);
  const uint64_t quads = cap * slot_bytes / 16;
  hipLaunchKernelGGL(k_init_slots, dim3(grid_cu(cu, quads, 256, 32)), dim3(256), 0, s, (uint32_t*)v.slots, cap,
                     slot_bytes / 4, (uint32_t)sizeof(K));
  if (nb) {
    if (v.preagg)
      hipLaunchKernelGGL(k_build_preagg<K>, dim3(grid_cu(cu, nb, kPreaggTile, 3)), dim3(256), 0, s, v, bc, nb, flags);
    else
      hipLaunchKernelGGL((k_build_unique_group<K, 8>), dim3(grid_cu(cu, nb, 256, 8)), dim3(256), 0, s, v, bc, nb,
                         flags);
  }
  if (q.n) {
    if (v.preagg)
      hipLaunchKernelGGL((k_probe<K, true, 4, kLayoutHash, false>), dim3(grid_cu(cu, q.n, 1024, 8)), dim3(256), 0, s, v, q, out);
    else
      hipLaunchKernelGGL((k_probe<K, false, 4, kLayoutHash, false>), dim3(grid_cu(cu, q.n, 1024, 8)), dim3(256), 0, s, v, q, out);
  }
}

}  // namespace vx

extern "C" vx_status vx_join_plain_noalloc(const vx_build_desc* b, const vx_probe_desc* p, void* stream,
                                           uint64_t* out) {
  using namespace vx;
  VX_CHECK(b && p && out, VX_EINVAL, "vx_join_plain_noalloc: null argument");
  const uint32_t kind = b->flags & ~(uint32_t)VX_HASHED;
  VX_CHECK(kind == VX_UNIQUE || kind == VX_PREAGG, VX_EINVAL,
           "vx_join_plain_noalloc: flags must be VX_UNIQUE or VX_PREAGG, optionally with VX_HASHED");
  VX_CHECK(b->n_pay <= kMaxPay && p->n_pay <= kMaxPay && b->n_pay + p->n_pay <= 8, VX_EINVAL,
           "vx_join_plain_noalloc: at most 4 payloads per side and 8 sums");
  VX_CHECK((b->n_pay == 0 || b->pay) && (p->n_pay == 0 || p->pay), VX_EINVAL, "vx_join_plain_noalloc: pay is NULL");
  VX_CHECK(b->key.type == p->key.type, VX_EINVAL, "vx_join_plain_noalloc: key types differ");
  const int ks = elsize_of(b->key.type);
  VX_CHECK(ks != 0, VX_EINVAL, "vx_join_plain_noalloc: key type %d is not VX_I32/VX_I64", b->key.type);
  int dev = 0;
  VX_HIP(hipGetDevice(&dev));
  NoAllocDevice* nd = nullptr;
  VX_TRY(noalloc_setup(dev, &nd));
  VX_TRY(noalloc_device_ptr(out, 1, dev, "out"));
  VX_TRY(noalloc_device_ptr(b->key.data, b->n, dev, "build key"));
  VX_TRY(noalloc_device_ptr(p->key.data, p->n, dev, "probe key"));
  BuildCols bc{};
  bc.key = b->key.data;
  int32_t pt[kMaxPay] = {0, 0, 0, 0};
  for (uint32_t c = 0; c < b->n_pay; ++c) {
    const int es = elsize_of(b->pay[c].type);
    VX_CHECK(es != 0, VX_EINVAL, "vx_join_plain_noalloc: build payload %u type %d", c, b->pay[c].type);
    VX_TRY(noalloc_device_ptr(b->pay[c].data, b->n, dev, "build payload"));
    pt[c] = b->pay[c].type;
    bc.pay[c] = b->pay[c].data;
    bc.pay_size[c] = (uint32_t)es;
  }
  ProbeCols q{};
  q.key = p->key.data;
  q.n = p->n;
  q.n_pay = p->n_pay;
  for (uint32_t c = 0; c < p->n_pay; ++c) {
    const int es = elsize_of(p->pay[c].type);
    VX_CHECK(es != 0, VX_EINVAL, "vx_join_plain_noalloc: probe payload %u type %d", c, p->pay[c].type);
    VX_TRY(noalloc_device_ptr(p->pay[c].data, p->n, dev, "probe payload"));
    q.pay[c] = p->pay[c].data;
    q.pay_size[c] = (uint32_t)es;
  }
  // a hash table (the direct layout would need the keys' range read back first)
  TableView v{};
  uint64_t cap = 0;
  uint32_t slot_bytes = 0;
  VX_TRY(plan_table(b->key.type, kind, pt, b->n_pay, b->n, b->load_factor, nullptr, &v, &cap, &slot_bytes));
  const uint64_t limit = VX_NOALLOC_SCRATCH_BYTES - kNaSlotsOff;
  VX_CHECK(cap * slot_bytes <= limit, VX_EBUDGET,
           "vx_join_plain_noalloc: %llu build rows need a table of %llu slots x %u B = %llu B; the fixed scratch "
           "array holds %llu B of slots",
           (unsigned long long)b->n, (unsigned long long)cap, slot_bytes, (unsigned long long)(cap * slot_bytes),
           (unsigned long long)limit);
  v.side = (unsigned long long*)nd->ptr;
  v.slots = nd->ptr + kNaSlotsOff;
  const hipStream_t s = (hipStream_t)stream;
  // the aggregate row, the error word and the side record start at zero (fill kernels, no memset)
  fill_zero(out, 10, s);
  fill_zero((uint64_t*)nd->ptr, kNaSlotsOff / 8, s);
  if (ks == 8) noalloc_launch<int64_t>(v, cap, slot_bytes, bc, b->n, q, nd->cu_count, (unsigned long long*)out, s);
  else noalloc_launch<int32_t>(v, cap, slot_bytes, bc, b->n, q, nd->cu_count, (unsigned long long*)out, s);
  VX_HIP(hipGetLastError());
  return VX_OK;
}
