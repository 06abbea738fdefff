// Device-side helpers shared by the kernels of several translation units.
#pragma once

#include "vx_table.h"

namespace vx {

template <typename K>
__device__ __forceinline__ uint64_t key_bits(K k) {
  return (uint64_t)(typename KeyTraits<K>::U)k;
}

// order-preserving unsigned form of a key (sign-extended, sign bit flipped)
template <typename K>
__device__ __forceinline__ unsigned long long key_ord(K k) {
  return (unsigned long long)(long long)k ^ 0x8000000000000000ull;
}

// First slot of k's probe sequence in t, for a layout known at compile time (DIRECT) or read
// from the table.  False when k cannot be in a direct table (outside its key range); then no
// slot is read.
template <bool DIRECT, typename K>
__device__ __forceinline__ bool first_slot_as(const TableView& t, K k, uint64_t& h) {
  if (DIRECT) {
    h = key_ord(k) - t.kmin_ord;
    return h < t.direct_range;
  }
  h = slot_of(key_bits(k), t.log2cap);
  return true;
}

template <typename K>
__device__ __forceinline__ bool first_slot(const TableView& t, K k, uint64_t& h) {
  return t.direct ? first_slot_as<true>(t, k, h) : first_slot_as<false>(t, k, h);
}

__device__ __forceinline__ long long load_signed(const void* base, uint64_t idx, uint32_t size) {
  if (size == 4) return (long long)((const int*)base)[idx];
  return ((const long long*)base)[idx];
}

__device__ __forceinline__ long long slot_signed(const uint8_t* slot, uint32_t off, uint32_t size) {
  if (size == 4) return (long long)*(const int*)(slot + off);
  return *(const long long*)(slot + off);
}

// Zero-copy traffic, counted: the number of distinct granules of 2^shift bytes that hold the
// elements this wave reads, where lane l reads the element at device address a0 + l * es
// (consecutive rows in consecutive lanes) when `active`.  A granule is the unit a zero-copy
// read moves over the host link, so this is what the wave's gather costs on the wire.  Every
// lane must call it; every lane gets the same count.
__device__ __forceinline__ uint32_t wave_granules(bool active, uint64_t a0, uint32_t es, uint32_t shift) {
  const unsigned long long m = __ballot(active);
  if (m == 0) return 0;
  const uint32_t lane = threadIdx.x & 63;
  const unsigned long long below = m & ((1ull << lane) - 1ull);
  bool first = false;
  if (active) {
    if (below == 0) {
      first = true;
    } else {   // the granule differs from that of the nearest active lane below
      const uint32_t prev = 63u - (uint32_t)__clzll(below);
      first = ((a0 + (uint64_t)prev * es) >> shift) != ((a0 + (uint64_t)lane * es) >> shift);
    }
  }
  return (uint32_t)__popcll(__ballot(first));
}

template <int NACC>
__device__ __forceinline__ void block_flush(unsigned long long (&acc)[NACC], int nacc,
                                            unsigned long long* out) {
  __shared__ unsigned long long red[NACC][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int a = 0; a < NACC; ++a) {
    unsigned long long v = acc[a];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[a][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)nacc) {
    unsigned long long s = 0;
    for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
    if (s) atomicAdd(out + threadIdx.x, s);
  }
}


// Find `k` in a unique table.  Returns the slot, or nullptr when absent; keys equal to the
// empty marker are looked up in the side record by the caller.  find_slot_hashed is for tables
// known to be hashed: it carries no test of the layout, which would change the loop's code.
template <typename K>
__device__ __forceinline__ const uint8_t* find_slot_hashed(const TableView& t, K k) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  const U kb = (U)k;
  uint64_t h = slot_of(key_bits(k), t.log2cap);
  for (uint64_t step = 0; step <= t.mask; ++step) {
    const uint8_t* slot = t.slots + (h << t.slot_shift);
    U sk = *(const U*)slot;
    if (sk == kb) return slot;
    if (sk == kEmpty) return nullptr;
    h = (h + 1) & t.mask;
  }
  return nullptr;
}

template <typename K>
__device__ __forceinline__ const uint8_t* find_slot(const TableView& t, K k) {
  if (!t.direct) return find_slot_hashed(t, k);
  using U = typename KeyTraits<K>::U;
  uint64_t h;
  if (!first_slot_as<true>(t, k, h)) return nullptr;
  const uint8_t* slot = t.slots + (h << t.slot_shift);
  return *(const U*)slot == (U)k ? slot : nullptr;   // a direct slot holds k or the empty marker
}

template <typename K>
__device__ __forceinline__ K load_key(const void* base, uint64_t idx) {
  return ((const K*)base)[idx];
}

// Add (cnt, sums) to key k's record of a pre-aggregated table, claiming a slot if needed.
template <typename K>
__device__ __forceinline__ void global_preagg_add(const TableView& t, K k, unsigned long long cnt,
                                                  const unsigned long long* sums,
                                                  unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  U kb = (U)k;
  if (kb == kEmpty) {
    atomicAdd(t.side, cnt);
    for (uint32_t p = 0; p < t.n_pay; ++p) atomicAdd(t.side + 1 + p, sums[p]);
    return;
  }
  uint64_t h;
  if (!first_slot(t, k, h)) {
    atomicOr(flags, kFlagFull);
    return;
  }
  for (uint64_t step = 0; step <= t.mask; ++step) {
    uint8_t* slot = t.slots + (h << t.slot_shift);
    U prev = atomicCAS((U*)slot, kEmpty, kb);
    if (prev == kEmpty || prev == kb) {
      unsigned long long* w = (unsigned long long*)(slot + 8);
      atomicAdd(w, cnt);
      for (uint32_t p = 0; p < t.n_pay; ++p) atomicAdd(w + 1 + p, sums[p]);
      return;
    }
    h = (h + 1) & t.mask;
  }
  atomicOr(flags, kFlagFull);
}

}  // namespace vx
