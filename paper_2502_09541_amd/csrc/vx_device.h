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
// lane must call it; every lane gets the same count.  es is a power of two no larger than the
// granule, a0 a multiple of es.  The work is on the wave's ballot mask (scalar operations): with
// L = lanes per granule and r = the lanes of the first granule that lie before lane 0, the mask
// shifted up by r splits into whole L-bit groups, one per granule, and the count is the number
// of nonzero groups.
__device__ __forceinline__ uint32_t mask_groups(unsigned long long x, uint32_t log2_l) {
  for (uint32_t s = (1u << log2_l) >> 1; s; s >>= 1) x |= x >> s;   // bit g*L: group g nonzero
  unsigned long long pick = 1;
  for (uint32_t s = 1u << log2_l; s < 64; s <<= 1) pick |= pick << s;
  return (uint32_t)__popcll(x & pick);
}

// The same count from the wave's ballot mask m of active lanes.
__device__ __forceinline__ uint32_t mask_granules(unsigned long long m, uint64_t a0, uint32_t es, uint32_t shift) {
  if (m == 0) return 0;
  const uint64_t a = __builtin_amdgcn_readfirstlane((uint32_t)a0) |
                     ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(a0 >> 32)) << 32);
  const uint32_t log2_es = 31u - (uint32_t)__clz(es);
  const uint32_t log2_l = shift - log2_es;                  // lanes per granule, log2
  if (log2_l > 6) {   // a granule wider than the wave: it spans at most two
    const uint32_t first = (uint32_t)__builtin_ctzll(m), last = 63u - (uint32_t)__clzll(m);
    return ((a + (uint64_t)first * es) >> shift) == ((a + (uint64_t)last * es) >> shift) ? 1u : 2u;
  }
  const uint32_t r = (uint32_t)((a >> log2_es) & ((1u << log2_l) - 1u));
  if (r == 0) {   // the wave starts on a granule: 8-byte or 4-byte rows in 128-byte granules
    if (log2_l == 4) {
      unsigned long long x = m | (m >> 1);
      x |= x >> 2;
      x |= x >> 4;
      x |= x >> 8;
      return (uint32_t)__popcll(x & 0x0001000100010001ull);
    }
    if (log2_l == 5) {
      unsigned long long x = m | (m >> 1);
      x |= x >> 2;
      x |= x >> 4;
      x |= x >> 8;
      x |= x >> 16;
      return (uint32_t)__popcll(x & 0x0000000100000001ull);
    }
  }
  const unsigned long long lo = m << r, hi = r ? m >> (64u - r) : 0ull;
  return mask_groups(lo, log2_l) + mask_groups(hi, log2_l);
}

__device__ __forceinline__ uint32_t wave_granules(bool active, uint64_t a0, uint32_t es, uint32_t shift) {
  return mask_granules(__ballot(active), a0, es, shift);
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
