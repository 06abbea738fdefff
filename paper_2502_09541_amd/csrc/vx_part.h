// Stable multisplit: partition ids, per-wave histograms, exclusive scan, stable scatter.
//
// Rows are split into contiguous wave tiles (wave w owns rows [w*T, (w+1)*T)).  Pass 1 counts
// each wave's rows per partition into hist[p * W + w] (partition-major).  An exclusive scan
// of that array gives every (partition, wave) pair its output offset, so partition p's rows
// land contiguously, in input order.  Pass 2 walks each wave tile in 64-row steps: ten
// ballots give each lane the mask of lanes with the same partition id, its rank among them
// is a popcount, and a per-wave running counter in LDS advances by the step's count.
#pragma once

#include "vx_internal.h"

namespace vx {

constexpr uint32_t kMaxParts = 1024;
constexpr uint32_t kMaxPartIdBits = 10;

enum PartFn : uint32_t {
  kPartHash = 0,      // top log2 P bits of the MurmurHash3 64-bit finalizer
  kPartBits = 1,      // raw key bits [shift, shift + log2 P); flip_sign orders signed keys
  kPartRange = 2      // number of splitters <= key
};

struct PartSpec {
  uint32_t fn;
  uint32_t n_parts;
  uint32_t log2p;
  uint32_t shift;
  uint32_t flip_sign;
  uint32_t n_split;
  const long long* splitters;   // device, ascending
};

struct PartIO {
  const void* key;               // keys of this launch (row 0 = first row)
  uint32_t key_size;
  uint32_t n_pay;
  const void* pay[4];
  uint32_t pay_size[4];
  uint64_t n;
  void* out_key;                 // clustered outputs (device or host-mapped), may be null
  void* out_pay[4];
  uint64_t out_base;             // row offset added to every output position
};

// Partition id of key k: hash, raw bits, or the count of splitters <= k (split[] ascending,
// ps.n_split entries, usually staged in LDS by the caller).
__device__ __forceinline__ unsigned long long fmix64(unsigned long long h) {
  h ^= h >> 33;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  return h;
}

__device__ __forceinline__ uint32_t part_of(const PartSpec& ps, long long k, const long long* split) {
  if (ps.fn == kPartHash) {
    return ps.log2p ? (uint32_t)(fmix64((unsigned long long)k) >> (64 - ps.log2p)) : 0u;
  }
  if (ps.fn == kPartBits) {
    unsigned long long u = (unsigned long long)k;
    if (ps.flip_sign) u ^= 0x8000000000000000ull;
    return (uint32_t)((u >> ps.shift) & (unsigned long long)(ps.n_parts - 1));
  }
  uint32_t lo = 0, hi = ps.n_split;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (split[mid] <= k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Launch geometry shared by hist and scatter: waves and rows per wave tile.
struct PartGeom {
  uint32_t blocks;
  uint32_t waves;     // blocks * 4
  uint64_t tile;      // rows per wave (multiple of 64)
};

PartGeom part_geom(const vx_ctx* ctx, uint64_t n);

constexpr uint32_t kMaxSumSlots = 64;

// hist: n_parts * waves uint32 (partition-major).  totals (optional, n_parts u64) accumulates
// each partition's row count.  sums (optional): for partitions with sum_slot[p] >= 0 (a
// device int array of n_parts entries, slots < kMaxSumSlots), the row count and the SUM of
// payload 0 are added to sums[2*slot] and sums[2*slot+1].
vx_status part_hist(vx_ctx* ctx, const PartSpec& ps, const PartIO& io, const PartGeom& g,
                    uint32_t* hist, unsigned long long* totals, const int* sum_slot,
                    unsigned long long* sums, hipStream_t s);
// Exclusive scan of hist (n_parts * waves) into offs (uint64).  Without part_base, one scan
// over the whole array (chunk-local clustering) and boundary (optional, n_parts + 1) receives
// each partition's first offset and the total.  With part_base (device, n_parts u64), each
// partition is scanned on its own and starts at part_base[p] (global placement).
vx_status part_scan(vx_ctx* ctx, const uint32_t* hist, uint32_t n_parts, uint32_t waves,
                    const unsigned long long* part_base, unsigned long long* offs,
                    unsigned long long* boundary, hipStream_t s);
vx_status part_scatter(vx_ctx* ctx, const PartSpec& ps, const PartIO& io, const PartGeom& g,
                       const unsigned long long* offs, hipStream_t s);

}  // namespace vx
