// Device hash table: open addressing, linear probing, power-of-two capacity.
//
// Slot layout (slot_bytes = 2^slot_shift):
//   unique table:   [key][pay 0][pay 1]...   each payload at its own width, naturally aligned
//   pre-aggregated: [key (8 bytes)][count (8)][sum 0 (8)][sum 1 (8)]...
// The all-ones-high-bit pattern (INT32_MIN / INT64_MIN) marks an empty slot; rows whose
// key equals it are aggregated into a side record instead: side[0] = count,
// side[1 + c] = SUM of payload c (and, for unique tables, side[5 + c] holds nothing more).
#pragma once

#include "vx_internal.h"

namespace vx {

template <typename K> struct KeyTraits;
template <> struct KeyTraits<int32_t> {
  using U = unsigned int;
  static constexpr U kEmpty = 0x80000000u;
};
template <> struct KeyTraits<int64_t> {
  using U = unsigned long long;
  static constexpr U kEmpty = 0x8000000000000000ull;
};

// Fibonacci hashing: the top log2(capacity) bits of key * 2^64/phi.
__device__ __host__ __forceinline__ uint64_t slot_of(uint64_t key_bits, uint32_t log2cap) {
  return (key_bits * 0x9E3779B97F4A7C15ull) >> (64 - log2cap);
}

constexpr uint32_t kMaxPay = 4;

// Error flags raised by kernels (ctx->dev_flags[0]).
enum : unsigned int { kFlagDup = 1u, kFlagFull = 2u, kFlagGroupOverflow = 4u };

struct TableView {
  uint8_t* slots;
  uint64_t mask;          // capacity - 1
  uint32_t log2cap;
  uint32_t slot_shift;
  unsigned long long* side;   // 1 + kMaxPay words
  uint32_t n_pay;
  uint32_t pay_off[kMaxPay];  // byte offset within the slot
  uint32_t pay_size[kMaxPay]; // 4 or 8 (unique); 8 (pre-aggregated sums)
  uint32_t preagg;
  uint32_t key_size;
  // Direct layout (direct == 1): key k lives in slot ord(k) - kmin_ord, where ord is the
  // order-preserving unsigned form of the key, and keys outside [kmin, kmin + direct_range) are
  // absent.  A slot then holds k or the empty marker, never another key, so every probe ends at
  // its first slot.
  // Dense layout (direct == 2): a unique build whose n keys are exactly the n values of their
  // range.  Every key of the range is present, so a slot holds only the payloads (at pay_off,
  // from offset 0; no slots at all without payloads) and a probe in range is a match.  `present`
  // holds one byte per key of the range, set by plain stores while building: a repeated key
  // leaves another key's byte unset, so fewer set bytes than rows catches it.
  uint32_t direct;
  unsigned long long kmin_ord;
  uint64_t direct_range;
  uint8_t* present;
};

enum : uint32_t { kLayoutHash = 0, kLayoutDirect = 1, kLayoutDense = 2 };

}  // namespace vx

struct vx_table {
  vx_ctx* ctx = nullptr;
  uint8_t* mem = nullptr;     // arena block: slots then side record
  uint64_t bytes = 0;
  uint64_t capacity = 0;
  uint64_t n_rows = 0;
  int32_t key_type = VX_I64;
  uint32_t flags = 0;
  uint32_t pay_type[vx::kMaxPay] = {0, 0, 0, 0};
  vx::TableView view{};
};

namespace vx {
// The build keys' range in order-preserving unsigned form (the empty-marker key excluded), or
// `known == false` when it was not measured.
struct KeyRange {
  bool known = false;
  unsigned long long min_ord = 0, max_ord = 0;
  uint64_t empty_rows = 0;    // rows whose key is the empty marker
  bool allow_dense = false;   // the caller's build is unique and may take the dense layout
};

// Launch helpers implemented in vx_join.hip and used by the other executors.
// make_table lays the table out directly (slot = key - min) when `kr` holds a measured range no
// wider than the hash table's capacity, so the direct table is never the larger of the two.
vx_status make_table(vx_ctx* ctx, int32_t key_type, uint32_t flags, const int32_t* pay_types,
                     uint32_t n_pay, uint64_t expected_rows, float load_factor, vx_table** out,
                     const KeyRange* kr = nullptr);
// Measure the range of n device-resident keys (one pass over them, then a 16-byte read back).
vx_status key_range(vx_ctx* ctx, int32_t key_type, const void* dev_keys, uint64_t n, KeyRange* out);
vx_status table_insert(vx_ctx* ctx, vx_table* t, const ColInfo& key, const ColInfo* pays,
                       uint64_t n, hipStream_t s, int group_lanes);
vx_status check_flags(vx_ctx* ctx, const char* what);
}  // namespace vx
