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
};

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
// Launch helpers implemented in vx_join.hip and used by the other executors.
vx_status make_table(vx_ctx* ctx, int32_t key_type, uint32_t flags, const int32_t* pay_types,
                     uint32_t n_pay, uint64_t expected_rows, float load_factor, vx_table** out);
vx_status table_insert(vx_ctx* ctx, vx_table* t, const ColInfo& key, const ColInfo* pays,
                       uint64_t n, hipStream_t s, int group_lanes);
vx_status check_flags(vx_ctx* ctx, const char* what);
}  // namespace vx
