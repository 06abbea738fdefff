// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "vx.h"

namespace vx {

// ---------------------------------------------------------------- errors

void set_error(const char* fmt, ...);

struct Fail {
  vx_status st;
};

#define VX_TRY(expr)                  \
  do {                                \
    vx_status st__ = (expr);          \
    if (st__ != VX_OK) return st__;   \
  } while (0)

#define VX_HIP(expr)                                                              \
  do {                                                                            \
    hipError_t e__ = (expr);                                                      \
    if (e__ != hipSuccess) {                                                      \
      ::vx::set_error("HIP error '%s' in %s (%s:%d)", hipGetErrorString(e__), #expr, \
                      __FILE__, __LINE__);                                        \
      return VX_EHIP;                                                             \
    }                                                                             \
  } while (0)

#define VX_CHECK(cond, status, ...)   \
  do {                                \
    if (!(cond)) {                    \
      ::vx::set_error(__VA_ARGS__);   \
      return status;                  \
    }                                 \
  } while (0)

// ---------------------------------------------------------------- arena

// First-fit allocator over the caller's device buffer.  Blocks are 256-byte aligned.
class Arena {
 public:
  void init(uint8_t* base, uint64_t bytes);
  uint8_t* alloc(uint64_t bytes);   // nullptr when it does not fit
  void release(uint8_t* p);
  uint64_t used() const { return used_; }
  uint64_t largest_free() const;
  uint64_t capacity() const { return bytes_; }

 private:
  uint8_t* base_ = nullptr;
  uint64_t bytes_ = 0;
  uint64_t used_ = 0;
  std::map<uint64_t, uint64_t> free_;   // offset -> size
  std::map<uint64_t, uint64_t> live_;   // offset -> size
};

// Allocation that returns to the arena at scope exit.
struct ArenaBlock {
  Arena* a = nullptr;
  uint8_t* p = nullptr;
  ArenaBlock() = default;
  ArenaBlock(const ArenaBlock&) = delete;
  ArenaBlock& operator=(const ArenaBlock&) = delete;
  ~ArenaBlock() { reset(); }
  void reset() {
    if (a && p) a->release(p);
    p = nullptr;
  }
};

// ---------------------------------------------------------------- columns

enum class Where { Device, Host };

struct ColInfo {
  Where where;
  const void* dev;    // device-accessible address (device memory or host mapping)
  const void* host;   // host address when Where::Host
  int elsize;         // 4 or 8
};

}  // namespace vx

struct vx_ctx {
  int device = 0;
  hipStream_t compute = nullptr;
  hipStream_t copy = nullptr;
  bool own_compute = false;
  vx::Arena arena;
  // device scratch for results: per-chunk aggregate rows etc. (carved at create)
  uint64_t* dev_acc = nullptr;
  uint64_t dev_acc_words = 0;
  unsigned int* dev_flags = nullptr;   // error flags written by kernels
  uint64_t* dev_scan = nullptr;        // kScanTilesMax + 1 words: tile sums of the partition scan
  int cu_count = 256;
  uint64_t l2_bytes = 4u << 20;
  // pinned host mirror of results (dev_acc_words words), then kHostSmallWords words for small
  // readbacks (error flags) that are read beside it
  uint64_t* host_acc = nullptr;
  uint64_t* host_small = nullptr;
  // device-to-host copies of intermediate results (partition pass write-back)
  hipStream_t d2h = nullptr;
  // pinned host memory for intermediates that live in CPU memory (grow-only, kept until destroy)
  uint8_t* host_scratch = nullptr;
  uint64_t host_scratch_bytes = 0;
  std::vector<hipEvent_t> ev_pool;
  uint32_t zc_line = 128;   // zero-copy transfer granule (bytes), measured by vx_calibrate
};

namespace vx {

// Drop the batch join's cached graph and tables held for this context.
void batch_release_ctx(const vx_ctx* ctx);
// Give back arena memory that a call keeps for reuse by the next call of its kind (the batch
// join's graph and tables): every entry point that does not reuse it calls this first, so its
// working set sees the whole arena.
inline void release_cached(vx_ctx* ctx) { batch_release_ctx(ctx); }

// Pinned host scratch of at least `bytes` (grows by reallocation; contents not kept).
vx_status host_scratch(vx_ctx* ctx, uint64_t bytes, uint8_t** out);

vx_status classify(const vx_ctx* ctx, const vx_col& c, uint64_t n, ColInfo* out, const char* what);
int elsize_of(int32_t type);
double now_ms();

// Acquire/return HIP events from the context pool.
hipEvent_t get_event(vx_ctx* ctx);
void put_event(vx_ctx* ctx, hipEvent_t e);

// Zero a device range on a stream with a fill kernel (no memset nodes: safe to capture).
void fill_zero(uint64_t* p, uint64_t words, hipStream_t s);

// Estimated zero-copy wire bytes of reading `count` matching rows, of elsize bytes each,
// spread over `n` rows: the touched lines of `line` bytes under independent selection.
double zc_wire_bytes(uint64_t n, uint64_t count, int elsize, uint32_t line);
constexpr uint32_t kScanTilesMax = 1024;
constexpr uint64_t kHostSmallWords = 32;
constexpr int kAccWords = 10;           // count + 8 sums + zero-copy granules per aggregate row

}  // namespace vx
