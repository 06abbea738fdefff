// The chunk pipeline: host-resident columns streamed through n_buffers device buffers.
//
// Chunk c uses buffer c % n_buffers.  Its copies go on the context's copy stream and are
// enqueued only once the kernel that last read that buffer has finished (the host waits on
// that kernel's event first), so a copy never sits in a hardware queue behind other work;
// the kernel for chunk c waits for its copies on the device and then runs on the compute
// stream while later copies proceed.  Columns that are not copied (device-resident, or read
// by zero-copy) are handed to the kernel as base pointers indexed by global row.
#pragma once

#include <functional>
#include <utility>
#include <vector>

#include "vx_internal.h"

namespace vx {

constexpr int kMaxPipeCols = 12;
constexpr uint32_t kMaxBuffers = 128;

struct PipeCol {
  ColInfo info;
  bool may_copy = false;   // buffers reserve room for this column
  bool copy = false;       // currently streamed by the copy stream (requires may_copy)
};

struct ChunkView {
  uint64_t index = 0, row0 = 0, rows = 0;
  const void* ptr[kMaxPipeCols] = {};
  uint32_t global_mask = 0;   // bit i: ptr[i] is a base pointer indexed by global row
};

class Pipeline {
 public:
  using KernelFn = std::function<vx_status(const ChunkView&)>;
  // Called once after chunk 0 has completed; may change PipeCol::copy of may_copy columns.
  using DecideFn = std::function<vx_status(std::vector<PipeCol>&)>;

  ~Pipeline();
  // Sizes chunks (auto: chunk_bytes of the widest copied column) and carves buffers from the
  // arena, halving the chunk while the buffers do not fit (unless chunk_rows was given).
  vx_status plan(vx_ctx* ctx, uint64_t n, uint64_t chunk_rows, uint32_t n_buffers,
                 std::vector<PipeCol> cols, uint64_t default_chunk_bytes = 64ull << 20);
  vx_status run(const KernelFn& fn, const DecideFn& decide = nullptr);
  // Enqueues the copies of the first min(k, buffers - 1, chunks) chunks now, so that they proceed
  // while the caller runs other work on the compute stream; the next run() starts from them.
  vx_status prefetch(uint64_t k);

  std::vector<PipeCol>& cols() { return cols_; }
  uint64_t chunk_rows() const { return chunk_rows_; }
  uint64_t n_chunks() const { return n_chunks_; }
  uint32_t n_buffers() const { return nbuf_; }
  bool streamed() const { return streamed_; }
  uint64_t sdma_bytes() const { return sdma_bytes_; }
  double kernel_ms() const;
  uint64_t kernel_launches() const { return kev_.size(); }

 private:
  vx_status issue_copy(uint64_t c);
  vx_status issue_kernel(uint64_t c, const KernelFn& fn);
  ChunkView view(uint64_t c) const;
  void release_events();

  vx_ctx* ctx_ = nullptr;
  uint64_t n_ = 0, chunk_rows_ = 0, n_chunks_ = 0, sdma_bytes_ = 0;
  uint32_t nbuf_ = 2;
  bool streamed_ = false;
  std::vector<PipeCol> cols_;
  uint64_t prefetched_ = 0;
  ArenaBlock bufs_[kMaxBuffers];
  hipEvent_t ev_copied_[kMaxBuffers] = {}, ev_free_[kMaxBuffers] = {};
  bool free_pending_[kMaxBuffers] = {};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> kev_;
};

uint64_t env_u64(const char* name, uint64_t dflt);

}  // namespace vx
