// The chunk pipeline (the double-buffered executor); see vx_pipeline.h.
#include <algorithm>
#include <cstdlib>

#include "vx_pipeline.h"

namespace vx {

uint64_t env_u64(const char* name, uint64_t dflt) {
  const char* e = getenv(name);
  return e ? strtoull(e, nullptr, 10) : dflt;
}

Pipeline::~Pipeline() {
  if (ctx_) {
    // buffers return to the arena only once no copy or kernel can still touch them
    (void)hipStreamSynchronize(ctx_->copy);
    (void)hipStreamSynchronize(ctx_->compute);
  }
  release_events();
}

void Pipeline::release_events() {
  if (!ctx_) return;
  for (uint32_t b = 0; b < kMaxBuffers; ++b) {
    put_event(ctx_, ev_copied_[b]);
    put_event(ctx_, ev_free_[b]);
    ev_copied_[b] = ev_free_[b] = nullptr;
  }
  for (auto& pr : kev_) {
    put_event(ctx_, pr.first);
    put_event(ctx_, pr.second);
  }
  kev_.clear();
}

static uint64_t align256(uint64_t v) { return (v + 255) / 256 * 256; }

constexpr uint64_t kMinChunks = 4;

vx_status Pipeline::plan(vx_ctx* ctx, uint64_t n, uint64_t chunk_rows, uint32_t n_buffers,
                         std::vector<PipeCol> cols, uint64_t default_chunk_bytes) {
  ctx_ = ctx;
  n_ = n;
  cols_ = std::move(cols);
  VX_CHECK(cols_.size() <= (size_t)kMaxPipeCols, VX_EINVAL, "pipeline: %zu columns (max %d)",
           cols_.size(), kMaxPipeCols);
  nbuf_ = n_buffers ? n_buffers : (uint32_t)env_u64("VX_BUFFERS", 2);
  VX_CHECK(nbuf_ >= 2 && nbuf_ <= kMaxBuffers, VX_EINVAL, "pipeline: n_buffers %u outside 2..%u", nbuf_,
           kMaxBuffers);
  uint64_t row_bytes = 0;
  int widest = 0;
  streamed_ = false;
  for (auto& c : cols_) {
    if (c.info.where != Where::Host) {
      c.may_copy = c.copy = false;
      continue;
    }
    if (c.copy) c.may_copy = true;
    if (c.may_copy) {
      row_bytes += (uint64_t)c.info.elsize;
      widest = std::max(widest, c.info.elsize);
      streamed_ = true;
    }
  }
  bool given = chunk_rows != 0;
  if (!given) {
    const bool env = getenv("VX_CHUNK_BYTES") != nullptr;
    uint64_t cb = env_u64("VX_CHUNK_BYTES", default_chunk_bytes);
    // a short column still gets kMinChunks chunks, so that its copies overlap the kernels, but
    // no chunk under 8 MiB (shorter copies lose rate to their fixed cost)
    if (!env && streamed_) cb = std::min(cb, std::max<uint64_t>(8ull << 20, n * (uint64_t)widest / kMinChunks));
    chunk_rows = streamed_ ? std::max<uint64_t>(1, cb / (uint64_t)std::max(widest, 1)) : (n ? n : 1);
  }
  if (n && chunk_rows > n) chunk_rows = n;
  if (chunk_rows == 0) chunk_rows = 1;
  if (streamed_ && n) {
    for (;;) {
      uint64_t bytes = 256;
      for (auto& c : cols_)
        if (c.may_copy) bytes += align256(chunk_rows * (uint64_t)c.info.elsize);
      bool ok = true;
      for (uint32_t b = 0; b < nbuf_; ++b) {
        bufs_[b].a = &ctx->arena;
        bufs_[b].p = ctx->arena.alloc(bytes);
        if (!bufs_[b].p) ok = false;
      }
      if (ok) break;
      for (uint32_t b = 0; b < nbuf_; ++b) bufs_[b].reset();
      VX_CHECK(!given && chunk_rows > 1024, VX_EBUDGET,
               "pipeline: %u chunk buffers of %llu rows x %llu B do not fit the arena (%llu B free, "
               "largest block %llu B)",
               nbuf_, (unsigned long long)chunk_rows, (unsigned long long)row_bytes,
               (unsigned long long)(ctx->arena.capacity() - ctx->arena.used()),
               (unsigned long long)ctx->arena.largest_free());
      chunk_rows /= 2;
    }
  }
  chunk_rows_ = chunk_rows;
  n_chunks_ = n ? (n + chunk_rows - 1) / chunk_rows : 0;
  for (uint32_t b = 0; b < nbuf_; ++b) {
    ev_copied_[b] = get_event(ctx);
    ev_free_[b] = get_event(ctx);
    VX_CHECK(ev_copied_[b] && ev_free_[b], VX_EHIP, "pipeline: event creation failed");
    free_pending_[b] = false;
  }
  return VX_OK;
}

ChunkView Pipeline::view(uint64_t c) const {
  ChunkView v;
  v.index = c;
  v.row0 = c * chunk_rows_;
  v.rows = std::min(chunk_rows_, n_ - v.row0);
  uint32_t b = (uint32_t)(c % nbuf_);
  uint64_t off = 0;
  for (size_t i = 0; i < cols_.size(); ++i) {
    const PipeCol& col = cols_[i];
    if (col.may_copy && col.copy) {
      v.ptr[i] = bufs_[b].p + off;
    } else {
      v.ptr[i] = col.info.dev;
      v.global_mask |= 1u << i;
    }
    if (col.may_copy) off += align256(chunk_rows_ * (uint64_t)col.info.elsize);
  }
  return v;
}

vx_status Pipeline::issue_copy(uint64_t c) {
  uint32_t b = (uint32_t)(c % nbuf_);
  if (free_pending_[b]) {
    VX_HIP(hipEventSynchronize(ev_free_[b]));
    free_pending_[b] = false;
  }
  ChunkView v = view(c);
  for (size_t i = 0; i < cols_.size(); ++i) {
    const PipeCol& col = cols_[i];
    if (!(col.may_copy && col.copy)) continue;
    uint64_t es = (uint64_t)col.info.elsize;
    VX_HIP(hipMemcpyAsync(const_cast<void*>(v.ptr[i]), (const uint8_t*)col.info.host + v.row0 * es,
                          v.rows * es, hipMemcpyHostToDevice, ctx_->copy));
    sdma_bytes_ += v.rows * es;
  }
  VX_HIP(hipEventRecord(ev_copied_[b], ctx_->copy));
  return VX_OK;
}

vx_status Pipeline::issue_kernel(uint64_t c, const KernelFn& fn) {
  uint32_t b = (uint32_t)(c % nbuf_);
  if (streamed_) VX_HIP(hipStreamWaitEvent(ctx_->compute, ev_copied_[b], 0));
  hipEvent_t a = get_event(ctx_), e = get_event(ctx_);
  VX_CHECK(a && e, VX_EHIP, "pipeline: event creation failed");
  kev_.push_back({a, e});
  VX_HIP(hipEventRecord(a, ctx_->compute));
  VX_TRY(fn(view(c)));
  VX_HIP(hipEventRecord(e, ctx_->compute));
  if (streamed_) {
    VX_HIP(hipEventRecord(ev_free_[b], ctx_->compute));
    free_pending_[b] = true;
  }
  return VX_OK;
}

vx_status Pipeline::prefetch(uint64_t k) {
  if (!streamed_) return VX_OK;
  // one buffer stays free, so run() always has a kernel queued ahead of the copy it waits to issue
  k = std::min<uint64_t>(std::min<uint64_t>(k, nbuf_ - 1), n_chunks_);
  for (uint64_t c = prefetched_; c < k; ++c) VX_TRY(issue_copy(c));
  prefetched_ = std::max(prefetched_, k);
  return VX_OK;
}

vx_status Pipeline::run(const KernelFn& fn, const DecideFn& decide) {
  if (n_chunks_ == 0) return VX_OK;
  if (!streamed_) {
    for (uint64_t c = 0; c < n_chunks_; ++c) VX_TRY(issue_kernel(c, fn));
    return VX_OK;
  }
  uint64_t start = 0, issued = prefetched_;
  prefetched_ = 0;
  if (decide && n_chunks_ > 1) {
    // the decision may change which columns are copied: nothing past chunk 0 may be in flight
    VX_CHECK(issued <= 1, VX_EINVAL, "pipeline: prefetch and a chunk-0 decision do not combine");
    if (issued == 0) {
      VX_TRY(issue_copy(0));
      issued = 1;
    }
    VX_TRY(issue_kernel(0, fn));
    VX_HIP(hipStreamSynchronize(ctx_->compute));
    VX_TRY(decide(cols_));
    for (auto& c : cols_)
      if (c.copy && !c.may_copy) c.copy = false;
    start = 1;
  }
  uint64_t ahead = std::min<uint64_t>(n_chunks_, start + nbuf_ - 1);
  for (uint64_t c = issued; c < ahead; ++c) VX_TRY(issue_copy(c));
  issued = std::max(issued, ahead);
  for (uint64_t c = start; c < n_chunks_; ++c) {
    VX_TRY(issue_kernel(c, fn));
    if (issued < n_chunks_) {
      VX_TRY(issue_copy(issued));
      ++issued;
    }
  }
  return VX_OK;
}

double Pipeline::kernel_ms() const {
  double t = 0;
  for (auto& pr : kev_) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) t += ms;
  }
  return t;
}

}  // namespace vx
