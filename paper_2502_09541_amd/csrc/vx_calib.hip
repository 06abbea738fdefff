// Link and memory calibration: the denominators of the late-materialization model and of the
// roofline fractions, measured on the machine the library runs on.
#include <algorithm>
#include <cstring>

#include "vx_internal.h"

namespace vx {

// Reads one 8-byte element every `step` elements; the sum keeps the loads alive.
__global__ void k_calib_read(const unsigned long long* p, uint64_t n_elems, uint64_t step,
                             unsigned long long* sink) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t n = n_elems / step;
  unsigned long long acc = 0;
  for (; i < n; i += stride) acc += p[i * step];
  if (acc == 0x9E3779B97F4A7C15ull) atomicAdd(sink, 1ull);
}

// Writes n 8-byte words of device memory with vector stores.
__global__ void k_calib_fill(unsigned long long* p, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = i * 0x9E3779B97F4A7C15ull;
}

// Writes n16 16-byte words of mapped host memory, the form the library's stores to host
// memory take.
__global__ void k_calib_write16(uint4* p, uint64_t n16) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n16;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = make_uint4((uint32_t)i, (uint32_t)(i >> 32), 0u, 1u);
}

static vx_status time_read(vx_ctx* ctx, const void* p, uint64_t bytes, uint64_t step, unsigned grid,
                           unsigned long long* sink, float* ms) {
  hipEvent_t a = get_event(ctx), b = get_event(ctx);
  hipLaunchKernelGGL(k_calib_read, dim3(grid), dim3(256), 0, ctx->compute, (const unsigned long long*)p,
                     bytes / 8, step, sink);
  VX_HIP(hipEventRecord(a, ctx->compute));
  hipLaunchKernelGGL(k_calib_read, dim3(grid), dim3(256), 0, ctx->compute, (const unsigned long long*)p,
                     bytes / 8, step, sink);
  VX_HIP(hipEventRecord(b, ctx->compute));
  VX_HIP(hipEventSynchronize(b));
  VX_HIP(hipEventElapsedTime(ms, a, b));
  put_event(ctx, a);
  put_event(ctx, b);
  return VX_OK;
}

}  // namespace vx

using namespace vx;

extern "C" vx_status vx_calibrate(vx_ctx* ctx, void* pinned, uint64_t bytes, vx_link_calib* out) {
  VX_CHECK(ctx && pinned && out, VX_EINVAL, "vx_calibrate: null argument");
  VX_CHECK(bytes >= (64u << 20), VX_EINVAL, "vx_calibrate: at least 64 MiB of pinned memory");
  vx::release_cached(ctx);
  VX_HIP(hipSetDevice(ctx->device));
  std::memset(out, 0, sizeof *out);
  vx_col c{pinned, VX_I64, 0};
  ColInfo hi;
  VX_TRY(classify(ctx, c, bytes / 8, &hi, "calibration buffer"));
  VX_CHECK(hi.where == Where::Host, VX_EINVAL, "vx_calibrate: buffer must be pinned host memory");
  const uint64_t chunk = 64u << 20;
  uint64_t dbytes = std::min<uint64_t>(bytes, ctx->arena.largest_free() / 2) / chunk * chunk;
  VX_CHECK(dbytes >= chunk, VX_EBUDGET, "vx_calibrate: the arena needs 128 MiB free");
  ArenaBlock d;
  d.a = &ctx->arena;
  d.p = ctx->arena.alloc(dbytes);
  VX_CHECK(d.p, VX_EBUDGET, "vx_calibrate: no room for the device buffer");
  unsigned long long* sink = (unsigned long long*)ctx->dev_acc;
  const unsigned grid = (unsigned)ctx->cu_count * 16;
  // host-to-device by the copy engines, 64 MiB copies (the pipeline's default chunk)
  {
    hipEvent_t a = get_event(ctx), b = get_event(ctx);
    VX_HIP(hipMemcpyAsync(d.p, hi.host, chunk, hipMemcpyHostToDevice, ctx->copy));
    VX_HIP(hipEventRecord(a, ctx->copy));
    for (uint64_t off = 0; off < dbytes; off += chunk)
      VX_HIP(hipMemcpyAsync(d.p + off, (const uint8_t*)hi.host + off, chunk, hipMemcpyHostToDevice, ctx->copy));
    VX_HIP(hipEventRecord(b, ctx->copy));
    VX_HIP(hipEventSynchronize(b));
    float ms = 0;
    VX_HIP(hipEventElapsedTime(&ms, a, b));
    out->h2d_gbs = dbytes / (ms * 1e6);
    put_event(ctx, a);
    put_event(ctx, b);
  }
  // zero-copy reads: contiguous, then one 8-byte element every 16 .. 1024 bytes
  const uint64_t zbytes = bytes / 8 * 8;
  float ms = 0;
  VX_TRY(time_read(ctx, hi.dev, zbytes, 1, grid, sink, &ms));
  out->zc_read_gbs = zbytes / (ms * 1e6);
  uint32_t granule = 8;
  for (int s = 0; s < 8; ++s) {
    uint64_t step = 2ull << s;   // 2 .. 256 elements = 16 .. 2048 bytes
    VX_TRY(time_read(ctx, hi.dev, zbytes, step, grid, sink, &ms));
    double elems = (double)(zbytes / 8 / step);
    out->zc_stride_bytes[s] = (uint32_t)(step * 8);
    out->zc_stride_gelems[s] = elems / (ms * 1e6);
    // while every line of the span still crosses the link, the span rate stays at the
    // contiguous rate; past the transfer granule it rises (fewer lines move)
    double span = zbytes / (ms * 1e6);
    if (granule == (uint32_t)(step * 4) && span <= 1.25 * out->zc_read_gbs) granule = (uint32_t)(step * 8);
  }
  out->zc_granule = granule;
  // device streaming read
  hipLaunchKernelGGL(k_calib_fill, dim3(grid), dim3(256), 0, ctx->compute, (unsigned long long*)d.p, dbytes / 8);
  VX_TRY(time_read(ctx, d.p, dbytes, 1, grid / 2, sink, &ms));
  out->hbm_read_gbs = dbytes / (ms * 1e6);
  ctx->zc_line = granule;

  // device-to-host: copies alone, both copy directions at once, kernel stores alone, and
  // host-to-device copies beside kernel stores
  uint8_t* hs = nullptr;
  VX_TRY(host_scratch(ctx, dbytes, &hs));
  void* hs_dev = nullptr;
  VX_HIP(hipHostGetDevicePointer(&hs_dev, hs, 0));
  VX_HIP(hipDeviceSynchronize());
  hipEvent_t e0 = get_event(ctx), e1 = get_event(ctx), e2 = get_event(ctx);
  VX_CHECK(e0 && e1 && e2, VX_EHIP, "vx_calibrate: event creation failed");
  auto span_ms = [&](hipEvent_t a, hipEvent_t b, hipEvent_t c, float* out_ms) -> vx_status {
    VX_HIP(hipEventSynchronize(b));
    VX_HIP(hipEventSynchronize(c));
    float x = 0, y = 0;
    VX_HIP(hipEventElapsedTime(&x, a, b));
    VX_HIP(hipEventElapsedTime(&y, a, c));
    *out_ms = std::max(x, y);
    return VX_OK;
  };
  auto d2h_copies = [&]() -> vx_status {
    for (uint64_t off = 0; off < dbytes; off += chunk)
      VX_HIP(hipMemcpyAsync(hs + off, d.p + off, chunk, hipMemcpyDeviceToHost, ctx->d2h));
    return VX_OK;
  };
  auto h2d_copies = [&]() -> vx_status {
    for (uint64_t off = 0; off < dbytes; off += chunk)
      VX_HIP(hipMemcpyAsync(d.p + off, (const uint8_t*)hi.host + off, chunk, hipMemcpyHostToDevice, ctx->copy));
    return VX_OK;
  };
  // warm the device-to-host path, then time it alone
  VX_HIP(hipMemcpyAsync(hs, d.p, chunk, hipMemcpyDeviceToHost, ctx->d2h));
  VX_HIP(hipEventRecord(e0, ctx->d2h));
  VX_TRY(d2h_copies());
  VX_HIP(hipEventRecord(e1, ctx->d2h));
  VX_TRY(span_ms(e0, e1, e1, &ms));
  out->d2h_gbs = dbytes / (ms * 1e6);
  // both directions: the two copy streams start from one event
  VX_HIP(hipEventRecord(e0, ctx->compute));
  VX_HIP(hipStreamWaitEvent(ctx->copy, e0, 0));
  VX_HIP(hipStreamWaitEvent(ctx->d2h, e0, 0));
  VX_TRY(h2d_copies());
  VX_TRY(d2h_copies());
  VX_HIP(hipEventRecord(e1, ctx->copy));
  VX_HIP(hipEventRecord(e2, ctx->d2h));
  VX_TRY(span_ms(e0, e1, e2, &ms));
  out->duplex_sdma_gbs = 2.0 * dbytes / (ms * 1e6);
  // kernel stores to mapped host memory, alone: 16-byte stores from one workgroup per 16 compute
  // units, the form the library's stores to host memory take (more workgroups slow the kernels
  // beside them and gain nothing)
  const unsigned wgrid = (unsigned)std::max(1, ctx->cu_count / 16);
  hipLaunchKernelGGL(k_calib_write16, dim3(wgrid), dim3(256), 0, ctx->compute, (uint4*)hs_dev, chunk / 16);
  VX_HIP(hipEventRecord(e0, ctx->compute));
  hipLaunchKernelGGL(k_calib_write16, dim3(wgrid), dim3(256), 0, ctx->compute, (uint4*)hs_dev, dbytes / 16);
  VX_HIP(hipEventRecord(e1, ctx->compute));
  VX_TRY(span_ms(e0, e1, e1, &ms));
  out->zc_write_gbs = dbytes / (ms * 1e6);
  // host-to-device copies beside kernel stores to host: the best of three runs (the rate the
  // sort and the partition passes move at, so its peak is taken as a maximum)
  out->duplex_zcw_gbs = 0;
  for (int trial = 0; trial < 3; ++trial) {
    VX_HIP(hipEventRecord(e0, ctx->compute));
    VX_HIP(hipStreamWaitEvent(ctx->copy, e0, 0));
    VX_TRY(h2d_copies());
    hipLaunchKernelGGL(k_calib_write16, dim3(wgrid), dim3(256), 0, ctx->compute, (uint4*)hs_dev, dbytes / 16);
    VX_HIP(hipEventRecord(e1, ctx->copy));
    VX_HIP(hipEventRecord(e2, ctx->compute));
    VX_TRY(span_ms(e0, e1, e2, &ms));
    out->duplex_zcw_gbs = std::max(out->duplex_zcw_gbs, 2.0 * dbytes / (ms * 1e6));
  }
  // kernel reads of mapped host memory beside device-to-host copies
  VX_HIP(hipEventRecord(e0, ctx->compute));
  VX_HIP(hipStreamWaitEvent(ctx->d2h, e0, 0));
  VX_TRY(d2h_copies());
  hipLaunchKernelGGL(k_calib_read, dim3(grid), dim3(256), 0, ctx->compute, (const unsigned long long*)hi.dev,
                     dbytes / 8, 1ull, sink);
  VX_HIP(hipEventRecord(e1, ctx->d2h));
  VX_HIP(hipEventRecord(e2, ctx->compute));
  VX_TRY(span_ms(e0, e1, e2, &ms));
  out->duplex_zcr_gbs = 2.0 * dbytes / (ms * 1e6);
  put_event(ctx, e0);
  put_event(ctx, e1);
  put_event(ctx, e2);
  return VX_OK;
}
