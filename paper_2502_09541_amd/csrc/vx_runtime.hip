// Context, arena, error reporting, host memory and column classification.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "vx_internal.h"

namespace vx {

static thread_local std::string g_err = "no error";

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int elsize_of(int32_t type) {
  if (type == VX_I32) return 4;
  if (type == VX_I64) return 8;
  return 0;
}

// ---------------------------------------------------------------- arena

static constexpr uint64_t kAlign = 256;

void Arena::init(uint8_t* base, uint64_t bytes) {
  uint64_t off = (kAlign - ((uintptr_t)base % kAlign)) % kAlign;
  base_ = base + off;
  bytes_ = bytes > off ? ((bytes - off) / kAlign) * kAlign : 0;
  used_ = 0;
  free_.clear();
  live_.clear();
  if (bytes_) free_[0] = bytes_;
}

uint8_t* Arena::alloc(uint64_t bytes) {
  if (bytes == 0) bytes = kAlign;
  bytes = (bytes + kAlign - 1) / kAlign * kAlign;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      uint64_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      live_[off] = bytes;
      used_ += bytes;
      return base_ + off;
    }
  }
  return nullptr;
}

void Arena::release(uint8_t* p) {
  if (!p) return;
  uint64_t off = (uint64_t)(p - base_);
  auto it = live_.find(off);
  if (it == live_.end()) return;
  uint64_t sz = it->second;
  live_.erase(it);
  used_ -= sz;
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && off + sz == nx->first) {
    sz += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {
    auto pv = std::prev(nx);
    if (pv->first + pv->second == off) {
      pv->second += sz;
      return;
    }
  }
  free_[off] = sz;
}

uint64_t Arena::largest_free() const {
  uint64_t m = 0;
  for (auto& kv : free_) m = kv.second > m ? kv.second : m;
  return m;
}

// ---------------------------------------------------------------- columns

vx_status classify(const vx_ctx* ctx, const vx_col& c, uint64_t n, ColInfo* out, const char* what) {
  int es = elsize_of(c.type);
  VX_CHECK(es != 0, VX_EINVAL, "%s: column type %d is not VX_I32/VX_I64", what, c.type);
  out->elsize = es;
  if (n == 0) {
    out->where = Where::Device;
    out->dev = c.data;
    out->host = nullptr;
    return VX_OK;
  }
  VX_CHECK(c.data != nullptr, VX_EINVAL, "%s: null column with %llu rows", what,
           (unsigned long long)n);
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  hipError_t e = hipPointerGetAttributes(&attr, c.data);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("%s: host pointer %p is not pinned (hipPointerGetAttributes: %s)", what, c.data,
              hipGetErrorString(e));
    return VX_ENOTPINNED;
  }
  if (attr.type == hipMemoryTypeDevice) {
    VX_CHECK(attr.device == ctx->device, VX_EINVAL, "%s: device pointer of device %d, context is on %d",
             what, attr.device, ctx->device);
    out->where = Where::Device;
    out->dev = c.data;
    out->host = nullptr;
    return VX_OK;
  }
  if (attr.type == hipMemoryTypeHost) {
    void* dp = attr.devicePointer;
    if (!dp) {
      if (hipHostGetDevicePointer(&dp, const_cast<void*>(c.data), 0) != hipSuccess) {
        (void)hipGetLastError();
        set_error("%s: pinned host pointer %p has no device mapping", what, c.data);
        return VX_ENOTPINNED;
      }
    }
    out->where = Where::Host;
    out->dev = dp;
    out->host = c.data;
    return VX_OK;
  }
  set_error("%s: pointer %p is pageable host memory (type %d); use vx_host_alloc or pinned memory",
            what, c.data, (int)attr.type);
  return VX_ENOTPINNED;
}

vx_status host_scratch(vx_ctx* ctx, uint64_t bytes, uint8_t** out) {
  if (ctx->host_scratch_bytes < bytes) {
    if (ctx->host_scratch) {
      VX_HIP(hipStreamSynchronize(ctx->d2h));
      VX_HIP(hipHostFree(ctx->host_scratch));
      ctx->host_scratch = nullptr;
      ctx->host_scratch_bytes = 0;
    }
    void* p = nullptr;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocMapped | hipHostMallocPortable);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("host scratch of %llu bytes: %s", (unsigned long long)bytes, hipGetErrorString(e));
      return VX_ENOMEM;
    }
    ctx->host_scratch = (uint8_t*)p;
    ctx->host_scratch_bytes = bytes;
  }
  *out = ctx->host_scratch;
  return VX_OK;
}

hipEvent_t get_event(vx_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void put_event(vx_ctx* ctx, hipEvent_t e) {
  if (e) ctx->ev_pool.push_back(e);
}

__global__ void k_fill_zero(uint64_t* p, uint64_t words) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

void fill_zero(uint64_t* p, uint64_t words, hipStream_t s) {
  if (!words) return;
  uint64_t blocks = (words + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, words);
}

double zc_wire_bytes(uint64_t n, uint64_t count, int elsize, uint32_t line) {
  if (n == 0 || count == 0) return 0.0;
  double s = (double)count / (double)n;
  if (s > 1.0) s = 1.0;
  double per_line = std::max(1.0, (double)line / elsize);
  double lines = (double)n / per_line;
  double touched = 1.0 - std::pow(1.0 - s, per_line);
  return lines * touched * per_line * elsize;
}

}  // namespace vx

using namespace vx;

extern "C" {

const char* vx_last_error(void) { return g_err.c_str(); }

static constexpr uint64_t kAccRows = 1u << 14;   // per-chunk aggregate rows held on the device

vx_status vx_ctx_create(int device, void* arena, uint64_t arena_bytes, void* stream, vx_ctx** out) {
  VX_CHECK(out != nullptr, VX_EINVAL, "vx_ctx_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  VX_HIP(hipGetDeviceCount(&ndev));
  VX_CHECK(device >= 0 && device < ndev, VX_EINVAL, "vx_ctx_create: device %d of %d", device, ndev);
  VX_CHECK(arena != nullptr, VX_EINVAL, "vx_ctx_create: arena is NULL");
  VX_HIP(hipSetDevice(device));
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  if (hipPointerGetAttributes(&attr, arena) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    set_error("vx_ctx_create: arena %p is not device memory", arena);
    return VX_EINVAL;
  }
  vx_ctx* c = new vx_ctx;
  c->device = device;
  c->arena.init((uint8_t*)arena, arena_bytes);
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, device) == hipSuccess) {
    c->cu_count = pr.multiProcessorCount;
    c->l2_bytes = (uint64_t)pr.l2CacheSize;
  }
  c->dev_acc_words = kAccRows * kAccWords;
  const uint64_t scratch_bytes = c->dev_acc_words * 8 + 256 + (kScanTilesMax + 1) * 8;
  uint8_t* scratch = c->arena.alloc(scratch_bytes);
  if (!scratch) {
    delete c;
    set_error("vx_ctx_create: arena of %llu bytes cannot hold the %llu-byte result scratch",
              (unsigned long long)arena_bytes, (unsigned long long)scratch_bytes);
    return VX_EBUDGET;
  }
  c->dev_acc = (uint64_t*)scratch;
  c->dev_flags = (unsigned int*)(scratch + c->dev_acc_words * 8);
  c->dev_scan = (uint64_t*)(scratch + c->dev_acc_words * 8 + 256);
  if (stream) {
    c->compute = (hipStream_t)stream;
  } else {
    // a blocking stream: ordered after work the caller put on the null stream
    if (hipStreamCreate(&c->compute) != hipSuccess) {
      delete c;
      set_error("vx_ctx_create: stream creation failed");
      return VX_EHIP;
    }
    c->own_compute = true;
  }
  if (hipStreamCreateWithFlags(&c->copy, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->d2h, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc((void**)&c->host_acc, (c->dev_acc_words + kHostSmallWords) * 8, hipHostMallocDefault) !=
          hipSuccess) {
    if (c->own_compute) (void)hipStreamDestroy(c->compute);
    if (c->copy) (void)hipStreamDestroy(c->copy);
    if (c->d2h) (void)hipStreamDestroy(c->d2h);
    delete c;
    set_error("vx_ctx_create: stream or pinned scratch creation failed");
    return VX_EHIP;
  }
  c->host_small = c->host_acc + c->dev_acc_words;
  *out = c;
  return VX_OK;
}

vx_status vx_ctx_destroy(vx_ctx* c) {
  if (!c) return VX_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->compute);
  (void)hipStreamSynchronize(c->copy);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own_compute) (void)hipStreamDestroy(c->compute);
  (void)hipStreamSynchronize(c->d2h);
  batch_release_ctx(c);
  (void)hipStreamDestroy(c->copy);
  (void)hipStreamDestroy(c->d2h);
  (void)hipHostFree(c->host_acc);
  if (c->host_scratch) (void)hipHostFree(c->host_scratch);
  delete c;
  return VX_OK;
}

uint64_t vx_ctx_arena_used(const vx_ctx* c) { return c ? c->arena.used() : 0; }

vx_status vx_host_alloc(uint64_t bytes, void** out) {
  VX_CHECK(out != nullptr, VX_EINVAL, "vx_host_alloc: out is NULL");
  *out = nullptr;
  if (bytes == 0) bytes = 1;
  void* p = nullptr;
  hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocMapped | hipHostMallocPortable);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("vx_host_alloc(%llu): %s", (unsigned long long)bytes, hipGetErrorString(e));
    return VX_ENOMEM;
  }
  *out = p;
  return VX_OK;
}

vx_status vx_host_free(void* p) {
  if (p) VX_HIP(hipHostFree(p));
  return VX_OK;
}

}  // extern "C"
