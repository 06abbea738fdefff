// Hash-table build, probe with fused aggregation, and the streamed probe executor.
//
// Build: open addressing with linear probing.  A lane group of G lanes (G = 1, 4 or 8)
// inspects G consecutive slots at once; __ballot finds the first matching or empty slot
// of the window and the lowest such lane claims it with one compare-and-swap.
// Probe: one lane per probe row, several rows per lane in flight, the streamed key
// column read with non-temporal loads so the table stays in L2 / MALL.  Matches are
// aggregated in registers, reduced across the workgroup in LDS and flushed with one
// 64-bit atomic per accumulator per workgroup.  Probe payload columns are read only for
// matching rows, from the chunk buffer or by zero-copy from pinned host memory.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "vx_table.h"

namespace vx {

// ---------------------------------------------------------------- device helpers

template <typename K>
__device__ __forceinline__ uint64_t key_bits(K k) {
  return (uint64_t)(typename KeyTraits<K>::U)k;
}

__device__ __forceinline__ long long load_signed(const void* base, uint64_t idx, uint32_t size) {
  if (size == 4) return (long long)((const int*)base)[idx];
  return ((const long long*)base)[idx];
}

__device__ __forceinline__ long long slot_signed(const uint8_t* slot, uint32_t off, uint32_t size) {
  if (size == 4) return (long long)*(const int*)(slot + off);
  return *(const long long*)(slot + off);
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

// ---------------------------------------------------------------- table init

__global__ void k_init_slots(uint32_t* slots, uint64_t capacity, uint32_t slot_words,
                             uint32_t key_size) {
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < capacity;
       s += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t* w = slots + s * slot_words;
    for (uint32_t i = 0; i < slot_words; ++i) w[i] = 0;
    if (key_size == 4) w[0] = 0x80000000u;
    else w[1] = 0x80000000u;    // little-endian INT64_MIN: low word 0, high word 0x80000000
  }
}

// ---------------------------------------------------------------- build (unique keys)

struct BuildCols {
  const void* key;
  const void* pay[kMaxPay];
  uint32_t pay_size[kMaxPay];
};

template <typename K>
__device__ __forceinline__ void write_unique_payloads(const TableView& t, uint8_t* slot,
                                                      const BuildCols& c, uint64_t row) {
  for (uint32_t p = 0; p < t.n_pay; ++p) {
    if (t.pay_size[p] == 4) *(int*)(slot + t.pay_off[p]) = ((const int*)c.pay[p])[row];
    else *(long long*)(slot + t.pay_off[p]) = ((const long long*)c.pay[p])[row];
  }
}

template <typename K>
__device__ __forceinline__ void side_add(const TableView& t, const BuildCols& c, uint64_t row,
                                         unsigned int* flags, bool unique) {
  unsigned long long prev = atomicAdd(t.side, 1ull);
  if (unique && prev != 0) atomicOr(flags, kFlagDup);
  for (uint32_t p = 0; p < t.n_pay; ++p)
    atomicAdd(t.side + 1 + p, (unsigned long long)load_signed(c.pay[p], row, c.pay_size[p]));
}

// One lane per row.
template <typename K>
__global__ void k_build_unique_lane(TableView t, BuildCols c, uint64_t n, unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    K k = ((const K*)c.key)[i];
    U kb = (U)k;
    if (kb == kEmpty) {
      side_add<K>(t, c, i, flags, true);
      continue;
    }
    uint64_t h = slot_of(key_bits(k), t.log2cap);
    bool done = false;
    for (uint64_t step = 0; step <= t.mask; ++step) {
      uint8_t* slot = t.slots + (h << t.slot_shift);
      U prev = atomicCAS((U*)slot, kEmpty, kb);
      if (prev == kEmpty) {
        write_unique_payloads<K>(t, slot, c, i);
        done = true;
        break;
      }
      if (prev == kb) {
        atomicOr(flags, kFlagDup);
        done = true;
        break;
      }
      h = (h + 1) & t.mask;
    }
    if (!done) atomicOr(flags, kFlagFull);
  }
}

// A group of G lanes per row: the group loads G consecutive slots, ballots for the key
// or an empty slot, and the first empty lane claims it.  Rows of the G lanes of a group
// are handled one after the other.
template <typename K, int G>
__global__ void k_build_unique_group(TableView t, BuildCols c, uint64_t n, unsigned int* flags) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int gbase = lane - gl;
  const unsigned long long gmask = ((G == 64) ? ~0ull : ((1ull << G) - 1)) << gbase;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  // every lane of a wave runs the same number of outer iterations (ballots stay convergent)
  uint64_t first = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t wave_first = first - lane;
  for (uint64_t wb = wave_first; wb < n; wb += stride) {
    uint64_t i = wb + lane;
    bool valid = i < n;
    K mykey = valid ? ((const K*)c.key)[i] : (K)0;
    for (int r = 0; r < G; ++r) {
      int src = gbase + r;
      bool v = __shfl(valid ? 1 : 0, src, 64) != 0;
      if (!v) continue;                       // uniform within the group
      K k = __shfl(mykey, src, 64);
      uint64_t row = wb + src;
      U kb = (U)k;
      if (kb == kEmpty) {
        if (gl == 0) side_add<K>(t, c, row, flags, true);
        continue;
      }
      uint64_t h = slot_of(key_bits(k), t.log2cap);
      bool done = false;
      for (uint64_t step = 0; step <= t.mask; step += G) {
        uint64_t pos = (h + gl) & t.mask;
        uint8_t* slot = t.slots + (pos << t.slot_shift);
        U sk = __atomic_load_n((U*)slot, __ATOMIC_RELAXED);
        unsigned long long hit = __ballot(sk == kb) & gmask;
        unsigned long long emp = __ballot(sk == kEmpty) & gmask;
        // the earliest event in probe order decides
        if (hit && (!emp || __ffsll((long long)hit) <= __ffsll((long long)emp))) {
          if (gl == 0) atomicOr(flags, kFlagDup);
          done = true;
          break;
        }
        if (emp) {
          int leader = __ffsll((long long)emp) - 1;
          int won = 0;
          if (lane == leader) {
            U prev = atomicCAS((U*)slot, kEmpty, kb);
            if (prev == kEmpty) {
              write_unique_payloads<K>(t, slot, c, row);
              won = 1;
            } else if (prev == kb) {
              atomicOr(flags, kFlagDup);
              won = 2;
            }
          }
          won = __shfl(won, leader, 64);
          if (won) {
            done = true;
            break;
          }
          step -= G;          // lost the race: re-read the same window
          continue;
        }
        h = (h + G) & t.mask;
      }
      if (!done && gl == 0) atomicOr(flags, kFlagFull);
    }
  }
}

// ---------------------------------------------------------------- build (pre-aggregated)

// Rows are first combined per workgroup tile in an LDS table (so a hot key costs one
// global update per tile), then flushed into the global table with 64-bit atomics.
constexpr int kPreaggLds = 1024;
constexpr int kPreaggTile = 4096;
constexpr int kPreaggProbe = 32;

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
  uint64_t h = slot_of(key_bits(k), t.log2cap);
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

template <typename K>
__global__ void __launch_bounds__(256) k_build_preagg(TableView t, BuildCols c, uint64_t n,
                                                      unsigned int* flags) {
  __shared__ unsigned long long lkey[kPreaggLds];
  __shared__ unsigned long long lcnt[kPreaggLds];
  __shared__ unsigned long long lsum[kMaxPay][kPreaggLds];
  const unsigned long long kFree = ~0ull;     // LDS marker; real keys are stored as 64-bit
  const unsigned long long kFreeAlt = ~0ull - 1;
  for (uint64_t base = (uint64_t)blockIdx.x * kPreaggTile; base < n;
       base += (uint64_t)gridDim.x * kPreaggTile) {
    for (int j = threadIdx.x; j < kPreaggLds; j += blockDim.x) {
      lkey[j] = kFree;
      lcnt[j] = 0;
      for (uint32_t p = 0; p < kMaxPay; ++p) lsum[p][j] = 0;
    }
    __syncthreads();
    uint64_t end = base + kPreaggTile < n ? base + kPreaggTile : n;
    for (uint64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
      K k = ((const K*)c.key)[i];
      unsigned long long kb = (unsigned long long)(long long)k;
      unsigned long long vals[kMaxPay];
      for (uint32_t p = 0; p < t.n_pay; ++p)
        vals[p] = (unsigned long long)load_signed(c.pay[p], i, c.pay_size[p]);
      bool placed = false;
      if (kb != kFree && kb != kFreeAlt) {     // those two key values bypass LDS
        uint32_t h = (uint32_t)(slot_of(kb, 10));
        for (int s = 0; s < kPreaggProbe; ++s) {
          uint32_t j = (h + s) & (kPreaggLds - 1);
          unsigned long long prev = atomicCAS(&lkey[j], kFree, kb);
          if (prev == kFree || prev == kb) {
            atomicAdd(&lcnt[j], 1ull);
            for (uint32_t p = 0; p < t.n_pay; ++p) atomicAdd(&lsum[p][j], vals[p]);
            placed = true;
            break;
          }
        }
      }
      if (!placed) global_preagg_add<K>(t, k, 1ull, vals, flags);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kPreaggLds; j += blockDim.x) {
      if (lkey[j] != kFree) {
        unsigned long long sums[kMaxPay];
        for (uint32_t p = 0; p < kMaxPay; ++p) sums[p] = lsum[p][j];
        global_preagg_add<K>(t, (K)(long long)lkey[j], lcnt[j], sums, flags);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- probe

struct ProbeCols {
  const void* key;            // keys of this launch, key[0] is global row row0
  uint64_t n;
  uint64_t row0;
  uint32_t n_pay;
  uint32_t pay_global;        // bit c: pay[c] is indexed by global row (resident / zero-copy)
  const void* pay[kMaxPay];
  uint32_t pay_size[kMaxPay];
};

template <typename K, bool PREAGG, int ITEMS>
__global__ void __launch_bounds__(256) k_probe(TableView t, ProbeCols q, unsigned long long* acc_out) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  constexpr int NACC = 9;
  unsigned long long acc[NACC];
#pragma unroll
  for (int a = 0; a < NACC; ++a) acc[a] = 0;
  const uint32_t nb = t.n_pay;
  const uint64_t tile = (uint64_t)blockDim.x * ITEMS;
  for (uint64_t base = blockIdx.x * tile; base < q.n; base += (uint64_t)gridDim.x * tile) {
    unsigned long long mb[ITEMS];
    K keys[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      keys[j] = i < q.n ? __builtin_nontemporal_load(((const K*)q.key) + i) : (K)0;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      mb[j] = 0;
      if (i >= q.n) continue;
      U kb = (U)keys[j];
      if (kb == kEmpty) {
        unsigned long long c = t.side[0];
        if (c) {
          mb[j] = c;
          acc[0] += c;
          for (uint32_t p = 0; p < nb; ++p) acc[1 + p] += t.side[1 + p];
        }
        continue;
      }
      uint64_t h = slot_of(key_bits(keys[j]), t.log2cap);
      for (uint64_t step = 0; step <= t.mask; ++step) {
        const uint8_t* slot = t.slots + (h << t.slot_shift);
        U sk = *(const U*)slot;
        if (sk == kb) {
          if (PREAGG) {
            const unsigned long long* w = (const unsigned long long*)(slot + 8);
            mb[j] = w[0];
            acc[0] += w[0];
            for (uint32_t p = 0; p < nb; ++p) acc[1 + p] += w[1 + p];
          } else {
            mb[j] = 1;
            acc[0] += 1;
            for (uint32_t p = 0; p < nb; ++p)
              acc[1 + p] += (unsigned long long)slot_signed(slot, t.pay_off[p], t.pay_size[p]);
          }
          break;
        }
        if (sk == kEmpty) break;
        h = (h + 1) & t.mask;
      }
    }
    // late materialization: probe payloads of matching rows only
    for (uint32_t p = 0; p < q.n_pay; ++p) {
      const bool glob = (q.pay_global >> p) & 1u;
      long long v[ITEMS];
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
        v[j] = mb[j] ? load_signed(q.pay[p], glob ? q.row0 + i : i, q.pay_size[p]) : 0;
      }
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) acc[1 + nb + p] += mb[j] * (unsigned long long)v[j];
    }
  }
  block_flush<NACC>(acc, 1 + (int)nb + (int)q.n_pay, acc_out);
}

// ---------------------------------------------------------------- host side

static int ilog2(uint64_t v) {
  int r = 0;
  while ((1ull << r) < v) ++r;
  return r;
}

vx_status make_table(vx_ctx* ctx, int32_t key_type, uint32_t flags, const int32_t* pay_types,
                     uint32_t n_pay, uint64_t expected_rows, float load_factor, vx_table** out) {
  *out = nullptr;
  VX_CHECK(n_pay <= kMaxPay, VX_EINVAL, "build: at most %u payload columns", kMaxPay);
  int ks = elsize_of(key_type);
  VX_CHECK(ks != 0, VX_EINVAL, "build: bad key type %d", key_type);
  bool preagg = (flags & VX_PREAGG) != 0;
  float lf = load_factor > 0 ? load_factor : 0.5f;
  VX_CHECK(lf > 0.05f && lf <= 0.95f, VX_EINVAL, "build: load factor %f outside (0.05, 0.95]", lf);
  uint64_t want = (uint64_t)std::ceil((double)(expected_rows ? expected_rows : 1) / lf);
  uint64_t cap = 64;
  while (cap < want) cap <<= 1;
  TableView v{};
  v.n_pay = n_pay;
  v.preagg = preagg ? 1 : 0;
  v.key_size = (uint32_t)ks;
  uint32_t off;
  if (preagg) {
    off = 16;   // key (8), count (8)
    for (uint32_t p = 0; p < n_pay; ++p) {
      v.pay_off[p] = off;
      v.pay_size[p] = 8;
      off += 8;
    }
  } else {
    off = (uint32_t)ks;
    for (uint32_t p = 0; p < n_pay; ++p) {
      int ps = elsize_of(pay_types[p]);
      VX_CHECK(ps != 0, VX_EINVAL, "build: bad payload type %d", pay_types[p]);
      off = (off + ps - 1) / ps * ps;
      v.pay_off[p] = off;
      v.pay_size[p] = (uint32_t)ps;
      off += ps;
    }
  }
  uint32_t slot_bytes = 8;
  while (slot_bytes < off) slot_bytes <<= 1;
  v.slot_shift = (uint32_t)ilog2(slot_bytes);
  v.log2cap = (uint32_t)ilog2(cap);
  v.mask = cap - 1;
  uint64_t bytes = cap * slot_bytes + 256;
  uint8_t* mem = ctx->arena.alloc(bytes);
  VX_CHECK(mem != nullptr, VX_EBUDGET,
           "build: hash table of %llu slots x %u B = %llu B does not fit the arena (%llu B free, "
           "largest block %llu B)",
           (unsigned long long)cap, slot_bytes, (unsigned long long)bytes,
           (unsigned long long)(ctx->arena.capacity() - ctx->arena.used()),
           (unsigned long long)ctx->arena.largest_free());
  v.slots = mem;
  v.side = (unsigned long long*)(mem + cap * slot_bytes);
  vx_table* t = new vx_table;
  t->ctx = ctx;
  t->mem = mem;
  t->bytes = bytes;
  t->capacity = cap;
  t->key_type = key_type;
  t->flags = flags;
  for (uint32_t p = 0; p < n_pay; ++p) t->pay_type[p] = (uint32_t)pay_types[p];
  t->view = v;
  uint64_t blocks = std::min<uint64_t>((cap + 255) / 256, 8192);
  hipLaunchKernelGGL(k_init_slots, dim3((unsigned)blocks), dim3(256), 0, ctx->compute,
                     (uint32_t*)mem, cap, slot_bytes / 4, (uint32_t)ks);
  fill_zero((uint64_t*)v.side, 32, ctx->compute);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->arena.release(mem);
    delete t;
    set_error("build: init kernel launch failed: %s", hipGetErrorString(e));
    return VX_EHIP;
  }
  *out = t;
  return VX_OK;
}

vx_status check_flags(vx_ctx* ctx, const char* what) {
  unsigned int f = 0;
  VX_HIP(hipMemcpyAsync(&f, ctx->dev_flags, sizeof f, hipMemcpyDeviceToHost, ctx->compute));
  VX_HIP(hipStreamSynchronize(ctx->compute));
  if (f & kFlagDup) {
    set_error("%s: duplicate key in a build declared unique", what);
    return VX_EDUPKEY;
  }
  if (f & kFlagFull) {
    set_error("%s: hash table full (internal sizing error)", what);
    return VX_ECAPACITY;
  }
  if (f & kFlagGroupOverflow) {
    set_error("%s: group table overflow", what);
    return VX_ECAPACITY;
  }
  return VX_OK;
}

static unsigned grid_for(vx_ctx* ctx, uint64_t work_items, uint64_t per_block, unsigned per_cu) {
  uint64_t blocks = (work_items + per_block - 1) / per_block;
  uint64_t cap = (uint64_t)ctx->cu_count * per_cu;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

vx_status table_insert(vx_ctx* ctx, vx_table* t, const ColInfo& key, const ColInfo* pays,
                       uint64_t n, hipStream_t s, int group_lanes) {
  if (n == 0) return VX_OK;
  BuildCols c{};
  c.key = key.dev;
  for (uint32_t p = 0; p < t->view.n_pay; ++p) {
    c.pay[p] = pays[p].dev;
    c.pay_size[p] = (uint32_t)pays[p].elsize;
  }
  const bool k64 = t->key_type == VX_I64;
  if (t->view.preagg) {
    unsigned g = grid_for(ctx, n, kPreaggTile, 3);
    if (k64) hipLaunchKernelGGL(k_build_preagg<int64_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
    else hipLaunchKernelGGL(k_build_preagg<int32_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
  } else {
    unsigned g = grid_for(ctx, n, 256, 8);
    switch (group_lanes) {
      case 1:
        if (k64) hipLaunchKernelGGL(k_build_unique_lane<int64_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        else hipLaunchKernelGGL(k_build_unique_lane<int32_t>, dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        break;
      case 4:
        if (k64) hipLaunchKernelGGL((k_build_unique_group<int64_t, 4>), dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        else hipLaunchKernelGGL((k_build_unique_group<int32_t, 4>), dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        break;
      default:
        if (k64) hipLaunchKernelGGL((k_build_unique_group<int64_t, 8>), dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        else hipLaunchKernelGGL((k_build_unique_group<int32_t, 8>), dim3(g), dim3(256), 0, s, t->view, c, n, ctx->dev_flags);
        break;
    }
  }
  VX_HIP(hipGetLastError());
  t->n_rows += n;
  return VX_OK;
}

// Launch one probe kernel over q.n rows, accumulating into acc (9 words).
static vx_status launch_probe(vx_ctx* ctx, const vx_table* t, const ProbeCols& q,
                              unsigned long long* acc, hipStream_t s) {
  if (q.n == 0) return VX_OK;
  constexpr int ITEMS = 4;
  unsigned g = grid_for(ctx, q.n, 256 * ITEMS, 8);
  const bool k64 = t->key_type == VX_I64;
  if (t->view.preagg) {
    if (k64) hipLaunchKernelGGL((k_probe<int64_t, true, ITEMS>), dim3(g), dim3(256), 0, s, t->view, q, acc);
    else hipLaunchKernelGGL((k_probe<int32_t, true, ITEMS>), dim3(g), dim3(256), 0, s, t->view, q, acc);
  } else {
    if (k64) hipLaunchKernelGGL((k_probe<int64_t, false, ITEMS>), dim3(g), dim3(256), 0, s, t->view, q, acc);
    else hipLaunchKernelGGL((k_probe<int32_t, false, ITEMS>), dim3(g), dim3(256), 0, s, t->view, q, acc);
  }
  VX_HIP(hipGetLastError());
  return VX_OK;
}

int build_group_lanes() {
  const char* e = getenv("VX_BUILD_LANES");
  int g = e ? atoi(e) : 8;
  return (g == 1 || g == 4 || g == 8) ? g : 8;
}

// ---------------------------------------------------------------- streamed probe executor

struct ProbePlan {
  uint64_t chunk_rows = 0;
  uint32_t n_buffers = 2;
  uint64_t buf_bytes = 0;
};

static uint64_t env_u64(const char* name, uint64_t dflt) {
  const char* e = getenv(name);
  return e ? strtoull(e, nullptr, 10) : dflt;
}

vx_status probe_impl(vx_ctx* ctx, const vx_table* t, const vx_probe_desc* d, vx_agg* out,
                     vx_stats* st) {
  double t0 = now_ms();
  VX_CHECK(d->key.type == t->key_type, VX_EINVAL, "probe: key type %d differs from the table's %d",
           d->key.type, t->key_type);
  VX_CHECK(d->n_pay <= kMaxPay, VX_EINVAL, "probe: at most %u payload columns", kMaxPay);
  VX_CHECK(d->n_pay == 0 || d->pay != nullptr, VX_EINVAL, "probe: pay is NULL");
  VX_CHECK(t->view.n_pay + d->n_pay <= 8, VX_EINVAL, "probe: more than 8 aggregate sums");
  VX_CHECK(d->late_mat >= -1 && d->late_mat <= 2, VX_EINVAL, "probe: late_mat %d", d->late_mat);
  ColInfo kc;
  VX_TRY(classify(ctx, d->key, d->n, &kc, "probe key"));
  ColInfo pc[kMaxPay];
  for (uint32_t p = 0; p < d->n_pay; ++p) VX_TRY(classify(ctx, d->pay[p], d->n, &pc[p], "probe payload"));
  VX_HIP(hipSetDevice(ctx->device));
  const uint64_t n = d->n;
  const int ks = kc.elsize;
  const uint32_t nacc = 1 + t->view.n_pay + d->n_pay;
  vx_stats s{};
  s.rows = n;
  s.table_bytes = t->bytes;
  std::vector<unsigned long long> total(kAccWords, 0);

  // chunking
  bool streamed = kc.where == Where::Host;
  uint64_t chunk_rows;
  if (d->chunk_rows) chunk_rows = d->chunk_rows;
  else if (streamed) chunk_rows = env_u64("VX_CHUNK_BYTES", 64ull << 20) / (uint64_t)ks;
  else chunk_rows = n ? n : 1;
  if (chunk_rows == 0) chunk_rows = 1;
  uint64_t n_chunks = n ? (n + chunk_rows - 1) / chunk_rows : 0;
  uint64_t acc_rows_cap = ctx->dev_acc_words / kAccWords;

  // per-column late materialization decision (streamed path only): zero-copy or SDMA
  uint32_t zc_mask = 0;
  bool decide_after_first = false;
  if (streamed) {
    if (d->late_mat == VX_LATE_ZC) zc_mask = (1u << d->n_pay) - 1;
    else if (d->late_mat == VX_LATE_SDMA) zc_mask = 0;
    else {
      zc_mask = (1u << d->n_pay) - 1;    // the first chunk runs zero-copy and measures selectivity
      decide_after_first = d->n_pay > 0 && n_chunks > 1;
    }
  }
  // payload columns that are device-resident are always read in place
  for (uint32_t p = 0; p < d->n_pay; ++p)
    if (pc[p].where == Where::Device) zc_mask |= 1u << p;

  uint32_t nbuf = d->n_buffers ? d->n_buffers : (uint32_t)env_u64("VX_BUFFERS", 2);
  VX_CHECK(nbuf >= 2 && nbuf <= 4, VX_EINVAL, "probe: n_buffers %u outside 2..4", nbuf);

  // buffers: keys + every payload column that may be copied
  uint64_t row_bytes = (uint64_t)ks;
  for (uint32_t p = 0; p < d->n_pay; ++p)
    if (pc[p].where == Where::Host && d->late_mat != VX_LATE_ZC) row_bytes += (uint64_t)pc[p].elsize;
  ArenaBlock bufs[4];
  uint64_t buf_bytes = 0;
  if (streamed && n) {
    if (chunk_rows > n) chunk_rows = n;
    // shrink chunks until the pipeline fits the free arena
    for (;;) {
      buf_bytes = chunk_rows * row_bytes + 256 * (1 + kMaxPay);
      bool ok = true;
      for (uint32_t b = 0; b < nbuf; ++b) {
        bufs[b].a = &ctx->arena;
        bufs[b].p = ctx->arena.alloc(buf_bytes);
        if (!bufs[b].p) ok = false;
      }
      if (ok) break;
      for (uint32_t b = 0; b < nbuf; ++b) bufs[b].reset();
      VX_CHECK(chunk_rows > 1024 && !d->chunk_rows, VX_EBUDGET,
               "probe: %u chunk buffers of %llu rows x %llu B do not fit the arena (%llu B free)",
               nbuf, (unsigned long long)chunk_rows, (unsigned long long)row_bytes,
               (unsigned long long)(ctx->arena.capacity() - ctx->arena.used()));
      chunk_rows /= 2;
    }
    n_chunks = (n + chunk_rows - 1) / chunk_rows;
  }
  s.chunk_rows = chunk_rows;
  s.chunks = streamed ? n_chunks : 0;
  s.n_buffers = streamed ? nbuf : 0;

  uint64_t acc_rows = std::min<uint64_t>(std::max<uint64_t>(n_chunks, 1), acc_rows_cap);
  fill_zero((uint64_t*)ctx->dev_acc, acc_rows * kAccWords, ctx->compute);
  fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);

  std::vector<hipEvent_t> ev_copied(nbuf), ev_free(nbuf);
  std::vector<bool> free_pending(nbuf, false);
  hipEvent_t k_beg = get_event(ctx), k_end = get_event(ctx);
  std::vector<std::pair<hipEvent_t, hipEvent_t>> kev;
  for (uint32_t b = 0; b < nbuf; ++b) {
    ev_copied[b] = get_event(ctx);
    ev_free[b] = get_event(ctx);
  }
  auto cleanup = [&]() {
    for (uint32_t b = 0; b < nbuf; ++b) {
      put_event(ctx, ev_copied[b]);
      put_event(ctx, ev_free[b]);
    }
    for (auto& pr : kev) {
      put_event(ctx, pr.first);
      put_event(ctx, pr.second);
    }
    put_event(ctx, k_beg);
    put_event(ctx, k_end);
  };

  auto chunk_layout = [&](uint32_t b, uint64_t rows, const void** key_dst, const void** pay_dst) {
    uint8_t* base = bufs[b].p;
    *key_dst = base;
    uint64_t off = (rows * (uint64_t)ks + 255) / 256 * 256;
    for (uint32_t p = 0; p < d->n_pay; ++p) {
      pay_dst[p] = nullptr;
      if (pc[p].where == Where::Host && !((zc_mask >> p) & 1u)) {
        pay_dst[p] = base + off;
        off += (rows * (uint64_t)pc[p].elsize + 255) / 256 * 256;
      }
    }
  };

  vx_status status = VX_OK;
  double tk0 = now_ms();
  if (!streamed) {
    // device-resident keys: probe in place, one launch per chunk (chunks only matter for
    // per-chunk aggregates)
    for (uint64_t c = 0; c < n_chunks && status == VX_OK; ++c) {
      uint64_t r0 = c * chunk_rows, rows = std::min(chunk_rows, n - r0);
      ProbeCols q{};
      q.key = (const uint8_t*)kc.dev + r0 * ks;
      q.n = rows;
      q.row0 = r0;
      q.n_pay = d->n_pay;
      for (uint32_t p = 0; p < d->n_pay; ++p) {
        q.pay[p] = pc[p].dev;
        q.pay_size[p] = (uint32_t)pc[p].elsize;
        q.pay_global |= 1u << p;
      }
      hipEvent_t a = get_event(ctx), b2 = get_event(ctx);
      kev.push_back({a, b2});
      (void)hipEventRecord(a, ctx->compute);
      status = launch_probe(ctx, t, q, (unsigned long long*)ctx->dev_acc + (c % acc_rows) * kAccWords,
                            ctx->compute);
      (void)hipEventRecord(b2, ctx->compute);
    }
  } else {
    // Pipelined executor: buffer b = chunk % nbuf.  A copy is enqueued only once its buffer
    // is free (the host waits for the kernel that last read it), so it starts at once.
    uint64_t issued = 0;
    auto issue_copy = [&](uint64_t c) -> vx_status {
      uint32_t b = (uint32_t)(c % nbuf);
      if (free_pending[b]) {
        VX_HIP(hipEventSynchronize(ev_free[b]));
        free_pending[b] = false;
      }
      uint64_t r0 = c * chunk_rows, rows = std::min(chunk_rows, n - r0);
      const void* kd;
      const void* pd[kMaxPay];
      chunk_layout(b, rows, &kd, pd);
      VX_HIP(hipMemcpyAsync(const_cast<void*>(kd), (const uint8_t*)kc.host + r0 * ks, rows * ks,
                            hipMemcpyHostToDevice, ctx->copy));
      s.sdma_bytes += rows * ks;
      for (uint32_t p = 0; p < d->n_pay; ++p) {
        if (!pd[p]) continue;
        uint64_t es = (uint64_t)pc[p].elsize;
        VX_HIP(hipMemcpyAsync(const_cast<void*>(pd[p]), (const uint8_t*)pc[p].host + r0 * es,
                              rows * es, hipMemcpyHostToDevice, ctx->copy));
        s.sdma_bytes += rows * es;
      }
      VX_HIP(hipEventRecord(ev_copied[b], ctx->copy));
      return VX_OK;
    };
    auto issue_kernel = [&](uint64_t c) -> vx_status {
      uint32_t b = (uint32_t)(c % nbuf);
      uint64_t r0 = c * chunk_rows, rows = std::min(chunk_rows, n - r0);
      const void* kd;
      const void* pd[kMaxPay];
      chunk_layout(b, rows, &kd, pd);
      VX_HIP(hipStreamWaitEvent(ctx->compute, ev_copied[b], 0));
      ProbeCols q{};
      q.key = kd;
      q.n = rows;
      q.row0 = r0;
      q.n_pay = d->n_pay;
      for (uint32_t p = 0; p < d->n_pay; ++p) {
        q.pay_size[p] = (uint32_t)pc[p].elsize;
        if (pd[p]) q.pay[p] = pd[p];
        else {
          q.pay[p] = pc[p].dev;
          q.pay_global |= 1u << p;
        }
      }
      hipEvent_t a = get_event(ctx), e2 = get_event(ctx);
      kev.push_back({a, e2});
      VX_HIP(hipEventRecord(a, ctx->compute));
      VX_TRY(launch_probe(ctx, t, q, (unsigned long long*)ctx->dev_acc + (c % acc_rows) * kAccWords,
                          ctx->compute));
      VX_HIP(hipEventRecord(e2, ctx->compute));
      VX_HIP(hipEventRecord(ev_free[b], ctx->compute));
      free_pending[b] = true;
      return VX_OK;
    };
    auto run = [&]() -> vx_status {
      if (n_chunks == 0) return VX_OK;
      uint64_t start = 0;
      if (decide_after_first) {
        VX_TRY(issue_copy(0));
        VX_TRY(issue_kernel(0));
        unsigned long long first[kAccWords];
        VX_HIP(hipMemcpyAsync(first, ctx->dev_acc, sizeof first, hipMemcpyDeviceToHost, ctx->compute));
        VX_HIP(hipStreamSynchronize(ctx->compute));
        uint64_t rows0 = std::min(chunk_rows, n);
        double sel = rows0 ? (double)first[0] / (double)rows0 : 0.0;
        // note: match_count counts pairs; for unique build keys it is the matching-row count
        for (uint32_t p = 0; p < d->n_pay; ++p) {
          if (pc[p].where != Where::Host) continue;
          int es = pc[p].elsize;
          bool zc;
          if (d->late_mat == VX_LATE_PAPER) {
            zc = sel < (double)es / (double)kZcLine;       // TH = E / (C_l2 * N_exchange), N = 1
          } else {
            double wire = zc_wire_bytes(rows0, first[0] < rows0 ? first[0] : rows0, es) / rows0;
            zc = wire < 0.95 * es;
          }
          if (!zc) zc_mask &= ~(1u << p);
        }
        start = 1;
        issued = 1;
      }
      // prologue: fill the buffers
      uint64_t ahead = std::min<uint64_t>(n_chunks, start + nbuf - 1);
      for (uint64_t c = std::max(issued, start); c < ahead; ++c) VX_TRY(issue_copy(c));
      issued = std::max(issued, ahead);
      for (uint64_t c = start; c < n_chunks; ++c) {
        VX_TRY(issue_kernel(c));
        if (issued < n_chunks) {
          VX_TRY(issue_copy(issued));
          ++issued;
        }
      }
      return VX_OK;
    };
    status = run();
  }
  if (status != VX_OK) {
    (void)hipStreamSynchronize(ctx->copy);
    (void)hipStreamSynchronize(ctx->compute);
    cleanup();
    return status;
  }
  // per-chunk aggregates back to the host
  hipError_t e = hipMemcpyAsync(ctx->host_acc, ctx->dev_acc, acc_rows * kAccWords * 8,
                                hipMemcpyDeviceToHost, ctx->compute);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->compute);
  if (e != hipSuccess) {
    cleanup();
    set_error("probe: %s", hipGetErrorString(e));
    return VX_EHIP;
  }
  double tk1 = now_ms();
  double kms = 0;
  for (auto& pr : kev) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) kms += ms;
  }
  s.kernel_ms = kms;
  s.kernel_launches = kev.size();
  cleanup();
  for (uint64_t r = 0; r < acc_rows; ++r)
    for (int a = 0; a < kAccWords; ++a) total[a] += ctx->host_acc[r * kAccWords + a];
  if (d->chunk_aggs) {
    VX_CHECK(n_chunks <= d->chunk_aggs_cap && n_chunks <= acc_rows_cap, VX_ECAPACITY,
             "probe: %llu chunks exceed chunk_aggs_cap %llu", (unsigned long long)n_chunks,
             (unsigned long long)d->chunk_aggs_cap);
    for (uint64_t c = 0; c < n_chunks; ++c) {
      vx_agg& ca = d->chunk_aggs[c];
      std::memset(&ca, 0, sizeof ca);
      ca.match_count = ctx->host_acc[c * kAccWords];
      for (uint32_t a = 1; a < nacc; ++a) ca.sum[a - 1] = ctx->host_acc[c * kAccWords + a];
    }
  }
  std::memset(out, 0, sizeof *out);
  out->match_count = total[0];
  for (uint32_t a = 1; a < nacc; ++a) out->sum[a - 1] = total[a];
  // zero-copy wire estimate from per-chunk match counts (unique keys: matches = rows)
  for (uint32_t p = 0; p < d->n_pay; ++p) {
    if (pc[p].where != Where::Host || !((zc_mask >> p) & 1u)) continue;
    for (uint64_t c = 0; c < n_chunks; ++c) {
      uint64_t rows = std::min(chunk_rows, n - c * chunk_rows);
      uint64_t m = c < acc_rows ? ctx->host_acc[c * kAccWords] : 0;
      s.zc_bytes_est += (uint64_t)zc_wire_bytes(rows, std::min(m, rows), pc[p].elsize);
    }
  }
  s.zc_mask = zc_mask;
  s.probe_ms = tk1 - tk0;
  s.total_ms = now_ms() - t0;
  if (st) *st = s;
  return VX_OK;
}

vx_status build_impl(vx_ctx* ctx, const vx_build_desc* d, vx_table** out, double* ms) {
  double t0 = now_ms();
  VX_CHECK(d != nullptr && out != nullptr, VX_EINVAL, "vx_build: null argument");
  *out = nullptr;
  VX_CHECK(d->flags == VX_UNIQUE || d->flags == VX_PREAGG, VX_EINVAL,
           "vx_build: flags must be VX_UNIQUE or VX_PREAGG");
  VX_CHECK(d->n_pay <= kMaxPay, VX_EINVAL, "vx_build: at most %u payload columns", kMaxPay);
  VX_CHECK(d->n_pay == 0 || d->pay != nullptr, VX_EINVAL, "vx_build: pay is NULL");
  ColInfo kc;
  VX_TRY(classify(ctx, d->key, d->n, &kc, "build key"));
  ColInfo pc[kMaxPay];
  int32_t pt[kMaxPay];
  for (uint32_t p = 0; p < d->n_pay; ++p) {
    VX_TRY(classify(ctx, d->pay[p], d->n, &pc[p], "build payload"));
    pt[p] = d->pay[p].type;
  }
  VX_HIP(hipSetDevice(ctx->device));
  vx_table* t = nullptr;
  VX_TRY(make_table(ctx, d->key.type, d->flags, pt, d->n_pay, d->n, d->load_factor, &t));
  fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);
  vx_status st = table_insert(ctx, t, kc, pc, d->n, ctx->compute, build_group_lanes());
  if (st == VX_OK) st = check_flags(ctx, "vx_build");
  if (st != VX_OK) {
    ctx->arena.release(t->mem);
    delete t;
    return st;
  }
  *out = t;
  if (ms) *ms = now_ms() - t0;
  return VX_OK;
}

vx_status join_star(vx_ctx* ctx, const vx_star_join* d, vx_join_out* out);
vx_status join_batch(vx_ctx* ctx, const vx_batch_join* d, vx_join_out* out);
vx_status join_partitioned(vx_ctx* ctx, const vx_partitioned_join* d, vx_join_out* out);

}  // namespace vx

using namespace vx;

extern "C" {

vx_status vx_build(vx_ctx* ctx, const vx_build_desc* d, vx_table** out) {
  VX_CHECK(ctx != nullptr, VX_EINVAL, "vx_build: ctx is NULL");
  return build_impl(ctx, d, out, nullptr);
}

vx_status vx_table_destroy(vx_table* t) {
  if (!t) return VX_OK;
  (void)hipStreamSynchronize(t->ctx->compute);
  t->ctx->arena.release(t->mem);
  delete t;
  return VX_OK;
}

vx_status vx_probe_stream(vx_ctx* ctx, const vx_table* t, const vx_probe_desc* d, vx_agg* out,
                          vx_stats* st) {
  VX_CHECK(ctx && t && d && out, VX_EINVAL, "vx_probe_stream: null argument");
  VX_CHECK(t->ctx == ctx, VX_EINVAL, "vx_probe_stream: table belongs to another context");
  return probe_impl(ctx, t, d, out, st);
}

vx_status vx_join_agg(vx_ctx* ctx, const vx_join_desc* d, vx_join_out* out) {
  VX_CHECK(ctx && d && out, VX_EINVAL, "vx_join_agg: null argument");
  std::memset(out, 0, sizeof *out);
  switch (d->kind) {
    case VX_JOIN_PLAIN: {
      double t0 = now_ms(), bms = 0;
      vx_table* t = nullptr;
      VX_TRY(build_impl(ctx, &d->u.plain.build, &t, &bms));
      vx_status st = probe_impl(ctx, t, &d->u.plain.probe, &out->agg, &out->stats);
      vx_table_destroy(t);
      out->stats.build_ms = bms;
      out->stats.total_ms = now_ms() - t0;
      return st;
    }
    case VX_JOIN_STAR: return join_star(ctx, &d->u.star, out);
    case VX_JOIN_BATCH: return join_batch(ctx, &d->u.batch, out);
    case VX_JOIN_PARTITIONED: return join_partitioned(ctx, &d->u.part, out);
    default: break;
  }
  set_error("vx_join_agg: unknown kind %d", d->kind);
  return VX_EINVAL;
}

}  // extern "C"
