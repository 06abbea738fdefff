// Partitioned join for a build side larger than the device budget.
//
// Pass 1 (the paper's radix-partition step, Sec. 6.2.1): both tables stream through the chunk
// pipeline; each chunk is clustered by partition on the GPU (stable multisplit) and written back
// to pinned host memory together with its boundary array, on a device-to-host stream that runs
// beside the host-to-device copies.  Pass 2 (Sec. 6.2.2): for each partition, its segments of
// every clustered chunk are located through the boundary arrays and read in place by zero-copy;
// a pre-aggregating hash table (key -> count, payload sums) is built from the build segments
// and probed with the probe segments.
//
// With range partitioning (learned or sample-quantile splitters) a key that carries several
// quantiles gets a partition of its own.  Such a singleton partition never goes through
// pass 2: pass 1 already counts its build rows, sums their payload and counts its probe rows,
// and its contribution is count_b * count_p pairs and sum_b * count_p.
#include <algorithm>
#include <cstring>
#include <vector>

#include "vx_cdf.h"
#include "vx_device.h"
#include "vx_part.h"
#include "vx_pipeline.h"

namespace vx {

vx_status make_spec(vx_ctx* ctx, const vx_part_opts& o, uint32_t n_parts, const int64_t* host_split,
                    uint32_t n_split, ArenaBlock& split_mem, PartSpec* ps);

constexpr uint32_t kMaxSegs = 1024;

struct SegList {
  const unsigned long long* start;    // first source row of each segment
  const unsigned long long* prefix;   // flattened start of each segment; prefix[nseg] = total
  uint32_t nseg;
  uint64_t total;
};

// source row of flattened index idx (the last segment whose prefix is <= idx)
__device__ __forceinline__ uint64_t seg_source(const unsigned long long* st,
                                               const unsigned long long* pre, uint32_t nseg,
                                               uint64_t idx) {
  uint32_t lo = 0, hi = nseg;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= idx) lo = mid;
    else hi = mid;
  }
  return st[lo] + (idx - pre[lo]);
}

__global__ void k_pj_init(uint32_t* slots, uint64_t capacity, uint32_t slot_words, uint32_t key_size,
                          unsigned long long* side) {
  for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < capacity;
       s += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t* w = slots + s * slot_words;
    for (uint32_t i = 0; i < slot_words; ++i) w[i] = 0;
    if (key_size == 4) w[0] = 0x80000000u;
    else w[1] = 0x80000000u;
  }
  if (blockIdx.x == 0 && threadIdx.x < 1 + kMaxPay) side[threadIdx.x] = 0;
}

constexpr int kPjLds = 1024;
constexpr int kPjTile = 4096;

template <typename K>
__global__ void __launch_bounds__(256) k_pj_build(TableView t, const void* key, const void* pay0,
                                                  uint32_t pay_size, SegList sl, unsigned int* flags) {
  __shared__ unsigned long long sst[kMaxSegs], spre[kMaxSegs + 1];
  __shared__ unsigned long long lkey[kPjLds], lcnt[kPjLds], lsum[kPjLds];
  const unsigned long long kFree = ~0ull;
  for (uint32_t j = threadIdx.x; j < sl.nseg; j += blockDim.x) sst[j] = sl.start[j];
  for (uint32_t j = threadIdx.x; j <= sl.nseg; j += blockDim.x) spre[j] = sl.prefix[j];
  __syncthreads();
  for (uint64_t base = (uint64_t)blockIdx.x * kPjTile; base < sl.total;
       base += (uint64_t)gridDim.x * kPjTile) {
    for (int j = threadIdx.x; j < kPjLds; j += blockDim.x) {
      lkey[j] = kFree;
      lcnt[j] = 0;
      lsum[j] = 0;
    }
    __syncthreads();
    uint64_t end = base + kPjTile < sl.total ? base + kPjTile : sl.total;
    for (uint64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
      uint64_t src = seg_source(sst, spre, sl.nseg, i);
      K k = load_key<K>(key, src);
      unsigned long long v = t.n_pay ? (unsigned long long)load_signed(pay0, src, pay_size) : 0ull;
      unsigned long long kb = (unsigned long long)(long long)k;
      bool placed = false;
      if (kb != kFree) {
        uint32_t h = (uint32_t)slot_of(kb, 10);
        for (int s = 0; s < 32; ++s) {
          uint32_t j = (h + s) & (kPjLds - 1);
          unsigned long long prev = atomicCAS(&lkey[j], kFree, kb);
          if (prev == kFree || prev == kb) {
            atomicAdd(&lcnt[j], 1ull);
            atomicAdd(&lsum[j], v);
            placed = true;
            break;
          }
        }
      }
      if (!placed) {
        unsigned long long sums[kMaxPay] = {v, 0, 0, 0};
        global_preagg_add<K>(t, k, 1ull, sums, flags);
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kPjLds; j += blockDim.x) {
      if (lkey[j] != kFree) {
        unsigned long long sums[kMaxPay] = {lsum[j], 0, 0, 0};
        global_preagg_add<K>(t, (K)(long long)lkey[j], lcnt[j], sums, flags);
      }
    }
    __syncthreads();
  }
}

template <typename K>
__global__ void __launch_bounds__(256) k_pj_probe(TableView t, const void* key, SegList sl,
                                                  unsigned long long* acc_out) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  __shared__ unsigned long long sst[kMaxSegs], spre[kMaxSegs + 1];
  for (uint32_t j = threadIdx.x; j < sl.nseg; j += blockDim.x) sst[j] = sl.start[j];
  for (uint32_t j = threadIdx.x; j <= sl.nseg; j += blockDim.x) spre[j] = sl.prefix[j];
  __syncthreads();
  unsigned long long acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  constexpr int ITEMS = 4;
  const uint64_t tile = (uint64_t)blockDim.x * ITEMS;
  for (uint64_t base = blockIdx.x * tile; base < sl.total; base += (uint64_t)gridDim.x * tile) {
    K keys[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      keys[j] = i < sl.total ? load_key<K>(key, seg_source(sst, spre, sl.nseg, i)) : (K)0;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      if (i >= sl.total) continue;
      const unsigned long long* w;
      if ((U)keys[j] == kEmpty) {
        w = t.side;
      } else {
        const uint8_t* s = find_slot<K>(t, keys[j]);
        if (!s) continue;
        w = (const unsigned long long*)(s + 8);
      }
      acc[0] += w[0];
      for (uint32_t p = 0; p < t.n_pay; ++p) acc[1 + p] += w[1 + p];
    }
  }
  block_flush<9>(acc, 1 + (int)t.n_pay, acc_out);
}

// ---------------------------------------------------------------- host side

namespace {

struct Side {
  ColInfo key;
  ColInfo pay[kMaxPay];
  uint32_t n_pay = 0;
  uint64_t n = 0;
  uint8_t* host_key = nullptr;          // clustered copy in pinned host memory
  uint8_t* host_pay[kMaxPay] = {};
  uint64_t chunk_rows = 0, n_chunks = 0;
  std::vector<unsigned long long> bnd;  // n_chunks * (P + 1)
  std::vector<unsigned long long> slot_sums;   // 2 * kMaxSumSlots: count, payload-0 sum
  uint64_t sdma = 0;
};

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// Pass 1 for one table: stream, cluster each chunk by partition, write it back with its
// boundary array.
vx_status cluster_side(vx_ctx* ctx, const PartSpec& ps, const int* sum_slot_dev, Side& sd) {
  const uint32_t P = ps.n_parts;
  std::vector<PipeCol> cols(1 + sd.n_pay);
  cols[0].info = sd.key;
  cols[0].may_copy = cols[0].copy = true;
  for (uint32_t c = 0; c < sd.n_pay; ++c) {
    cols[1 + c].info = sd.pay[c];
    cols[1 + c].may_copy = cols[1 + c].copy = true;
  }
  uint64_t min_rows = (sd.n + kMaxSegs - 1) / kMaxSegs;
  uint64_t want = env_u64("VX_CHUNK_BYTES", 64ull << 20) / 8;
  Pipeline pipe;
  VX_TRY(pipe.plan(ctx, sd.n, std::max(min_rows, std::min<uint64_t>(want, std::max<uint64_t>(sd.n, 1))), 0, cols));
  sd.chunk_rows = pipe.chunk_rows();
  sd.n_chunks = pipe.n_chunks();
  uint64_t row_bytes = (uint64_t)sd.key.elsize;
  for (uint32_t c = 0; c < sd.n_pay; ++c) row_bytes += (uint64_t)sd.pay[c].elsize;
  // staging for clustered chunks (double-buffered against the write-back), per-wave
  // histograms, offsets, per-chunk boundaries and singleton sums
  PartGeom g0 = part_geom(ctx, sd.chunk_rows);
  uint64_t stage_bytes = align_up(sd.chunk_rows * row_bytes + 256 * (1 + kMaxPay), 256);
  uint64_t scratch = 2 * stage_bytes + (uint64_t)P * g0.waves * 12 +
                     std::max<uint64_t>(sd.n_chunks, 1) * (P + 1) * 8 + 2 * kMaxSumSlots * 8 + 1024;
  ArenaBlock blk;
  blk.a = &ctx->arena;
  blk.p = ctx->arena.alloc(scratch);
  VX_CHECK(blk.p, VX_EBUDGET, "partitioned join: no room for the partition pass scratch (%llu B)",
           (unsigned long long)scratch);
  uint8_t* stage[2] = {blk.p, blk.p + stage_bytes};
  uint32_t* hist = (uint32_t*)(blk.p + 2 * stage_bytes);
  unsigned long long* offs = (unsigned long long*)((uint8_t*)hist + (uint64_t)P * g0.waves * 4);
  unsigned long long* bnd = offs + (uint64_t)P * g0.waves;
  unsigned long long* sums = bnd + std::max<uint64_t>(sd.n_chunks, 1) * (P + 1);
  fill_zero((uint64_t*)sums, 2 * kMaxSumSlots, ctx->compute);
  hipEvent_t done[2] = {get_event(ctx), get_event(ctx)};
  hipEvent_t wrote[2] = {get_event(ctx), get_event(ctx)};
  bool pending[2] = {false, false};
  auto kernel = [&](const ChunkView& v) -> vx_status {
    uint32_t b = (uint32_t)(v.index % 2);
    if (pending[b]) VX_HIP(hipStreamWaitEvent(ctx->compute, wrote[b], 0));
    PartIO io{};
    io.key = (v.global_mask & 1u) ? (const uint8_t*)v.ptr[0] + v.row0 * sd.key.elsize : v.ptr[0];
    io.key_size = (uint32_t)sd.key.elsize;
    io.n = v.rows;
    io.n_pay = sd.n_pay;
    uint8_t* out = stage[b];
    io.out_key = out;
    uint64_t off = align_up(v.rows * sd.key.elsize, 256);
    for (uint32_t c = 0; c < sd.n_pay; ++c) {
      io.pay[c] = ((v.global_mask >> (1 + c)) & 1u)
                      ? (const uint8_t*)v.ptr[1 + c] + v.row0 * sd.pay[c].elsize
                      : v.ptr[1 + c];
      io.pay_size[c] = (uint32_t)sd.pay[c].elsize;
      io.out_pay[c] = out + off;
      off += align_up(v.rows * sd.pay[c].elsize, 256);
    }
    PartGeom g = part_geom(ctx, v.rows);
    VX_TRY(part_hist(ctx, ps, io, g, hist, nullptr, sum_slot_dev, sum_slot_dev ? sums : nullptr,
                     ctx->compute));
    VX_TRY(part_scan(ctx, hist, P, g.waves, nullptr, offs, bnd + v.index * (P + 1), ctx->compute));
    VX_TRY(part_scatter(ctx, ps, io, g, offs, ctx->compute));
    VX_HIP(hipEventRecord(done[b], ctx->compute));
    // write the clustered chunk back to host memory at the chunk's own rows
    VX_HIP(hipStreamWaitEvent(ctx->d2h, done[b], 0));
    VX_HIP(hipMemcpyAsync(sd.host_key + v.row0 * sd.key.elsize, io.out_key, v.rows * sd.key.elsize,
                          hipMemcpyDeviceToHost, ctx->d2h));
    for (uint32_t c = 0; c < sd.n_pay; ++c)
      VX_HIP(hipMemcpyAsync(sd.host_pay[c] + v.row0 * sd.pay[c].elsize, io.out_pay[c],
                            v.rows * sd.pay[c].elsize, hipMemcpyDeviceToHost, ctx->d2h));
    VX_HIP(hipEventRecord(wrote[b], ctx->d2h));
    pending[b] = true;
    return VX_OK;
  };
  vx_status st = pipe.run(kernel);
  (void)hipStreamSynchronize(ctx->compute);
  (void)hipStreamSynchronize(ctx->d2h);
  for (int b = 0; b < 2; ++b) {
    put_event(ctx, done[b]);
    put_event(ctx, wrote[b]);
  }
  VX_TRY(st);
  sd.sdma = pipe.sdma_bytes();
  sd.bnd.assign(sd.n_chunks * (P + 1), 0);
  sd.slot_sums.assign(2 * kMaxSumSlots, 0);
  if (sd.n_chunks) VX_HIP(hipMemcpy(sd.bnd.data(), bnd, sd.bnd.size() * 8, hipMemcpyDeviceToHost));
  VX_HIP(hipMemcpy(sd.slot_sums.data(), sums, sd.slot_sums.size() * 8, hipMemcpyDeviceToHost));
  return VX_OK;
}

// segments of partition p across the chunks of one side (row starts in the clustered copy)
uint64_t segments(const Side& sd, uint32_t P, uint32_t p, std::vector<unsigned long long>& start,
                  std::vector<unsigned long long>& prefix) {
  start.clear();
  prefix.clear();
  uint64_t tot = 0;
  for (uint64_t c = 0; c < sd.n_chunks; ++c) {
    const unsigned long long* b = sd.bnd.data() + c * (P + 1);
    uint64_t len = b[p + 1] - b[p];
    if (!len) continue;
    start.push_back(c * sd.chunk_rows + b[p]);
    prefix.push_back(tot);
    tot += len;
  }
  prefix.push_back(tot);
  return tot;
}

}  // namespace

vx_status join_partitioned(vx_ctx* ctx, const vx_partitioned_join* d, vx_join_out* out) {
  double t0 = now_ms();
  const vx_build_desc& B = d->build;
  const vx_probe_desc& Q = d->probe;
  VX_CHECK(B.key.type == Q.key.type, VX_EINVAL, "partitioned join: key types differ");
  VX_CHECK(B.n_pay <= 1, VX_EUNSUPPORTED, "partitioned join: at most one build payload");
  VX_CHECK(B.n_pay == 0 || B.pay, VX_EINVAL, "partitioned join: build pay is NULL");
  VX_CHECK(Q.n_pay == 0, VX_EUNSUPPORTED, "partitioned join: probe payloads are not supported");
  VX_HIP(hipSetDevice(ctx->device));
  Side bs, qs;
  bs.n = B.n;
  qs.n = Q.n;
  VX_TRY(classify(ctx, B.key, B.n, &bs.key, "partitioned build key"));
  bs.n_pay = B.n_pay;
  for (uint32_t c = 0; c < B.n_pay; ++c) VX_TRY(classify(ctx, B.pay[c], B.n, &bs.pay[c], "partitioned build payload"));
  VX_TRY(classify(ctx, Q.key, Q.n, &qs.key, "partitioned probe key"));
  const int ks = bs.key.elsize;

  // partitioner
  vx_part_opts o = d->part;
  uint32_t req = o.n_parts ? o.n_parts : 256;
  std::vector<int64_t> split;
  CdfReport rep{};
  uint32_t method = o.method;
  double tt0 = now_ms();
  if (method == VX_PART_LEARNED || method == VX_PART_QUANTILE || method == VX_PART_UNTRAINED ||
      method == VX_PART_AUTO) {
    VX_TRY(cdf_splitters(ctx, bs.key, B.n, o, req, &split, &rep, nullptr));
    if (method == VX_PART_AUTO) {
      bool singleton = false;
      for (size_t i = 1; i < split.size(); ++i) singleton |= split[i] == split[i - 1] + 1;
      method = singleton ? VX_PART_LEARNED : VX_PART_RADIX_HASH;
    }
  }
  double train_ms = now_ms() - tt0;
  vx_part_opts eff = o;
  eff.method = (method == VX_PART_LEARNED || method == VX_PART_QUANTILE || method == VX_PART_UNTRAINED)
                   ? VX_PART_RANGE
                   : method;
  if (eff.method == VX_PART_RANGE && o.method == VX_PART_RANGE) {
    VX_CHECK(o.n_splitters == 0 || o.splitters, VX_EINVAL, "partitioned join: splitters is NULL");
    split.assign(o.splitters, o.splitters + o.n_splitters);
  }
  ArenaBlock split_mem;
  PartSpec ps;
  VX_TRY(make_spec(ctx, eff, req, split.data(), (uint32_t)split.size(), split_mem, &ps));
  const uint32_t P = ps.n_parts;

  // singleton partitions (range methods): [s_{p-1}, s_p) holding exactly one key value
  std::vector<int> slot(P, -1);
  uint32_t n_single = 0;
  if (ps.fn == kPartRange) {
    for (uint32_t p = 1; p + 1 < P && n_single < kMaxSumSlots; ++p)
      if (split[p] == split[p - 1] + 1) slot[p] = (int)n_single++;
  }
  ArenaBlock slot_mem;
  const int* slot_dev = nullptr;
  if (n_single) {
    slot_mem.a = &ctx->arena;
    slot_mem.p = ctx->arena.alloc(P * sizeof(int));
    VX_CHECK(slot_mem.p, VX_EBUDGET, "partitioned join: no room for singleton slots");
    VX_HIP(hipMemcpyAsync(slot_mem.p, slot.data(), P * sizeof(int), hipMemcpyHostToDevice, ctx->compute));
    slot_dev = (const int*)slot_mem.p;
  }

  // pinned host memory for the clustered tables
  uint64_t hbytes = align_up(B.n * ks, 256) + align_up(Q.n * ks, 256);
  for (uint32_t c = 0; c < B.n_pay; ++c) hbytes += align_up(B.n * bs.pay[c].elsize, 256);
  uint8_t* hs = nullptr;
  VX_TRY(host_scratch(ctx, hbytes + 256, &hs));
  bs.host_key = hs;
  uint64_t off = align_up(B.n * ks, 256);
  for (uint32_t c = 0; c < B.n_pay; ++c) {
    bs.host_pay[c] = hs + off;
    off += align_up(B.n * bs.pay[c].elsize, 256);
  }
  qs.host_key = hs + off;

  // pass 1
  double tp0 = now_ms();
  VX_TRY(cluster_side(ctx, ps, slot_dev, bs));
  VX_TRY(cluster_side(ctx, ps, slot_dev, qs));
  double part_ms = now_ms() - tp0;

  // per-partition sizes
  std::vector<uint64_t> brows(P, 0), qrows(P, 0);
  for (uint64_t c = 0; c < bs.n_chunks; ++c)
    for (uint32_t p = 0; p < P; ++p) brows[p] += bs.bnd[c * (P + 1) + p + 1] - bs.bnd[c * (P + 1) + p];
  for (uint64_t c = 0; c < qs.n_chunks; ++c)
    for (uint32_t p = 0; p < P; ++p) qrows[p] += qs.bnd[c * (P + 1) + p + 1] - qs.bnd[c * (P + 1) + p];

  // pass 2: one pre-aggregating table, sized for the largest non-singleton partition
  double tj0 = now_ms();
  uint64_t max_rows = 0;
  for (uint32_t p = 0; p < P; ++p)
    if (slot[p] < 0 && qrows[p]) max_rows = std::max(max_rows, brows[p]);
  const uint32_t slot_bytes = 32;   // key, count, payload sum (+ padding)
  uint64_t max_cap = 64;
  while (max_cap < 2 * max_rows) max_cap <<= 1;
  ArenaBlock tmem, segmem;
  uint64_t pass2_rows = 0;
  for (uint32_t p = 0; p < P; ++p)
    if (slot[p] < 0 && brows[p] && qrows[p]) pass2_rows += brows[p] + qrows[p];
  tmem.a = &ctx->arena;
  tmem.p = ctx->arena.alloc(max_cap * slot_bytes + 256);
  VX_CHECK(tmem.p, VX_EBUDGET,
           "partitioned join: the largest partition (%llu build rows, %llu slots) does not fit the "
           "arena; use more partitions", (unsigned long long)max_rows, (unsigned long long)max_cap);
  // segment lists of every partition, uploaded once: [p][start | prefix] for build, then probe
  const uint64_t seg_stride = 4 * (uint64_t)(kMaxSegs + 1);
  segmem.a = &ctx->arena;
  segmem.p = ctx->arena.alloc((uint64_t)P * seg_stride * 8);
  VX_CHECK(segmem.p, VX_EBUDGET, "partitioned join: no room for segment lists");
  std::vector<unsigned long long> hseg((uint64_t)P * seg_stride, 0);
  std::vector<uint64_t> nb_of(P, 0), nq_of(P, 0), sb_of(P, 0), sq_of(P, 0);
  {
    std::vector<unsigned long long> st, pre;
    for (uint32_t p = 0; p < P; ++p) {
      unsigned long long* h = hseg.data() + (uint64_t)p * seg_stride;
      nb_of[p] = segments(bs, P, p, st, pre);
      sb_of[p] = st.size();
      std::copy(st.begin(), st.end(), h);
      std::copy(pre.begin(), pre.end(), h + (kMaxSegs + 1));
      nq_of[p] = segments(qs, P, p, st, pre);
      sq_of[p] = st.size();
      std::copy(st.begin(), st.end(), h + 2 * (kMaxSegs + 1));
      std::copy(pre.begin(), pre.end(), h + 3 * (kMaxSegs + 1));
    }
  }
  VX_HIP(hipMemcpyAsync(segmem.p, hseg.data(), hseg.size() * 8, hipMemcpyHostToDevice, ctx->compute));
  const uint64_t acc_rows = std::min<uint64_t>(P, ctx->dev_acc_words / kAccWords);
  fill_zero((uint64_t*)ctx->dev_acc, acc_rows * kAccWords, ctx->compute);
  fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);
  const bool k64 = B.key.type == VX_I64;
  uint64_t launches = 0;
  void* hs_dev = nullptr;
  VX_HIP(hipHostGetDevicePointer(&hs_dev, hs, 0));
  const uint8_t* dk_b = (const uint8_t*)hs_dev + (bs.host_key - hs);
  const uint8_t* dp_b = B.n_pay ? (const uint8_t*)hs_dev + (bs.host_pay[0] - hs) : nullptr;
  const uint8_t* dk_q = (const uint8_t*)hs_dev + (qs.host_key - hs);
  const uint32_t psz = B.n_pay ? (uint32_t)bs.pay[0].elsize : 8;
  for (uint32_t p = 0; p < P; ++p) {
    if (slot[p] >= 0 || brows[p] == 0 || qrows[p] == 0) continue;
    const uint64_t nb = nb_of[p], nq = nq_of[p];
    TableView t{};
    uint64_t cap = 64;
    while (cap < 2 * nb) cap <<= 1;
    t.slots = tmem.p;
    t.mask = cap - 1;
    while ((1ull << t.log2cap) < cap) ++t.log2cap;
    t.slot_shift = 5;
    t.side = (unsigned long long*)(tmem.p + max_cap * slot_bytes);
    t.n_pay = B.n_pay;
    t.pay_off[0] = 16;
    t.pay_size[0] = 8;
    t.preagg = 1;
    t.key_size = (uint32_t)ks;
    const unsigned long long* h = (const unsigned long long*)segmem.p + (uint64_t)p * seg_stride;
    SegList lb{h, h + (kMaxSegs + 1), (uint32_t)sb_of[p], nb};
    SegList lq{h + 2 * (kMaxSegs + 1), h + 3 * (kMaxSegs + 1), (uint32_t)sq_of[p], nq};
    unsigned ig = (unsigned)std::min<uint64_t>((cap + 255) / 256, (uint64_t)ctx->cu_count * 8);
    hipLaunchKernelGGL(k_pj_init, dim3(ig), dim3(256), 0, ctx->compute, (uint32_t*)tmem.p, cap,
                       slot_bytes / 4, (uint32_t)ks, t.side);
    unsigned gb = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((nb + kPjTile - 1) / kPjTile,
                                                                     (uint64_t)ctx->cu_count * 3));
    unsigned gq = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((nq + 1023) / 1024, (uint64_t)ctx->cu_count * 8));
    unsigned long long* acc = (unsigned long long*)ctx->dev_acc + (p % acc_rows) * kAccWords;
    if (k64) {
      hipLaunchKernelGGL(k_pj_build<int64_t>, dim3(gb), dim3(256), 0, ctx->compute, t, dk_b, dp_b, psz, lb,
                         ctx->dev_flags);
      hipLaunchKernelGGL(k_pj_probe<int64_t>, dim3(gq), dim3(256), 0, ctx->compute, t, dk_q, lq, acc);
    } else {
      hipLaunchKernelGGL(k_pj_build<int32_t>, dim3(gb), dim3(256), 0, ctx->compute, t, dk_b, dp_b, psz, lb,
                         ctx->dev_flags);
      hipLaunchKernelGGL(k_pj_probe<int32_t>, dim3(gq), dim3(256), 0, ctx->compute, t, dk_q, lq, acc);
    }
    VX_HIP(hipGetLastError());
    launches += 3;
  }
  VX_HIP(hipStreamSynchronize(ctx->compute));
  VX_TRY(check_flags(ctx, "partitioned join"));
  std::vector<unsigned long long> accs(acc_rows * kAccWords);
  VX_HIP(hipMemcpy(accs.data(), ctx->dev_acc, accs.size() * 8, hipMemcpyDeviceToHost));
  double join_ms = now_ms() - tj0;

  // per-partition aggregates: pass 2 results, or the singleton closed form
  std::vector<vx_agg> per(P);
  uint64_t single_rows = 0;
  for (uint32_t p = 0; p < P; ++p) {
    std::memset(&per[p], 0, sizeof(vx_agg));
    if (slot[p] >= 0) {
      uint64_t cb = bs.slot_sums[2 * slot[p]], sb = bs.slot_sums[2 * slot[p] + 1];
      uint64_t cq = qs.slot_sums[2 * slot[p]];
      per[p].match_count = cb * cq;
      per[p].sum[0] = sb * cq;
      single_rows += cb + cq;
    } else if (P <= acc_rows) {
      per[p].match_count = accs[p * kAccWords];
      for (uint32_t c = 0; c < B.n_pay; ++c) per[p].sum[c] = accs[p * kAccWords + 1 + c];
    }
  }
  std::memset(&out->agg, 0, sizeof out->agg);
  for (uint32_t p = 0; p < P; ++p) {
    out->agg.match_count += per[p].match_count;
    for (uint32_t c = 0; c < B.n_pay; ++c) out->agg.sum[c] += per[p].sum[c];
  }
  if (Q.chunk_aggs) {
    VX_CHECK(Q.chunk_aggs_cap >= P, VX_ECAPACITY, "partitioned join: chunk_aggs_cap %llu < %u partitions",
             (unsigned long long)Q.chunk_aggs_cap, P);
    std::copy(per.begin(), per.end(), Q.chunk_aggs);
  }
  double mx = 0, tot = 0;
  for (uint32_t p = 0; p < P; ++p) {
    mx = std::max(mx, (double)(brows[p] + qrows[p]));
    tot += (double)(brows[p] + qrows[p]);
  }
  vx_stats& s = out->stats;
  std::memset(&s, 0, sizeof s);
  s.rows = Q.n;
  s.n_parts = P;
  s.imbalance = tot > 0 ? mx / (tot / P) : 0.0;
  s.part_ms = part_ms;
  s.train_ms = train_ms;
  s.singleton_rows = single_rows;
  s.sdma_bytes = bs.sdma + qs.sdma;
  uint64_t pass2_bytes = 0;
  for (uint32_t p = 0; p < P; ++p)
    if (slot[p] < 0 && brows[p] && qrows[p])
      pass2_bytes += brows[p] * (ks + (B.n_pay ? bs.pay[0].elsize : 0)) + qrows[p] * ks;
  s.zc_bytes_est = pass2_bytes;
  s.build_ms = 0;
  s.probe_ms = join_ms;
  s.kernel_launches = launches;
  s.total_ms = now_ms() - t0;
  out->part_method_used = method;
  return VX_OK;
}

}  // namespace vx
