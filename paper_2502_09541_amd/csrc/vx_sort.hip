// Out-of-core sort of a key column larger than the device budget (Sec. 6.1).
//
// Pass 1 (the paper's SortExKernel): the column streams through the chunk pipeline in runs of
// chunk_rows keys.  Each run is sorted on the GPU by an LSD radix sort of 8-bit digits (the sign
// bit flipped so that signed order comes out) whose stable passes sort tiles of 8192 keys in LDS
// and write each digit's keys of a tile as one run, and is stored to pinned host scratch by a
// kernel on a second stream: kernel stores to mapped host memory run beside the host-to-device
// copies.
// Pass 2 (the paper's MergeExKernel): every run is cut at the same global ranks (multiples of the
// run length), found by binary search over the runs on the host.  Output range i then holds one
// sorted segment of every run.  Its segments are copied in, merged in a tree of pairwise
// merge-path launches (two device buffers used in turn), and the result is stored to its final
// place in the key column.  Up to three ranges are in flight: one copies in, one merges, one is
// stored.
#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "vx_part.h"
#include "vx_pipeline.h"

namespace vx {

namespace {

constexpr int kMergeThreads = 256;
constexpr int kMergeItems = 8;
constexpr int kMergeTile = kMergeThreads * kMergeItems;   // outputs per workgroup tile

// Number of the first d outputs of merge(a, b) that come from a (ties: a first).
template <typename K>
__device__ __forceinline__ uint64_t merge_split(const K* a, uint64_t na, const K* b, uint64_t nb, uint64_t d) {
  uint64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] <= b[d - 1 - mid]) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// split[t] = merge_split at output min(t * tile, na + nb), for t = 0 .. tiles: where every tile
// of the merge starts, found by all the tiles' binary searches at once.
template <typename K>
__global__ void k_merge_splits(const K* a, uint64_t na, const K* b, uint64_t nb, uint64_t tiles,
                               unsigned long long* split) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t > tiles) return;
  const uint64_t d = t * kMergeTile < na + nb ? t * kMergeTile : na + nb;
  split[t] = merge_split(a, na, b, nb, d);
}

// out[0, na + nb) = the stable merge of sorted a and b.  A workgroup takes a tile of 2048
// outputs whose ends on the merge path are split[t] and split[t + 1], stages the tile's inputs
// in LDS with coalesced loads, lets every lane merge 8 outputs from LDS (its own start found by
// a binary search in LDS) into an LDS output tile, and stores the tile with coalesced writes.
template <typename K>
__global__ void __launch_bounds__(kMergeThreads) k_merge(const K* a, uint64_t na, const K* b, uint64_t nb,
                                                         const unsigned long long* split, K* out) {
  __shared__ K sa[kMergeTile], sb[kMergeTile], so[kMergeTile];
  const uint64_t n = na + nb;
  for (uint64_t t = blockIdx.x; t * kMergeTile < n; t += gridDim.x) {
    const uint64_t d0 = t * kMergeTile;
    const uint64_t d1 = d0 + kMergeTile < n ? d0 + kMergeTile : n;
    const uint64_t s0 = split[t], s1 = split[t + 1];
    const uint64_t ia = s0, ib = d0 - s0;
    const uint32_t ma = (uint32_t)(s1 - s0), mb = (uint32_t)((d1 - s1) - ib);
    for (uint32_t k = threadIdx.x; k < ma; k += kMergeThreads) sa[k] = a[ia + k];
    for (uint32_t k = threadIdx.x; k < mb; k += kMergeThreads) sb[k] = b[ib + k];
    __syncthreads();
    const uint32_t m = ma + mb, t0 = threadIdx.x * kMergeItems;
    if (t0 < m) {
      uint32_t lo = t0 > mb ? t0 - mb : 0, hi = t0 < ma ? t0 : ma;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sa[mid] <= sb[t0 - 1 - mid]) lo = mid + 1;
        else hi = mid;
      }
      uint32_t i = lo, j = t0 - lo;
      const uint32_t e1 = t0 + kMergeItems < m ? t0 + kMergeItems : m;
      for (uint32_t e = t0; e < e1; ++e) {
        const bool take_a = j >= mb || (i < ma && sa[i] <= sb[j]);
        so[e] = take_a ? sa[i++] : sb[j++];
      }
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < m; k += kMergeThreads) out[d0 + k] = so[k];
    __syncthreads();
  }
}

// dst[0, bytes) = src[0, bytes) with 16-byte vector stores (dst may be mapped host memory); both
// 16-byte aligned, bytes a multiple of 4.
__global__ void __launch_bounds__(256) k_store(const uint8_t* src, uint8_t* dst, uint64_t bytes) {
  const uint64_t n16 = bytes / 16;
  const uint4* s = (const uint4*)src;
  uint4* d = (uint4*)dst;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
  for (uint64_t i = n16 * 4 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < bytes / 4;
       i += (uint64_t)gridDim.x * blockDim.x)
    ((uint32_t*)dst)[i] = ((const uint32_t*)src)[i];
}

// The same for any 4-byte-aligned pointers, element by element.
__global__ void __launch_bounds__(256) k_store4(const uint32_t* src, uint32_t* dst, uint64_t words) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---------------------------------------------------------------- LSD radix digit pass
//
// One workgroup per tile of 8192 consecutive keys; wave w holds keys [w*1024, (w+1)*1024) of the
// tile, 16 per lane in steps of 64.  The histogram launch counts each tile's keys per digit into
// hist[t * 256 + d] (tile-major: a workgroup's 256 counts are one contiguous store).  A column
// scan turns them into offs[t * 256 + d], where tile t's first key of digit d goes: the keys of
// every lower digit plus those of digit d in earlier tiles.  It walks the tiles in blocks, one
// thread per digit, so its loads and stores are contiguous across the threads.  The scatter
// launch ranks the tile's keys by digit in input order
// (ballots give a lane its rank among the step's lanes of the same digit, a per-wave LDS counter
// carries the count across steps), sorts the tile into LDS by that rank, and writes it out in
// LDS order: each digit's keys of the tile form one run of consecutive output addresses, about 32
// keys long, so the stores fill whole lines.  A stable pass, as LSD radix sorting needs.
constexpr uint32_t kDigitThreads = 512;
constexpr uint32_t kDigitWaves = kDigitThreads / 64;
constexpr uint32_t kDigitItems = 16;                            // keys per lane
constexpr uint32_t kDigitTile = kDigitThreads * kDigitItems;    // keys per workgroup tile
constexpr uint32_t kWaveKeys = 64 * kDigitItems;                // keys per wave, contiguous

uint64_t digit_tiles(uint64_t rows) { return std::max<uint64_t>(1, (rows + kDigitTile - 1) / kDigitTile); }

// 8 bits at `shift` of the key's order-preserving unsigned image (sign bit flipped)
__device__ __forceinline__ uint32_t digit_of(int32_t k, uint32_t shift) {
  return (((uint32_t)k ^ 0x80000000u) >> shift) & 255u;
}
__device__ __forceinline__ uint32_t digit_of(int64_t k, uint32_t shift) {
  return (uint32_t)((((uint64_t)k ^ 0x8000000000000000ull) >> shift) & 255u);
}

// the valid lanes of the wave whose digit equals this lane's
__device__ __forceinline__ unsigned long long same_digit(uint32_t d, bool valid) {
  unsigned long long m = __ballot(valid);
#pragma unroll
  for (uint32_t b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const unsigned long long v = __ballot(bit);
    m &= bit ? v : ~v;
  }
  return m;
}

// this lane's keys of tile t (zero past n); a full tile loads unconditionally
template <typename K>
__device__ __forceinline__ void digit_load(const K* in, uint64_t n, uint64_t first, bool full,
                                           K (&k)[kDigitItems]) {
  if (full) {
#pragma unroll
    for (uint32_t j = 0; j < kDigitItems; ++j) k[j] = __builtin_nontemporal_load(in + first + j * 64);
  } else {
#pragma unroll
    for (uint32_t j = 0; j < kDigitItems; ++j) k[j] = first + j * 64 < n ? in[first + j * 64] : K(0);
  }
}

// rank[j] = number of this wave's earlier keys with key j's digit; cnt[d] ends as the wave's
// count of digit d (cnt is the wave's own row, zeroed by the caller)
template <typename K>
__device__ __forceinline__ void digit_rank(const K (&k)[kDigitItems], uint64_t n, uint64_t first,
                                           uint32_t shift, uint32_t* cnt, uint32_t (&rank)[kDigitItems]) {
  const uint32_t lane = threadIdx.x & 63;
  const unsigned long long lower = (1ull << lane) - 1;
#pragma unroll
  for (uint32_t j = 0; j < kDigitItems; ++j) {
    const bool valid = first + j * 64 < n;
    const uint32_t d = digit_of(k[j], shift);
    const unsigned long long peers = same_digit(d, valid);
    const uint32_t below = (uint32_t)__popcll(peers & lower);
    const uint32_t c = valid ? cnt[d] : 0u;
    rank[j] = c + below;
    // every lane has read cnt[] before the group's first lane advances it
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0) cnt[d] = c + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
}

template <typename K>
__global__ void __launch_bounds__(kDigitThreads) k_digit_hist(const K* in, uint64_t n, uint32_t shift,
                                                             uint32_t* hist) {
  __shared__ uint32_t cnt[kDigitWaves][256];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t t = blockIdx.x;
  for (uint32_t i = threadIdx.x; i < kDigitWaves * 256; i += kDigitThreads) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const uint64_t first = t * kDigitTile + wave * kWaveKeys + lane;
  K k[kDigitItems];
  uint32_t rank[kDigitItems];
  digit_load(in, n, first, (t + 1) * kDigitTile <= n, k);
  digit_rank(k, n, first, shift, cnt[wave], rank);
  __syncthreads();
  if (threadIdx.x < 256) {
    uint32_t c = 0;
#pragma unroll
    for (uint32_t w = 0; w < kDigitWaves; ++w) c += cnt[w][threadIdx.x];
    hist[t * 256 + threadIdx.x] = c;
  }
}

// Column scan of the tile-major histogram, in blocks of `per` tiles (at most kColBlocks blocks;
// thread d of every launch handles digit d).  part holds kColBlocks * 256 words.
constexpr uint32_t kColBlocks = 128;

uint64_t col_per(uint64_t tiles) { return std::max<uint64_t>(1, (tiles + kColBlocks - 1) / kColBlocks); }

// part[b * 256 + d] = block b's keys of digit d
__global__ void __launch_bounds__(256) k_digit_colsum(const uint32_t* hist, uint64_t tiles, uint64_t per,
                                                      unsigned long long* part) {
  const uint64_t t0 = blockIdx.x * per, t1 = t0 + per < tiles ? t0 + per : tiles;
  unsigned long long s = 0;
  uint64_t t = t0;
  for (; t + 8 <= t1; t += 8) {   // eight independent loads in flight
    uint32_t v[8];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) v[u] = hist[(t + u) * 256 + threadIdx.x];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) s += v[u];
  }
  for (; t < t1; ++t) s += hist[t * 256 + threadIdx.x];
  part[(uint64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// One workgroup: part[b * 256 + d] becomes the output position of block b's first key of digit d.
__global__ void __launch_bounds__(256) k_digit_colbase(unsigned long long* part, uint32_t nb) {
  __shared__ unsigned long long ws[4];
  const uint32_t d = threadIdx.x, lane = d & 63, wave = d >> 6;
  unsigned long long total = 0;
  uint32_t b = 0;
  for (; b + 8 <= nb; b += 8) {   // eight independent loads in flight
    unsigned long long v[8];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) v[u] = part[(uint64_t)(b + u) * 256 + d];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) {
      part[(uint64_t)(b + u) * 256 + d] = total;
      total += v[u];
    }
  }
  for (; b < nb; ++b) {
    const unsigned long long v = part[(uint64_t)b * 256 + d];
    part[(uint64_t)b * 256 + d] = total;
    total += v;
  }
  unsigned long long x = total;   // exclusive scan of the digits' totals over the workgroup
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[wave] = x;
  __syncthreads();
  unsigned long long base = x - total;
  for (uint32_t w = 0; w < wave; ++w) base += ws[w];
  for (uint32_t b = 0; b < nb; ++b) part[(uint64_t)b * 256 + d] += base;
}

// offs[t * 256 + d] = output position of tile t's first key of digit d
__global__ void __launch_bounds__(256) k_digit_colapply(const uint32_t* hist, uint64_t tiles, uint64_t per,
                                                        const unsigned long long* part, unsigned long long* offs) {
  const uint64_t t0 = blockIdx.x * per, t1 = t0 + per < tiles ? t0 + per : tiles;
  unsigned long long run = part[(uint64_t)blockIdx.x * 256 + threadIdx.x];
  uint64_t t = t0;
  for (; t + 8 <= t1; t += 8) {
    uint32_t v[8];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) v[u] = hist[(t + u) * 256 + threadIdx.x];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) {
      offs[(t + u) * 256 + threadIdx.x] = run;
      run += v[u];
    }
  }
  for (; t < t1; ++t) {
    offs[t * 256 + threadIdx.x] = run;
    run += hist[t * 256 + threadIdx.x];
  }
}

// offs[t * 256 + d] = output position of tile t's first key of digit d
template <typename K>
__global__ void __launch_bounds__(kDigitThreads) k_digit_scatter(const K* in, K* out, uint64_t n, uint32_t shift,
                                                                const unsigned long long* offs) {
  __shared__ K stage[kDigitTile];
  __shared__ uint32_t cnt[kDigitWaves][256];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t wsum[4];
  __shared__ unsigned long long gbase[256];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t t = blockIdx.x;
  for (uint32_t i = threadIdx.x; i < kDigitWaves * 256; i += kDigitThreads) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const uint64_t first = t * kDigitTile + wave * kWaveKeys + lane;
  const bool full = (t + 1) * kDigitTile <= n;
  K k[kDigitItems];
  uint32_t rank[kDigitItems];
  digit_load(in, n, first, full, k);
  digit_rank(k, n, first, shift, cnt[wave], rank);
  __syncthreads();
  // per digit: the waves' exclusive offsets, then the digits' exclusive offsets in the tile
  uint32_t tot = 0;
  if (threadIdx.x < 256) {
#pragma unroll
    for (uint32_t w = 0; w < kDigitWaves; ++w) {
      const uint32_t c = cnt[w][threadIdx.x];
      cnt[w][threadIdx.x] = tot;
      tot += c;
    }
  }
  uint32_t x = tot;
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (threadIdx.x < 256 && lane == 63) wsum[wave] = x;
  __syncthreads();
  if (threadIdx.x < 256) {
    uint32_t e = x - tot;
    for (uint32_t w = 0; w < wave; ++w) e += wsum[w];
    dstart[threadIdx.x] = e;
    gbase[threadIdx.x] = offs[t * 256 + threadIdx.x] - e;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t j = 0; j < kDigitItems; ++j)
    if (first + j * 64 < n) {
      const uint32_t d = digit_of(k[j], shift);
      stage[dstart[d] + cnt[wave][d] + rank[j]] = k[j];
    }
  __syncthreads();
  const uint32_t m = full ? kDigitTile : (uint32_t)(n - t * kDigitTile);
#pragma unroll
  for (uint32_t j = 0; j < kDigitItems; ++j) {
    const uint32_t p = j * kDigitThreads + threadIdx.x;
    if (p < m) {
      const K v = stage[p];
      out[gbase[digit_of(v, shift)] + p] = v;
    }
  }
}

unsigned grid_of(const vx_ctx* ctx, uint64_t items, uint64_t per_block, uint64_t per_cu) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((items + per_block - 1) / per_block,
                                                            (uint64_t)ctx->cu_count * per_cu));
}

// The order-preserving map of a signed key to an unsigned one.
inline uint64_t ord(int64_t v) { return (uint64_t)v ^ 0x8000000000000000ull; }
inline int64_t unord(uint64_t u) { return (int64_t)(u ^ 0x8000000000000000ull); }

// Per-run cut at global rank r: the r smallest elements of the union of the sorted runs, ties
// taken from lower-numbered runs first.  Finds the smallest value v with at least r elements
// <= v (binary search over the value range, each step a binary search in every run), takes
// every element below v, then the elements equal to v run by run.
template <typename K>
void merge_cuts_t(const K* const* runs, const uint64_t* len, uint32_t n_runs, uint64_t r, uint64_t* cut) {
  uint64_t total = 0;
  for (uint32_t j = 0; j < n_runs; ++j) total += len[j];
  if (r == 0 || r >= total) {
    for (uint32_t j = 0; j < n_runs; ++j) cut[j] = r == 0 ? 0 : len[j];
    return;
  }
  uint64_t lo = ~0ull, hi = 0;
  for (uint32_t j = 0; j < n_runs; ++j)
    if (len[j]) {
      lo = std::min(lo, ord((int64_t)runs[j][0]));
      hi = std::max(hi, ord((int64_t)runs[j][len[j] - 1]));
    }
  auto count_le = [&](uint64_t u) {
    const int64_t v = unord(u);
    uint64_t c = 0;
    for (uint32_t j = 0; j < n_runs; ++j)
      c += (uint64_t)(std::upper_bound(runs[j], runs[j] + len[j], v,
                                       [](int64_t x, const K& y) { return x < (int64_t)y; }) - runs[j]);
    return c;
  };
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (count_le(mid) >= r) hi = mid;
    else lo = mid + 1;
  }
  const int64_t v = unord(lo);
  uint64_t need = r;
  std::vector<uint64_t> eq(n_runs);
  for (uint32_t j = 0; j < n_runs; ++j) {
    const K* b = runs[j];
    const K* e = runs[j] + len[j];
    const K* l = std::lower_bound(b, e, v, [](const K& x, int64_t y) { return (int64_t)x < y; });
    const K* u = std::upper_bound(b, e, v, [](int64_t x, const K& y) { return x < (int64_t)y; });
    cut[j] = (uint64_t)(l - b);
    eq[j] = (uint64_t)(u - l);
    need -= cut[j];
  }
  for (uint32_t j = 0; j < n_runs && need; ++j) {
    const uint64_t t = std::min(need, eq[j]);
    cut[j] += t;
    need -= t;
  }
}

// LSD radix sort of rows keys from src (left unchanged) into dst, through alt: digit passes of 8
// bits over the key's order-preserving image (int64: 8 passes, int32: 4), each a histogram
// launch, the three-launch column scan and a tile scatter.  Passes alternate between dst and alt
// so the last one writes dst.  hist holds 256 * digit_tiles(rows) entries, offs that many plus
// 256 * kColBlocks (the column scan's block sums, after the offsets).
template <typename K>
vx_status radix_sort_keys(const K* src, K* alt, K* dst, uint64_t rows, uint32_t* hist, unsigned long long* offs,
                          vx_ctx* ctx, hipStream_t s) {
  const uint32_t passes = sizeof(K);
  const uint64_t tiles = digit_tiles(rows);
  VX_CHECK(tiles < (1ull << 31), VX_EINVAL, "sort: run of %llu keys is too long", (unsigned long long)rows);
  const uint64_t per = col_per(tiles);
  const unsigned nb = (unsigned)((tiles + per - 1) / per);   // <= kColBlocks
  unsigned long long* part = offs + 256 * tiles;
  (void)ctx;
  const K* in = src;
  for (uint32_t p = 0; p < passes; ++p) {
    K* out = ((passes - 1 - p) % 2 == 0) ? dst : alt;
    hipLaunchKernelGGL(k_digit_hist<K>, dim3((unsigned)tiles), dim3(kDigitThreads), 0, s, in, rows, 8 * p, hist);
    hipLaunchKernelGGL(k_digit_colsum, dim3(nb), dim3(256), 0, s, hist, tiles, per, part);
    hipLaunchKernelGGL(k_digit_colbase, dim3(1), dim3(256), 0, s, part, nb);
    hipLaunchKernelGGL(k_digit_colapply, dim3(nb), dim3(256), 0, s, hist, tiles, per, part, offs);
    hipLaunchKernelGGL(k_digit_scatter<K>, dim3((unsigned)tiles), dim3(kDigitThreads), 0, s, in, out, rows, 8 * p,
                       offs);
    VX_HIP(hipGetLastError());
    in = out;
  }
  return VX_OK;
}

vx_status radix_sort_run(vx_ctx* ctx, const void* src, void* alt, void* dst, uint64_t rows, uint32_t ks,
                         uint32_t* hist, unsigned long long* offs, hipStream_t s) {
  if (ks == 8)
    return radix_sort_keys((const int64_t*)src, (int64_t*)alt, (int64_t*)dst, rows, hist, offs, ctx, s);
  return radix_sort_keys((const int32_t*)src, (int32_t*)alt, (int32_t*)dst, rows, hist, offs, ctx, s);
}

uint64_t align_to(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// Stores of a sorted run or merged range to its place (host or device memory), on a second stream
// beside the sort and merge kernels.  One workgroup per 16 compute units: the stores slow the
// kernels beside them (on the full-size sort, 256 workgroups took 1077 ms per sort, 64 took
// 1030, 16 took 1001 and 8 took 1041, where the stores themselves became the limit).
vx_status launch_store(const vx_ctx* ctx, const uint8_t* src, uint8_t* dst, uint64_t bytes, hipStream_t s) {
  const unsigned g = (unsigned)std::max(1, ctx->cu_count / 16);
  if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0)
    hipLaunchKernelGGL(k_store, dim3(g), dim3(256), 0, s, src, dst, bytes);
  else
    hipLaunchKernelGGL(k_store4, dim3(g), dim3(256), 0, s, (const uint32_t*)src, (uint32_t*)dst, bytes / 4);
  VX_HIP(hipGetLastError());
  return VX_OK;
}

vx_status sort_impl(vx_ctx* ctx, const vx_sort_desc* d, vx_stats* stats) {
  const double t0 = now_ms();
  VX_HIP(hipSetDevice(ctx->device));
  ColInfo kc;
  VX_TRY(classify(ctx, d->key, d->n, &kc, "sort key"));
  const uint64_t n = d->n;
  const uint32_t ks = (uint32_t)kc.elsize;
  vx_stats st;
  std::memset(&st, 0, sizeof st);
  st.rows = n;
  if (n < 2) {
    if (stats) *stats = st;
    return VX_OK;
  }
  // run length: the largest power of two whose pass-1 buffers (2 pipeline buffers, one radix
  // buffer, two staging runs) and digit histograms fit the free arena; pass 2 needs 4 runs' room
  const uint64_t free0 = ctx->arena.capacity() - ctx->arena.used();
  auto pass1_bytes = [&](uint64_t rows) {
    return 5 * align_to(rows * ks, 256) + (uint64_t)256 * (digit_tiles(rows) * 12 + kColBlocks * 8) + (1ull << 20);
  };
  uint64_t C = d->chunk_rows;
  if (!C) {
    C = 1024;
    while (C * 2 <= n && pass1_bytes(C * 2) <= free0) C *= 2;
    if (C < n && pass1_bytes(n) <= free0) C = n;
    if (C > n) C = n;
  }
  VX_CHECK(C >= 1, VX_EINVAL, "sort: chunk_rows is 0");
  const uint64_t runs = (n + C - 1) / C;
  const uint64_t tiles_max = digit_tiles(std::min(C, n));
  const uint64_t run_bytes = align_to(std::min(C, n) * ks, 256);
  // host scratch for the sorted runs (several runs only)
  uint8_t* hs = nullptr;
  if (runs > 1) VX_TRY(host_scratch(ctx, n * ks + 256, &hs));
  void* hs_dev = nullptr;
  if (hs) VX_HIP(hipHostGetDevicePointer(&hs_dev, hs, 0));
  uint8_t* out_dev = (uint8_t*)kc.dev;   // the key column as a device address (sorted in place)

  // ---------------- pass 1: sorted runs
  const double tp0 = now_ms();
  double sort_k_ms = 0;
  uint64_t launches = 0, sdma = 0;
  uint32_t nbuf_used = 0;
  {
    ArenaBlock blk;
    blk.a = &ctx->arena;
    const uint64_t hist_bytes = align_to((uint64_t)256 * tiles_max * 4, 256);
    blk.p = ctx->arena.alloc(3 * run_bytes + hist_bytes + (uint64_t)256 * (tiles_max + kColBlocks) * 8 + 256);
    VX_CHECK(blk.p, VX_EBUDGET, "sort: no room for runs of %llu keys (radix and staging buffers)",
             (unsigned long long)C);
    uint8_t* alt = blk.p;
    uint8_t* stage[2] = {blk.p + run_bytes, blk.p + 2 * run_bytes};
    uint32_t* hist = (uint32_t*)(blk.p + 3 * run_bytes);
    unsigned long long* offs = (unsigned long long*)(blk.p + 3 * run_bytes + hist_bytes);
    std::vector<PipeCol> cols(1);
    cols[0].info = kc;
    cols[0].may_copy = cols[0].copy = true;
    Pipeline pipe;
    VX_TRY(pipe.plan(ctx, n, C, d->n_buffers, cols));
    nbuf_used = pipe.n_buffers();
    hipEvent_t sorted_ev[2] = {get_event(ctx), get_event(ctx)}, wrote[2] = {get_event(ctx), get_event(ctx)};
    std::vector<hipEvent_t> kev;
    bool pending[2] = {false, false};
    auto kernel = [&](const ChunkView& v) -> vx_status {
      for (int b = 0; b < 2; ++b) VX_CHECK(sorted_ev[b] && wrote[b], VX_EHIP, "sort: no HIP event");
      const uint32_t b = (uint32_t)(v.index % 2);
      if (pending[b]) VX_HIP(hipStreamWaitEvent(ctx->compute, wrote[b], 0));
      const uint8_t* src = (v.global_mask & 1u) ? (const uint8_t*)v.ptr[0] + v.row0 * ks : (const uint8_t*)v.ptr[0];
      hipEvent_t e0 = get_event(ctx), e1 = get_event(ctx);
      VX_CHECK(e0 && e1, VX_EHIP, "sort: no HIP event");
      kev.push_back(e0);
      kev.push_back(e1);
      VX_HIP(hipEventRecord(e0, ctx->compute));
      VX_TRY(radix_sort_run(ctx, src, alt, stage[b], v.rows, ks, hist, offs, ctx->compute));
      VX_HIP(hipEventRecord(e1, ctx->compute));
      launches += 5 * ks;   // per digit pass: histogram, three scan launches, scatter
      VX_HIP(hipEventRecord(sorted_ev[b], ctx->compute));
      // a single run is the result: store it in place; otherwise to its rows of the scratch
      uint8_t* dst = (runs > 1 ? (uint8_t*)hs_dev : out_dev) + v.row0 * ks;
      VX_HIP(hipStreamWaitEvent(ctx->d2h, sorted_ev[b], 0));
      VX_TRY(launch_store(ctx, stage[b], dst, v.rows * ks, ctx->d2h));
      ++launches;
      VX_HIP(hipEventRecord(wrote[b], ctx->d2h));
      pending[b] = true;
      return VX_OK;
    };
    vx_status rs = pipe.run(kernel);
    (void)hipStreamSynchronize(ctx->compute);
    (void)hipStreamSynchronize(ctx->d2h);
    for (size_t i = 0; i + 1 < kev.size(); i += 2) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, kev[i], kev[i + 1]) == hipSuccess) sort_k_ms += ms;
    }
    for (auto e : kev) put_event(ctx, e);
    for (int b = 0; b < 2; ++b) {
      put_event(ctx, sorted_ev[b]);
      put_event(ctx, wrote[b]);
    }
    VX_TRY(rs);
    sdma = pipe.sdma_bytes();
  }
  const double pass1_ms = now_ms() - tp0;

  // ---------------- pass 2: regroup and merge
  const double tm0 = now_ms();
  double merge_k_ms = 0;
  uint64_t max_part = 0;
  if (runs > 1) {
    // cuts of every run at ranks 0, C, 2C, ..., n (host binary search over the pinned runs)
    const uint64_t M = runs;
    std::vector<uint64_t> rank(M + 1), len(runs);
    for (uint64_t i = 0; i <= M; ++i) rank[i] = std::min(i * C, n);
    for (uint64_t j = 0; j < runs; ++j) len[j] = std::min(C, n - j * C);
    std::vector<uint64_t> cuts((M + 1) * runs);
    {
      const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
      std::vector<std::thread> th;
      for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
          if (ks == 8) {
            std::vector<const long long*> rp(runs);
            for (uint64_t j = 0; j < runs; ++j) rp[j] = (const long long*)hs + j * C;
            for (uint64_t i = t; i <= M; i += nt)
              merge_cuts_t<long long>(rp.data(), len.data(), (uint32_t)runs, rank[i], &cuts[i * runs]);
          } else {
            std::vector<const int*> rp(runs);
            for (uint64_t j = 0; j < runs; ++j) rp[j] = (const int*)hs + j * C;
            for (uint64_t i = t; i <= M; i += nt)
              merge_cuts_t<int>(rp.data(), len.data(), (uint32_t)runs, rank[i], &cuts[i * runs]);
          }
        });
      for (auto& x : th) x.join();
    }
    for (uint64_t i = 0; i < M; ++i) max_part = std::max(max_part, rank[i + 1] - rank[i]);
    // three sets of (input, alternate) buffers when they fit, else two: a range holds its set from
    // its copy in to the end of its store, so with three the copies of the next ranges run while
    // one range merges and another is stored
    const uint64_t pbytes = align_to(max_part * ks, 256);
    ArenaBlock blk;
    blk.a = &ctx->arena;
    uint32_t nset = 3;
    blk.p = ctx->arena.largest_free() >= 6 * pbytes + (1u << 20) ? ctx->arena.alloc(6 * pbytes) : nullptr;
    if (!blk.p) {
      nset = 2;
      blk.p = ctx->arena.alloc(4 * pbytes);
    }
    VX_CHECK(blk.p, VX_EBUDGET, "sort: no room for the merge buffers (4 x %llu B)", (unsigned long long)pbytes);
    uint8_t* X[3] = {blk.p, blk.p + pbytes, blk.p + 2 * pbytes};
    uint8_t* Y[3] = {blk.p + nset * pbytes, blk.p + (nset + 1) * pbytes, blk.p + (nset + 2) * pbytes};
    ArenaBlock sp;
    sp.a = &ctx->arena;
    sp.p = ctx->arena.alloc((max_part / kMergeTile + 2) * 8);
    VX_CHECK(sp.p, VX_EBUDGET, "sort: no room for the merge splits");
    unsigned long long* splits = (unsigned long long*)sp.p;
    hipEvent_t copied[3] = {get_event(ctx), get_event(ctx), get_event(ctx)},
               merged[3] = {get_event(ctx), get_event(ctx), get_event(ctx)},
               stored[3] = {get_event(ctx), get_event(ctx), get_event(ctx)};
    std::vector<hipEvent_t> kev;
    // one output range; on an error the streams are still drained before the buffers go back
    auto range = [&](uint64_t i) -> vx_status {
      for (int b = 0; b < 3; ++b) VX_CHECK(copied[b] && merged[b] && stored[b], VX_EHIP, "sort: no HIP event");
      const uint32_t b = (uint32_t)(i % nset);
      if (i >= nset) VX_HIP(hipEventSynchronize(stored[b]));   // range i - nset has left these buffers
      // copy in the range's segment of every run, back to back
      std::vector<uint64_t> off(runs + 1, 0);
      for (uint64_t j = 0; j < runs; ++j) {
        const uint64_t a = cuts[i * runs + j], e = cuts[(i + 1) * runs + j];
        off[j + 1] = off[j] + (e - a);
        if (e > a) {
          VX_HIP(hipMemcpyAsync(X[b] + off[j] * ks, hs + (j * C + a) * ks, (e - a) * ks, hipMemcpyHostToDevice,
                                ctx->copy));
          sdma += (e - a) * ks;
        }
      }
      VX_HIP(hipEventRecord(copied[b], ctx->copy));
      VX_HIP(hipStreamWaitEvent(ctx->compute, copied[b], 0));
      // merge rounds: pairs of neighbouring segments, X and Y in turn
      std::vector<uint64_t> seg;
      for (uint64_t j = 0; j <= runs; ++j)
        if (j == 0 || j == runs || off[j] != off[j - 1]) seg.push_back(off[j]);
      uint8_t* src = X[b];
      uint8_t* dst = Y[b];
      hipEvent_t e0 = get_event(ctx), e1 = get_event(ctx);
      VX_CHECK(e0 && e1, VX_EHIP, "sort: no HIP event");
      kev.push_back(e0);
      kev.push_back(e1);
      VX_HIP(hipEventRecord(e0, ctx->compute));
      while (seg.size() > 2) {
        std::vector<uint64_t> next;
        for (size_t k = 0; k + 1 < seg.size(); k += 2) {
          const uint64_t a0 = seg[k], a1 = seg[k + 1], b1 = k + 2 < seg.size() ? seg[k + 2] : a1;
          const uint64_t tiles = (b1 - a0 + kMergeTile - 1) / kMergeTile;
          const unsigned g = grid_of(ctx, b1 - a0, kMergeTile, 4);
          const unsigned gs = (unsigned)((tiles + 1 + 255) / 256);
          if (ks == 8) {
            const long long* pa = (const long long*)src + a0;
            const long long* pb = (const long long*)src + a1;
            hipLaunchKernelGGL(k_merge_splits<long long>, dim3(gs), dim3(256), 0, ctx->compute, pa, a1 - a0, pb,
                               b1 - a1, tiles, splits);
            hipLaunchKernelGGL(k_merge<long long>, dim3(g), dim3(kMergeThreads), 0, ctx->compute, pa, a1 - a0, pb,
                               b1 - a1, (const unsigned long long*)splits, (long long*)dst + a0);
          } else {
            const int* pa = (const int*)src + a0;
            const int* pb = (const int*)src + a1;
            hipLaunchKernelGGL(k_merge_splits<int>, dim3(gs), dim3(256), 0, ctx->compute, pa, a1 - a0, pb, b1 - a1,
                               tiles, splits);
            hipLaunchKernelGGL(k_merge<int>, dim3(g), dim3(kMergeThreads), 0, ctx->compute, pa, a1 - a0, pb, b1 - a1,
                               (const unsigned long long*)splits, (int*)dst + a0);
          }
          VX_HIP(hipGetLastError());
          launches += 2;
          next.push_back(a0);
        }
        next.push_back(seg.back());
        seg.swap(next);
        std::swap(src, dst);
      }
      VX_HIP(hipEventRecord(e1, ctx->compute));
      VX_HIP(hipEventRecord(merged[b], ctx->compute));
      // store the merged range to its place in the key column
      VX_HIP(hipStreamWaitEvent(ctx->d2h, merged[b], 0));
      const uint64_t rows = rank[i + 1] - rank[i];
      VX_TRY(launch_store(ctx, src, out_dev + rank[i] * ks, rows * ks, ctx->d2h));
      ++launches;
      VX_HIP(hipEventRecord(stored[b], ctx->d2h));
      return VX_OK;
    };
    vx_status rs = VX_OK;
    for (uint64_t i = 0; i < M && rs == VX_OK; ++i) rs = range(i);
    (void)hipStreamSynchronize(ctx->copy);
    (void)hipStreamSynchronize(ctx->compute);
    (void)hipStreamSynchronize(ctx->d2h);
    for (size_t k = 0; k + 1 < kev.size(); k += 2) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, kev[k], kev[k + 1]) == hipSuccess) merge_k_ms += ms;
    }
    for (auto e : kev) put_event(ctx, e);
    for (int b = 0; b < 3; ++b) {
      put_event(ctx, copied[b]);
      put_event(ctx, merged[b]);
      put_event(ctx, stored[b]);
    }
    VX_TRY(rs);
  }
  VX_HIP(hipGetLastError());
  st.chunks = runs;
  st.chunk_rows = C;
  st.n_buffers = nbuf_used;
  st.part_ms = pass1_ms;
  st.probe_ms = runs > 1 ? now_ms() - tm0 : 0;
  st.kernel_ms = sort_k_ms;
  st.build_ms = merge_k_ms;
  st.sdma_bytes = sdma;
  st.kernel_launches = launches;
  st.total_ms = now_ms() - t0;
  if (stats) *stats = st;
  return VX_OK;
}

}  // namespace
}  // namespace vx

extern "C" vx_status vx_sort(vx_ctx* ctx, const vx_sort_desc* d, vx_stats* stats) {
  VX_CHECK(ctx && d, VX_EINVAL, "vx_sort: null argument");
  vx::release_cached(ctx);
  return vx::sort_impl(ctx, d, stats);
}

extern "C" vx_status vx_merge_cuts(const int64_t* const* runs, const uint64_t* run_len, uint32_t n_runs,
                                   uint64_t rank, uint64_t* cut) {
  VX_CHECK(n_runs == 0 || (runs && run_len && cut), VX_EINVAL, "vx_merge_cuts: null argument");
  uint64_t total = 0;
  for (uint32_t j = 0; j < n_runs; ++j) {
    VX_CHECK(run_len[j] == 0 || runs[j], VX_EINVAL, "vx_merge_cuts: run %u is NULL", j);
    total += run_len[j];
  }
  VX_CHECK(rank <= total, VX_EINVAL, "vx_merge_cuts: rank %llu exceeds the %llu elements",
           (unsigned long long)rank, (unsigned long long)total);
  vx::merge_cuts_t<int64_t>(runs, run_len, n_runs, rank, cut);
  return VX_OK;
}
