// Star join with GROUP BY.
//
// The dimension tables are filtered and hashed on the GPU and stay resident; the fact table
// is streamed (the paper's star-schema plan).  Once the dimension tables are built, the
// fraction of rows that passed each filter is the selectivity estimate of the matching fact
// foreign key; dimensions are probed in ascending selectivity, so each later column is read
// only for rows still alive.  The first probed foreign key is streamed through the chunk
// pipeline; each other fact column is streamed too or read by zero-copy for the surviving
// rows only, chosen from the running selectivity before the scan starts (late
// materialization).  Survivors are aggregated into a device group table with 64-bit atomics.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "vx_device.h"
#include "vx_pipeline.h"

namespace vx {


// ---------------------------------------------------------------- dimension build

template <typename K>
__global__ void k_build_dim(TableView t, const void* key, const void* filt, uint32_t filt_size,
                            long long lo, long long hi, const void* grp, uint64_t n,
                            unsigned int* flags, unsigned long long* passed) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t first = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  for (uint64_t wb = first - (threadIdx.x & 63); wb < n; wb += stride) {
    uint64_t i = wb + (threadIdx.x & 63);
    bool pass = false;
    if (i < n) {
      long long f = load_signed(filt, i, filt_size);
      pass = f >= lo && f <= hi;
    }
    unsigned long long m = __ballot(pass);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(passed, (unsigned long long)__popcll(m));
    if (!pass) continue;
    K k = load_key<K>(key, i);
    U kb = (U)k;
    int g = grp ? ((const int*)grp)[i] : 0;
    if (kb == kEmpty) {
      atomicAdd(t.side, 1ull);
      if (grp) atomicAdd(t.side + 1, (unsigned long long)(long long)g);
      continue;
    }
    uint64_t h;
    bool done = false;
    if (!first_slot(t, k, h)) {    // cannot happen: the range was measured over every dimension row
      atomicOr(flags, kFlagFull);
      continue;
    }
    for (uint64_t step = 0; step <= t.mask; ++step) {
      uint8_t* slot = t.slots + (h << t.slot_shift);
      U prev = atomicCAS((U*)slot, kEmpty, kb);
      if (prev == kEmpty) {
        if (grp) *(int*)(slot + t.pay_off[0]) = g;
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

// ---------------------------------------------------------------- group table

// Slot: key (8), count (8), sums (4 x 8), padding -> 64 bytes.  Key = (u32)g0 << 32 | (u32)g1;
// all-ones marks an empty slot, so group (-1, -1) lives in the side record after the slots.
struct GroupTable {
  unsigned long long* slots;
  uint64_t mask;
  uint32_t log2cap;
  uint32_t n_meas;
};
constexpr unsigned long long kGroupEmpty = ~0ull;
constexpr int kGroupWords = 8;

__global__ void k_init_groups(unsigned long long* slots, uint64_t words) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x)
    slots[i] = (i % kGroupWords) == 0 ? kGroupEmpty : 0ull;
}

__device__ __forceinline__ void group_add(const GroupTable& g, unsigned long long key,
                                          const long long* meas, unsigned int* flags) {
  unsigned long long* w = nullptr;
  if (key == kGroupEmpty) {
    w = g.slots + (g.mask + 1) * kGroupWords;   // side record
  } else {
    uint64_t h = slot_of(key, g.log2cap);
    for (uint64_t step = 0; step <= g.mask; ++step) {
      unsigned long long* s = g.slots + h * kGroupWords;
      unsigned long long prev = atomicCAS(s, kGroupEmpty, key);
      if (prev == kGroupEmpty || prev == key) {
        w = s;
        break;
      }
      h = (h + 1) & g.mask;
    }
    if (!w) {
      atomicOr(flags, kFlagGroupOverflow);
      return;
    }
  }
  atomicAdd(w + 1, 1ull);
  for (uint32_t m = 0; m < g.n_meas; ++m) atomicAdd(w + 2 + m, (unsigned long long)meas[m]);
}

// ---------------------------------------------------------------- fact scan

struct StarArgs {
  uint32_t n_dims;
  uint32_t n_meas;
  TableView dim[4];            // probe order
  int gsel[4];                 // -1: no group; 0 / 1: writes g0 / g1
  const void* fk[4];           // probe order; chunk-local unless fk_global bit set
  uint32_t fk_global;
  const void* meas[4];
  uint32_t meas_size[4];
  uint32_t meas_global;
  uint64_t n, row0;
  GroupTable groups;
  unsigned int* flags;
  unsigned long long* survivors;   // [0] fact rows that pass every dimension, [1] zero-copy granules
  uint32_t fk_zc, meas_zc;         // bit set: the column is host memory read in place (count granules)
  uint32_t zc_shift;               // log2 of the zero-copy granule in bytes
};

// COUNT: count the zero-copy granules of the gathers (compiled in only when asked for).
template <typename K, int kStarItems, bool COUNT>
__global__ void __launch_bounds__(256) k_star(StarArgs a) {
  using U = typename KeyTraits<K>::U;
  const U kEmpty = KeyTraits<K>::kEmpty;
  unsigned long long alive_count = 0, granules = 0;
  const uint64_t tile = (uint64_t)blockDim.x * kStarItems;
  const uint64_t wave_row = threadIdx.x & ~63u;
  for (uint64_t base = blockIdx.x * tile; base < a.n; base += (uint64_t)gridDim.x * tile) {
    bool alive[kStarItems];
    int g[kStarItems][2];
#pragma unroll
    for (int j = 0; j < kStarItems; ++j) {
      alive[j] = base + (uint64_t)j * blockDim.x + threadIdx.x < a.n;
      g[j][0] = g[j][1] = 0;
    }
    for (uint32_t d = 0; d < a.n_dims; ++d) {
      const bool glob = (a.fk_global >> d) & 1u;
      K fk[kStarItems];
#pragma unroll
      for (int j = 0; j < kStarItems; ++j) {
        uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
        fk[j] = 0;
        if (alive[j]) {
          if (d == 0 && !glob) fk[j] = __builtin_nontemporal_load(((const K*)a.fk[0]) + i);
          else fk[j] = load_key<K>(a.fk[d], glob ? a.row0 + i : i);
        }
      }
      if (COUNT && ((a.fk_zc >> d) & 1u)) {
#pragma unroll
        for (int j = 0; j < kStarItems; ++j) {
          const uint64_t r0 = a.row0 + base + (uint64_t)j * blockDim.x + wave_row;
          granules += wave_granules(alive[j], (uint64_t)(uintptr_t)a.fk[d] + r0 * sizeof(K), sizeof(K), a.zc_shift);
        }
      }
#pragma unroll
      for (int j = 0; j < kStarItems; ++j) {
        if (!alive[j]) continue;
        const TableView& t = a.dim[d];
        int grp = 0;
        bool found;
        if ((U)fk[j] == kEmpty) {
          found = t.side[0] != 0;
          grp = (int)t.side[1];
        } else {
          const uint8_t* s = find_slot<K>(t, fk[j]);
          found = s != nullptr;
          if (found && t.n_pay) grp = *(const int*)(s + t.pay_off[0]);
        }
        alive[j] = found;
        if (found && a.gsel[d] >= 0) g[j][a.gsel[d]] = grp;
      }
    }
    for (uint32_t c = 0; COUNT && c < a.n_meas; ++c) {
      if (!((a.meas_zc >> c) & 1u)) continue;
#pragma unroll
      for (int j = 0; j < kStarItems; ++j) {
        const uint64_t r0 = a.row0 + base + (uint64_t)j * blockDim.x + wave_row;
        granules += wave_granules(alive[j], (uint64_t)(uintptr_t)a.meas[c] + r0 * a.meas_size[c], a.meas_size[c],
                                  a.zc_shift);
      }
    }
#pragma unroll
    for (int j = 0; j < kStarItems; ++j) {
      if (!alive[j]) continue;
      uint64_t i = base + (uint64_t)j * blockDim.x + threadIdx.x;
      long long m[4] = {0, 0, 0, 0};
      for (uint32_t c = 0; c < a.n_meas; ++c)
        m[c] = load_signed(a.meas[c], ((a.meas_global >> c) & 1u) ? a.row0 + i : i, a.meas_size[c]);
      unsigned long long key = ((unsigned long long)(unsigned int)g[j][0] << 32) |
                               (unsigned long long)(unsigned int)g[j][1];
      group_add(a.groups, key, m, a.flags);
      ++alive_count;
    }
  }
  for (int o = 32; o > 0; o >>= 1) alive_count += __shfl_xor(alive_count, o, 64);
  if ((threadIdx.x & 63) == 0 && alive_count) atomicAdd(a.survivors, alive_count);
  // every lane holds its wave's granule count
  if (COUNT && (threadIdx.x & 63) == 0 && granules) atomicAdd(a.survivors + 1, granules);
}

// ---------------------------------------------------------------- host side

template <int ITEMS>
static void launch_star(bool k64, bool count, unsigned g, const StarArgs& a, hipStream_t s) {
  if (k64) {
    if (count) hipLaunchKernelGGL((k_star<int64_t, ITEMS, true>), dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_star<int64_t, ITEMS, false>), dim3(g), dim3(256), 0, s, a);
  } else {
    if (count) hipLaunchKernelGGL((k_star<int32_t, ITEMS, true>), dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_star<int32_t, ITEMS, false>), dim3(g), dim3(256), 0, s, a);
  }
}

// rows per lane in flight in the fact scan (VX_STAR_ITEMS = 4 or 8; default 8)
static int star_items() {
  const char* e = getenv("VX_STAR_ITEMS");
  return e && atoi(e) == 4 ? 4 : 8;
}

vx_status join_star(vx_ctx* ctx, const vx_star_join* d, vx_join_out* out) {
  double t0 = now_ms();
  VX_CHECK(d->n_dims >= 1 && d->n_dims <= 4, VX_EINVAL, "star: n_dims %u outside 1..4", d->n_dims);
  VX_CHECK(d->n_measures <= 4, VX_EINVAL, "star: n_measures %u > 4", d->n_measures);
  VX_CHECK(d->late_mat >= -1 && d->late_mat <= 2, VX_EINVAL, "star: late_mat %d", d->late_mat);
  VX_CHECK(d->groups != nullptr || d->groups_cap == 0, VX_EINVAL, "star: groups is NULL");
  VX_CHECK((d->flags & ~(uint32_t)VX_PROBE_COUNT_ZC) == 0, VX_EINVAL, "star: unknown flags %u", d->flags);
  const bool count_zc = (d->flags & VX_PROBE_COUNT_ZC) != 0;
  const int32_t ktype = d->dims[0].key.type;
  const uint32_t nd = d->n_dims;
  VX_HIP(hipSetDevice(ctx->device));
  for (uint32_t k = 0; k < nd; ++k) {
    VX_CHECK(d->dims[k].key.type == ktype && d->fact_fk[k].type == ktype, VX_EINVAL,
             "star: dimension keys and fact foreign keys must share one type");
    VX_CHECK(d->dims[k].group.data == nullptr || d->dims[k].group.type == VX_I32, VX_EINVAL,
             "star: group attributes must be VX_I32");
  }
  // group attribute slots: the first two dimensions (in dimension order) that carry one
  int gsel_dim[4] = {-1, -1, -1, -1};
  int ng = 0;
  for (uint32_t k = 0; k < nd; ++k)
    if (d->dims[k].group.data && ng < 2) gsel_dim[k] = ng++;

  // dimension tables: uniqueness over all rows, then the filtered table
  struct Dim {
    vx_table* t = nullptr;
    double sel = 1.0;
  } dims[4];
  auto free_dims = [&]() {
    for (uint32_t k = 0; k < nd; ++k)
      if (dims[k].t) {
        ctx->arena.release(dims[k].t->mem);
        delete dims[k].t;
        dims[k].t = nullptr;
      }
  };
  vx_stats s{};
  for (uint32_t k = 0; k < nd; ++k) {
    const vx_star_dim& sd = d->dims[k];
    ColInfo kc, fc, gc{};
    vx_status st = classify(ctx, sd.key, sd.n, &kc, "star dimension key");
    if (st == VX_OK) st = classify(ctx, sd.filter, sd.n, &fc, "star dimension filter");
    if (st == VX_OK && sd.group.data) st = classify(ctx, sd.group, sd.n, &gc, "star dimension group");
    if (st != VX_OK) {
      free_dims();
      return st;
    }
    // device-resident keys that fill a narrow range get direct tables (slot = key - min)
    KeyRange kr;
    if (kc.where == Where::Device) st = key_range(ctx, ktype, kc.dev, sd.n, &kr);
    if (st != VX_OK) {
      free_dims();
      return st;
    }
    // uniqueness of the dimension's keys (primary key), over every row
    {
      vx_table* u = nullptr;
      st = make_table(ctx, ktype, VX_UNIQUE, nullptr, 0, sd.n, 0.5f, &u, &kr);
      if (st == VX_OK) {
        fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);
        st = table_insert(ctx, u, kc, nullptr, sd.n, ctx->compute, 1);
        if (st == VX_OK) st = check_flags(ctx, "star dimension");
        ctx->arena.release(u->mem);
        delete u;
      }
      if (st != VX_OK) {
        free_dims();
        return st;
      }
    }
    int32_t pt[1] = {VX_I32};
    // worst case every row passes; size the table for all rows
    st = make_table(ctx, ktype, VX_UNIQUE, pt, sd.group.data ? 1 : 0, sd.n, 0.5f, &dims[k].t, &kr);
    if (st != VX_OK) {
      free_dims();
      return st;
    }
    s.table_bytes += dims[k].t->bytes;
    unsigned long long* passed = (unsigned long long*)ctx->dev_acc;
    fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);
    fill_zero((uint64_t*)passed, 1, ctx->compute);
    if (sd.n) {
      unsigned g = (unsigned)std::min<uint64_t>((sd.n + 255) / 256, (uint64_t)ctx->cu_count * 8);
      const void* grp = sd.group.data ? gc.dev : nullptr;
      if (ktype == VX_I64)
        hipLaunchKernelGGL(k_build_dim<int64_t>, dim3(g), dim3(256), 0, ctx->compute, dims[k].t->view,
                           kc.dev, fc.dev, (uint32_t)fc.elsize, (long long)sd.lo, (long long)sd.hi, grp,
                           sd.n, ctx->dev_flags, passed);
      else
        hipLaunchKernelGGL(k_build_dim<int32_t>, dim3(g), dim3(256), 0, ctx->compute, dims[k].t->view,
                           kc.dev, fc.dev, (uint32_t)fc.elsize, (long long)sd.lo, (long long)sd.hi, grp,
                           sd.n, ctx->dev_flags, passed);
      st = hipGetLastError() == hipSuccess ? VX_OK : VX_EHIP;
      if (st != VX_OK) set_error("star: dimension build launch failed");
    }
    unsigned long long np = 0;
    if (st == VX_OK && hipMemcpy(&np, passed, 8, hipMemcpyDeviceToHost) != hipSuccess) {
      set_error("star: reading the filter count failed");
      st = VX_EHIP;
    }
    if (st == VX_OK) st = check_flags(ctx, "star dimension");
    if (st != VX_OK) {
      free_dims();
      return st;
    }
    dims[k].t->n_rows = np;
    dims[k].sel = sd.n ? (double)np / (double)sd.n : 0.0;
  }
  s.build_ms = now_ms() - t0;

  // probe order: ascending estimated selectivity (stable)
  uint32_t order[4];
  std::iota(order, order + nd, 0u);
  std::stable_sort(order, order + nd, [&](uint32_t a, uint32_t b) { return dims[a].sel < dims[b].sel; });

  // pipeline columns: FKs in probe order, then measures
  std::vector<PipeCol> cols(nd + d->n_measures);
  std::vector<double> col_sel(cols.size());
  double run = 1.0;
  for (uint32_t k = 0; k < nd; ++k) {
    uint32_t dk = order[k];
    vx_status st = classify(ctx, d->fact_fk[dk], d->n_fact, &cols[k].info, "star fact key");
    if (st != VX_OK) {
      free_dims();
      return st;
    }
    col_sel[k] = run;
    run *= dims[dk].sel;
  }
  for (uint32_t c = 0; c < d->n_measures; ++c) {
    vx_status st = classify(ctx, d->measure[c], d->n_fact, &cols[nd + c].info, "star measure");
    if (st != VX_OK) {
      free_dims();
      return st;
    }
    col_sel[nd + c] = run;
  }
  for (size_t c = 0; c < cols.size(); ++c) {
    bool zc;
    int es = cols[c].info.elsize;
    if (c == 0) zc = false;                         // the first probed key is always streamed
    else if (d->late_mat == VX_LATE_SDMA) zc = false;
    else if (d->late_mat == VX_LATE_ZC) zc = true;
    else if (d->late_mat == VX_LATE_PAPER) zc = col_sel[c] < (double)es / (double)ctx->zc_line;
    else zc = zc_wire_bytes(1000000, (uint64_t)(col_sel[c] * 1e6), es, ctx->zc_line) / 1e6 < 0.95 * es;
    cols[c].copy = cols[c].may_copy = !zc;
  }

  // group table
  uint64_t want = std::max<uint64_t>(1024, 2 * std::max<uint64_t>(d->groups_cap, 1));
  uint64_t gcap = 1;
  while (gcap < want) gcap <<= 1;
  uint64_t gwords = (gcap + 1) * kGroupWords;
  ArenaBlock gblock;
  gblock.a = &ctx->arena;
  gblock.p = ctx->arena.alloc(gwords * 8);
  if (!gblock.p) {
    free_dims();
    set_error("star: group table of %llu slots does not fit the arena", (unsigned long long)gcap);
    return VX_EBUDGET;
  }
  GroupTable gt{(unsigned long long*)gblock.p, gcap - 1, 0, d->n_measures};
  while ((1ull << gt.log2cap) < gcap) ++gt.log2cap;
  {
    unsigned g = (unsigned)std::min<uint64_t>((gwords + 255) / 256, 4096);
    hipLaunchKernelGGL(k_init_groups, dim3(g), dim3(256), 0, ctx->compute, gt.slots, gwords);
  }
  unsigned long long* survivors = (unsigned long long*)ctx->dev_acc;
  fill_zero((uint64_t*)survivors, 2, ctx->compute);
  fill_zero((uint64_t*)ctx->dev_flags, 1, ctx->compute);

  StarArgs base{};
  base.n_dims = nd;
  base.n_meas = d->n_measures;
  for (uint32_t k = 0; k < nd; ++k) {
    base.dim[k] = dims[order[k]].t->view;
    base.gsel[k] = gsel_dim[order[k]];
  }
  for (uint32_t c = 0; c < d->n_measures; ++c) base.meas_size[c] = (uint32_t)cols[nd + c].info.elsize;
  base.groups = gt;
  base.flags = ctx->dev_flags;
  base.survivors = survivors;
  while ((2u << base.zc_shift) <= ctx->zc_line) ++base.zc_shift;

  vx_status status;
  double tp0 = now_ms();
  uint64_t n_chunks = 0, chunk_rows = 0, sdma = 0, kl = 0;
  double kms = 0;
  uint32_t nbuf = 0;
  bool streamed = false;
  {
    Pipeline pipe;
    status = pipe.plan(ctx, d->n_fact, d->chunk_rows, 0, cols);
    if (status == VX_OK) {
      auto kernel = [&](const ChunkView& v) -> vx_status {
        StarArgs a = base;
        a.n = v.rows;
        a.row0 = v.row0;
        for (uint32_t k = 0; k < nd; ++k) {
          a.fk[k] = v.ptr[k];
          if ((v.global_mask >> k) & 1u) {
            a.fk_global |= 1u << k;
            if (cols[k].info.where == Where::Host) a.fk_zc |= 1u << k;
          }
        }
        for (uint32_t c = 0; c < d->n_measures; ++c) {
          a.meas[c] = v.ptr[nd + c];
          if ((v.global_mask >> (nd + c)) & 1u) {
            a.meas_global |= 1u << c;
            if (cols[nd + c].info.where == Where::Host) a.meas_zc |= 1u << c;
          }
        }
        if (a.n == 0) return VX_OK;
        const int items = star_items();
        unsigned g = (unsigned)std::min<uint64_t>((a.n + 256 * items - 1) / (256 * items),
                                                  (uint64_t)ctx->cu_count * 8);
        if (items == 8) launch_star<8>(ktype == VX_I64, count_zc, g, a, ctx->compute);
        else launch_star<4>(ktype == VX_I64, count_zc, g, a, ctx->compute);
        VX_HIP(hipGetLastError());
        return VX_OK;
      };
      status = pipe.run(kernel);
      if (status == VX_OK) {
        VX_HIP(hipStreamSynchronize(ctx->compute));
        n_chunks = pipe.n_chunks();
        chunk_rows = pipe.chunk_rows();
        sdma = pipe.sdma_bytes();
        kms = pipe.kernel_ms();
        kl = pipe.kernel_launches();
        nbuf = pipe.n_buffers();
        streamed = pipe.streamed();
      }
    }
  }
  if (status == VX_OK) status = check_flags(ctx, "star");
  if (status != VX_OK) {
    free_dims();
    return status;
  }
  // groups back to the host, compacted and sorted by (g0, g1)
  std::vector<unsigned long long> host(gwords);
  unsigned long long nsurv[2] = {0, 0};
  if (hipMemcpy(host.data(), gt.slots, gwords * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(nsurv, survivors, 16, hipMemcpyDeviceToHost) != hipSuccess) {
    free_dims();
    set_error("star: reading the group table failed");
    return VX_EHIP;
  }
  free_dims();
  std::vector<vx_group_row> rows;
  for (uint64_t i = 0; i <= gcap; ++i) {
    const unsigned long long* w = host.data() + i * kGroupWords;
    if (w[1] == 0) continue;
    unsigned long long key = i == gcap ? kGroupEmpty : w[0];
    vx_group_row r{};
    r.g0 = (int32_t)(uint32_t)(key >> 32);
    r.g1 = (int32_t)(uint32_t)(key & 0xffffffffull);
    r.count = w[1];
    for (uint32_t m = 0; m < 4; ++m) r.sum[m] = m < d->n_measures ? w[2 + m] : 0;
    rows.push_back(r);
  }
  std::sort(rows.begin(), rows.end(), [](const vx_group_row& a, const vx_group_row& b) {
    return a.g0 != b.g0 ? a.g0 < b.g0 : a.g1 < b.g1;
  });
  out->n_groups = rows.size();
  s.rows = d->n_fact;
  s.chunks = streamed ? n_chunks : 0;
  s.chunk_rows = chunk_rows;
  s.n_buffers = streamed ? nbuf : 0;
  s.sdma_bytes = sdma;
  s.kernel_ms = kms;
  s.kernel_launches = kl;
  for (size_t c = 0; c < cols.size(); ++c) {
    if (cols[c].info.where != Where::Host || cols[c].copy) continue;
    s.zc_mask |= 1u << c;
    if (!count_zc)   // not counted: the wire model's estimate from the estimated selectivities
      s.zc_bytes += (uint64_t)zc_wire_bytes(d->n_fact, (uint64_t)(col_sel[c] * d->n_fact), cols[c].info.elsize,
                                            ctx->zc_line);
  }
  if (count_zc) {
    s.zc_bytes = nsurv[1] << base.zc_shift;   // counted granules x granule
    s.zc_counted = s.zc_mask ? 1u : 0u;
  }
  s.probe_ms = now_ms() - tp0;
  s.total_ms = now_ms() - t0;
  s.survivors = nsurv[0];
  out->stats = s;
  VX_CHECK(rows.size() <= d->groups_cap, VX_ECAPACITY, "star: %zu groups exceed groups_cap %llu",
           rows.size(), (unsigned long long)d->groups_cap);
  std::copy(rows.begin(), rows.end(), d->groups);
  return VX_OK;
}

}  // namespace vx
