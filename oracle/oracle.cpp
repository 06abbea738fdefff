/*
 * CPU ORACLE — test infrastructure only.
 *
 * A plain, slow, single-threaded restatement of what the streamed
 * join / aggregate / partition path computes, written from the paper
 * ("Vortex: Overcoming Memory Capacity Limitations in GPU-Accelerated
 * Large-Scale Data Analytics", VLDB 2025) and from the textbook definitions
 * of an inner equi-join and GROUP BY.  It shares no code, header, table or
 * helper with the GPU library; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * Integer arithmetic: every SUM is taken in two's complement modulo 2^64
 * (int32 inputs are sign-extended first), so each aggregate has exactly one
 * correct value whatever the summation order.
 *
 * Floating point (the CDF model used to pick range-partition splitters):
 * computed in double from FP32 parameters and FP32 features.
 *
 * Parity status per function is stated in its comment.
 */
#include <cstdint>
#include <cstddef>
#include <cstring>
#include <cmath>
#include <vector>
#include <algorithm>
#include <unordered_map>
#include <map>
#include <utility>
#include <tuple>

extern "C" {

/* A borrowed column of signed integers, 4 or 8 bytes per element. */
typedef struct {
  const void* p;
  int32_t elsize;
  int32_t pad_;
} or_col;

}  // extern "C"

namespace {

inline int64_t at(const or_col& c, uint64_t i) {
  if (c.elsize == 4) return (int64_t)((const int32_t*)c.p)[i];
  return ((const int64_t*)c.p)[i];
}

constexpr uint32_t kMaxSums = 8;

struct BuildAgg {
  uint64_t count = 0;
  uint64_t sums[kMaxSums] = {0, 0, 0, 0, 0, 0, 0, 0};
};

/* Per distinct build key: its multiplicity mB(k) and the sum of each build
 * payload over its rows, sumB_c(k). */
using BuildMap = std::unordered_map<int64_t, BuildAgg>;

BuildMap make_build_map(or_col bkey, const or_col* bpay, uint32_t nbp, uint64_t nb) {
  BuildMap m;
  m.reserve(nb ? nb : 1);
  for (uint64_t i = 0; i < nb; ++i) {
    BuildAgg& a = m[at(bkey, i)];
    a.count += 1;
    for (uint32_t c = 0; c < nbp; ++c) a.sums[c] += (uint64_t)at(bpay[c], i);
  }
  return m;
}

}  // namespace

extern "C" {

/*
 * Inner equi-join on bitwise key equality with multiset semantics, reduced to
 * aggregates (the paper's join query of Sec. 7.1, SUM(A.val + B.val) over
 * A.key == B.key, generalised to several payload columns per side):
 *   out[0]              = |{(b, p) : b.key == p.key}|
 *   out[1 + c]          = SUM over those pairs of build payload c
 *   out[1 + nbp + c]    = SUM over those pairs of probe payload c
 * Hash-map formulation: for each probe row, the matching build rows are
 * exactly the rows stored under its key, so the pair count grows by mB(k),
 * the build sums by sumB_c(k) and each probe sum by mB(k) * p_c.
 * Pinned by: nested-loop brute force, the sort-merge formulation below,
 * the cardinality identity and generator closed forms (tests).
 */
int or_join_agg_hash(or_col bkey, const or_col* bpay, uint32_t nbp, uint64_t nb,
                     or_col pkey, const or_col* ppay, uint32_t npp, uint64_t np, uint64_t* out) {
  if (nbp > kMaxSums) return 1;
  BuildMap m = make_build_map(bkey, bpay, nbp, nb);
  std::memset(out, 0, sizeof(uint64_t) * (1 + nbp + npp));
  for (uint64_t i = 0; i < np; ++i) {
    auto it = m.find(at(pkey, i));
    if (it == m.end()) continue;
    const BuildAgg& a = it->second;
    out[0] += a.count;
    for (uint32_t c = 0; c < nbp; ++c) out[1 + c] += a.sums[c];
    for (uint32_t c = 0; c < npp; ++c) out[1 + nbp + c] += a.count * (uint64_t)at(ppay[c], i);
  }
  return 0;
}

/*
 * The inner equi-join's rows themselves (the join output before any aggregation): for every
 * pair (b, p) with b.key == p.key, in probe order and, within one probe row, in build order,
 * one output row (probe row index p, the build payloads of b, the probe payloads of p), payloads
 * sign-extended to int64.  Columns are written column-major: out_bpay[c * cap + r].
 * Returns the number of pairs; rows past `cap` are counted but not written.
 * Pinned by: a nested-loop brute force, and by its sums and count equalling or_join_agg_hash.
 */
uint64_t or_join_rows(or_col bkey, const or_col* bpay, uint32_t nbp, uint64_t nb, or_col pkey,
                      const or_col* ppay, uint32_t npp, uint64_t np, uint64_t cap, uint64_t* out_row,
                      int64_t* out_bpay, int64_t* out_ppay) {
  std::unordered_map<int64_t, std::vector<uint64_t>> rows_of;
  rows_of.reserve(nb ? nb : 1);
  for (uint64_t b = 0; b < nb; ++b) rows_of[at(bkey, b)].push_back(b);
  uint64_t n = 0;
  for (uint64_t i = 0; i < np; ++i) {
    auto it = rows_of.find(at(pkey, i));
    if (it == rows_of.end()) continue;
    for (uint64_t b : it->second) {
      if (n < cap) {
        out_row[n] = i;
        for (uint32_t c = 0; c < nbp; ++c) out_bpay[c * cap + n] = at(bpay[c], b);
        for (uint32_t c = 0; c < npp; ++c) out_ppay[c * cap + n] = at(ppay[c], i);
      }
      ++n;
    }
  }
  return n;
}

/* A prepared build side, so one build can serve several probe slices (used to
 * check sampled probe chunks of a full-size run). */
struct or_build {
  BuildMap m;
  uint32_t nbp;
};

or_build* or_build_create(or_col bkey, const or_col* bpay, uint32_t nbp, uint64_t nb) {
  if (nbp > kMaxSums) return nullptr;
  or_build* b = new or_build;
  b->m = make_build_map(bkey, bpay, nbp, nb);
  b->nbp = nbp;
  return b;
}

void or_build_free(or_build* b) { delete b; }

/* Same aggregates as or_join_agg_hash for the probe rows given. */
int or_build_probe(const or_build* b, or_col pkey, const or_col* ppay, uint32_t npp, uint64_t np,
                   uint64_t* out) {
  std::memset(out, 0, sizeof(uint64_t) * (1 + b->nbp + npp));
  for (uint64_t i = 0; i < np; ++i) {
    auto it = b->m.find(at(pkey, i));
    if (it == b->m.end()) continue;
    const BuildAgg& a = it->second;
    out[0] += a.count;
    for (uint32_t c = 0; c < b->nbp; ++c) out[1 + c] += a.sums[c];
    for (uint32_t c = 0; c < npp; ++c) out[1 + b->nbp + c] += a.count * (uint64_t)at(ppay[c], i);
  }
  return 0;
}

uint64_t or_build_distinct(const or_build* b) { return (uint64_t)b->m.size(); }

/*
 * The same join aggregates by sort-merge: sort both sides by key, walk the
 * two sorted runs, and for each key present on both sides add
 * mB*mP pairs, mP*sumB_c and mB*sumP_c.  An independent second formulation.
 */
int or_join_agg_sortmerge(or_col bkey, const or_col* bpay, uint32_t nbp, uint64_t nb,
                          or_col pkey, const or_col* ppay, uint32_t npp, uint64_t np,
                          uint64_t* out) {
  std::vector<std::pair<int64_t, uint64_t>> bs(nb), ps(np);
  for (uint64_t i = 0; i < nb; ++i) bs[i] = {at(bkey, i), i};
  for (uint64_t i = 0; i < np; ++i) ps[i] = {at(pkey, i), i};
  std::sort(bs.begin(), bs.end());
  std::sort(ps.begin(), ps.end());
  std::memset(out, 0, sizeof(uint64_t) * (1 + nbp + npp));
  uint64_t i = 0, j = 0;
  while (i < nb && j < np) {
    if (bs[i].first < ps[j].first) { ++i; continue; }
    if (ps[j].first < bs[i].first) { ++j; continue; }
    int64_t k = bs[i].first;
    uint64_t i1 = i, j1 = j;
    while (i1 < nb && bs[i1].first == k) ++i1;
    while (j1 < np && ps[j1].first == k) ++j1;
    uint64_t mb = i1 - i, mp = j1 - j;
    out[0] += mb * mp;
    for (uint32_t c = 0; c < nbp; ++c) {
      uint64_t s = 0;
      for (uint64_t r = i; r < i1; ++r) s += (uint64_t)at(bpay[c], bs[r].second);
      out[1 + c] += mp * s;
    }
    for (uint32_t c = 0; c < npp; ++c) {
      uint64_t s = 0;
      for (uint64_t r = j; r < j1; ++r) s += (uint64_t)at(ppay[c], ps[r].second);
      out[1 + nbp + c] += mb * s;
    }
    i = i1;
    j = j1;
  }
  return 0;
}

/*
 * Star join with GROUP BY (the paper's star-schema plan, Sec. 7.1: the
 * dimensions are filtered and hashed, the fact table is joined against every
 * dimension and aggregated).  A fact row survives iff, for every dimension d,
 * its foreign key equals the key of a dimension row whose filter attribute
 * lies in [lo_d, hi_d].  The group of a survivor is the pair of group
 * attributes of the (at most two) dimensions that carry a group column, in
 * dimension order; missing attributes read as 0.  Output: one row per group
 * with count > 0, ascending by (g0, g1), holding the row count and the
 * mod-2^64 SUM of each measure.  Dimension keys must be unique (primary
 * keys): returns 1 on a duplicate key, 2 if more than cap groups, else 0.
 */
typedef struct {
  or_col key;
  uint64_t n;
  or_col filt;
  int64_t lo, hi;
  or_col group; /* p == NULL: no group attribute */
} or_dim;

int or_star_groupby(const or_dim* dims, uint32_t ndims, const or_col* fks, const or_col* meas,
                    uint32_t nmeas, uint64_t nfact, int64_t* out_g, uint64_t* out_cnt,
                    uint64_t* out_sums, uint64_t cap, uint64_t* n_groups) {
  struct DimRow { bool pass; int64_t g; };
  std::vector<std::unordered_map<int64_t, DimRow>> maps(ndims);
  for (uint32_t d = 0; d < ndims; ++d) {
    for (uint64_t r = 0; r < dims[d].n; ++r) {
      int64_t k = at(dims[d].key, r);
      int64_t f = at(dims[d].filt, r);
      DimRow row{f >= dims[d].lo && f <= dims[d].hi,
                 dims[d].group.p ? at(dims[d].group, r) : 0};
      if (!maps[d].emplace(k, row).second) return 1;
    }
  }
  struct Acc { uint64_t count = 0; std::vector<uint64_t> sums; };
  std::map<std::pair<int64_t, int64_t>, Acc> groups;
  for (uint64_t i = 0; i < nfact; ++i) {
    int64_t g[2] = {0, 0};
    int ng = 0;
    bool ok = true;
    for (uint32_t d = 0; d < ndims && ok; ++d) {
      auto it = maps[d].find(at(fks[d], i));
      if (it == maps[d].end() || !it->second.pass) { ok = false; break; }
      if (dims[d].group.p && ng < 2) g[ng++] = it->second.g;
    }
    if (!ok) continue;
    Acc& a = groups[{g[0], g[1]}];
    if (a.sums.empty()) a.sums.assign(nmeas, 0);
    a.count += 1;
    for (uint32_t c = 0; c < nmeas; ++c) a.sums[c] += (uint64_t)at(meas[c], i);
  }
  *n_groups = groups.size();
  if (groups.size() > cap) return 2;
  uint64_t r = 0;
  for (auto& kv : groups) {
    out_g[2 * r] = kv.first.first;
    out_g[2 * r + 1] = kv.first.second;
    out_cnt[r] = kv.second.count;
    for (uint32_t c = 0; c < nmeas; ++c) out_sums[r * nmeas + c] = kv.second.sums[c];
    ++r;
  }
  return 0;
}

/*
 * Partitioning (Sec. 6.2, RadixPartitionExKer).
 *
 * Radix partition by raw key bits: the paper groups tuples by the low bits of
 * the key (bits 0..23 in its join); here bits [shift, shift + log2p).
 */
void or_part_ids_bits(or_col keys, uint64_t n, uint32_t shift, uint32_t log2p, uint32_t* ids) {
  uint64_t mask = log2p >= 64 ? ~0ULL : ((1ULL << log2p) - 1);
  for (uint64_t i = 0; i < n; ++i) ids[i] = (uint32_t)(((uint64_t)at(keys, i) >> shift) & mask);
}

/* The MurmurHash3 64-bit finalizer (Appleby, public domain): a bijection of
 * the 64-bit words.  Pinned by its published inverse (tests). */
static uint64_t fmix64(uint64_t h) {
  h ^= h >> 33;
  h *= 0xff51afd7ed558ccdULL;
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ULL;
  h ^= h >> 33;
  return h;
}

/* The whole 64-bit finalizer value of each key, so that it can be pinned. */
void or_hash64(or_col keys, uint64_t n, uint64_t* out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = fmix64((uint64_t)at(keys, i));
}

/* Radix partition by a hash of the key, for skewed keys (the paper leaves a
 * better hash for skew out of its scope; this reading takes the MurmurHash3
 * 64-bit finalizer and keeps its top log2p bits). */
void or_part_ids_hash(or_col keys, uint64_t n, uint32_t log2p, uint32_t* ids) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t h = fmix64((uint64_t)at(keys, i));
    ids[i] = log2p == 0 ? 0u : (uint32_t)(h >> (64 - log2p));
  }
}

/* Range partition: the id of a key is the number of splitters <= key, so
 * partition p holds [s_{p-1}, s_p) with s_{-1} = -inf, s_{P-1} = +inf. */
void or_part_ids_range(or_col keys, uint64_t n, const int64_t* splitters, uint32_t nsplit,
                       uint32_t* ids) {
  for (uint64_t i = 0; i < n; ++i) {
    int64_t k = at(keys, i);
    uint32_t c = 0;
    for (uint32_t s = 0; s < nsplit; ++s) c += splitters[s] <= k ? 1u : 0u;
    ids[i] = c;
  }
}

void or_histogram(const uint32_t* ids, uint64_t n, uint32_t nparts, uint64_t* hist) {
  for (uint32_t p = 0; p < nparts; ++p) hist[p] = 0;
  for (uint64_t i = 0; i < n; ++i) hist[ids[i]] += 1;
}

/*
 * Clustering followed by find_boundary, as the paper describes it
 * (Sec. 6.2.1): rows are reordered so that equal group ids are contiguous,
 * keeping input order inside a group (a stable sort by group id); then
 * boundary[h] is set at every position where the id differs from the
 * previous one, and every entry still unset is filled with the next valid
 * boundary, with boundary[nparts] = n.  Writes the clustered row order
 * (order[j] = input row at clustered position j) and the boundary array.
 * Pinned by the closed form boundary = exclusive prefix sum of the
 * per-group histogram (tests).
 */
void or_cluster_boundary(const uint32_t* ids, uint64_t n, uint32_t nparts, uint64_t* order,
                         uint64_t* boundary) {
  std::vector<uint64_t> idx(n);
  for (uint64_t i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](uint64_t a, uint64_t b) { return ids[a] < ids[b]; });
  for (uint64_t j = 0; j < n; ++j) order[j] = idx[j];
  const uint64_t NA = ~0ULL;
  for (uint32_t h = 0; h <= nparts; ++h) boundary[h] = NA;
  for (uint64_t j = 0; j < n; ++j) {
    uint32_t h = ids[idx[j]];
    if (j == 0 || ids[idx[j - 1]] != h) boundary[h] = j;
  }
  boundary[nparts] = n;
  for (int64_t h = (int64_t)nparts - 1; h >= 0; --h)
    if (boundary[h] == NA) boundary[h] = boundary[h + 1];
}

/*
 * Late-materialization threshold (Sec. 6.3): a column whose estimated
 * selectivity is below TH = E / (C_l2 * N_exchange) is read on demand by
 * zero-copy access instead of being streamed.
 */
double or_late_mat_threshold(double elem_bytes, double line_bytes, double n_exchange) {
  return elem_bytes / (line_bytes * n_exchange);
}

/*
 * Bernoulli row sample: row i is kept iff the (i+1)-th output of the SplitMix64 generator
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * started from state `seed` is below frac * 2^64.  Keys of kept rows are written in row
 * order; returns their count.
 */
static uint64_t splitmix64_next(uint64_t* state) {
  *state += 0x9E3779B97F4A7C15ULL;
  uint64_t z = *state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* The first n outputs of the SplitMix64 generator started from state `seed`,
 * so that the stream the sampler draws from can be pinned. */
void or_splitmix64(uint64_t seed, uint64_t n, uint64_t* out) {
  uint64_t state = seed;
  for (uint64_t i = 0; i < n; ++i) out[i] = splitmix64_next(&state);
}

uint64_t or_sample_bernoulli(or_col keys, uint64_t n, uint64_t seed, double frac, int64_t* out) {
  uint64_t thr = frac >= 1.0 ? ~0ULL : (uint64_t)(frac * 18446744073709551616.0);
  uint64_t state = seed, m = 0;
  for (uint64_t i = 0; i < n; ++i)
    if (splitmix64_next(&state) < thr) out[m++] = at(keys, i);
  return m;
}

/*
 * Learned range-partition splitters: a cumulative-distribution model of the
 * key sample (not in the paper, which leaves skew handling out of scope).
 *
 * Feature of a key: a piecewise-linear base-2 logarithm of its offset above
 * the sample minimum (Mitchell's approximation: the exponent plus the next 23
 * mantissa bits, read as a fixed-point number), as an FP32 value in [0, 1):
 *   u = key - kmin (0 if key < kmin, at most 2^63 - 1), l = floor(log2(u + 1)),
 *   m = the 23 bits of (u + 1) below its leading one,
 *   x = float(l * 2^23 + m) * scale, scale = 1 / (L * 2^23) as FP32.
 * Exact in FP32 up to the single int->float rounding (round to nearest even).
 */
float or_cdf_feature(int64_t key, int64_t kmin, float scale) {
  uint64_t u = key < kmin ? 0ULL : (uint64_t)key - (uint64_t)kmin;
  if (u > 0x7FFFFFFFFFFFFFFFULL) u = 0x7FFFFFFFFFFFFFFFULL;   /* saturate: v <= 2^63 */
  uint64_t v = u + 1;
  uint32_t l = 63;
  while (!((v >> l) & 1ULL)) --l;
  uint64_t m = l >= 23 ? (v >> (l - 23)) & 0x7FFFFFULL : (v << (23 - l)) & 0x7FFFFFULL;
  int64_t fixed = ((int64_t)l << 23) | (int64_t)m;
  return (float)fixed * scale;
}

/* Mid-CDF targets of a sorted sample: t_i = (#{< k_i} + #{<= k_i}) / (2n),
 * evaluated in double and rounded to FP32; equal keys get equal targets. */
void or_cdf_targets(const int64_t* sorted, uint64_t n, float* t) {
  uint64_t i = 0;
  while (i < n) {
    uint64_t j = i;
    while (j < n && sorted[j] == sorted[i]) ++j;
    double v = ((double)i + (double)j) / (2.0 * (double)n);
    for (uint64_t r = i; r < j; ++r) t[r] = (float)v;
    i = j;
  }
}

/*
 * One-hidden-layer ReLU network y(x) = b2 + sum_j w2_j * relu(w1_j * x + b1_j),
 * hidden width H.  Parameter layout: w1[H], b1[H], w2[H], b2.
 * Mean squared error L = (1/n) sum_i (y_i - t_i)^2 and its gradient, in
 * double.  relu'(0) is taken as 0.  grad has the same layout as params.
 */
double or_mlp_loss_grad(const float* params, uint32_t H, const float* x, const float* t, uint64_t n,
                        double* grad) {
  const float* w1 = params;
  const float* b1 = params + H;
  const float* w2 = params + 2 * H;
  double b2 = params[3 * H];
  for (uint32_t j = 0; j < 3 * H + 1; ++j) grad[j] = 0.0;
  double loss = 0.0;
  std::vector<double> z(H), h(H);
  for (uint64_t i = 0; i < n; ++i) {
    double y = b2;
    for (uint32_t j = 0; j < H; ++j) {
      z[j] = (double)w1[j] * (double)x[i] + (double)b1[j];
      h[j] = z[j] > 0.0 ? z[j] : 0.0;
      y += (double)w2[j] * h[j];
    }
    double e = y - (double)t[i];
    loss += e * e;
    double r = 2.0 * e / (double)n;
    grad[3 * H] += r;
    for (uint32_t j = 0; j < H; ++j) {
      grad[2 * H + j] += r * h[j];
      if (z[j] > 0.0) {
        double g = r * (double)w2[j];
        grad[H + j] += g;
        grad[j] += g * (double)x[i];
      }
    }
  }
  return loss / (double)n;
}

/* Network output at each x, in double from FP32 parameters. */
void or_mlp_forward(const float* params, uint32_t H, const float* x, uint64_t n, double* y) {
  for (uint64_t i = 0; i < n; ++i) {
    double acc = params[3 * H];
    for (uint32_t j = 0; j < H; ++j) {
      double z = (double)params[j] * (double)x[i] + (double)params[H + j];
      if (z > 0.0) acc += (double)params[2 * H + j] * z;
    }
    y[i] = acc;
  }
}

/*
 * One Adam step (Kingma and Ba, 2015) on FP32 parameters with FP32 moments,
 * evaluated in double and rounded back:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 */
void or_adam_step(float* params, float* m, float* v, const float* grad, uint32_t np, uint32_t t,
                  double lr, double b1, double b2, double eps) {
  double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
  for (uint32_t j = 0; j < np; ++j) {
    double g = grad[j];
    double mj = b1 * (double)m[j] + (1.0 - b1) * g;
    double vj = b2 * (double)v[j] + (1.0 - b2) * g * g;
    m[j] = (float)mj;
    v[j] = (float)vj;
    params[j] = (float)((double)params[j] - lr * (mj / c1) / (std::sqrt(vj / c2) + eps));
  }
}

/*
 * Splitters from a CDF model over a sorted sample: y_env is the running
 * maximum of the model output along the sorted sample (a monotone envelope);
 * splitter j (j = 1..P-1) is the smallest sample key whose envelope reaches
 * j/P.  Where one key carries the envelope across several quantiles, that key
 * is isolated in a partition of its own by also emitting key + 1.  Splitters
 * are strictly increasing; fewer than P-1 may result.  Returns their count.
 */
uint32_t or_splitters_from_cdf(const int64_t* sorted, const double* y, uint64_t n, uint32_t P,
                               int64_t* out) {
  std::vector<int64_t> s;
  double env = -INFINITY;
  uint32_t j = 1;
  for (uint64_t i = 0; i < n && j < P; ++i) {
    if (y[i] > env) env = y[i];
    if (env >= (double)j / (double)P) {
      int64_t k = sorted[i];
      uint32_t crossed = 0;
      while (j < P && env >= (double)j / (double)P) { ++j; ++crossed; }
      if (s.empty() || s.back() < k) s.push_back(k);
      if (crossed > 1 && k < INT64_MAX && s.back() < k + 1) s.push_back(k + 1);
    }
  }
  for (size_t i = 0; i < s.size(); ++i) out[i] = s[i];
  return (uint32_t)s.size();
}

/* ---------------------------------------------------------------- out-of-core sort (Sec. 6.1)
 *
 * The external sort's result has a plain definition: the input keys in
 * ascending signed order.  or_sort writes that order with the C++ library
 * sort.  Pinned by tests against numpy's sort and by the permutation and
 * order invariants on random, duplicate-heavy, extreme and empty inputs.
 */
void or_sort(or_col keys, uint64_t n, int64_t* out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = at(keys, i);
  std::sort(out, out + n);
}

/* The regroup step of the merge phase (Sec. 6.1.3): sorted runs are cut at a
 * global rank r so that the r smallest elements of their union (ties taken
 * from the lower-numbered run first, and in run order within a run) lie in
 * front of the cuts.  Written as that definition: every element becomes
 * (value, run, position), the triples are sorted, and the first r are counted
 * per run.  Pinned by tests of its invariants (cut sums, order across the cut,
 * tie order) on small runs. */
void or_merge_cuts(const int64_t* const* runs, const uint64_t* len, uint32_t n_runs, uint64_t r,
                   uint64_t* cut) {
  std::vector<std::tuple<int64_t, uint32_t, uint64_t>> all;
  for (uint32_t j = 0; j < n_runs; ++j)
    for (uint64_t i = 0; i < len[j]; ++i) all.emplace_back(runs[j][i], j, i);
  std::sort(all.begin(), all.end());
  for (uint32_t j = 0; j < n_runs; ++j) cut[j] = 0;
  for (uint64_t k = 0; k < r && k < all.size(); ++k) ++cut[std::get<1>(all[k])];
}

}  // extern "C"
