/*
 * Seeded synthetic input generators for the streamed join / star join /
 * batched join / skewed partitioned join workloads.
 *
 * This module holds no step of the join method itself: it only produces
 * input columns.  Every value is a pure function of (seed, column id, row),
 * so any slice of any column can be regenerated independently and in
 * parallel, and the GPU library and the CPU oracle see identical inputs.
 *
 * Random source: the SplitMix64 output function (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014), used as a
 * counter-based generator: the (row+1)-th SplitMix64 output of a stream whose
 * initial state is itself a SplitMix64 output of (seed, column).
 */
#include <stdint.h>
#include <stddef.h>
#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_state(uint64_t seed, uint64_t col) {
  return sm64_out(seed + GOLDEN * (col + 1));
}

static inline uint64_t draw(uint64_t state, uint64_t row) {
  return sm64_out(state + GOLDEN * (row + 1));
}

/* floor(u * n / 2^64): maps a uniform 64-bit word onto [0, n). */
static inline uint64_t mulhi(uint64_t u, uint64_t n) {
  return (uint64_t)(((unsigned __int128)u * n) >> 64);
}

uint64_t dg_u64(uint64_t seed, uint64_t col, uint64_t row) {
  return draw(stream_state(seed, col), row);
}

void dg_fill_u64(uint64_t seed, uint64_t col, uint64_t row0, uint64_t cnt, uint64_t* out) {
  uint64_t st = stream_state(seed, col);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)cnt; ++i) out[i] = draw(st, row0 + (uint64_t)i);
}

static inline void store(void* out, int elsize, uint64_t i, int64_t v) {
  if (elsize == 4) ((int32_t*)out)[i] = (int32_t)v;
  else ((int64_t*)out)[i] = v;
}

/* Uniform integers in [lo, hi). */
void dg_uniform(uint64_t seed, uint64_t col, uint64_t row0, uint64_t cnt,
                int64_t lo, int64_t hi, void* out, int elsize) {
  uint64_t st = stream_state(seed, col);
  uint64_t span = (uint64_t)hi - (uint64_t)lo;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)cnt; ++i) {
    uint64_t u = draw(st, row0 + (uint64_t)i);
    int64_t v = span ? (int64_t)((uint64_t)lo + mulhi(u, span)) : (int64_t)u;
    store(out, elsize, (uint64_t)i, v);
  }
}

/* 4-round balanced Feistel network on 2*h bits: a bijection of [0, 2^(2h)). */
static inline uint64_t feistel(uint64_t fst, int h, uint64_t x) {
  uint64_t mask = (1ULL << h) - 1;
  uint64_t l = (x >> h) & mask, r = x & mask;
  for (uint64_t round = 0; round < 4; ++round) {
    uint64_t f = draw(fst, (round << 40) | r) & mask;
    uint64_t nl = r;
    r = l ^ f;
    l = nl;
  }
  return (l << h) | r;
}

static inline int half_bits(uint64_t n) {
  int b = 0;
  while (b < 62 && (1ULL << b) < n) ++b;  /* 2^b >= n */
  return (b + 1) / 2;                     /* 2^(2h) >= n */
}

/* A pseudorandom permutation of [0, n) by cycle-walking a Feistel network. */
static inline uint64_t perm_at(uint64_t fst, int h, uint64_t n, uint64_t i) {
  uint64_t x = feistel(fst, h, i);
  while (x >= n) x = feistel(fst, h, x);
  return x;
}

void dg_perm(uint64_t seed, uint64_t col, uint64_t n, uint64_t row0, uint64_t cnt,
             void* out, int elsize) {
  uint64_t fst = stream_state(seed, col);
  int h = half_bits(n < 2 ? 2 : n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)cnt; ++i)
    store(out, elsize, (uint64_t)i, (int64_t)perm_at(fst, h, n, row0 + (uint64_t)i));
}

/* Feistel40: a fixed bijection of [0, 2^40); distinct rows give distinct keys. */
void dg_feistel40(uint64_t seed, uint64_t col, uint64_t row0, uint64_t cnt, int64_t* out) {
  uint64_t fst = stream_state(seed, col);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)cnt; ++i)
    out[i] = (int64_t)feistel(fst, 20, row0 + (uint64_t)i);
}

/*
 * Streamed-join probe side.  Row r matches with probability match_frac: then
 * its key is Feistel40(j) for a build row j uniform in [0, n_build); otherwise
 * it is Feistel40 of an index in [n_build, 2^40), which no build key uses.
 * Payload columns are uniform in [-2^32, 2^32).  key_col is the column id of
 * the build keys' Feistel network, so both sides share one bijection.
 * hit_row (optional) receives the matched build row, or -1.
 */
void dg_probe_fk(uint64_t seed, uint64_t key_col, uint64_t n_build, double match_frac,
                 uint64_t row0, uint64_t cnt, int64_t* keys, int64_t* pay0, int64_t* pay1,
                 int64_t* hit_row) {
  uint64_t fst = stream_state(seed, key_col);
  uint64_t s_sel = stream_state(seed, 100), s_hit = stream_state(seed, 101);
  uint64_t s_miss = stream_state(seed, 102);
  uint64_t s_p0 = stream_state(seed, 103), s_p1 = stream_state(seed, 104);
  double thr_d = match_frac * 18446744073709551616.0;
  uint64_t thr = match_frac >= 1.0 ? UINT64_MAX : (uint64_t)thr_d;
  uint64_t miss_span = (1ULL << 40) - n_build;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)cnt; ++i) {
    uint64_t r = row0 + (uint64_t)i;
    int hit = draw(s_sel, r) < thr;
    uint64_t idx = hit ? mulhi(draw(s_hit, r), n_build) : n_build + mulhi(draw(s_miss, r), miss_span);
    if (keys) keys[i] = (int64_t)feistel(fst, 20, idx);
    if (pay0) pay0[i] = (int64_t)(draw(s_p0, r) >> 31) - (1LL << 32);
    if (pay1) pay1[i] = (int64_t)(draw(s_p1, r) >> 31) - (1LL << 32);
    if (hit_row) hit_row[i] = hit ? (int64_t)idx : -1;
  }
}

/*
 * Zipf(s) over ranks [1, n] by rejection-inversion (W. Hormann and
 * G. Derflinger, "Rejection-inversion to generate variates from monotone
 * discrete distributions", ACM TOMACS 6(3), 1996).  The uniform draws of row r
 * come from a private SplitMix64 sequence seeded by (seed, col, r).
 */
static inline double zh(double x, double s) {            /* integral of x^-s */
  double lx = log(x);
  double t = (1.0 - s) * lx;
  return fabs(t) > 1e-8 ? expm1(t) / (1.0 - s) : lx * (1.0 + 0.5 * t);
}
static inline double zh_inv(double x, double s) {
  double t = x * (1.0 - s);
  if (t < -1.0) t = -1.0;
  return exp(fabs(t) > 1e-8 ? log1p(t) / (1.0 - s) : x * (1.0 - 0.5 * t));
}
static inline double zh_pt(double x, double s) { return exp(-s * log(x)); }

void dg_zipf(uint64_t seed, uint64_t col, double s, uint64_t n, uint64_t row0, uint64_t cnt,
             int64_t* out) {
  uint64_t st = stream_state(seed, col);
  double dn = (double)n;
  double hx1 = zh(1.5, s) - 1.0;
  double hn = zh(dn + 0.5, s);
  double sq = 2.0 - zh_inv(zh(2.5, s) - zh_pt(2.0, s), s);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)cnt; ++i) {
    uint64_t rs = draw(st, row0 + (uint64_t)i);
    uint64_t k = 1;
    for (uint64_t it = 0;; ++it) {
      double u01 = (double)(sm64_out(rs + GOLDEN * (it + 1)) >> 11) * 0x1.0p-53;
      double u = hn + u01 * (hx1 - hn);
      double x = zh_inv(u, s);
      double kd = floor(x + 0.5);
      if (kd < 1.0) kd = 1.0;
      if (kd > dn) kd = dn;
      if (kd - x <= sq || u >= zh(kd + 0.5, s) - zh_pt(kd, s)) { k = (uint64_t)kd; break; }
    }
    out[i] = (int64_t)k;
  }
}

/* Log-uniform integer sizes: floor(exp(U[ln lo, ln hi))). */
void dg_loguniform(uint64_t seed, uint64_t col, uint64_t row0, uint64_t cnt, double lo, double hi,
                   double* out) {
  uint64_t st = stream_state(seed, col);
  double a = log(lo), b = log(hi);
  for (uint64_t i = 0; i < cnt; ++i) {
    double u01 = (double)(draw(st, row0 + i) >> 11) * 0x1.0p-53;
    out[i] = exp(a + u01 * (b - a));
  }
}
