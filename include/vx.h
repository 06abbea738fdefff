/*
 * vx.h — C ABI of an MI355X (gfx950) streamed equi-join / aggregate library.
 *
 * The operations follow "Vortex: Overcoming Memory Capacity Limitations in
 * GPU-Accelerated Large-Scale Data Analytics" (VLDB 2025):
 *   - an equi-join reduced to aggregates, SUM(A.val + B.val) over
 *     A.key == B.key (Sec. 7.1, hash join query), where the probe side lives in
 *     host memory and is larger than the device (Sec. 1, 3: data starts in CPU
 *     memory, nothing is cached on the GPU);
 *   - the probe side streamed in chunks through two device buffers while the
 *     kernel works on the previous chunk (Sec. 5.3, Pipelined Executor), with
 *     copies submitted only when they can run at once (Sec. 4.3, first design
 *     principle);
 *   - columns of low estimated selectivity read by zero-copy access instead of
 *     being copied, with the threshold TH = E / (C_l2 * N_exchange) (Sec. 6.3);
 *   - a star join of small filtered dimension tables kept on the GPU against a
 *     streamed fact table, with GROUP BY (Sec. 7.1, Star Schema Benchmark plan);
 *   - radix partitioning into groups with a boundary array (Sec. 6.2.1) for the
 *     case where the build side exceeds device memory (Sec. 6.2).
 * Learned (CDF-model) range partitioning, the batched join (queue-draining
 * kernels in one HIP graph) and directly indexed tables for keys that fill a
 * narrow range are additions of this library; the paper leaves skew-aware
 * partitioning out of its scope (Sec. 6.2.1).
 *
 * Conventions for every entry point:
 *   - Every call returns a vx_status; nothing throws across the ABI.  On a
 *     status other than VX_OK, vx_last_error() returns a thread-local message.
 *   - Calls are synchronous: they return after their results are on the host
 *     (or written to the caller's output arrays).
 *   - Column pointers (vx_col.data) may point to device memory of the context's
 *     device, or to pinned, device-mapped host memory (hipHostMalloc or
 *     vx_host_alloc).  Pageable host memory is rejected with VX_ENOTPINNED.
 *     Inputs are borrowed for the duration of the call and never written.
 *   - All device memory the library uses comes from the caller's arena given
 *     to vx_ctx_create; if a call's working set does not fit, it returns
 *     VX_EBUDGET and leaves the context usable.  The library calls no device
 *     allocator of its own.
 *   - Integer SUMs are two's-complement modulo 2^64; int32 values are
 *     sign-extended first.  Key equality is bitwise; every key value is legal.
 *   - A context is bound to one device and is not thread-safe.
 */
#ifndef VX_H
#define VX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VX_OK = 0,
  VX_EINVAL = 1,        /* bad argument (null pointer, type mismatch, size) */
  VX_EBUDGET = 2,       /* the arena cannot hold the call's working set */
  VX_ENOMEM = 3,        /* host allocation failed */
  VX_EHIP = 4,          /* a HIP runtime call failed */
  VX_ENOTPINNED = 5,    /* a host column is not pinned / device-mapped */
  VX_ECAPACITY = 6,     /* an output array is too small (its required size is reported) */
  VX_EUNSUPPORTED = 7,  /* a valid request the library does not handle */
  VX_EDUPKEY = 8        /* duplicate key in a build declared unique */
} vx_status;

typedef enum { VX_I32 = 1, VX_I64 = 2 } vx_type;

/* A borrowed column: data points to n elements of type `type`. */
typedef struct {
  const void* data;
  int32_t type;     /* vx_type */
  int32_t reserved; /* must be 0 */
} vx_col;

/* ------------------------------------------------------------------------ context */

typedef struct vx_ctx vx_ctx;

/*
 * Create a context on `device` over the caller's device buffer `arena` of
 * `arena_bytes` (the device-memory budget; 256-byte aligned).  `stream` is a
 * hipStream_t for compute work, or NULL for a library-owned stream; a second,
 * library-owned stream carries the host-to-device copies.  The arena stays
 * owned by the caller and must outlive the context.
 */
vx_status vx_ctx_create(int device, void* arena, uint64_t arena_bytes, void* stream, vx_ctx** out);
vx_status vx_ctx_destroy(vx_ctx* ctx);

/* Thread-local text describing the last non-OK status (never NULL). */
const char* vx_last_error(void);

/* Bytes of the arena currently held by the context and live tables. */
uint64_t vx_ctx_arena_used(const vx_ctx* ctx);

/* Pinned, device-mapped host memory for columns (page-locked; freed with vx_host_free). */
vx_status vx_host_alloc(uint64_t bytes, void** out);
vx_status vx_host_free(void* p);

/*
 * Measure the host link and device memory on this machine: host-to-device copy rate (64 MiB
 * copies), zero-copy read rate (contiguous and strided) and the zero-copy transfer granule (the
 * largest stride at which every touched line still crosses the link), and a device streaming
 * read, plus the device-to-host direction (copies and kernel stores) alone and beside
 * host-to-device copies.  `pinned` is caller-owned pinned host memory of `bytes` (>= 64 MiB) whose
 * contents are read only; the device-to-host legs write into the context's own pinned scratch.
 * The granule becomes the line size of the context's late-materialization model (Sec. 6.3,
 * C_l2); before a calibration it is 128 bytes.
 */
typedef struct {
  double h2d_gbs;
  double zc_read_gbs;
  double hbm_read_gbs;
  uint32_t zc_granule;
  uint32_t zc_stride_bytes[8];
  double zc_stride_gelems[8];   /* elements per ns at each stride */
  double d2h_gbs;               /* device-to-host copy rate (64 MiB copies) */
  double duplex_sdma_gbs;       /* host-to-device and device-to-host copies at once, both directions summed */
  double zc_write_gbs;          /* kernel stores to mapped pinned host memory (16-byte stores,
                                   one workgroup per 16 compute units) */
  double duplex_zcw_gbs;        /* host-to-device copies beside such kernel stores to host, summed;
                                   the best of three runs */
  double duplex_zcr_gbs;        /* kernel reads of host memory beside device-to-host copies, summed */
} vx_link_calib;

vx_status vx_calibrate(vx_ctx* ctx, void* pinned, uint64_t bytes, vx_link_calib* out);

/* ------------------------------------------------------------------------ statistics */

/* Statistics of one call.  The radix join (VX_JOIN_RADIX) and vx_sort give some fields their
 * own meaning; their declarations below say which. */
typedef struct {
  uint64_t rows;            /* probe (or fact) rows processed */
  uint64_t chunks;          /* chunks streamed (0: device-resident input) */
  uint64_t chunk_rows;      /* rows per chunk used */
  uint64_t sdma_bytes;      /* bytes copied host-to-device by the copy stream */
  uint64_t zc_bytes;        /* bytes read from host memory in place (zero-copy).  Gathers (probe
                               payloads, star fact columns): granules touched x granule size,
                               counted by the kernels under VX_PROBE_COUNT_ZC (each wave counts the
                               distinct granules holding the rows it reads), else estimated by
                               the wire model; in-place scans: bytes read */
  uint32_t zc_mask;         /* bit c set: probe payload / fact column c read by zero-copy */
  uint32_t n_buffers;       /* chunk buffers used by the pipeline */
  double build_ms;          /* wall time of the build phase */
  double probe_ms;          /* wall time of the probe / stream phase */
  double total_ms;
  double kernel_ms;         /* summed device time of the main kernels (HIP events) */
  uint64_t kernel_launches; /* main-kernel launches timed in kernel_ms */
  uint64_t table_bytes;     /* device bytes of the hash table(s) */
  uint64_t n_parts;         /* partitions used (partitioned join) */
  double imbalance;         /* max/mean rows per partition (partitioned join) */
  double part_ms;           /* partition pass wall time */
  double train_ms;          /* CDF model training wall time */
  uint64_t singleton_rows;  /* rows resolved through singleton partitions */
  uint64_t survivors;       /* star join: fact rows that pass every dimension; partitioned join:
                               probe rows routed to a partition table (not a singleton) */
  double imbalance_tables;  /* partitioned join: max/mean build + probe rows over the partitions
                               joined through a table (singletons excluded) */
  double imbalance_distinct; /* partitioned join: max/mean distinct build keys over the same
                                partitions (their pre-aggregating tables grow with it) */
  uint32_t zc_counted;      /* 1: zc_bytes of the gathers was counted by the kernels */
  uint32_t reserved;
} vx_stats;

/* ------------------------------------------------------------------------ build / probe */

enum {
  VX_UNIQUE = 1,  /* keys are unique; a duplicate fails the build with VX_EDUPKEY */
  VX_PREAGG = 2,  /* duplicates allowed: the table stores per key its count and payload sums */
  VX_HASHED = 4   /* OR-ed with one of the above: always a hash table, never a direct one */
};

typedef struct {
  vx_col key;
  const vx_col* pay;   /* n_pay payload columns (NULL if n_pay == 0) */
  uint32_t n_pay;      /* <= 4 */
  uint32_t flags;      /* VX_UNIQUE or VX_PREAGG, optionally | VX_HASHED */
  uint64_t n;          /* rows */
  float load_factor;   /* 0 = default (0.5); table capacity is a power of two */
  uint32_t reserved;
} vx_build_desc;

typedef struct vx_table vx_table;

/*
 * Build a device hash table over the build side (the table the paper keeps in
 * GPU memory while the other side streams, Sec. 5.1, 7.1).  Host-resident
 * build columns are read in place by zero-copy.  The table is carved from the
 * arena and owned by the library until vx_table_destroy.
 *
 * Direct tables: when the keys are device-resident and VX_HASHED is not set,
 * the build first measures their range (min..max, leaving out the key equal to
 * the table's empty marker, INT32_MIN or INT64_MIN, which has a record of its
 * own).  If the range is no wider than the hash table's capacity at the load
 * factor, key k is stored in slot k - min instead of a hashed slot, with a
 * power-of-two capacity no smaller than the range.  A VX_UNIQUE build whose n
 * keys are exactly the n values of their range (no empty-marker key) is dense:
 * every key of the range is present, so its slots hold only the payloads (none
 * without payloads) and a presence byte per key of the range catches a repeated key.
 * Results are the same for every layout; a probe then reads one slot, or none
 * for keys outside the range.  Host-resident keys always get a hash table.
 */
vx_status vx_build(vx_ctx* ctx, const vx_build_desc* desc, vx_table** out);
vx_status vx_table_destroy(vx_table* table);

/* Aggregates of one join: count, then per build payload, then per probe payload. */
typedef struct {
  uint64_t match_count;
  uint64_t sum[8]; /* sum[c] for build payload c (c < n_build_pay), then probe payloads */
} vx_agg;

enum {
  VX_LATE_AUTO = -1,   /* per column: zero-copy if the wire-byte model says it moves fewer bytes
                          than streaming, with the selectivity measured on the first chunk */
  VX_LATE_SDMA = 0,    /* stream every payload column with the keys */
  VX_LATE_ZC = 1,      /* read payload columns of matching rows by zero-copy */
  VX_LATE_PAPER = 2    /* the paper's rule: zero-copy iff selectivity < E / (C_l2 * 1), with C_l2 the
                          context's zero-copy granule */
};

typedef struct {
  vx_col key;
  const vx_col* pay;   /* probe payload columns, read only for matching rows */
  uint32_t n_pay;      /* <= 4; n_build_pay + n_pay <= 8 */
  int32_t late_mat;    /* VX_LATE_* */
  uint64_t n;
  uint64_t chunk_rows; /* 0 = auto */
  uint32_t n_buffers;  /* chunk buffers in the pipeline, 2..4; 0 = 2 (the paper's mem A / mem B) */
  uint32_t flags;      /* 0 or VX_PROBE_COUNT_ZC */
  vx_agg* chunk_aggs;  /* optional host array: per-chunk aggregates (cap chunk_aggs_cap) */
  uint64_t chunk_aggs_cap;
} vx_probe_desc;

enum {
  /* The probe kernels count the zero-copy traffic of their gathers exactly: per wave, the
     distinct granules that hold a matching row, per zero-copied column; vx_stats.zc_bytes is
     then that count times the granule (zc_counted = 1).  Without it zc_bytes is the wire model's
     estimate from the per-chunk match counts.  The count makes the gather loop about 4% slower,
     so it is asked for, not always on. */
  VX_PROBE_COUNT_ZC = 1
};

/*
 * Probe `table` with every probe row and aggregate the matches: the probe side
 * of the paper's hash join (Sec. 7.1) run by its pipelined executor (Sec. 5.3).
 * Device-resident keys are probed in place.  Host-resident keys are streamed
 * through n_buffers chunk buffers carved from the arena (the executor's mem A /
 * mem B; VX_EBUDGET if two chunks of one row do not fit): the copy of chunk
 * c + 1 runs while the kernel works on chunk c, and each copy is submitted only
 * once its buffer is free, so it never waits in a hardware queue (Sec. 4.3,
 * the immediate-execution principle).  Probe payload columns in host memory are
 * read only for matching rows, by zero-copy loads, or streamed with the keys,
 * as late_mat chooses (Sec. 6.3).
 * Arguments: `table` from vx_build on the same context; desc->key of the
 * table's key type; desc->pay[c] of n rows each, int32 or int64.  Results:
 * *out = count and sums (build payloads, then probe payloads), mod 2^64; per
 * chunk in desc->chunk_aggs when given (VX_ECAPACITY if there are more chunks
 * than chunk_aggs_cap).  `stats` may be NULL.
 * Errors: VX_EINVAL (type mismatch, more than 4 payloads or 8 sums, n_buffers
 * outside 2..4, a table of another context), VX_ENOTPINNED, VX_EBUDGET.
 */
vx_status vx_probe_stream(vx_ctx* ctx, const vx_table* table, const vx_probe_desc* desc,
                          vx_agg* out, vx_stats* stats);

/*
 * The join's rows themselves (an ExKernel's outputs, Sec. 5.2, saved back as the executor runs,
 * Sec. 5.3): probe like vx_probe_stream, against a table built with VX_UNIQUE, and also write
 * one output row per probe row whose key is in the table:
 *   row[r] = the probe row's index, build_pay[c][r] = the table's payload c, probe_pay[c][r] =
 *   the probe's payload c (payloads sign-extended to int64), in no particular order.
 * Each column is caller-owned memory of `cap` rows, device memory or pinned host memory; the
 * probe kernel writes it directly (stores to host memory run beside the host-to-device
 * copies).  NULL payload columns are skipped.  `n_out` receives the number of output rows;
 * when it exceeds `cap` the call returns VX_ECAPACITY and nothing past `cap` is written.
 * `out` and `stats` are as for vx_probe_stream.  VX_EUNSUPPORTED for a pre-aggregating table.
 */
typedef struct {
  uint64_t* row;               /* probe row index per output row */
  int64_t* build_pay[4];       /* one column per table payload (NULL: skipped) */
  int64_t* probe_pay[4];       /* one column per probe payload (NULL: skipped) */
  uint64_t cap;                /* rows each column holds */
  uint64_t n_out;              /* [out] output rows */
} vx_join_rows;

vx_status vx_probe_rows(vx_ctx* ctx, const vx_table* table, const vx_probe_desc* desc, vx_join_rows* rows,
                        vx_agg* out, vx_stats* stats);


/* ------------------------------------------------------------------------ one-shot joins */

typedef enum {
  VX_JOIN_PLAIN = 1,        /* build + probe of two tables */
  VX_JOIN_STAR = 2,         /* star join with GROUP BY */
  VX_JOIN_BATCH = 3,        /* many independent device-resident joins in one launch */
  VX_JOIN_PARTITIONED = 4,  /* build side too large for the budget: partition, then join */
  VX_JOIN_RADIX = 5         /* both tables too large for the budget: cluster both, join per partition */
} vx_join_kind;

typedef struct {
  vx_col key;
  uint64_t n;
  vx_col filter;       /* filter attribute; a row passes iff lo <= filter <= hi */
  int64_t lo, hi;
  vx_col group;        /* group attribute, or data == NULL for none */
} vx_star_dim;

typedef struct {
  int32_t g0, g1;      /* group attributes of the first two dimensions that have one (0 if absent) */
  uint64_t count;
  uint64_t sum[4];     /* per measure */
} vx_group_row;

typedef struct {
  uint32_t n_dims;             /* 1..4 */
  uint32_t n_measures;         /* 0..4 */
  vx_star_dim dims[4];         /* device or host; keys unique (VX_EDUPKEY otherwise) */
  vx_col fact_fk[4];           /* fact foreign key per dimension */
  vx_col measure[4];
  uint64_t n_fact;
  uint64_t chunk_rows;         /* 0 = auto */
  int32_t late_mat;            /* VX_LATE_*: fact columns after the first probed one */
  uint32_t flags;              /* 0 or VX_PROBE_COUNT_ZC (counts the fact columns' gathers) */
  vx_group_row* groups;        /* host output, ascending (g0, g1), count > 0 only */
  uint64_t groups_cap;
} vx_star_join;

/*
 * Batched join: many independent device-resident joins in one call.  A job whose build keys fill
 * their value range exactly (n unique keys from min to min + n - 1, measured on every call) is
 * joined through a direct table indexed by key - min; other jobs through hash tables, which drop
 * probe keys outside the build keys' range.  Mode 0 probes tables from LDS: a table of at most
 * 128 KiB whole, a larger one by regions of 128 KiB, for which the job's probe keys are first
 * partitioned by region into arena memory (about 4 or 8 bytes per probe row; a job whose buffers
 * do not fit the arena is probed from device memory instead).  Results do not depend on any of
 * this.  Mode-0 stats: n_parts = jobs whose probe side was partitioned, survivors = jobs probed
 * by regions, kernel_launches = kernels in the graph.  Errors: VX_EDUPKEY when a job's build keys
 * repeat; VX_EINVAL for host-resident columns, mixed key types or more than 4096 jobs.
 */
typedef struct {
  uint32_t n_jobs;
  int32_t mode;                /* 0: one HIP graph launch of queue-draining kernels (build phase,
                                  probe-side partitioning beside it, probe phase); 1: two launches
                                  per job.
                                  Mode 0 keeps its graph, tables and descriptors in the arena after
                                  the call, for the next mode-0 call with the same jobs
                                  (vx_ctx_arena_used counts them); every other call on the context
                                  gives them back before it allocates */
  const vx_col* build_key;     /* per job, device-resident, unique keys */
  const vx_col* build_pay;     /* per job one payload column (data may be NULL) */
  const uint64_t* n_build;
  const vx_col* probe_key;     /* per job, device-resident */
  const uint64_t* n_probe;
  vx_agg* out;                 /* per job: match_count and sum[0] = SUM(build payload) */
  uint32_t tile_rows;          /* 0 = autotuned */
  uint32_t block;              /* workgroup size, 0 = autotuned */
  float load_factor;           /* 0 = autotuned */
  uint32_t flags;              /* 0, or VX_HASHED: hash tables for every job (no direct tables) */
} vx_batch_join;

typedef enum {
  VX_PART_AUTO = 0,            /* range splitters from the trained model, or from the sample
                                  quantiles when their singleton partitions hold 5 points more of
                                  the sample; then vx_partition: the lower imbalance on the key
                                  sample (those splitters or radix-hash); partitioned join: the
                                  range splitters when they isolate a heavy key (a singleton
                                  partition), else radix-hash.  method_used reports the choice */
  VX_PART_RADIX_HASH = 1,      /* top bits of a 64-bit mix of the key */
  VX_PART_RADIX_BITS = 2,      /* raw key bits [shift, shift + log2 P) as in the paper */
  VX_PART_LEARNED = 3,         /* CDF-model range splitters, trained on the GPU */
  VX_PART_QUANTILE = 4,        /* range splitters from sample quantiles (no model) */
  VX_PART_UNTRAINED = 5,       /* CDF model at its initial weights (control) */
  VX_PART_RANGE = 6            /* caller-given splitters */
} vx_part_method;

typedef struct {
  uint32_t method;             /* vx_part_method */
  uint32_t n_parts;            /* 0 = 256; radix methods round up to 2^k; range methods may
                                  return fewer (repeated quantiles merge) */
  uint32_t shift;              /* VX_PART_RADIX_BITS */
  uint32_t train_steps;        /* 0 = 1000 */
  float sample_frac;           /* 0 = 0.01 */
  float lr;                    /* 0 = 1e-2 */
  uint64_t seed;               /* sampling seed */
  const int64_t* splitters;    /* VX_PART_RANGE: n_splitters ascending keys */
  uint32_t n_splitters;
  uint32_t reserved;
} vx_part_opts;

/*
 * Partitioned join (Sec. 6.2): count and SUM(build payload) over all matching pairs, for a build
 * side whose table would not fit the budget.  The build side (key + at most one payload, host
 * or device) is clustered by partition in one pass.  The clustered copy goes in the arena when
 * the range splitters' key sample predicts that the partition tables fit beside it, else in
 * the context's pinned host scratch.  Each partition is pre-aggregated per key (duplicates
 * allowed) into a table sized by its distinct keys.  The probe keys (host or device, no
 * payloads) then stream once through the chunk pipeline.  Keys that carry several quantiles of
 * the sample get singleton partitions, which are resolved from counts alone.  When
 * probe.chunk_aggs is set it receives one vx_agg per partition (chunk_aggs_cap >= n_parts).
 * stats: n_parts, imbalance (max/mean build + probe rows per partition), singleton_rows,
 * survivors (probe rows routed to a table), part_ms (pass 1), train_ms (splitters),
 * probe_ms (pass 2), sdma_bytes and zc_bytes (host-link bytes).
 * Errors: VX_EBUDGET when the largest partition's transient table or the partition scratch
 * does not fit; VX_ENOMEM when pinned host scratch cannot be had; VX_EUNSUPPORTED for more than
 * one build payload or any probe payload.
 */
typedef struct {
  vx_build_desc build;         /* host or device; VX_PREAGG implied */
  vx_probe_desc probe;         /* host or device keys; no probe payloads; chunk_aggs per partition */
  vx_part_opts part;
} vx_partitioned_join;

/*
 * Radix-partitioned join of two large tables A and B (Sec. 6.2, the hash-join case study):
 * count and SUM(payload) of each side over all pairs with A.key == B.key, so that
 * SUM(A.val + B.val) = agg.sum[0] + agg.sum[1] (mod 2^64) with one payload per side.
 * Pass 1 clusters each table by partition, chunk by chunk through the chunk pipeline (the
 * paper's radix-partition step: raw key bits [shift, shift + log2 n_parts), or the top bits
 * of a 64-bit mix of the key), and keeps each chunk's boundary array.  The clustered copies go
 * in pinned host scratch (written by a kernel that stores to mapped memory beside the
 * host-to-device copies) or, when both fit beside pass 2, in the arena.  Pass 2 takes the
 * partitions in turn: A's rows of partition p, read in place from every clustered chunk, are
 * pre-aggregated per key (count, payload sum) into a table in the arena, and B's rows of p look
 * it up.  A partition whose A rows exceed the largest table the arena holds is built in slices,
 * each probed by all of B's rows of that partition.  With one partition nothing is clustered:
 * both tables are read in place.
 * Keys: any value, duplicates on both sides (multiset semantics); both sides share one type.
 * Payloads: at most one per side; sums wrap mod 2^64 (int32 sign-extended).
 * agg: match_count; sum[0..n_pay_a) A's payload, then B's.  When b.chunk_aggs is set it receives
 * one vx_agg per partition (chunk_aggs_cap >= n_parts), partition p holding the pairs whose key
 * maps to p.
 * stats: n_parts, imbalance (max/mean A + B rows per partition), part_ms (pass 1), probe_ms
 * (pass 2), build_ms and kernel_ms (pass 2's build and probe kernels, summed from HIP events
 * around each launch), sdma_bytes (pass 1 copies), zc_bytes (bytes read in place from host
 * memory), table_bytes (the pass-2 table), chunks (pass-2 build slices: one build and one probe
 * launch each), rows = b.n.
 * Errors: VX_EINVAL for a bad argument (n_parts not a power of two or above 1024, shift > 63,
 * key types that differ); VX_EUNSUPPORTED for more than one payload on a side; VX_EBUDGET when
 * the arena cannot hold pass 1's buffers or a pass-2 table of 64 slots; VX_ENOMEM when pinned
 * host scratch cannot be had.
 */
typedef struct {
  vx_build_desc a;             /* host or device; flags ignored (duplicates allowed) */
  vx_probe_desc b;             /* host or device; chunk_aggs: one per partition */
  uint32_t n_parts;            /* power of two <= 1024; 0 = the fewest whose expected largest
                                  table fits the arena */
  uint32_t shift;              /* first key bit of the partition id (raw-bits partitioning) */
  uint32_t hash;               /* 0: raw key bits as in the paper; 1: top bits of a 64-bit mix */
  int32_t placement;           /* clustered copies: 0 auto, 1 pinned host scratch, 2 arena */
} vx_radix_join;

typedef struct {
  int32_t kind;                /* vx_join_kind */
  int32_t reserved;
  union {
    struct { vx_build_desc build; vx_probe_desc probe; } plain;
    vx_star_join star;
    vx_batch_join batch;
    vx_partitioned_join part;
    vx_radix_join radix;
  } u;
} vx_join_desc;

typedef struct {
  vx_agg agg;                  /* PLAIN, PARTITIONED, RADIX */
  uint64_t n_groups;           /* STAR: groups with count > 0 (required capacity on VX_ECAPACITY) */
  uint32_t part_method_used;   /* PARTITIONED */
  uint32_t reserved;
  vx_stats stats;
} vx_join_out;

/*
 * One-shot join of any kind.  PLAIN is the paper's join query SUM(A.val + B.val) over
 * A.key == B.key, reduced to the match count and per-column sums (Sec. 7.1): vx_build of the
 * build side, then vx_probe_stream of the probe side, then the table is freed.  STAR is the
 * Star Schema Benchmark plan of Sec. 7.1 (filter the dimensions, build their tables on the GPU,
 * stream the fact table, aggregate per group).  PARTITIONED and RADIX are the partitioned joins
 * of Sec. 6.2 for build sides that do not fit the budget; BATCH runs many small joins in one
 * graph.  Each kind's descriptor above states its layout, ownership and errors.  `out` must not
 * be NULL; out->stats is filled on success.
 */
vx_status vx_join_agg(vx_ctx* ctx, const vx_join_desc* desc, vx_join_out* out);

/* ------------------------------------------------------------------------ partitioning */

typedef struct {
  vx_col key;                  /* device or pinned host */
  const vx_col* pay;           /* payload columns carried by the scatter */
  uint32_t n_pay;              /* <= 4 */
  uint32_t reserved;
  uint64_t n;
  vx_part_opts opts;
  void* out_key;               /* optional: clustered keys (host or device, n elements) */
  void* const* out_pay;        /* optional: clustered payloads, one per column */
} vx_partition_desc;

typedef struct {
  uint32_t method_used;
  uint32_t n_parts;
  uint64_t* hist;              /* caller array [n_parts_cap] */
  uint64_t* boundary;          /* caller array [n_parts_cap + 1]: exclusive prefix, boundary[P] = n */
  int64_t* splitters;          /* caller array [n_parts_cap] for range methods (count in n_splitters) */
  uint32_t n_parts_cap;
  uint32_t n_splitters;
  double imbalance;            /* max/mean of hist */
  double est_imbalance_radix;  /* on the sample */
  double est_imbalance_range;  /* on the sample */
  double final_loss;           /* learned: training loss after the last step */
  float* model;                /* optional caller array [193]: w1[64], b1[64], w2[64], b2 */
} vx_partition_out;

/*
 * Assign every row to a partition, histogram the assignment, and write the
 * boundary array (Sec. 6.2.1: boundary[h] is the first clustered position of
 * group h, empty groups take the next boundary, boundary[P] = n).  If out_key
 * is given, rows are scattered stably (input order kept within a partition).
 */
vx_status vx_partition(vx_ctx* ctx, const vx_partition_desc* desc, vx_partition_out* out);

/* ------------------------------------------------------------------------ out-of-core sort */

typedef struct {
  vx_col key;                  /* pinned host or device; sorted in place */
  uint64_t n;
  uint64_t chunk_rows;         /* pass-1 run length; 0 = the largest power of two whose buffers fit */
  uint32_t n_buffers;          /* pass-1 pipeline buffers; 0 = 2 */
  uint32_t reserved;
} vx_sort_desc;

/*
 * Out-of-core sort (Sec. 6.1): the n keys (int32 or int64) in ascending signed order, written
 * back in place.
 * Pass 1 (the paper's SortExKernel) streams runs of chunk_rows keys through the chunk pipeline.
 * Each run is sorted on the GPU by an LSD radix sort (stable passes of 8-bit digits over tiles of
 * 8192 keys sorted in LDS) and stored to the context's pinned host scratch by a kernel on a
 * second stream.
 * Pass 2 (the paper's MergeExKernel) cuts every run at the ranks 0, chunk_rows, 2 chunk_rows, ...
 * (vx_merge_cuts).  For each output range it copies the runs' segments in, merges them in a
 * tree of merge-path kernels, and stores the result to its place in the key column.  One run is
 * stored in place directly.
 * Needs about 5 runs of device memory for pass 1 and 4 for pass 2, plus n keys of pinned host
 * scratch when there are several runs.
 * stats (nullable): rows = n, chunks = runs, chunk_rows, n_buffers, part_ms (pass 1), probe_ms
 * (pass 2), kernel_ms (pass-1 sort kernels) and build_ms (pass-2 merge kernels), both summed from
 * HIP events; sdma_bytes (host-to-device copies), kernel_launches, total_ms.
 * Errors: VX_EINVAL (bad column type; NULL column with n > 0); VX_ENOTPINNED; VX_EBUDGET when a
 * run's buffers do not fit the arena; VX_ENOMEM when pinned host scratch cannot be had.
 */
vx_status vx_sort(vx_ctx* ctx, const vx_sort_desc* desc, vx_stats* stats);

/*
 * The regroup step of the sort's merge phase (Sec. 6.1.3), for callers that merge sorted runs
 * themselves.  runs[j] holds run_len[j] int64 keys in ascending order (host memory).  cut[j]
 * receives how many of run j's keys are among the `rank` smallest keys of all runs, with equal
 * keys taken from lower-numbered runs first.  So cut sums to rank, and every key in front of a
 * cut is <= every key behind one.  Host work only (binary searches).
 * Errors: VX_EINVAL for NULL arrays or rank above the total length.
 */
vx_status vx_merge_cuts(const int64_t* const* runs, const uint64_t* run_len, uint32_t n_runs, uint64_t rank,
                        uint64_t* cut);

/* ------------------------------------------------------------------------ CDF model kernels */

/*
 * The kernels behind VX_PART_LEARNED, exported so their numerics can be checked on their
 * own.  The model is y(x) = b2 + sum_{j<64} w2_j * relu(w1_j * x + b1_j) in FP32, with
 * parameters laid out as float[193] = {w1[64], b1[64], w2[64], b2} in host memory; x, t are
 * n floats in device or pinned host memory; outputs are host arrays.
 *
 * vx_cdf_loss_grad: the mean squared error (1/n) sum (y_i - t_i)^2 and its gradient, from
 *   one forward/backward pass (relu'(0) = 0); gradient accumulated in FP64 in a fixed order
 *   and rounded to FP32.  Deterministic.
 * vx_cdf_forward: y_i for every x_i (the evaluation used to place splitters).
 * vx_cdf_train: `steps` full-batch Adam steps (beta 0.9 / 0.999, eps 1e-8) from the given
 *   parameters, updated in place; the learning rate at step k is lr * (1 + cos(pi (k-1) / steps)) / 2
 *   (lr at the first step; lr 0 = 1e-2); *final_loss = loss after training.
 */
vx_status vx_cdf_loss_grad(vx_ctx* ctx, const float* x, const float* t, uint64_t n,
                           const float* params, float* grad, double* loss);
vx_status vx_cdf_forward(vx_ctx* ctx, const float* x, uint64_t n, const float* params, float* y);
vx_status vx_cdf_train(vx_ctx* ctx, const float* x, const float* t, uint64_t n, float* params,
                       uint32_t steps, float lr, double* final_loss);

/* ------------------------------------------------------------------------ no device allocation */

/* Bytes of the fixed device array behind vx_join_plain_noalloc, per GPU. */
#define VX_NOALLOC_SCRATCH_BYTES (32ull << 20)

/*
 * For callers that cannot allocate device memory at all, not even a context's arena: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  The PLAIN join of
 * vx_join_agg (build a table over the build side, probe it with every probe row, count and sum
 * the matches) on device-resident columns, with the hash table in a fixed array of the library
 * (VX_NOALLOC_SCRATCH_BYTES on each GPU the library runs on, held until the process ends)
 * instead of in an arena.  It needs no context, allocates nothing (no device or host memory, no
 * stream, no event), and does not synchronize: the work is enqueued on `stream` (a hipStream_t;
 * NULL for the null stream) on the calling thread's current device, and the call returns.
 *   b, p: as for VX_JOIN_PLAIN; every column device memory of the current device; the table is
 *         always hashed (VX_HASHED implied), VX_UNIQUE or VX_PREAGG, load_factor as for vx_build.
 *   out:  caller-owned device memory of 10 uint64 words, written in stream order:
 *         out[0] match count, out[1 .. 8] the sums (build payloads, then probe payloads,
 *         mod 2^64, unused words 0), out[9] error flags: bit 0 a duplicate key in a VX_UNIQUE
 *         build, bit 1 a full table (neither leaves the aggregates meaningful).
 * Errors (returned before anything is enqueued): VX_EINVAL for a bad argument or a column that is
 * not device memory of the current device; VX_EBUDGET when the build side's table (capacity the
 * next power of two >= n / load_factor, 8-64 B slots) exceeds the array, e.g. more than 2^20
 * unique int32 rows with one int32 payload at the default load factor; VX_EHIP.
 * Every call on a GPU shares that GPU's array and keeps the last call's table in it: calls that
 * overlap on one GPU (other streams, other threads) race and must be ordered by the caller.
 */
vx_status vx_join_plain_noalloc(const vx_build_desc* b, const vx_probe_desc* p, void* stream, uint64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* VX_H */
