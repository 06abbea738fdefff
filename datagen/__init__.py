"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the oracle.

Holds none of the join method's arithmetic: only counter-based random columns
(SplitMix64), Feistel permutations, a Zipf sampler and the workload recipes
built from them.  ``datagen.c`` is compiled into ``libdatagen.so`` by
:func:`build` (OpenMP-parallel; every value depends only on
``(seed, column, row)``, so results do not depend on the thread count).

Every ``fill_*`` function writes into a caller-provided numpy array, which may
wrap pinned host memory.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdatagen.so")
_lib = None


def build() -> str:
    src = os.path.join(_HERE, "datagen.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise RuntimeError(f"datagen library not built: {_SO} (run datagen.build())")
    lib = C.CDLL(_SO)
    u64, vp, i64, dbl = C.c_uint64, C.c_void_p, C.c_int64, C.c_double
    lib.dg_u64.argtypes = [u64, u64, u64]
    lib.dg_u64.restype = u64
    lib.dg_fill_u64.argtypes = [u64, u64, u64, u64, vp]
    lib.dg_uniform.argtypes = [u64, u64, u64, u64, i64, i64, vp, C.c_int]
    lib.dg_perm.argtypes = [u64, u64, u64, u64, u64, vp, C.c_int]
    lib.dg_feistel40.argtypes = [u64, u64, u64, u64, vp]
    lib.dg_probe_fk.argtypes = [u64, u64, u64, dbl, u64, u64, vp, vp, vp, vp]
    lib.dg_zipf.argtypes = [u64, u64, dbl, u64, u64, u64, vp]
    lib.dg_loguniform.argtypes = [u64, u64, u64, u64, dbl, dbl, vp]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data


def _chk(a, dtypes):
    if a is not None:
        if a.dtype not in dtypes:
            raise TypeError(f"bad dtype {a.dtype}")
        if not a.flags.c_contiguous:
            raise ValueError("arrays must be contiguous")


def u64(seed, col, row):
    return int(_load().dg_u64(seed, col, row))


def fill_u64(out, seed, col, row0=0):
    """out[i] = the 64-bit SplitMix output for row row0 + i (an int64 view: uniform over all values)."""
    _chk(out, (np.int64,))
    _load().dg_fill_u64(seed, col, row0, len(out), _p(out))
    return out


def fill_uniform(out, seed, col, lo, hi, row0=0):
    """out[i] = uniform integer in [lo, hi) for row row0 + i."""
    _chk(out, (np.int32, np.int64))
    _load().dg_uniform(seed, col, row0, len(out), int(lo), int(hi), _p(out), out.dtype.itemsize)
    return out


def fill_perm(out, seed, col, n, row0=0):
    """out[i] = perm_n(row0 + i) for a seeded permutation of [0, n)."""
    _chk(out, (np.int32, np.int64))
    _load().dg_perm(seed, col, n, row0, len(out), _p(out), out.dtype.itemsize)
    return out


def fill_feistel40(out, seed, col, row0=0):
    _chk(out, (np.int64,))
    _load().dg_feistel40(seed, col, row0, len(out), _p(out))
    return out


def fill_probe_fk(seed, key_col, n_build, match_frac, keys=None, pay0=None, pay1=None,
                  hit_row=None, row0=0):
    """Streamed-join probe rows: keys matching a Feistel40 build key w.p. match_frac.

    hit_row (optional int64) receives the matched build row index, or -1."""
    n = next(len(a) for a in (keys, pay0, pay1, hit_row) if a is not None)
    for a in (keys, pay0, pay1, hit_row):
        _chk(a, (np.int64,))
    _load().dg_probe_fk(seed, key_col, n_build, float(match_frac), row0, n, _p(keys), _p(pay0),
                        _p(pay1), _p(hit_row))


def fill_zipf(out, seed, col, s, n, row0=0):
    """Zipf(s) ranks in [1, n] (rejection-inversion)."""
    _chk(out, (np.int64,))
    _load().dg_zipf(seed, col, float(s), int(n), row0, len(out), _p(out))
    return out


def loguniform(seed, col, cnt, lo, hi):
    out = np.zeros(cnt, dtype=np.float64)
    _load().dg_loguniform(seed, col, 0, cnt, float(lo), float(hi), _p(out))
    return out


# ---------------------------------------------------------------------------
# Workload recipes (sizes and distributions of the five benchmark workloads).
# ---------------------------------------------------------------------------

SEED_PLAIN, SEED_STREAM, SEED_STAR, SEED_BATCH, SEED_SKEW = 0xC1, 0xC2, 0xC3, 0xC4, 0xC5
SEED_RADIX = 0xC6
SEED_SORT = 0xC7

# column ids
COL_BKEY, COL_BPAY0, COL_BPAY1, COL_PKEY, COL_PPAY0 = 1, 2, 3, 4, 5


def plain_join(n_build=1 << 20, n_probe=1 << 24, seed=SEED_PLAIN, key_range_mult=2):
    """Plain in-memory join: unique int32 build keys (a permutation of [0, n_build)),
    one uniform int32 payload, probe keys uniform over [0, 2*n_build)."""
    bkey = fill_perm(np.empty(n_build, np.int32), seed, COL_BKEY, n_build)
    bpay = fill_uniform(np.empty(n_build, np.int32), seed, COL_BPAY0, -(1 << 31), 1 << 31)
    pkey = fill_uniform(np.empty(n_probe, np.int32), seed, COL_PKEY, 0, key_range_mult * n_build)
    return bkey, bpay, pkey


def stream_build(n_build, seed=SEED_STREAM, out=None):
    """Streamed-join build side: Feistel40 unique int64 keys, two int32 payloads."""
    if out is None:
        out = (np.empty(n_build, np.int64), np.empty(n_build, np.int32), np.empty(n_build, np.int32))
    k, p0, p1 = out
    fill_feistel40(k, seed, COL_BKEY)
    fill_uniform(p0, seed, COL_BPAY0, -(1 << 31), 1 << 31)
    fill_uniform(p1, seed, COL_BPAY1, -(1 << 31), 1 << 31)
    return out


def stream_probe(n_build, n_probe, seed=SEED_STREAM, match_frac=0.1, out=None, row0=0,
                 hit_row=None):
    """Streamed-join probe side: int64 keys (match_frac hit a build key), two int64 payloads."""
    if out is None:
        out = (np.empty(n_probe, np.int64), np.empty(n_probe, np.int64), np.empty(n_probe, np.int64))
    k, p0, p1 = out
    fill_probe_fk(seed, COL_BKEY, n_build, match_frac, k, p0, p1, hit_row, row0=row0)
    return out


STAR_DIM_ROWS = (2556, 200_000, 3_000_000, 2_000_000)
STAR_FILTER_Q = (7, 5, 25, 1)      # filter attribute uniform in [0, q); filter keeps f == 0
STAR_GROUPS = (7, None, None, 100)  # group attribute cardinality per dimension (None: no group)


def star_dims(seed=SEED_STAR, rows=STAR_DIM_ROWS, q=STAR_FILTER_Q, groups=STAR_GROUPS):
    """Dimension tables: dense int32 keys 0..n-1, a filter attribute, optional group attribute."""
    dims = []
    for d, n in enumerate(rows):
        key = np.arange(n, dtype=np.int32)
        filt = fill_uniform(np.empty(n, np.int32), seed, 10 + d, 0, q[d])
        grp = None
        if groups[d] is not None:
            grp = fill_uniform(np.empty(n, np.int32), seed, 20 + d, 0, groups[d])
        dims.append(dict(key=key, filt=filt, lo=0, hi=0, group=grp))
    return dims


def star_fact(n_fact, seed=SEED_STAR, rows=STAR_DIM_ROWS, n_meas=3, out=None, row0=0):
    """Fact table: one int32 FK per dimension (uniform over its keys), int32 measures in [0, 2^20)."""
    if out is None:
        out = ([np.empty(n_fact, np.int32) for _ in rows], [np.empty(n_fact, np.int32) for _ in range(n_meas)])
    fks, meas = out
    for d, n in enumerate(rows):
        fill_uniform(fks[d], seed, 30 + d, 0, n, row0=row0)
    for m in range(n_meas):
        fill_uniform(meas[m], seed, 40 + m, 0, 1 << 20, row0=row0)
    return out


def batch_sizes(n_jobs=256, seed=SEED_BATCH, b_lo=1 << 10, b_hi=1 << 22, r_lo=10.0, r_hi=100.0):
    """Per-join (build rows, probe rows): build log-uniform in [b_lo, b_hi), probe = ratio * build
    with the ratio log-uniform in [r_lo, r_hi)."""
    b = np.floor(loguniform(seed, 50, n_jobs, b_lo, b_hi)).astype(np.int64)
    r = loguniform(seed, 51, n_jobs, r_lo, r_hi)
    p = np.round(r * b).astype(np.int64)
    return b, p


def batch_job(j, n_build, n_probe, seed=SEED_BATCH):
    """One batched join: keys as in the plain join, on a per-job seed."""
    s = seed * 1000003 + j
    bkey = fill_perm(np.empty(n_build, np.int32), s, COL_BKEY, n_build)
    bpay = fill_uniform(np.empty(n_build, np.int32), s, COL_BPAY0, -(1 << 31), 1 << 31)
    pkey = fill_uniform(np.empty(n_probe, np.int32), s, COL_PKEY, 0, 2 * n_build)
    return bkey, bpay, pkey


ZIPF_S = 1.1
ZIPF_N = 1 << 40


def skew_build(n, seed=SEED_SKEW, out=None, row0=0):
    """Skewed build side: Zipf(1.1) int64 keys over [1, 2^40], int64 payload in [0, 2^32)."""
    if out is None:
        out = (np.empty(n, np.int64), np.empty(n, np.int64))
    k, p = out
    fill_zipf(k, seed, COL_BKEY, ZIPF_S, ZIPF_N, row0=row0)
    fill_uniform(p, seed, COL_BPAY0, 0, 1 << 32, row0=row0)
    return out


def scramble40(k):
    """A bijection of [0, 2^40) applied in place to int64 keys (taken mod 2^40): an odd multiply,
    an xor-shift and another odd multiply, each invertible mod 2^40.  Scrambled Zipf keys keep
    their frequencies but lose their order."""
    m = np.uint64((1 << 40) - 1)
    u = k.view(np.uint64)
    u &= m
    u *= np.uint64(0x9E3779B97F4A7C15)
    u &= m
    u ^= u >> np.uint64(20)
    u *= np.uint64(0xC2B2AE3D27D4EB4F)
    u &= m
    return k


def skew_probe(n, seed=SEED_SKEW, out=None, row0=0):
    """Skewed probe side: Zipf(1.1) int64 keys over [1, 2^40]."""
    if out is None:
        out = np.empty(n, np.int64)
    fill_zipf(out, seed, COL_PKEY, ZIPF_S, ZIPF_N, row0=row0)
    return out


def radix_a(n_a, seed=SEED_RADIX, out=None, row0=0):
    """Two-table join, table A: unique int64 keys (a seeded permutation of [0, n_a)) and int64
    values uniform in [0, 2^32)."""
    if out is None:
        out = (np.empty(n_a, np.int64), np.empty(n_a, np.int64))
    k, v = out
    fill_perm(k, seed, COL_BKEY, n_a, row0=row0)
    fill_uniform(v, seed, COL_BPAY0, 0, 1 << 32, row0=row0)
    return out


def radix_b(n_a, n_b, seed=SEED_RADIX, out=None, row0=0):
    """Two-table join, table B: int64 foreign keys uniform over A's keys [0, n_a) and int64
    values uniform in [0, 2^32)."""
    if out is None:
        out = (np.empty(n_b, np.int64), np.empty(n_b, np.int64))
    k, v = out
    fill_uniform(k, seed, COL_PKEY, 0, n_a, row0=row0)
    fill_uniform(v, seed, COL_PPAY0, 0, 1 << 32, row0=row0)
    return out


def sort_keys(n, seed=SEED_SORT, out=None, row0=0):
    """Out-of-core sort input: int64 keys uniform over all 2^64 values."""
    if out is None:
        out = np.empty(n, np.int64)
    return fill_u64(out, seed, COL_BKEY, row0=row0)
