"""Pins for the oracle's join aggregates (CPU only).

The oracle's hash-map join is checked against things it does not share code
with: a numpy nested-loop brute force on tiny inputs, the cardinality identity
count = sum_k mB(k) * mP(k), exact big-integer sums reduced mod 2^64, and the
generators' own closed forms (dense permutation keys; generator-known match
rows of the streamed workload).
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import datagen
import oracle

M64 = 1 << 64


def brute(bkey, bpays, pkey, ppays):
    """Nested loop over all (build, probe) pairs: the definition itself."""
    eq = np.equal.outer(np.asarray(bkey, np.int64), np.asarray(pkey, np.int64))  # [nb, np]
    bi, pi = np.nonzero(eq)
    out = [len(bi)]
    out += [sum(int(v) for v in np.asarray(c, np.int64)[bi]) % M64 for c in bpays]
    out += [sum(int(v) for v in np.asarray(c, np.int64)[pi]) % M64 for c in ppays]
    return out


def _rand_cols(rng, n, key_lo, key_hi, kdt, ndt_b, ndt_p, nb_cols=2, np_cols=2, nprobe=None):
    bkey = rng.integers(key_lo, key_hi, n).astype(kdt)
    pkey = rng.integers(key_lo, key_hi, nprobe if nprobe is not None else 2 * n).astype(kdt)
    info_b = np.iinfo(ndt_b)
    info_p = np.iinfo(ndt_p)
    bp = [rng.integers(info_b.min, info_b.max, n, dtype=ndt_b, endpoint=True) for _ in range(nb_cols)]
    pp = [rng.integers(info_p.min, info_p.max, len(pkey), dtype=ndt_p, endpoint=True) for _ in range(np_cols)]
    return bkey, bp, pkey, pp


@pytest.mark.parametrize("method", ["hash", "sortmerge"])
@pytest.mark.parametrize("kdt", [np.int32, np.int64])
def test_brute_force_random_duplicates(method, kdt):
    rng = np.random.default_rng(1)
    for trial in range(20):
        n = int(rng.integers(0, 300))
        span = int(rng.integers(1, 50))
        bkey, bp, pkey, pp = _rand_cols(rng, n, -span, span, kdt, np.int32, np.int64,
                                        nprobe=int(rng.integers(0, 600)))
        assert oracle.join_agg(bkey, bp, pkey, pp, method) == brute(bkey, bp, pkey, pp)


@settings(max_examples=60, deadline=None)
@given(st.lists(st.integers(-3, 3), max_size=40), st.lists(st.integers(-3, 3), max_size=60),
       st.integers(0, 2**32))
def test_brute_force_hypothesis(bk, pk, seed):
    rng = np.random.default_rng(seed)
    bkey = np.array(bk, np.int64)
    pkey = np.array(pk, np.int64)
    bp = [rng.integers(-2**63, 2**63 - 1, len(bk), dtype=np.int64, endpoint=True)]
    pp = [rng.integers(-2**31, 2**31 - 1, len(pk), dtype=np.int64, endpoint=True)]
    exp = brute(bkey, bp, pkey, pp)
    assert oracle.join_agg(bkey, bp, pkey, pp, "hash") == exp
    assert oracle.join_agg(bkey, bp, pkey, pp, "sortmerge") == exp


def test_extreme_keys_and_sentinels():
    """Every key value is legal, including the extremes a GPU table may use as an empty marker."""
    i64 = np.iinfo(np.int64)
    i32 = np.iinfo(np.int32)
    bkey = np.array([i64.min, i64.max, 0, -1, i64.min, 5], np.int64)
    pkey = np.array([i64.min, i64.max, i64.max, 7, -1, i64.min, i64.min], np.int64)
    bp = [np.array([1, 2, 3, 4, 5, 6], np.int64)]
    pp = [np.array([10, 20, 30, 40, 50, 60, 70], np.int64)]
    exp = brute(bkey, bp, pkey, pp)
    # i64.min appears twice in build and three times in probe: 6 pairs; i64.max 1x2; -1 1x1.
    assert exp[0] == 6 + 2 + 1
    assert oracle.join_agg(bkey, bp, pkey, pp) == exp
    bk32 = np.array([i32.min, i32.max, 0], np.int32)
    pk32 = np.array([i32.min, i32.min, i32.max], np.int32)
    assert oracle.join_agg(bk32, [], pk32, []) == [3]


def test_empty_sides():
    e64 = np.zeros(0, np.int64)
    k = np.arange(10, dtype=np.int64)
    assert oracle.join_agg(e64, [e64], k, [k]) == [0, 0, 0]
    assert oracle.join_agg(k, [k], e64, [e64]) == [0, 0, 0]
    assert oracle.join_agg(e64, [], e64, []) == [0]


def test_cardinality_identity():
    """count == sum over keys of mB(k) * mP(k), counted with np.unique."""
    rng = np.random.default_rng(7)
    bkey = rng.zipf(1.3, 20000).astype(np.int64)
    pkey = rng.zipf(1.3, 50000).astype(np.int64)
    ub, cb = np.unique(bkey, return_counts=True)
    up, cp = np.unique(pkey, return_counts=True)
    common, ib, ip = np.intersect1d(ub, up, return_indices=True)
    expect = int(np.sum(cb[ib].astype(object) * cp[ip].astype(object)))
    assert oracle.join_agg(bkey, [], pkey, [])[0] == expect
    assert oracle.join_agg(bkey, [], pkey, [], "sortmerge")[0] == expect


def test_mod_2_64_wraparound():
    """Sums wrap modulo 2^64 exactly as big-integer sums reduced mod 2^64."""
    n = 1000
    bkey = np.zeros(n, np.int64)            # one key, n copies
    pkey = np.zeros(3 * n, np.int64)        # 3n probes of it: 3n^2 pairs
    bp = [np.full(n, np.iinfo(np.int64).max, np.int64)]
    pp = [np.full(3 * n, np.iinfo(np.int64).min, np.int64)]
    out = oracle.join_agg(bkey, bp, pkey, pp)
    assert out[0] == 3 * n * n
    assert out[1] == (3 * n * n * (2**63 - 1)) % M64
    assert out[2] == (3 * n * n * (-2**63)) % M64


def test_plain_workload_closed_form():
    """Dense permutation build keys: pay_of_key[] is a direct array, so
    count = #{probe < n_build} and SUM = sum of pay_of_key[probe] over those."""
    nb, np_ = 1 << 14, 1 << 18
    bkey, bpay, pkey = datagen.plain_join(nb, np_, seed=11)
    assert np.array_equal(np.sort(bkey), np.arange(nb, dtype=np.int32))
    pay_of_key = np.empty(nb, np.int64)
    pay_of_key[bkey] = bpay
    hit = pkey < nb
    cnt = int(hit.sum())
    s = int(pay_of_key[pkey[hit]].sum()) % M64
    assert oracle.join_agg(bkey, [bpay], pkey, []) == [cnt, s]
    assert 0.45 < cnt / np_ < 0.55


def test_stream_workload_closed_form():
    """Generator-known match rows: count = #hits, build sums from the hit rows,
    probe sums over hit rows; misses are disjoint from build keys by construction."""
    nb, np_ = 1 << 13, 1 << 17
    bk, b0, b1 = datagen.stream_build(nb, seed=21)
    hit_row = np.empty(np_, np.int64)
    pk, p0, p1 = datagen.stream_probe(nb, np_, seed=21, hit_row=hit_row)
    h = hit_row >= 0
    exp = [int(h.sum()),
           int(b0.astype(np.int64)[hit_row[h]].sum()) % M64,
           int(b1.astype(np.int64)[hit_row[h]].sum()) % M64,
           int(p0[h].sum()) % M64, int(p1[h].sum()) % M64]
    assert len(np.unique(bk)) == nb
    assert np.array_equal(pk[h], bk[hit_row[h]])
    assert oracle.join_agg(bk, [b0, b1], pk, [p0, p1]) == exp
    assert 0.08 < h.mean() < 0.12


def test_prepared_build_slices_sum_to_whole():
    rng = np.random.default_rng(3)
    bkey = rng.integers(0, 500, 3000).astype(np.int64)
    bp = [rng.integers(-1000, 1000, 3000).astype(np.int32)]
    pkey = rng.integers(0, 700, 10000).astype(np.int64)
    pp = [rng.integers(-10**12, 10**12, 10000).astype(np.int64)]
    whole = oracle.join_agg(bkey, bp, pkey, pp)
    pb = oracle.PreparedBuild(bkey, bp)
    parts = [pb.probe(pkey[a:b], [pp[0][a:b]]) for a, b in ((0, 1234), (1234, 9000), (9000, 10000))]
    assert [sum(c) % M64 for c in zip(*parts)] == whole
    assert pb.distinct() == len(np.unique(bkey))
