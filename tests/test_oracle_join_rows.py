"""Pins of the oracle's materialized join output (the join's rows before aggregation).

Each output row is (probe row index, build payloads, probe payloads) for one pair (b, p) with
b.key == p.key, in probe order and then build order.  Checked against a nested-loop brute force
written here, and against the aggregate oracle (count and sums of the same pairs).
"""
import numpy as np
import pytest

import datagen
import oracle

M64 = 1 << 64


def _brute(bk, bps, pk, pps):
    rows, ob, op = [], [[] for _ in bps], [[] for _ in pps]
    for i in range(len(pk)):
        for b in range(len(bk)):
            if bk[b] == pk[i]:
                rows.append(i)
                for c, col in enumerate(bps):
                    ob[c].append(int(col[b]))
                for c, col in enumerate(pps):
                    op[c].append(int(col[i]))
    return rows, ob, op


@pytest.mark.parametrize("kdt", [np.int32, np.int64])
def test_rows_brute_force_with_duplicates(kdt):
    rng = np.random.default_rng(5)
    bk = rng.integers(-20, 20, 300).astype(kdt)
    pk = rng.integers(-25, 25, 500).astype(kdt)
    bps = [rng.integers(-2**31, 2**31, 300).astype(np.int32), rng.integers(-2**62, 2**62, 300).astype(np.int64)]
    pps = [rng.integers(-2**40, 2**40, 500).astype(np.int64)]
    rows, ob, op = oracle.join_rows(bk, bps, pk, pps)
    erows, eob, eop = _brute(bk, bps, pk, pps)
    assert rows.tolist() == erows
    assert [c.tolist() for c in ob] == eob
    assert [c.tolist() for c in op] == eop


def test_rows_match_the_aggregates():
    """Count and every SUM over the emitted rows equal the aggregate oracle's (mod 2^64)."""
    bk, b0, b1 = datagen.stream_build(5000, seed=3)
    pk, p0, p1 = datagen.stream_probe(5000, 60_000, seed=3, match_frac=0.3)
    rows, ob, op = oracle.join_rows(bk, [b0, b1], pk, [p0, p1])
    agg = oracle.join_agg(bk, [b0, b1], pk, [p0, p1])
    got = [len(rows)] + [int(c.astype(np.uint64).sum(dtype=np.uint64)) for c in ob + op]
    assert got == [a % M64 for a in agg]
    assert np.all(np.diff(rows.astype(np.int64)) > 0)        # unique build keys: one row per hit, in order


def test_rows_extremes_and_empty():
    i64 = np.iinfo(np.int64)
    bk = np.array([i64.min, i64.max, 0], np.int64)
    pk = np.array([i64.max, 1, i64.min, i64.min], np.int64)
    rows, ob, op = oracle.join_rows(bk, [bk], pk, [pk])
    assert rows.tolist() == [0, 2, 3]
    assert ob[0].tolist() == [i64.max, i64.min, i64.min] and op[0].tolist() == [i64.max, i64.min, i64.min]
    e = np.zeros(0, np.int64)
    assert len(oracle.join_rows(e, [], pk, [])[0]) == 0
    assert len(oracle.join_rows(bk, [], e, [])[0]) == 0
